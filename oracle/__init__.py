"""CPU oracle for the MORSE map-build + trajectory-search path (McDougall & Albrow 2015).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library under
``paper_1511_01157_amd`` and its Python binding) may import, link or execute anything
in this package.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` use it.  It shares no code, headers, tables or constants with the HIP
path; the only common dependency is the seeded input generator in ``workloads``, which
holds none of the method's arithmetic.

Modules, each citing the passage of the paper it follows:

* ``lens``      lens placement (sec. 4.1), Eq. 2 lens equation, quintic image
                positions and point-source magnification (Eqs. 3-4), Paczynski limit.
* ``caustics``  critical curves / caustics and the caustic-pixel mask.
* ``rays``      inverse ray shooting into a source-plane histogram (the ray-shooting
                map family the paper cites in sec. 3): FP32 FMA-free mirror (numpy and
                an independent C build) and an FP64 version.
* ``maps``      normalisation by the no-lens ray density and uniform-disk convolution
                (sec. 4.1 convolution of the point-source map by a source profile).
* ``sampling``  trajectory geometry (sec. 4.1 parameters, sec. 4.2 trajectories) and
                bilinear map sampling.
* ``fit``       profiled linear flux fit (Eqs. 5-6), chi-square, best / top-k selection.
* ``adjoint``   chi-square gradient with respect to (t0, u0, tE, alpha).
* ``lbfgs``     batched L-BFGS refinement state machine.

Parity status of each function is stated in its docstring; functions without an
independent pin say "parity unpinned".
"""
