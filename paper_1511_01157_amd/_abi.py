"""ctypes declarations of include/morse.h and the loader of libmorse.so."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmorse.so")

MORSE_OK, MORSE_EINVAL, MORSE_ENOMEM, MORSE_EHIP, MORSE_ERANGE, MORSE_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
TRAJ_GRID, TRAJ_LIST = 0, 1
SEARCH_PLAIN, SEARCH_BATCHED = 0, 1


class Grid2D(ctypes.Structure):
    _fields_ = [("cx", c_double), ("cy", c_double), ("wx", c_double), ("wy", c_double),
                ("nx", c_int32), ("ny", c_int32)]


class MapStats(ctypes.Structure):
    _fields_ = [("rays_total", c_uint64), ("rays_in", c_uint64), ("rays_out", c_uint64),
                ("rays_nonfinite", c_uint64), ("rays_zero_axis", c_uint64),
                ("max_count", c_uint32), ("reserved", c_uint32)]


class MapView(ctypes.Structure):
    _fields_ = [("d_map", c_void_p), ("window", Grid2D)]


class FsOpts(ctypes.Structure):
    _fields_ = [("n_b", c_int32), ("n_crit", c_int32), ("n_side", c_int32), ("n_grow", c_int32),
                ("n_r", c_int32), ("n_theta", c_int32), ("n_shrink", c_int32), ("reserved", c_int32),
                ("near", c_double), ("gap", c_double)]


class LightCurves(ctypes.Structure):
    _fields_ = [("n_events", c_int32), ("reserved", c_int32), ("h_offsets", c_void_p),
                ("h_t_ref", c_void_p), ("d_t", c_void_p), ("d_flux", c_void_p),
                ("d_weight", c_void_p)]


class Trajectories(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("n_u0", c_int32), ("n_alpha", c_int32), ("n_t0", c_int32),
                ("n_tE", c_int32), ("shared", c_int32), ("h_u0", c_void_p), ("h_alpha", c_void_p),
                ("h_t0", c_void_p), ("h_tE", c_void_p), ("n", c_int64), ("d_params", c_void_p)]


class SearchOut(ctypes.Structure):
    _fields_ = [("d_chi2", c_void_p), ("d_fs", c_void_p), ("d_fb", c_void_p),
                ("d_best_chi2", c_void_p), ("d_best_idx", c_void_p), ("top_k", c_int32),
                ("reserved", c_int32), ("d_topk_chi2", c_void_p), ("d_topk_idx", c_void_p)]


class SimplexOpts(ctypes.Structure):
    _fields_ = [("max_iter", c_int32), ("reserved", c_int32), ("step_t0", c_double),
                ("step_ln_tE", c_double), ("ftol", c_double)]


class LbfgsOpts(ctypes.Structure):
    _fields_ = [("steps", c_int32), ("history", c_int32), ("max_ls", c_int32),
                ("reserved", c_int32), ("c1", c_double), ("shrink", c_double)]


# name -> (restype, argtypes)
SIGNATURES = {
    "morse_abi_version": (c_int32, []),
    "morse_ctx_create": (c_int32, [c_int32, c_void_p, POINTER(c_void_p)]),
    "morse_ctx_destroy": (c_int32, [c_void_p]),
    "morse_ctx_set_stream": (c_int32, [c_void_p, c_void_p]),
    "morse_ctx_synchronize": (c_int32, [c_void_p]),
    "morse_ctx_set_timing": (c_int32, [c_void_p, ctypes.c_uint32]),
    "morse_autotune_load": (c_int32, [c_void_p, c_char_p, ctypes.POINTER(c_int32)]),
    "morse_ctx_kernel_time": (c_int32, [c_void_p, c_int32, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(c_int64), c_int32]),
    "morse_last_error": (c_char_p, [c_void_p]),
    "morse_rayshoot": (c_int32, [c_void_p, c_double, c_double, POINTER(Grid2D), POINTER(Grid2D),
                                 c_int32, c_int32, c_void_p, c_int32, c_void_p]),
    "morse_normalize_convolve": (c_int32, [c_void_p, c_void_p, POINTER(Grid2D), POINTER(Grid2D),
                                           c_double, c_void_p]),
    "morse_convolve_stack": (c_int32, [c_void_p, c_void_p, POINTER(Grid2D), POINTER(Grid2D),
                                       c_void_p, c_int32, c_double, c_int32, c_void_p]),
    "morse_profile_weights": (c_int32, [c_double, c_double, c_double, c_double, c_void_p, c_int64,
                                        POINTER(c_int32), POINTER(c_int32)]),
    "morse_caustics": (c_int32, [c_double, c_double, c_int32, c_void_p, c_int32, POINTER(c_int32)]),
    "morse_caustic_lines": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_void_p, c_int32, c_void_p]),
    "morse_line_filter": (c_int32, [c_void_p, POINTER(MapView), c_void_p, c_int64, c_double, c_void_p,
                                    c_void_p, c_void_p, c_void_p, POINTER(c_int64)]),
    "morse_line_peaks": (c_int32, [c_void_p, POINTER(MapView), c_void_p, c_int64, c_double, c_int32,
                                   c_double, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p, POINTER(c_int64)]),
    "morse_peak_starts": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p,
                                    c_void_p, c_int32, c_void_p, c_int32, c_double, c_void_p]),
    "morse_fs_magnification": (c_int32, [c_void_p, c_double, c_double, c_void_p, c_int64, c_double,
                                         c_double, POINTER(FsOpts), c_void_p, c_void_p]),
    "morse_trajectory_positions": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p]),
    "morse_lines_to_trajectories": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_int32,
                                              c_void_p, c_int32, c_void_p]),
    "morse_line_simplex": (c_int32, [c_void_p, POINTER(MapView), c_int32, POINTER(LightCurves), c_int32,
                                     c_void_p, c_int64, c_void_p, POINTER(SimplexOpts), c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_void_p]),
    "morse_build_map": (c_int32, [c_void_p, c_double, c_double, POINTER(Grid2D), POINTER(Grid2D),
                                  c_double, c_void_p, c_void_p, POINTER(MapStats)]),
    "morse_search": (c_int32, [c_void_p, POINTER(MapView), c_int32, POINTER(LightCurves),
                               POINTER(Trajectories), c_int32, POINTER(SearchOut)]),
    "morse_autotune": (c_int32, [c_void_p, POINTER(MapView), c_int32, POINTER(LightCurves),
                                 POINTER(Trajectories), c_char_p, POINTER(c_int32)]),
    "morse_candidates_from_topk": (c_int32, [c_void_p, POINTER(Trajectories), c_int32, c_int32,
                                             c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "morse_chi2_grad": (c_int32, [c_void_p, POINTER(MapView), c_int32, POINTER(LightCurves),
                                  c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p]),
    "morse_chi2_grad_noalloc": (c_int32, [c_void_p, POINTER(MapView), c_int32,
                                          POINTER(LightCurves), c_int64, c_void_p, c_void_p,
                                          c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "morse_refine": (c_int32, [c_void_p, POINTER(MapView), c_int32, POINTER(LightCurves), c_int64,
                               c_void_p, c_void_p, c_void_p, POINTER(LbfgsOpts), c_void_p,
                               c_void_p]),
}

_LIB = None


def load():
    """Load libmorse.so (raises if it is missing: there is no fallback path)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB
