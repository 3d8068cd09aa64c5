"""GPU parity of the image-centred finite-source magnification (sec. 5) against the
oracle's own implementation of the same steps, through the C ABI: the branch taken
(point source or image-centred, and the number of regions) must agree and the
magnification must agree to 1e-8 relative (both FP64; they differ only in rounding:
libm angles, the complex division, the quintic's root solver, the order of the sums).
The physics of the method is pinned on the oracle (tests/test_oracle_fsmag.py); one
single-lens case is also checked here against the reduced disk integral."""
import math

import numpy as np
import pytest
import torch

import paper_1511_01157_amd as M
from oracle.caustics import caustic_points
from oracle.fsmag import FsOptions, fs_magnification, single_lens_disk
from tests.helpers import note

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def sources(s, q, rho, seed):
    cc = np.asarray(caustic_points(s, q, 4096)).reshape(-1)
    cc = cc[np.isfinite(cc)]
    c0 = cc[np.argmax(cc.real)]
    rng = np.random.default_rng(seed)
    near = cc[rng.integers(0, len(cc), 6)] + rho * (rng.normal(0, 1.0, 6) + 1j * rng.normal(0, 1.0, 6))
    pts = [c0, c0 + 0.5j * rho, c0 + 3j * rho, c0 - 0.9 * rho, c0 + 6j * rho, 0.7 + 0.6j, -1.1 + 0.1j]
    return np.concatenate([np.array(pts), near])


@pytest.mark.parametrize("s,q,rho,gamma", [(0.8, 5e-3, 0.01, 0.0), (0.8, 5e-3, 0.05, 0.53),
                                           (1.2, 0.3, 0.02, 0.53), (1.0, 1e-2, 0.005, 0.0)])
def test_fs_magnification_matches_the_oracle(s, q, rho, gamma):
    z = sources(s, q, rho, 7)
    note(f"fsmag: s={s} q={q} rho={rho} gamma={gamma}, {len(z)} sources")
    zt = torch.from_numpy(np.stack([z.real, z.imag], 1).copy()).to(DEV)
    A, nreg = M.fs_magnification(s, q, zt, rho, gamma)
    A, nreg = A.cpu().numpy(), nreg.cpu().numpy()
    opt = FsOptions()
    for k, zk in enumerate(z):
        oA, d = fs_magnification(zk, rho, gamma, s, q, opt=opt, details=True)
        if d["point_source"]:
            assert nreg[k] == -1, k
        else:
            assert nreg[k] == len(d["regions"]), (k, nreg[k], d["regions"])
        assert abs(A[k] / oA - 1) < 1e-8, (k, A[k], oA)
    assert (nreg > 0).sum() >= 6 and (nreg == -1).sum() >= 2


@pytest.mark.parametrize("kw", [dict(n_b=64, n_side=50, n_grow=20, n_r=200, n_theta=300, n_shrink=3),
                                dict(n_b=40, n_side=16, n_grow=5, n_r=96, n_theta=700, n_shrink=0)])
def test_fs_magnification_options_match_the_oracle(kw):
    """Grids whose column count is not a multiple of the integration workgroup's 512
    lanes (300, 700), more and no shrink passes, fewer boundary seeds."""
    s, q, rho, gamma = 1.2, 0.3, 0.02, 0.53
    z = sources(s, q, rho, 3)[:9]
    note(f"fsmag options {kw}")
    zt = torch.from_numpy(np.stack([z.real, z.imag], 1).copy()).to(DEV)
    A, nreg = M.fs_magnification(s, q, zt, rho, gamma, **kw)
    A, nreg = A.cpu().numpy(), nreg.cpu().numpy()
    opt = FsOptions(**kw)
    for k, zk in enumerate(z):
        oA, d = fs_magnification(zk, rho, gamma, s, q, opt=opt, details=True)
        assert nreg[k] == (-1 if d["point_source"] else len(d["regions"])), (k, nreg[k])
        assert abs(A[k] / oA - 1) < 1e-8, (k, A[k], oA)
    assert (nreg > 0).sum() >= 4


def test_more_near_sources_than_one_pass():
    """4500 sources within 3 rho of the caustic: two passes of the image-centred kernels
    (at most 4096 sources each).  Splitting the call elsewhere gives the same bits, and
    sampled sources match the oracle."""
    s, q, rho, gamma = 0.8, 5e-3, 0.01, 0.53
    kw = dict(n_b=32, n_side=32, n_grow=10, n_r=64, n_theta=64, n_shrink=1)
    cc = np.asarray(caustic_points(s, q, 4096)).reshape(-1)
    cc = cc[np.isfinite(cc)]
    rng = np.random.default_rng(11)
    z = cc[rng.integers(0, len(cc), 4500)] + rho * (rng.uniform(-2, 2, 4500) + 1j * rng.uniform(-2, 2, 4500))
    zt = torch.from_numpy(np.stack([z.real, z.imag], 1).copy()).to(DEV)
    note("fsmag: 4500 near sources, two passes")
    A, nreg = M.fs_magnification(s, q, zt, rho, gamma, **kw)
    A1, n1 = M.fs_magnification(s, q, zt[:1700].contiguous(), rho, gamma, **kw)
    A2, n2 = M.fs_magnification(s, q, zt[1700:].contiguous(), rho, gamma, **kw)
    A, nreg = A.cpu().numpy(), nreg.cpu().numpy()
    assert (nreg > 0).sum() > 4096
    assert np.array_equal(A, np.concatenate([A1.cpu().numpy(), A2.cpu().numpy()]), equal_nan=True)
    assert np.array_equal(nreg, np.concatenate([n1.cpu().numpy(), n2.cpu().numpy()]))
    opt = FsOptions(**kw)
    for k in (0, 17, 4095, 4096, 4100, 4499):
        oA, d = fs_magnification(z[k], rho, gamma, s, q, opt=opt, details=True)
        assert nreg[k] == (-1 if d["point_source"] else len(d["regions"])), k
        assert abs(A[k] / oA - 1) < 1e-8, (k, A[k], oA)


def test_single_lens_against_the_disk_integral_on_the_gpu():
    s, q = 3.0, 1e-10
    b = np.array([0.0, 0.05, 0.1, 0.2, 0.5])
    zt = torch.from_numpy(np.stack([b, np.zeros_like(b)], 1)).to(DEV)
    for gamma in (0.0, 0.53):
        note(f"fsmag: single lens gamma={gamma}")
        A, nreg = M.fs_magnification(s, q, zt, 0.1, gamma)
        for k, bk in enumerate(b):
            tol = 5e-4 if bk == 0.1 else 2e-4
            assert abs(float(A[k]) / single_lens_disk(bk, 0.1, gamma) - 1) < tol, (bk, gamma)


def test_fs_magnification_argument_errors():
    zt = torch.zeros((1, 2), dtype=torch.float64, device=DEV)
    with pytest.raises(M.MorseError):
        M.fs_magnification(1.0, 1e-3, zt, -0.1)
    with pytest.raises(M.MorseError):
        M.fs_magnification(1.0, 1e-3, zt, 0.1, gamma=1.5)
    with pytest.raises(M.MorseError):
        M.fs_magnification(1.0, 1e-3, zt, 0.1, n_r=1)
    A, nreg = M.fs_magnification(1.0, 1e-3, zt[:0], 0.1)
    assert A.numel() == 0


def test_trajectory_positions():
    t = np.linspace(-40.0, 40.0, 1001) + 2456000.0
    p = (2456003.0, 0.07, 23.0, 1.1)
    z = M.trajectory_positions(p, torch.from_numpy(t).to(DEV)).cpu().numpy()
    tau = (t - p[0]) / p[2]
    ref = np.stack([tau * math.cos(p[3]) - p[1] * math.sin(p[3]),
                    tau * math.sin(p[3]) + p[1] * math.cos(p[3])], 1)
    assert np.max(np.abs(z - ref)) < 1e-13
