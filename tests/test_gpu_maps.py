"""GPU parity of the map build: ray counts bit-exact vs the FP32 mirror oracle,
normalised/convolved maps within the map gate (relative 1e-3 outside caustic pixels,
expected ~1e-7), statistics, symmetry and conservation at full size."""
import numpy as np
import pytest
import torch

import paper_1511_01157_amd as M
import workloads as W
from oracle.caustics import caustic_mask
from oracle.maps import disk_pixel_weights, map_scale, normalize_convolve_exact64, normalize_convolve_mirror32
from oracle.rays import rayshoot_mirror32_c
from tests.helpers import note

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def gpu_counts(s, q, rays, window, rows=None):
    counts = torch.empty((window[5], window[4]), dtype=torch.int32, device=DEV)
    stats = torch.zeros(3, dtype=torch.int64, device=DEV)
    M.rayshoot(s, q, rays, window, counts, rows=rows, stats=stats)
    torch.cuda.synchronize()
    c = counts.cpu().numpy().view(np.uint32)
    st = stats.cpu().numpy()
    return c, dict(out=int(st[0]), nonfinite=int(st[1]), zero_axis=int(st[2]))


def test_tiny_counts_bit_exact_and_stats():
    c = W.config("tiny")
    note("rayshoot tiny full")
    g, gst = gpu_counts(c["s"], c["q"], c["rays"], c["window"])
    o, ost = rayshoot_mirror32_c(c["s"], c["q"], c["rays"], c["window"], nthreads=8)
    assert np.array_equal(g, o)
    assert gst == ost


@pytest.mark.parametrize("s,q,rays,window", [
    (0.8, 5e-3, (0.1, -0.05, 3.0, 2.5, 650, 514), (0.02, 0.01, 1.5, 1.2, 202, 160)),  # ragged tiles
    (2.0, 1.0, (0.0, 0.0, 6.0, 6.0, 1030, 1026), (0.5, 0.0, 3.0, 3.0, 256, 256)),      # equal masses
    (1.0, 0.0, (0.0, 0.0, 4.0, 4.0, 1024, 1024), (0.0, 0.0, 2.0, 2.0, 128, 128)),      # single lens
    (1.0, 1e-3, (0.0, 0.0, 0.5, 0.5, 256, 256), (5.0, 5.0, 1.0, 1.0, 64, 64)),         # window missed
    (0.3, 0.1, (0.0, 0.0, 2.0, 2.0, 2, 2), (0.0, 0.0, 2.0, 2.0, 2, 2)),                # minimal grids
    (0.5, 0.0, (-0.3, 0.0, 4.0, 4.0, 1026, 1026), (0.0, 0.0, 2.0, 2.0, 128, 128)),    # zero-axis rays
    (2.0, 1.0, (-0.3, 0.0, 1.0, 1.0, 768, 768), (0.2, 0.0, 2.0, 2.0, 128, 128)),      # zero-axis rays
])
def test_counts_bit_exact_edge_cases(s, q, rays, window):
    """Lattices and windows centred on the lens axis go through mirror pairs (the last
    two cases have rays whose window y offset is exactly zero, which the pairing counts
    twice in their own bin); the others shoot every ray."""
    note(f"rayshoot edge s={s} q={q} rays={rays} window={window}")
    g, gst = gpu_counts(s, q, rays, window)
    o, ost = rayshoot_mirror32_c(s, q, rays, window, nthreads=8)
    assert np.array_equal(g, o)
    assert gst == ost
    if rays[0] == -0.3:
        assert ost["zero_axis"] > 0


def test_large_counts_row_slices_bit_exact():
    """Full-size lattice (32768^2 rays into 2048^2): row slices through the lens axis
    (all rows paired with their mirror rows; a ragged part paired, the rest not; the two
    middle rows), the lattice edge and a ragged end, each bit-exact against the mirror."""
    c = W.config("large")
    for rows in [(16320, 16448), (16000, 16500), (16383, 16385), (0, 64), (32700, 32768),
                 (9000, 9037)]:
        note(f"rayshoot large rows {rows}")
        g, gst = gpu_counts(c["s"], c["q"], c["rays"], c["window"], rows=rows)
        o, ost = rayshoot_mirror32_c(c["s"], c["q"], c["rays"], c["window"], rows=rows, nthreads=16)
        assert np.array_equal(g, o), rows
        assert gst == ost


def test_large_full_build_bit_exact_conservation_symmetry_and_map_gate():
    """The whole large workload: 32768^2 rays -> 2048^2 counts bit-exact against the
    oracle's own full run; the GPU map within the map gate of the oracle's FP64
    normalise/convolve of the oracle counts outside caustic pixels."""
    c = W.config("large")
    note("oracle rayshoot large full")
    o, ost = rayshoot_mirror32_c(c["s"], c["q"], c["rays"], c["window"], nthreads=16)
    note("build_map large full")
    counts = torch.empty((2048, 2048), dtype=torch.int32, device=DEV)
    amap, st = M.build_map(c["s"], c["q"], c["rays"], c["window"], c["rho"], device=DEV,
                           counts=counts, stats=True)
    torch.cuda.synchronize()
    cnt = counts.cpu().numpy().view(np.uint32)
    assert np.array_equal(cnt, o)
    n = c["rays"][4] * c["rays"][5]
    assert st["rays_total"] == n
    assert (st["rays_out"], st["rays_nonfinite"], st["rays_zero_axis"]) == (ost["out"], ost["nonfinite"], ost["zero_axis"])
    assert int(cnt.sum(dtype=np.uint64)) == st["rays_in"]
    assert st["rays_in"] + st["rays_out"] + st["rays_nonfinite"] == n
    assert st["max_count"] == int(cnt.max())
    if st["rays_zero_axis"] == 0:
        assert np.array_equal(cnt, cnt[::-1, :])
    dx = c["window"][2] / 2048
    w = disk_pixel_weights(c["rho"], dx, dx)
    ref64 = normalize_convolve_exact64(o, map_scale(c["rays"], c["window"], fp32=False), w)
    ref32 = normalize_convolve_mirror32(o, map_scale(c["rays"], c["window"]), w)
    A = amap.cpu().numpy()
    mask = caustic_mask(c["s"], c["q"], *c["window"], margin_px=2, rho=c["rho"])
    ok = ~mask & (ref64 > 0)
    err = np.abs(A[ok] / ref64[ok] - 1)
    assert err.max() < 1e-3   # the stated map gate
    assert err.max() < 1e-6   # what binary32 rounding alone allows
    assert np.max(np.abs(A.astype(np.float64) - ref32) / np.maximum(ref32, 1e-30)) < 2e-7


@pytest.mark.parametrize("rho", [0.0, 1e-3, 2e-3, 0.01])
def test_normalize_convolve_vs_mirror(rho):
    c = W.config("tiny")
    note(f"normalize_convolve tiny rho={rho}")
    o, _ = rayshoot_mirror32_c(c["s"], c["q"], c["rays"], c["window"], nthreads=8)
    cnt = torch.from_numpy(o.view(np.int32)).to(DEV)
    A = M.normalize_convolve(cnt, c["rays"], c["window"], rho).cpu().numpy()
    dx = c["window"][2] / c["window"][4]
    w = disk_pixel_weights(rho, dx, dx)
    ref32 = normalize_convolve_mirror32(o, map_scale(c["rays"], c["window"]), w)
    ref64 = normalize_convolve_exact64(o, map_scale(c["rays"], c["window"], fp32=False), w)
    pos = ref64 > 0
    assert np.max(np.abs(A[pos] / ref64[pos] - 1)) < 1e-6
    # the weights are computed independently on both sides; when they round to the
    # same binary32 values the maps agree bit for bit
    assert np.max(np.abs(A - ref32)) <= 2e-7 * max(1.0, float(ref32.max()))


@pytest.mark.parametrize("window,rho,shift", [
    ((0.1, -0.05, 2.0, 1.3, 334, 218), 0.0, 0),     # 16-byte loads and stores
    ((0.1, -0.05, 2.0, 1.3, 334, 218), 0.0, 1),     # buffers 4 B off 16: the scalar path
    ((0.1, -0.05, 2.0, 1.3, 334, 218), 0.02, 0),    # ragged 64 x 32 tiles, a 3-pixel stencil
    ((0.1, -0.05, 2.0, 1.3, 334, 218), 0.0862, 1),  # the widest stencil (15 pixels)
    ((0.0, 0.0, 0.2, 2.0, 8, 70), 0.05, 0)])        # narrower than one tile, halo beyond both edges
def test_build_map_ragged_tiles_bit_exact(window, rho, shift):
    """Maps whose sides are not multiples of the 64 x 32 output tile, and buffers not
    16-byte aligned: every pixel, the clamped halo and the largest count against the
    binary32 mirror."""
    s, q, rays = 1.0, 1e-3, (0.0, 0.0, 4.0, 4.0, 1600, 1600)
    note(f"build_map ragged window={window} rho={rho} shift={shift}")
    o, _ = rayshoot_mirror32_c(s, q, rays, window, nthreads=8)
    npx = window[4] * window[5]
    cbuf = torch.empty(npx + 4, dtype=torch.int32, device=DEV)
    abuf = torch.empty(npx + 4, dtype=torch.float32, device=DEV)
    cnt = cbuf[shift:shift + npx].view(window[5], window[4])
    out = abuf[shift:shift + npx].view(window[5], window[4])
    A, st = M.build_map(s, q, rays, window, rho, device=DEV, out=out, counts=cnt, stats=True)
    assert np.array_equal(cnt.cpu().numpy().view(np.uint32), o)
    assert st["max_count"] == int(o.max())
    w = disk_pixel_weights(rho, window[2] / window[4], window[3] / window[5])
    assert max(w.shape) <= 31
    ref32 = normalize_convolve_mirror32(o, map_scale(rays, window), w)
    A = A.cpu().numpy()
    assert np.max(np.abs(A - ref32)) <= 2e-7 * max(1.0, float(ref32.max()))
    B = M.normalize_convolve(cnt, rays, window, rho).cpu().numpy()
    assert np.array_equal(A, B)


@pytest.mark.parametrize("window,rho,shift", [
    ((0.1, -0.05, 2.0, 1.3, 334, 218), 0.005, 0),   # 3 x 3, nine taps, ragged wavefront tiles
    ((0.1, -0.05, 2.0, 1.3, 334, 218), 0.0033, 1),  # 3 x 3, five taps, buffers 4 B off 16
    ((0.0, 0.0, 0.2, 2.0, 8, 70), 0.02, 0),         # narrower than one wavefront's columns
    ((0.0, 0.0, 2.0, 5.0, 100, 100), 0.015, 0),     # reach 1 in x, 0 in y
    ((0.1, -0.05, 2.0, 1.3, 334, 218), 0.02, 0)])   # 7 x 7: the LDS-tiled kernel
def test_normalize_bitwise_with_the_library_weights(window, rho, shift):
    """Every pixel bit for bit against the binary32 mirror run with the library's own
    FP64 weights: the taps' order, their offsets' directions and the edge clamp."""
    s, q, rays = 1.0, 1e-3, (0.0, 0.0, 4.0, 4.0, 1600, 1600)
    note(f"normalize bitwise window={window} rho={rho} shift={shift}")
    o, _ = rayshoot_mirror32_c(s, q, rays, window, nthreads=8)
    npx = window[4] * window[5]
    cbuf = torch.empty(npx + 4, dtype=torch.int32, device=DEV)
    abuf = torch.empty(npx + 4, dtype=torch.float32, device=DEV)
    cnt = cbuf[shift:shift + npx].view(window[5], window[4])
    out = abuf[shift:shift + npx].view(window[5], window[4])
    cnt.copy_(torch.from_numpy(o.view(np.int32)))
    M.normalize_convolve(cnt, rays, window, rho, out=out)
    w = M.profile_weights(rho, window[2] / window[4], window[3] / window[5], 0.0)
    ref32 = normalize_convolve_mirror32(o, map_scale(rays, window), w)
    A = out.cpu().numpy()
    assert np.array_equal(A, ref32), int(np.count_nonzero(A != ref32))


def test_build_map_rejects_bad_arguments():
    note("build_map argument errors")
    with pytest.raises(M.MorseError) as e:
        M.build_map(1.0, 2.0, (0, 0, 4, 4, 64, 64), (0, 0, 2, 2, 16, 16), device=DEV)
    assert e.value.code == -1
    with pytest.raises(M.MorseError) as e:
        M.build_map(1.0, 0.1, (0, 0, 4, 4, 63, 64), (0, 0, 2, 2, 16, 16), device=DEV)
    assert e.value.code == -1
    with pytest.raises(M.MorseError) as e:
        M.build_map(1.0, 0.1, (0, 0, 4, 4, 64, 64), (0, 0, 2, 2, 16, 16), rho=-1.0, device=DEV)
    assert e.value.code == -1
    with pytest.raises(M.MorseError) as e:
        # rho / pixel = 16 > 15: the stencil would exceed 31 x 31
        M.build_map(1.0, 0.1, (0, 0, 4, 4, 64, 64), (0, 0, 2, 2, 16, 16), rho=2.0, device=DEV)
    assert e.value.code == -4
