"""Pins of the oracle's real-space (affine) deskew against what the
geometry fixes, independently of its formula:

* frame: the scan-coordinate range of the stack's corners, both scan
  directions;
* a sheet along the scan axis with unit steps turns the resampling into a
  pure index shear, equal to NumPy indexing bit for bit;
* images varying linearly along the scan are reproduced exactly;
* a dense hat-kernel matrix built element by element;
* a bright spot at a physical position lands at its scan coordinate, and at
  the same physical point the remap places it (rotation into the sheet
  frame).
"""
import math

import numpy as np
import pytest

import oracle


def test_frame_is_the_scan_range_of_the_corners():
    a = math.radians(35.0)
    y0, ny = oracle.affine_frame(512, 2048, 35.0, 0.4, 0.115, 0.115)
    span = 511 * 0.4 + 2047 * 0.115 * math.cos(a)
    assert y0 == 0.0 and ny == math.floor(span / 0.115) + 1
    y0, ny = oracle.affine_frame(10, 50, 30.0, -0.3, 0.1, 0.05)
    assert y0 == pytest.approx(-2.7, abs=1e-12)
    assert ny == math.floor((49 * 0.1 * math.cos(math.radians(30)) + 2.7) / 0.05) + 1


@pytest.mark.parametrize("n,c,ang,step,pix,dy", [(7, 13, 35.0, 0.4, 0.115, 0.115),
                                                 (10, 50, 30.0, -0.3, 0.1, 0.05),
                                                 (5, 9, 60.0, 0.25, 0.2, 0.07),
                                                 (1, 6, 45.0, 0.4, 0.1, 0.03),
                                                 (12, 1, 20.0, -0.5, 0.1, 0.2)])
def test_frame_is_the_smallest_grid_covering_every_pixel(n, c, ang, step, pix, dy):
    """Brute force over every raw pixel's scan coordinate n z + c p cos(alpha):
    the grid starts at the smallest, its last slice lies at or before the
    largest and one more slice would lie beyond it."""
    pc = pix * math.cos(math.radians(ang))
    ys = [k * step + j * pc for k in range(n) for j in range(c)]
    y0, ny = oracle.affine_frame(n, c, ang, step, pix, dy)
    assert y0 == pytest.approx(min(ys), abs=1e-12)
    top = max(ys)
    assert y0 + (ny - 1) * dy <= top + 1e-12
    assert y0 + ny * dy > top + 1e-12


def test_sheet_along_scan_axis_is_an_index_shear():
    """alpha = 0, unit pixel, step and y-step: image coordinate u = y - z
    exactly, so V[y, x, z] = S[y - z, x, z] (zero outside)."""
    rng = np.random.default_rng(0)
    s = rng.integers(0, 65535, (7, 3, 5), dtype=np.uint16)
    v, (y0, ny) = oracle.affine(s, 0.0, 1.0, 1.0, 1.0)
    assert y0 == 0.0 and ny == 7 + 4
    ref = np.zeros((ny, 3, 5), np.float32)
    for y in range(ny):
        for z in range(5):
            n = y - z
            if 0 <= n < 7:
                ref[y, :, z] = s[n, :, z]
    assert np.array_equal(v, ref)


def test_linear_scan_profile_is_reproduced():
    n, r, c = 12, 2, 9
    a, b = 3.25, 0.75
    s = np.broadcast_to((a + b * np.arange(n, dtype=np.float64))[:, None, None],
                        (n, r, c)).astype(np.float32)
    ang, step, pix, dy = 40.0, 0.5, 0.2, 0.13
    v, (y0, ny) = oracle.affine(s, ang, step, pix, dy, vol64=True)
    pc = pix * math.cos(math.radians(ang))
    for y in range(ny):
        for z in range(c):
            u = (y0 + y * dy - z * pc) / step
            if 0.0 <= u <= n - 1 - 1e-9:
                assert v[y, 0, z] == pytest.approx(a + b * u, rel=1e-12), (y, z)


@pytest.mark.parametrize("seed", [1, 2])
def test_dense_hat_matrix(seed):
    rng = np.random.default_rng(seed)
    n, r, c = 5, 2, 6
    s = rng.random((n, r, c)).astype(np.float32)
    ang = float(rng.uniform(20, 60))
    step = float(rng.choice([-1, 1]) * rng.uniform(0.2, 0.6))
    pix, dy = 0.15, float(rng.uniform(0.05, 0.3))
    v, (y0, ny) = oracle.affine(s, ang, step, pix, dy, vol64=True)
    pc = pix * math.cos(math.radians(ang))
    s64 = s.astype(np.float64)
    want = np.zeros((ny, r, c))
    for y in range(ny):
        for z in range(c):
            u = (y0 + y * dy - z * pc) / step
            for k in range(n):
                want[y, :, z] += max(0.0, 1.0 - abs(u - k)) * s64[k, :, z]
    np.testing.assert_allclose(v, want, rtol=1e-12, atol=1e-14)


def _spot(shape, n0, r0, c0, sigma=3.0, amp=1000.0):
    n, r, c = shape
    nn, rr, cc = np.meshgrid(np.arange(n), np.arange(r), np.arange(c), indexing="ij")
    return (amp * np.exp(-((nn - n0) ** 2 + (rr - r0) ** 2 + (cc - c0) ** 2)
                         / (2 * sigma ** 2))).astype(np.float32)


@pytest.mark.parametrize("ang", [30.0, 35.0, 50.0])
def test_spot_lands_at_its_scan_coordinate(ang):
    shape = (40, 3, 64)
    step, pix, dy = 0.4, 0.115, 0.05
    st = _spot(shape, 19.6, 1, 31.3)
    s = st[:, 1, :].astype(np.float64)
    m = s.sum()
    n_bar = (s.sum(1) * np.arange(shape[0])).sum() / m
    c_bar = (s.sum(0) * np.arange(shape[2])).sum() / m
    a = math.radians(ang)
    y_phys = n_bar * step + c_bar * pix * math.cos(a)      # scan coordinate
    z_phys = c_bar * pix * math.sin(a)                     # height
    v, (y0, ny) = oracle.affine(st, ang, step, pix, dy, vol64=True)
    row = v[:, 1, :]
    got_y = (row.sum(1) * np.arange(ny)).sum() / row.sum() * dy + y0
    got_z = (row.sum(0) * np.arange(shape[2])).sum() / row.sum() * pix * math.sin(a)
    assert got_y == pytest.approx(y_phys, abs=0.05 * dy)
    assert got_z == pytest.approx(z_phys, abs=1e-3 * pix)
    # the remap puts the same spot at (Y cos a + Z sin a) / p in its columns
    offs = oracle.offsets_uniform(shape[0], oracle.shift_px(ang, step, pix))
    d = oracle.deskew(st, offs, vol=False)
    p = d["psum"][1].astype(np.float64)
    x_bar = (p * np.arange(p.size)).sum() / p.sum()
    assert x_bar + d["origin"] == pytest.approx(
        (y_phys * math.cos(a) + z_phys * math.sin(a)) / pix, abs=1e-6)
