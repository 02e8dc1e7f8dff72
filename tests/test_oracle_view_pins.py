"""Pins of the oracle's shear-warp rotated view (Fig. 3) against what the
geometry and the mathematics fix, independently of the oracle's formulas:

* view geometry at the three angles with a known answer (theta = alpha is
  Eq. 1 with no stretch, theta = 0 looks down the optical axis, theta = 90
  degrees is the side view along the scan axis);
* the stretch is the identity at factor 1, reproduces linear rows exactly
  and equals a dense hat-kernel resampling matrix built element by element;
* a bright spot placed at a physical position (Y, Z) lands, in the view at
  angle theta, at the rotated coordinate (Y cos theta + Z sin theta) / p,
  and two spots on one line of sight collapse onto one view column.
"""
import math

import numpy as np
import pytest

import oracle

ALPHA, STEP, PIXEL = 30.0, 0.4, 0.115


def test_view_geometry_special_angles():
    s, w = oracle.view_geometry(ALPHA, ALPHA, STEP, PIXEL)
    assert s == oracle.shift_px(ALPHA, STEP, PIXEL) and w == 1.0
    a = math.radians(ALPHA)
    s, w = oracle.view_geometry(0.0, ALPHA, STEP, PIXEL)
    assert s == pytest.approx(STEP / (PIXEL * math.cos(a)), rel=1e-15)
    assert w == pytest.approx(math.cos(a), rel=1e-15)
    s, w = oracle.view_geometry(90.0, ALPHA, STEP, PIXEL)
    assert abs(s) < 1e-15 and w == pytest.approx(math.sin(a), rel=1e-15)


def test_warp_factor_one_is_identity():
    rng = np.random.default_rng(0)
    p = rng.random((5, 37))
    out = oracle.warp(p, 1.0)
    assert out.shape == p.shape
    assert np.array_equal(out, p)


@pytest.mark.parametrize("wf", [0.9999, 0.8660254037844387, 0.5, 0.31])
def test_warp_reproduces_linear_rows(wf):
    x = np.arange(200, dtype=np.float64)
    p = np.stack([3.5 + 0.25 * x, 100.0 - 0.4 * x])
    out = oracle.warp(p, wf)
    j = np.arange(out.shape[1], dtype=np.float64)
    assert out.shape[1] == math.floor(199 * wf) + 1
    assert (out.shape[1] - 1) / wf <= 199 + 1e-9
    np.testing.assert_allclose(out[0], 3.5 + 0.25 * j / wf, rtol=1e-12)
    np.testing.assert_allclose(out[1], 100.0 - 0.4 * j / wf, rtol=1e-12, atol=1e-11)


@pytest.mark.parametrize("w_in,wf", [(200, 0.9999), (200, 0.8660254037844387), (3504, 0.5),
                                     (37, 0.31), (1, 0.7), (2, 1.0), (4218, 0.8191520442889918),
                                     (11, 0.5)])
def test_view_width_is_the_largest_inside_the_row(w_in, wf):
    """The view keeps exactly the columns j = 0, 1, ... whose sample point
    j / wf lies on the projection row (at most the last column's centre
    w_in - 1): counted one by one, and the next column falls outside."""
    w = oracle.view_width(w_in, wf)
    inside = 0
    while inside / wf <= w_in - 1:
        inside += 1
    assert w == inside
    assert (w - 1) / wf <= w_in - 1 < w / wf


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_warp_equals_dense_hat_matrix(seed):
    rng = np.random.default_rng(seed)
    w_in = int(rng.integers(3, 24))
    wf = float(rng.uniform(0.3, 1.0))
    w_out = int(rng.integers(1, w_in + 4))          # also longer than the support
    p = rng.random((3, w_in))
    m = np.zeros((w_out, w_in))
    for j in range(w_out):
        for x in range(w_in):
            m[j, x] = max(0.0, 1.0 - abs(j / wf - x))
    np.testing.assert_allclose(oracle.warp(p, wf, w_out), p @ m.T, rtol=1e-13, atol=1e-15)


def _spot_stack(spots, shape, sigma=3.0):
    """Float32 stack with Gaussian spots at raw (n, r, c) index positions."""
    n, r, c = shape
    nn, rr, cc = np.meshgrid(np.arange(n), np.arange(r), np.arange(c), indexing="ij")
    s = np.zeros(shape, np.float64)
    for (n0, r0, c0, a) in spots:
        s += a * np.exp(-((nn - n0) ** 2 + (rr - r0) ** 2 + (cc - c0) ** 2) / (2 * sigma ** 2))
    return s.astype(np.float32)


def _physical(n, c):
    """(Y, Z) in um of raw image n, column c: the sheet at angle alpha to
    the scan axis records height Z at column Z / (p sin alpha), and image n
    sits n scan steps along Y."""
    a = math.radians(ALPHA)
    z = c * PIXEL * math.sin(a)
    return n * STEP + z / math.tan(a), z


def _centroid(stack, row):
    """Mass-weighted raw (n, c) centroid of one row of the float32 stack."""
    s = stack[:, row, :].astype(np.float64)
    m = s.sum()
    return (s.sum(1) * np.arange(s.shape[0])).sum() / m, (s.sum(0) * np.arange(s.shape[1])).sum() / m


@pytest.mark.parametrize("theta", [-20.0, 0.0, 15.0, ALPHA, 60.0, 85.0])
def test_spot_lands_at_rotated_coordinate(theta):
    shape = (48, 3, 96)
    st = _spot_stack([(23.3, 1, 47.6, 1000.0)], shape)
    v = oracle.view(st, theta, ALPHA, STEP, PIXEL)
    n_bar, c_bar = _centroid(st, 1)
    y, z = _physical(n_bar, c_bar)
    t = math.radians(theta)
    expect = (y * math.cos(t) + z * math.sin(t)) / PIXEL - v["warp"] * v["origin"]
    row = v["psum"][1]
    got = (row * np.arange(row.size)).sum() / row.sum()
    assert got == pytest.approx(expect, abs=0.05), (theta, got, expect)


def test_line_of_sight_collapses():
    """Two spots at one scan position Y and different heights Z: one view
    column looking down the optical axis, two columns at theta = alpha."""
    shape = (64, 20, 112)
    a = math.radians(ALPHA)
    n1, c1 = 40.0, 30.0
    c2 = 80.0
    n2 = n1 - (c2 - c1) * PIXEL * math.cos(a) / STEP      # same Y
    assert 15 < n2 < 48          # spots stay 5 sigma inside the stack
    st = _spot_stack([(n1, 3, c1, 1000.0), (n2, 16, c2, 1000.0)], shape)
    cen = {}
    for theta in (0.0, ALPHA):
        v = oracle.view(st, theta, ALPHA, STEP, PIXEL)
        cen[theta] = [(v["psum"][r] * np.arange(v["width"])).sum() / v["psum"][r].sum()
                      for r in (3, 16)]
    assert cen[0.0][0] == pytest.approx(cen[0.0][1], abs=0.05)
    assert abs(cen[ALPHA][0] - cen[ALPHA][1]) > 8
