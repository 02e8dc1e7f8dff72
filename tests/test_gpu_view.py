"""Shear-warp rotated views (Fig. 3) on the GPU against the FP64 oracle:
remap with the view's shift, projections, column stretch."""
import numpy as np
import pytest
import torch

import oracle
import paper_2211_00645_amd as dsk
from paper_2211_00645_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ALPHA, STEP, PIXEL = 30.0, 0.4, 0.115


def _close(got, want, rel=2e-5, abs_=1e-6):
    got = np.asarray(got, np.float64)
    err = np.abs(got - want)
    bad = err > rel * np.abs(want) + abs_
    assert not bad.any(), (int(bad.sum()), float(err.max()))


@pytest.fixture(scope="module")
def stack():
    s = synth.blob_stack((64, 128, 256), 50, 0, device=DEV)
    torch.cuda.synchronize()
    return s


@pytest.mark.parametrize("theta", [-20.0, 0.0, 15.0, 45.0, 60.0, 85.0])
def test_view_matches_oracle(stack, theta):
    v = dsk.view(stack, theta, ALPHA, STEP, PIXEL)
    torch.cuda.synchronize()
    o = oracle.view(stack.cpu().numpy(), theta, ALPHA, STEP, PIXEL)
    assert (v["origin"], v["proj_width"], v["width"]) == (o["origin"], o["proj_width"], o["width"])
    _close(v["vsum"].cpu().numpy(), o["psum"])
    _close(v["vmax"].cpu().numpy(), o["pmax"])


def test_view_at_sheet_angle_is_the_plain_projection(stack):
    v = dsk.view(stack, ALPHA, ALPHA, STEP, PIXEL)
    d = dsk.deskew(stack, ALPHA, STEP, PIXEL, vol=False)
    torch.cuda.synchronize()
    assert v["stretch"] == 1.0 and v["width"] == d["width"]
    assert torch.equal(v["vsum"], d["psum"]) and torch.equal(v["vmax"], d["pmax"])


@pytest.mark.parametrize("shape,theta", [((37, 13, 101), 10.0), ((5, 3, 9), -40.0),
                                         ((1, 4, 33), 0.0), ((90, 2, 64), 70.0)])
def test_view_ragged_shapes(shape, theta):
    s = synth.blob_stack(shape, 6, 3, device=DEV)
    v = dsk.view(s, theta, ALPHA, STEP, PIXEL)
    torch.cuda.synchronize()
    o = oracle.view(s.cpu().numpy(), theta, ALPHA, STEP, PIXEL)
    _close(v["vsum"].cpu().numpy(), o["psum"])
    _close(v["vmax"].cpu().numpy(), o["pmax"])


@pytest.mark.parametrize("factor,width", [(0.8660254037844387, None), (0.31, None), (1.0, None),
                                          (0.5, 700), (1.7, 40)])
def test_stretch_matches_oracle(factor, width):
    g = torch.Generator().manual_seed(7)
    p = torch.rand((9, 333), generator=g, dtype=torch.float32) * 1000
    out = dsk.stretch(p.to(DEV), factor, width)
    torch.cuda.synchronize()
    want = oracle.warp(p.numpy().astype(np.float64), factor, out.shape[1])
    if width is None:
        assert out.shape[1] == oracle.view_width(333, factor)
    _close(out.cpu().numpy(), want, rel=1e-6)


def test_view_full_size_sampled_rows():
    """The 512x512x2048 stack viewed down the optical axis: rows sampled
    across the stack against the oracle on those rows (rows are
    independent)."""
    s = synth.blob_stack((512, 512, 2048), 2000, 2, device=DEV)
    v = dsk.view(s, 0.0, 35.0, STEP, PIXEL)
    torch.cuda.synchronize()
    rows = [0, 1, 255, 511]
    sub = np.concatenate([s[:, r:r + 1, :].cpu().numpy() for r in rows], axis=1)
    o = oracle.view(sub, 0.0, 35.0, STEP, PIXEL)
    assert o["width"] == v["width"]
    _close(v["vsum"][rows].cpu().numpy(), o["psum"])
    _close(v["vmax"][rows].cpu().numpy(), o["pmax"])
    del s
