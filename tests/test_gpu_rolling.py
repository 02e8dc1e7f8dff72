"""Rolling display mode: after every image the projections equal those of
the stack made of the latest image at every index."""
import numpy as np
import pytest
import torch

import oracle
import paper_2211_00645_amd as dsk
from paper_2211_00645_amd import synth
from paper_2211_00645_amd.rolling import RollingView

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _fwd(stack, shift):
    n = stack.shape[0]
    return dsk.deskew(stack, offsets=np.arange(n) * shift)


@pytest.mark.parametrize("shape", [(64, 128, 256), (13, 7, 61)])   # 7 x W odd: one pixel per thread
def test_in_order_equals_forward_bitwise(shape):
    n_img = shape[0]
    st = synth.blob_stack(shape, 50, 0).to(DEV)
    rv = RollingView(*shape, 30.0, 0.4, 0.115)
    for n in range(n_img):
        rv.update(n, st[n])
    ref = dsk.deskew(st, 30.0, 0.4, 0.115)
    torch.cuda.synchronize()
    assert torch.equal(rv.vol, ref["vol"])
    assert torch.equal(rv.pmax, ref["pmax"])
    assert torch.equal(rv.psum, ref["psum"])


def test_replacements_and_random_order_match_oracle():
    a = synth.blob_stack((40, 48, 200), 30, 1).to(DEV)
    b = synth.blob_stack((40, 48, 200), 30, 2).to(DEV)
    rv = RollingView(40, 48, 200, 35.0, 0.4, 0.115)
    rng = np.random.default_rng(5)
    for n in rng.permutation(40):
        rv.update(int(n), a[int(n)])
    cur = a.clone()
    for n in (5, 17, 39, 5, 0):
        src = b if n != 0 else a
        rv.update(n, src[n])
        cur[n] = src[n]
    torch.cuda.synchronize()
    ref = dsk.deskew(cur, 35.0, 0.4, 0.115)
    assert torch.equal(rv.vol, ref["vol"])
    assert torch.equal(rv.pmax, ref["pmax"])
    torch.testing.assert_close(rv.psum, ref["psum"], rtol=1e-6, atol=0)
    o = oracle.deskew(cur.cpu().numpy(), oracle.offsets_uniform(40, oracle.shift_px(35.0, 0.4, 0.115)))
    g = rv.psum.cpu().numpy().astype(np.float64)
    assert (np.abs(g - o["psum"]) <= 1e-5 * np.abs(o["psum"])).all()
    g = rv.pmax.cpu().numpy().astype(np.float64)
    assert (np.abs(g - o["pmax"]) <= 1e-5 * np.abs(o["pmax"])).all()


@pytest.mark.parametrize("n", [1, 2, 3, 50])
def test_paper_display_shape(n):
    """The paper's live-view region: 1304 x 87 px images spread over a
    3652-px display (for 50 images); odd image counts exercise the tree."""
    shift = (3652 - 87) / 49
    st = synth.blob_stack((n, 1304, 87), 20, 3).to(DEV)
    rv = RollingView(n, 1304, 87, shift_px=shift)
    if n == 50:
        assert rv.width == 3652
    for i in range(n):
        rv.update(i, st[i])
    ref = _fwd(st, shift)
    torch.cuda.synchronize()
    assert torch.equal(rv.pmax, ref["pmax"]) and torch.equal(rv.psum, ref["psum"])
    rv.reset()
    torch.cuda.synchronize()
    assert not rv.pmax.any() and not rv.vol.any()


def test_full_stack_512x512x2048():
    """The benchmark stack's shape, updated image by image in order and then
    with a few images replaced: bitwise the fused deskew of the stack the
    display holds (the running FP64 sum of an in-order build equals the
    plane-ordered sum)."""
    st = synth.blob_stack((512, 512, 2048), 2000, 2, device=DEV)
    rv = RollingView(512, 512, 2048, 35.0, 0.4, 0.115)
    for n in range(512):
        rv.update(n, st[n])
    ref = dsk.deskew(st, 35.0, 0.4, 0.115)
    torch.cuda.synchronize()
    assert rv.width == ref["width"] == 3504
    assert torch.equal(rv.vol, ref["vol"])
    assert torch.equal(rv.pmax, ref["pmax"])
    assert torch.equal(rv.psum, ref["psum"])
    del ref
    # replace three images by other ones
    alt = synth.blob_stack((3, 512, 2048), 40, 9, device=DEV)
    cur = st.clone()
    for i, n in enumerate((0, 255, 511)):
        rv.update(n, alt[i])
        cur[n] = alt[i]
    ref = dsk.deskew(cur, 35.0, 0.4, 0.115)
    torch.cuda.synchronize()
    assert torch.equal(rv.vol, ref["vol"])
    assert torch.equal(rv.pmax, ref["pmax"])
    torch.testing.assert_close(rv.psum, ref["psum"], rtol=1e-6, atol=0)
