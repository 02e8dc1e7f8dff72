"""Parity of the HIP forward deskew + projections with the CPU oracle.

Bar: bit-exact where every plane sits at an integer offset; otherwise, per
voxel, |gpu - oracle| <= 1e-5 * (whi*|a| + wlo*|b|) (for uint16 input this
is <= 1e-5 * |oracle|), padding voxels exactly zero, and the FP64-summed
projection within 1e-5 relative.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2211_00645_amd as dsk
from paper_2211_00645_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-5
DEV = "cuda:0"


def _say(msg):
    print(msg, flush=True)


def _to_np(t):
    return t.detach().cpu().numpy()


def _interp_scale(stack, offsets, origin, width, rows=None):
    """Per-voxel magnitude whi*|a| + wlo*|b| (the oracle on |stack|)."""
    return oracle.deskew(np.abs(stack) if stack.dtype != np.uint16 else stack, offsets,
                         origin=origin, width=width, rows=rows)["vol"].astype(np.float64)


def _check_close(gpu, ref, scale, what):
    g = gpu.astype(np.float64)
    r = ref.astype(np.float64)
    err = np.abs(g - r)
    bound = RTOL * scale + 1e-30
    bad = err > bound
    assert not bad.any(), (f"{what}: {bad.sum()} voxels over tolerance, worst "
                           f"{(err / np.maximum(scale, 1e-30)).max():.3e}")


def _check_zero_padding(gpu_vol, ref_vol, what):
    z = ref_vol == 0
    assert (gpu_vol[z] == 0).all(), f"{what}: nonzero where the oracle has padding"


@pytest.fixture(scope="module")
def cfg1():
    s = synth.blob_stack((64, 128, 256), 50, 0)
    return s, s.numpy()


def test_config1_integer_shift_bit_exact(cfg1):
    st, sn = cfg1
    _say("forward: config 1, integer shift 3 px/plane")
    off = np.arange(64, dtype=np.float64) * 3.0
    ref = oracle.deskew(sn, off)
    out = dsk.deskew(st.to(DEV), offsets=off)
    torch.cuda.synchronize()
    assert (out["origin"], out["width"]) == (ref["origin"], ref["width"]) == (0, 445)
    assert _to_np(out["vol"]).tobytes() == ref["vol"].tobytes()
    assert _to_np(out["psum"]).tobytes() == ref["psum"].tobytes()
    assert _to_np(out["pmax"]).tobytes() == ref["pmax"].tobytes()


def test_config1_fractional(cfg1):
    st, sn = cfg1
    _say("forward: config 1, 30 deg, 0.4 um, 0.115 um")
    s = oracle.shift_px(30.0, 0.4, 0.115)
    off = oracle.offsets_uniform(64, s)
    ref = oracle.deskew(sn, off)
    out = dsk.deskew(st.to(DEV), 30.0, 0.4, 0.115)
    torch.cuda.synchronize()
    assert (out["origin"], out["width"]) == (ref["origin"], ref["width"]) == (0, 446)
    v = _to_np(out["vol"])
    _check_close(v, ref["vol"], np.abs(ref["vol"]).astype(np.float64), "vol")
    _check_zero_padding(v, ref["vol"], "vol")
    _check_close(_to_np(out["psum"]), ref["psum"], np.abs(ref["psum"]).astype(np.float64),
                 "psum")
    _check_close(_to_np(out["pmax"]), ref["pmax"], np.abs(ref["pmax"]).astype(np.float64),
                 "pmax")


TUNES = [dict(block=b, per_thread=j, nt_store=nt, unroll=u)
         for b in (64, 128, 256) for j in (1, 2, 4, 8) for nt in (0, 1) for u in (1, 2, 4)
         if not (j < 4 and u > 1)]
# plane pacing only delays wavefronts: slow, default and never-binding paces
TUNES += [dict(block=b, per_thread=j, nt_store=1, unroll=4, pace_gbs=p)
          for b in (64, 256) for j in (4, 8) for p in (500, 6000, 100000)]


def test_every_launch_shape_is_bitwise_identical(cfg1):
    st, _ = cfg1
    _say("forward: launch shapes")
    x = st.to(DEV)
    off = oracle.offsets_uniform(64, oracle.shift_px(30.0, 0.4, 0.115))
    base = dsk.deskew(x, offsets=off)
    for t in TUNES:
        o = dsk.deskew(x, offsets=off, tune=t)
        for k in ("vol", "psum", "pmax"):
            assert torch.equal(o[k], base[k]), (t, k)
        # the projections-only pass (its own loop) gives the same projections
        p = dsk.deskew(x, offsets=off, tune=t, vol=False)
        for k in ("psum", "pmax"):
            assert torch.equal(p[k], base[k]), (t, k, "projections only")
    # the uniform-scan path (offsets computed on the device) matches too
    o = dsk.deskew(x, 30.0, 0.4, 0.115)
    for k in ("vol", "psum", "pmax"):
        assert torch.equal(o[k], base[k]), k


def test_misaligned_buffers_match_aligned(cfg1):
    """Stacks and volumes that are not 16-byte aligned take the scalar kernel;
    results are bitwise those of the aligned vector kernel."""
    st, _ = cfg1
    x = st.to(DEV)
    off = oracle.offsets_uniform(64, oracle.shift_px(30.0, 0.4, 0.115))
    base = dsk.deskew(x, offsets=off)
    flat = torch.empty(x.numel() + 1, dtype=torch.uint16, device=DEV)
    xm = flat[1:].view(x.shape)
    xm.copy_(x)
    assert xm.data_ptr() % 16 != 0
    w = base["width"]
    vflat = torch.empty(64 * 128 * w + 1, dtype=torch.float32, device=DEV)
    vm = vflat[1:].view(64, 128, w)
    o = dsk.deskew(xm, offsets=off, out={"vol": vm})
    for k in ("psum", "pmax"):
        assert torch.equal(o[k], base[k]), k
    assert torch.equal(vm, base["vol"])


@pytest.mark.parametrize("width,lead", [(1256, 0), (1272, 0), (1276, 0), (1280, 0), (1280, 4),
                                        (1112, 12)])
def test_aligned_tile_grids_match_the_scalar_kernel(width, lead):
    """Frames with rows*W a multiple of 32, where the vector kernel starts
    each row's tiles on a 128-byte boundary of the volume if the shifted
    grids fit the row's tiles: they fit for 1256 (shifts 0-6 groups, 58 + 6
    of the last tile's 64), 1280 on a boundary (no shift) and 1112 twelve
    floats after one (shifts up to 7, 22 + 7 of 64); they do not for 1272,
    1276 and 1280 four floats after a boundary (shift 1, 64 + 1), which keep
    the plain grid.  Each is bitwise the scalar kernel's result (a volume 4
    bytes off alignment)."""
    shape = (8, 32, 1024)
    _say(f"forward: aligned tile grids W {width} lead {lead}")
    st = synth.blob_stack(shape, synth.blobs_for_volume(*shape), 23)
    g = st.to(DEV)
    n, r = shape[0], shape[1]
    vflat = torch.full((n * r * width + 16,), -1.0, device=DEV)
    assert vflat.data_ptr() % 128 == 0
    va = vflat[lead:lead + n * r * width].view(n, r, width)
    sflat = torch.full((n * r * width + 1,), -1.0, device=DEV)
    vs = sflat[1:].view(n, r, width)
    a = dsk.deskew(g, 35.0, 0.4, 0.115, width=width, out={"vol": va})
    b = dsk.deskew(g, 35.0, 0.4, 0.115, width=width, out={"vol": vs})
    torch.cuda.synchronize()
    assert torch.equal(va, vs)
    for k in ("psum", "pmax"):
        assert torch.equal(a[k], b[k]), k


def test_determinism(cfg1):
    st, _ = cfg1
    x = st.to(DEV)
    a = dsk.deskew(x, 35.0, 0.4, 0.115)
    b = dsk.deskew(x, 35.0, 0.4, 0.115)
    for k in ("vol", "psum", "pmax"):
        assert torch.equal(a[k], b[k])


RAGGED = [
    # (planes, rows, cols, offsets kind, seed)
    (1, 1, 1, "frac", 1),
    (1, 3, 17, "frac", 2),
    (7, 5, 33, "neg", 3),
    (13, 9, 257, "frac", 4),
    (33, 7, 513, "jitter", 5),
    (5, 3, 1000, "int", 6),
    (64, 4, 64, "big", 7),         # W = 64 + 63*40 = 2584: many tiles, mostly padding
    (3, 2, 5, "zero", 8),
    (4, 4, 7, "frac", 9),          # rows*cols % 4 == 0, W odd
    (9, 12, 300, "neg", 10),       # vector kernel with negative offsets
    (2, 2, 2, "frac", 11),         # tiny stack: scalar kernel
    (150, 6, 400, "shuffle", 12),  # offsets out of order: padding planes between others
    (200, 8, 300, "frac", 13),     # several 64-plane chunks, partial last chunk
    # stack-end planes in the vector kernel: one plane holding both the
    # first and the last rows, a last chunk of one plane, and a last chunk
    # of one plane after two full ones with negative offsets
    (1, 4, 64, "frac", 14),
    (65, 4, 64, "frac", 15),
    (129, 4, 96, "neg", 16),
]


# projections-only shapes beside the default: two groups per lane side by
# side (one walk over the union of their plane ranges), paced, and a
# 256-thread workgroup
PROJ_TUNES = [dict(block=64, per_thread=8, nt_store=1, unroll=2),
              dict(block=256, per_thread=8, nt_store=1, unroll=4, pace_gbs=9000),
              dict(block=64, per_thread=4, nt_store=1, unroll=4, pace_gbs=9000)]


def _offsets(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == "frac":
        return oracle.offsets_uniform(n, 2.718281828)
    if kind == "neg":
        return oracle.offsets_uniform(n, -1.4142135)
    if kind == "jitter":
        return np.cumsum(np.r_[0.0, rng.uniform(0.5, 3.5, n - 1)])
    if kind == "int":
        return np.arange(n, dtype=np.float64) * -7.0
    if kind == "big":
        return oracle.offsets_uniform(n, 40.0)
    if kind == "zero":
        return np.zeros(n)
    if kind == "shuffle":
        return rng.permutation(n).astype(np.float64) * 5.3 + rng.uniform(0, 1, n)
    raise ValueError(kind)


@pytest.mark.parametrize("n,r,c,kind,seed", RAGGED)
@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_ragged_shapes(n, r, c, kind, seed, dtype):
    _say(f"forward: ragged {n}x{r}x{c} {kind} {dtype}")
    if dtype == "u16":
        st = synth.blob_stack((n, r, c), max(1, n * r * c // 20000), seed)
    else:
        st = synth.blob_stack((n, r, c), max(1, n * r * c // 20000), seed, dtype="f32")
        st = st - 0.25 * st.mean()          # signed values
    sn = st.numpy()
    off = _offsets(kind, n, seed)
    ref = oracle.deskew(sn, off)
    out = dsk.deskew(st.to(DEV), offsets=off)
    proj = dsk.deskew(st.to(DEV), offsets=off, vol=False)
    torch.cuda.synchronize()
    assert (out["origin"], out["width"]) == (ref["origin"], ref["width"])
    for k in ("psum", "pmax"):
        assert torch.equal(proj[k], out[k]), f"projections-only {k}"
    for t in PROJ_TUNES:
        p2 = dsk.deskew(st.to(DEV), offsets=off, vol=False, tune=t)
        for k in ("psum", "pmax"):
            assert torch.equal(p2[k], out[k]), (t, k)
    v = _to_np(out["vol"])
    if kind in ("int", "zero"):
        assert v.tobytes() == ref["vol"].tobytes()
        assert _to_np(out["psum"]).tobytes() == ref["psum"].tobytes()
        assert _to_np(out["pmax"]).tobytes() == ref["pmax"].tobytes()
        return
    scale = _interp_scale(sn, off, ref["origin"], ref["width"])
    _check_close(v, ref["vol"], scale, "vol")
    _check_zero_padding(v, ref["vol"], "vol")
    pscale = scale.sum(0)
    _check_close(_to_np(out["psum"]), ref["psum"], pscale, "psum")
    _check_close(_to_np(out["pmax"]), ref["pmax"], scale.max(0), "pmax")


def test_clipped_and_padded_width_and_projection_only(cfg1):
    st, sn = cfg1
    x = st.to(DEV)
    off = oracle.offsets_uniform(64, oracle.shift_px(30.0, 0.4, 0.115))
    for w in (300, 446, 500):
        ref = oracle.deskew(sn, off, origin=0, width=w)
        out = dsk.deskew(x, offsets=off, origin=0, width=w)
        torch.cuda.synchronize()
        _check_close(_to_np(out["vol"]), ref["vol"], np.abs(ref["vol"]).astype(np.float64),
                     f"vol w={w}")
        _check_zero_padding(_to_np(out["vol"]), ref["vol"], f"vol w={w}")
    full = dsk.deskew(x, offsets=off)
    proj = dsk.deskew(x, offsets=off, vol=False)
    assert "vol" not in proj
    assert torch.equal(proj["psum"], full["psum"]) and torch.equal(proj["pmax"], full["pmax"])
    vol_only = dsk.deskew(x, offsets=off, psum=False, pmax=False)
    assert torch.equal(vol_only["vol"], full["vol"])


def test_live_scale_config2_sampled_rows():
    """512 x 512 x 2048 uint16 at 35 deg: every output of sampled rows, in the
    launch configuration the benchmark times (the tuner's shape for this
    frame), and the whole result bitwise equal to the default shape's."""
    _say("forward: config 2 (512x512x2048), generating")
    st = synth.blob_stack((512, 512, 2048), 2000, 2, device=DEV)
    torch.cuda.synchronize()
    _say("forward: config 2 deskew, tuned shape")
    out = dsk.deskew(st, 35.0, 0.4, 0.115, tune="auto")
    torch.cuda.synchronize()
    assert out["width"] == 3504 and out["origin"] == 0
    _say("forward: config 2 deskew, default shape")
    dflt = dsk.deskew(st, 35.0, 0.4, 0.115)
    torch.cuda.synchronize()
    for k in ("vol", "psum", "pmax"):
        assert torch.equal(out[k], dflt[k]), k
    del dflt
    _say("forward: config 2 projections only")
    proj = dsk.deskew(st, 35.0, 0.4, 0.115, vol=False)
    torch.cuda.synchronize()
    for k in ("psum", "pmax"):
        assert torch.equal(proj[k], out[k]), f"projections-only {k}"
    del proj
    torch.cuda.empty_cache()
    rows = [0, 1, 137, 255, 256, 400, 511]
    sn = st.cpu().numpy()
    off = oracle.offsets_uniform(512, oracle.shift_px(35.0, 0.4, 0.115))
    vol = out["vol"]
    for r in rows:
        _say(f"forward: config 2 row {r}")
        ref = oracle.deskew(sn, off, rows=(r, r + 1))
        g = _to_np(vol[:, r:r + 1, :])
        _check_close(g, ref["vol"], np.abs(ref["vol"]).astype(np.float64), f"vol row {r}")
        _check_zero_padding(g, ref["vol"], f"vol row {r}")
        _check_close(_to_np(out["psum"][r:r + 1]), ref["psum"],
                     np.abs(ref["psum"]).astype(np.float64), f"psum row {r}")
        _check_close(_to_np(out["pmax"][r:r + 1]), ref["pmax"],
                     np.abs(ref["pmax"]).astype(np.float64), f"pmax row {r}")
    # integral property over the whole stack: sum of Psum == sum of the stack
    tot_in = float(st.to(torch.int64).sum())
    tot_out = float(out["psum"].double().sum())
    assert tot_out == pytest.approx(tot_in, rel=1e-6)


@pytest.mark.parametrize("step", [0.0, 0.4])
def test_signed_stack_maximum(step):
    """Float32 stack of negative values: with zero shift there is no
    padding, so the maximum projection is the largest (negative) value;
    with a shift, columns that some image does not cover get the padding's
    0.  Both passes agree with the oracle."""
    n, r, c = 70, 5, 96
    st = -1.0 - synth.blob_stack((n, r, c), 8, 14, dtype="f32")
    off = oracle.offsets_uniform(n, oracle.shift_px(35.0, step, 0.115))
    ref = oracle.deskew(st.numpy(), off)
    for vol, tune in ((True, None), (False, None), (False, PROJ_TUNES[0])):
        out = dsk.deskew(st.to(DEV), offsets=off, vol=vol, tune=tune)
        torch.cuda.synchronize()
        pm = _to_np(out["pmax"])
        _check_close(pm, ref["pmax"], np.abs(ref["pmax"]).astype(np.float64),
                     f"pmax vol={vol} tune={tune}")
        if step == 0.0:
            assert (pm < 0).all()


def test_invalid_arguments_raise():
    x = torch.zeros((4, 2, 8), dtype=torch.uint16, device=DEV)
    with pytest.raises(ValueError):
        dsk.deskew(x.cpu(), 30.0, 0.4, 0.115)
    with pytest.raises(Exception):
        dsk.deskew(x, 30.0, 0.4, -1.0)
    with pytest.raises(ValueError):
        dsk.deskew(x.transpose(1, 2), 30.0, 0.4, 0.115)


def test_row_bands_of_a_frame_wider_than_the_resident_tiles():
    """1028 rows x 9 column tiles (W = 2091, edge columns) exceed the
    workgroups an MI355X holds at once (8192 in the default shape), so the
    paced default launch goes out as two bands of rows (516 + 512).  The
    result equals, bit for bit, the unpaced launch of the whole frame at once,
    and the oracle within the forward's bar."""
    shape = (16, 1028, 2048)
    _say(f"forward: row bands {shape}")
    st = synth.blob_stack(shape, synth.blobs_for_volume(*shape), 21)
    s = oracle.shift_px(35.0, 0.4, 0.115)
    off = oracle.offsets_uniform(shape[0], s)
    g = st.to(DEV)
    banded = dsk.deskew(g, 35.0, 0.4, 0.115)
    whole = dsk.deskew(g, 35.0, 0.4, 0.115,
                       tune={"block": 64, "per_thread": 4, "nt_store": 1, "unroll": 2,
                             "wg_per_cu": 0, "pace_gbs": 0})
    torch.cuda.synchronize()
    assert banded["width"] == 2091
    for k in ("vol", "psum", "pmax"):
        assert torch.equal(banded[k], whole[k]), k
    sn = st.numpy()
    ref = oracle.deskew(sn, off)
    assert (banded["origin"], banded["width"]) == (ref["origin"], ref["width"])
    vol = _to_np(banded["vol"])
    _check_close(vol, ref["vol"], _interp_scale(sn, off, ref["origin"], ref["width"]), "vol")
    _check_zero_padding(vol, ref["vol"], "vol")
    for k in ("psum", "pmax"):
        r = ref[k].astype(np.float64)
        assert (np.abs(_to_np(banded[k]).astype(np.float64) - r) <= RTOL * np.abs(r)).all(), k


def test_row_bands_float32():
    """The float32 path through the same row bands (1028 rows x 9 column
    tiles, W = 2091): bitwise the unpaced whole-frame launch, and the
    oracle within the forward's bar on the projections."""
    shape = (16, 1028, 2048)
    _say(f"forward: row bands, float32 {shape}")
    st = synth.blob_stack(shape, synth.blobs_for_volume(*shape), 22).to(torch.float32)
    g = st.to(DEV)
    banded = dsk.deskew(g, 35.0, 0.4, 0.115)
    whole = dsk.deskew(g, 35.0, 0.4, 0.115,
                       tune={"block": 64, "per_thread": 4, "nt_store": 1, "unroll": 2,
                             "wg_per_cu": 0, "pace_gbs": 0})
    torch.cuda.synchronize()
    assert banded["width"] == 2091
    for k in ("vol", "psum", "pmax"):
        assert torch.equal(banded[k], whole[k]), k
    off = oracle.offsets_uniform(shape[0], oracle.shift_px(35.0, 0.4, 0.115))
    ref = oracle.deskew(st.numpy(), off)
    for k in ("psum", "pmax"):
        r = ref[k].astype(np.float64)
        assert (np.abs(_to_np(banded[k]).astype(np.float64) - r) <= RTOL * np.abs(r)).all(), k


def test_projections_only_wider_than_the_resident_tiles():
    """Without a volume (the live view) a frame whose tiles do not all fit at
    once (1028 rows x 9 tiles) is launched unpaced even in the paced default
    shape: projections bitwise those of the explicitly unpaced launch and of
    the fused pass with the volume (which goes out as row bands)."""
    shape = (16, 1028, 2048)
    _say(f"forward: projections only, more tiles than resident {shape}")
    g = synth.blob_stack(shape, synth.blobs_for_volume(*shape), 23, device=DEV)
    banded = dsk.deskew(g, 35.0, 0.4, 0.115, vol=False)
    whole = dsk.deskew(g, 35.0, 0.4, 0.115, vol=False,
                       tune={"block": 64, "per_thread": 4, "nt_store": 1, "unroll": 4,
                             "wg_per_cu": 0, "pace_gbs": 0})
    full = dsk.deskew(g, 35.0, 0.4, 0.115)
    torch.cuda.synchronize()
    for k in ("psum", "pmax"):
        assert torch.equal(banded[k], whole[k]), k
        assert torch.equal(banded[k], full[k]), k
