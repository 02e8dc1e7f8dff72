"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no deskew arithmetic: it only draws stacks, batch shapes and
arrival traces.  The paper's own data (live OPM recordings of Vero cells) is
not available, so every workload is a synthetic stand-in with the structure of
a fluorescence stack: a Poisson photon background plus bright Gaussian spots.

Recipe (all draws seeded):
  1. blob centres, continuous U[0,N) x U[0,R) x U[0,C)   (numpy PCG64, seed)
  2. blob amplitudes U[1000, 4000]                        (same generator)
  3. background Poisson(100) per voxel                    (torch generator on
                                                           the target device,
                                                           same seed)
  voxel = clip(round(bg + sum_b A_b exp(-|v - mu_b|^2 / (2 sigma^2))), 0, 65535)
with sigma = 1.5 px in index space, each blob rendered in the voxels within
5 sigma of its centre along every axis.  Float32 stacks are noise-free (no
background, no rounding).
"""
from __future__ import annotations

import math

import numpy as np
import torch

SIGMA = 1.5
BOX_HALF = 8          # voxels on each side of the rounded centre; >= 5 sigma
_BLOB_CHUNK = 4096


def blob_params(shape, n_blobs: int, seed: int):
    """Blob centres (float64 [B,3], index space) and amplitudes ([B])."""
    rng = np.random.default_rng(seed)
    dims = np.asarray(shape, np.float64)
    centres = rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * dims
    amps = rng.uniform(1000.0, 4000.0, size=n_blobs)
    return centres, amps


def _render_blobs(buf: torch.Tensor, centres: np.ndarray, amps: np.ndarray,
                  sigma: float):
    """Add every blob into ``buf`` (float32, [N][R][C]) on its device."""
    n, r, c = buf.shape
    dev = buf.device
    flat = buf.view(-1)
    k = torch.arange(-BOX_HALF, BOX_HALF + 1, device=dev, dtype=torch.float64)
    lim = 5.0 * sigma
    dims = torch.tensor([n, r, c], device=dev, dtype=torch.int64)
    for s in range(0, len(amps), _BLOB_CHUNK):
        mu = torch.as_tensor(centres[s:s + _BLOB_CHUNK], device=dev)
        a = torch.as_tensor(amps[s:s + _BLOB_CHUNK], device=dev)
        base = torch.round(mu)                                   # [B,3]
        idx = base[:, :, None] + k[None, None, :]                # [B,3,K]
        d = idx - mu[:, :, None]
        g = torch.exp(-(d * d) / (2.0 * sigma * sigma))
        ok = (d.abs() <= lim) & (idx >= 0) & (idx < dims[None, :, None])
        g = torch.where(ok, g, torch.zeros_like(g))
        vals = (a[:, None, None, None] * g[:, 0, :, None, None]
                * g[:, 1, None, :, None] * g[:, 2, None, None, :])
        ii = idx.clamp(min=0).to(torch.int64)
        ii = torch.minimum(ii, (dims - 1)[None, :, None])
        lin = ((ii[:, 0, :, None, None] * r + ii[:, 1, None, :, None]) * c
               + ii[:, 2, None, None, :])
        keep = vals != 0
        flat.index_put_((lin[keep],), vals[keep].to(torch.float32),
                        accumulate=True)


def blob_stack(shape, n_blobs: int, seed: int, device="cpu", dtype="u16",
               background: float = 100.0, sigma: float = SIGMA) -> torch.Tensor:
    """A [N][R][C] stack on ``device``: uint16 (Poisson background + blobs,
    rounded and clipped) or float32 (noise-free blobs)."""
    n, r, c = (int(v) for v in shape)
    centres, amps = blob_params((n, r, c), n_blobs, seed)
    dev = torch.device(device)
    if dtype == "u16":
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed)
        buf = torch.empty((n, r, c), dtype=torch.float32, device=dev)
        step = max(1, (1 << 25) // max(1, r * c))
        for p in range(0, n, step):
            q = min(n, p + step)
            lam = torch.full((q - p, r, c), background, dtype=torch.float32,
                             device=dev)
            buf[p:q] = torch.poisson(lam, generator=gen)
            del lam
        _render_blobs(buf, centres, amps, sigma)
        out = torch.empty((n, r, c), dtype=torch.uint16, device=dev)
        for p in range(0, n, 64):
            out[p:p + 64] = buf[p:p + 64].round_().clamp_(0, 65535).to(
                torch.int32).to(torch.uint16)
        del buf
        return out
    if dtype == "f32":
        buf = torch.zeros((n, r, c), dtype=torch.float32, device=dev)
        _render_blobs(buf, centres, amps, sigma)
        return buf
    raise ValueError("dtype must be 'u16' or 'f32'")


def uniform_f32(shape, seed: int, device="cpu") -> torch.Tensor:
    """U[0,1) float32 values (used by the adjoint dot-product test)."""
    gen = torch.Generator(device=torch.device(device))
    gen.manual_seed(seed)
    return torch.rand(tuple(int(v) for v in shape), generator=gen,
                      dtype=torch.float32, device=device)


def blobs_for_volume(n: int, r: int, c: int, per: int = 50,
                     ref=(64, 128, 256)) -> int:
    """Blob count scaled by volume: ``per`` blobs per ``ref`` voxels."""
    return max(1, int(round(per * (n * r * c) / float(np.prod(ref)))))


def ragged_jobs(n_jobs: int = 64, seed: int = 0, pixel_um: float = 0.115,
                scale: float = 1.0):
    """Shapes and geometry of a ragged batch, drawn per job in the order
    (planes, rows, cols, angle, step).  ``scale`` < 1 shrinks every dimension
    (for small test batches) after the draw, so the draw itself is unchanged.
    """
    rng = np.random.default_rng(seed)
    jobs = []
    for _ in range(n_jobs):
        n = int(rng.integers(50, 401))
        r = int(rng.choice([256, 512, 1024]))
        c = int(rng.integers(512, 2049))
        ang = float(rng.choice([30.0, 35.0, 45.0]))
        step = float(rng.uniform(0.2, 0.8))
        if scale != 1.0:
            n = max(1, int(math.ceil(n * scale)))
            r = max(1, int(math.ceil(r * scale)))
            c = max(1, int(math.ceil(c * scale)))
        jobs.append(dict(planes=n, rows=r, cols=c, angle_deg=ang,
                         step_um=step, pixel_um=pixel_um))
    return jobs


def serving_trace(n_requests: int, rate_hz: float, seed: int,
                  planes=(100, 400), rows=(512, 1024), cols=(1024, 2048),
                  channels: int = 2):
    """Poisson arrival times (s) and per-request stack shapes for the live
    serving loop.  Returns a list of dicts with ``t``, ``planes``, ``rows``,
    ``cols`` and ``channels``."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        n = int(rng.integers(planes[0], planes[1] + 1))
        r = int(rng.choice(list(rows)))
        c = int(rng.choice(list(cols)))
        out.append(dict(t=float(t[i]), planes=n, rows=r, cols=c,
                        channels=channels))
    return out
