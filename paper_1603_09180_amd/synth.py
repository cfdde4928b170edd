"""Seeded synthetic grayscale images shaped like the paper's workload.

The paper measures on one 512x512 brain MRI and its Deriche-gradient image
(section 5.2, Fig. 1); neither is available, so these generators stand in for
them.  This module holds no part of the thinning method: it only draws images
and workload descriptions, and both the GPU path and the oracle consume what
it returns.

gen_blobs   -- sum of Gaussian blobs plus uniform noise, clipped to 0..255
gen_ridges  -- Gaussian-filtered white noise rescaled to 0..255 with bright
               1-pixel-wide polylines (a gradient-like image with thin crests)
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

U8 = np.uint8
U16 = np.uint16


def _to_dtype(f: np.ndarray, dtype) -> np.ndarray:
    f = np.clip(f, 0.0, 255.0)
    if np.dtype(dtype) == np.uint8:
        return np.rint(f).astype(np.uint8)
    if np.dtype(dtype) == np.uint16:
        return np.rint(f * 257.0).astype(np.uint16)
    raise ValueError(f"unsupported dtype {dtype}")


def gen_blobs(h: int, w: int, seed: int, dtype=U8, nblobs: int = 12,
              sigma=(4.0, 16.0), amplitude=(40.0, 200.0), noise: float = 10.0) -> np.ndarray:
    """Sum of `nblobs` Gaussian blobs + i.i.d. uniform noise in [-noise, noise].

    sigma is a (low, high) range drawn per blob, or one number for a fixed
    width.  Values are computed in float64, clipped to [0, 255], then rounded
    (u8) or rounded after scaling by 257 (u16, so 255 maps to 65535).
    """
    rng = np.random.default_rng(seed)
    f = np.zeros((h, w), np.float64)
    rows = np.arange(h, dtype=np.float64)
    cols = np.arange(w, dtype=np.float64)
    for _ in range(nblobs):
        ci = rng.uniform(0.0, h)
        cj = rng.uniform(0.0, w)
        if isinstance(sigma, (tuple, list)):
            s = rng.uniform(sigma[0], sigma[1])
        else:
            s = float(sigma)
        a = rng.uniform(amplitude[0], amplitude[1])
        gi = np.exp(-((rows - ci) ** 2) / (2.0 * s * s))
        gj = np.exp(-((cols - cj) ** 2) / (2.0 * s * s))
        f += a * np.outer(gi, gj)
    f += rng.uniform(-noise, noise, size=(h, w))
    return _to_dtype(f, dtype)


def _bresenham(r0: int, c0: int, r1: int, c1: int):
    """Integer points of the 8-connected segment from (r0, c0) to (r1, c1)."""
    pts = []
    dr, dc = abs(r1 - r0), abs(c1 - c0)
    sr = 1 if r1 >= r0 else -1
    sc = 1 if c1 >= c0 else -1
    err = dc - dr
    r, c = r0, c0
    while True:
        pts.append((r, c))
        if r == r1 and c == c1:
            break
        e2 = 2 * err
        if e2 > -dr:
            err -= dr
            c += sc
        if e2 < dc:
            err += dc
            r += sr
    return pts


def gen_ridges(h: int, w: int, seed: int, dtype=U8, sigma: float = 4.0,
               npolylines: int = 20) -> np.ndarray:
    """Gaussian-filtered white noise rescaled to 0..255, plus `npolylines`
    1-pixel-wide polylines (3-6 vertices, 8-connected), each written with one
    value drawn from 230..255."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    f = gaussian_filter(rng.standard_normal((h, w)), sigma=sigma)
    lo, hi = float(f.min()), float(f.max())
    f = (f - lo) / (hi - lo) * 255.0 if hi > lo else np.zeros_like(f)
    g = np.rint(f)
    for _ in range(npolylines):
        nv = int(rng.integers(3, 7))
        rs = rng.integers(0, h, size=nv)
        cs = rng.integers(0, w, size=nv)
        val = float(rng.integers(230, 256))
        for k in range(nv - 1):
            for r, c in _bresenham(int(rs[k]), int(cs[k]), int(rs[k + 1]), int(cs[k + 1])):
                g[r, c] = val
    return _to_dtype(g, dtype)


# --------------------------------------------------------------------------
# Workloads.  Adjacency code: 0 = (8,4), 1 = (4,8).


@dataclass
class Job:
    """One image to thin: a seed-reproducible description, materialised on demand."""
    h: int
    w: int
    dtype: type
    lam: int
    adj: int
    seed: int
    kind: str = "blobs"
    sigma: object = (4.0, 16.0)
    arrival: float = 0.0          # seconds from trace start (serving only)
    op: str = "leveling"          # "leveling" or "skeleton"
    front: tuple = None           # (alpha, gain): thin the image's gradient instead

    def image(self) -> np.ndarray:
        if self.kind == "blobs":
            return gen_blobs(self.h, self.w, self.seed, self.dtype, sigma=self.sigma)
        if self.kind == "ridges":
            return gen_ridges(self.h, self.w, self.seed, self.dtype)
        raise ValueError(self.kind)

    @property
    def bytes_per_pixel(self) -> int:
        return np.dtype(self.dtype).itemsize


def blobs_128() -> Job:
    """Single 128x128 u8 blob image, lambda 0, (8,4): the small case."""
    return Job(128, 128, U8, 0, 0, seed=1)


def ridges_512() -> Job:
    """Single 512x512 u8 ridge image, lambda 20, (8,4): the paper-shaped case."""
    return Job(512, 512, U8, 20, 0, seed=2, kind="ridges")


def skeleton_512() -> Job:
    """The 512x512 ridge image under the lambda-skeleton with lambda 10 (the
    value of the paper's filtered-skeleton illustration), (8,4)."""
    return Job(512, 512, U8, 10, 0, seed=2, kind="ridges", op="skeleton")


def gradient_skeleton_512() -> Job:
    """The pipeline of the paper's illustration on a synthetic gray image: the
    512x512 u8 blob image's gradient (alpha 1, gain 12), then its
    lambda-skeleton with lambda 10, (8,4)."""
    return Job(512, 512, U8, 10, 0, seed=6, op="skeleton", front=(1.0, 12.0))


def blobs_8192_u16() -> Job:
    """Single 8192x8192 u16 blob image (sigma fixed at 16), lambda 500, (4,8)."""
    return Job(8192, 8192, U16, 500, 1, seed=3, sigma=16.0)


def batch_512_uneven(n: int = 512, seed: int = 4, lo: int = 64, hi: int = 2048):
    """n u8 blob images, sides log-uniform in [lo, hi] drawn independently,
    lambda drawn from {0, 5, 20, 50}, (8,4); image seeds 4000 + i."""
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        hh = int(np.rint(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        ww = int(np.rint(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        lam = int(rng.choice([0, 5, 20, 50]))
        jobs.append(Job(hh, ww, U8, lam, 0, seed=4000 + i))
    return jobs


def serving_trace(duration_s: float = 10.0, rate: float = 2000.0, seed: int = 5,
                  lo: int = 64, hi: int = 4096):
    """Poisson arrivals at `rate` images/s for `duration_s` seconds: u8 or u16
    with probability 1/2, sides log-uniform in [lo, hi], lambda uniform in
    0..50, (8,4); image seeds 5,000,000 + i."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    i = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration_s:
            break
        dt = U8 if rng.random() < 0.5 else U16
        hh = int(np.rint(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        ww = int(np.rint(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        lam = int(rng.integers(0, 51))
        jobs.append(Job(hh, ww, dt, lam, 0, seed=5_000_000 + i, arrival=t))
        i += 1
    return jobs


def random_small(seed: int, max_side: int = 40, levels: int = 256, dtype=U8):
    """A small random test image: random side lengths (1..max_side), values
    drawn from a few smooth blobs and noise, quantised to `levels` levels."""
    rng = np.random.default_rng(seed)
    h = int(rng.integers(1, max_side + 1))
    w = int(rng.integers(1, max_side + 1))
    f = gen_blobs(h, w, seed + 17, U8, nblobs=int(rng.integers(1, 6)),
                  sigma=(1.0, 6.0), noise=float(rng.uniform(0, 30))).astype(np.int64)
    if levels < 256:
        f = f * levels // 256
    if np.dtype(dtype) == np.uint16:
        f = f * 257 if levels == 256 else f
    return f.astype(dtype)


def gen_blobs_device(h: int, w: int, seed: int, dtype=U8, device="cuda", nblobs: int = 12,
                     sigma=(4.0, 16.0), amplitude=(40.0, 200.0), noise: float = 10.0):
    """gen_blobs's recipe drawn on the GPU, for workloads too large to draw
    on the host (thousands of images up to 4096x4096).

    Blob centres, widths and amplitudes come from the same numpy stream as in
    gen_blobs; the noise comes from torch's generator seeded with `seed`, so
    the pixels differ from gen_blobs(h, w, seed) while the distribution is the
    same.  Returns a 2-D uint8/uint16 tensor on `device`.
    """
    import torch

    rng = np.random.default_rng(seed)
    rows = torch.arange(h, dtype=torch.float64, device=device)
    cols = torch.arange(w, dtype=torch.float64, device=device)
    f = torch.zeros((h, w), dtype=torch.float64, device=device)
    for _ in range(nblobs):
        ci = rng.uniform(0.0, h)
        cj = rng.uniform(0.0, w)
        s = rng.uniform(sigma[0], sigma[1]) if isinstance(sigma, (tuple, list)) else float(sigma)
        a = rng.uniform(amplitude[0], amplitude[1])
        gi = torch.exp(-((rows - ci) ** 2) / (2.0 * s * s))
        gj = torch.exp(-((cols - cj) ** 2) / (2.0 * s * s))
        f += a * torch.outer(gi, gj)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    f += (torch.rand((h, w), dtype=torch.float64, device=device, generator=g) * 2.0 - 1.0) * noise
    f.clamp_(0.0, 255.0)
    if np.dtype(dtype) == np.uint8:
        return torch.round(f).to(torch.uint8)
    if np.dtype(dtype) == np.uint16:
        return torch.round(f * 257.0).to(torch.int32).to(torch.uint16)
    raise ValueError(f"unsupported dtype {dtype}")
