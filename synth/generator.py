"""Seeded generator of synthetic frames and block-loss patterns.

The paper measures on natural images and coded video that are not available
here; these planes stand in for them.  Every draw comes from one
``numpy.random.default_rng(seed)`` in a fixed order, so a (workload, seed)
pair always yields the same arrays.

Luma model (all terms added in float64, then rounded and clipped to uint8):

* smooth field: a sum of Gaussian bumps (amplitude U[20, 120], centre uniform
  over the frame, isotropic std U[0.02, 0.06] * min(H, W)), shifted so that
  its mean is 128;
* straight step edges: contrast +-U[30, 90], a line through a uniform point
  at angle U[0, pi), +c/2 on one side and -c/2 on the other, confined to a
  disc of radius U[0.1, 0.3] * min(H, W) around that point (a full-plane step
  clips a large part of the frame to 0 or 255; ``full_plane_edges`` keeps the
  literal variant available);
* optional band-limited texture: white noise smoothed by a Gaussian of
  std 1.5 px, scaled to std 8, applied where a second bump field exceeds its
  70th percentile (30 % of the area);
* Gaussian noise of std 2, then floor(v + 0.5) and clipping to [0, 255].

Loss masks are uint8 planes, 1 = lost pixel, built from whole B x B cells of
the block grid that lie completely inside the frame.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "seed_for", "make_luma", "make_chroma", "loss_isolated", "loss_dispersed",
    "loss_random", "loss_slices", "loss_random_bursts", "workload_plain_512",
    "workload_layered_1080p", "workload_batch", "workload_stream_4k",
]


def seed_for(workload: int, frame: int = 0) -> int:
    """Seed of frame ``frame`` of workload number ``workload`` (1..5)."""
    return 1000 * int(workload) + int(frame)


def _gauss1d(n: int, c: float, s: float) -> np.ndarray:
    t = (np.arange(n, dtype=np.float64) - c) / s
    return np.exp(-0.5 * t * t)


def _bump_field(rng, h: int, w: int, n: int, amp=(20.0, 120.0), rel_sigma=(0.02, 0.06)):
    m = float(min(h, w))
    f = np.zeros((h, w), dtype=np.float64)
    for _ in range(n):
        a = rng.uniform(*amp)
        cx = rng.uniform(0.0, w)
        cy = rng.uniform(0.0, h)
        s = rng.uniform(*rel_sigma) * m
        f += a * np.outer(_gauss1d(h, cy, s), _gauss1d(w, cx, s))
    return f


def _smooth(noise: np.ndarray, sigma: float) -> np.ndarray:
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(noise, sigma=sigma, mode="reflect")


def make_luma(h: int, w: int, seed: int, n_bumps: int = 40, n_edges: int = 12,
              texture: bool = False, noise_std: float = 2.0,
              full_plane_edges: bool = False) -> np.ndarray:
    """Synthetic 8-bit luma plane of shape (h, w)."""
    rng = np.random.default_rng(seed)
    m = float(min(h, w))
    f = _bump_field(rng, h, w, n_bumps)
    f += 128.0 - f.mean()
    yy = np.arange(h, dtype=np.float64)[:, None]
    xx = np.arange(w, dtype=np.float64)[None, :]
    for _ in range(n_edges):
        px = rng.uniform(0.0, w)
        py = rng.uniform(0.0, h)
        th = rng.uniform(0.0, np.pi)
        sign = 1.0 if rng.uniform() < 0.5 else -1.0
        c = sign * rng.uniform(30.0, 90.0)
        rad = rng.uniform(0.1, 0.3) * m
        side = (xx - px) * np.sin(th) - (yy - py) * np.cos(th)
        step = np.where(side >= 0.0, 0.5 * c, -0.5 * c)
        if not full_plane_edges:
            step = np.where((xx - px) ** 2 + (yy - py) ** 2 <= rad * rad, step, 0.0)
        f += step
    if texture:
        tex = _smooth(rng.standard_normal((h, w)), 1.5)
        tex *= 8.0 / max(tex.std(), 1e-12)
        sel = _bump_field(rng, h, w, max(8, n_bumps // 4))
        f += np.where(sel > np.percentile(sel, 70.0), tex, 0.0)
    f += rng.normal(0.0, noise_std, size=(h, w))
    return np.clip(np.floor(f + 0.5), 0, 255).astype(np.uint8)


def make_chroma(h: int, w: int, seed: int, n_bumps: int = 24) -> np.ndarray:
    """Smooth chroma plane (bump field around 128 plus std-1 noise)."""
    rng = np.random.default_rng(seed)
    f = _bump_field(rng, h, w, n_bumps, amp=(10.0, 40.0), rel_sigma=(0.04, 0.12))
    f += 128.0 - f.mean()
    f += rng.normal(0.0, 1.0, size=(h, w))
    return np.clip(np.floor(f + 0.5), 0, 255).astype(np.uint8)


def _grid(h: int, w: int, b: int):
    return h // b, w // b  # full cells only


def _mask_from_cells(h: int, w: int, b: int, cells) -> np.ndarray:
    mask = np.zeros((h, w), dtype=np.uint8)
    for by, bx in cells:
        mask[by * b:(by + 1) * b, bx * b:(bx + 1) * b] = 1
    return mask


def loss_isolated(h: int, w: int, b: int, count: int, seed: int, min_cheb: int = 2,
                  max_tries: int = 200000) -> np.ndarray:
    """``count`` lost cells, pairwise Chebyshev cell distance >= ``min_cheb``."""
    rng = np.random.default_rng(seed)
    gh, gw = _grid(h, w, b)
    taken = np.zeros((gh, gw), dtype=bool)
    cells = []
    tries = 0
    while len(cells) < count and tries < max_tries:
        tries += 1
        by = int(rng.integers(0, gh))
        bx = int(rng.integers(0, gw))
        y0, y1 = max(0, by - min_cheb + 1), min(gh, by + min_cheb)
        x0, x1 = max(0, bx - min_cheb + 1), min(gw, bx + min_cheb)
        if taken[y0:y1, x0:x1].any():
            continue
        taken[by, bx] = True
        cells.append((by, bx))
    return _mask_from_cells(h, w, b, cells)


def loss_dispersed(h: int, w: int, b: int, ox: int = 0, oy: int = 0) -> np.ndarray:
    """Checkerboard lattice: cell (by, bx) lost iff bx = ox and by = oy (mod 2).

    Exactly 25 % of the full cells; every lost cell has its 8 neighbours
    received.
    """
    gh, gw = _grid(h, w, b)
    cells = [(by, bx) for by in range(gh) for bx in range(gw)
             if by % 2 == oy % 2 and bx % 2 == ox % 2]
    return _mask_from_cells(h, w, b, cells)


def loss_random(h: int, w: int, b: int, rate: float, seed: int) -> np.ndarray:
    """Each full cell lost independently with probability ``rate``."""
    rng = np.random.default_rng(seed)
    gh, gw = _grid(h, w, b)
    lost = rng.uniform(size=(gh, gw)) < rate
    return _mask_from_cells(h, w, b, list(zip(*np.nonzero(lost))))


def loss_partial_cells(h: int, w: int, b: int, rate: float, seed: int,
                       frac: float = 0.5) -> np.ndarray:
    """Arbitrary-shape loss: each full cell is hit with probability ``rate``;
    a share ``frac`` of the hit cells lose a random subset of their pixels
    (each pixel with a per-cell probability in [0.3, 0.9), at least one),
    the others lose every pixel."""
    rng = np.random.default_rng(seed)
    gh, gw = _grid(h, w, b)
    m = np.zeros((h, w), dtype=np.uint8)
    for by in range(gh):
        for bx in range(gw):
            if rng.uniform() < rate:
                c = np.ones((b, b), dtype=np.uint8)
                if rng.uniform() < frac:
                    c = (rng.uniform(size=(b, b)) < rng.uniform(0.3, 0.9)).astype(np.uint8)
                    c[rng.integers(b), rng.integers(b)] = 1
                m[by * b:(by + 1) * b, bx * b:(bx + 1) * b] = c
    return m


def loss_slices(h: int, w: int, b: int, rate: float, seed: int) -> np.ndarray:
    """Whole rows of cells lost; round(rate * rows) distinct rows, uniform."""
    rng = np.random.default_rng(seed)
    gh, gw = _grid(h, w, b)
    n = max(1, min(gh - 1, int(round(rate * gh))))
    rows = sorted(int(r) for r in rng.choice(gh, size=n, replace=False))
    return _mask_from_cells(h, w, b, [(by, bx) for by in rows for bx in range(gw)])


def loss_random_bursts(h: int, w: int, b: int, rate: float, seed: int,
                       max_burst: int = 4) -> np.ndarray:
    """Random horizontal bursts of 1..max_burst cells until ``rate`` is reached."""
    rng = np.random.default_rng(seed)
    gh, gw = _grid(h, w, b)
    lost = np.zeros((gh, gw), dtype=bool)
    target = int(round(rate * gh * gw))
    while lost.sum() < target:
        by = int(rng.integers(0, gh))
        bx = int(rng.integers(0, gw))
        n = int(rng.integers(1, max_burst + 1))
        lost[by, bx:min(gw, bx + n)] = True
    return _mask_from_cells(h, w, b, list(zip(*np.nonzero(lost))))


# ---------------------------------------------------------------- workloads

def workload_plain_512(seed: int | None = None):
    """512 x 512 luma, 40 bumps + 12 edges + noise, 64 isolated 16 x 16 cells."""
    s = seed_for(1) if seed is None else seed
    frame = make_luma(512, 512, s, n_bumps=40, n_edges=12)
    mask = loss_isolated(512, 512, 16, 64, s + 500)
    return frame, mask


def workload_layered_1080p(seed: int | None = None):
    """1920 x 1080 luma (150 bumps, 40 edges, texture), 25 % dispersed lattice."""
    s = seed_for(2) if seed is None else seed
    frame = make_luma(1080, 1920, s, n_bumps=150, n_edges=40, texture=True)
    mask = loss_dispersed(1080, 1920, 16)
    return frame, mask


def workload_batch(n_frames: int = 64, seed: int | None = None, sizes=None):
    """Mixed batch: 24 x 720p, 32 x 1080p, 8 x 2160p (by default).

    Per frame the seed picks the cell size (8 or 16) and either scattered cell
    loss at 10-30 % or slice loss at 5-50 %.  Returns a list of dicts with
    ``frame``, ``mask``, ``block`` and ``kind``.
    """
    base = seed_for(3) if seed is None else seed
    if sizes is None:
        sizes = [(720, 1280)] * 24 + [(1080, 1920)] * 32 + [(2160, 3840)] * 8
    sizes = list(sizes)[:n_frames]
    out = []
    for f, (h, w) in enumerate(sizes):
        s = base + f
        rng = np.random.default_rng(s + 777)
        b = 8 if rng.uniform() < 0.5 else 16
        if rng.uniform() < 0.5:
            kind = "scattered"
            mask = loss_random(h, w, b, rng.uniform(0.10, 0.30), s + 500)
        else:
            kind = "slices"
            mask = loss_slices(h, w, b, rng.uniform(0.05, 0.50), s + 500)
        big = h * w >= 1920 * 1080
        frame = make_luma(h, w, s, n_bumps=150 if big else 40, n_edges=40 if big else 12,
                          texture=big)
        out.append({"frame": frame, "mask": mask, "block": b, "kind": kind})
    return out


def workload_stream_4k(frame_index: int, seed: int | None = None):
    """One 3840 x 2160 YUV 4:2:0 frame with 30 % random-burst 16 x 16 loss.

    Returns ((Y, U, V), (mask_Y, mask_U, mask_V)); chroma loses the 8 x 8
    cells co-located with the lost luma macroblocks.
    """
    s = (seed_for(5) if seed is None else seed) + frame_index
    h, w = 2160, 3840
    y = make_luma(h, w, s, n_bumps=150, n_edges=40, texture=True)
    u = make_chroma(h // 2, w // 2, s + 100)
    v = make_chroma(h // 2, w // 2, s + 200)
    my = loss_random_bursts(h, w, 16, 0.30, s + 500)
    mc = my[::2, ::2].copy()
    return (y, u, v), (my, mc, mc.copy())
