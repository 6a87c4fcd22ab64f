"""Float64 reference of the learned layer manager — TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use
this module.

The network predicts, from a 48 x 48 window centred on a lost block, the
PSNR gain (dB) of the next refinement layer over the one below:
g1 = PSNR(IDL over the whole window) - PSNR(BRL) and
g2 = PSNR(HQL) - PSNR(IDL), 0 where HQL is not available (Sec. "Scalable
K-MMSE estimator" defines the layers; the gate replaces the profile rule of
Sec. "Layer switching and profile selection").

Input channels: c0 = (u - 128) / 128 at known pixels, 0 elsewhere; c1 = 1 at
unknown pixels (lost or outside the frame), 0 elsewhere.  The (2, 48, 48)
input is rearranged without loss into (8, 24, 24): channel 4 c + 2 dy + dx
at (Y, X) holds channel c at pixel (2 Y + dy, 2 X + dx) (space to depth).
Layers: three 3x3 convolutions, stride 2, zero padding 1, 32 channels, ReLU
(24 -> 12 -> 6 -> 3), global average pool, linear 32 -> 2.
Precision model of the GPU network: weights and the inputs of every
convolution are rounded to bfloat16 (round to nearest even); sums are exact
here (float64) and FP32 on the GPU; pooling and head in full precision.
The backward pass treats the bfloat16 rounding of activations as identity.
"""
from __future__ import annotations

import numpy as np

SHAPES = {
    "w1": (32, 8, 3, 3), "b1": (32,),
    "w2": (32, 32, 3, 3), "b2": (32,),
    "w3": (32, 32, 3, 3), "b3": (32,),
    "wh": (2, 32), "bh": (2,),
}
ORDER = ("w1", "b1", "w2", "b2", "w3", "b3", "wh", "bh")
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES.values())
PATCH = 48


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def unpack(flat: np.ndarray) -> dict:
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(SHAPES[k]))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(SHAPES[k])
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in ORDER])


def block_input(u: np.ndarray, avail: np.ndarray, by: int, bx: int, b: int) -> np.ndarray:
    """(2, 48, 48) input for block (by, bx): window centred on the block."""
    h, w = u.shape
    y0 = by * b + b // 2 - PATCH // 2
    x0 = bx * b + b // 2 - PATCH // 2
    ys = np.arange(y0, y0 + PATCH)[:, None]
    xs = np.arange(x0, x0 + PATCH)[None, :]
    inside = (ys >= 0) & (ys < h) & (xs >= 0) & (xs < w)
    yc, xc = np.clip(ys, 0, h - 1), np.clip(xs, 0, w - 1)
    known = inside & avail[yc, xc]
    c0 = np.where(known, (u[yc, xc].astype(np.float64) - 128.0) / 128.0, 0.0)
    c1 = np.where(known, 0.0, 1.0)
    return np.stack([c0, c1])


def space_to_depth(x: np.ndarray) -> np.ndarray:
    """(N, 2, 48, 48) -> (N, 8, 24, 24); channel 4 c + 2 dy + dx at (Y, X) is
    channel c at pixel (2 Y + dy, 2 X + dx)."""
    n, c, h, w = x.shape
    out = np.empty((n, 4 * c, h // 2, w // 2), dtype=x.dtype)
    for ch in range(c):
        for dy in range(2):
            for dx in range(2):
                out[:, 4 * ch + 2 * dy + dx] = x[:, ch, dy::2, dx::2]
    return out


def _conv_s2(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """3x3 convolution, stride 2, zero padding 1: x (N, C, H, H) -> (N, K, H/2, H/2)."""
    n, c, hh, _ = x.shape
    ho = hh // 2
    xp = np.zeros((n, c, hh + 2, hh + 2))
    xp[:, :, 1:-1, 1:-1] = x
    out = np.zeros((n, w.shape[0], ho, ho))
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + 2 * ho:2, kx:kx + 2 * ho:2]      # (N, C, ho, ho)
            out += np.einsum("nchw,kc->nkhw", patch, w[:, :, ky, kx])
    return out + b[None, :, None, None]


def _conv_s2_back(x, w, gout):
    """Gradients of _conv_s2 w.r.t. x, w, b for upstream gradient gout."""
    n, c, hh, _ = x.shape
    ho = hh // 2
    xp = np.zeros((n, c, hh + 2, hh + 2))
    xp[:, :, 1:-1, 1:-1] = x
    gx = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, :, ky:ky + 2 * ho:2, kx:kx + 2 * ho:2]
            gw[:, :, ky, kx] = np.einsum("nkhw,nchw->kc", gout, patch)
            gx[:, :, ky:ky + 2 * ho:2, kx:kx + 2 * ho:2] += np.einsum("nkhw,kc->nchw", gout,
                                                                     w[:, :, ky, kx])
    gb = gout.sum(axis=(0, 2, 3))
    return gx[:, :, 1:-1, 1:-1], gw, gb


def forward(params: dict, x: np.ndarray, keep=False, quant=True):
    """x (N, 2, 48, 48) -> predictions (N, 2); with keep, also the cache.
    quant=False skips the bfloat16 rounding (exact float64 network)."""
    rq = bf16 if quant else (lambda v: np.asarray(v, dtype=np.float64))
    q = {k: rq(v) if k.startswith("w") and k != "wh" else v for k, v in params.items()}
    a0 = rq(space_to_depth(x))
    z1 = _conv_s2(a0, q["w1"], q["b1"])
    a1 = rq(np.maximum(z1, 0.0))
    z2 = _conv_s2(a1, q["w2"], q["b2"])
    a2 = rq(np.maximum(z2, 0.0))
    z3 = _conv_s2(a2, q["w3"], q["b3"])
    a3 = np.maximum(z3, 0.0)
    g = a3.mean(axis=(2, 3))                                       # (N, 32)
    y = g @ q["wh"].T + q["bh"]
    if keep:
        return y, dict(q=q, a0=a0, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, a3=a3, g=g)
    return y


def loss_and_grads(params: dict, x: np.ndarray, t: np.ndarray, quant=True):
    """Mean squared error over the batch and both outputs, and its gradients
    with respect to every parameter (hand-derived backward)."""
    y, c = forward(params, x, keep=True, quant=quant)
    n = x.shape[0]
    diff = y - t
    loss = float((diff * diff).mean())
    gy = 2.0 * diff / diff.size                                    # (N, 2)
    q = c["q"]
    grads = {"wh": gy.T @ c["g"], "bh": gy.sum(axis=0)}
    gg = gy @ q["wh"]                                              # (N, 32)
    ga3 = np.repeat(np.repeat(gg[:, :, None, None] / 9.0, 3, axis=2), 3, axis=3)
    gz3 = ga3 * (c["z3"] > 0)
    ga2, grads["w3"], grads["b3"] = _conv_s2_back(c["a2"], q["w3"], gz3)
    gz2 = ga2 * (c["z2"] > 0)
    ga1, grads["w2"], grads["b2"] = _conv_s2_back(c["a1"], q["w2"], gz2)
    gz1 = ga1 * (c["z1"] > 0)
    _, grads["w1"], grads["b1"] = _conv_s2_back(c["a0"], q["w1"], gz1)
    assert n == x.shape[0]
    return loss, grads


def init_params(seed: int) -> dict:
    """He-uniform initialisation, zero biases (same recipe as the GPU)."""
    rng = np.random.default_rng(seed)
    p = {}
    for k in ORDER:
        s = SHAPES[k]
        if k.startswith("b"):
            p[k] = np.zeros(s)
        else:
            fan_in = int(np.prod(s[1:]))
            lim = np.sqrt(6.0 / fan_in)
            p[k] = rng.uniform(-lim, lim, size=s)
    return p


def block_psnr_gain(est_a: np.ndarray, est_b: np.ndarray, truth: np.ndarray) -> float:
    """PSNR(est_b) - PSNR(est_a) over one block, MSE floored at 1/12 (the
    variance of uniform rounding error), peak 255."""
    def ps(e):
        d = e.astype(np.float64) - truth.astype(np.float64)
        mse = max(float((d * d).mean()), 1.0 / 12.0)
        return 10.0 * np.log10(255.0 * 255.0 / mse)
    return ps(est_b) - ps(est_a)
