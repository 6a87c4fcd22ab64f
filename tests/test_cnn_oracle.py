"""Pins of the float64 CNN reference: finite differences, an independent
(torch, CPU) convolution and forward, bfloat16 rounding and the input map."""
import numpy as np
import pytest
import torch

from oracle import cnn


def _rand(seed, n=3):
    rng = np.random.default_rng(seed)
    x = np.stack([rng.uniform(-1, 1, size=(n, 48, 48)), (rng.uniform(size=(n, 48, 48)) < 0.3)],
                 axis=1).astype(np.float64)
    t = rng.normal(size=(n, 2))
    return x, t


def test_backward_matches_central_differences():
    p = cnn.init_params(5)
    for k in p:                         # non-zero biases exercise their gradients
        if k.startswith("b"):
            p[k] = np.random.default_rng(1).normal(0, 0.1, size=p[k].shape)
    x, t = _rand(7)
    _, g = cnn.loss_and_grads(p, x, t, quant=False)
    rng = np.random.default_rng(9)
    eps = 1e-6
    for k in cnn.ORDER:
        flat = p[k].ravel()
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = cnn.loss_and_grads(p, x, t, quant=False)[0]
            flat[idx] = old - eps
            lm = cnn.loss_and_grads(p, x, t, quant=False)[0]
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = g[k].ravel()[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, idx, fd, an)


def test_conv_matches_torch_conv2d():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 3, 12, 12))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b),
                                     stride=2, padding=1).numpy()
    np.testing.assert_allclose(cnn._conv_s2(x, w, b), ref, rtol=0, atol=1e-12)


def test_forward_matches_torch_network():
    p = cnn.init_params(3)
    x, _ = _rand(4)
    ours = cnn.forward(p, x, quant=False)
    t = {k: torch.from_numpy(v) for k, v in p.items()}
    # space to depth by torch's own pixel_unshuffle (channel c*4 + dy*2 + dx)
    h = torch.nn.functional.pixel_unshuffle(torch.from_numpy(x), 2)
    for i in (1, 2, 3):
        h = torch.relu(torch.nn.functional.conv2d(h, t[f"w{i}"], t[f"b{i}"], stride=2, padding=1))
    ref = (h.mean(dim=(2, 3)) @ t["wh"].T + t["bh"]).numpy()
    np.testing.assert_allclose(ours, ref, rtol=0, atol=1e-12)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.normal(size=2000) * 10, [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -0.0, 0.5]])
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16(v), ref)


def test_input_map_centres_the_block_and_hides_lost_pixels():
    u = np.arange(64 * 64, dtype=np.int64).reshape(64, 64) % 256
    avail = np.ones((64, 64), bool)
    avail[0:16, 0:16] = False
    x = cnn.block_input(u, avail, 0, 0, 16)        # window origin (-16, -16)
    assert x.shape == (2, 48, 48)
    assert (x[1, 16:32, 16:32] == 1).all() and (x[0, 16:32, 16:32] == 0).all()
    assert x[1, :16, :].all() and x[1, :, :16].all()        # outside the frame
    assert x[0, 32, 40] == (u[16, 24] - 128) / 128.0 and x[1, 32, 40] == 0
    x8 = cnn.block_input(u, np.ones((64, 64), bool), 2, 3, 8)   # origin (y, x) = (-4, 4)
    assert x8[1, 3, 0] == 1 and x8[0, 3, 0] == 0                # row -1: outside
    assert x8[1, 4, 0] == 0 and x8[0, 4, 0] == (u[0, 4] - 128) / 128.0
    assert cnn.N_PARAMS == 20898


def test_space_to_depth_is_a_lossless_rearrangement():
    x, _ = _rand(11, n=2)
    s = cnn.space_to_depth(x)
    assert s.shape == (2, 8, 24, 24)
    np.testing.assert_array_equal(np.sort(s.ravel()), np.sort(x.ravel()))
    assert s[1, 4 * 1 + 2 * 1 + 0, 5, 7] == x[1, 1, 11, 14]
