"""GPU: the allocation-free entry point (skm_conceal_device_noalloc) against
skm_conceal_device.

Both run the same kernels; the allocation-free one takes its workspace from
the library's fixed per-GPU array and launches eagerly, so its output, block
records and pre-rounding estimates must equal the other entry point's bit for
bit.  Each case makes two calls in a row, the second on a smaller frame (the
array keeps the first call's contents), and checks that the calls leave the
device's free memory unchanged."""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_2205_11226_amd", "weights",
                       "gate_1080p.skm")


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2205_11226_amd as skm
    assert torch.cuda.is_available()
    c = skm.Context(0)
    c.cnn_load(WEIGHTS)
    yield c
    c.close()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def frames(kind):
    """(big, small) frame/mask pairs of one loss kind."""
    if kind == "lattice":
        big = (synth.make_luma(720, 1280, 5101, n_bumps=80, n_edges=24, texture=True),
               synth.loss_dispersed(720, 1280, 16))
        small = (synth.make_luma(256, 320, 5102, n_bumps=20, n_edges=8),
                 synth.loss_dispersed(256, 320, 16, 1, 0))
    elif kind == "isolated":                       # HQL blocks (complete candidates)
        big = (synth.make_luma(512, 512, 5103), synth.loss_isolated(512, 512, 16, 64, 5104))
        small = (synth.make_luma(192, 256, 5105, n_bumps=12, n_edges=6),
                 synth.loss_isolated(192, 256, 16, 8, 5106))
    else:                                          # slices: several rounds
        big = (synth.make_luma(480, 640, 5107, n_bumps=40, n_edges=12),
               synth.loss_slices(480, 640, 16, 0.4, 5108))
        small = (synth.make_luma(160, 224, 5109, n_bumps=12, n_edges=6),
                 synth.loss_slices(160, 224, 16, 0.5, 5110))
    return big, small


def run(ctx, entry, f, m, prm):
    import torch
    fd, md = to_dev(f), to_dev(m)
    out, info, xh = entry(fd, md, prm)
    torch.cuda.synchronize()
    return out.cpu().numpy(), info, xh.cpu().numpy()


@pytest.mark.parametrize("mode,kind", [("plain", "lattice"), ("cnn", "lattice"),
                                       ("profile", "isolated"), ("full", "isolated"),
                                       ("profile", "slices")])
def test_noalloc_matches_conceal_device(ctx, mode, kind):
    import torch
    import paper_2205_11226_amd as skm
    prm = skm.default_params(mode=mode)
    big, small = frames(kind)
    print(f"noalloc case: mode={mode} loss={kind} shapes={big[0].shape},{small[0].shape}",
          flush=True)
    # references first (they may grow the context's own workspace)
    ref_big = run(ctx, ctx.conceal_device, *big, prm)
    ref_small = run(ctx, ctx.conceal_device, *small, prm)
    # inputs of the calls under test allocated up front, so that only the
    # library could change the device's free memory during the calls
    fb, mb, fs, ms = (to_dev(a) for a in (*big, *small))
    ob, os_ = torch.empty_like(fb), torch.empty_like(fs)
    b = prm.block
    cb, cs = (fb.shape[0] // b) * (fb.shape[1] // b), (fs.shape[0] // b) * (fs.shape[1] // b)
    # warm-up call: loads kernels the context has not launched yet
    ctx.conceal_device_noalloc(fs, ms, prm, out=os_, want_info=False, want_xhat=False)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got_big = ctx.conceal_device_noalloc(fb, mb, prm, out=ob)
    got_small = ctx.conceal_device_noalloc(fs, ms, prm, out=os_)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    for ref, got, cap in ((ref_big, got_big, cb), (ref_small, got_small, cs)):
        out, info, xh = got[0].cpu().numpy(), got[1], got[2].cpu().numpy()
        assert 0 < len(info) <= cap
        assert np.array_equal(out, ref[0])
        assert info.tobytes() == ref[1].tobytes()
        assert np.array_equal(xh, ref[2])
    if mode in ("profile", "full") and kind == "isolated":
        assert (ref_big[1]["layer"] == skm.LAYER_HQL).any()
    if kind == "slices":
        assert ref_big[1]["round"].max() > 1
    assert free1 == free0, (free0, free1)


def test_noalloc_rejects_frames_beyond_its_workspace(ctx):
    import torch
    import paper_2205_11226_amd as skm
    f = torch.zeros((4096, 8192), dtype=torch.uint8, device="cuda")   # 64 MiB value plane
    m = torch.zeros_like(f)
    m[:16, :16] = 1
    with pytest.raises(skm.SkmError) as e:
        ctx.conceal_device_noalloc(f, m, skm.default_params(mode="plain"))
    assert e.value.status == -1
    assert "skm_conceal_device_noalloc has" in skm.lib.skm_last_error().decode()
    # the same frame through the allocating entry point still works
    out, info, _ = ctx.conceal_device(f, m, skm.default_params(mode="plain"))
    assert len(info) == 1
