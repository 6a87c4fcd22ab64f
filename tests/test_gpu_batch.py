"""GPU: captured-graph replays, the batch entry point and the autotuner.

Graph replays and batch results are compared bit for bit with the eager
single-frame path (itself compared with the float64 oracle in
test_gpu_parity); the full-size mixed batch and the 4K YUV 4:2:0 stream frame
are checked against the oracle on sampled round-1 blocks."""
import math
import os

import numpy as np
import pytest

import synth
from oracle import cnn as ocnn
from oracle.skmmse import Params, estimate_block, lost_cells
from tests.parity import XHAT_TOL, device_params

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


def run_single(ctx, f, m, prm):
    out, info, xh = ctx.conceal_device(to_dev(f), to_dev(m), prm)
    return out.cpu().numpy(), info, xh.cpu().numpy()


@pytest.mark.parametrize("mode", ["plain", "profile", "cnn"])
def test_graph_replays_match_eager(ctx, mode):
    import torch
    import paper_2205_11226_amd as skm
    f = synth.make_luma(240, 320, 71, n_bumps=20, n_edges=8)
    m = synth.loss_slices(240, 320, 16, 0.5, 72)          # two rounds
    prm = device_params(mode)
    ctx.set_option(skm.OPT_GRAPHS, 0)
    ref = run_single(ctx, f, m, prm)
    ctx.set_option(skm.OPT_GRAPHS, 1)
    try:
        for rep in range(5):
            got = run_single(ctx, f, m, prm)
            assert np.array_equal(got[0], ref[0]), rep
            assert got[1].tobytes() == ref[1].tobytes(), rep
            assert np.array_equal(got[2], ref[2]), rep
            # eager work and a synchronisation between replays
            ctx.set_option(skm.OPT_GRAPHS, 0)
            run_single(ctx, f, m, prm)
            torch.cuda.synchronize()
            ctx.set_option(skm.OPT_GRAPHS, 1)
    finally:
        ctx.set_option(skm.OPT_GRAPHS, 1)
    assert ref[1]["round"].max() >= 2


def _batch_jobs(frames, prms):
    import torch
    jobs, outs = [], []
    for (f, m), prm in zip(frames, prms):
        fd, md = to_dev(f), to_dev(m)
        b = prm.block
        cap = (f.shape[0] // b) * (f.shape[1] // b)
        info = torch.zeros(max(cap, 1) * 48, dtype=torch.uint8, device="cuda")
        xh = torch.zeros((max(cap, 1), b, b), dtype=torch.float32, device="cuda")
        out = torch.empty_like(fd)
        jobs.append((fd, md, out, prm, info, xh, cap))
        outs.append((out, info, xh))
    return jobs, outs


def test_batch_matches_single_frames(ctx):
    import paper_2205_11226_amd as skm
    wl = synth.workload_batch(n_frames=6, sizes=[(360, 640)] * 3 + [(540, 960)] * 3)
    frames = [(w["frame"], w["mask"]) for w in wl]
    modes = ["profile", "cnn", "plain", "profile", "cnn", "idl"]
    prms = [device_params(md, block=w["block"]) for md, w in zip(modes, wl)]
    refs = [run_single(ctx, f, m, prm) for (f, m), prm in zip(frames, prms)]
    for streams in (1, 3, 4):
        ctx.set_option(skm.OPT_BATCH_STREAMS, streams)
        for rep in range(2):
            jobs, outs = _batch_jobs(frames, prms)
            res = ctx.conceal_batch(jobs)
            for k, ((out, info, xh), ref) in enumerate(zip(outs, refs)):
                n, rounds, st = res[k]
                assert st == 0 and n == len(ref[1]), (streams, k)
                assert rounds == int(ref[1]["round"].max()), (streams, k)
                assert np.array_equal(out.cpu().numpy(), ref[0]), (streams, rep, k)
                gi = info.cpu().numpy().view(skm.BLOCK_INFO_DTYPE)[:n]
                assert gi.tobytes() == ref[1].tobytes(), (streams, rep, k)
                assert np.array_equal(xh[:n].cpu().numpy(), ref[2]), (streams, rep, k)
    ctx.set_option(skm.OPT_BATCH_STREAMS, 4)


def test_batch_arbitrary_shape_loss_matches_single_frames(ctx):
    """Cells that keep received pixels, in a batch of mixed geometry and
    modes (graph replay on and off): bit-identical to single-frame runs."""
    import paper_2205_11226_amd as skm
    frames, prms = [], []
    for k, (h, w, b, mode) in enumerate([(144, 176, 16, "profile"), (120, 152, 8, "plain"),
                                          (144, 176, 16, "cnn"), (96, 128, 8, "full")]):
        f = synth.make_luma(h, w, 300 + k, n_bumps=10, n_edges=5)
        m = synth.loss_partial_cells(h, w, b, 0.35, 310 + k, frac=0.6)
        frames.append((f, m))
        prms.append(device_params(mode, block=b, min_hql_cands=8))
    refs = [run_single(ctx, f, m, prm) for (f, m), prm in zip(frames, prms)]
    for (f, m), ref in zip(frames, refs):
        assert np.array_equal(ref[0][m == 0], f[m == 0])
    for graphs in (0, 1):
        ctx.set_option(skm.OPT_GRAPHS, graphs)
        jobs, outs = _batch_jobs(frames, prms)
        res = ctx.conceal_batch(jobs)
        for k, ((out, info, xh), ref) in enumerate(zip(outs, refs)):
            n, rounds, st = res[k]
            assert st == 0 and n == len(ref[1]), (graphs, k)
            assert np.array_equal(out.cpu().numpy(), ref[0]), (graphs, k)
            gi = info.cpu().numpy().view(skm.BLOCK_INFO_DTYPE)[:n]
            assert gi.tobytes() == ref[1].tobytes(), (graphs, k)
            assert np.array_equal(xh[:n].cpu().numpy(), ref[2]), (graphs, k)
    ctx.set_option(skm.OPT_GRAPHS, 1)


def test_batch_reports_errors_per_frame(ctx):
    import paper_2205_11226_amd as skm
    f = synth.make_luma(128, 128, 5)
    good = synth.loss_random(128, 128, 16, 0.2, 6)
    f2 = synth.make_luma(136, 128, 5)                  # 8 rows below the last cell row
    bad = np.zeros((136, 128), np.uint8)
    bad[:128] = good
    bad[130, 5] = 1                                    # a lost pixel outside the cells
    prm = device_params("plain")
    jobs, _ = _batch_jobs([(f, good), (f2, bad), (f, good)], [prm] * 3)
    with pytest.raises(skm.SkmError):
        ctx.conceal_batch(jobs)
    descs, keep = ctx._frame_descs(jobs)
    st = skm.api.lib.skm_conceal_batch(ctx._h, descs, 3, None)
    assert st != 0
    assert [d.status for d in descs] == [0, st, 0]


def _sampled_oracle(f, m, b, info, xh, mode, n_samples, seed, gate=None, t_nu=0.1):
    """Oracle estimates of sampled round-1 blocks (the round-1 state is the
    received frame), compared with the GPU's."""
    rng = np.random.default_rng(seed)
    idx = [k for k in range(len(info)) if int(info["round"][k]) == 1]
    pick = rng.choice(idx, size=min(n_samples, len(idx)), replace=False)
    u = np.where(m == 0, f, 0).astype(np.int64)
    avail = m == 0
    p = Params(mode=mode, block=b, t_nu=t_nu)
    checked = 0
    for k in pick:
        by, bx = int(info["by"][k]), int(info["bx"][k])
        near = {}
        g = None
        if gate is not None:
            def g(uu, aa, yy, xx):
                choice, is_near = gate(uu, aa, yy, xx)
                near["v"] = is_near
                return choice
        xo, io = estimate_block(u, avail, by, bx, p, g)
        if near.get("v"):
            continue
        assert int(info["layer"][k]) == io["layer"], (by, bx, int(info["layer"][k]), io)
        err = float(np.abs(xh[k].astype(np.float64) - xo.reshape(b, b)).max())
        assert err <= XHAT_TOL, (by, bx, err)
        checked += 1
    return checked


def test_full_size_mixed_batch_sampled_oracle(ctx):
    """One frame of each size of the mixed 64-frame batch (720p, 1080p,
    2160p; cell size and loss kind from the seed), concealed in one batch
    with the paper's profile gating."""
    import paper_2205_11226_amd as skm
    base = synth.seed_for(3)
    # frames 0, 24 and 56 of the batch (its frame f uses seed base + f)
    pick = [synth.workload_batch(1, seed=base + f, sizes=[hw])[0]
            for f, hw in ((0, (720, 1280)), (24, (1080, 1920)), (56, (2160, 3840)))]
    frames = [(w["frame"], w["mask"]) for w in pick]
    prms = [device_params("profile", block=w["block"]) for w in pick]
    jobs, outs = _batch_jobs(frames, prms)
    res = ctx.conceal_batch(jobs)
    for k, ((f, m), w) in enumerate(zip(frames, pick)):
        n = res[k][0]
        info = outs[k][1].cpu().numpy().view(skm.BLOCK_INFO_DTYPE)[:n]
        xh = outs[k][2][:n].cpu().numpy()
        assert n == len(lost_cells(m, w["block"]))
        keep = info["layer"] != 2          # keep the oracle's HQL cost bounded
        got = _sampled_oracle(f, m, w["block"], info[keep], xh[keep], "profile", 6, 100 + k)
        print(f"frame {k}: {f.shape} B={w['block']} {w['kind']} lost {n}, "
              f"rounds {res[k][1]}, oracle-checked {got}", flush=True)
        assert got >= 3


def test_stream_4k_yuv_sampled_oracle(ctx):
    """One frame of the 4K YUV 4:2:0 stream (30% bursty 16x16 loss, chroma
    losing the co-located 8x8 cells), the three planes in one batch with CNN
    gating; sampled round-1 blocks against the oracle running the same
    network (blocks within 1e-3 of a threshold are skipped)."""
    import paper_2205_11226_amd as skm
    from bench import read_gate
    planes, masks = synth.workload_stream_4k(0)
    t1, t2, w = read_gate(WEIGHTS)
    pw = ocnn.unpack(w)
    prms = [device_params("cnn", block=16), device_params("cnn", block=8),
            device_params("cnn", block=8)]
    jobs, outs = _batch_jobs(list(zip(planes, masks)), prms)
    res = ctx.conceal_batch(jobs)
    for k, (f, m) in enumerate(zip(planes, masks)):
        b = prms[k].block

        def gate(u, avail, by, bx):
            y = ocnn.forward(pw, ocnn.block_input(u, avail, by, bx, b)[None])[0]
            near = min(abs(y[0] - t1), abs(y[1] - t2)) < 1e-3
            return (0 if y[0] <= t1 else (2 if y[1] > t2 else 1)), near
        n = res[k][0]
        info = outs[k][1].cpu().numpy().view(skm.BLOCK_INFO_DTYPE)[:n]
        xh = outs[k][2][:n].cpu().numpy()
        hql = info["layer"] == 2
        if hql.any():                      # keep the oracle's HQL cost bounded
            info, xh = info[~hql], xh[~hql]
        got = _sampled_oracle(f, m, b, info, xh, "cnn", 5, 200 + k, gate=gate)
        print(f"plane {k}: {f.shape} B={b} lost {n}, rounds {res[k][1]}, "
              f"oracle-checked {got}", flush=True)
        assert got >= 2


def test_autotune_keeps_results(ctx):
    import paper_2205_11226_amd as skm
    f, m = synth.workload_plain_512()
    prm = device_params("cnn")
    ref = run_single(ctx, f, m, prm)
    jobs, outs = _batch_jobs([(f, m)] * 3, [prm] * 3)
    best = ctx.autotune(jobs, reps=2)
    assert best > 0.0
    assert ctx.get_option(skm.OPT_BATCH_STREAMS) in (1, 2, 4, 8)
    assert ctx.get_option(skm.OPT_GRAPHS) in (0, 1)
    assert ctx.get_option(skm.OPT_GATE_GRID) in (640, 1280, 2560)
    for out, info, xh in outs:
        assert np.array_equal(out.cpu().numpy(), ref[0])
    got = run_single(ctx, f, m, prm)
    assert np.array_equal(got[0], ref[0]) and got[1].tobytes() == ref[1].tobytes()
    ctx.set_option(skm.OPT_BATCH_STREAMS, 4)
    ctx.set_option(skm.OPT_GRAPHS, 1)
    ctx.set_option(skm.OPT_GATE_GRID, 1280)


def test_batch_patch_geometry_matches_single_frames(ctx):
    """The paper's 2x2 patches (several rounds per frame) next to a block
    frame in one batch; graphs off, then on twice (the second call replays
    the captured graphs): bit-identical to single-frame runs."""
    import paper_2205_11226_amd as skm
    frames, prms = [], []
    for k, (h, w, mode, win) in enumerate([(80, 112, "profile", 24), (64, 96, "full", 12),
                                           (96, 128, "plain", 24)]):
        f = synth.make_luma(h, w, 400 + k, n_bumps=10, n_edges=5)
        m = synth.loss_random(h, w, 16, 0.3, 410 + k)
        frames.append((f, m))
        prms.append(skm.patch_params(mode=mode, window=win, min_hql_cands=16))
    f = synth.make_luma(144, 176, 420, n_bumps=10, n_edges=5)
    frames.append((f, synth.loss_random(144, 176, 16, 0.3, 421)))
    prms.append(device_params("profile"))
    refs = [run_single(ctx, f, m, prm) for (f, m), prm in zip(frames, prms)]
    assert max(int(r[1]["round"].max()) for r in refs[:3]) >= 4
    for graphs in (0, 1, 1):
        ctx.set_option(skm.OPT_GRAPHS, graphs)
        jobs, outs = _batch_jobs(frames, prms)
        res = ctx.conceal_batch(jobs)
        for k, ((out, info, xh), ref) in enumerate(zip(outs, refs)):
            n, rounds, st = res[k]
            assert st == 0 and n == len(ref[1]), (graphs, k)
            assert np.array_equal(out.cpu().numpy(), ref[0]), (graphs, k)
            gi = info.cpu().numpy().view(skm.BLOCK_INFO_DTYPE)[:n]
            assert gi.tobytes() == ref[1].tobytes(), (graphs, k)
            assert np.array_equal(xh[:n].cpu().numpy(), ref[2]), (graphs, k)
    ctx.set_option(skm.OPT_GRAPHS, 1)
