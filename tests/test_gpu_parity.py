"""GPU parity of the HIP concealment path against the float64 oracle.

Every call goes through the C ABI (ctypes binding).  Inputs are the seeded
synthetic workloads; the oracle never sees anything the GPU produced.
"""
import math

import numpy as np
import pytest

import synth
from oracle.skmmse import block_distances, conceal as oracle_conceal, lost_cells
from tests.parity import compare, device_params, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2205_11226_amd as skm
    assert torch.cuda.is_available()
    c = skm.Context(0)
    yield c
    c.close()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_both(ctx, frame, mask, mode, **kw):
    pg = device_params(mode, **kw)
    out, info, xh = ctx.conceal_device(to_dev(frame), to_dev(mask), pg)
    out_o, xh_o, info_o = oracle_conceal(frame, mask, oracle_params(mode, **kw))
    return out.cpu().numpy(), info, xh.cpu().numpy(), out_o, xh_o, info_o


def check(ctx, frame, mask, mode, **kw):
    out_g, info_g, xh_g, out_o, xh_o, info_o = run_both(ctx, frame, mask, mode, **kw)
    t_nu = kw.get("t_nu", 0.1)
    b = kw.get("block", 16)
    st = compare(frame, mask, out_g, info_g, xh_g, out_o, xh_o, info_o, t_nu, b,
                 ring=kw.get("ring", 4), window=kw.get("window", 24))
    print(mode, kw, st, flush=True)
    return st, info_g


# ------------------------------------------------------------- distances

def test_distances_bit_exact_plain_512(ctx):
    f, m = synth.workload_plain_512()
    p = device_params("plain")
    d, n = ctx.distances_device(to_dev(f), to_dev(m), p)
    d, n = d.cpu().numpy(), n.cpu().numpy()
    cells = lost_cells(m, 16)
    assert d.shape[0] == len(cells) == 64
    op = oracle_params("plain")
    avail = m == 0
    for i, (by, bx) in enumerate(cells):
        do, no = block_distances(f.astype(np.int64), avail, by, bx, op)
        assert np.array_equal(d[i], do), (by, bx)
        assert np.array_equal(n[i][do >= 0], no[do >= 0])


def test_distances_bit_exact_borders_and_neighbours(ctx):
    f = synth.make_luma(72, 88, 7, n_bumps=6, n_edges=4)
    m = synth.loss_random(72, 88, 8, 0.3, 8)
    p = device_params("plain", block=8, ring=3, window=10)
    d, n = ctx.distances_device(to_dev(f), to_dev(m), p)
    d, n = d.cpu().numpy(), n.cpu().numpy()
    op = oracle_params("plain", block=8, ring=3, window=10)
    for i, (by, bx) in enumerate(lost_cells(m, 8)):
        do, no = block_distances(f.astype(np.int64), m == 0, by, bx, op)
        assert np.array_equal(d[i], do), (by, bx)
        assert np.array_equal(n[i][do >= 0], no[do >= 0])


# --------------------------------------------------------- whole frames

def test_plain_512_parity(ctx):
    f, m = synth.workload_plain_512()
    st, info = check(ctx, f, m, "plain")
    assert (info["layer"] == 1).all()


def test_idl_expansion_512_parity(ctx):
    f, m = synth.workload_plain_512()
    for tnu in (0.01, 0.1, 100.0):
        check(ctx, f, m, "idl", t_nu=tnu)


def test_profile_1080p_dispersed_parity(ctx):
    f, m = synth.workload_layered_1080p()
    for prof, tnu in (("efficient", 0.1), ("express", 0.01)):
        st, info = check(ctx, f, m, "profile", t_nu=tnu)
        layers = np.bincount(info["layer"] + 1, minlength=4)
        assert layers[1] > 0 and layers[2] > 0   # some BRL, some IDL


def test_plain_1080p_dispersed_parity(ctx):
    f, m = synth.workload_layered_1080p()
    check(ctx, f, m, "plain")


@pytest.mark.parametrize("b,r,w", [(8, 4, 24), (8, 2, 12), (4, 1, 6), (16, 3, 17)])
def test_random_loss_multiround_parity(ctx, b, r, w):
    f = synth.make_luma(120, 152, 40 + b, n_bumps=10, n_edges=5)
    m = synth.loss_random(120, 152, b, 0.35, 41 + b)
    st, info = check(ctx, f, m, "profile", block=b, ring=r, window=w, t_nu=0.1)


@pytest.mark.parametrize("b,r,w,mode", [
    (16, 4, 24, "plain"), (16, 4, 24, "profile"), (16, 4, 24, "brl"),
    (8, 2, 12, "full"), (8, 4, 24, "idl"), (8, 3, 10, "profile"),
])
def test_arbitrary_shape_loss_parity(ctx, b, r, w, mode):
    """Cells that keep some received pixels: those join the context and are
    never overwritten."""
    f = synth.make_luma(112, 144, 80 + b, n_bumps=10, n_edges=5)
    m = synth.loss_partial_cells(112, 144, b, 0.35, 81 + b + r, frac=0.6)
    st, info = check(ctx, f, m, mode, block=b, ring=r, window=w, t_nu=0.1,
                     min_hql_cands=8)
    own = [(int(i["by"]), int(i["bx"])) for i in info
           if (m[int(i["by"]) * b:(int(i["by"]) + 1) * b,
                 int(i["bx"]) * b:(int(i["bx"]) + 1) * b] == 0).any()]
    assert own, "the mask should leave received pixels in some lost cells"
    if mode == "full":
        layer = {(int(i["by"]), int(i["bx"])): int(i["layer"]) for i in info}
        assert any(layer[k] == 2 for k in own), "some partly received cell should take HQL"


@pytest.mark.parametrize("grid", [64, 0])
def test_more_hql_blocks_than_hql_workgroups_parity(ctx, grid):
    """150 HQL blocks in one round on 64 HQL workgroups: each takes two or
    three blocks, so nothing of one block may leak into the next (grid 0:
    the automatic count, one block each)."""
    import paper_2205_11226_amd as skm
    f = synth.make_luma(256, 320, 170, n_bumps=20, n_edges=8)
    m = synth.loss_isolated(256, 320, 8, 150, 171)
    for bad in (-1, 1025):
        with pytest.raises(skm.SkmError):
            ctx.set_option(skm.OPT_HQL_GRID, bad)
    ctx.set_option(skm.OPT_HQL_GRID, grid)
    try:
        assert ctx.get_option(skm.OPT_HQL_GRID) == grid
        st, info = check(ctx, f, m, "full", block=8, ring=2, window=12, min_hql_cands=16)
    finally:
        ctx.set_option(skm.OPT_HQL_GRID, 0)
    assert len(info) == 150 and (info["layer"] == 2).all() and (info["round"] == 1).all()


def test_arbitrary_shape_loss_distances_bit_exact(ctx):
    f = synth.make_luma(96, 128, 90, n_bumps=8, n_edges=4)
    m = synth.loss_partial_cells(96, 128, 16, 0.4, 91, frac=0.7)
    p = device_params("plain")
    d, n = ctx.distances_device(to_dev(f), to_dev(m), p)
    d, n = d.cpu().numpy(), n.cpu().numpy()
    op = oracle_params("plain")
    cells = lost_cells(m, 16)
    assert d.shape[0] == len(cells) > 0
    for i, (by, bx) in enumerate(cells):
        do, no = block_distances(f.astype(np.int64), m == 0, by, bx, op)
        assert np.array_equal(d[i], do), (by, bx)
        assert np.array_equal(n[i][do >= 0], no[do >= 0])


def test_slice_loss_rounds_parity(ctx):
    f = synth.make_luma(160, 192, 50, n_bumps=10, n_edges=5)
    m = synth.loss_slices(160, 192, 16, 0.5, 51)
    st, info = check(ctx, f, m, "plain")
    assert info["round"].max() >= 2


def test_brl_mode_parity(ctx):
    f, m = synth.workload_plain_512()
    check(ctx, f, m, "brl")


def test_round_limit_fill_parity(ctx):
    f = synth.make_luma(128, 128, 60, n_bumps=8, n_edges=4)
    m = synth.loss_slices(128, 128, 16, 0.6, 61)
    st, info = check(ctx, f, m, "plain", max_rounds=1)
    assert (info["layer"] == -1).any()


# ----------------------------------------------------------- boundary

def test_host_and_device_entry_points_agree(ctx):
    import paper_2205_11226_amd as skm
    f = synth.make_luma(96, 112, 70, n_bumps=8, n_edges=4)
    m = synth.loss_random(96, 112, 8, 0.3, 71)
    p = skm.default_params(block=8)
    out_h, info_h = ctx.conceal(f, m, p)
    out_d, info_d, _ = ctx.conceal_device(to_dev(f), to_dev(m), p)
    assert np.array_equal(out_h, out_d.cpu().numpy())
    assert info_h.tobytes() == info_d.tobytes()       # NaN log nu for BRL blocks


def test_lost_pixels_are_never_read(ctx):
    import paper_2205_11226_amd as skm
    f, m = synth.workload_plain_512()
    g = f.copy()
    g[m > 0] = np.random.default_rng(3).integers(0, 256, int(m.sum()))
    p = skm.default_params()
    a, _, _ = ctx.conceal_device(to_dev(f), to_dev(m), p)
    b, _, _ = ctx.conceal_device(to_dev(g), to_dev(m), p)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_in_place_and_deterministic(ctx):
    import paper_2205_11226_amd as skm
    f, m = synth.workload_plain_512()
    p = skm.default_params(mode="idl")
    ref, info1, x1 = ctx.conceal_device(to_dev(f), to_dev(m), p)
    t = to_dev(f)
    out, info2, x2 = ctx.conceal_device(t, to_dev(m), p, out=t)
    assert out.data_ptr() == t.data_ptr()
    assert np.array_equal(ref.cpu().numpy(), t.cpu().numpy())
    assert info1.tobytes() == info2.tobytes()
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())


def test_strided_frame(ctx):
    import torch
    import paper_2205_11226_amd as skm
    f = synth.make_luma(96, 112, 72, n_bumps=8, n_edges=4)
    m = synth.loss_random(96, 112, 16, 0.3, 73)
    p = skm.default_params(mode="plain")
    big_f = torch.zeros((96, 160), dtype=torch.uint8, device="cuda")
    big_m = torch.zeros((96, 160), dtype=torch.uint8, device="cuda")
    big_f[:, :112] = to_dev(f)
    big_m[:, :112] = to_dev(m)
    out_s = torch.zeros_like(big_f)
    o1, i1, _ = ctx.conceal_device(big_f[:, :112], big_m[:, :112], p, out=out_s[:, :112])
    o2, i2, _ = ctx.conceal_device(to_dev(f), to_dev(m), p)
    assert np.array_equal(o1.cpu().numpy(), o2.cpu().numpy())
    assert i1.tobytes() == i2.tobytes()
    assert (out_s[:, 112:] == 0).all()


def test_odd_width_misaligned_frame(ctx):
    """A width and a row pitch that are not multiples of 4 and a frame that
    starts one byte into its allocation: the geometry kernel's per-column
    path.  The result must match the oracle and a contiguous copy."""
    import torch
    import paper_2205_11226_amd as skm
    h, w, pitch = 88, 117, 123
    f = synth.make_luma(h, w, 76, n_bumps=8, n_edges=4)
    m = np.zeros((h, w), dtype=np.uint8)
    m[:, :112] = synth.loss_random(h, 112, 8, 0.3, 77)
    big_f = torch.zeros((h * pitch + 1,), dtype=torch.uint8, device="cuda")
    big_m = torch.zeros_like(big_f)
    big_o = torch.zeros_like(big_f)
    vf = big_f[1:].as_strided((h, w), (pitch, 1))
    vm = big_m[1:].as_strided((h, w), (pitch, 1))
    vo = big_o[1:].as_strided((h, w), (pitch, 1))
    vf.copy_(to_dev(f))
    vm.copy_(to_dev(m))
    p = skm.default_params(mode="plain", block=8)
    o1, i1, x1 = ctx.conceal_device(vf, vm, p, out=vo)
    o2, i2, x2 = ctx.conceal_device(to_dev(f), to_dev(m), p)
    assert np.array_equal(o1.cpu().numpy(), o2.cpu().numpy())
    assert i1.tobytes() == i2.tobytes()
    check(ctx, f, m, "plain", block=8)


def test_no_loss_copies_frame(ctx):
    import paper_2205_11226_amd as skm
    f = synth.make_luma(64, 80, 74)
    m = np.zeros_like(f)
    out, info, _ = ctx.conceal_device(to_dev(f), to_dev(m), skm.default_params())
    assert np.array_equal(out.cpu().numpy(), f) and len(info) == 0


def test_error_codes(ctx):
    import paper_2205_11226_amd as skm
    f = synth.make_luma(64, 64, 75)
    allm = np.ones_like(f)
    with pytest.raises(skm.SkmError) as e:
        ctx.conceal_device(to_dev(f), to_dev(allm), skm.default_params())
    assert e.value.status == -1
    part = np.zeros_like(f)
    part[3:9, 5:20] = 1                    # cells with received pixels: accepted
    out, info, _ = ctx.conceal_device(to_dev(f), to_dev(part), skm.default_params())
    assert len(info) == 2 and np.array_equal(out.cpu().numpy()[part == 0], f[part == 0])
    edge = np.zeros((70, 64), np.uint8)
    edge[66:, :16] = 1                     # partial bottom cell row
    with pytest.raises(skm.SkmError) as e:
        ctx.conceal_device(to_dev(np.zeros((70, 64), np.uint8)), to_dev(edge),
                           skm.default_params())
    assert e.value.status == -4
    for bad in (dict(block=12), dict(ring=0), dict(window=40), dict(sigma2=0.0),
                dict(min_hql_cands=1), dict(mode=9), dict(t_nu=-1.0), dict(expand_step=1),
                dict(ridge_rel=-1.5)):
        with pytest.raises(skm.SkmError) as e:
            ctx.conceal_device(to_dev(f), to_dev(np.zeros_like(f)), skm.default_params(**bad))
        assert e.value.status == -1, bad


def test_small_info_capacity_is_rejected(ctx):
    import ctypes
    import torch
    import paper_2205_11226_amd as skm
    f, m = synth.workload_plain_512()
    tf, tm = to_dev(f), to_dev(m)
    out = torch.empty_like(tf)
    info = torch.zeros(10 * 48, dtype=torch.uint8, device="cuda")
    p = skm.default_params()
    n = ctypes.c_int32(0)
    st = skm.lib.skm_conceal_device(ctx._h, tf.data_ptr(), tm.data_ptr(), 512, 512, 512,
                                    ctypes.byref(p), out.data_ptr(), info.data_ptr(), None, 10,
                                    ctypes.byref(n), None)
    torch.cuda.synchronize()
    assert st == -1 and n.value == 64


# ------------------------------------------------------------------- HQL

def compare_sampled(ctx, frame, mask, mode, n_sample, seed=0, **kw):
    """Full-frame GPU run; oracle on a sample of blocks (single-round loss,
    so each block depends on the received frame only)."""
    import math as _m
    from oracle.skmmse import estimate_block
    pg = device_params(mode, **kw)
    out, info, xh = ctx.conceal_device(to_dev(frame), to_dev(mask), pg)
    out, xh = out.cpu().numpy(), xh.cpu().numpy()
    assert (info["round"] == 1).all()
    po = oracle_params(mode, **kw)
    u = frame.astype(np.int64)
    avail = mask == 0
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(info), size=min(n_sample, len(info)), replace=False)
    b = po.block
    t_nu = kw.get("t_nu", 0.1)
    log_tnu = _m.log(t_nu) if t_nu > 0 else -_m.inf
    worst = 0.0
    for k in sorted(idx):
        ig = info[k]
        by, bx = int(ig["by"]), int(ig["bx"])
        xo, io = estimate_block(u, avail, by, bx, po)
        if int(ig["layer"]) != io["layer"]:
            assert abs(io["log_nu"] - log_tnu) < 1e-9, (by, bx, int(ig["layer"]), io)
            continue
        for f in ("n_cand", "n_complete", "phi", "n_ctx", "flags", "radius"):
            assert int(ig[f]) == io[f], (by, bx, f, int(ig[f]), io[f])
        err = float(np.abs(xh[k].astype(np.float64).ravel() - xo).max())
        worst = max(worst, err)
        assert err <= 1e-3, (by, bx, io["layer"], err)
        g = out[by * b:(by + 1) * b, bx * b:(bx + 1) * b].ravel().astype(int)
        o = np.clip(np.floor(xo + 0.5), 0, 255).astype(int)
        for gv, ov, xv in zip(g, o, xo):
            if gv != ov:
                assert abs((xv - _m.floor(xv)) - 0.5) < 1e-3
    print(mode, kw, "sampled", len(idx), "max err", worst, flush=True)
    return info


def test_full_kmmse_512_sampled(ctx):
    f, m = synth.workload_plain_512()
    info = compare_sampled(ctx, f, m, "full", 12)
    assert (info["layer"] == 2).all()


def test_profile_512_sampled(ctx):
    f, m = synth.workload_plain_512()
    for tnu in (0.1, 100.0):
        info = compare_sampled(ctx, f, m, "profile", 16, t_nu=tnu)
        assert (info["layer"] == 2).any()


@pytest.mark.parametrize("b,r,w", [(8, 2, 12), (8, 3, 14), (4, 2, 9)])
def test_full_small_frames_parity(ctx, b, r, w):
    f = synth.make_luma(80, 96, 90 + b + r, n_bumps=6, n_edges=4)
    m = synth.loss_random(80, 96, b, 0.15, 91 + b + r)
    st, info = check(ctx, f, m, "full", block=b, ring=r, window=w, min_hql_cands=8)
    assert (info["layer"] == 2).any()


def test_hql_ramp_is_exact(ctx):
    yy, xx = np.mgrid[0:96, 0:96]
    f = (2 * xx + yy // 2 + 5).astype(np.uint8)
    m = np.zeros_like(f)
    m[40:48, 40:48] = 1
    pg = device_params("full", block=8, ring=2, window=12, min_hql_cands=8)
    out, info, xh = ctx.conceal_device(to_dev(f), to_dev(m), pg)
    assert int(info[0]["layer"]) == 2
    np.testing.assert_allclose(xh.cpu().numpy()[0], f[40:48, 40:48], rtol=0, atol=1e-3)


def test_hql_indefinite_covariance_falls_back_to_context_mean(ctx):
    """A negative ridge makes C_YY + lambda I indefinite: the Cholesky
    factorisation meets a pivot <= 0 and every HQL block takes the context
    mean, flagged, as in the oracle (forced from the host through ridge_rel)."""
    import paper_2205_11226_amd as skm
    f = synth.make_luma(80, 96, 98, n_bumps=6, n_edges=4)
    m = synth.loss_random(80, 96, 8, 0.15, 99)
    st, info = check(ctx, f, m, "full", block=8, ring=2, window=12, min_hql_cands=8,
                     ridge_rel=-1.0)
    sing = (info["flags"] & skm.FLAG_HQL_SINGULAR) != 0
    assert sing.sum() >= 3 and (info["layer"][sing] == 0).all()
    assert not (info["layer"] == 2).any()
