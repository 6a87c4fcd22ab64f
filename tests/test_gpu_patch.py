"""Parity of the paper's 2 x 2 patch geometry (B 2, ring 2: a 6 x 6 context)
against the float64 oracle, through the C ABI.

Lost 16 x 16 blocks are concealed patch by patch; a patch waits until its
ring holds ring*block known pixels, so the rounds run from the border of a
lost region towards its centre (Sec. "Reconstruction framework").
"""
import numpy as np
import pytest

import synth
from oracle.skmmse import block_distances, lost_cells
from tests.parity import oracle_params
from tests.test_gpu_parity import check, ctx, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu

PATCH = dict(block=2, ring=2)


def _dispersed(h, w, seed):
    f = synth.make_luma(h, w, seed, n_bumps=10, n_edges=5)
    return f, synth.loss_dispersed(h, w, 16, ox=1, oy=1)


@pytest.mark.parametrize("mode,win,tnu,hql", [
    ("plain", 24, 0.1, 64),
    ("profile", 24, 0.1, 64),           # the efficient profile
    ("profile", 12, 100.0, 16),         # the excellent profile, reaching HQL
    ("full", 12, 0.1, 16),
    ("brl", 24, 0.1, 64),
])
def test_patch_mode_dispersed_parity(ctx, mode, win, tnu, hql):
    f, m = _dispersed(80, 112, 100 + win)
    st, info = check(ctx, f, m, mode, window=win, t_nu=tnu, min_hql_cands=hql, **PATCH)
    assert len(info) == 6 * 64
    if mode == "full":
        assert (info["layer"] == 2).sum() > len(info) // 2


def test_patch_mode_rounds_run_from_border_to_centre(ctx):
    """Patch (i, j) of an isolated lost 16 x 16 block is concealed in round
    1 + min(i, j, 7 - i, 7 - j)."""
    f, m = _dispersed(80, 112, 120)
    st, info = check(ctx, f, m, "plain", window=24, **PATCH)
    for i in info:
        pi, pj = int(i["by"]) % 8, int(i["bx"]) % 8
        assert int(i["round"]) == 1 + min(pi, pj, 7 - pi, 7 - pj), (int(i["by"]), int(i["bx"]))
        assert int(i["n_ctx"]) >= 4


@pytest.mark.parametrize("mode", ["plain", "profile"])
def test_patch_mode_random_loss_parity(ctx, mode):
    """Adjacent lost blocks form larger holes: more rounds, same order."""
    f = synth.make_luma(80, 112, 130, n_bumps=10, n_edges=5)
    m = synth.loss_random(80, 112, 16, 0.3, 131)
    st, info = check(ctx, f, m, mode, window=24, t_nu=0.1, **PATCH)
    assert info["round"].max() >= 4


def test_patch_mode_arbitrary_shape_loss_parity(ctx):
    """2 x 2 cells that keep some received pixels."""
    f = synth.make_luma(64, 80, 140, n_bumps=8, n_edges=4)
    m = synth.loss_partial_cells(64, 80, 2, 0.3, 141, frac=0.6)
    check(ctx, f, m, "profile", window=12, t_nu=0.1, min_hql_cands=16, **PATCH)


def test_patch_mode_distances_bit_exact(ctx):
    import paper_2205_11226_amd as skm
    f, m = _dispersed(80, 112, 150)
    p = skm.patch_params(mode="plain", window=12)
    d, n = ctx.distances_device(to_dev(f), to_dev(m), p)
    d, n = d.cpu().numpy(), n.cpu().numpy()
    op = oracle_params("plain", window=12, **PATCH)
    cells = lost_cells(m, 2)
    assert d.shape[0] == len(cells) == 6 * 64
    for i, (by, bx) in enumerate(cells):
        do, no = block_distances(f.astype(np.int64), m == 0, by, bx, op)
        assert np.array_equal(d[i], do), (by, bx)
        assert np.array_equal(n[i][do >= 0], no[do >= 0])


def test_patch_params_and_cnn_rejection(ctx):
    import paper_2205_11226_amd as skm
    p = skm.patch_params()
    q = skm.default_params()
    assert (p.block, p.ring) == (2, 2)
    assert (p.window, p.expand_step, p.sigma2, p.t_phi, p.t_nu) == \
        (q.window, q.expand_step, q.sigma2, q.t_phi, q.t_nu)
    f = synth.make_luma(64, 64, 160)
    m = synth.loss_dispersed(64, 64, 16)
    with pytest.raises(skm.SkmError) as e:
        ctx.conceal_device(to_dev(f), to_dev(m), skm.patch_params(mode="cnn"))
    assert e.value.status == -1
