"""GPU parity of HQL over partly known candidate contexts (hql_partial)
against the float64 oracle: lattice loss (no complete candidate), slice loss
over several rounds, isolated loss (complete and partial candidates), the
profile rule, and the repair of an indefinite covariance reaching the
context-mean fallback.  The reduction to the complete-context HQL is pinned
on the CPU (tests/test_oracle_partial_hql.py)."""
import numpy as np
import pytest

import synth
from oracle.skmmse import conceal as oracle_conceal
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


def check(ctx, frame, mask, mode, **kw):
    pg = device_params(mode, hql_partial=1, **kw)
    out, info, xh = ctx.conceal_device(to_dev(frame), to_dev(mask), pg)
    out_o, xh_o, info_o = oracle_conceal(frame, mask, oracle_params(mode, hql_partial=True, **kw))
    st = compare(frame, mask, out.cpu().numpy(), info, xh.cpu().numpy(), out_o, xh_o, info_o,
                 kw.get("t_nu", 0.1), kw.get("block", 16), ring=kw.get("ring", 4),
                 window=kw.get("window", 24))
    print(mode, kw, st, flush=True)
    return info, info_o


@pytest.mark.parametrize("b,r,w", [(16, 4, 24), (8, 2, 12)])
def test_lattice_loss_takes_partial_hql(ctx, b, r, w):
    f = synth.make_luma(128, 160, 60 + b, n_bumps=10, n_edges=5, texture=True)
    m = synth.loss_dispersed(128, 160, b)
    info, info_o = check(ctx, f, m, "full", block=b, ring=r, window=w, min_hql_cands=16)
    assert (info["n_complete"] == 0).all()
    assert (info["layer"] == 2).all()


def test_slice_loss_rounds_partial_hql(ctx):
    f = synth.make_luma(96, 128, 70, n_bumps=8, n_edges=4)
    m = synth.loss_slices(96, 128, 8, 0.4, 71)
    info, info_o = check(ctx, f, m, "full", block=8, ring=2, window=12, min_hql_cands=8)
    assert info["round"].max() >= 2
    assert (info["layer"] == 2).sum() >= len(info) // 2


def test_profile_mode_partial_hql_parity(ctx):
    f = synth.make_luma(128, 160, 72, n_bumps=10, n_edges=5, texture=True)
    m = synth.loss_dispersed(128, 160, 16, 1, 1)
    info, _ = check(ctx, f, m, "profile", t_nu=100.0, min_hql_cands=16)
    assert (info["layer"] == 2).any()


def test_isolated_loss_partial_hql_parity(ctx):
    """Isolated blocks: candidates near the block have rings over the block
    itself, so the partial reading takes them next to the complete ones."""
    f = synth.make_luma(256, 256, 74, n_bumps=16, n_edges=6)
    m = np.zeros((256, 256), np.uint8)
    for by, bx in ((3, 3), (3, 12), (12, 3), (12, 12)):
        m[by * 16:(by + 1) * 16, bx * 16:(bx + 1) * 16] = 1
    info, _ = check(ctx, f, m, "full")
    assert (info["layer"] == 2).all()
    assert (info["n_cand"] > info["n_complete"]).all()


def test_partial_hql_indefinite_covariance_falls_back_after_the_repair(ctx):
    """ridge_rel = -1 keeps C_YY + lambda I indefinite at every repair step:
    after the last retry every HQL block takes the context mean, flagged, as
    in the oracle."""
    import paper_2205_11226_amd as skm
    f = synth.make_luma(80, 96, 98, n_bumps=6, n_edges=4)
    m = synth.loss_dispersed(80, 96, 8)
    info, _ = check(ctx, f, m, "full", block=8, ring=2, window=12, min_hql_cands=8,
                    ridge_rel=-1.0)
    sing = (info["flags"] & skm.FLAG_HQL_SINGULAR) != 0
    assert sing.sum() >= 3 and (info["layer"][sing] == 0).all()
