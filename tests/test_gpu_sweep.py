"""GPU: the limiting cases of the layer gate that the threshold sweeps rest
on, and one small run of every sweep setting.

With T_nu out of reach no block accepts IDL, so the profile rule must give
full K-MMSE exactly (HQL where enough complete candidates exist, else IDL over
the whole window); with T_phi above any flatness every block takes BRL.  Both
are compared bit for bit with the forced modes (themselves compared with the
oracle in test_gpu_parity)."""
import math

import numpy as np
import pytest

import sweep
import synth
from tests.parity import device_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    import paper_2205_11226_amd as skm
    assert torch.cuda.is_available()
    c = skm.Context(0)
    yield c
    c.close()


def run(ctx, f, m, prm):
    import torch
    out, info, xh = ctx.conceal_device(torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda(),
                                       prm)
    return out.cpu().numpy(), info, xh.cpu().numpy()


def test_gate_limits_equal_forced_layers(ctx):
    f = synth.make_luma(256, 320, 91, n_bumps=20, n_edges=8, texture=True)
    m = synth.loss_random(256, 320, 16, 0.25, 92)
    o_full, i_full, x_full = run(ctx, f, m, device_params("full"))
    o_lim, i_lim, x_lim = run(ctx, f, m, device_params("profile", t_phi=-1.0, t_nu=sweep.BIG))
    assert np.sum(i_full["layer"] == 2) > 0, "random loss should leave HQL blocks"
    assert np.array_equal(o_full, o_lim)
    assert np.array_equal(x_full, x_lim)
    assert np.array_equal(i_full["layer"], i_lim["layer"])
    assert np.array_equal(i_full["flags"], i_lim["flags"])

    o_brl, i_brl, x_brl = run(ctx, f, m, device_params("brl"))
    o_all, i_all, x_all = run(ctx, f, m, device_params("profile", t_phi=1e9, t_nu=0.1))
    assert np.all(i_all["layer"] == 0)
    assert np.array_equal(o_brl, o_all)
    assert np.array_equal(x_brl, x_all)


def test_sweep_runs_every_setting(ctx):
    rows = sweep.sweep(n_frames=1, reps=1, h=128, w=192)
    summ = sweep.summarise(rows)
    assert len(summ) == 2 * len(sweep.settings())
    for s in summ:
        assert math.isfinite(s["dpsnr"]) and s["speedup"] > 0
        assert s["brl"] + s["idl"] + s["hql"] + s["idl_full"] == pytest.approx(1.0)
    by = {(s["study"], s["label"], s["pattern"]): s for s in summ}
    # the dispersed lattice is concealed in one round, so raising T_phi can
    # only move blocks to BRL (later rounds of random loss start from other
    # concealed pixels)
    brl = [by[("flatness", f"T_phi={t:g}", "dispersed")]["brl"] for t in sweep.T_PHI_SWEEP]
    assert all(b1 >= b0 for b0, b1 in zip(brl, brl[1:]))
    # and raising T_nu can only move blocks from IDL to full K-MMSE, which on
    # the lattice is IDL over the whole window (no complete candidates)
    d2 = [by[("normalisation", f"T_nu={t:g}", "dispersed")] for t in sweep.T_NU_SWEEP]
    assert all(s["hql"] == 0 for s in d2)
    full = [s["idl_full"] for s in d2]
    assert all(b1 >= b0 for b0, b1 in zip(full, full[1:]))
    # BRL only where a block has no admissible candidate, whatever T_nu
    assert len({s["brl"] for s in d2}) == 1
    md = sweep.markdown(summ)
    assert "flatness" in md and "profiles" in md and "excellent" in md


def test_patch_geometry_gate_limit_and_sweep(ctx):
    """The paper's 2x2 patches: with T_nu out of reach and T_phi below any
    flatness the profile rule is full K-MMSE bit for bit, and the sweep runs
    every setting in that geometry."""
    import paper_2205_11226_amd as skm
    f = synth.make_luma(80, 112, 93, n_bumps=10, n_edges=5, texture=True)
    m = synth.loss_dispersed(80, 112, 16, ox=1, oy=1)
    o_full, i_full, x_full = run(ctx, f, m, skm.patch_params(mode="full"))
    o_lim, i_lim, x_lim = run(ctx, f, m, skm.patch_params(mode="profile", t_phi=-1.0,
                                                          t_nu=sweep.BIG))
    assert np.all(i_full["layer"] == 2)
    assert np.array_equal(o_full, o_lim) and np.array_equal(x_full, x_lim)
    assert np.array_equal(i_full["layer"], i_lim["layer"])
    rows = sweep.sweep(n_frames=1, reps=1, h=96, w=128, geometry="patch")
    summ = sweep.summarise(rows)
    assert len(summ) == 2 * len(sweep.settings())
    for s in summ:
        assert math.isfinite(s["dpsnr"]) and s["speedup"] > 0
        assert s["brl"] + s["idl"] + s["hql"] + s["idl_full"] == pytest.approx(1.0)
