"""Pins of the float64 oracle against facts the paper and the mathematics fix.

None of these re-types the oracle's formulas: each checks a closed form, an
invariant, a limit, a special case that reduces to a textbook result, or an
independent loop implementation (``oracle.brute``) on tiny frames.
"""
import json
import math
import os
from dataclasses import replace

import numpy as np
import pytest

import synth
from oracle import brute
from oracle.skmmse import (
    LAYER_BRL, LAYER_HQL, LAYER_IDL, PROFILES, Params, UnsupportedLoss,
    block_context, block_distances, candidate_set, conceal, estimate_block,
    hql_estimate, idl_estimate, idl_radii, log_nu_by_radius, log_weights,
    lost_cells, _cov,
)

GOLD = os.path.join(os.path.dirname(__file__), "golden")
SMALL = dict(block=8, ring=2, window=8, min_hql_cands=8)


def tiny_frame(seed, h=32, w=32):
    return synth.make_luma(h, w, seed, n_bumps=4, n_edges=3, noise_std=3.0)


def cells_mask(h, w, b, cells):
    m = np.zeros((h, w), np.uint8)
    for by, bx in cells:
        m[by * b:(by + 1) * b, bx * b:(bx + 1) * b] = 1
    return m


# ------------------------------------------------------------ fixtures / table

def test_profile_table_matches_paper():
    g = json.load(open(os.path.join(GOLD, "profiles.json")))
    for name in ("express", "efficient", "excellent"):
        assert PROFILES[name] == (g[name]["t_phi"], g[name]["t_nu"])


def test_default_constants_match_paper():
    g = json.load(open(os.path.join(GOLD, "constants.json")))
    p = Params()
    assert p.sigma2 == g["sigma2"] and p.block == g["block"]


def test_dispersed_pattern_is_quarter_loss_with_received_neighbours():
    m = synth.loss_dispersed(1080, 1920, 16)
    cells = lost_cells(m, 16)
    assert len(cells) == 2040
    s = set(cells)
    for by, bx in cells:
        for ddy in (-1, 0, 1):
            for ddx in (-1, 0, 1):
                if (ddy, ddx) != (0, 0):
                    assert (by + ddy, bx + ddx) not in s


def test_lost_pixels_outside_the_cells_are_rejected():
    m = np.zeros((36, 32), np.uint8)
    m[33, 5] = 1                          # rows 32..35 hold no full 8 x 8 cell
    with pytest.raises(UnsupportedLoss):
        lost_cells(m, 8)


def test_any_lost_pixel_makes_its_cell_a_block():
    m = np.zeros((32, 32), np.uint8)
    m[3:9, 3:9] = 1                       # touches cells (0,0) (0,1) (1,0) (1,1)
    m[20, 30] = 1                         # one pixel of cell (2,3)
    assert lost_cells(m, 8) == [(0, 0), (0, 1), (1, 0), (1, 1), (2, 3)]


def partial_mask(h, w, b, seed, frac=0.5, rate=0.25):
    return synth.loss_partial_cells(h, w, b, rate, seed, frac=frac)


def test_received_pixels_of_a_lost_cell_are_kept():
    f = tiny_frame(31, 48, 48)
    m = partial_mask(48, 48, 8, 32, frac=1.0, rate=0.3)
    assert ((m != 0).sum() > 0) and len(lost_cells(m, 8)) > 0
    for mode in ("plain", "profile", "full"):
        out, _, _ = conceal(f, m, Params(block=8, ring=2, window=8, min_hql_cands=8,
                                         mode=mode))
        assert np.array_equal(out[m == 0], f[m == 0])


def test_constant_frame_with_arbitrary_loss_is_restored():
    # every context and prototype holds the same value: BRL gives it, and all
    # IDL distances are 0 so the weighted average of equal prototypes gives it
    f = np.full((48, 48), 93, np.uint8)
    m = partial_mask(48, 48, 8, 33, frac=0.7, rate=0.4)
    for mode in ("plain", "profile", "idl", "brl"):
        out, xh, _ = conceal(f, m, Params(block=8, ring=2, window=8, mode=mode))
        assert np.array_equal(out, f)
        for v in xh.values():
            np.testing.assert_allclose(v, 93.0, rtol=0, atol=1e-12)


def test_received_pixels_of_a_cell_join_the_hql_context():
    f = tiny_frame(34, 40, 40)
    m = cells_mask(40, 40, 8, [(2, 2)])
    m[16, 16] = 0                          # one received pixel in the cell
    p = Params(block=8, ring=2, window=12, min_hql_cands=8, mode="full")
    out, xh, info = conceal(f, m, p)
    (i,) = info
    assert i["layer"] == LAYER_HQL
    assert i["n_ctx"] == (8 + 4) ** 2 - 64 + 1
    assert out[16, 16] == f[16, 16]
    # an affine ramp is reproduced exactly by HQL with the extra context pixel
    yy, xx = np.mgrid[0:40, 0:40]
    ramp = (40 + 2 * yy + 3 * xx).astype(np.uint8)
    out_r, xh_r, info_r = conceal(ramp, m, p)
    assert info_r[0]["layer"] == LAYER_HQL
    np.testing.assert_allclose(xh_r[(2, 2)], ramp[16:24, 16:24], rtol=0, atol=1e-6)


# ------------------------------------------------------------------ distances

def test_distance_equals_norm_decomposition():
    """d_j = |m_j o s0|^2 + |m0 o s_j|^2 - 2 <m0 o s0, m_j o s_j>, s = u - 128."""
    u = tiny_frame(3, 48, 48).astype(np.int64)
    mask = cells_mask(48, 48, 8, [(2, 2), (1, 4), (4, 1)])
    avail = mask == 0
    p = Params(**SMALL)
    for by, bx in [(2, 2), (1, 4), (4, 1)]:
        y0, m0 = block_context(u, avail, by, bx, p)
        c = candidate_set(u, avail, by, bx, p, y0, m0)
        assert c.size > 0
        s0 = np.where(m0, y0 - 128, 0)
        for j in range(c.size):
            sj = np.where(c.m[j], c.y[j] - 128, 0)
            t1 = int((c.m[j] * s0 * s0).sum())
            t2 = int((m0 * sj * sj).sum())
            x = int((s0 * sj).sum())
            assert c.d[j] == t1 + t2 - 2 * x


def test_distance_is_symmetric():
    u = tiny_frame(5, 40, 40)
    b, p = 8, Params(block=8, ring=2, window=16)
    a, bpos = (1, 1), (3, 3)        # 16 px apart: rings do not touch the other block
    d_ab, _ = block_distances(u, cells_mask(40, 40, b, [a]) == 0, a[0], a[1], p)
    d_ba, _ = block_distances(u, cells_mask(40, 40, b, [bpos]) == 0, bpos[0], bpos[1], p)
    dy, dx = (bpos[0] - a[0]) * b, (bpos[1] - a[1]) * b
    W = p.window
    assert d_ab[dy + W, dx + W] == d_ba[-dy + W, -dx + W] >= 0


# --------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed,cells,mode,tnu,win", [
    (11, [(1, 1)], "plain", 0.1, 8),
    (12, [(1, 2), (2, 0)], "profile", 0.1, 8),
    (13, [(0, 0), (2, 2), (3, 1)], "profile", 0.01, 8),
    (14, [(1, 1), (1, 2)], "profile", 100.0, 8),     # adjacent: two rounds
    (15, [(2, 1)], "full", 0.1, 12),                 # |d| >= 10 gives complete rings
    (18, [(1, 1), (2, 2)], "profile", 100.0, 12),    # profile reaching HQL
    (16, [(1, 1), (2, 3)], "idl", 1.0, 8),
    (17, [(1, 1), (2, 1), (3, 1)], "plain", 0.1, 8),  # vertical slice piece
])
def test_vectorised_oracle_equals_loop_oracle(seed, cells, mode, tnu, win):
    f = tiny_frame(seed)
    m = cells_mask(32, 32, 8, cells)
    p = Params(block=8, ring=2, window=win, min_hql_cands=8, t_nu=tnu, mode=mode)
    out, xh, info = conceal(f, m, p)
    bu, bxh, blay = brute.conceal(f.tolist(), m.tolist(), 8, 2, win, t_nu=tnu, min_hql=8,
                                  mode=mode)
    assert np.array_equal(out, np.array(bu, dtype=np.uint8))
    for i in info:
        k = (i["by"], i["bx"])
        assert i["layer"] == blay[k]
        np.testing.assert_allclose(xh[k].ravel(), np.array(bxh[k]), rtol=0, atol=1e-9)


@pytest.mark.parametrize("seed,mode,tnu,win,frac", [
    (41, "plain", 0.1, 8, 1.0),
    (42, "profile", 0.1, 8, 0.5),
    (43, "profile", 100.0, 12, 0.5),
    (44, "idl", 1.0, 8, 0.8),
    (45, "full", 0.1, 12, 0.5),
    (46, "brl", 0.1, 8, 1.0),
])
def test_partial_loss_vectorised_oracle_equals_loop_oracle(seed, mode, tnu, win, frac):
    f = tiny_frame(seed)
    m = partial_mask(32, 32, 8, seed + 100, frac=frac, rate=0.35)
    p = Params(block=8, ring=2, window=win, min_hql_cands=8, t_nu=tnu, mode=mode)
    out, xh, info = conceal(f, m, p)
    bu, bxh, blay = brute.conceal(f.tolist(), m.tolist(), 8, 2, win, t_nu=tnu, min_hql=8,
                                  mode=mode)
    assert len(info) == len(lost_cells(m, 8)) > 0
    assert np.array_equal(out, np.array(bu, dtype=np.uint8))
    for i in info:
        k = (i["by"], i["bx"])
        assert i["layer"] == blay[k]
        # HQL: Cholesky solves and 40 golden-section steps in two summation
        # orders differ by up to ~2e-8
        tol = 1e-7 if i["layer"] == LAYER_HQL else 1e-9
        np.testing.assert_allclose(xh[k].ravel(), np.array(bxh[k]), rtol=0, atol=tol)


def test_hql_vectorised_equals_loop_version():
    f = tiny_frame(21, 40, 40)
    m = cells_mask(40, 40, 8, [(2, 2)])
    p = Params(block=8, ring=2, window=12, min_hql_cands=8, mode="full")
    u = f.astype(np.int64)
    avail = m == 0
    y0, m0 = block_context(u, avail, 2, 2, p)
    c = candidate_set(u, avail, 2, 2, p, y0, m0)
    comp = c.n == m0.sum()
    assert comp.sum() >= 20
    xs, ys = c.x[comp], c.y[comp][:, m0]
    v = hql_estimate(xs, ys, y0[m0], c.d[comp], p.ridge_rel)
    w = brute.hql(xs.tolist(), ys.tolist(), y0[m0].tolist(), c.d[comp].tolist(), p.ridge_rel)
    np.testing.assert_allclose(v, w, rtol=0, atol=1e-8)


# ------------------------------------------------------------ IDL invariants

def _block_cands(seed=7, sigma2=10.0):
    u = tiny_frame(seed, 48, 48).astype(np.int64)
    m = cells_mask(48, 48, 8, [(2, 3)])
    p = Params(block=8, ring=2, window=8, sigma2=sigma2)
    y0, m0 = block_context(u, m == 0, 2, 3, p)
    return candidate_set(u, m == 0, 2, 3, p, y0, m0), p


def test_idl_weights_sum_to_one():
    c, p = _block_cands()
    c.x = np.ones_like(c.x)
    v = idl_estimate(c, np.ones(c.size, bool), p.sigma2)
    np.testing.assert_allclose(v, 1.0, rtol=0, atol=1e-12)


def test_bandwidth_to_zero_gives_nearest_patch_copy():
    c, p = _block_cands()
    delta = c.d / c.n
    best = delta == delta.min()
    v = idl_estimate(c, np.ones(c.size, bool), 1e-9)
    np.testing.assert_allclose(v, c.x[best].mean(axis=0), rtol=0, atol=1e-9)


def test_bandwidth_to_infinity_gives_candidate_mean():
    c, p = _block_cands()
    v = idl_estimate(c, np.ones(c.size, bool), 1e15)
    np.testing.assert_allclose(v, c.x.mean(axis=0), rtol=0, atol=1e-6)


def test_single_candidate_returns_its_own_block():
    f = tiny_frame(9, 8, 24)
    m = cells_mask(8, 24, 8, [(0, 2)])
    p = Params(block=8, ring=2, window=8, mode="plain")
    out, xh, info = conceal(f, m, p)
    assert info[0]["n_cand"] == 1
    np.testing.assert_array_equal(xh[(0, 2)], f[:, 8:16].astype(float))


def test_log_nu_is_monotone_and_matches_naive_sum():
    c, p = _block_cands(seed=8)
    lnu = log_nu_by_radius(c, p)
    assert all(b >= a for a, b in zip(lnu, lnu[1:]))
    ell = log_weights(c, p.sigma2)
    for rho, v in zip(idl_radii(p), lnu):
        s = float(np.exp(ell[c.radius <= rho]).sum())
        if s > 1e-300:
            assert abs(math.log(s) - v) < 1e-9


def test_expansion_threshold_limits():
    f = tiny_frame(31)
    m = cells_mask(32, 32, 8, [(1, 1), (2, 2)])
    base = dict(block=8, ring=2, window=8, min_hql_cands=8, t_phi=-1.0)
    p0 = Params(**base, t_nu=0.0, mode="profile")
    _, _, inf0 = conceal(f, m, p0)
    for i in inf0:
        # first schedule radius that holds a candidate (B = 8: none within 4 px)
        u = f.astype(np.int64)
        y0, m0 = block_context(u, m == 0, i["by"], i["bx"], p0)
        rmin = candidate_set(u, m == 0, i["by"], i["bx"], p0, y0, m0).radius.min()
        first = min(r for r in idl_radii(p0) if r >= rmin)
        assert i["layer"] == LAYER_IDL and i["radius"] == first == 8
    _, _, infi = conceal(f, m, Params(**base, t_nu=math.inf, mode="profile"))
    assert all(i["layer"] in (LAYER_HQL,) or i["flags"] for i in infi)


def test_gate_limits():
    f = tiny_frame(32)
    m = cells_mask(32, 32, 8, [(1, 1), (2, 3)])
    base = dict(block=8, ring=2, window=8, min_hql_cands=8)
    _, _, inf = conceal(f, m, Params(**base, t_phi=255, mode="profile"))
    assert all(i["layer"] == LAYER_BRL for i in inf)
    o1, x1, _ = conceal(f, m, Params(**base, t_phi=-1, t_nu=math.inf, mode="profile"))
    o2, x2, _ = conceal(f, m, Params(**base, mode="full"))
    assert np.array_equal(o1, o2)
    for k in x1:
        assert np.array_equal(x1[k], x2[k])


def test_brl_is_context_mean_and_phi_is_range():
    f = tiny_frame(33)
    m = cells_mask(32, 32, 8, [(1, 1)])
    _, xh, inf = conceal(f, m, Params(block=8, ring=2, window=8, mode="brl"))
    ring = f[6:18, 6:18].astype(float).copy()
    ring[2:10, 2:10] = np.nan
    vals = ring[~np.isnan(ring)]
    assert vals.size == 12 * 12 - 64
    np.testing.assert_allclose(xh[(1, 1)], vals.mean(), rtol=0, atol=1e-12)
    assert inf[0]["phi"] == vals.max() - vals.min()


# ------------------------------------------------------- whole-method pins

@pytest.mark.parametrize("mode", ["plain", "profile", "full", "brl", "idl"])
def test_constant_image_is_reproduced(mode):
    f = np.full((40, 40), 77, np.uint8)
    m = cells_mask(40, 40, 8, [(1, 1), (3, 2)])
    out, xh, _ = conceal(f, m, Params(block=8, ring=2, window=8, min_hql_cands=8,
                                      t_phi=-1, mode=mode))
    assert np.array_equal(out, f)
    for v in xh.values():
        np.testing.assert_allclose(v, 77.0, rtol=0, atol=1e-9)


@pytest.mark.parametrize("mode", ["plain", "profile", "full"])
def test_brightness_shift_shifts_estimate(mode):
    f = (tiny_frame(41, 40, 40).astype(np.int64) * 150 // 255 + 20).astype(np.uint8)
    m = cells_mask(40, 40, 8, [(1, 1), (3, 3)])
    p = Params(block=8, ring=2, window=8, min_hql_cands=8, mode=mode)
    _, x1, i1 = conceal(f, m, p)
    _, x2, i2 = conceal(f + 17, m, p)
    for k in x1:
        np.testing.assert_allclose(x2[k], x1[k] + 17.0, rtol=0, atol=1e-7)
    assert [i["layer"] for i in i1] == [i["layer"] for i in i2]


def test_lost_pixels_are_never_read():
    f = tiny_frame(42)
    m = cells_mask(32, 32, 8, [(1, 1), (2, 2)])
    g = f.copy()
    g[m > 0] = np.random.default_rng(0).integers(0, 256, size=int(m.sum()))
    p = Params(block=8, ring=2, window=8, min_hql_cands=8, mode="profile")
    assert np.array_equal(conceal(f, m, p)[0], conceal(g, m, p)[0])


# -------------------------------------------------------------------- HQL

def _ramp_case():
    yy, xx = np.mgrid[0:64, 0:64]
    f = (2 * xx + yy + 10).astype(np.uint8)
    m = cells_mask(64, 64, 8, [(3, 3)])
    p = Params(block=8, ring=2, window=12, min_hql_cands=8, mode="full")
    return f, m, p


def test_hql_reproduces_affine_ramp():
    f, m, p = _ramp_case()
    _, xh, inf = conceal(f, m, p)
    assert inf[0]["layer"] == LAYER_HQL
    np.testing.assert_allclose(xh[(3, 3)], f[24:32, 24:32], rtol=0, atol=1e-6)


def _hql_parts(seed=51):
    u = tiny_frame(seed, 48, 48).astype(np.int64)
    m = cells_mask(48, 48, 8, [(2, 2)])
    p = Params(block=8, ring=2, window=12)
    y0, m0 = block_context(u, m == 0, 2, 2, p)
    c = candidate_set(u, m == 0, 2, 2, p, y0, m0)
    comp = c.n == m0.sum()
    xs, ys = c.x[comp].astype(float), c.y[comp][:, m0].astype(float)
    v, parts = hql_estimate(xs, ys, y0[m0], c.d[comp], p.ridge_rel, return_parts=True)
    return xs, ys, y0[m0].astype(float), c.d[comp], v, parts, p


def test_hql_is_kde_conditional_mean_when_alpha_is_one():
    """x~ + A (y0 - y~) = sum_j w_j (x_j + A (y0 - y_j)) (identity behind eq. kmmse)."""
    xs, ys, y0, d, _, parts, p = _hql_parts()
    v1 = hql_estimate(xs, ys, y0, d, p.ridge_rel, alpha_override=1.0)
    w, A = parts["w"], parts["A"]
    ref = np.zeros(xs.shape[1])
    for j in range(xs.shape[0]):
        ref += w[j] * (xs[j] + A @ (y0 - ys[j]))
    np.testing.assert_allclose(v1, ref, rtol=0, atol=1e-9)


def test_hql_alpha_zero_is_mahalanobis_kernel_regression():
    xs, ys, y0, d, _, parts, p = _hql_parts()
    v0 = hql_estimate(xs, ys, y0, d, p.ridge_rel, alpha_override=0.0)
    np.testing.assert_allclose(v0, parts["w"] @ xs, rtol=0, atol=1e-9)


def test_hql_alpha_is_argmin_of_eps_x():
    _, _, _, _, _, parts, _ = _hql_parts()
    ci, ei, a = parts["ci"], parts["ei"], parts["alpha"]

    def epsx(al):
        return float(((ei - al * ci) ** 2).sum())
    for da in (1e-3, 1e-2, 0.1, 1.0):
        assert epsx(a) <= epsx(a + da) and epsx(a) <= epsx(a - da)
    scan = np.linspace(a - 2, a + 2, 4001)
    assert abs(scan[np.argmin([epsx(s) for s in scan])] - a) <= 1e-3 + 1e-12


def test_hql_beta_not_worse_than_any_grid_point():
    _, _, _, _, _, parts, _ = _hql_parts(52)
    e = parts["eps_y"](parts["beta"])
    assert all(e <= g + 1e-12 * max(1.0, g) for g in parts["eps_grid"])


def test_hql_with_indefinite_covariance_falls_back_to_context_mean():
    """A negative ridge (lambda = -tr(C_YY)/N_y + 1e-12) makes C_YY + lambda I
    indefinite for any non-isotropic covariance: the Cholesky factorisation
    meets a pivot <= 0, and the block takes the context mean of eq. mean,
    flagged (both oracles)."""
    from oracle.skmmse import FLAG_HQL_SINGULAR
    f, m = tiny_frame(51, 48, 48), cells_mask(48, 48, 8, [(2, 2), (3, 4)])
    p = Params(block=8, ring=2, window=12, min_hql_cands=8, mode="full", ridge_rel=-1.0)
    out, xh, info = conceal(f, m, p)
    u, av = f.astype(np.int64), m == 0
    for i in info:
        assert i["layer"] == LAYER_BRL and i["flags"] & FLAG_HQL_SINGULAR, i
        assert i["n_complete"] >= 8
        y0, m0 = block_context(u, av, i["by"], i["bx"], p)
        np.testing.assert_allclose(xh[(i["by"], i["bx"])], y0[m0].mean(), rtol=0, atol=1e-12)
    bu, bxh, blay = brute.conceal(f.tolist(), m.tolist(), 8, 2, 12, min_hql=8, mode="full",
                                  ridge_rel=-1.0)
    assert np.array_equal(out, np.array(bu, dtype=np.uint8))
    assert all(v == LAYER_BRL for v in blay.values())
    # the default ridge keeps the same blocks on HQL
    _, _, info_d = conceal(f, m, replace(p, ridge_rel=1e-3))
    assert all(i["layer"] == LAYER_HQL and not i["flags"] for i in info_d)


def test_covariance_matches_numpy_cov():
    z = np.random.default_rng(3).integers(0, 256, size=(50, 7)).astype(float)
    np.testing.assert_allclose(_cov(z), np.cov(z, rowvar=False, bias=True), atol=1e-9)


def test_oracle_runs_plain_512_workload_in_seconds():
    f, m = synth.workload_plain_512()
    assert len(lost_cells(m, 16)) == 64
    out, xh, inf = conceal(f, m, Params(mode="plain"))
    assert len(inf) == 64 and all(i["layer"] == LAYER_IDL for i in inf)
    assert all(i["n_cand"] > 0 for i in inf)


# -------------------------------------------- the paper's 2 x 2 patch mode

PATCH = dict(block=2, ring=2)


def test_patch_mode_fills_a_lost_block_from_its_border_to_its_centre():
    """2 x 2 patches with a 6 x 6 context (Sec. "Reconstruction framework"):
    a patch is concealed once its ring holds ring*block known pixels, so the
    round of patch (i, j) of a lost 16 x 16 block is its layer,
    1 + min(i, j, 7 - i, 7 - j) -- the border-to-centre filling order of the
    paper's filling-order figure."""
    f = tiny_frame(61, 48, 48)
    m = cells_mask(48, 48, 16, [(1, 1)])
    p = Params(window=12, mode="plain", **PATCH)
    out, xh, info = conceal(f, m, p)
    assert len(info) == 64
    for i in info:
        pi, pj = i["by"] - 8, i["bx"] - 8
        assert i["round"] == 1 + min(pi, pj, 7 - pi, 7 - pj)
        assert i["n_ctx"] >= 4
    assert np.array_equal(out[m == 0], f[m == 0])


@pytest.mark.parametrize("seed,mode,tnu,win", [
    (71, "plain", 0.1, 8),
    (72, "profile", 0.1, 8),
    (73, "profile", 100.0, 10),        # profile reaching HQL
    (74, "full", 0.1, 10),
])
def test_patch_mode_vectorised_oracle_equals_loop_oracle(seed, mode, tnu, win):
    f = tiny_frame(seed)
    m = cells_mask(32, 32, 8, [(1, 1), (2, 3)])
    p = Params(window=win, min_hql_cands=8, t_nu=tnu, mode=mode, **PATCH)
    out, xh, info = conceal(f, m, p)
    bu, bxh, blay = brute.conceal(f.tolist(), m.tolist(), 2, 2, win, t_nu=tnu, min_hql=8,
                                  mode=mode)
    assert np.array_equal(out, np.array(bu, dtype=np.uint8))
    assert len(info) == 32
    for i in info:
        k = (i["by"], i["bx"])
        assert i["layer"] == blay[k]
        # HQL: eps_y is flat to rounding (1e-14 relative) within ~1e-7 of
        # log beta at the minimum, so a search by function values fixes beta
        # only that far, and x-hat moves by up to ~15 per unit of log beta
        # with 32 context pixels: two summation orders agree to ~1e-5
        tol = 1e-5 if i["layer"] == LAYER_HQL else 1e-9
        np.testing.assert_allclose(xh[k].ravel(), np.array(bxh[k]), rtol=0, atol=tol)
    if mode == "full":
        assert any(i["layer"] == LAYER_HQL for i in info)


def test_hql_flat_eps_minimum_takes_its_smallest_beta():
    """As beta -> 0 the weights of eq. weights become one-hot on the nearest
    candidate and eps_y (eq. epsy) saturates at ||y0 - y_nearest||^2, so its
    argmin is not unique; the smallest grid beta on the flat part is taken
    (the refinement inside the flat part does not count as better)."""
    f = synth.make_luma(80, 112, 112, n_bumps=10, n_edges=5)
    m = synth.loss_dispersed(80, 112, 16, ox=1, oy=1)
    p = Params(window=12, **PATCH)
    u, av = f.astype(np.int64), m == 0
    y0, m0 = block_context(u, av, 12, 24, p)
    c = candidate_set(u, av, 12, 24, p, y0, m0)
    comp = c.n == m0.sum()
    ys = c.y[comp][:, m0].astype(float)
    _, parts = hql_estimate(c.x[comp].astype(float), ys, y0[m0].astype(float), c.d[comp],
                            p.ridge_rel, return_parts=True)
    eg = parts["eps_grid"]
    near = float(((ys[np.argmin(parts["dmah0"])] - y0[m0]) ** 2).sum())
    assert eg[0] == pytest.approx(near, rel=1e-12)          # saturated at the nearest context
    assert abs(eg[1] - eg[0]) < 1e-9 * eg[0] and min(eg) >= eg[0] * (1 - 1e-12)
    assert parts["beta"] == parts["grid"][0]


@pytest.mark.parametrize("seed,mode,tnu", [(81, "profile", 0.1), (82, "full", 0.1)])
def test_patch_mode_partial_cells_vectorised_oracle_equals_loop_oracle(seed, mode, tnu):
    """2 x 2 cells that keep some received pixels: those join the context,
    are never overwritten, and both oracles agree."""
    f = tiny_frame(seed)
    m = synth.loss_partial_cells(32, 32, 2, 0.3, seed + 100, frac=0.6)
    p = Params(window=8, min_hql_cands=8, t_nu=tnu, mode=mode, **PATCH)
    out, xh, info = conceal(f, m, p)
    bu, bxh, blay = brute.conceal(f.tolist(), m.tolist(), 2, 2, 8, t_nu=tnu, min_hql=8,
                                  mode=mode)
    assert len(info) == len(lost_cells(m, 2)) > 0
    assert np.array_equal(out, np.array(bu, dtype=np.uint8))
    assert np.array_equal(out[m == 0], f[m == 0])
    for i in info:
        k = (i["by"], i["bx"])
        assert i["layer"] == blay[k]
        tol = 1e-5 if i["layer"] == LAYER_HQL else 1e-9
        np.testing.assert_allclose(xh[k].ravel(), np.array(bxh[k]), rtol=0, atol=tol)


def test_cnn_mode_takes_the_flatness_test_before_the_gate():
    """CNN mode: a block whose known context is flat (phi = max - min <=
    T_phi, the profile rule's BRL test) takes BRL, the context mean, and the
    gate is never asked; every other block gets exactly the gate's layer.
    A gate that always answers IDL pins the order: with it, flat blocks must
    still be BRL and no non-flat block may be BRL."""
    f = tiny_frame(71, 48, 48)
    f[:16, :16] = 120                          # a flat corner region
    f[2:6, 2:6] = 128                          # phi = 8 around the corner cell
    m = cells_mask(48, 48, 8, [(0, 0), (1, 4), (4, 1), (4, 4)])
    u = np.where(m == 0, f, 0).astype(np.int64)
    avail = m == 0
    p = Params(mode="cnn", t_phi=20.0, **SMALL)
    asked = []

    def gate_idl(uu, aa, by, bx):
        asked.append((by, bx))
        return LAYER_IDL

    flat_seen = 0
    for by, bx in lost_cells(m, 8):
        y0, m0 = block_context(u, avail, by, bx, p)
        known = y0[m0]
        phi = int(known.max() - known.min()) if m0.any() else 0
        n_asked = len(asked)
        xh, info = estimate_block(u, avail, by, bx, p, gate_idl)
        assert info["phi"] == phi
        if phi <= p.t_phi:
            flat_seen += 1
            assert len(asked) == n_asked, (by, bx)
            assert info["layer"] == LAYER_BRL
            assert np.array_equal(xh, np.full(64, known.mean()))
        else:
            assert asked[-1] == (by, bx)
            assert info["layer"] == LAYER_IDL
    assert flat_seen >= 1 and len(asked) >= 1
