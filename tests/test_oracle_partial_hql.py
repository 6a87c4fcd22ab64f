"""CPU pins of the oracle's HQL over partly known candidate contexts
(reading of Sec. "K-MMSE overview" for candidates whose context ring is not
fully received): the pairwise-complete covariance against loops over
coordinate pairs, the context completion against loops, the PSD repair, and
the reduction to the complete-context HQL."""
import numpy as np
import pytest

import synth
from oracle.skmmse import (Params, block_context, candidate_set, complete_contexts, conceal,
                           hql_estimate, hql_estimate_partial, lost_cells, pairwise_covariance)


def _random_case(seed, m=30, nx=4, ny=9, p_known=0.7):
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 256, size=(m, nx))
    y = rng.integers(0, 256, size=(m, ny))
    o = rng.uniform(size=(m, ny)) < p_known
    return x, y, o


def _pair_cov(za, ka, zb, kb):
    """Covariance of two coordinates over the candidates that know both,
    1/N normalised, written as a loop over candidates."""
    sel = [j for j in range(len(za)) if ka[j] and kb[j]]
    if not sel:
        return 0.0
    n = float(len(sel))
    ma = sum(float(za[j]) for j in sel) / n
    mb = sum(float(zb[j]) for j in sel) / n
    return sum((float(za[j]) - ma) * (float(zb[j]) - mb) for j in sel) / n


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_pairwise_covariance_matches_pair_loops(seed):
    x, y, o = _random_case(seed)
    cxy, cyy = pairwise_covariance(x, y, o)
    m, ny = y.shape
    ones = np.ones(m, dtype=bool)
    for a in range(ny):
        for b in range(ny):
            ref = _pair_cov(y[:, a], o[:, a], y[:, b], o[:, b])
            assert abs(cyy[a, b] - ref) <= 1e-9 * max(1.0, abs(ref)), (a, b)
    for q in range(x.shape[1]):
        for b in range(ny):
            ref = _pair_cov(x[:, q], ones, y[:, b], o[:, b])
            assert abs(cxy[q, b] - ref) <= 1e-9 * max(1.0, abs(ref)), (q, b)


def test_pairwise_covariance_of_complete_data_is_the_covariance():
    x, y, _ = _random_case(7, m=40)
    o = np.ones_like(y, dtype=bool)
    cxy, cyy = pairwise_covariance(x, y, o)
    c = np.cov(np.concatenate([x, y], axis=1).T.astype(np.float64), bias=True)
    nx = x.shape[1]
    np.testing.assert_allclose(cyy, c[nx:, nx:], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(cxy, c[:nx, nx:], rtol=1e-12, atol=1e-9)


def test_pairwise_covariance_without_common_candidates_is_zero():
    y = np.array([[10, 0], [20, 0], [0, 5], [0, 9]])
    o = np.array([[1, 0], [1, 0], [0, 1], [0, 1]], dtype=bool)
    x = np.array([[1], [2], [3], [4]])
    _, cyy = pairwise_covariance(x, y, o)
    assert cyy[0, 1] == 0.0 and cyy[1, 0] == 0.0
    assert cyy[0, 0] == 25.0 and cyy[1, 1] == 4.0


def test_complete_contexts_matches_loops():
    x, y, o = _random_case(11, m=20, ny=7, p_known=0.5)
    o[:, 3] = False                                   # a coordinate nobody knows
    y0 = np.arange(7) * 10
    yc = complete_contexts(y, o, y0)
    for a in range(7):
        known = [int(y[j, a]) for j in range(20) if o[j, a]]
        if known:
            s, n = sum(known), len(known)
            fill = (2 * s + n) // (2 * n)             # round half up
            assert fill == int(np.floor(s / n + 0.5))
        else:
            fill = int(y0[a])
        for j in range(20):
            assert yc[j, a] == (y[j, a] if o[j, a] else fill), (j, a)


def _complete_block():
    f, m = synth.workload_plain_512()
    p = Params(mode="full")
    u = np.where(m == 0, f, 0).astype(np.int64)
    av = m == 0
    by, bx = lost_cells(m, 16)[0]
    y0, m0 = block_context(u, av, by, bx, p)
    c = candidate_set(u, av, by, bx, p, y0, m0)
    return c, y0, m0


def test_partial_hql_reduces_to_hql_on_complete_contexts():
    c, y0, m0 = _complete_block()
    comp = c.n == int(m0.sum())
    assert comp.sum() >= 64
    xs, ys = c.x[comp], c.y[comp][:, m0]
    ref = hql_estimate(xs, ys, y0[m0], c.d[comp], 1e-3)
    got = hql_estimate_partial(xs, ys, np.ones_like(ys, dtype=bool), y0[m0], c.d[comp],
                               c.n[comp], 1e-3)
    assert np.abs(got - ref).max() <= 1e-7


def test_psd_repair_raises_lambda_until_the_factorisation_holds():
    # three coordinates whose pairs are seen by disjoint candidate sets: a = b
    # (candidates 0-5), b = c (6-11), c = 255 - a (12-17) -- no joint
    # distribution has these pairwise correlations, the estimate is indefinite
    rng = np.random.default_rng(5)
    v = rng.integers(0, 256, size=18)
    y = np.zeros((18, 3), dtype=np.int64)
    o = np.zeros((18, 3), dtype=bool)
    y[:6, 0] = y[:6, 1] = v[:6]; o[:6, :2] = True
    y[6:12, 1] = y[6:12, 2] = v[6:12]; o[6:12, 1:] = True
    y[12:, 0] = v[12:]; y[12:, 2] = 255 - v[12:]; o[12:, 0] = o[12:, 2] = True
    x = rng.integers(0, 256, size=(18, 2))
    _, cyy = pairwise_covariance(x, y, o)
    assert np.linalg.eigvalsh(cyy).min() < 0.0
    y0 = np.array([100, 110, 120])
    d = np.arange(18) + 1
    n = o.sum(axis=1)
    xh, parts = hql_estimate_partial(x, y, o, y0, d, n, 1e-3, return_parts=True)
    lam0 = 1e-3 * np.trace(cyy) / 3 + 1e-12
    lam = parts["lam"]
    k = round(np.log10(lam / lam0))
    assert k >= 1 and abs(lam - lam0 * 10.0 ** k) <= 1e-9 * lam
    with pytest.raises(np.linalg.LinAlgError):
        np.linalg.cholesky(cyy + (lam / 10.0) * np.eye(3))
    assert np.all(np.isfinite(xh))


def test_partial_hql_on_a_lattice_frame():
    """On a 25 % lattice no candidate context is complete: HQL over partial
    contexts is available; a constant frame is reproduced and a brightness
    shift shifts the estimate."""
    f = synth.make_luma(96, 96, 41, n_bumps=6, n_edges=3)
    f = np.clip(f, 20, 200).astype(np.uint8)
    m = synth.loss_dispersed(96, 96, 16)
    p = Params(mode="full", hql_partial=True, min_hql_cands=16)
    out, xh, info = conceal(f, m, p)
    assert all(i["n_complete"] == 0 for i in info)
    assert all(i["layer"] == 2 for i in info)
    out2, xh2, _ = conceal((f.astype(np.int64) + 30).astype(np.uint8), m, p)
    for k in xh:
        assert np.abs(xh2[k] - xh[k] - 30.0).max() <= 1e-6, k
    c = np.full((96, 96), 77, np.uint8)
    out3, xh3, _ = conceal(c, m, p)
    for k in xh3:
        assert np.abs(xh3[k] - 77.0).max() <= 1e-9, k
    # the complete-context reading keeps its IDL fallback on the same frame
    _, _, info4 = conceal(f, m, Params(mode="full", min_hql_cands=16))
    assert all(i["layer"] == 1 for i in info4)
