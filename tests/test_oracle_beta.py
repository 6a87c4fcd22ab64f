"""Pin of the oracle's beta search (Sec. "K-MMSE overview", eq. epsy).

The bandwidth scale beta minimises the context prediction error
eps_y(beta) = ||y0 - sum_j w_j(beta) y_j||^2 with w_j proportional to
exp(-D(y0, y_j) / (2 beta)) and D the Mahalanobis distance in C_YY.  The
oracle finds it with a coarse grid and a golden-section refinement.  These
tests recompute eps_y independently (np.cov, a direct linear solve, a
log-sum-exp softmax; none of the oracle's helpers) and scan it densely over
log beta:

* over the whole grid range (>= 10^4 points) no scanned beta beats the
  oracle's beta;
* on a fine scan (10^4 points) of one grid step either side of the oracle's
  beta, the oracle's beta lies within one scan step of the scan's argmin
  wherever eps_y is not flat there to 1e-12 (relative).

A search that stops short, walks the wrong way or keeps the grid point fails
the first check or the second; ``test_reversed_golden_comparison_is_caught``
plants such a mistake in the oracle and checks that it is caught.
"""
import math

import numpy as np
import pytest

import synth
from oracle import skmmse
from oracle.skmmse import Params, block_context, candidate_set, hql_estimate

FLAT_REL = 1e-12
N_FULL = 12001
N_FINE = 10001


def _hql_inputs(seed, geom):
    """Complete-candidate HQL inputs (x, y, y0, d) of one block."""
    if geom == "block8":
        u = synth.make_luma(48, 48, seed, n_bumps=4, n_edges=3, noise_std=3.0).astype(np.int64)
        m = np.zeros((48, 48), np.uint8)
        m[16:24, 16:24] = 1
        p = Params(block=8, ring=2, window=12)
        by, bx = 2, 2
    else:                                       # the paper's 2 x 2 patch, 6 x 6 context
        u = synth.make_luma(64, 64, seed, n_bumps=6, n_edges=4, noise_std=2.0).astype(np.int64)
        m = np.zeros((64, 64), np.uint8)
        m[32:34, 30:32] = 1
        p = Params(block=2, ring=2, window=12)
        by, bx = 16, 15
    av = m == 0
    y0, m0 = block_context(u, av, by, bx, p)
    c = candidate_set(u, av, by, bx, p, y0, m0)
    comp = c.n == m0.sum()
    return (c.x[comp].astype(float), c.y[comp][:, m0].astype(float),
            y0[m0].astype(float), c.d[comp], p.ridge_rel)


def _independent_eps(ys, y0, ridge_rel):
    """eps_y(beta) for an array of betas, from the definitions."""
    ny = ys.shape[1]
    cyy = np.atleast_2d(np.cov(ys, rowvar=False, bias=True))
    cyy = cyy + (ridge_rel * np.trace(cyy) / ny + 1e-12) * np.eye(ny)
    diff = y0[None, :] - ys
    dm = np.einsum("jk,jk->j", diff, np.linalg.solve(cyy, diff.T).T)

    def eps(betas):
        betas = np.atleast_1d(np.asarray(betas, dtype=np.float64))
        out = np.empty(betas.shape[0])
        for s in range(0, betas.shape[0], 512):
            lg = -dm[None, :] / (2.0 * betas[s:s + 512, None])
            lg -= lg.max(axis=1, keepdims=True)
            w = np.exp(lg)
            w /= w.sum(axis=1, keepdims=True)
            r = y0[None, :] - w @ ys
            out[s:s + 512] = (r * r).sum(axis=1)
        return out
    return dm, eps


def check_beta(xs, ys, y0, d, ridge_rel):
    """Assert the dense-scan properties; returns whether the location check ran."""
    _, parts = hql_estimate(xs, ys, y0, d, ridge_rel, return_parts=True)
    beta, grid = parts["beta"], parts["grid"]
    dm, eps = _independent_eps(ys, y0, ridge_rel)
    # the Mahalanobis distances through another route (solve, not whitening)
    np.testing.assert_allclose(parts["dmah0"], dm, rtol=1e-8, atol=1e-8)
    e_beta = float(eps(beta)[0])
    # 1. over the whole grid range
    tf = np.linspace(math.log(grid[0]), math.log(grid[-1]), N_FULL)
    ef = eps(np.exp(tf))
    assert e_beta <= float(ef.min()) * (1.0 + FLAT_REL) + 1e-300, (e_beta, float(ef.min()))
    # 2. one grid step (2^(1/2)) either side of beta, finely
    h = 0.5 * math.log(2.0)
    tl = max(math.log(grid[0]), math.log(beta) - h)
    th = min(math.log(grid[-1]), math.log(beta) + h)
    ts = np.linspace(tl, th, N_FINE)
    step = ts[1] - ts[0]
    es = eps(np.exp(ts))
    k = int(np.argmin(es))
    emin = float(es[k])
    assert e_beta <= emin * (1.0 + FLAT_REL) + 1e-300, (e_beta, emin)
    flat = np.nonzero(es <= emin * (1.0 + FLAT_REL))[0]
    if flat.max() - flat.min() > 2:            # flat to 1e-12 over several steps
        return False
    assert abs(math.log(beta) - ts[k]) <= step * (1.0 + 1e-9), (math.log(beta), ts[k], step)
    return True


# blocks whose eps_y minimum lies strictly inside the grid range (the
# refinement decides beta there), in both geometries
INTERIOR = [(57, "block8"), (60, "block8"), (61, "block8"), (64, "block8"), (65, "block8"),
            (69, "block8"), (62, "patch"), (65, "patch"), (66, "patch"), (68, "patch"),
            (72, "patch"), (74, "patch"), (76, "patch"), (78, "patch")]
# the minimum at an end of the grid: beta -> 0 saturation (reading S4b) and
# eps_y still falling at the largest beta
EDGE = [(51, "block8"), (52, "block8")]
CASES = INTERIOR + EDGE


@pytest.mark.parametrize("seed,geom", CASES)
def test_beta_is_the_dense_scan_minimiser(seed, geom):
    xs, ys, y0, d, rr = _hql_inputs(seed, geom)
    assert xs.shape[0] >= 16
    check_beta(xs, ys, y0, d, rr)


def test_dense_scan_location_check_runs_on_non_flat_minima():
    """The location check must not be vacuous: most cases have an isolated
    minimum."""
    ran = sum(check_beta(*_hql_inputs(s, g)) for s, g in INTERIOR)
    assert ran == len(INTERIOR), ran


def _reversed_golden_section(f, a, b, steps):
    # a planted mistake: the bracket moves towards the larger value
    invphi = (math.sqrt(5.0) - 1.0) / 2.0
    c = b - invphi * (b - a)
    d = a + invphi * (b - a)
    fc, fd = f(c), f(d)
    for _ in range(steps):
        if fc >= fd:
            b, d, fd = d, c, fc
            c = b - invphi * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + invphi * (b - a)
            fd = f(d)
    return a, b


def test_reversed_golden_comparison_is_caught(monkeypatch):
    monkeypatch.setattr(skmmse, "golden_section", _reversed_golden_section)
    caught = 0
    for s, g in INTERIOR:
        try:
            check_beta(*_hql_inputs(s, g))
        except AssertionError:
            caught += 1
    assert caught == len(INTERIOR), caught


def test_truncated_golden_search_is_caught(monkeypatch):
    orig = skmmse.golden_section
    monkeypatch.setattr(skmmse, "golden_section", lambda f, a, b, steps: orig(f, a, b, 3))
    caught = 0
    for s, g in INTERIOR:
        try:
            check_beta(*_hql_inputs(s, g))
        except AssertionError:
            caught += 1
    assert caught == len(INTERIOR), caught
