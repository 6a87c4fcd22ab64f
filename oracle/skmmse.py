"""Float64 CPU oracle of K-MMSE and scalable K-MMSE concealment.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Paper: Koloda, Seiler, Peinado, Kaup, "Scalable Kernel-Based Minimum Mean
Square Error Estimator for Accelerated Image Error Concealment" (arXiv
2205.11226).  Section names below refer to it.

Geometry (block mode).  The paper estimates 2x2 patches from a 6x6 context
(Sec. "Reconstruction framework").  Here a B x B cell of the block grid that
holds any lost pixel is x0; its context y0 is the ring of width r around it
and the cell's own received pixels (the paper's loss patterns may have any
shape, Sec. "Reconstruction framework"), restricted to available pixels (mask
m0); candidates z_j are all displacements (dx, dy) in [-W, W]^2 whose B x B
prototype does not overlap the cell, lies in the frame and is fully
available.  A candidate's
ring may be partly unavailable: its distance to y0 is taken over the pixels
known in both rings (count n_j) and normalised by n_j, the "average
distortion per context pixel" that the IDL bandwidth sigma^2 N_y expresses
(Sec. "Intermediate dynamic layer").  Candidates with n_j below
ceil(min_overlap_pct * |m0| / 100) are dropped.  HQL, whose covariance needs
every coordinate, uses only candidates whose context covers all of m0.

Layers and gate (Sec. "Scalable K-MMSE estimator", Sec. "Layer switching"):
* BRL: mean of y0 (eq. "mean"), chosen when phi = max(y0) - min(y0) <= T_phi;
* IDL: fixed bandwidth sigma^2 = 10 kernel regression (eq. "slpe") over the
  candidates within Chebyshev radius rho, rho growing in steps of
  ``expand_step`` up to W; accepted at the first rho whose
  nu = sum of raw weights (eq. "factor", read with a negative exponent)
  reaches T_nu;
* HQL: full K-MMSE with covariance-scaled bandwidth (eqs. "kmmse",
  "weights", "bandwidthScaled", "epsy", "epsx").

Lost blocks are concealed in Jacobi rounds: every block whose available
context holds at least r*B pixels is estimated from the state at the start of
the round, then its lost pixels take the rounded estimates and become
available (the transfer of x0 into S, end of Sec. "K-MMSE overview"); its
received pixels are never changed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np

LAYER_FILL = -1
LAYER_BRL = 0
LAYER_IDL = 1
LAYER_HQL = 2

FLAG_CTX_RELAXED = 1   # block proceeded with fewer than r*B context pixels
FLAG_NO_HQL = 2        # HQL wanted but too few complete candidates: full IDL
FLAG_NO_CAND = 4       # no candidate at all: BRL
FLAG_EMPTY_CTX = 8     # forced fill with no context pixel: frame mean
FLAG_HQL_SINGULAR = 16  # HQL's C_YY + lambda I not positive definite in float64: BRL

# Profile table of the paper (Table "Profile definitions"): (T_phi, T_nu).
PROFILES = {
    "express": (20.0, 0.01),
    "efficient": (20.0, 0.1),
    "excellent": (20.0, 100.0),
}

MODES = ("plain", "full", "profile", "brl", "idl", "cnn")


class UnsupportedLoss(ValueError):
    """Loss mask with lost pixels outside the in-frame B x B cells."""


@dataclass(frozen=True)
class Params:
    block: int = 16
    ring: int = 4
    window: int = 24
    sigma2: float = 10.0          # IDL decay factor (Sec. IDL: set to 10)
    t_phi: float = 20.0
    t_nu: float = 0.1
    expand_step: int = 4
    min_overlap_pct: int = 50
    min_hql_cands: int = 64
    ridge_rel: float = 1e-3
    mode: str = "profile"
    max_rounds: int = 0           # 0 = until every block is concealed
    # HQL over every admissible candidate, completing partly known candidate
    # contexts (hql_estimate_partial); False: complete candidates only
    hql_partial: bool = False

    def with_profile(self, name: str) -> "Params":
        tphi, tnu = PROFILES[name]
        return replace(self, t_phi=tphi, t_nu=tnu)


# ------------------------------------------------------------------ geometry

def ring_offsets(b: int, r: int) -> np.ndarray:
    """(oy, ox) of the context ring around a B x B block, raster order."""
    out = [(oy, ox) for oy in range(-r, b + r) for ox in range(-r, b + r)
           if not (0 <= oy < b and 0 <= ox < b)]
    return np.asarray(out, dtype=np.int64).reshape(-1, 2)


def context_offsets(b: int, r: int) -> np.ndarray:
    """(oy, ox) of every context position: the ring (raster order), then the
    block's own B x B positions (raster order), which count where received."""
    inner = [(oy, ox) for oy in range(b) for ox in range(b)]
    return np.concatenate([ring_offsets(b, r),
                           np.asarray(inner, dtype=np.int64).reshape(-1, 2)])


def lost_cells(mask: np.ndarray, b: int) -> list[tuple[int, int]]:
    """Cells (by, bx) in raster order that hold at least one lost pixel; every
    lost pixel must lie in a B x B cell that is entirely inside the frame."""
    h, w = mask.shape
    lost = mask != 0
    gh, gw = h // b, w // b
    cells = []
    covered = np.zeros_like(lost)
    covered[:gh * b, :gw * b] = True
    if (lost & ~covered).any():
        raise UnsupportedLoss("lost pixels outside the in-frame B x B cells")
    for by in range(gh):
        for bx in range(gw):
            if lost[by * b:(by + 1) * b, bx * b:(bx + 1) * b].any():
                cells.append((by, bx))
    return cells


def _gather(u: np.ndarray, avail: np.ndarray, ys: np.ndarray, xs: np.ndarray):
    """Pixel values and availability at (ys, xs); out-of-frame = unavailable."""
    h, w = u.shape
    inside = (ys >= 0) & (ys < h) & (xs >= 0) & (xs < w)
    yc = np.clip(ys, 0, h - 1)
    xc = np.clip(xs, 0, w - 1)
    m = inside & avail[yc, xc]
    v = np.where(m, u[yc, xc], 0).astype(np.int64)
    return v, m


def block_context(u, avail, by, bx, p: Params):
    """Context y0 and its mask m0 over the ring and the block's own positions
    (values 0 where unknown)."""
    off = context_offsets(p.block, p.ring)
    return _gather(u, avail, by * p.block + off[:, 0], bx * p.block + off[:, 1])



@dataclass
class Candidates:
    dx: np.ndarray        # displacement, raster order (dy, then dx)
    dy: np.ndarray
    n: np.ndarray         # |m0 and m_j|
    d: np.ndarray         # sum over m0 and m_j of (y0 - y_j)^2, exact integer
    x: np.ndarray         # (M, B*B) prototypes
    y: np.ndarray         # (M, N_ctx) context vectors (0 where unknown)
    m: np.ndarray         # (M, N_ctx) candidate context availability

    @property
    def size(self) -> int:
        return int(self.dx.shape[0])

    @property
    def radius(self) -> np.ndarray:
        return np.maximum(np.abs(self.dx), np.abs(self.dy))


def candidate_set(u, avail, by, bx, p: Params, y0, m0) -> Candidates:
    """All admissible candidates of block (by, bx) with their exact distances.

    A displacement is admissible when its prototype does not overlap the
    block, is in the frame and fully available, and its context shares at
    least ceil(min_overlap_pct |m0| / 100) (and at least one) known pixels
    with m0.  At the block's own positions a candidate's context is its
    prototype (always available).
    """
    b, W = p.block, p.window
    h, w = u.shape
    off = context_offsets(b, p.ring)
    n0 = int(m0.sum())
    nmin = max(1, (p.min_overlap_pct * n0 + 99) // 100)
    dys, dxs = np.meshgrid(np.arange(-W, W + 1), np.arange(-W, W + 1), indexing="ij")
    dys = dys.ravel()
    dxs = dxs.ravel()
    keep = ~((np.abs(dys) < b) & (np.abs(dxs) < b))
    dys, dxs = dys[keep], dxs[keep]
    py = by * b + dys
    px = bx * b + dxs
    inside = (py >= 0) & (px >= 0) & (py + b <= h) & (px + b <= w)
    # prototype availability from an integral image of the lost indicator,
    # taken over the part of the frame the prototypes can reach
    y_lo, x_lo = max(0, by * b - W), max(0, bx * b - W)
    y_hi, x_hi = min(h, by * b + b + W), min(w, bx * b + b + W)
    lost = ~avail[y_lo:y_hi, x_lo:x_hi]
    lost_ii = np.zeros((lost.shape[0] + 1, lost.shape[1] + 1), dtype=np.int64)
    lost_ii[1:, 1:] = np.cumsum(np.cumsum(lost, axis=0), axis=1)
    pyc = np.clip(py, y_lo, max(y_lo, y_hi - b)) - y_lo
    pxc = np.clip(px, x_lo, max(x_lo, x_hi - b)) - x_lo
    nlost = (lost_ii[pyc + b, pxc + b] - lost_ii[pyc, pxc + b]
             - lost_ii[pyc + b, pxc] + lost_ii[pyc, pxc])
    ok = inside & (nlost == 0)
    dys, dxs, py, px = dys[ok], dxs[ok], py[ok], px[ok]
    ry = py[:, None] + off[None, :, 0]
    rx = px[:, None] + off[None, :, 1]
    yj, mj = _gather(u, avail, ry, rx)
    both = mj & m0[None, :]
    n = both.sum(axis=1)
    diff = np.where(both, y0[None, :] - yj, 0)
    d = (diff * diff).sum(axis=1)
    sel = n >= nmin
    ii = np.arange(b)
    xy = py[sel][:, None, None] + ii[None, :, None]
    xx = px[sel][:, None, None] + ii[None, None, :]
    xproto = u[xy, xx].reshape(-1, b * b).astype(np.int64)
    return Candidates(dx=dxs[sel], dy=dys[sel], n=n[sel], d=d[sel], x=xproto,
                      y=yj[sel], m=mj[sel])


def block_distances(u, avail, by, bx, p: Params):
    """Exact integer distance table over every displacement, for parity.

    Returns (d, n) of shape (2W+1, 2W+1) indexed [dy+W, dx+W]; d = -1 where
    the displacement is not an admissible candidate.
    """
    y0, m0 = block_context(u, avail, by, bx, p)
    c = candidate_set(u, avail, by, bx, p, y0, m0)
    W = p.window
    d = np.full((2 * W + 1, 2 * W + 1), -1, dtype=np.int64)
    n = np.zeros((2 * W + 1, 2 * W + 1), dtype=np.int64)
    d[c.dy + W, c.dx + W] = c.d
    n[c.dy + W, c.dx + W] = c.n
    return d, n


# ---------------------------------------------------------------- IDL / nu

def log_weights(c: Candidates, sigma2: float) -> np.ndarray:
    """ell_j = -(d_j / n_j) / (2 sigma^2): log of the raw IDL weight (eq. slpe
    with N_y replaced by the per-candidate overlap n_j)."""
    return -(c.d.astype(np.float64) / c.n.astype(np.float64)) / (2.0 * sigma2)


def _logsumexp(v: np.ndarray) -> float:
    if v.size == 0:
        return -math.inf
    m = float(v.max())
    return m + math.log(float(np.exp(v - m).sum()))


def idl_radii(p: Params) -> list[int]:
    """Expansion schedule of the support area: Chebyshev radii step, 2 step,
    ..., W (the expansion map itself is not legible in the paper)."""
    rs = list(range(p.expand_step, p.window, p.expand_step))
    rs.append(p.window)
    return rs


def log_nu_by_radius(c: Candidates, p: Params) -> list[float]:
    """log nu(rho) = log sum_{rho_j <= rho} exp(ell_j) for each rho (eq. factor)."""
    ell = log_weights(c, p.sigma2)
    rad = c.radius
    return [_logsumexp(ell[rad <= rho]) for rho in idl_radii(p)]


def idl_estimate(c: Candidates, sel: np.ndarray, sigma2: float) -> np.ndarray:
    """Normalised-weight average of the selected prototypes (eq. slpe)."""
    ell = log_weights(c, sigma2)[sel]
    wgt = np.exp(ell - ell.max())
    wgt /= wgt.sum()
    return wgt @ c.x[sel].astype(np.float64)


# ---------------------------------------------------------------------- HQL

def _cov(z: np.ndarray) -> np.ndarray:
    """Sample covariance with 1/M normalisation (eq. covariance)."""
    zc = z - z.mean(axis=0, keepdims=True)
    return (zc.T @ zc) / z.shape[0]


def _softmax_rows(logits: np.ndarray) -> np.ndarray:
    m = logits.max(axis=-1, keepdims=True)
    e = np.exp(logits - m)
    return e / e.sum(axis=-1, keepdims=True)


BETA_G_LO, BETA_G_HI, GOLDEN_STEPS = -8, 24, 40
# eps_y values within this relative margin count as equal: where eps_y is
# flat (as beta -> 0 the weights become one-hot on the nearest candidate and
# eps_y saturates), the argmin of eq. epsy is not unique and rounding alone
# would pick among the flat betas, which alpha then depends on
EPS_TIE_REL = 1e-12


def golden_section(f, a: float, b: float, steps: int) -> tuple[float, float]:
    """Golden-section search for a minimiser of f on [a, b] (Kiefer 1953):
    two interior points at the golden ratio; each step keeps the sub-interval
    on the side of the lower value and reuses the surviving point.  Returns
    the final bracket."""
    invphi = (math.sqrt(5.0) - 1.0) / 2.0
    c = b - invphi * (b - a)
    d = a + invphi * (b - a)
    fc, fd = f(c), f(d)
    for _ in range(steps):
        if fc <= fd:
            b, d, fd = d, c, fc
            c = b - invphi * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + invphi * (b - a)
            fd = f(d)
    return a, b


def hql_estimate(x: np.ndarray, y: np.ndarray, y0: np.ndarray, d_euclid: np.ndarray,
                 ridge_rel: float, return_parts: bool = False, alpha_override=None):
    """Full-featured K-MMSE (HQL) for one block.

    x: (M, Nx) prototypes, y: (M, Ny) complete contexts, y0: (Ny,) context,
    d_euclid: (M,) exact Euclidean distances, raster-ordered candidates.

    Steps (Sec. "K-MMSE overview"):
    1. C_ZZ from z_j = (x_j, y_j), 1/M normalised; C_YY gets a ridge
       lambda = ridge_rel tr(C_YY)/Ny + 1e-12 (the paper does not regularise;
       C_YY is singular whenever M <= Ny or the content is flat).  If the
       Cholesky factorisation meets a pivot <= 0 (possible only through
       rounding when ridge_rel >= 0, and always when a negative ridge_rel
       makes the matrix indefinite) np.linalg.LinAlgError propagates;
    2.-6. as in hql_core.
    """
    x = x.astype(np.float64)
    y = y.astype(np.float64)
    nx = x.shape[1]
    z = np.concatenate([x, y], axis=1)
    c = _cov(z)
    cyy = c[nx:, nx:].copy()
    ny = cyy.shape[0]
    lam = ridge_rel * np.trace(cyy) / ny + 1e-12
    cyy[np.diag_indices(ny)] += lam
    chol = np.linalg.cholesky(cyy)
    return hql_core(x, y, y0, d_euclid.astype(np.float64), c[:nx, nx:], cyy, chol, lam,
                    return_parts, alpha_override)


def hql_core(x, y, y0, order_key, cxy, cyy, chol, lam, return_parts=False, alpha_override=None):
    """The estimate of eq. kmmse given the covariance blocks C_XY and the
    regularised C_YY (with its Cholesky factor):
    2. A = C_XY C_YY^-1 (the correction matrix of eq. kmmse with H = beta C);
    3. Mahalanobis distances D(u, v) = (u-v)^T C_YY^-1 (u-v), weights
       proportional to exp(-D / (2 beta)) (eq. weights with H_YY = beta C_YY);
    4. beta = argmin eps_y(beta) (eq. epsy): first minimiser on the grid
       D0 2^(g/2), g = -8..24, D0 = max(min_j D(y0, y_j), 1e-9), refined by
       40 golden-section steps on log beta between the neighbouring grid
       points; grid values within a relative EPS_TIE_REL of the smallest count
       as minimisers, and the refined value is kept only if it is better than
       the grid's by that margin (a flat minimum keeps its smallest beta);
    5. alpha = argmin eps_x(alpha) (eq. epsx) over I0 = the Ny + 1 candidates
       with the smallest order_key (ties by raster index); each x_i is
       predicted leave-one-out from the other candidates with the same beta
       and A.  x_i_hat is affine in alpha, so the argmin is closed form;
    6. x0_hat = x~(beta) + alpha A (y0 - y~(beta)).
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    y0 = np.asarray(y0, dtype=np.float64)
    m = x.shape[0]
    ny = y.shape[1]
    amat = np.linalg.solve(cyy, cxy.T).T            # C_XY C_YY^-1  (Nx x Ny)

    def whiten(v):                                    # L^-1 v  (rows)
        return np.linalg.solve(chol, v.T).T

    vy = whiten(y)
    v0 = whiten(y0[None, :])[0]
    dmah0 = ((vy - v0[None, :]) ** 2).sum(axis=1)     # D(y0, y_j)

    def weights(beta):
        return _softmax_rows(-dmah0 / (2.0 * beta))

    def eps_y(beta):
        r = y0 - weights(beta) @ y
        return float(r @ r)

    d0 = max(float(dmah0.min()), 1e-9)
    grid = [d0 * 2.0 ** (g / 2.0) for g in range(BETA_G_LO, BETA_G_HI + 1)]
    eg = [eps_y(bt) for bt in grid]
    emin = min(eg)
    # first minimiser; a flat minimum resolves to its smallest beta
    gstar = next(g for g, e in enumerate(eg) if e <= emin * (1.0 + EPS_TIE_REL))
    a_t, b_t = golden_section(lambda t: eps_y(math.exp(t)),
                              math.log(grid[max(gstar - 1, 0)]),
                              math.log(grid[min(gstar + 1, len(grid) - 1)]), GOLDEN_STEPS)
    beta = math.exp(0.5 * (a_t + b_t))
    if not eps_y(beta) < eg[gstar] * (1.0 - EPS_TIE_REL):    # kept only if better
        beta = grid[gstar]

    w0 = weights(beta)
    xt = w0 @ x
    yt = w0 @ y

    # I0: Ny + 1 candidates with the smallest key, ties by index
    k = min(ny + 1, m)
    order = np.argsort(order_key, kind="stable")[:k]
    vi = vy[order]
    dmah = ((vi[:, None, :] - vy[None, :, :]) ** 2).sum(axis=2)   # (k, M)
    logits = -dmah / (2.0 * beta)
    logits[np.arange(k), order] = -np.inf                         # leave one out
    wl = _softmax_rows(logits)
    xt_i = wl @ x
    yt_i = wl @ y
    ci = (y[order] - yt_i) @ amat.T                                # A r_i
    ei = x[order] - xt_i
    den = float((ci * ci).sum())
    alpha = float((ci * ei).sum()) / den if den > 0.0 else 0.0
    if alpha_override is not None:
        alpha = float(alpha_override)
    xhat = xt + alpha * (amat @ (y0 - yt))
    if return_parts:
        return xhat, {"beta": beta, "alpha": alpha, "A": amat, "xt": xt, "yt": yt,
                      "w": w0, "grid": grid, "eps_grid": eg, "eps_y": eps_y,
                      "dmah0": dmah0, "I0": order, "ci": ci, "ei": ei, "lam": lam}
    return xhat


PSD_REPAIR_STEPS = 6


def pairwise_covariance(x: np.ndarray, y: np.ndarray, o: np.ndarray):
    """Pairwise-complete covariance of z_j = (x_j, y_j) when y_j is known only
    where o_j is set (x_j always known).  For coordinates a, b the estimate
    uses the candidates that know both: with N_ab their count,
    C_ab = (1/N_ab) sum z_a z_b - (1/N_ab) sum z_a * (1/N_ab) sum z_b, each sum
    over those candidates (0 where N_ab = 0).  With every coordinate known it
    is the 1/M covariance of eq. covariance.  Returns (C_XY, C_YY)."""
    x = x.astype(np.float64)
    yz = np.where(o, y, 0).astype(np.float64)
    of = o.astype(np.float64)
    n_yy = of.T @ of                                   # candidates knowing a and b
    s_yy = yz.T @ of                                   # [a, b]: sum of y_a where both known
    g_yy = yz.T @ yz
    with np.errstate(divide="ignore", invalid="ignore"):
        cyy = np.where(n_yy > 0, g_yy / n_yy - (s_yy * s_yy.T) / (n_yy * n_yy), 0.0)
    n_b = of.sum(axis=0)                               # x known everywhere: N_qb = N_b
    sx_b = x.T @ of                                    # [q, b]: sum of x_q where y_b known
    sy_b = yz.sum(axis=0)                              # sum of y_b where known
    g_xy = x.T @ yz
    with np.errstate(divide="ignore", invalid="ignore"):
        cxy = np.where(n_b[None, :] > 0,
                       g_xy / n_b[None, :] - (sx_b / n_b[None, :]) * (sy_b / n_b)[None, :], 0.0)
    return cxy, cyy


def complete_contexts(y: np.ndarray, o: np.ndarray, y0: np.ndarray) -> np.ndarray:
    """Unknown context pixels of a candidate take the mean of that coordinate
    over the candidates that know it, rounded half up to an integer (the
    coordinate of y0 where no candidate knows it)."""
    yz = np.where(o, y, 0).astype(np.int64)
    cnt = o.sum(axis=0).astype(np.int64)
    tot = yz.sum(axis=0)
    safe = np.maximum(cnt, 1)
    mean = np.where(cnt > 0, (2 * tot + safe) // (2 * safe), np.asarray(y0, dtype=np.int64))
    return np.where(o, y, mean[None, :]).astype(np.int64)


def hql_estimate_partial(x, y, o, y0, d, n, ridge_rel, return_parts=False):
    """HQL over candidates whose contexts are known only where o is set
    (reading of Sec. "K-MMSE overview" for partly lost supports; the paper's
    candidates always have complete contexts):
    1. C_ZZ pairwise complete (pairwise_covariance), C_YY + lambda I with
       lambda as in hql_estimate; where the Cholesky factorisation meets a
       pivot <= 0 (a pairwise estimate need not be positive semi-definite)
       lambda is multiplied by 10 and the factorisation repeated, at most
       PSD_REPAIR_STEPS times, then np.linalg.LinAlgError propagates;
    2. unknown context pixels are completed (complete_contexts);
    3. hql_core on the completed contexts, with I0 ordered by the normalised
       distance d_j / n_j of the candidates (d_j over the pixels both
       contexts know).
    With every context complete it is hql_estimate."""
    x = np.asarray(x, dtype=np.float64)
    cxy, cyy0 = pairwise_covariance(x, y, o)
    ny = cyy0.shape[0]
    lam0 = ridge_rel * np.trace(cyy0) / ny + 1e-12
    chol, cyy, lam = None, None, lam0
    for k in range(PSD_REPAIR_STEPS + 1):
        lam = lam0 * 10.0 ** k
        cyy = cyy0.copy()
        cyy[np.diag_indices(ny)] += lam
        try:
            chol = np.linalg.cholesky(cyy)
            break
        except np.linalg.LinAlgError:
            if k == PSD_REPAIR_STEPS:
                raise
    yc = complete_contexts(y, o, y0).astype(np.float64)
    key = np.asarray(d, dtype=np.float64) / np.asarray(n, dtype=np.float64)
    return hql_core(x, yc, y0, key, cxy, cyy, chol, lam, return_parts)


# ---------------------------------------------------------------- one block

def estimate_block(u, avail, by, bx, p: Params, cnn_gate=None):
    """Estimate lost block (by, bx) from the current state.

    Returns (xhat (B*B,) float64, info dict).
    """
    b = p.block
    y0, m0 = block_context(u, avail, by, bx, p)
    n0 = int(m0.sum())
    info = {"bx": bx, "by": by, "layer": LAYER_BRL, "n_cand": -1, "n_complete": -1,
            "phi": 0, "log_nu": math.nan, "radius": 0, "flags": 0, "n_ctx": n0}
    known = y0[m0]
    phi = int(known.max() - known.min()) if n0 else 0
    info["phi"] = phi
    brl = np.full(b * b, float(known.mean()) if n0 else 0.0)

    mode = p.mode
    if mode == "brl":
        return brl, info
    want_hql = None
    if mode == "profile" and phi <= p.t_phi:
        return brl, info
    cnn_choice = None
    if mode == "cnn":
        # the profile rule's flatness test first (it needs only the ring):
        # a flat ring takes BRL without asking the network
        if phi <= p.t_phi:
            return brl, info
        # learned gate: BRL, IDL with the support-area expansion (never
        # escalating), or HQL (full-window IDL when HQL is not available)
        if cnn_gate is None:
            raise ValueError("cnn mode needs a gate callable")
        cnn_choice = cnn_gate(u, avail, by, bx)
        if cnn_choice == LAYER_BRL:
            return brl, info

    c = candidate_set(u, avail, by, bx, p, y0, m0)
    complete = c.n == n0
    info["n_cand"] = c.size
    info["n_complete"] = int(complete.sum())
    if c.size == 0:
        info["flags"] |= FLAG_NO_CAND
        return brl, info
    ell = log_weights(c, p.sigma2)
    full_sel = np.ones(c.size, dtype=bool)
    info["log_nu"] = _logsumexp(ell)
    info["radius"] = p.window

    if mode in ("profile", "idl") or cnn_choice == LAYER_IDL:
        log_tnu = math.log(p.t_nu) if p.t_nu > 0 else -math.inf
        rad = c.radius
        for rho, lnu in zip(idl_radii(p), log_nu_by_radius(c, p)):
            sel = rad <= rho
            if sel.any() and lnu >= log_tnu:
                info["layer"] = LAYER_IDL
                info["log_nu"] = lnu
                info["radius"] = rho
                return idl_estimate(c, sel, p.sigma2), info
        want_hql = mode == "profile"
    elif mode == "plain":
        want_hql = False
    elif mode == "full" or cnn_choice == LAYER_HQL:
        want_hql = True

    if want_hql:
        avail_hql = c.size if p.hql_partial else info["n_complete"]
        if avail_hql >= max(2, p.min_hql_cands):
            try:
                if p.hql_partial:
                    xh = hql_estimate_partial(c.x, c.y[:, m0], c.m[:, m0], y0[m0], c.d, c.n,
                                              p.ridge_rel)
                else:
                    xh = hql_estimate(c.x[complete], c.y[complete][:, m0], y0[m0],
                                      c.d[complete], p.ridge_rel)
            except np.linalg.LinAlgError:
                # a Cholesky pivot <= 0: the covariance model of eq. kmmse does
                # not exist for this block; the paper gives no rule, the reading
                # is the context mean of eq. mean, flagged
                info["flags"] |= FLAG_HQL_SINGULAR
                return brl, info
            info["layer"] = LAYER_HQL
            return xh, info
        info["flags"] |= FLAG_NO_HQL
    info["layer"] = LAYER_IDL
    return idl_estimate(c, full_sel, p.sigma2), info


# -------------------------------------------------------------- frame driver

def _round_pixel(v: np.ndarray) -> np.ndarray:
    return np.clip(np.floor(v + 0.5), 0, 255).astype(np.uint8)


def conceal(frame: np.ndarray, mask: np.ndarray, p: Params, cnn_gate=None):
    """Conceal every lost block of ``frame`` (uint8, HxW); ``mask`` != 0 = lost.

    Returns (out uint8 HxW, xhat {(by, bx): float64 (B, B)}, info list in
    processing order).
    """
    if p.mode not in MODES:
        raise ValueError(f"unknown mode {p.mode}")
    b, r = p.block, p.ring
    frame = np.asarray(frame, dtype=np.uint8)
    cells = lost_cells(mask, b)
    avail = mask == 0
    if cells and not avail.any():
        raise ValueError("frame has no received pixel")
    u = np.where(avail, frame, 0).astype(np.int64)
    out = frame.copy()
    out[~avail] = 0
    xhats: dict = {}
    infos: list = []
    pending = list(cells)
    rnd = 0
    while pending:
        rnd += 1
        if p.max_rounds and rnd > p.max_rounds:
            fill_mean = float(u[avail].mean())
            for (by, bx) in pending:
                y0, m0 = block_context(u, avail, by, bx, p)
                info = {"bx": bx, "by": by, "layer": LAYER_FILL, "n_cand": -1,
                        "n_complete": -1, "phi": 0, "log_nu": math.nan, "radius": 0,
                        "flags": 0, "round": rnd, "n_ctx": int(m0.sum())}
                if m0.any():
                    v = float(y0[m0].mean())
                else:
                    v = fill_mean
                    info["flags"] |= FLAG_EMPTY_CTX
                xh = np.full((b, b), v)
                xhats[(by, bx)] = xh
                lost = ~avail[by * b:(by + 1) * b, bx * b:(bx + 1) * b]
                out[by * b:(by + 1) * b, bx * b:(bx + 1) * b][lost] = _round_pixel(xh)[lost]
                infos.append(info)
            break
        counts = {c: int(block_context(u, avail, c[0], c[1], p)[1].sum()) for c in pending}
        thr = r * b
        eligible = [c for c in pending if counts[c] >= thr]
        relaxed = False
        if not eligible:
            mx = max(counts.values())
            if mx <= 0:
                raise ValueError("no lost block touches a known pixel")
            eligible = [c for c in pending if counts[c] == mx]
            relaxed = True
        results = []
        for (by, bx) in eligible:
            xh, info = estimate_block(u, avail, by, bx, p, cnn_gate)
            info["round"] = rnd
            if relaxed:
                info["flags"] |= FLAG_CTX_RELAXED
            results.append(((by, bx), xh.reshape(b, b), info))
        for (by, bx), xh, info in results:
            v = _round_pixel(xh)
            sl = (slice(by * b, (by + 1) * b), slice(bx * b, (bx + 1) * b))
            lost = ~avail[sl]                 # received pixels keep their values
            out[sl][lost] = v[lost]
            u[sl][lost] = v[lost]
            avail[sl] = True
            xhats[(by, bx)] = xh
            infos.append(info)
        done = set(eligible)
        pending = [c for c in pending if c not in done]
    return out, xhats, infos


def psnr(a: np.ndarray, b: np.ndarray, sel=None) -> float:
    """Luma PSNR with peak 255 over the whole frame or the pixels in ``sel``."""
    d = a.astype(np.float64) - b.astype(np.float64)
    if sel is not None:
        d = d[sel]
    mse = float((d * d).mean())
    return math.inf if mse == 0.0 else 10.0 * math.log10(255.0 * 255.0 / mse)
