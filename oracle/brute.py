"""Pure-Python loop version of the concealment oracle, for tiny frames.

TEST INFRASTRUCTURE ONLY.  It re-derives every quantity of ``skmmse`` with
explicit loops, hand-written Cholesky and triangular solves and the ``math``
module, without NumPy, so that a vectorisation slip in ``skmmse`` (a wrong
axis, a transposed operand, a dropped mask) shows up as a mismatch.  It is
only meant for frames of a few dozen pixels a side.

Same definitions as ``skmmse`` (block mode of the paper's Sec.
"Reconstruction framework", layers of Sec. "Scalable K-MMSE estimator", gate
of Sec. "Layer switching").
"""
from __future__ import annotations

import math


def _ring(b, r):
    """Context positions relative to the block origin: the ring of width r,
    then the block's own positions (they count where received)."""
    ring = [(oy, ox) for oy in range(-r, b + r) for ox in range(-r, b + r)
            if not (0 <= oy < b and 0 <= ox < b)]
    return ring + [(oy, ox) for oy in range(b) for ox in range(b)]


def _px(u, av, y, x):
    h, w = len(u), len(u[0])
    if 0 <= y < h and 0 <= x < w and av[y][x]:
        return u[y][x], True
    return 0, False


def context(u, av, by, bx, b, r):
    ys, ms = [], []
    for oy, ox in _ring(b, r):
        v, k = _px(u, av, by * b + oy, bx * b + ox)
        ys.append(v)
        ms.append(k)
    return ys, ms


def candidates(u, av, by, bx, b, r, W, pct):
    """List of dicts (dx, dy, n, d, x, y, m) in raster order (dy, then dx)."""
    h, w = len(u), len(u[0])
    y0, m0 = context(u, av, by, bx, b, r)
    n0 = sum(m0)
    nmin = max(1, (pct * n0 + 99) // 100)
    ring = _ring(b, r)
    out = []
    for dy in range(-W, W + 1):
        for dx in range(-W, W + 1):
            if abs(dx) < b and abs(dy) < b:      # overlaps the block itself
                continue
            py, px = by * b + dy, bx * b + dx
            if py < 0 or px < 0 or py + b > h or px + b > w:
                continue
            full = True
            for i in range(b):
                for j in range(b):
                    if not av[py + i][px + j]:
                        full = False
            if not full:
                continue
            yj, mj = [], []
            for oy, ox in ring:
                v, k = _px(u, av, py + oy, px + ox)
                yj.append(v)
                mj.append(k)
            n = 0
            d = 0
            for k in range(len(ring)):
                if m0[k] and mj[k]:
                    n += 1
                    d += (y0[k] - yj[k]) ** 2
            if n < nmin:
                continue
            xj = [u[py + i][px + j] for i in range(b) for j in range(b)]
            out.append({"dx": dx, "dy": dy, "n": n, "d": d, "x": xj, "y": yj, "m": mj})
    return out


def _lse(vals):
    if not vals:
        return -math.inf
    m = max(vals)
    return m + math.log(sum(math.exp(v - m) for v in vals))


def radii(W, step):
    rs = []
    rho = step
    while rho < W:
        rs.append(rho)
        rho += step
    rs.append(W)
    return rs


def ell(c, sigma2):
    return -(c["d"] / c["n"]) / (2.0 * sigma2)


def log_nu(cands, rho, sigma2):
    return _lse([ell(c, sigma2) for c in cands if max(abs(c["dx"]), abs(c["dy"])) <= rho])


def idl(cands, rho, sigma2, nx):
    sel = [c for c in cands if max(abs(c["dx"]), abs(c["dy"])) <= rho]
    ls = [ell(c, sigma2) for c in sel]
    m = max(ls)
    ws = [math.exp(v - m) for v in ls]
    s = sum(ws)
    return [sum(ws[j] * sel[j]["x"][p] for j in range(len(sel))) / s for p in range(nx)]


# ----------------------------------------------------------- linear algebra

class NotPositiveDefinite(ArithmeticError):
    """A Cholesky pivot came out <= 0 (or NaN)."""


def _cholesky(a):
    n = len(a)
    L = [[0.0] * n for _ in range(n)]
    for i in range(n):
        for j in range(i + 1):
            s = a[i][j]
            for k in range(j):
                s -= L[i][k] * L[j][k]
            if i == j:
                if not s > 0.0:
                    raise NotPositiveDefinite(i)
                L[i][i] = math.sqrt(s)
            else:
                L[i][j] = s / L[j][j]
    return L


def _fwd(L, v):
    n = len(L)
    out = [0.0] * n
    for i in range(n):
        s = v[i]
        for k in range(i):
            s -= L[i][k] * out[k]
        out[i] = s / L[i][i]
    return out


def _bwd(L, v):          # solve L^T x = v
    n = len(L)
    out = [0.0] * n
    for i in range(n - 1, -1, -1):
        s = v[i]
        for k in range(i + 1, n):
            s -= L[k][i] * out[k]
        out[i] = s / L[i][i]
    return out


def _softmax(vals):
    m = max(vals)
    e = [math.exp(v - m) if v != -math.inf else 0.0 for v in vals]
    s = sum(e)
    return [v / s for v in e]


def hql(xs, ys, y0, deu, ridge_rel):
    """Same six steps as ``skmmse.hql_estimate``, written with loops."""
    M = len(xs)
    nx, ny = len(xs[0]), len(ys[0])
    zs = [list(map(float, xs[j])) + list(map(float, ys[j])) for j in range(M)]
    D = nx + ny
    mean = [sum(zs[j][a] for j in range(M)) / M for a in range(D)]
    C = [[sum((zs[j][a] - mean[a]) * (zs[j][c] - mean[c]) for j in range(M)) / M
          for c in range(D)] for a in range(D)]
    cyy = [[C[nx + a][nx + c] for c in range(ny)] for a in range(ny)]
    lam = ridge_rel * sum(cyy[a][a] for a in range(ny)) / ny + 1e-12
    for a in range(ny):
        cyy[a][a] += lam
    L = _cholesky(cyy)
    # A = C_XY C_YY^-1: row p of A solves C_YY a_p = C_YX[:, p]
    A = []
    for p in range(nx):
        col = [C[nx + a][p] for a in range(ny)]
        A.append(_bwd(L, _fwd(L, col)))

    def mah(u, v):
        t = _fwd(L, [u[a] - v[a] for a in range(ny)])
        return sum(q * q for q in t)

    yf = [list(map(float, y)) for y in ys]
    y0f = list(map(float, y0))
    dm0 = [mah(y0f, yf[j]) for j in range(M)]

    def wts(beta):
        return _softmax([-dm / (2.0 * beta) for dm in dm0])

    def eps(beta):
        w = wts(beta)
        s = 0.0
        for a in range(ny):
            r = y0f[a] - sum(w[j] * yf[j][a] for j in range(M))
            s += r * r
        return s

    d0 = max(min(dm0), 1e-9)
    grid = [d0 * 2.0 ** (g / 2.0) for g in range(-8, 25)]
    eg = [eps(bt) for bt in grid]
    emin = min(eg)
    gs = 0
    while eg[gs] > emin * (1.0 + 1e-12):          # flat minimum: smallest beta
        gs += 1
    a_t = math.log(grid[max(gs - 1, 0)])
    b_t = math.log(grid[min(gs + 1, len(grid) - 1)])
    ip = (math.sqrt(5.0) - 1.0) / 2.0
    c_t = b_t - ip * (b_t - a_t)
    d_t = a_t + ip * (b_t - a_t)
    fc, fd = eps(math.exp(c_t)), eps(math.exp(d_t))
    for _ in range(40):
        if fc <= fd:
            b_t, d_t, fd = d_t, c_t, fc
            c_t = b_t - ip * (b_t - a_t)
            fc = eps(math.exp(c_t))
        else:
            a_t, c_t, fc = c_t, d_t, fd
            d_t = a_t + ip * (b_t - a_t)
            fd = eps(math.exp(d_t))
    beta = math.exp(0.5 * (a_t + b_t))
    if not eps(beta) < eg[gs] * (1.0 - 1e-12):
        beta = grid[gs]
    w = wts(beta)
    xt = [sum(w[j] * xs[j][p] for j in range(M)) for p in range(nx)]
    yt = [sum(w[j] * yf[j][a] for j in range(M)) for a in range(ny)]
    k = min(ny + 1, M)
    order = sorted(range(M), key=lambda j: (deu[j], j))[:k]
    num = 0.0
    den = 0.0
    for i in order:
        lg = [(-mah(yf[i], yf[j]) / (2.0 * beta)) if j != i else -math.inf for j in range(M)]
        wl = _softmax(lg)
        xti = [sum(wl[j] * xs[j][p] for j in range(M)) for p in range(nx)]
        yti = [sum(wl[j] * yf[j][a] for j in range(M)) for a in range(ny)]
        r = [yf[i][a] - yti[a] for a in range(ny)]
        ci = [sum(A[p][a] * r[a] for a in range(ny)) for p in range(nx)]
        for p in range(nx):
            num += ci[p] * (xs[i][p] - xti[p])
            den += ci[p] * ci[p]
    alpha = num / den if den > 0.0 else 0.0
    corr = [y0f[a] - yt[a] for a in range(ny)]
    return [xt[p] + alpha * sum(A[p][a] * corr[a] for a in range(ny)) for p in range(nx)]


# ------------------------------------------------------------------ driver

def conceal(frame, mask, b, r, W, sigma2=10.0, t_phi=20.0, t_nu=0.1, step=4, pct=50,
            min_hql=64, ridge_rel=1e-3, mode="profile"):
    """Loop version of ``skmmse.conceal`` (no CNN, no round limit).

    frame, mask: lists of lists.  Returns (out, {(by, bx): xhat list}, layers).
    """
    h, w = len(frame), len(frame[0])
    av = [[mask[y][x] == 0 for x in range(w)] for y in range(h)]
    u = [[frame[y][x] if av[y][x] else 0 for x in range(w)] for y in range(h)]
    cells = [(by, bx) for by in range(h // b) for bx in range(w // b)
             if any(mask[by * b + i][bx * b + j] for i in range(b) for j in range(b))]
    xh_all, layers = {}, {}
    pending = list(cells)
    while pending:
        cnt = {c: sum(context(u, av, c[0], c[1], b, r)[1]) for c in pending}
        elig = [c for c in pending if cnt[c] >= r * b]
        if not elig:
            mx = max(cnt.values())
            elig = [c for c in pending if cnt[c] == mx]
        res = []
        for (by, bx) in elig:
            y0, m0 = context(u, av, by, bx, b, r)
            known = [y0[k] for k in range(len(y0)) if m0[k]]
            phi = max(known) - min(known)
            brl = [sum(known) / len(known)] * (b * b)
            layer, xh = 0, brl
            if mode == "brl" or (mode == "profile" and phi <= t_phi):
                res.append(((by, bx), xh, layer))
                continue
            cs = candidates(u, av, by, bx, b, r, W, pct)
            if not cs:
                res.append(((by, bx), brl, 0))
                continue
            done = False
            if mode in ("profile", "idl"):
                ltn = math.log(t_nu) if t_nu > 0 else -math.inf
                for rho in radii(W, step):
                    sel = [c for c in cs if max(abs(c["dx"]), abs(c["dy"])) <= rho]
                    if sel and log_nu(cs, rho, sigma2) >= ltn:
                        layer, xh, done = 1, idl(cs, rho, sigma2, b * b), True
                        break
            if not done:
                want = mode in ("full", "profile")
                comp = [c for c in cs if c["n"] == sum(m0)]
                if want and len(comp) >= max(2, min_hql):
                    ys = [[c["y"][k] for k in range(len(m0)) if m0[k]] for c in comp]
                    try:
                        xh = hql([c["x"] for c in comp], ys, known, [c["d"] for c in comp],
                                 ridge_rel)
                        layer = 2
                    except NotPositiveDefinite:
                        layer, xh = 0, brl     # no covariance model: context mean
                else:
                    layer, xh = 1, idl(cs, W, sigma2, b * b)
            res.append(((by, bx), xh, layer))
        for (by, bx), xh, layer in res:
            for i in range(b):
                for j in range(b):
                    if av[by * b + i][bx * b + j]:
                        continue                 # a received pixel of the block
                    v = min(255, max(0, math.floor(xh[i * b + j] + 0.5)))
                    u[by * b + i][bx * b + j] = v
                    av[by * b + i][bx * b + j] = True
            xh_all[(by, bx)] = xh
            layers[(by, bx)] = layer
        pending = [c for c in pending if c not in set(elig)]
    return u, xh_all, layers
