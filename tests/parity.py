"""Helpers that compare the HIP path with the float64 oracle.

Bars: exact integers (distances, counts, layer decisions), max |xhat| error
<= 1e-3 before rounding, uint8 pixels equal except where the oracle's value
lies within 1e-3 of a rounding tie, log nu within 1e-9 (absolute, on values
of order 1-100), and layer decisions equal except where log nu is within
1e-9 of log T_nu.

Rounds: the estimates of a round become known pixels of the next ones (end
of the K-MMSE overview), as rounded integers.  Where a pixel of an earlier
round was rounded the other way at a tie, the blocks of later rounds whose
search window holds it start from different inputs; they are exempt from
the value bars (xhat, log nu, layer) and counted instead.
"""
import math

import numpy as np

XHAT_TOL = 1e-3
TIE_TOL = 1e-3
LNU_TOL = 1e-9

ORACLE_MODE = {"profile": "profile", "plain": "plain", "full": "full", "brl": "brl",
               "idl": "idl", "cnn": "profile"}


def oracle_params(mode="profile", **kw):
    from oracle.skmmse import Params
    return Params(mode=ORACLE_MODE[mode], **kw)


def device_params(mode="profile", **kw):
    import paper_2205_11226_amd as skm
    return skm.default_params(mode=mode, **kw)


def tie_affected(out_g, out_o, xh_o, info_o, b, ring, window):
    """Blocks of later rounds whose search window holds a pixel that differs
    from the oracle's because an earlier round rounded it the other way at a
    tie, or because it belongs to such a block (transitively, round by
    round)."""
    rnd = {(io["by"], io["bx"]): io["round"] for io in info_o}
    diffs = [(int(y), int(x)) for y, x in np.argwhere(out_g != out_o)]
    ext = ring + window
    out = set()
    for rk in sorted(set(rnd.values())):
        src = []
        for y, x in diffs:
            key = (y // b, x // b)
            if rnd.get(key, 10 ** 9) >= rk:
                continue
            v = xh_o[key][y % b, x % b]
            if key in out or abs((v - math.floor(v)) - 0.5) < TIE_TOL:
                src.append((y, x))
        for key, r_ in rnd.items():
            if r_ != rk:
                continue
            y0, x0 = key[0] * b - ext, key[1] * b - ext
            if any(y0 <= y < y0 + b + 2 * ext and x0 <= x < x0 + b + 2 * ext for y, x in src):
                out.add(key)
    return out


def compare(frame, mask, out_g, info_g, xhat_g, out_o, xh_o, info_o, t_nu, b,
            check_pixels=True, ring=4, window=24):
    """Assert parity of one concealed frame; returns a dict of statistics."""
    byk = {(int(i["by"]), int(i["bx"])): i for i in info_g}
    assert len(byk) == len(info_o), (len(byk), len(info_o))
    log_tnu = math.log(t_nu) if t_nu > 0 else -math.inf
    max_err = 0.0
    near = 0
    affected = tie_affected(out_g, out_o, xh_o, info_o, b, ring, window)
    assert len(affected) <= max(2, len(info_o) // 10), len(affected)
    for k, io in enumerate(info_o):
        key = (io["by"], io["bx"])
        ig = byk[key]
        if key in affected:
            assert int(ig["round"]) == io["round"], key
            continue
        lnu_o = io["log_nu"]
        tie = (math.isfinite(lnu_o) and abs(lnu_o - log_tnu) < LNU_TOL)
        if int(ig["layer"]) != io["layer"] or int(ig["radius"]) != io["radius"]:
            assert tie, (key, dict(zip(ig.dtype.names, ig.tolist())), io)
            near += 1
            continue
        for f in ("phi", "n_ctx", "flags", "n_cand", "n_complete", "round"):
            if f in io:
                assert int(ig[f]) == io[f], (key, f, int(ig[f]), io[f])
        lg = float(ig["log_nu"])
        if math.isnan(lnu_o):
            assert math.isnan(lg), (key, lg)
        else:
            assert abs(lg - lnu_o) <= LNU_TOL * max(1.0, abs(lnu_o)), (key, lg, lnu_o)
    if not check_pixels:
        return {"max_err": None, "near_ties": near}
    # per-block pixel estimates (xhat_g in lost-cell raster order = info_g order)
    for idx, ig in enumerate(info_g):
        key = (int(ig["by"]), int(ig["bx"]))
        if key in affected:
            continue
        xo = xh_o[key]
        xg = xhat_g[idx]
        err = float(np.abs(xg.astype(np.float64) - xo).max())
        max_err = max(max_err, err)
        assert err <= XHAT_TOL, (key, err)
    diff = out_g != out_o
    if diff.any():
        ys, xs = np.nonzero(diff)
        for y, x in zip(ys, xs):
            key = (y // b, x // b)
            if key in affected:
                continue
            v = xh_o[key][y % b, x % b]
            assert abs((v - math.floor(v)) - 0.5) < TIE_TOL, ((y, x), v, out_g[y, x], out_o[y, x])
    keep = mask == 0
    assert np.array_equal(out_g[keep], frame[keep])
    return {"max_err": max_err, "near_ties": near, "pix_diff": int(diff.sum()),
            "tie_affected": len(affected)}
