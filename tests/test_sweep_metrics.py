"""Host checks of the sweep tool: PSNR and SSIM pinned to their definitions
(closed forms and a window-by-window brute force), and the settings of the
three studies (flatness sweep, normalisation sweep, named profiles)."""
import math

import numpy as np
import pytest

import sweep


def test_psnr_closed_form():
    a = np.full((40, 50), 100, dtype=np.uint8)
    b = a.copy()
    b[:10, :] = 110                      # a quarter of the pixels off by 10
    mse = 0.25 * 100.0
    assert sweep.psnr(a, b) == pytest.approx(10 * math.log10(255.0 ** 2 / mse), abs=1e-12)
    assert sweep.psnr(a, a) == math.inf


def test_ssim_identical_is_one():
    rng = np.random.default_rng(1)
    x = rng.integers(0, 256, size=(37, 41)).astype(np.uint8)
    assert sweep.ssim(x, x) == pytest.approx(1.0, abs=1e-12)


def test_ssim_constant_planes_closed_form():
    # no variance: the structure term is C2 / C2 = 1, the luminance term
    # (2ab + C1) / (a^2 + b^2 + C1) holds in every window
    c1 = (0.01 * 255) ** 2
    for a, b in ((100, 100), (100, 120), (0, 255), (37, 3)):
        x = np.full((20, 30), a, dtype=np.uint8)
        y = np.full((20, 30), b, dtype=np.uint8)
        want = (2 * a * b + c1) / (a * a + b * b + c1)
        assert sweep.ssim(x, y) == pytest.approx(want, rel=1e-12)


def test_ssim_matches_window_brute_force():
    rng = np.random.default_rng(7)
    x = rng.integers(0, 256, size=(19, 23)).astype(np.float64)
    y = np.clip(x + rng.normal(0, 20, size=x.shape), 0, 255)
    t = np.arange(-5, 6, dtype=np.float64)
    g1 = np.exp(-0.5 * (t / 1.5) ** 2)
    g = np.outer(g1, g1)
    g /= g.sum()
    c1, c2 = (0.01 * 255) ** 2, (0.03 * 255) ** 2
    vals = []
    for i in range(x.shape[0] - 10):
        for j in range(x.shape[1] - 10):
            wx, wy = x[i:i + 11, j:j + 11], y[i:i + 11, j:j + 11]
            mx, my = (g * wx).sum(), (g * wy).sum()
            vx = (g * (wx - mx) ** 2).sum()
            vy = (g * (wy - my) ** 2).sum()
            cxy = (g * (wx - mx) * (wy - my)).sum()
            vals.append((2 * mx * my + c1) * (2 * cxy + c2) /
                        ((mx * mx + my * my + c1) * (vx + vy + c2)))
    assert sweep.ssim(x, y) == pytest.approx(float(np.mean(vals)), abs=1e-12)


def test_ssim_rejects_small_planes():
    with pytest.raises(ValueError):
        sweep.ssim(np.zeros((10, 40)), np.zeros((10, 40)))


def test_study_settings():
    st = sweep.settings()
    flat = [s for s in st if s[0] == "flatness"]
    norm = [s for s in st if s[0] == "normalisation"]
    prof = {s[1]: (s[2], s[3]) for s in st if s[0] == "profiles"}
    # flatness sweep: IDL never accepted; the paper's profile value 20 included
    assert all(s[3] == sweep.BIG for s in flat) and any(s[2] == 20.0 for s in flat)
    # normalisation sweep: BRL never taken (phi >= 0 > T_phi), log-spaced T_nu
    assert all(s[2] < 0 for s in norm)
    tn = [s[3] for s in norm]
    assert np.allclose(np.diff(np.log10(tn)), 1.0)
    assert {0.01, 0.1, 100.0} <= set(np.round(tn, 12))
    # the three named profiles of the paper
    assert prof == {"express": (20.0, 0.01), "efficient": (20.0, 0.1),
                  "excellent": (20.0, 100.0)}


def test_summary_gains_and_reduction():
    lay = {"brl": 1, "idl": 2, "hql": 1, "idl_full": 0}
    rows = [dict(study="profiles", label="x", pattern="random", frame=f, psnr=30.0 + f, ssim=0.9,
                 ms=1.0, layers=lay, full_psnr=31.0 + f, full_ssim=0.95, full_ms=4.0,
                 full_layers=lay) for f in range(2)]
    (s,) = sweep.summarise(rows)
    assert s["dpsnr"] == pytest.approx(-1.0)
    assert s["dssim100"] == pytest.approx(-5.0)
    assert s["speedup"] == pytest.approx(4.0)
    assert (s["brl"], s["idl"], s["hql"], s["idl_full"]) == (0.25, 0.5, 0.25, 0.0)


def test_layer_counts_split_the_hql_fallback():
    info = np.zeros(6, dtype=[("layer", "<i4"), ("flags", "<i4")])
    info["layer"] = [0, 1, 1, 2, 1, 0]
    info["flags"] = [4, 0, 2, 0, 3, 0]          # NO_CAND, -, NO_HQL, -, NO_HQL|RELAXED, -
    assert sweep.layer_counts(info) == dict(brl=2, idl=1, hql=1, idl_full=2)
