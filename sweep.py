"""Threshold and profile sweeps of the layered estimator on synthetic frames.

Re-runs, on synthetic frames, the three studies of the paper's section on
layer switching and profile selection and of its still-image results:

* flatness threshold T_phi: BRL where phi(y0) <= T_phi, full K-MMSE
  elsewhere (IDL switched off), quality gain and time reduction relative to
  full K-MMSE as T_phi grows;
* normalisation threshold T_nu (log scale): IDL where nu(y0) >= T_nu,
  full K-MMSE elsewhere (BRL switched off);
* the three named profiles (express, efficient, excellent: T_phi = 20 and
  T_nu = 0.01, 0.1, 100), as in the profile table.

"Full K-MMSE" is mode ``full``: HQL where the block has enough candidates
with a complete ring, else IDL over the whole window.  Both loss patterns of
the paper are used: dispersed (the 25 % lattice of lost cells) and random
(25 % of the cells, uniform).  Quality is PSNR and SSIM over the whole frame
against the original; time is the GPU time of one ``conceal_device`` call
(HIP events on its stream, median of ``reps`` after a warm-up), with the
inputs resident in device memory.

    python sweep.py [--frames 4] [--reps 3] [--json out.json]

prints one markdown table per study.
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

# ------------------------------------------------------------------ metrics


def psnr(ref: np.ndarray, img: np.ndarray, peak: float = 255.0) -> float:
    """10 log10(peak^2 / MSE) over the whole plane; inf for identical planes."""
    d = ref.astype(np.float64) - img.astype(np.float64)
    mse = float(np.mean(d * d))
    return math.inf if mse == 0.0 else 10.0 * math.log10(peak * peak / mse)


SSIM_SIGMA = 1.5          # Gaussian window of Wang et al. (2004): sigma 1.5, 11 x 11
SSIM_RADIUS = 5
SSIM_K1, SSIM_K2 = 0.01, 0.03


def _gauss_window() -> np.ndarray:
    t = np.arange(-SSIM_RADIUS, SSIM_RADIUS + 1, dtype=np.float64)
    g = np.exp(-0.5 * (t / SSIM_SIGMA) ** 2)
    return g / g.sum()


def _filter_valid(x: np.ndarray) -> np.ndarray:
    """Separable Gaussian filter, 'valid' part only (no padding)."""
    g = _gauss_window()
    n = g.size
    h, w = x.shape
    rows = sum(g[k] * x[:, k:w - n + 1 + k] for k in range(n))
    return sum(g[k] * rows[k:h - n + 1 + k, :] for k in range(n))


def ssim(ref: np.ndarray, img: np.ndarray, peak: float = 255.0) -> float:
    """Mean SSIM index (Wang, Bovik, Sheikh, Simoncelli 2004) over every
    11 x 11 Gaussian window (sigma 1.5) that fits in the plane, with
    C1 = (0.01 peak)^2 and C2 = (0.03 peak)^2 and weighted (biased) local
    moments."""
    x = ref.astype(np.float64)
    y = img.astype(np.float64)
    if min(x.shape) < 2 * SSIM_RADIUS + 1:
        raise ValueError("plane smaller than the SSIM window")
    c1, c2 = (SSIM_K1 * peak) ** 2, (SSIM_K2 * peak) ** 2
    mx, my = _filter_valid(x), _filter_valid(y)
    sxx = _filter_valid(x * x) - mx * mx
    syy = _filter_valid(y * y) - my * my
    sxy = _filter_valid(x * y) - mx * my
    s = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    return float(np.mean(s))


# ---------------------------------------------------------------- settings

BIG = 1e300               # a threshold no nu reaches (IDL never accepted)
T_PHI_SWEEP = (0.0, 5.0, 10.0, 15.0, 20.0, 25.0, 30.0, 40.0, 50.0, 60.0, 80.0)
T_NU_SWEEP = tuple(10.0 ** k for k in range(-4, 4))
PROFILES = (("express", 20.0, 0.01), ("efficient", 20.0, 0.1), ("excellent", 20.0, 100.0))


def settings():
    """(study, label, t_phi, t_nu) for every setting of the three studies."""
    out = [("flatness", f"T_phi={t:g}", t, BIG) for t in T_PHI_SWEEP]
    out += [("normalisation", f"T_nu={t:g}", -1.0, t) for t in T_NU_SWEEP]
    out += [("profiles", name, tphi, tnu) for name, tphi, tnu in PROFILES]
    return out


def workloads(n_frames: int, h: int = 512, w: int = 768, block: int = 16):
    """(pattern, index, frame, mask): half textured, half smooth frames, each
    under the dispersed lattice and under uniform random cell loss (25 %)."""
    import synth
    out = []
    for f in range(n_frames):
        seed = synth.seed_for(6, f)
        frame = synth.make_luma(h, w, seed, n_bumps=40, n_edges=12, texture=(f % 2 == 0))
        out.append(("dispersed", f, frame, synth.loss_dispersed(h, w, block)))
        out.append(("random", f, frame, synth.loss_random(h, w, block, 0.25, seed + 1)))
    return out


# --------------------------------------------------------------------- run

def run_one(ctx, fd, md, prm, reps: int):
    """Median GPU time (ms) of conceal_device, its output and the layer counts."""
    import torch
    out = torch.empty_like(fd)
    _, info, _ = ctx.conceal_device(fd, md, prm, out=out, want_info=True, want_xhat=False)
    torch.cuda.synchronize()
    times = []
    s = torch.cuda.current_stream()
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        ctx.conceal_device(fd, md, prm, out=out, want_info=False, want_xhat=False)
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times)), out.cpu().numpy(), layer_counts(info)


LAYER_KEYS = ("brl", "idl", "hql", "idl_full")


def layer_counts(info) -> dict:
    """Blocks per layer: BRL, IDL accepted by the nu test, HQL, and IDL over the
    whole window where HQL was wanted but too few complete candidates exist."""
    lay, fl = info["layer"], info["flags"]
    fb = (lay == 1) & ((fl & 2) != 0)
    return dict(brl=int(np.sum(lay == 0)), idl=int(np.sum((lay == 1) & ~fb)),
                hql=int(np.sum(lay == 2)), idl_full=int(np.sum(fb)))


def sweep(n_frames: int = 4, reps: int = 3, block: int = 16, h: int = 512, w: int = 768,
          geometry: str = "block"):
    """geometry "patch": the same 16 x 16 loss, concealed as the paper's 2x2
    patches with 6x6 contexts."""
    import torch
    import paper_2205_11226_amd as skm
    if geometry == "patch":
        def mk(**kw):
            return skm.patch_params(**kw)
    else:
        def mk(**kw):
            return skm.default_params(block=block, **kw)
    ctx = skm.Context(0)
    rows = []
    for pattern, f, frame, mask in workloads(n_frames, h, w, block):
        fd = torch.from_numpy(frame).cuda()
        md = torch.from_numpy(mask).cuda()
        t_full, o_full, l_full = run_one(ctx, fd, md, mk(mode="full"), reps)
        ref = dict(psnr=psnr(frame, o_full), ssim=ssim(frame, o_full), ms=t_full)
        for study, label, tphi, tnu in settings():
            prm = mk(mode="profile", t_phi=tphi, t_nu=tnu)
            t, o, lay = run_one(ctx, fd, md, prm, reps)
            rows.append(dict(study=study, label=label, pattern=pattern, frame=f,
                             psnr=psnr(frame, o), ssim=ssim(frame, o), ms=t, layers=lay,
                             full_psnr=ref["psnr"], full_ssim=ref["ssim"], full_ms=ref["ms"],
                             full_layers=l_full))
        print(f"# {pattern} frame {f}: full K-MMSE {ref['psnr']:.2f} dB, {t_full:.2f} ms, "
              f"layers {l_full}", file=sys.stderr, flush=True)
    ctx.close()
    return rows


def summarise(rows):
    """Per (study, setting, pattern): mean PSNR and SSIM gains over the
    frames and the time reduction (sum of full K-MMSE times / sum of times)."""
    out = []
    keys = []
    for r in rows:
        k = (r["study"], r["label"], r["pattern"])
        if k not in keys:
            keys.append(k)
    for k in keys:
        rs = [r for r in rows if (r["study"], r["label"], r["pattern"]) == k]
        lay = {n: sum(r["layers"][n] for r in rs) for n in LAYER_KEYS}
        tot = max(1, sum(lay.values()))
        out.append(dict(study=k[0], label=k[1], pattern=k[2],
                        dpsnr=float(np.mean([r["psnr"] - r["full_psnr"] for r in rs])),
                        dssim100=float(np.mean([100 * (r["ssim"] - r["full_ssim"]) for r in rs])),
                        speedup=sum(r["full_ms"] for r in rs) / max(1e-9, sum(r["ms"] for r in rs)),
                        ms=float(np.mean([r["ms"] for r in rs])),
                        **{k: lay[k] / tot for k in LAYER_KEYS}))
    return out


def markdown(summary) -> str:
    lines = []
    for study in ("flatness", "normalisation", "profiles"):
        lines.append(f"\n{study}\n")
        lines.append("| setting | loss | dPSNR (dB) | dSSIM x100 | time reduction (x) | ms/frame |"
                     " BRL | IDL | HQL | IDL, no HQL |")
        lines.append("|---|---|---:|---:|---:|---:|---:|---:|---:|---:|")
        for s in summary:
            if s["study"] != study:
                continue
            lines.append(f"| {s['label']} | {s['pattern']} | {s['dpsnr']:+.3f} | "
                         f"{s['dssim100']:+.3f} | {s['speedup']:.2f} | {s['ms']:.2f} | "
                         f"{100 * s['brl']:.0f}% | {100 * s['idl']:.0f}% | {100 * s['hql']:.0f}% | "
                         f"{100 * s['idl_full']:.0f}% |")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--frames", type=int, default=4)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--json", default=None)
    ap.add_argument("--geometry", choices=("block", "patch"), default="block")
    a = ap.parse_args(argv)
    rows = sweep(a.frames, a.reps, geometry=a.geometry)
    summ = summarise(rows)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(dict(rows=rows, summary=summ), f, indent=1)
    print(markdown(summ))


if __name__ == "__main__":
    main()
