"""Training of the learned layer manager (the CNN gate).

Labels come from the concealment method itself: for every lost block of a
training frame the library conceals the frame in BRL, full-window IDL (plain),
IDL with support-area expansion and full K-MMSE modes, and the block's PSNR
gains are
    g1 = PSNR(IDL, whole window) - PSNR(BRL)
    g2 = PSNR(HQL) - PSNR(IDL), 0 where HQL is not available,
with the block MSE floored at 1/12 (the error of rounding to integers).
The network is trained with the library's own kernels (Adam on FP32 master
weights, bfloat16 forward).  The decision thresholds (tau1, tau2) are then
fitted on held-out frames: the largest share of cheap layers such that the
frame PSNR stays within `max_dpsnr` dB of full K-MMSE.

Usage:  python -m paper_2205_11226_amd.gate --out gate.skm
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

# relative cost of a block per layer, for choosing thresholds (order of
# magnitude measured on MI355X: a context mean is nearly free next to the
# distances and weights of IDL, and full K-MMSE costs thousands of IDL blocks)
LAYER_COST = {"brl": 0.2, "idl": 1.0, "hql": 2000.0}


def _psnr_from_sse(sse, npx):
    mse = max(sse / npx, 1e-12)
    return 10.0 * math.log10(255.0 * 255.0 / mse)


def block_labels(ctx, frame, mask, b=16, t_nu=0.1):
    """Per-block SSE of each layer, labels (g1, g2) and HQL availability."""
    import torch
    import paper_2205_11226_amd as skm
    fd = torch.from_numpy(np.ascontiguousarray(frame)).cuda()
    md = torch.from_numpy(np.ascontiguousarray(mask)).cuda()
    outs, infos = {}, {}
    for mode in ("brl", "plain", "idl", "full"):
        p = skm.default_params(mode=mode, block=b, t_nu=t_nu)
        o, info, _ = ctx.conceal_device(fd, md, p, want_xhat=False)
        outs[mode] = o.cpu().numpy().astype(np.float64)
        infos[mode] = info
    info = infos["full"]
    truth = frame.astype(np.float64)
    n = len(info)
    sse = {m: np.zeros(n) for m in outs}
    for k, ig in enumerate(info):
        by, bx = int(ig["by"]), int(ig["bx"])
        sl = (slice(by * b, (by + 1) * b), slice(bx * b, (bx + 1) * b))
        for m in outs:
            d = outs[m][sl] - truth[sl]
            sse[m][k] = float((d * d).sum())
    floor = b * b / 12.0

    def ps(s):
        return 10.0 * np.log10(255.0 * 255.0 * b * b / np.maximum(s, floor))
    hql = info["layer"] == 2
    g1 = ps(sse["plain"]) - ps(sse["brl"])
    g2 = np.where(hql, ps(sse["full"]) - ps(sse["plain"]), 0.0)
    # blocks that CNN mode sends to BRL by the flatness test, before the gate
    flat = info["phi"] <= skm.default_params(mode="cnn", block=b).t_phi
    return {"g": np.stack([g1, g2], 1).astype(np.float32), "sse": sse, "hql": hql,
            "flat": flat, "npx": frame.size}


KINDS = ("lattice", "isolated", "smooth")


def _gen(args):
    """One training frame: 1080p textured luma with 25% dispersed loss
    (lattice), 720p textured luma with isolated loss (isolated), or 720p
    luma without texture with isolated loss (smooth)."""
    import synth
    kind, seed = args
    if kind == "lattice":
        f = synth.make_luma(1080, 1920, seed, n_bumps=150, n_edges=40, texture=True)
        r = np.random.default_rng(seed + 1)
        m = synth.loss_dispersed(1080, 1920, 16, int(r.integers(2)), int(r.integers(2)))
    elif kind == "isolated":
        f = synth.make_luma(720, 1280, seed, n_bumps=80, n_edges=24, texture=True)
        m = synth.loss_isolated(720, 1280, 16, 420, seed + 1)
    else:
        f = synth.make_luma(720, 1280, seed, n_bumps=80, n_edges=24, texture=False)
        m = synth.loss_isolated(720, 1280, 16, 420, seed + 1)
    return f, m


def make_frames(counts, seed0, workers=8):
    """counts: frames per kind, in KINDS order."""
    import multiprocessing as mp
    jobs = [(k, seed0 + 5000 * j + i) for j, (k, n) in enumerate(zip(KINDS, counts))
            for i in range(n)]
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_gen, jobs)


def build_dataset(ctx, frames, b=16):
    """Inputs (bf16 bits, device) and labels of every lost block, plus the
    per-frame label records."""
    import torch
    import paper_2205_11226_amd as skm
    xs, ys, recs = [], [], []
    for f, m in frames:
        p = skm.default_params(block=b)
        x = ctx.cnn_inputs(torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda(), p)
        rec = block_labels(ctx, f, m, b)
        xs.append(x)
        ys.append(torch.from_numpy(rec["g"]).cuda())
        recs.append(rec)
    return torch.cat(xs), torch.cat(ys), recs


def train(ctx, x, y, epochs=8, batch=256, lr=1e-3, seed=0, log=print):
    import torch
    ctx.cnn_init(seed)
    n = x.shape[0]
    rng = np.random.default_rng(seed)
    steps = 0
    total = epochs * ((n + batch - 1) // batch)
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        run = 0.0
        nb = 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            xb = x.index_select(0, idx).contiguous()
            yb = y.index_select(0, idx).contiguous()
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * steps / total))
            want = (nb % 50) == 0
            loss = ctx.cnn_train_step(xb, yb, cur, want_loss=want)
            if want:
                run += loss
            nb += 1
            steps += 1
        log(f"epoch {ep}: mean sampled loss {run / max(1, (nb + 49) // 50):.4f}")


def fit_thresholds(pred, recs, max_dpsnr=0.05, margin=0.01):
    """Thresholds minimising the layer cost subject to a PSNR loss against
    full K-MMSE of at most max_dpsnr - margin dB on every frame."""
    q1 = np.unique(np.quantile(pred[:, 0], np.linspace(0, 1, 121)))
    q2 = np.unique(np.quantile(pred[:, 1], np.linspace(0, 1, 61)))
    best = None
    o = 0
    spans = []
    for r in recs:
        n = len(r["g"])
        spans.append((o, o + n))
        o += n
    full_ps = [_psnr_from_sse(r["sse"]["full"].sum(), r["npx"]) for r in recs]
    for t1 in np.concatenate([[-np.inf], q1]):
        for t2 in np.concatenate([q2, [np.inf]]):
            dps, cost = [], 0.0
            for (a, b), r, fp in zip(spans, recs, full_ps):
                p = pred[a:b]
                brl = (p[:, 0] <= t1) | r["flat"]
                hql = ~brl & (p[:, 1] > t2) & r["hql"]
                idl = ~brl & ~hql
                sse = (r["sse"]["brl"] * brl + r["sse"]["full"] * hql + r["sse"]["idl"] * idl).sum()
                dps.append(fp - _psnr_from_sse(sse, r["npx"]))
                cost += (LAYER_COST["brl"] * brl.sum() + LAYER_COST["idl"] * idl.sum() +
                         LAYER_COST["hql"] * hql.sum())
            dworst = float(np.max(dps))
            if dworst <= max_dpsnr - margin and (best is None or cost < best[0]):
                best = (cost, float(t1), float(t2), dworst)
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--lattice", type=int, default=80)
    ap.add_argument("--isolated", type=int, default=60)
    ap.add_argument("--smooth", type=int, default=60)
    ap.add_argument("--val", type=int, default=6, help="validation frames per kind")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--seed", type=int, default=4000)
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    import torch
    import paper_2205_11226_amd as skm
    t0 = time.time()
    frames = make_frames((args.lattice, args.isolated, args.smooth), args.seed, args.workers)
    vframes = make_frames((args.val,) * len(KINDS), args.seed + 20000, args.workers)
    print(f"frames generated in {time.time() - t0:.1f}s", flush=True)
    ctx = skm.Context(0)
    t0 = time.time()
    x, y, _ = build_dataset(ctx, frames)
    xv, yv, vrecs = build_dataset(ctx, vframes)
    torch.cuda.synchronize()
    print(f"dataset: {x.shape[0]} training blocks, {xv.shape[0]} validation blocks, "
          f"labels in {time.time() - t0:.1f}s; mean g1 {y[:, 0].mean().item():.3f} dB, "
          f"mean g2 {y[:, 1].mean().item():.3f} dB", flush=True)
    t0 = time.time()
    train(ctx, x, y, epochs=args.epochs, log=lambda s: print(s, flush=True))
    torch.cuda.synchronize()
    print(f"trained in {time.time() - t0:.1f}s", flush=True)
    pv = ctx.cnn_forward(xv).cpu().numpy()
    mse = float(((pv - yv.cpu().numpy()) ** 2).mean())
    var = float(yv.cpu().numpy().var(axis=0).mean())
    print(f"validation mse {mse:.4f} (label variance {var:.4f})", flush=True)
    best = fit_thresholds(pv, vrecs)
    if best is None:
        print("no threshold pair meets the PSNR bound; keeping the profile rule", flush=True)
        sys.exit(1)
    cost, t1, t2, dps = best
    print(f"thresholds tau1 {t1:.4f} tau2 {t2:.4f}: worst-frame dPSNR {dps:.4f} dB, "
          f"cost {cost:.0f}", flush=True)
    ctx.cnn_set_thresholds(t1 if math.isfinite(t1) else -1e30, t2 if math.isfinite(t2) else 1e30)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    ctx.cnn_save(args.out)
    print(f"saved {args.out}", flush=True)


if __name__ == "__main__":
    main()
