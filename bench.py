"""Throughput benchmark: concealed 16x16 blocks/s on a 1080p frame with 25 %
dispersed block loss (one MI355X).

One step = the whole concealment of one 1920x1080 luma frame through the C
ABI (loss geometry, rounds, context/flatness gate, candidate distances,
weights, weighted averages, write-back), with the frame and mask already in
HBM.  Prints ONE JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode cnn|profile|plain|...]
       python bench.py --traffic-run --steps 3          (under rocprofv3 --pmc)
       python bench.py --traffic-parse FETCH_DIR WRITE_DIR OUT.json
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "concealed 16x16 blocks/s @1080p 25% loss, layered+CNN vs plain, ΔPSNR≤0.05dB"
VALU_PEAK_TOPS = 78.6   # 256 CU x 64 lanes x 2 ops (mul+add) x 2.4 GHz, no packed math
KERNEL = "k_round_main"


# ----------------------------------------------------------- CPU baseline

_CPU = {}


def read_gate(path):
    """Thresholds and float32 weights of a gate file written by skm_save_cnn:
    8-byte magic, four uint32 (version, count, 0, 0), two float32 thresholds,
    then the weights, all little-endian."""
    raw = open(path, "rb").read()
    if raw[:8] != b"SKMGATE1":
        raise ValueError(f"{path}: not a gate weight file")
    hdr = np.frombuffer(raw, "<u4", 4, 8)
    tau = np.frombuffer(raw, "<f4", 2, 24).astype(np.float64)
    w = np.frombuffer(raw, "<f4", int(hdr[1]), 32).astype(np.float64)
    return float(tau[0]), float(tau[1]), w


def _cpu_init(frame, mask, mode, t_nu, gate_path):
    import oracle.skmmse as o
    _CPU["f"] = frame.astype(np.int64)
    _CPU["a"] = mask == 0
    _CPU["p"] = o.Params(mode=mode, t_nu=t_nu)
    _CPU["est"] = o.estimate_block
    _CPU["gate"] = None
    if mode == "cnn":
        import oracle.cnn as oc
        t1, t2, w = read_gate(gate_path)
        pw = oc.unpack(w)

        def gate(u, avail, by, bx):
            y = oc.forward(pw, oc.block_input(u, avail, by, bx, 16)[None])[0]
            return 0 if y[0] <= t1 else (2 if y[1] > t2 else 1)
        _CPU["gate"] = gate


def _cpu_work(cells):
    for by, bx in cells:
        _CPU["est"](_CPU["f"], _CPU["a"], by, bx, _CPU["p"], _CPU["gate"])
    return len(cells)


def cpu_baseline(frame, mask, mode, t_nu, workers, gate_path, frac=1.0, passes=4):
    """Time the float64 oracle on the lost blocks of the frame (one round: all
    blocks are independent) over a process pool of ``workers``; ``frac`` keeps
    an evenly spaced share of the blocks, ``passes`` repeats the list (about
    4 s of CPU work per pass of the whole frame)."""
    import multiprocessing as mp
    from oracle.skmmse import lost_cells
    cells = lost_cells(mask, 16)
    step = max(1, int(round(1.0 / frac)))
    cells = cells[::step] * passes
    chunks = [cells[i::workers * 4] for i in range(workers * 4)]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_cpu_init,
                  initargs=(frame, mask, mode, t_nu, gate_path)) as pool:
        pool.map(_cpu_work, [c[:2] for c in chunks[:workers]])     # warm the workers
        t0 = time.perf_counter()
        n = sum(pool.map(_cpu_work, chunks))
        dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "blocks/s", "cores": workers, "kind": "oracle",
            "sample": f"{passes} passes over {n // passes} of the lost blocks of the 1080p frame "
                      f"(every {step}), float64 NumPy oracle, mode={mode}, {workers} worker "
                      f"processes, {dt:.2f} s wall"}


# ------------------------------------------------------------ algorithmic

def algorithmic_ops(d_tab, n_tab, info, b):
    """Ops of one launch of the estimation kernel on this frame.

    Per block that computes distances: 3 ops (difference, multiply, add) per
    pair of ring pixels compared, summed over candidates; plus 2 ops (FMA)
    per prototype pixel per candidate inside the accepted radius.  Context-
    mean blocks count one add per known ring pixel."""
    W = (d_tab.shape[1] - 1) // 2
    yy, xx = np.mgrid[-W:W + 1, -W:W + 1]
    rad = np.maximum(np.abs(yy), np.abs(xx))
    total = 0
    for k, inf in enumerate(info):
        if inf["layer"] == 0 and inf["n_cand"] < 0:
            total += int(inf["n_ctx"])
            continue
        ok = d_tab[k] >= 0
        total += 3 * int(n_tab[k][ok].sum())
        if inf["layer"] == 1:
            total += 2 * b * b * int((ok & (rad <= inf["radius"])).sum())
    return total


def traffic_from_profile(kernel_src_hash):
    path = os.path.join(ROOT, "profiles", "traffic_k_round_main_1080p.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha1") != kernel_src_hash:
        return None
    return rec.get("bytes_per_launch")


def kernel_source_hash():
    h = hashlib.sha1()
    for n in ("skm_kernels.hip", "skm_device.h", "skm_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2205_11226_amd", "csrc", n), "rb").read())
    return h.hexdigest()


def psnr(a, b):
    d = a.astype(np.float64) - b.astype(np.float64)
    mse = float((d * d).mean())
    return math.inf if mse == 0 else 10 * math.log10(255 * 255 / mse)


# ------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--mode", default="cnn")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2205_11226_amd", "weights",
                                                      "gate_1080p.skm"))
    ap.add_argument("--profile", default="efficient")
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-run", action="store_true",
                    help="only conceal --steps frames and copy a known size (counter runs)")
    ap.add_argument("--geometry", choices=("block", "patch"), default="block",
                    help="patch: the paper's 2x2 patches with a 6x6 context on the same frame "
                         "(a line of its own; the default line is the block workload)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(blocks of a round are independent; frames or bands would shard "
              "across GPUs).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    t_nu = {"express": 0.01, "efficient": 0.1, "excellent": 100.0}[args.profile]
    frame, mask = synth.workload_layered_1080p()
    if args.traffic_run:
        return traffic_run(args, frame, mask)
    if args.geometry == "patch":
        return bench_patch(args, frame, mask)

    cpu = None
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or max(1, min(os.cpu_count() or 1, 16))
        cpu = cpu_baseline(frame, mask, args.mode, t_nu, workers, args.weights)
        print(f"# cpu baseline: {cpu['value']:.1f} blocks/s on {workers} cores", file=sys.stderr,
              flush=True)

    import torch
    import paper_2205_11226_amd as skm

    dev = torch.device("cuda:0")
    fd = torch.from_numpy(frame).to(dev)
    md = torch.from_numpy(mask).to(dev)
    out = torch.empty_like(fd)
    ctx = skm.Context(0)
    if args.mode == "cnn":
        ctx.cnn_load(args.weights)          # fails loudly when the weights are missing
    p_lay = skm.default_params(mode=args.mode, profile=args.profile)
    p_prof = skm.default_params(mode="profile", profile=args.profile)
    p_plain = skm.default_params(mode="plain")

    outs = [torch.empty_like(fd) for _ in range(8)]

    def jobs_for(p, k):
        return [(fd, md, outs[j % len(outs)], p) for j in range(k)]

    def timed_batch(p, events=False):
        """One skm_conceal_batch over `steps` frames (frames in flight on the
        context's streams, graphs replayed), after an untimed warm-up batch."""
        ctx.conceal_batch(jobs_for(p, max(args.warmup, 1)))
        jobs = jobs_for(p, args.steps)
        torch.cuda.synchronize()
        ctx.profile_enable(events)
        ctx.profile_read()                  # drop earlier event pairs
        t0 = time.perf_counter()
        res = ctx.conceal_batch(jobs)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        ctx.profile_enable(False)
        assert all(r[2] == 0 and r[0] == res[0][0] for r in res)
        return dt

    def timed_single(p, k):
        """Synchronous single-frame calls: latency per frame."""
        for _ in range(max(args.warmup, 1)):
            ctx.conceal_device(fd, md, p, out=out, want_info=False, want_xhat=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            ctx.conceal_device(fd, md, p, out=out, want_info=False, want_xhat=False)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    # launch configuration picked by the library's autotuner on a short batch
    tune_ms = ctx.autotune(jobs_for(p_lay, 16), reps=3)
    tuned = {"batch_streams": ctx.get_option(skm.OPT_BATCH_STREAMS),
             "graphs": ctx.get_option(skm.OPT_GRAPHS),
             "gate_grid": ctx.get_option(skm.OPT_GATE_GRID), "tune_batch16_ms": tune_ms}
    print(f"# autotune: {tuned}", file=sys.stderr, flush=True)

    sec_lay = timed_batch(p_lay)
    # the estimation kernel bracketed by HIP events on its own stream, over
    # the same batch again with one frame in flight (event timing makes the
    # library launch eagerly; no other frame's kernels overlap the pair)
    streams = ctx.get_option(skm.OPT_BATCH_STREAMS)
    ctx.set_option(skm.OPT_BATCH_STREAMS, 1)
    sec_lay_ev = timed_batch(p_lay, events=True)
    ctx.set_option(skm.OPT_BATCH_STREAMS, streams)
    ms_tot, launches = ctx.profile_read()
    k_ms = ms_tot / max(launches, 1)
    print(f"# layered ({args.mode}): {sec_lay * 1e3:.3f} ms/frame ({sec_lay_ev * 1e3:.3f} with "
          f"event timing), estimation kernel {k_ms * 1e3:.1f} us x {launches / args.steps:.0f} "
          f"per frame", file=sys.stderr, flush=True)
    lat_lay = timed_single(p_lay, min(args.steps, 20))
    sec_plain = timed_batch(p_plain)
    print(f"# plain: {sec_plain * 1e3:.3f} ms/frame", file=sys.stderr, flush=True)
    sec_prof = timed_batch(p_prof)
    print(f"# profile rule: {sec_prof * 1e3:.3f} ms/frame", file=sys.stderr, flush=True)

    # statistics of one frame per mode (not timed)
    o_lay, info_lay, _ = ctx.conceal_device(fd, md, p_lay, want_xhat=False)
    o_prof, info_prof, _ = ctx.conceal_device(fd, md, p_prof, want_xhat=False)
    o_plain, _, _ = ctx.conceal_device(fd, md, p_plain, want_xhat=False)
    o_full, _, _ = ctx.conceal_device(fd, md, skm.default_params(mode="full"), want_xhat=False)
    d_tab, n_tab = ctx.distances_device(fd, md, p_plain)
    d_tab, n_tab = d_tab.cpu().numpy(), n_tab.cpu().numpy()
    n_lost = len(info_lay)
    ops = algorithmic_ops(d_tab, n_tab, info_lay, 16)
    achieved = ops / (k_ms * 1e-3) / 1e12
    ps_lay = psnr(o_lay.cpu().numpy(), frame)
    ps_full = psnr(o_full.cpu().numpy(), frame)
    ps_prof = psnr(o_prof.cpu().numpy(), frame)
    ps_plain = psnr(o_plain.cpu().numpy(), frame)

    def layer_counts(info):
        c = np.bincount(info["layer"] + 1, minlength=4)
        return {"brl": int(c[1]), "idl": int(c[2]), "hql": int(c[3]), "fill": int(c[0])}

    res = {
        "metric": METRIC,
        "value": n_lost / sec_lay,
        "unit": "blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_lay * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32+f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "1920x1080 luma (150 bumps, 40 edges, texture), 25% dispersed "
                        "16x16 loss (2040 blocks), one frame per step",
            "mode": args.mode, "profile": args.profile,
            "lost_blocks": n_lost,
            "frames_per_s": 1.0 / sec_lay,
            "timed": f"one skm_conceal_batch call over {args.steps} frames (the same input, "
                     f"outputs in 8 rotating buffers), launch configuration from skm_autotune",
            "launch_config": tuned,
            "single_frame_latency_ms": lat_lay * 1e3,
            "psnr_layered_db": ps_lay,
            "psnr_full_kmmse_db": ps_full,
            "delta_psnr_db": ps_full - ps_lay,
            "layers": layer_counts(info_lay),
            "plain": {"blocks_per_s": n_lost / sec_plain, "ms_per_frame": sec_plain * 1e3,
                      "delta_psnr_db": ps_full - ps_plain},
            "speedup_vs_plain": sec_plain / sec_lay,
            "profile_rule": {"blocks_per_s": n_lost / sec_prof, "ms_per_frame": sec_prof * 1e3,
                             "delta_psnr_db": ps_full - ps_prof,
                             "layers": layer_counts(info_prof)},
        },
        "roofline": {
            "kernel": KERNEL,
            "bound": "alu",
            "achieved": achieved,
            "peak": VALU_PEAK_TOPS,
            "unit": "TOP/s",
            "frac": achieved / VALU_PEAK_TOPS,
            "traffic": traffic_from_profile(kernel_source_hash()),
            "ops_per_launch": ops,
            "kernel_ms": k_ms,
            "launches_timed": launches,
            "kernel_timing": "HIP events around each launch, over a second run of the timed "
                             "batch with one frame in flight (eager launches)",
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    ctx.close()


# ------------------------------------------------------ 2x2 patch geometry

def bench_patch(args, frame, mask):
    """The paper's own geometry on the same 1080p frame and loss: every lost
    16x16 block is 64 patches of 2x2 pixels with a 6x6 context, concealed
    over rounds from the border of each lost region to its centre.  Timed as
    the block workload (one skm_conceal_batch over --steps frames) for the
    efficient, excellent and plain profiles."""
    import torch
    import paper_2205_11226_amd as skm

    dev = torch.device("cuda:0")
    fd = torch.from_numpy(frame).to(dev)
    md = torch.from_numpy(mask).to(dev)
    outs = [torch.empty_like(fd) for _ in range(8)]
    ctx = skm.Context(0)
    res = {}
    for name, p in (("efficient", skm.patch_params(mode="profile", profile="efficient")),
                    ("excellent", skm.patch_params(mode="profile", profile="excellent")),
                    ("plain", skm.patch_params(mode="plain"))):
        o, info, _ = ctx.conceal_device(fd, md, p, want_xhat=False)
        ctx.conceal_batch([(fd, md, outs[j % 8], p) for j in range(max(args.warmup, 1))])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.conceal_batch([(fd, md, outs[j % 8], p) for j in range(args.steps)])
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.steps
        assert all(x[2] == 0 and x[0] == len(info) for x in r)
        c = np.bincount(info["layer"] + 1, minlength=4)
        res[name] = {"patches_per_s": len(info) / sec, "ms_per_frame": sec * 1e3,
                     "rounds": int(info["round"].max()), "psnr_db": psnr(o.cpu().numpy(), frame),
                     "layers": {"brl": int(c[1]), "idl": int(c[2]), "hql": int(c[3])}}
        print(f"# patch {name}: {sec * 1e3:.3f} ms/frame", file=sys.stderr, flush=True)
    n = len(info)
    print(json.dumps({
        "metric": "concealed 2x2 patches/s @1080p 25% loss (efficient profile)",
        "value": res["efficient"]["patches_per_s"], "unit": "patches/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["efficient"]["ms_per_frame"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "i32+f32+f64", "data": "synthetic",
        "config": {"workload": "1920x1080 luma (150 bumps, 40 edges, texture), 25% dispersed "
                               f"16x16 loss as {n} 2x2 patches with 6x6 contexts, window +-24, "
                               "one frame per step", "profiles": res},
    }), flush=True)
    ctx.close()


# ---------------------------------------------------------------- traffic
#
# HBM traffic of the estimation kernel comes from two rocprofv3 counter runs
# of `bench.py --traffic-run` (FETCH_SIZE, then WRITE_SIZE).  Each run also
# times a plain device-to-device copy of a known size, whose counter reading
# gives the factor that turns the counter into bytes.

COPY_BYTES = 256 << 20


def traffic_run(args, frame, mask):
    import torch
    import paper_2205_11226_amd as skm
    fd = torch.from_numpy(frame).cuda()
    md = torch.from_numpy(mask).cuda()
    out = torch.empty_like(fd)
    ctx = skm.Context(0)
    if args.mode == "cnn":
        ctx.cnn_load(args.weights)
    p = skm.default_params(mode=args.mode, profile=args.profile)
    for _ in range(args.steps):
        ctx.conceal_device(fd, md, p, out=out, want_info=False, want_xhat=False)
    src = torch.ones(COPY_BYTES, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ctx.close()
    print(f"# traffic run: {args.steps} frames, 3 copies of {COPY_BYTES} bytes", flush=True)


def _counter_rows(d):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        rows += list(csv.DictReader(open(f)))
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return rows


def traffic_parse(fetch_dir, write_dir, out_path):
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        per = {}
        for r in _counter_rows(d):
            if r["Counter_Name"] != counter:
                continue
            per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        main = [v for k, v in per.items() if KERNEL in k]
        copy = [v for k, v in per.items() if "copy" in k.lower() and "skm" not in k]
        if not main or not copy:
            raise SystemExit(f"{counter}: kernels found {sorted(per)}")
        main_avg = float(np.mean(main[0]))
        # the copies of COPY_BYTES are the largest copy dispatches of the run
        big = sorted(copy[0])[-3:]
        copy_avg = float(np.mean(big))
        # a copy of COPY_BYTES reads and writes COPY_BYTES once each
        scale = COPY_BYTES / copy_avg
        res[counter] = {"kernel_counter_avg": main_avg, "copy_counter_avg": copy_avg,
                        "bytes_per_unit": scale, "bytes": main_avg * scale,
                        "dispatches": len(main[0])}
    rec = {"kernel": KERNEL, "kernel_source_sha1": kernel_source_hash(),
           "bytes_per_launch": res["FETCH_SIZE"]["bytes"] + res["WRITE_SIZE"]["bytes"],
           "counters": res}
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--traffic-parse":
        traffic_parse(sys.argv[2], sys.argv[3], sys.argv[4])
    else:
        main()
