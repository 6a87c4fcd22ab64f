"""Throughput benchmark: concealed 16x16 blocks/s on a 1080p frame with 25 %
dispersed block loss (one MI355X).

One step = the whole concealment of one 1920x1080 luma frame through the C
ABI (loss geometry, rounds, context/flatness gate, candidate distances,
weights, weighted averages, write-back), with the frame and mask already in
HBM.  Prints ONE JSON line.

Other workloads print a line of their own (not the headline):
  --workload plain512   plain and full K-MMSE on a 512x512 image, 64 isolated blocks
  --workload batch      64 mixed frames (720p, 1080p, 2160p; B 8 or 16; scattered
                        or slice loss) in one skm_conceal_batch call
  --workload stream4k   120 frames of 3840x2160 YUV 4:2:0, 30 % bursty loss
  --geometry patch      the paper's 2x2 patches on the headline frame

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode cnn|profile|plain|...]
       python bench.py --traffic-run --steps 3          (under rocprofv3 --pmc)
       python bench.py --traffic-parse FETCH_DIR WRITE_DIR OUT.json FRAMES_PER_LAUNCH
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
# Published MI355X peaks.  The estimation kernel's arithmetic runs on the
# vector ALUs (int16 dot products for the distances, FP32 FMA for the
# weighted sums): its roofline is the FP32 vector peak.  The int8 MFMA peak is
# reported beside it for the distance stage, the HBM peak for the gather and
# weighted-sum traffic.
VALU_PEAK_TOPS = 157.3      # FP32 vector, TFLOP/s
INT8_MFMA_PEAK_TOPS = 5000.0
HBM_PEAK_GBS = 8000.0
KERNEL = "k_round_main"   # matches the batched k_round_main_b too


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
    """Algorithmic work of one launch of the estimation kernel on this frame.

    Distance stage: one multiply-accumulate per pair of context pixels
    compared, summed over every admissible candidate (2 ops per MAC).
    Weighted sum: one FMA per prototype pixel per candidate inside the
    accepted radius (2 ops).  Context-mean blocks: one add per known context
    pixel.  Returns a dict of op counts."""
    W = (d_tab.shape[1] - 1) // 2
    yy, xx = np.mgrid[-W:W + 1, -W:W + 1]
    rad = np.maximum(np.abs(yy), np.abs(xx))
    dist = wsum = brl = 0
    for k, inf in enumerate(info):
        if inf["layer"] == 0 and inf["n_cand"] < 0:
            brl += int(inf["n_ctx"])
            continue
        ok = d_tab[k] >= 0
        dist += 2 * int(n_tab[k][ok].sum())
        if inf["layer"] == 1:
            wsum += 2 * b * b * int((ok & (rad <= inf["radius"])).sum())
    return {"distance_ops": dist, "weighted_sum_ops": wsum, "brl_ops": brl,
            "total": dist + wsum + brl}


def algorithmic_bytes(frame, n_lost, b):
    """HBM bytes of one launch of the estimation kernel that the method needs:
    one read of the 8-bit plane and one write of the lost blocks' pixels."""
    return int(frame.size) + int(n_lost) * b * b


def roofline_record(ops, nbytes, k_ms, traffic, launches, frames_per_launch):
    sec = k_ms * 1e-3
    achieved = ops["total"] / sec / 1e12
    hbm = nbytes / sec / 1e9
    rec = {
        "kernel": KERNEL,
        "bound": "alu",
        "achieved": achieved,
        "peak": VALU_PEAK_TOPS,
        "unit": "TOP/s",
        "frac": achieved / VALU_PEAK_TOPS,
        "traffic": traffic,
        "ops_per_launch": ops,
        "int8_mfma_distance_stage": {
            "achieved_tops": ops["distance_ops"] / sec / 1e12, "peak_tops": INT8_MFMA_PEAK_TOPS,
            "frac": ops["distance_ops"] / sec / 1e12 / INT8_MFMA_PEAK_TOPS,
            "note": "distances run on VALU int16 dot products, not MFMA"},
        "hbm": {"algorithmic_bytes": nbytes, "achieved_gbs": hbm, "peak_gbs": HBM_PEAK_GBS,
                "frac": hbm / HBM_PEAK_GBS,
                "counter_bytes": traffic,
                "counter_frac": (traffic / sec / 1e9 / HBM_PEAK_GBS) if traffic else None,
                "counter_over_algorithmic": (traffic / nbytes) if traffic else None},
        "kernel_ms": k_ms,
        "launches_timed": launches,
        "frames_per_launch": frames_per_launch,
        "kernel_timing": "HIP events around each launch on the stream it is launched on, over "
                         "a second run of the timed batch (eager launches, one batch in flight)",
    }
    return rec


def traffic_from_profile(kernel_src_hash, frames_per_launch):
    """Counter bytes of one estimation-kernel launch covering
    frames_per_launch frames, from the committed counter record (None when
    it was taken on other kernel sources)."""
    path = os.path.join(ROOT, "profiles", "traffic_k_round_main_1080p.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha1") != kernel_src_hash:
        return None
    per_frame = rec.get("bytes_per_frame")
    return None if per_frame is None else per_frame * frames_per_launch


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
    ap.add_argument("--kernel-run", action="store_true",
                    help="only single-frame calls of the 1080p frame for kernel traces and "
                         "counters: plain and CNN mode, the gate at several grids, the gate "
                         "network alone, the distance table")
    ap.add_argument("--geometry", choices=("block", "patch"), default="block",
                    help="patch: the paper's 2x2 patches with a 6x6 context on the same frame "
                         "(a line of its own; the default line is the block workload)")
    ap.add_argument("--workload", choices=("layered1080p", "plain512", "batch", "stream4k"),
                    default="layered1080p",
                    help="layered1080p: the headline line; the others print a line of their own")
    ap.add_argument("--distinct", type=int, default=16,
                    help="stream4k: distinct generated frames, cycled over the 120-frame stream")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(blocks of a round are independent; frames or bands would shard "
              "across GPUs).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    t_nu = {"express": 0.01, "efficient": 0.1, "excellent": 100.0}[args.profile]
    if args.workload == "plain512":
        return bench_plain512(args)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "stream4k":
        return bench_stream4k(args)
    frame, mask = synth.workload_layered_1080p()
    if args.traffic_run:
        return traffic_run(args, frame, mask)
    if args.kernel_run:
        return kernel_run(args, frame, mask)
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

    # launch configuration picked by the library's autotuner on a batch of the
    # timed size (this also sizes the workspaces, so that no allocation falls
    # in the timed region)
    tune_ms = ctx.autotune(jobs_for(p_lay, args.steps), reps=3)
    tuned = {"batch_mode": ctx.get_option(skm.OPT_BATCH_MODE),
             "group_split": ctx.get_option(skm.OPT_GROUP_SPLIT),
             "batch_streams": ctx.get_option(skm.OPT_BATCH_STREAMS),
             "graphs": ctx.get_option(skm.OPT_GRAPHS),
             "gate_grid": ctx.get_option(skm.OPT_GATE_GRID), "tune_batch_ms": tune_ms}
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
    # every frame of this workload takes one round: a launch of the batched
    # estimation kernel covers steps / launches frames (1 in frame-pipeline mode)
    frames_per_launch = args.steps / max(launches, 1)
    print(f"# layered ({args.mode}): {sec_lay * 1e3:.3f} ms/frame ({sec_lay_ev * 1e3:.3f} with "
          f"event timing), estimation kernel {k_ms * 1e3:.1f} us per launch of "
          f"{frames_per_launch:.0f} frames", file=sys.stderr, flush=True)
    lat_lay = timed_single(p_lay, min(args.steps, 20))
    sec_plain = timed_batch(p_plain)
    print(f"# plain: {sec_plain * 1e3:.3f} ms/frame", file=sys.stderr, flush=True)
    sec_prof = timed_batch(p_prof)
    print(f"# profile rule: {sec_prof * 1e3:.3f} ms/frame", file=sys.stderr, flush=True)

    # statistics of one frame per mode (not timed)
    o_lay, info_lay, _ = ctx.conceal_device(fd, md, p_lay, want_xhat=False)
    o_prof, info_prof, _ = ctx.conceal_device(fd, md, p_prof, want_xhat=False)
    o_plain, _, _ = ctx.conceal_device(fd, md, p_plain, want_xhat=False)
    o_full, info_full, _ = ctx.conceal_device(fd, md, skm.default_params(mode="full"),
                                              want_xhat=False)
    d_tab, n_tab = ctx.distances_device(fd, md, p_plain)
    d_tab, n_tab = d_tab.cpu().numpy(), n_tab.cpu().numpy()
    n_lost = len(info_lay)
    ops = algorithmic_ops(d_tab, n_tab, info_lay, 16)
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
                     f"outputs in 8 rotating buffers), launch configuration from skm_autotune "
                     f"on a batch of the same size",
            "launch_config": tuned,
            "single_frame_latency_ms": lat_lay * 1e3,
            "psnr_layered_db": ps_lay,
            "psnr_full_kmmse_db": ps_full,
            "delta_psnr_db": ps_full - ps_lay,
            # layers of the reference itself: on this lattice no block has an
            # HQL candidate set, so full K-MMSE conceals every block by IDL
            "full_kmmse_layers": layer_counts(info_full),
            "layers": layer_counts(info_lay),
            "plain": {"blocks_per_s": n_lost / sec_plain, "ms_per_frame": sec_plain * 1e3,
                      "delta_psnr_db": ps_full - ps_plain},
            "speedup_vs_plain": sec_plain / sec_lay,
            "profile_rule": {"blocks_per_s": n_lost / sec_prof, "ms_per_frame": sec_prof * 1e3,
                             "delta_psnr_db": ps_full - ps_prof,
                             "layers": layer_counts(info_prof)},
        },
        "roofline": roofline_record(
            {k: v * frames_per_launch for k, v in ops.items()},
            algorithmic_bytes(frame, n_lost, 16) * frames_per_launch, k_ms,
            traffic_from_profile(kernel_source_hash(), frames_per_launch), launches,
            frames_per_launch),
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    ctx.close()


# ------------------------------------------------------ other workloads

def _line(metric, value, unit, args, ms_per_step, config, higher=True, **extra):
    rec = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": higher,
           "scaling": "weak", "vs_baseline": None, "dtype": "i32+f32+f64", "data": "synthetic",
           "config": config}
    rec.update(extra)
    print(json.dumps(rec), flush=True)


def _timed_batches(ctx, jobs, steps, warmup):
    """`warmup` untimed skm_conceal_batch calls over `jobs`, then `steps` timed
    ones; returns seconds per call and the last call's results.  Each call
    prints a progress line (after it returns)."""
    import torch
    for k in range(max(warmup, 1)):
        t = time.perf_counter()
        ctx.conceal_batch(jobs)
        print(f"# warm-up call {k}: {time.perf_counter() - t:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        res = ctx.conceal_batch(jobs)
        print(f"# timed call {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / max(steps, 1)
    if any(r[2] != 0 for r in res):
        raise SystemExit(f"batch status {[r[2] for r in res]}")
    return sec, res


def _oracle_blocks(args):
    f, m, mode = args
    from oracle.skmmse import Params, estimate_block, lost_cells
    u = np.where(m == 0, f, 0).astype(np.int64)
    t0 = time.perf_counter()
    cells = lost_cells(m, 16)
    for by, bx in cells:
        estimate_block(u, m == 0, by, bx, Params(mode=mode))
    return len(cells), time.perf_counter() - t0


def bench_plain512(args):
    """Plain (fixed-bandwidth IDL over the whole window) and full K-MMSE (HQL
    wherever 64 complete candidates exist) on the 512x512 image with 64
    isolated lost blocks: blocks/s and ms per block, one frame per step
    (frames of a step's batch in flight together)."""
    import torch
    import paper_2205_11226_amd as skm
    frame, mask = synth.workload_plain_512()
    fd, md = torch.from_numpy(frame).cuda(), torch.from_numpy(mask).cuda()
    outs = [torch.empty_like(fd) for _ in range(8)]
    ctx = skm.Context(0)
    res = {}
    for mode in ("plain", "full"):
        p = skm.default_params(mode=mode)
        o, info, _ = ctx.conceal_device(fd, md, p, want_xhat=False)
        jobs = [(fd, md, outs[j % 8], p) for j in range(args.steps)]
        sec, _ = _timed_batches(ctx, jobs, 1, args.warmup)
        sec /= args.steps
        n = len(info)
        res[mode] = {"blocks_per_s": n / sec, "ms_per_frame": sec * 1e3,
                     "ms_per_block_sequential_equiv": sec * 1e3 / n,
                     "psnr_db": psnr(o.cpu().numpy(), frame),
                     "layers": {"brl": int((info["layer"] == 0).sum()),
                                "idl": int((info["layer"] == 1).sum()),
                                "hql": int((info["layer"] == 2).sum())}}
        print(f"# {mode}: {sec * 1e3:.3f} ms/frame", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(2) as pool:
            r = pool.map(_oracle_blocks, [(frame, mask, "plain"), (frame, mask, "full")])
        cpu = {"value": r[1][0] / r[1][1], "unit": "blocks/s", "cores": 1, "kind": "oracle",
               "sample": f"all {r[1][0]} blocks of the frame, float64 NumPy oracle on one core "
                         f"each: full K-MMSE {r[1][1]:.2f} s, plain {r[0][1]:.2f} s "
                         f"({r[0][0] / r[0][1]:.1f} blocks/s)"}
    ctx.close()
    _line("full K-MMSE blocks/s, 512x512, 64 isolated 16x16 blocks", res["full"]["blocks_per_s"],
          "blocks/s", args, res["full"]["ms_per_frame"],
          {"workload": "512x512 luma (40 bumps, 12 edges), 64 isolated 16x16 lost blocks, "
                       "plain and full K-MMSE, one frame per step", "modes": res},
          cpu_baseline=cpu)


def _gen_batch(args):
    base, f, hw = args
    return synth.workload_batch(1, seed=base + f, sizes=[hw])[0]


def bench_batch(args):
    """The mixed batch: 24 x 1280x720, 32 x 1920x1080, 8 x 3840x2160 frames;
    per frame the seed picks B (8 or 16) and scattered (10-30 %) or slice
    (5-50 %) loss.  One step = one skm_conceal_batch call over the 64 frames
    in --mode (default: layered with the learned gate), launch configuration
    from skm_autotune."""
    import multiprocessing as mp
    import torch
    import paper_2205_11226_amd as skm
    sizes = [(720, 1280)] * 24 + [(1080, 1920)] * 32 + [(2160, 3840)] * 8
    base = synth.seed_for(3)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        frames = pool.map(_gen_batch, [(base, f, hw) for f, hw in enumerate(sizes)])
    print(f"# generated 64 frames in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    ctx = skm.Context(0)
    ctx.cnn_load(args.weights)
    jobs, n_px = [], 0
    for w in frames:
        fd = torch.from_numpy(w["frame"]).cuda()
        md = torch.from_numpy(w["mask"]).cuda()
        jobs.append((fd, md, torch.empty_like(fd), skm.default_params(mode=args.mode,
                                                                      block=w["block"])))
        n_px += w["frame"].size
    # launch configuration tuned on one frame of each size (the batch itself
    # takes seconds per call in CNN mode with HQL blocks)
    sub = [jobs[0], jobs[24], jobs[56]]
    tune_ms = ctx.autotune(sub, reps=1)
    print(f"# autotuned on 3 frames: {tune_ms:.2f} ms", file=sys.stderr, flush=True)
    sec, res = _timed_batches(ctx, jobs, args.steps, args.warmup)
    blocks = sum(r[0] for r in res)
    rounds = [r[1] for r in res]
    tuned = {"batch_mode": ctx.get_option(skm.OPT_BATCH_MODE),
             "group_split": ctx.get_option(skm.OPT_GROUP_SPLIT),
             "batch_streams": ctx.get_option(skm.OPT_BATCH_STREAMS),
             "graphs": ctx.get_option(skm.OPT_GRAPHS),
             "gate_grid": ctx.get_option(skm.OPT_GATE_GRID), "tune_batch_ms": tune_ms}
    ctx.close()
    kinds = {}
    for w in frames:
        key = f"B{w['block']}-{w['kind']}"
        kinds[key] = kinds.get(key, 0) + 1
    _line("concealed blocks/s, 64-frame mixed batch (720p/1080p/2160p, B 8|16, scattered|slice "
          "loss)", blocks / sec, "blocks/s", args, sec * 1e3,
          {"workload": "64 frames: 24 x 1280x720, 32 x 1920x1080, 8 x 3840x2160 luma; per frame "
                       "B 8|16 and scattered 10-30 % or slice 5-50 % loss by seed; one "
                       "skm_conceal_batch call over the 64 frames per step",
           "mode": args.mode, "frames_per_s": 64 / sec, "megapixels": n_px / 1e6,
           "lost_blocks": blocks, "rounds_max": max(rounds), "frame_kinds": kinds,
           "launch_config": tuned})


def _gen_stream(k):
    return synth.workload_stream_4k(k)


def bench_stream4k(args):
    """120 frames of 3840x2160 YUV 4:2:0 (Y in 16x16 blocks, U and V in 8x8
    cells co-located with the lost luma macroblocks), 30 % random loss in
    bursts of up to 4 blocks, layered with the learned gate.  `--distinct`
    frames are generated and cycled over the 120 (each a different input in
    HBM; more than the last-level cache holds).  One step = one
    skm_conceal_batch call over the 360 planes of the 120 frames.  Delta PSNR
    (full K-MMSE minus layered) over frames 0-9, untimed."""
    import multiprocessing as mp
    import torch
    import paper_2205_11226_amd as skm
    nd = max(10, args.distinct)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        gen = pool.map(_gen_stream, range(nd))
    print(f"# generated {nd} frames in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    ctx = skm.Context(0)
    ctx.cnn_load(args.weights)
    dev = []
    for planes, masks in gen:
        dev.append([(torch.from_numpy(p).cuda(), torch.from_numpy(m).cuda()) for p, m in
                    zip(planes, masks)])
    prm = {16: skm.default_params(mode=args.mode, block=16),
           8: skm.default_params(mode=args.mode, block=8)}
    full = {16: skm.default_params(mode="full", block=16),
            8: skm.default_params(mode="full", block=8)}
    jobs = []
    for k in range(120):
        for c, (fd, md) in enumerate(dev[k % nd]):
            jobs.append((fd, md, torch.empty_like(fd), prm[16 if c == 0 else 8]))
    tune_ms = ctx.autotune(jobs[:6], reps=1)
    print(f"# autotuned on 2 frames: {tune_ms:.2f} ms", file=sys.stderr, flush=True)
    sec, res = _timed_batches(ctx, jobs, args.steps, args.warmup)
    blocks = sum(r[0] for r in res)
    luma_blocks = sum(r[0] for r in res[0::3])
    # quality over frames 0-9 (untimed)
    d_lay, d_full = [], []
    for k in range(10):
        (yf, ym) = dev[k][0]
        o_l, _, _ = ctx.conceal_device(yf, ym, prm[16], want_info=False, want_xhat=False)
        o_f, _, _ = ctx.conceal_device(yf, ym, full[16], want_info=False, want_xhat=False)
        truth = gen[k][0][0]
        d_lay.append(psnr(o_l.cpu().numpy(), truth))
        d_full.append(psnr(o_f.cpu().numpy(), truth))
    ctx.close()
    _line("concealed 4K YUV 4:2:0 frames/s, 30% bursty 16x16 loss, layered+CNN",
          120 / sec, "frames/s", args, sec * 1e3 / 120,
          {"workload": f"120 frames of 3840x2160 YUV 4:2:0 ({nd} distinct generated frames "
                       "cycled), Y in 16x16 blocks, U/V in co-located 8x8 cells, 30 % random "
                       "loss in bursts of <= 4; one skm_conceal_batch over the 360 planes per "
                       "step", "mode": args.mode,
           "blocks_per_s": blocks / sec, "lost_blocks_per_frame": blocks / 120,
           "luma_blocks_per_frame": luma_blocks / 120, "tune_ms": tune_ms,
           "psnr_luma_layered_db_frames0_9": float(np.mean(d_lay)),
           "psnr_luma_full_kmmse_db_frames0_9": float(np.mean(d_full)),
           "delta_psnr_db_frames0_9": float(np.mean(d_full) - np.mean(d_lay))})


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
    # the timed configuration: one skm_conceal_batch over --steps frames
    # (batched kernels: one estimation launch covers every frame)
    outs = [torch.empty_like(fd) for _ in range(8)]
    ctx.conceal_batch([(fd, md, outs[j % 8], p) for j in range(args.steps)])
    src = torch.ones(COPY_BYTES, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ctx.close()
    print(f"# traffic run: one batch of {args.steps} frames, 3 copies of {COPY_BYTES} bytes",
          flush=True)


def kernel_run(args, frame, mask):
    """Single-frame calls in a fixed order, for `rocprofv3 --kernel-trace` or
    `--pmc` (one dispatch list per phase): 20 plain frames, 20 CNN frames at
    the default gate grid, 10 CNN frames at each of the gate grids 768, 1280,
    2560 and 4096, 10 runs of the gate network alone on the frame's lost
    blocks, 5 distance tables."""
    import torch
    import paper_2205_11226_amd as skm
    fd = torch.from_numpy(frame).cuda()
    md = torch.from_numpy(mask).cuda()
    ctx = skm.Context(0)
    ctx.cnn_load(args.weights)
    for mode in ("plain", "cnn"):
        p = skm.default_params(mode=mode)
        for _ in range(20):
            ctx.conceal_device(fd, md, p, want_info=False, want_xhat=False)
        torch.cuda.synchronize()
    p = skm.default_params(mode="cnn")
    default_grid = ctx.get_option(skm.OPT_GATE_GRID)
    for grid in (768, 1280, 2560, 4096):
        ctx.set_option(skm.OPT_GATE_GRID, grid)
        for _ in range(10):
            ctx.conceal_device(fd, md, p, want_info=False, want_xhat=False)
        torch.cuda.synchronize()
    ctx.set_option(skm.OPT_GATE_GRID, default_grid)
    x = ctx.cnn_inputs(fd, md, skm.default_params(mode="profile"))
    for _ in range(10):
        ctx.cnn_forward(x)
    pp = skm.default_params(mode="plain")
    for _ in range(5):
        ctx.distances_device(fd, md, pp)
    torch.cuda.synchronize()
    ctx.close()
    print(f"# kernel run: {x.shape[0]} lost blocks", flush=True)


def _counter_rows(d):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        rows += list(csv.DictReader(open(f)))
    if not rows:
        raise SystemExit(f"no counter_collection.csv under {d}")
    return rows


def traffic_parse(fetch_dir, write_dir, out_path, frames_per_launch):
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
    per_launch = res["FETCH_SIZE"]["bytes"] + res["WRITE_SIZE"]["bytes"]
    rec = {"kernel": KERNEL, "kernel_source_sha1": kernel_source_hash(),
           "frames_per_launch": frames_per_launch,
           "bytes_per_launch": per_launch, "bytes_per_frame": per_launch / frames_per_launch,
           "counters": res}
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--traffic-parse":
        traffic_parse(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]))
    else:
        main()
