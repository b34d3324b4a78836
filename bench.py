#!/usr/bin/env python3
"""Benchmark of the MI355X Difference-of-Gaussians blob detector.

Headline: Mpixel-scales/s of the whole detector path (blur stack, DoG,
3x3x3 local maxima with threshold, compaction, readback, host sort and
pruning) on one 1024x1024 fp32 camera frame (500 blobs, sigma 1..30, ratio
1.6 -> 8 DoG planes, threshold 0.05, overlap 0.5) already resident in HBM.
Mpixel-scales = H * W * k per frame.  A step is one frame from launch to its
pruned blob list on the host; three contexts, each on its own stream, are
used in turn, so steps i+1 and i+2 are queued before step i's blobs are
collected (three frames in flight, --inflight).

Also printed in the same JSON line:
  * the same steps one synchronous call at a time: per-frame latency p50/p99
    and the unpipelined rate;
  * roofline of the dominant kernel, from HIP start/end events of each
    kernel's dispatch on the stream it runs on, during a further run of the
    same steps (issued directly: events inside a replayed graph cannot be
    timed);
  * the autotuner's per-variant timings for the frame and its choice;
  * a uniform batch of 64 1024x1024 frames through the batched entry point
    vs one frame at a time (throughput ratio and latency);
  * an uneven batch of 128 frames (sides 256..2048, square and 2:1 crops):
    batched vs per-frame on device frames, and the server at saturation vs
    the plain host entry point frame by frame;
  * the server fed by a Poisson stream of mixed frames (200 frames/s):
    p50/p99 latency and sustained frames/s;
  * the paper's own configuration (arithmetic ladder of Eq. 1 with n_bin = 10,
    truncate 5, coalescing) on the same frame;
  * preprocessing (smoothing + 0.35 % contrast stretch) of the frame's raw
    counts alone and in front of the detector;
  * overlap pruning and the radius histogram of the frame's candidates on
    the device against the host step;
  * the server fed by the same stream under an admission budget of 2.5
    footprints of the largest frame, so admission binds;
  * the FP64 CPU oracle timed on this host on a bounded sample, on one
    thread and on every core.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-batch] [--no-mixed]
                    [--no-serve] [--no-paper] [--serve-seconds S] [--no-cpu] [--variant V]
                    [--dct MIN_TAPS] [--inflight N] [--only paper|preprocess]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X figures used for the roofline: 256 CUs at 2.4 GHz, 128 FP32 FMAs per
# CU per clock.  Plain v_fma_f32 / v_fmac_f32 with vector-register operands
# reach this rate on gfx950 (a probe measured 138-152 TFLOP/s); the blur
# kernels use that form, so the published 157.3 TFLOP/s is the peak.
N_CU = 256
CLOCK_HZ = 2.4e9
FP32_FMA_PER_CU_CLK = 128
PEAK_FP32_TFLOPS = N_CU * CLOCK_HZ * FP32_FMA_PER_CU_CLK * 2 / 1e12   # 157.3
PEAK_HBM_GBS = 8000.0

PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "dog_kernels_frame1k_counters.txt")



def pct(a, q):
    import numpy as np
    return float(np.percentile(np.asarray(a), q))


def kernel_source_hash() -> str:
    from paper_2010_08486_amd.build import kernel_hash
    return kernel_hash()


def measured_traffic(kernel: str, variant: int, min_taps: int = 0):
    """HBM bytes per launch of `kernel` in kernel variant `variant` at
    transform threshold `min_taps` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel build and covers that
    configuration (else None)."""
    if not os.path.exists(PROFILE_COUNTERS):
        return None
    vals = {}
    for line in open(PROFILE_COUNTERS):
        line = line.strip()
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    key = "v%d.m%d.%s_hbm_bytes_per_launch" % (variant, min_taps, kernel)
    return float(vals[key]) if key in vals else None


def _gen(args):
    import synth
    kind, a = args
    if kind == "batch64":
        return synth.batch64(n_frames=1, first_seed=1000 + a)[0]
    H, W = a[1], a[2]
    return synth.mixed_frame(a[0], H, W)


def generate_inputs(want_batch: bool, want_mixed: bool, workers: int):
    """Synthetic frames of the batch workloads, generated in worker processes
    before this process touches the GPU."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import synth
    jobs = []
    if want_batch:
        jobs += [("batch64", f) for f in range(64)]
    if want_mixed:
        jobs += [("mixed", (f, H, W)) for f, (H, W) in enumerate(synth.mixed_shapes())]
    if not jobs:
        return [], []
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        frames = list(ex.map(_gen, jobs, chunksize=2))
    nb = 64 if want_batch else 0
    return frames[:nb], frames[nb:]


def cpu_model() -> str:
    """Model name of the host CPU (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def roofline_entry(name, flop, nbytes, ms, traffic):
    """Roofline of one launch from its algorithmic flops and bytes and its
    mean duration: bound by HBM when its arithmetic intensity is below the
    ridge point (FP32 peak / HBM peak, 19.7 flop per byte), by FP32
    arithmetic above; the other ceiling's fraction rides along."""
    t = ms * 1e-3
    ai = flop / nbytes
    ridge = PEAK_FP32_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)
    tf = flop / t / 1e12
    gbs = nbytes / t / 1e9
    r = {"kernel": name, "traffic": traffic, "algorithmic_flop_per_launch": flop,
         "algorithmic_bytes_per_launch": nbytes, "arithmetic_intensity": round(ai, 2),
         "ridge_point": round(ridge, 2), "frac_fp32_peak": round(tf / PEAK_FP32_TFLOPS, 4),
         "frac_hbm_peak": round(gbs / PEAK_HBM_GBS, 4)}
    if ai < ridge:
        r.update({"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                  "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4)})
    else:
        r.update({"bound": "alu", "achieved": round(tf, 3), "peak": round(PEAK_FP32_TFLOPS, 1),
                  "unit": "TFLOP/s", "frac": round(tf / PEAK_FP32_TFLOPS, 4)})
    return {k: r[k] for k in ("bound", "kernel", "achieved", "peak", "unit", "frac", "traffic",
                              "arithmetic_intensity", "ridge_point", "frac_fp32_peak",
                              "frac_hbm_peak", "algorithmic_flop_per_launch",
                              "algorithmic_bytes_per_launch")}


def blur_flops(radii, H, W, min_taps, merged):
    """Algorithmic FP32 flops per launch of the blur kernels of one H x W
    frame: 2 per tap and output pixel for the planes blurred directly; for
    the planes taken in the cosine-transform domain (kernels of at least
    min_taps taps) the transforms' flops, counted per pair of lines of N
    values as 5 N log2 N per complex FFT (one forward per pair, one inverse
    per plane) plus 8 N for the cosine coefficients and 14 N per plane for
    the inverse sequence.  Pass 1 takes the frame's rows (N = W, H / 2
    pairs, every transform plane from one forward transform: the forward
    transforms the kernels repeat per plane are not counted); pass 2 the
    planes' columns (N = H, W / 2 pairs per plane).  merged: the jobs run in
    the blur passes' launches (their flops count there), else in fft1 / fft2."""
    import math
    taps = [2 * int(r) + 1 for r in radii]
    tr = [t for t in taps if min_taps > 0 and t >= min_taps]
    direct = 2.0 * (sum(taps) - sum(tr)) * H * W
    n_tr = len(tr)

    def job(N, planes):
        return 5.0 * N * math.log2(N) * (1 + planes) + 8.0 * N + 14.0 * N * planes

    f1 = (H / 2) * job(W, n_tr) if n_tr else 0.0
    f2 = n_tr * (W / 2) * job(H, 1) if n_tr else 0.0
    out = {"pass1": direct, "pass2": direct, "nms": 0.0, "fft1": f1, "fft2": f2,
           "merged": merged}
    if merged:
        out["pass1"] += f1
        out["pass2"] += f2
        out["fft1"] = out["fft2"] = 0.0
    return out


def cpu_baseline(img, prm, k, budget_s=10.0):
    """The FP64 C oracle on the same frame: once on one thread, then repeated
    on every core this process may use (OpenMP over rows), for about
    budget_s seconds."""
    import oracle
    oracle.build()
    cores = len(os.sched_getaffinity(0))
    H, W = img.shape

    def run():
        t0 = time.perf_counter()
        oracle.detect_c(img, prm.sigma_min, prm.sigma_max, prm.sigma_ratio, prm.threshold,
                        prm.overlap, 4.0)
        return time.perf_counter() - t0

    oracle.set_threads(1)
    t_one = run()
    oracle.set_threads(cores)
    n_threads = oracle.get_threads()
    reps, t_total = 0, 0.0
    while t_total < budget_s and reps < 50:
        t_total += run()
        reps += 1
    per = t_total / reps
    return {"value": round(H * W * k / per / 1e6, 3), "unit": "Mpixel-scales/s",
            "cores": n_threads, "kind": "oracle", "cpu_model": cpu_model(),
            "all_cores_s_per_frame": round(per, 3),
            "single_thread_s_per_frame": round(t_one, 3),
            "single_thread_mpx_scales_per_s": round(H * W * k / t_one / 1e6, 3),
            "sample": "the FP64 C oracle (ladder, planes, local maxima, pruning) on the same "
                      "1024x1024 frame: 1 run on one thread (%.1f s), then %d runs on %d threads "
                      "(%.1f s)" % (t_one, reps, n_threads, t_total)}


def bench_prune(dog, torch, ctx, t_img, prm, reps=50):
    """Overlap pruning and the radius histogram of the frame's candidates: on
    the device (dog_prune_device, the list already in HBM) against the host
    step (dog_prune, the list in host memory), same result."""
    raw = ctx.debug_candidates(t_img, prm)
    d = torch.from_numpy(raw.view("u1").reshape(-1).copy()).cuda()
    out = {"candidates": int(len(raw))}
    import dataclasses
    for name, par in (("prune", prm), ("coalesce", dataclasses.replace(prm, coalesce=True))):
        ref = dog.prune(par, raw)
        got, _ = ctx.prune_device(d, par)
        assert got.tobytes() == ref.tobytes()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.prune_device(d, par)
        t_dev = (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        for _ in range(reps):
            dog.prune(par, raw)
            dog.radius_histogram(par, ref)
        t_host = (time.perf_counter() - t0) / reps
        out[name] = {"kept": int(len(ref)), "device_call_us": round(t_dev * 1e6, 1),
                     "host_call_us": round(t_host * 1e6, 1)}
    return out


def bench_mixed(dog, torch, ctx, prm, k, frames, steps, tune_cache):
    """Uneven batch of 128 frames: one batched launch sequence vs a launch per
    frame (device frames), and the server at saturation vs the plain host
    entry point frame by frame (host frames)."""
    dev = torch.device("cuda:0")
    dfr = [torch.from_numpy(f).to(dev) for f in frames]
    tot = sum(f.shape[0] * f.shape[1] for f in frames) * k / 1e6
    shapes = sorted({f.shape for f in frames}, key=lambda s: s[0] * s[1])
    choice, transform = {}, {}
    for shp in shapes:   # the autotuner picks a variant and transform threshold per frame size
        f = next(t for t in dfr if tuple(t.shape) == shp)
        choice["%dx%d" % shp] = ctx.autotune(f, prm, reps=3)[0]
        transform["%dx%d" % shp] = ctx.autotune_transform(prm, shp[0], shp[1])
    ctx.autotune_save(tune_cache)   # the servers' slots load the same choices
    torch.cuda.synchronize()
    ctx.detect_batch(dfr, prm)
    ctx.detect_batch(dfr, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res, _ = ctx.detect_batch(dfr, prm)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / steps
    for f in dfr[:8]:
        ctx.detect_device(f, prm)
    torch.cuda.synchronize()
    per = []
    t0 = time.perf_counter()
    for f in dfr:
        s0 = time.perf_counter()
        ctx.detect_device(f, prm)
        per.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    # host frames: plain per-frame entry point vs the server fed all at once
    for f in frames[:4]:
        dog.detect(f, prm.sigma_min, prm.sigma_max, prm.sigma_ratio, prm.threshold, prm.overlap)
    t0 = time.perf_counter()
    for f in frames:
        dog.detect(f, prm.sigma_min, prm.sigma_max, prm.sigma_ratio, prm.threshold, prm.overlap)
    th = time.perf_counter() - t0

    def served(fr, reps=2):
        """Time the server on all frames submitted at once; the first pass
        warms its pinned request buffers and the slots' workspaces."""
        sv = dog.Server(prm, max_batch_frames=32, tune_cache=tune_cache)
        try:
            best, st = None, None
            for _ in range(reps):
                b0 = sv.stats()["batches"]
                t0 = time.perf_counter()
                tickets = [sv.submit(f) for f in fr]
                for tk in tickets:
                    sv.wait(tk)
                dt = time.perf_counter() - t0
                s1 = sv.stats()
                if best is None or dt < best:
                    best, st = dt, (len(fr) / max(1, s1["batches"] - b0))
            return best, st
        finally:
            sv.close()

    ts, mean_b = served(frames)
    tsd, mean_bd = served(dfr)
    del dfr
    return {"frames": len(frames), "mpixel_scales": round(tot, 1),
            "autotuned_variant_per_shape": choice,
            "autotuned_transform_min_taps_per_shape": transform,
            "batched_mpx_scales_per_s": round(tot / tb, 1),
            "per_frame_device_mpx_scales_per_s": round(tot / tp, 1),
            "batched_over_per_frame_device": round(tp / tb, 3),
            "batched_ms_per_batch": round(tb * 1e3, 3),
            "per_frame_device_p50_ms": round(pct(per, 50) * 1e3, 4),
            "per_frame_device_p99_ms": round(pct(per, 99) * 1e3, 4),
            "host_per_frame_mpx_scales_per_s": round(tot / th, 1),
            "served_host_frames_mpx_scales_per_s": round(tot / ts, 1),
            "served_host_over_host_per_frame": round(th / ts, 3),
            "served_host_mean_batch_frames": round(mean_b, 2),
            "served_device_frames_mpx_scales_per_s": round(tot / tsd, 1),
            "served_device_over_per_frame_device": round(tp / tsd, 3),
            "served_device_mean_batch_frames": round(mean_bd, 2)}


def bench_paper_config(dog, torch, t_img, steps, nf):
    """The paper's own configuration on the same frame: arithmetic ladder of
    Sec. 4 Eq. 1 (n_bin = 10 over sigma 1..30), truncate 5, coalescing by
    averaging the radius; threshold 0.05 as in the headline workload.  Same
    pipelined steps as the headline (nf frames in flight)."""
    prm = dog.Params.paper(1.0, 30.0, 10, threshold=0.05)
    info = dog.plan_info(prm)
    k = info["k"]
    H, W = t_img.shape
    ctxs = [dog.Context(0) for _ in range(nf)]
    streams = [torch.cuda.Stream() for _ in range(nf)]
    try:
        v, _ = ctxs[0].autotune(t_img, prm, reps=3)
        mt = ctxs[0].autotune_transform(prm, H, W)
        for c, st in zip(ctxs, streams):
            c.set_variant(v)
            c.set_dct(mt)
            for _ in range(3):
                c.detect_device(t_img, prm, stream=st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(nf - 1):
            ctxs[i].detect_device_async(t_img, prm, stream=streams[i])
        for i in range(nf - 1, steps + nf - 1):
            if i < steps:
                ctxs[i % nf].detect_device_async(t_img, prm, stream=streams[i % nf])
            blobs = ctxs[(i - nf + 1) % nf].finish()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        ctxs[0].set_profiling(True)
        for _ in range(20):
            ctxs[0].detect_device(t_img, prm)
        kms, n = ctxs[0].kernel_times_all()
        taps = int((2 * info["radii"] + 1).sum())
        avg = [m / max(n, 1) for m in kms]
        fl = blur_flops(info["radii"], H, W, mt, merged=avg[3] == 0.0 and avg[4] == 0.0)
        return {"ladder": "arithmetic n_bin=10, sigma 1..30, truncate 5, coalesce",
                "dog_planes": k, "taps_per_pass": taps, "variant": v,
                "transform_min_taps": mt,
                "mpx_scales_per_s": round(H * W * k / dt / 1e6, 1),
                "ms_per_frame": round(dt * 1e3, 4),
                "kernel_avg_us": {nm: round(m * 1e3, 2)
                                  for nm, m in zip(dog.Context.KERNEL_NAMES, avg)},
                "pass1_tflops": round(fl["pass1"] / (avg[0] * 1e-3) / 1e12, 2),
                "blobs": int(len(blobs))}
    finally:
        for c in ctxs:
            c.close()


def bench_preprocess(dog, torch, img, prm, k, steps, nf, variant, min_taps):
    """Sec. 4.1's optional first step on raw camera counts of the headline
    frame: smoothing (sigma 1) and a 0.35 % contrast stretch alone, then the
    whole pipeline (preprocess + detector, with the headline's blur variant,
    8 if none was tuned, and transform threshold) with nf frames in flight."""
    import numpy as np
    counts = torch.from_numpy((img * 65535.0).astype(np.float32)).cuda()
    H, W = counts.shape
    ctxs = [dog.Context(0) for _ in range(nf)]
    streams = [torch.cuda.Stream() for _ in range(nf)]
    outs = [torch.empty((H, W), dtype=torch.float32, device="cuda") for _ in range(nf)]
    try:
        c0 = ctxs[0]
        for _ in range(5):
            c0.preprocess(counts, 1.0, 0.0035, out=outs[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            c0.preprocess(counts, 1.0, 0.0035, out=outs[0])
        torch.cuda.synchronize()
        t_pre = (time.perf_counter() - t0) / steps
        for c, st, o in zip(ctxs, streams, outs):
            c.set_variant(variant if variant >= 0 else 8)
            c.set_dct(min_taps)
            for _ in range(3):
                c.preprocess(counts, 1.0, 0.0035, out=o, stream=st)
                c.detect_device(o, prm, stream=st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(nf - 1):
            ctxs[i].preprocess(counts, 1.0, 0.0035, out=outs[i], stream=streams[i])
            ctxs[i].detect_device_async(outs[i], prm, stream=streams[i])
        for i in range(nf - 1, steps + nf - 1):
            if i < steps:
                j = i % nf
                ctxs[j].preprocess(counts, 1.0, 0.0035, out=outs[j], stream=streams[j])
                ctxs[j].detect_device_async(outs[j], prm, stream=streams[j])
            blobs = ctxs[(i - nf + 1) % nf].finish()
        torch.cuda.synchronize()
        t_pipe = (time.perf_counter() - t0) / steps
        # bytes per pixel the four kernels move: smoothing 4 in + 4 out (its
        # top-digit histogram rides along), two select passes 4 each, the
        # stretch 4 in + 4 out
        algo = 24.0 * H * W
        return {"smooth_sigma": 1.0, "saturated": 0.0035,
                "preprocess_us_per_frame": round(t_pre * 1e6, 2),
                "preprocess_algorithmic_gbs": round(algo / t_pre / 1e9, 1),
                "pipeline_ms_per_frame": round(t_pipe * 1e3, 4),
                "pipeline_mpx_scales_per_s": round(H * W * k / t_pipe / 1e6, 1),
                "blobs": int(len(blobs))}
    finally:
        for c in ctxs:
            c.close()


def bench_serving(dog, prm, k, pool, rate, seconds, budget=0, tune_cache=None):
    """The server fed by a Poisson stream: frames drawn in turn from the pool
    of uneven frames, submitted at their arrival times.  budget: the
    admission budget in bytes (0: the server's default); tune_cache: the
    autotuner's choices for the slots (dog_autotune_save), or None."""
    import synth
    arrivals = synth.poisson_arrivals(rate=rate, duration=seconds)
    sv = dog.Server(prm, max_batch_frames=16, hbm_budget_bytes=budget, tune_cache=tune_cache)
    try:
        for f in pool[:8]:
            sv.wait(sv.submit(f))
        base = sv.stats()
        tickets = []
        t0 = time.perf_counter()
        for i, ta in enumerate(arrivals):
            while True:
                now = time.perf_counter() - t0
                if now >= ta:
                    break
                time.sleep(min(ta - now, 0.002))
            tickets.append(sv.submit(pool[i % len(pool)]))
        lat = []
        for tk in tickets:
            _, info = sv.wait(tk)
            lat.append((info["t_done_ns"] - info["t_arrive_ns"]) / 1e6)
        wall = time.perf_counter() - t0
        st = sv.stats()
    finally:
        sv.close()
    mpx = sum(pool[i % len(pool)].size for i in range(len(arrivals))) * k / 1e6
    return {"rate_fps": rate, "seconds": seconds, "frames": len(arrivals),
            "p50_ms": round(pct(lat, 50), 3), "p99_ms": round(pct(lat, 99), 3),
            "max_ms": round(max(lat), 3),
            "sustained_fps": round(len(arrivals) / wall, 1),
            "mpx_scales_per_s": round(mpx / wall, 1),
            "batches": st["batches"] - base["batches"],
            "mean_batch_frames": round(len(arrivals) / max(1, st["batches"] - base["batches"]), 2),
            "budget_gib": round(budget / 2**30, 3) if budget else "default (90% of free HBM)",
            "peak_reserved_gib": round(st["peak_reserved_bytes"] / 2**30, 3),
            "peak_held_gib": round(st["peak_held_bytes"] / 2**30, 3),
            "admission_waits": st["admission_waits"] - base["admission_waits"]}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-paper", action="store_true")
    ap.add_argument("--only", choices=("paper", "preprocess"), default=None,
                    help="run only the paper-configuration or the preprocessing section "
                         "(for a profile of its kernels) and print its JSON")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--tight-serve-seconds", type=float, default=10.0,
                    help="length of the serving leg whose admission budget binds")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--dct", type=int, default=-1,
                    help="transform threshold in kernel taps (0: every plane direct; "
                         "-1: the autotuner's choice)")
    ap.add_argument("--inflight", type=int, default=3,
                    help="frames in flight in the timed steps (contexts and streams used in turn)")
    ap.add_argument("--pmc-workload", type=int, default=0,
                    help="only run N detector steps on the 1024x1024 frame, then a plain 256 MiB "
                         "device copy (the calibration for rocprofv3 byte counters), and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: frames are independent, so several GPUs would take "
              "whole frames each with no collective, and only the one-GPU measurement is "
              "implemented. Use --gpus 1.", file=sys.stderr)
        return 2

    import numpy as np

    import paper_2010_08486_amd as dog
    import synth

    pmc = args.pmc_workload > 0 or args.only is not None
    want_mixed = not pmc and not (args.no_mixed and args.no_serve)
    batch_frames, mixed_frames = generate_inputs(not pmc and not args.no_batch, want_mixed,
                                                 workers=min(16, os.cpu_count() or 1))

    import torch
    dev = torch.device("cuda:0")
    prm = dog.Params(1.0, 30.0, 1.6, 0.05, 0.5)
    info = dog.plan_info(prm)
    k = info["k"]
    radii = info["radii"]
    img = synth.camera_frame(seed=1)
    H, W = img.shape
    t_img = torch.from_numpy(img).to(dev)
    ctx = dog.Context(0)
    tune = None
    if args.variant >= 0:
        ctx.set_variant(args.variant)
    if args.dct >= 0:
        ctx.set_dct(args.dct)
    if args.variant < 0 and not pmc:
        v, us = ctx.autotune(t_img, prm, reps=7)
        tune = {"variant": v, "geometry": dog.variant_info(v),
                "kernel_us_per_variant": [round(u, 2) for u in us]}
    variant = tune["variant"] if tune else args.variant
    min_taps = ctx.autotune_transform(prm, H, W)   # the pinned one, else the tuned one
    if tune:
        tune["transform_min_taps"] = min_taps
        tune["transform_planes"] = [int(p) for p in range(k + 1)
                                    if min_taps > 0 and 2 * radii[p] + 1 >= min_taps]

    if args.only:
        # one section alone (for a profile of its kernels), as its JSON line
        nf = max(1, args.inflight)
        if args.only == "paper":
            sec = bench_paper_config(dog, torch, t_img, args.steps, nf)
        else:
            sec = bench_preprocess(dog, torch, img, prm, k, args.steps, nf, variant, min_taps)
        ctx.close()
        print(json.dumps({"section": args.only, args.only: sec}))
        return 0

    if args.pmc_workload > 0:
        for _ in range(args.pmc_workload):
            ctx.detect_device(t_img, prm)
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        ctx.close()
        print("pmc workload done", flush=True)
        return 0

    # N contexts with the same kernel variant, each launching on its own
    # stream: frames i+1 .. i+N-1 are queued before frame i's blobs are
    # collected, so the host work of one frame and the kernels of the others
    # overlap, and kernels of different frames share the GPU (one frame's
    # local-maximum pass, bound by memory, beside another's blur)
    nf = args.inflight
    if nf < 1:
        print("--inflight must be at least 1", file=sys.stderr)
        return 2
    ctxs = [ctx] + [dog.Context(0) for _ in range(nf - 1)]
    for c in ctxs[1:]:
        c.set_variant(variant)
        c.set_dct(min_taps)
    streams = [torch.cuda.Stream(device=dev) for _ in range(nf)]
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        for c, st in zip(ctxs, streams):
            c.detect_device(t_img, prm, stream=st)
    torch.cuda.synchronize()

    # ---- timed region: K whole-path steps, each one frame from launch to its
    # pruned blob list on the host
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(nf - 1):
        ctxs[i].detect_device_async(t_img, prm, stream=streams[i])
    for i in range(nf - 1, args.steps + nf - 1):
        if i < args.steps:
            ctxs[i % nf].detect_device_async(t_img, prm, stream=streams[i % nf])
        blobs = ctxs[(i - nf + 1) % nf].finish()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # ---- the same K steps one synchronous call at a time: per-frame
    # latency (call to blobs on the host) and the unpipelined rate
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        blobs_sync = ctx.detect_device(t_img, prm)
        lat.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    dt_sync = time.perf_counter() - t0
    assert blobs_sync.tobytes() == blobs.tobytes()

    # ---- kernel-timing region: the same K steps with HIP start/end events of
    # each kernel's dispatch on the stream it runs on (events cannot be timed inside
    # a graph, so these steps issue the same kernels directly)
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        ctx.detect_device(t_img, prm)
    torch.cuda.synchronize()
    dt_eager = time.perf_counter() - t1
    kms, nseq = ctx.kernel_times_all()
    # the same steps with every plane blurred directly (the direct stencil's
    # roofline, beside the tuned configuration's)
    ctx.set_dct(0)
    ctx.set_profiling(True)
    for _ in range(args.steps):
        ctx.detect_device(t_img, prm)
    kms_direct, nseq_direct = ctx.kernel_times_all()
    ctx.set_profiling(False)
    ctx.set_dct(-1 if args.dct < 0 else args.dct)

    # ---- the host entry point on the same frame (host pixels: the upload
    # over PCIe is inside each call); reported beside, never as `value`
    n_host = max(10, args.steps // 10)
    for _ in range(3):
        dog.detect(img, prm.sigma_min, prm.sigma_max, prm.sigma_ratio, prm.threshold, prm.overlap)
    t2 = time.perf_counter()
    for _ in range(n_host):
        dog.detect(img, prm.sigma_min, prm.sigma_max, prm.sigma_ratio, prm.threshold, prm.overlap)
    dt_host = (time.perf_counter() - t2) / n_host

    mpx = H * W * k / 1e6
    value = mpx * args.steps / dt
    names = list(dog.Context.KERNEL_NAMES)
    avg_ms = [m / max(nseq, 1) for m in kms]
    flops = blur_flops(radii, H, W, min_taps, merged=avg_ms[3] == 0.0 and avg_ms[4] == 0.0)
    # the dominant blur launch (a pass, with the transform jobs it runs)
    blur = [n for n in names if n != "nms"]
    dname = max(blur, key=lambda n: avg_ms[names.index(n)])
    dom = names.index(dname)
    traffic = measured_traffic(dname, variant, min_taps)
    # every kernel against both ceilings: algorithmic flops and bytes per launch
    n_g = k + 1
    pitch = (H + 63) // 64 * 64
    plane_b = 4.0 * W * pitch
    n_tr = sum(1 for p in range(n_g) if min_taps > 0 and 2 * radii[p] + 1 >= min_taps)
    algo_bytes = {"pass1": 4.0 * H * W + n_g * plane_b, "pass2": 2.0 * n_g * plane_b,
                  "nms": n_g * plane_b,
                  "fft1": 4.0 * H * W + n_tr * plane_b, "fft2": 2.0 * n_tr * plane_b}
    if flops["merged"]:
        algo_bytes["pass1"] = 4.0 * H * W + n_g * plane_b
        algo_bytes["pass2"] = 2.0 * n_g * plane_b
    else:
        algo_bytes["pass1"] = 4.0 * H * W + (n_g - n_tr) * plane_b
        algo_bytes["pass2"] = 2.0 * (n_g - n_tr) * plane_b
    roofline = roofline_entry(dname, flops[dname], algo_bytes[dname], avg_ms[dom], traffic)
    roofline.update({"kernel_avg_us": {n: round(m * 1e3, 2) for n, m in zip(names, avg_ms)},
                     "transform_min_taps": min_taps})
    roofline["per_kernel"] = {
        n: {"us": round(m * 1e3, 2),
            "tflops": round(flops[n] / (m * 1e-3) / 1e12, 2),
            "frac_fp32_peak": round(flops[n] / (m * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
            "algorithmic_gbs": round(algo_bytes[n] / (m * 1e-3) / 1e9, 1),
            "frac_hbm_peak": round(algo_bytes[n] / (m * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
        for n, m in zip(names, avg_ms) if m > 0}
    avg_direct = [m / max(nseq_direct, 1) for m in kms_direct]
    fl_d = blur_flops(radii, H, W, 0, merged=False)
    d_dom = int(np.argmax(avg_direct[:2]))
    d_bytes = 4.0 * H * W + n_g * plane_b if d_dom == 0 else 2.0 * n_g * plane_b
    roofline_direct = roofline_entry(names[d_dom], fl_d[names[d_dom]], d_bytes,
                                     avg_direct[d_dom], measured_traffic(names[d_dom], variant, 0))
    roofline_direct.update({"kernel_avg_us": {n: round(m * 1e3, 2)
                                              for n, m in zip(names[:3], avg_direct[:3])},
                            "kernel_ms_per_frame": round(sum(avg_direct), 4)})
    kernel_sum_ms = sum(avg_ms)

    out = {"metric": "Mpixel-scales/s for DoG+NMS on 1 GPU; p99 frame latency, batched vs per-frame",
           "value": round(value, 1), "unit": "Mpixel-scales/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(dt / args.steps * 1e3, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "frame1k: one 1024x1024 fp32 camera frame (Poisson counts, "
                                  "500 blobs), sigma 1..30 ratio 1.6 (8 DoG planes), threshold "
                                  "0.05, overlap 0.5", "frames_per_step": 1, "height": H,
                      "width": W, "dog_planes": k, "parallelism": "single GPU",
                      "frames_in_flight": nf},
           "roofline": roofline,
           "roofline_direct_blur": roofline_direct,
           "latency_ms": {"p50": round(pct(lat, 50) * 1e3, 4), "p99": round(pct(lat, 99) * 1e3, 4)},
           "sync_ms_per_step": round(dt_sync / args.steps * 1e3, 4),
           "sync_mpx_scales_per_s": round(mpx * args.steps / dt_sync, 1),
           "kernel_ms_per_frame": round(kernel_sum_ms, 4),
           "eager_ms_per_step": round(dt_eager / args.steps * 1e3, 4),
           "kernel_only_mpx_scales_per_s": round(mpx / (kernel_sum_ms * 1e-3), 1),
           "host_entry_ms_per_frame": round(dt_host * 1e3, 4),
           "host_entry_mpx_scales_per_s": round(mpx / dt_host, 1),
           "blobs": int(len(blobs)),
           "autotune": tune}

    out["prune"] = bench_prune(dog, torch, ctx, t_img, prm)
    if not args.no_paper:
        out["paper_config"] = bench_paper_config(dog, torch, t_img, args.steps, nf)
        out["preprocess"] = bench_preprocess(dog, torch, img, prm, k, args.steps, nf,
                                             variant, min_taps)

    # ---- uniform batch of 64 frames: batched entry point vs frame by frame
    if not args.no_batch:
        frames = batch_frames
        dfr = [torch.from_numpy(f).to(dev) for f in frames]
        torch.cuda.synchronize()
        ctx.detect_batch(dfr, prm)
        for f in dfr[:4]:
            ctx.detect_device(f, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            res, _ = ctx.detect_batch(dfr, prm)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / args.batch_steps
        # the same batch as one launch sequence of all 64 frames
        ctx.set_batch_grouping(0)
        ctx.detect_batch(dfr, prm)
        ctx.detect_batch(dfr, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            ctx.detect_batch(dfr, prm)
        torch.cuda.synchronize()
        tb1 = (time.perf_counter() - t0) / args.batch_steps
        ctx.set_batch_grouping(1 << 20, 3)
        t0 = time.perf_counter()
        per = []
        for f in dfr:
            s0 = time.perf_counter()
            ctx.detect_device(f, prm)
            per.append(time.perf_counter() - s0)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        tot = sum(f.shape[0] * f.shape[1] for f in frames) * k / 1e6
        out["batch64"] = {"batched_mpx_scales_per_s": round(tot / tb, 1),
                          "batched_grouping": "groups of 2^20 px on 3 lanes",
                          "one_sequence_mpx_scales_per_s": round(tot / tb1, 1),
                          "per_frame_mpx_scales_per_s": round(tot / tp, 1),
                          "batched_over_per_frame": round(tp / tb, 3),
                          "batched_ms_per_batch": round(tb * 1e3, 3),
                          "per_frame_p50_ms": round(pct(per, 50) * 1e3, 4),
                          "per_frame_p99_ms": round(pct(per, 99) * 1e3, 4),
                          "batched_frame_latency_ms": round(tb * 1e3, 3)}
        del dfr

    # the autotuner's choices, for the servers' slot contexts
    import tempfile
    tune_cache = os.path.join(tempfile.gettempdir(), "dog_bench_tune_%d.json" % os.getpid())
    ctx.autotune_save(tune_cache)
    if not args.no_mixed:
        out["mixed128"] = bench_mixed(dog, torch, ctx, prm, k, mixed_frames, args.batch_steps,
                                      tune_cache)
    if not args.no_serve:
        out["serving"] = bench_serving(dog, prm, k, mixed_frames, args.serve_rate,
                                       args.serve_seconds, tune_cache=tune_cache)
        # the same stream under a budget of 2.5 footprints of the largest
        # frame of the pool, so admission by HBM footprint binds
        big = max(mixed_frames, key=lambda f: f.size)
        budget = int(2.5 * dog.footprint(prm, [big.shape]))
        out["serving_tight_budget"] = bench_serving(dog, prm, k, mixed_frames, args.serve_rate,
                                                    args.tight_serve_seconds, budget, tune_cache)
    try:
        os.remove(tune_cache)
    except OSError:
        pass

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(img, prm, k)
    for c in ctxs:
        c.close()
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
