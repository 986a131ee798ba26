#!/usr/bin/env python3
"""Throughput of the factored-LM registration on one MI355X.

One step = one complete coarse-to-fine registration of a brain-MRI-like pair
(160x192x224, FP32 images and field, LNCC window 7, gradient smoothing
sigma 1, lambda0 1, x2 on a bad step / x0.5 on a good one, rejection at
tau = 0, pyramid 4x/2x/1x with 200/100/50 attempts).  The images are resident
in HBM before the timed region.  `value` is voxel-attempts per second over the
timed steps: sum over levels of (voxels of the level x attempts evaluated).

Printed on one JSON line, with
  roofline      one LM attempt at full resolution (its five kernels): the
                method's algorithmic bytes (read F, M, u; write u~; write and
                read the persisted smoothed gradient: 56 B per voxel with FP32
                images, 52 with BF16) / the attempt's mean duration, the sum of
                the kernels' mean durations measured with HIP events the
                library records on its own stream inside the timed region,
                around every seventh fine-level attempt (--event-stride; the
                attempts in between run as graph launches, like the coarse
                levels; 7 is prime to the 50 fine attempts of a step, so the
                sample moves by one attempt from step to step and covers
                accepted and rejected attempts in their own proportion rather
                than a fixed subset);
                traffic = HBM bytes per attempt from the committed rocprofv3
                counter summaries when they were taken on the current kernel
                sources; per_kernel gives each kernel's own figure against the
                bytes its design reads and writes;
  cpu_baseline  the FP64 oracle on the host's cores on a bounded sample of the
                same workload (attempts at the full-resolution level, at the
                host's thread count and at one thread; the whole 50-attempt run
                of the 32^3 blob pair), with the CPU model;
  detail        per-level attempts and losses, and the wall time of one attempt
                at each level (the level's pooled pair alone, replayed from a
                HIP graph); for the brain workload also the learned
                initializer's time to the plain method's final LNCC on 16
                held-out seeds, the attempt time at 384^3 with BF16 images, and
                device memory and time per iteration of the LM step and of the
                Adam comparator on N^3 volumes, N = 64..512, and short runs of
                the lung, abdomen, 16-pair and small-pairs workloads below
                (--no-extra skips the per-level times and these).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--workload brain|lung|abdomen|batch|small|unet] [--accum f64|f32c]

The default workload is the brain registration above.  Five more workloads
print a line of the same form:
  lung     384^3 lung-CT-like pair with BF16 images (FP32 field, FP64 loss),
           pyramid 2x/1x with 100/50 attempts;
  abdomen  192x160x192 abdomen-like cross-modal pair (CT-like fixed, MR-like
           moving), FP32, the brain's pyramid and attempts;
  batch    16 brain-like pairs of uneven shapes (4 x 96^3, 4 x 128x160x128,
           4 x 160x192x224, 4 x 192x160x256) advanced together (the tuner
           picks a persistent launch per attempt or one launch per phase, and
           the tiling), replayed from a HIP graph, 150 attempts at full
           resolution, against the same pairs as stand-alone graph replays.
  small    64 brain-like 48^3 pairs, 50 attempts each: the batched form
           against the same pairs as stand-alone contexts (graph replays),
           one after another and on four streams.
  unet     the learned initializer's network at 80x96x112: forward passes/s
           and one training step, with its MFMA roofline (TFLOP/s of the 15
           convolutions against 2.5 PFLOP/s BF16).
--accum selects the LNCC box-sum accumulator: exact FP32 products summed in
FP64 (default) or compensated FP32 pairs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SHAPE = (160, 192, 224)
FACTORS = (4, 2, 1)
ITERS = (200, 100, 50)
WINDOW, SIGMA = 7, 1.0
HBM_PEAK_GBS = 8000.0
# box-sum accumulator of the LNCC passes (lmr_params.accum)
ACCUM = {"f64": 0, "f32c": 1}
ACCUM_TEXT = {"f64": "FP64 box sums", "f32c": "compensated FP32 box sums"}

# Algorithmic bytes per voxel that each kernel must move given its inputs and
# outputs (each array read or written once; s = bytes per image voxel).
def kernel_bytes(s):
    return {
        # g, u, M gather -> u~, warped M and its derivative (read by lncc_bwd)
        "update": 12 + 12 + s + 12 + 4 + 12,
        "lncc_fwd": s + 4 + 16 + 16,         # F, warped M, mu_F and sigma_FF -> 4 maps
        "decide": 0,
        "lncc_bwd": 16 + s + 4 + 12 + 12,    # maps, F, Mw, dMw -> g
        "smooth": 12 + 12,
    }


# Whole attempt (what the method itself must move): read F, M, u, write u~,
# persist the smoothed gradient between attempts (write + read).
def attempt_bytes(s):
    return 2 * s + 12 + 12 + 24


def source_sha() -> str:
    from paper_2603_19371_amd.pmc_summary import source_sha as sha
    return sha()


def traffic_for(kernel: str, workload: str):
    """HBM bytes per launch from profiles/<kernel>__<workload>.pmc.txt (written
    by paper_2603_19371_amd.pmc_summary from rocprofv3 counters), if they were
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}__{workload}.pmc.txt")
    if not os.path.exists(path):
        return None
    d = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                d[k.strip()] = v.strip()
    from paper_2603_19371_amd.pmc_summary import source_sha as sha
    files = d.get("source_files", "").split()
    if not files or d.get("source_sha") != sha(files):
        return None
    return float(d["hbm_bytes_per_launch"])


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(F, M, attempts=2, what="the full-resolution level", single_thread=True):
    """The FP64 oracle on the host: `attempts` attempts on (F, M) at the
    host's thread count (OMP_NUM_THREADS, else min(16, cpu_count)) and one at
    one thread, plus the whole 50-attempt run of the 32^3 blob pair at both
    thread counts."""
    import numpy as np
    import oracle
    from paper_2603_19371_amd import phantoms
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
    oracle.set_threads(threads)
    used = oracle.get_threads()
    p = oracle.Params(window=WINDOW, grad_sigma=SIGMA)
    t0 = time.perf_counter()
    pr = oracle.Pair(F, M, p).begin(lambda0=1.0)
    t1 = time.perf_counter()
    for _ in range(attempts):
        pr.attempt()
    t2 = time.perf_counter()
    n = int(np.prod(F.shape))
    sh = "x".join(str(d) for d in F.shape)
    out = {"value": n * attempts / (t2 - t1), "unit": "voxel-attempts/s",
           "cores": used, "kind": "oracle",
           "sample": f"{attempts} LM attempts of {what} ({sh}) after begin "
                     f"({t1 - t0:.1f} s), FP64 oracle, {used} threads",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count()}
    if single_thread and used > 1:
        oracle.set_threads(1)
        t3 = time.perf_counter()
        pr.attempt()
        t4 = time.perf_counter()
        out["single_thread_value"] = n / (t4 - t3)
    # the 32^3 blob pair of the small configuration, its whole run
    ph = phantoms.blobs((32, 32, 32), seed=0)
    runs = {}
    for th in sorted({1, used}):
        oracle.set_threads(th)
        t5 = time.perf_counter()
        q = oracle.Pair(ph.F, ph.M, oracle.Params(window=5)).begin(lambda0=1.0)
        for _ in range(50):
            q.attempt()
        runs[f"{th}_threads_s"] = round(time.perf_counter() - t5, 3)
    out["blobs32_50_attempts"] = runs
    oracle.set_threads(used)
    return out


def level_attempt_us(F, M, factor, n, img_dtype, a):
    """Mean wall time of one attempt of a pyramid level: the pair average-
    pooled by `factor`, n attempts as one graph replay, minus one attempt."""
    import torch
    import torch.nn.functional as tf
    from paper_2603_19371_amd import _lib

    def pool(x):
        x = x.float()
        if factor > 1:
            x = tf.avg_pool3d(x[None, None], factor)[0, 0]
        return x.to(img_dtype).contiguous()
    Fl, Ml = pool(F), pool(M)
    shape = tuple(Fl.shape)
    pyr = _lib.Pyramid(shape, (1,), img_dtype=img_dtype, window=WINDOW, grad_sigma=SIGMA,
                       accum=ACCUM[a.accum])
    out = torch.empty((3,) + shape, device="cuda")
    ms = {}
    for k in (1, n):
        for _ in range(2):
            pyr.run(Fl, Ml, [k], lambda0=1.0, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 10
        for _ in range(reps):
            pyr.run(Fl, Ml, [k], lambda0=1.0, out=out)
        torch.cuda.synchronize()
        ms[k] = (time.perf_counter() - t0) / reps * 1e3
    return (ms[n] - ms[1]) / (n - 1) * 1e3


def _pyramid_line(a, F, M, img_dtype, factors, iters, workload, s):
    """Times `steps` full coarse-to-fine registrations; roofline from the
    fine level's kernel events."""
    import numpy as np
    import torch
    from paper_2603_19371_amd import _lib

    shape = tuple(F.shape)
    pyr = _lib.Pyramid(shape, factors, img_dtype=img_dtype, window=WINDOW, grad_sigma=SIGMA,
                       accum=ACCUM[a.accum])
    out = torch.empty((3,) + shape, device="cuda")
    for _ in range(a.warmup):
        pyr.run(F, M, iters, lambda0=1.0, out=out)
    torch.cuda.synchronize()
    fine = pyr.level(len(factors) - 1)
    fine.profile_start(max_attempts=iters[-1] * a.steps // a.event_stride + 1,
                       stride=a.event_stride)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        pyr.run(F, M, iters, lambda0=1.0, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = fine.profile_stop()

    per_level = []
    vox_att = 0
    for l, f in enumerate(factors):
        st = pyr.level(l).state()
        n = int(np.prod([d // f for d in shape]))
        per_level.append({"factor": f, "voxels": n, "attempts": int(st["attempts"]),
                          "accepted_loss": st["loss"], "lambda": st["lambda_"]})
        vox_att += n * int(st["attempts"])
    # wall time per attempt at every level, outside the timed region: each
    # level's pooled pair alone as a one-level registration replayed from a
    # HIP graph, (T(n attempts) - T(1 attempt)) / (n - 1), which leaves out
    # the level's begin
    if not a.no_extra:
        for l, f in enumerate(factors):
            per_level[l]["attempt_us"] = round(
                level_attempt_us(F, M, f, iters[l], img_dtype, a), 2)
    elapsed = t1 - t0
    nfine = int(np.prod(shape))
    kb = kernel_bytes(s)
    timed = {k: v for k, v in prof.items() if v["count"]}
    attempt_ms = sum(v["avg_ms"] for v in timed.values())
    # measured HBM bytes per launch (rocprofv3 counters, averaged over accepted
    # and rejected attempts like the durations) while they match the sources
    moved = {k: traffic_for(k, workload) for k in ("update", "lncc_fwd", "lncc_bwd", "smooth")}
    complete = all(v is not None for v in moved.values())
    ab = attempt_bytes(s) * nfine
    achieved = ab / (attempt_ms * 1e-3) / 1e9
    per_kernel = {}
    for k, v in timed.items():
        e = {"design_bytes_per_voxel": kb[k], "mean_ms": round(v["avg_ms"], 5),
             "launches": v["count"]}
        if kb[k]:
            gbs = kb[k] * nfine / (v["avg_ms"] * 1e-3) / 1e9
            e.update({"achieved": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
        if moved.get(k) is not None:
            e["traffic"] = moved[k]
        per_kernel[k] = e
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": sum(moved.values()) if complete else None,
                "kernel": "one full-resolution LM attempt (update, lncc_fwd, decide, "
                          "lncc_bwd, smooth)",
                "algorithmic_bytes_per_voxel": attempt_bytes(s),
                "algorithmic_bytes_per_launch": ab,
                "mean_launch_ms": round(attempt_ms, 5),
                "launches_timed": max(v["count"] for v in timed.values()),
                "events_every": a.event_stride,
                "dominant_kernel": max(timed, key=lambda k: timed[k]["total_ms"]),
                "per_kernel": per_kernel}
    detail = {
        "levels": per_level,
        "fine_level_attempt_ms": round(attempt_ms, 5),
        "fine_level_voxel_attempts_per_s": round(nfine / (attempt_ms * 1e-3), 1),
        "kernel_source_sha": source_sha(),
    }
    if complete:
        b = sum(moved.values())
        t_ms = sum(prof[k]["avg_ms"] for k in moved if prof[k]["count"])
        detail["fine_level_attempt_hbm_bytes_per_voxel"] = round(b / nfine, 1)
        detail["fine_level_attempt_hbm_frac"] = round(b / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return vox_att * a.steps / elapsed, elapsed, vox_att, roofline, detail


def learned_detail(n_seeds=16):
    """Time to the plain method's final LNCC (within 1e-3) on held-out seeds
    5000.. with the committed network: plain coarse-to-fine LM vs prediction
    + LM refinement, both gates (per-seed plain run; training-set median
    folded count)."""
    import numpy as np
    from paper_2603_19371_amd import learned
    base = os.path.join(ROOT, "paper_2603_19371_amd", "weights", "unet_brain160x192x224")
    if not os.path.exists(base + ".npy"):
        return {"skipped": "no committed weights"}
    with open(base + ".json") as fh:
        meta = json.load(fh)
    sched = meta.get("schedule_selection", {}).get("chosen", "1:50")
    schedule = [tuple(int(v) for v in st.split(":")) for st in sched.split(",")]
    init = learned.LearnedInit(SHAPE, params=np.load(base + ".npy"))
    t0 = time.perf_counter()
    summary, _ = learned.evaluate(
        init, range(5000, 5000 + n_seeds), schedule=schedule, ablation=False,
        train_folded_median=meta.get("training", {}).get("plain_folded_median"),
        log=lambda *_: None)
    keys = ("seeds", "plain_ms_median", "plain_ms_p90", "learned_ms_median",
            "learned_ms_p90", "learned_speedup_median", "learned_fallback_rate",
            "learned_attempts_median", "learned_start_ms_median",
            "learned_train_gate_speedup_median", "learned_train_gate_fallback_rate",
            "plain_final_loss_median", "net_loss_median", "identity_loss_median",
            "gate", "train_gate")
    out = {k: (round(summary[k], 4) if isinstance(summary[k], float) else summary[k])
           for k in keys if k in summary}
    out.update({"schedule": sched, "held_out_seeds": f"5000..{5000 + n_seeds - 1}",
                "wall_s": round(time.perf_counter() - t0, 1)})
    return out


def attempt_detail(shape=(384, 384, 384), attempts=20):
    """Mean time of one LM attempt at `shape` with BF16 images (FP32 field,
    FP64 loss) for both box-sum accumulators: a brain-like pair generated on
    the device (the lung generator runs on the host, ~40 s at this size),
    kernel times from HIP events on the context's stream."""
    import torch
    from paper_2603_19371_amd import _lib, phantoms_torch
    F, M, _ = phantoms_torch.brain(shape, seed=0)
    F, M = F.to(torch.bfloat16), M.to(torch.bfloat16)
    n = F.numel()
    out = {"shape": "x".join(map(str, shape)), "images": "bf16"}
    for name, acc in ACCUM.items():
        ctx = _lib.Context(shape, img_dtype=torch.bfloat16, window=WINDOW, grad_sigma=SIGMA,
                           accum=acc)
        ctx.begin(F, M, lambda0=1.0)
        ctx.step(F, M, 5)
        ctx.profile_start(max_attempts=attempts)
        ctx.step(F, M, attempts)
        prof = ctx.profile_stop()
        ms = sum(v["avg_ms"] for v in prof.values() if v["count"])
        out[name] = {"attempt_ms": round(ms, 4),
                     "voxel_attempts_per_s": round(n / (ms * 1e-3), 1),
                     "algorithmic_frac": round(attempt_bytes(2) * n / (ms * 1e-3) / 1e9
                                               / HBM_PEAK_GBS, 4),
                     "kernel_ms": {k: round(v["avg_ms"], 4) for k, v in prof.items()
                                   if v["count"]}}
        ctx.close()
        torch.cuda.synchronize()
    return out


def adam_vs_lm_detail(sides=(64, 128, 192, 256, 320, 384, 448, 512), attempts=10):
    """Device memory and time per iteration of the LM step and of the Adam
    comparator in the same kernels, on N^3 brain-like pairs generated on the
    device (FP32 images, w = 7, sigma 1): the comparison of the paper's
    Sec. 3.5.  Memory = the context's workspace + the two images; the drop
    of free device memory when the context is created is reported beside
    it."""
    import torch
    from paper_2603_19371_amd import _lib, phantoms_torch
    rows = []
    for n in sides:
        shape = (n, n, n)
        F, M, _ = phantoms_torch.brain(shape, seed=0)
        del _
        img = 2 * F.numel() * 4
        row = {"N": n}
        for name, opt in (("lm", 0), ("adam", 1)):
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            ctx = _lib.Context(shape, window=WINDOW, grad_sigma=SIGMA, optimizer=opt)
            torch.cuda.synchronize()
            drop = free0 - torch.cuda.mem_get_info()[0]
            ws = ctx.workspace_bytes()
            ctx.begin(F, M, lambda0=1.0)
            ctx.step(F, M, 3)
            ctx.profile_start(max_attempts=attempts)
            ctx.step(F, M, attempts)
            prof = ctx.profile_stop()
            ms = sum(v["avg_ms"] for v in prof.values() if v["count"])
            row[name] = {"memory_MB": round((ws + img) / 1e6, 1),
                         "workspace_bytes_per_voxel": round(ws / F.numel(), 2),
                         "free_memory_drop_MB": round(drop / 1e6, 1),
                         "iteration_ms": round(ms, 4)}
            ctx.close()
        row["memory_saved_pct"] = round(100.0 * (1 - row["lm"]["memory_MB"] /
                                                 row["adam"]["memory_MB"]), 2)
        row["speedup"] = round(row["adam"]["iteration_ms"] / row["lm"]["iteration_ms"], 3)
        rows.append(row)
        del F, M
        torch.cuda.empty_cache()
    return rows


def run_brain(a):
    import torch
    from paper_2603_19371_amd import phantoms

    ph = phantoms.brain(SHAPE, seed=0)
    F = torch.from_numpy(ph.F).cuda()
    M = torch.from_numpy(ph.M).cuda()
    workload = "brain160x192x224_f32_w7" + ("" if a.accum == "f64" else "_f32c")
    value, elapsed, vox_att, roofline, detail = _pyramid_line(
        a, F, M, torch.float32, FACTORS, ITERS, workload, 4)
    if not a.no_extra:
        progress("learned initializer on held-out seeds")
        detail["learned_init"] = learned_detail()
        progress("384^3 attempt")
        detail["attempt_384_bf16"] = attempt_detail()
        progress("LM vs Adam memory and time")
        detail["adam_vs_lm"] = adam_vs_lm_detail()
        detail["other_workloads"] = other_workloads(a)
    cpu = None if a.no_cpu_baseline else cpu_baseline(ph.F, ph.M)
    config = {"workload": "brain-MRI-like phantom 160x192x224, FP32 images and field, "
                          f"{ACCUM_TEXT[a.accum]}, LNCC w=7, sigma_g=1, pyramid 4x/2x/1x "
                          "with 200/100/50 attempts, lambda0=1, x2/x0.5, tau=0",
              "pairs": 1, "voxel_attempts_per_step": vox_att}
    return "f32", value, elapsed, config, roofline, cpu, detail


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def other_workloads(a):
    """The lung, abdomen, 16-pair and many-small-pairs workloads in short runs
    (1 warm-up and 2 timed steps each, no CPU baseline), so that one default
    run carries their figures too."""
    import argparse as _ap
    out = {}
    for name, fn in (("lung", run_lung), ("abdomen", run_abdomen), ("batch", run_batch),
                     ("small", run_small)):
        progress(f"{name} workload")
        b = _ap.Namespace(**vars(a))
        b.steps, b.warmup, b.no_cpu_baseline, b.no_extra = 2, 1, True, True
        t0 = time.perf_counter()
        dtype, value, elapsed, config, roofline, _, det = fn(b)
        e = {"value": round(value, 1), "ms_per_step": round(elapsed / b.steps * 1e3, 3),
             "dtype": dtype, "workload": config["workload"],
             "attempt_ms": roofline.get("mean_launch_ms"), "frac": roofline.get("frac"),
             "wall_s": round(time.perf_counter() - t0, 1)}
        for k in ("batched_speedup_vs_sequential", "batched_speedup_vs_4_streams",
                  "per_pair_sequential", "per_pair_4_streams"):
            if k in det:
                e[k] = det[k]
        out[name] = e
    return out


def run_lung(a):
    import numpy as np
    import torch
    from paper_2603_19371_amd import phantoms

    shape = (384, 384, 384)
    ph = phantoms.lung(shape, seed=0)
    bits = phantoms.to_bf16_rne(ph.F)
    F = torch.from_numpy(bits.view(np.int16)).cuda().view(torch.bfloat16)
    M = torch.from_numpy(phantoms.to_bf16_rne(ph.M).view(np.int16)).cuda().view(torch.bfloat16)
    workload = "lung384_bf16_w7" + ("" if a.accum == "f64" else "_f32c")
    factors, iters = (2, 1), (100, 50)
    value, elapsed, vox_att, roofline, detail = _pyramid_line(
        a, F, M, torch.bfloat16, factors, iters, workload, 2)
    cpu = None
    if not a.no_cpu_baseline:
        c = tuple(slice(d // 2 - 64, d // 2 + 64) for d in shape)
        Fc = phantoms.bf16_to_f32(bits)[c].copy()
        Mc = phantoms.bf16_to_f32(phantoms.to_bf16_rne(ph.M))[c].copy()
        cpu = cpu_baseline(Fc, Mc, what="a centred 128^3 crop of the BF16 lung pair")
    config = {"workload": "lung-CT-like phantom 384^3, BF16 images, FP32 field, "
                          f"{ACCUM_TEXT[a.accum]}, FP64 loss reduction, LNCC w=7, "
                          "sigma_g=1, pyramid 2x/1x with 100/50 attempts, lambda0=1, "
                          "x2/x0.5, tau=0",
              "pairs": 1, "voxel_attempts_per_step": vox_att}
    return "bf16", value, elapsed, config, roofline, cpu, detail


def run_abdomen(a):
    import torch
    from paper_2603_19371_amd import phantoms

    shape = (192, 160, 192)
    ph = phantoms.abdomen(shape, seed=0)
    F = torch.from_numpy(ph.F).cuda()
    M = torch.from_numpy(ph.M).cuda()
    workload = "abdomen192x160x192_f32_w7" + ("" if a.accum == "f64" else "_f32c")
    value, elapsed, vox_att, roofline, detail = _pyramid_line(
        a, F, M, torch.float32, FACTORS, ITERS, workload, 4)
    cpu = None if a.no_cpu_baseline else cpu_baseline(
        ph.F, ph.M, what="the full-resolution level of the abdomen pair")
    config = {"workload": "abdomen-like cross-modal phantom 192x160x192 (CT-like fixed, "
                          "MR-like moving), FP32 images and field, "
                          f"{ACCUM_TEXT[a.accum]}, LNCC w=7, sigma_g=1, pyramid 4x/2x/1x "
                          "with 200/100/50 attempts, lambda0=1, x2/x0.5, tau=0",
              "pairs": 1, "voxel_attempts_per_step": vox_att}
    return "f32", value, elapsed, config, roofline, cpu, detail


BATCH_SHAPES = [(96, 96, 96)] * 4 + [(128, 160, 128)] * 4 + [(160, 192, 224)] * 4 + \
    [(192, 160, 256)] * 4
BATCH_ITERS = 150


def run_batch(a):
    import numpy as np
    import torch
    from paper_2603_19371_amd import _lib, phantoms_torch

    pairs = [phantoms_torch.brain(sh, seed=100 + i) for i, sh in enumerate(BATCH_SHAPES)]
    Fs = [p[0] for p in pairs]
    Ms = [p[1] for p in pairs]
    b = _lib.Batch(BATCH_SHAPES, window=WINDOW, grad_sigma=SIGMA, accum=ACCUM[a.accum])
    # autotuner cache: per machine, outside the source tree
    import tempfile
    cache = os.environ.get("LMR_TUNE_CACHE",
                           os.path.join(tempfile.gettempdir(), "lmr_batch_tune.txt"))
    tune_ms = b.tune(Fs, Ms, cache_path=cache, iters=3)
    cfg = b.config()
    for _ in range(a.warmup):
        b.begin(Fs, Ms)
        b.step(BATCH_ITERS, graph=True)
        b.sync()
    b.begin(Fs, Ms)
    b.sync()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        b.begin(Fs, Ms)
        b.step(BATCH_ITERS, graph=True)
    b.sync()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    ntot = sum(int(np.prod(sh)) for sh in BATCH_SHAPES)
    attempts = [b.pair(i).state()["attempts"] for i in range(len(BATCH_SHAPES))]
    vox_att = sum(int(np.prod(sh)) * n for sh, n in zip(BATCH_SHAPES, attempts))
    value = vox_att * a.steps / elapsed
    per_attempt_s = elapsed / (a.steps * BATCH_ITERS)
    achieved = attempt_bytes(4) * ntot / per_attempt_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_for("batch_attempt", "batch16_f32_w7"),
                "kernel": "one batched attempt (persistent launch or one launch per "
                          "phase, as tuned)",
                "algorithmic_bytes_per_launch": attempt_bytes(4) * ntot,
                "mean_launch_ms": round(per_attempt_s * 1e3, 5),
                "launches_timed": a.steps * BATCH_ITERS}
    # the same pairs as stand-alone contexts, one after another: a one-level
    # pyramid per pair replays its attempts as one HIP graph
    kw = dict(window=WINDOW, grad_sigma=SIGMA, accum=ACCUM[a.accum])
    pyrs = [_lib.Pyramid(sh, (1,), **kw) for sh in BATCH_SHAPES]
    outs = [torch.empty((3,) + tuple(sh), device="cuda") for sh in BATCH_SHAPES]

    def per_pair_once():
        for i, pyr in enumerate(pyrs):
            pyr.run(Fs[i], Ms[i], [BATCH_ITERS], lambda0=1.0, out=outs[i])
    progress("16 pairs as stand-alone graph replays")
    per_pair_once()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(a.steps):
        per_pair_once()
    torch.cuda.synchronize()
    seq_s = (time.perf_counter() - t2) / a.steps
    seq_att = sum(int(np.prod(sh)) * int(p.level(0).state()["attempts"])
                  for sh, p in zip(BATCH_SHAPES, pyrs))
    del pyrs, outs
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(Fs[0].cpu().numpy(), Ms[0].cpu().numpy(),
                           what="the smallest pair of the batch")
    config = {"workload": "16 brain-like pairs (4x96^3, 4x128x160x128, 4x160x192x224, "
                          "4x192x160x256), FP32, LNCC w=7, sigma_g=1, 150 attempts at "
                          "full resolution, batched form (persistent launch or one "
                          "launch per phase per attempt, and tiling, autotuned), HIP graph",
              "pairs": len(BATCH_SHAPES), "voxel_attempts_per_step": vox_att}
    detail = {"tuned_config": cfg, "tune_ms_per_attempt": tune_ms,
              "per_pair_sequential": {"value": round(seq_att / seq_s, 1),
                                      "ms_per_run": round(seq_s * 1e3, 3),
                                      "attempt_ms": round(seq_s / BATCH_ITERS * 1e3, 4)},
              "batched_speedup_vs_sequential": round(value / (seq_att / seq_s), 3),
              "accepted_losses": [b.pair(i).state()["loss"] for i in range(len(BATCH_SHAPES))],
              "kernel_source_sha": source_sha()}
    return "f32", value, elapsed, config, roofline, cpu, detail


SMALL_SHAPE = (48, 48, 48)
SMALL_PAIRS = 64
SMALL_ITERS = 50


def run_small(a):
    """Many small pairs, where one pair's kernels leave most of the GPU idle:
    64 brain-like 48^3 pairs, 50 LM attempts each at full resolution.  The
    batched form (one persistent launch, or one launch per phase, per attempt
    for all pairs, as tuned; the pairs on 4-plane bricks) against
    the same pairs run as stand-alone contexts (one HIP graph of 50 attempts
    per pair), one after another and spread over four streams."""
    import numpy as np
    import torch
    from paper_2603_19371_amd import _lib, phantoms_torch

    shapes = [SMALL_SHAPE] * SMALL_PAIRS
    pairs = [phantoms_torch.brain(SMALL_SHAPE, seed=300 + i) for i in range(SMALL_PAIRS)]
    Fs = [p[0] for p in pairs]
    Ms = [p[1] for p in pairs]
    nvox = int(np.prod(SMALL_SHAPE))
    kw = dict(window=WINDOW, grad_sigma=SIGMA, accum=ACCUM[a.accum])

    b = _lib.Batch(shapes, **kw)
    import tempfile
    cache = os.environ.get("LMR_TUNE_CACHE",
                           os.path.join(tempfile.gettempdir(), "lmr_batch_tune.txt"))
    # attempts of small pairs take about a millisecond: ten per trial keep
    # the tuner's choice above its timing noise
    b.tune(Fs, Ms, cache_path=cache, iters=10)
    for _ in range(a.warmup):
        b.begin(Fs, Ms)
        b.step(SMALL_ITERS, graph=True)
        b.sync()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        b.begin(Fs, Ms)
        b.step(SMALL_ITERS, graph=True)
    b.sync()
    elapsed = time.perf_counter() - t0
    attempts = [b.pair(i).state()["attempts"] for i in range(SMALL_PAIRS)]
    vox_att = nvox * sum(attempts)
    value = vox_att * a.steps / elapsed

    # the same pairs as stand-alone contexts: a one-level pyramid per pair
    # replays its 50 attempts as one HIP graph
    def per_pair(nstreams):
        streams = [torch.cuda.Stream() for _ in range(nstreams)]
        pyrs = [_lib.Pyramid(SMALL_SHAPE, (1,), stream=streams[i % nstreams], **kw)
                for i in range(SMALL_PAIRS)]
        outs = [torch.empty((3,) + SMALL_SHAPE, device="cuda") for _ in range(SMALL_PAIRS)]
        torch.cuda.synchronize()

        def once():
            for i, pyr in enumerate(pyrs):
                pyr.run(Fs[i], Ms[i], [SMALL_ITERS], lambda0=1.0, out=outs[i])
        for _ in range(max(1, a.warmup)):
            once()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(a.steps):
            once()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        n = nvox * sum(int(pyr.level(0).state()["attempts"]) for pyr in pyrs)
        return n * a.steps / dt, dt / a.steps * 1e3

    seq_v, seq_ms = per_pair(1)
    par_v, par_ms = per_pair(4)
    per_attempt_s = elapsed / (a.steps * SMALL_ITERS)
    achieved = attempt_bytes(4) * nvox * SMALL_PAIRS / per_attempt_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "one batched attempt (persistent launch or one launch per "
                          "phase, as tuned)",
                "algorithmic_bytes_per_launch": attempt_bytes(4) * nvox * SMALL_PAIRS,
                "mean_launch_ms": round(per_attempt_s * 1e3, 5),
                "launches_timed": a.steps * SMALL_ITERS}
    config = {"workload": f"{SMALL_PAIRS} brain-like pairs of 48^3, FP32, LNCC w=7, "
                          f"sigma_g=1, {SMALL_ITERS} attempts at full resolution, batched "
                          "form (persistent launch or one launch per phase per attempt, "
                          "autotuned; 4-plane bricks), HIP graph",
              "pairs": SMALL_PAIRS, "voxel_attempts_per_step": vox_att}
    detail = {"batched_ms_per_run": round(elapsed / a.steps * 1e3, 3),
              "per_pair_sequential": {"value": round(seq_v, 1), "ms_per_run": round(seq_ms, 3)},
              "per_pair_4_streams": {"value": round(par_v, 1), "ms_per_run": round(par_ms, 3)},
              "batched_speedup_vs_sequential": round(value / seq_v, 3),
              "batched_speedup_vs_4_streams": round(value / par_v, 3),
              "tuned_config": b.config(), "kernel_source_sha": source_sha()}
    return "f32", value, elapsed, config, roofline, None, detail


def unet_flops(shape):
    """Multiply-add FLOPs (2 per MAC) of the network's 15 convolutions at
    `shape` (its own resolution): forward, and forward + backward (input
    gradients of layers 1..14 and weight gradients of all)."""
    from paper_2603_19371_amd import _lib
    levels = (0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0)
    fwd = bwd = 0
    for l, (ci, co, _, _) in enumerate(_lib.unet_layers()):
        n = 1
        for d in shape:
            n *= d >> levels[l]
        f = 2 * n * 27 * ci * co
        fwd += f
        bwd += f * (2 if l else 1)
    return fwd, fwd + bwd


def run_unet(a):
    """The learned initializer's network at 80x96x112 (half of the brain
    shape): forward from a full-resolution pair (pooled by 2) and one training
    step (forward, MSE backward, Adam), timed with HIP events."""
    import numpy as np
    import torch
    from paper_2603_19371_amd import _lib, learned, phantoms_torch
    shape = tuple(d // 2 for d in SHAPE)
    F, M, t = phantoms_torch.brain(SHAPE, seed=5000)
    net = _lib.UNet(shape)
    base = os.path.join(ROOT, "paper_2603_19371_amd", "weights", "unet_brain160x192x224.npy")
    params = np.load(base) if os.path.exists(base) else learned.init_params(0)
    net.set_params(torch.from_numpy(params).cuda())
    target = torch.nn.functional.avg_pool3d(t[None], 2)[0].contiguous()

    def fwd():
        net.forward(F, M, pool=True)

    def train():
        net.forward(F, M, pool=True)
        net.backward(target, target_scale=0.5)
        net.adam(1e-4)

    out = {}
    for name, fn in (("forward", fwd), ("training_step", train)):
        for _ in range(max(a.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / a.steps
    net.set_params(torch.from_numpy(params).cuda())   # leave the weights as loaded
    f_fwd, f_train = unet_flops(shape)
    tf = f_fwd / (out["forward"] * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(tf, 2), "peak": 2500.0,
                "unit": "TFLOP/s", "frac": round(tf / 2500.0, 4), "traffic": None,
                "kernel": "U-Net forward (15 BF16 MFMA convolutions with their epilogues, "
                          "pooling, upsampling)",
                "algorithmic_flops_per_launch": f_fwd,
                "mean_launch_ms": round(out["forward"], 4), "launches_timed": a.steps}
    detail = {"forward_ms": round(out["forward"], 4),
              "training_step_ms": round(out["training_step"], 4),
              "forward_gflop": round(f_fwd / 1e9, 2),
              "training_step_gflop": round(f_train / 1e9, 2),
              "training_step_tflops": round(f_train / (out["training_step"] * 1e-3) / 1e12, 2),
              "kernel_source_sha": source_sha()}
    config = {"workload": "learned initializer U-Net (16/32/64/128 channels, 3x3x3, BF16 MFMA, "
                          "FP32 accumulation) at 80x96x112 on a brain-like pair pooled from "
                          "160x192x224", "pairs": 1}
    value = 1e3 / out["forward"]
    return "bf16", value, a.steps * out["forward"] * 1e-3, config, roofline, None, detail


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the per-level attempt times and, for the brain workload, "
                         "the learned-initializer, 384^3 and Adam legs")
    ap.add_argument("--workload",
                    choices=("brain", "lung", "abdomen", "batch", "small", "unet"),
                    default="brain")
    ap.add_argument("--event-stride", type=int, default=7,
                    help="HIP events around the kernels of every n-th fine-level attempt "
                         "(the attempts between two samples run as one graph launch; "
                         "1: every attempt, all enqueued kernel by kernel)")
    ap.add_argument("--accum", choices=tuple(ACCUM), default="f64",
                    help="box-sum accumulator of the LNCC passes")
    a = ap.parse_args()
    if a.event_stride < 1:
        ap.error("--event-stride must be at least 1")
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(one pair's registration runs on one device).", file=sys.stderr)
        sys.exit(2)

    run = {"brain": run_brain, "lung": run_lung, "abdomen": run_abdomen,
           "batch": run_batch, "small": run_small, "unet": run_unet}[a.workload]
    dtype, value, elapsed, config, roofline, cpu, detail = run(a)
    line = {
        "metric": {"batch": "voxel-attempts/s of the LM step (batched pairs)",
                   "small": "voxel-attempts/s of the LM step (batched pairs)",
                   "unet": "U-Net forward passes/s of the learned initializer"}.get(
                       a.workload,
                       "voxel-attempts/s of the LM step (full coarse-to-fine registration)"),
        "value": round(value, 1),
        "unit": "forward passes/s" if a.workload == "unet" else "voxel-attempts/s",
        "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": config,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
