#!/usr/bin/env python3
"""Throughput of the factored-LM registration on one MI355X.

One step = one complete coarse-to-fine registration of a brain-MRI-like pair
(160x192x224, FP32 images and field, LNCC window 7, gradient smoothing
sigma 1, lambda0 1, x2 on a bad step / x0.5 on a good one, rejection at
tau = 0, pyramid 4x/2x/1x with 200/100/50 attempts).  The images are resident
in HBM before the timed region.  `value` is voxel-attempts per second over the
timed steps: sum over levels of (voxels of the level x attempts evaluated).

Printed on one JSON line, with
  roofline      the dominant kernel of the full-resolution level: algorithmic
                bytes per launch / its mean duration, measured with HIP events
                the library records on its own stream inside the timed region;
                traffic = HBM bytes per launch from the committed rocprofv3
                counter summary when it was taken on the current kernel source;
  cpu_baseline  the FP64 oracle on the host's cores on a bounded sample of the
                same workload (attempts at the full-resolution level).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
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

# Algorithmic bytes per voxel that each kernel must move given its inputs and
# outputs (each array read or written once; s = bytes per image voxel).
def kernel_bytes(s):
    return {
        "update": 12 + 12 + s + 12 + 4,      # g, u, M gather, u~, warped M
        "lncc_fwd": s + 4 + 16,              # F, warped M -> 4 adjoint maps
        "decide": 0,
        "lncc_bwd": 16 + s + 4 + 12 + s + 12,  # maps, F, Mw, u, M gather -> g
        "smooth": 12 + 12,
    }


# Whole attempt (SURVEY-level algorithmic figure): read F, M, u, write u~,
# persist the smoothed gradient between attempts (write + read).
def attempt_bytes(s):
    return 2 * s + 12 + 12 + 24


def source_sha() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_19371_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, workload: str):
    """HBM bytes per launch from profiles/<kernel>__<workload>.pmc.json, if the
    counters were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}__{workload}.pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_sha") != source_sha():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(ph, attempts=2):
    import numpy as np
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(16, os.cpu_count() or 1)
    oracle.set_threads(threads)
    used = oracle.get_threads()
    p = oracle.Params(window=WINDOW, grad_sigma=SIGMA)
    t0 = time.perf_counter()
    pr = oracle.Pair(ph.F, ph.M, p).begin(lambda0=1.0)
    t1 = time.perf_counter()
    for _ in range(attempts):
        pr.attempt()
    t2 = time.perf_counter()
    n = int(np.prod(SHAPE))
    return {"value": n * attempts / (t2 - t1), "unit": "voxel-attempts/s",
            "cores": used, "kind": "oracle",
            "sample": f"{attempts} LM attempts of the full-resolution level "
                      f"({SHAPE[0]}x{SHAPE[1]}x{SHAPE[2]}) after begin "
                      f"({t1 - t0:.1f} s), FP64 oracle, {used} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(the registration of one pair runs on one device).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2603_19371_amd import _lib, phantoms

    ph = phantoms.brain(SHAPE, seed=0)
    F = torch.from_numpy(ph.F).cuda()
    M = torch.from_numpy(ph.M).cuda()
    pyr = _lib.Pyramid(SHAPE, FACTORS, window=WINDOW, grad_sigma=SIGMA)
    out = torch.empty((3,) + SHAPE, device="cuda")
    for _ in range(a.warmup):
        pyr.run(F, M, ITERS, lambda0=1.0, out=out)
    torch.cuda.synchronize()

    fine = pyr.level(len(FACTORS) - 1)
    fine.profile_start(max_attempts=ITERS[-1] * a.steps, stride=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        pyr.run(F, M, ITERS, lambda0=1.0, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = fine.profile_stop()

    per_level = []
    vox_att = 0
    for l, f in enumerate(FACTORS):
        st = pyr.level(l).state()
        n = int(np.prod([s // f for s in SHAPE]))
        per_level.append({"factor": f, "voxels": n, "attempts": int(st["attempts"]),
                          "accepted_loss": st["loss"], "lambda": st["lambda_"]})
        vox_att += n * int(st["attempts"])
    elapsed = t1 - t0
    value = vox_att * a.steps / elapsed

    s = 4
    nfine = int(np.prod(SHAPE))
    kb = kernel_bytes(s)
    dom = max((k for k in prof if prof[k]["count"]), key=lambda k: prof[k]["total_ms"])
    avg_s = prof[dom]["avg_ms"] * 1e-3
    achieved = kb[dom] * nfine / avg_s / 1e9
    attempt_ms = sum(v["avg_ms"] for v in prof.values() if v["count"])
    workload = "brain160x192x224_f32_w7"
    traffic = traffic_for(dom, workload)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": dom,
                "algorithmic_bytes_per_launch": kb[dom] * nfine,
                "mean_launch_ms": round(prof[dom]["avg_ms"], 5),
                "launches_timed": prof[dom]["count"]}

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(ph)

    line = {
        "metric": "voxel-attempts/s of the LM step (full coarse-to-fine registration)",
        "value": round(value, 1), "unit": "voxel-attempts/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "brain-MRI-like phantom 160x192x224, FP32 images "
                               "and field, LNCC w=7, sigma_g=1, pyramid 4x/2x/1x "
                               "with 200/100/50 attempts, lambda0=1, x2/x0.5, tau=0",
                   "pairs": 1, "voxel_attempts_per_step": vox_att},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {
            "levels": per_level,
            "fine_level_kernel_ms": {k: round(v["avg_ms"], 5) for k, v in prof.items()
                                     if v["count"]},
            "fine_level_attempt_ms": round(attempt_ms, 5),
            "fine_level_voxel_attempts_per_s": round(nfine / (attempt_ms * 1e-3), 1),
            "fine_level_attempt_algorithmic_frac": round(
                attempt_bytes(s) * nfine / (attempt_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "kernel_source_sha": source_sha(),
        },
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
