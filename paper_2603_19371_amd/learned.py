"""Learned initializer: a U-Net trained on fields the LM method converged to
predicts an initial displacement; LM refines from it and stays the fallback.

    python -m paper_2603_19371_amd.learned train --pairs 2000 --epochs 4 \\
        --out unet.npy
    python -m paper_2603_19371_amd.learned eval --weights unet.npy \\
        --seeds 5000:5200 --out eval.json

Pipeline (full-resolution pair of shape S, network at S/2):
  1. the network sees (F, M) average-pooled by 2 and predicts a field in
     voxels of the S/2 grid;
  2. the field is upsampled x2 (voxel-centre aligned, values doubled) to S;
  3. LM attempts at S start from it (lambda0 and the rules as for the plain
     method) until the loss reaches the target or the attempt budget ends;
  4. the result is kept only if it reached the target and folds no more
     voxels than allowed; otherwise the plain coarse-to-fine LM from the
     identity is run (the fallback).
Training targets are the plain method's converged full-resolution fields,
average-pooled by 2 (the halving of their values is applied in the loss).
Every network step runs in liblmreg's kernels (lmreg_unet.h); torch holds the
device buffers.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import _lib
from . import phantoms_torch

SHAPE = (160, 192, 224)
FACTORS = (4, 2, 1)
ITERS = (200, 100, 50)
WINDOW, SIGMA = 7, 1.0


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights (std sqrt(2 / (27 cin))), zero biases; the last
    layer's weights are scaled by 0.1 so that the first predictions are
    small.  Returned as the flat FP32 vector of lmreg_unet.h."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co, relu, _ in _lib.unet_layers():
        std = math.sqrt(2.0 / (27 * ci)) * (1.0 if relu else 0.1)
        parts.append((rng.standard_normal(27 * ci * co) * std).astype(np.float32))
        parts.append(np.zeros(co, np.float32))
    return np.concatenate(parts)


class LearnedInit:
    """The network at half the resolution of `shape` plus the x2 upsampling."""

    def __init__(self, shape=SHAPE, params=None, seed=0):
        self.shape = tuple(int(s) for s in shape)
        self.net_shape = tuple(s // 2 for s in self.shape)
        self.net = _lib.UNet(self.net_shape)
        p = params if params is not None else init_params(seed)
        self.set_params(p)

    def set_params(self, p):
        t = torch.as_tensor(np.asarray(p, np.float32)).cuda() if not torch.is_tensor(p) \
            else p.to("cuda", torch.float32).contiguous()
        self.net.set_params(t)

    def params(self) -> np.ndarray:
        return self.net.params().cpu().numpy()

    def predict(self, F, M) -> torch.Tensor:
        """Initial field at full resolution [3][S] for full-resolution images."""
        return _lib.upsample_field(self.net.forward(F, M, pool=True))


# ------------------------------------------------------------- training set
def plain_register(pyr, F, M, out=None):
    """The plain coarse-to-fine LM of the reference workload."""
    return pyr.run(F, M, ITERS, lambda0=1.0, out=out)


def make_training_set(seeds, shape=SHAPE, log=print):
    """Pooled images and pooled converged fields for every seed, resident on
    the device: dict(F, M [n][S/2] FP32, T [n][3][S/2] FP32 (not yet halved),
    loss [n], folded [n])."""
    n = len(seeds)
    half = tuple(s // 2 for s in shape)
    Fp = torch.empty((n,) + half, device="cuda")
    Mp = torch.empty((n,) + half, device="cuda")
    T = torch.empty((n, 3) + half, device="cuda")
    loss = np.zeros(n)
    folded = np.zeros(n, np.int64)
    pyr = _lib.Pyramid(shape, FACTORS, window=WINDOW, grad_sigma=SIGMA)
    u = torch.empty((3,) + shape, device="cuda")
    fine = pyr.level(len(FACTORS) - 1)
    t0 = time.time()
    last = t0
    for i, seed in enumerate(seeds):
        F, M, _ = phantoms_torch.brain(shape, seed=seed)
        plain_register(pyr, F, M, out=u)
        Fp[i] = _lib.avgpool(F, 2)
        Mp[i] = _lib.avgpool(M, 2)
        for c in range(3):
            T[i, c] = _lib.avgpool(u[c].contiguous(), 2)
        st = fine.state()
        loss[i] = st["loss"]
        folded[i] = fine.folded_count()
        if time.time() - last > 10 or i == n - 1:
            last = time.time()
            log(f"[data] {i + 1}/{n} pairs, {last - t0:.0f} s, "
                f"mean final loss {loss[:i + 1].mean():.4f}")
    return dict(F=Fp, M=Mp, T=T, loss=loss, folded=folded, seeds=list(seeds))


def train(net: _lib.UNet, data, epochs=4, batch=4, lr=1e-3, seed=0, log=print):
    """Adam on mini-batches (gradients accumulated over `batch` pairs), with a
    cosine decay of the learning rate.  Returns the mean loss per epoch."""
    n = data["F"].shape[0]
    steps = epochs * (n // batch)
    rng = np.random.default_rng(seed)
    lbuf = torch.zeros(n, dtype=torch.float64, device="cuda")
    hist = []
    step = 0
    t0 = time.time()
    last = t0
    for ep in range(epochs):
        order = rng.permutation(n)
        for b0 in range(0, n - batch + 1, batch):
            for j, k in enumerate(order[b0:b0 + batch]):
                net.forward(data["F"][k], data["M"][k])
                net.backward(data["T"][k], target_scale=0.5, accumulate=j > 0,
                             loss=lbuf[k:k + 1])
            lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * step / max(1, steps)))
            net.adam(max(lr_t, lr * 1e-3), grad_scale=1.0 / batch)
            step += 1
            if time.time() - last > 10:
                last = time.time()
                log(f"[train] epoch {ep + 1}/{epochs} step {step}/{steps} "
                    f"{last - t0:.0f} s")
        hist.append(float(lbuf.mean().item()))
        log(f"[train] epoch {ep + 1}: mean MSE {hist[-1]:.5f} (half-res voxels^2)")
    return hist


# ------------------------------------------------------------------ timing
class _Clock:
    """HIP events on torch's current stream (the library's stream here)."""

    def __init__(self):
        self.ev = []

    def mark(self):
        e = torch.cuda.Event(enable_timing=True)
        e.record()
        self.ev.append(e)
        return len(self.ev) - 1

    def ms(self, a, b):
        return self.ev[a].elapsed_time(self.ev[b])


def _first_reaching(losses, target):
    for k, L in enumerate(losses):
        if L <= target:
            return k
    return None


def _start(init, pyr, F, M, schedule):
    """Inference (init None: the identity instead) and every refinement stage
    but the last: returns the field the last (full-resolution) stage begins
    from.  schedule: (factor, attempts) stages, coarse to fine, the last at
    factor 1; a factor-2 stage begins from the network's field itself (it is
    on that grid)."""
    half = tuple(s // 2 for s in F.shape)
    if init is not None:
        u = init.net.forward(F, M, pool=True)
    else:
        u = torch.zeros((3,) + half, device="cuda")
    for f, n in schedule[:-1]:
        if f != 2:
            raise ValueError("refinement stages below full resolution run at factor 2")
        lv = pyr.level(FACTORS.index(2))
        Fp, Mp = _lib.avgpool(F, 2), _lib.avgpool(M, 2)
        lv.begin(Fp, Mp, field=u, lambda0=1.0)
        lv.step(Fp, Mp, n)
        u = lv.field(sync=False)
    return _lib.upsample_field(u)


def _refine(init, pyr, fine, F, M, schedule, target):
    """Tracked then timed run of start + full-resolution attempts until the
    target; returns (losses, first attempt at target or None, folded count,
    start ms, ms to the target or to the last attempt, begin loss)."""
    max_attempts = schedule[-1][1]
    u0 = _start(init, pyr, F, M, schedule)
    fine.begin(F, M, field=u0, lambda0=1.0)
    begin_loss = fine.state()["loss"]
    losses = []
    for _ in range(max_attempts):
        fine.step(F, M, 1)
        losses.append(fine.state()["loss"])
        if losses[-1] <= target:
            break
    k = _first_reaching(losses, target)
    folded = fine.folded_count()
    torch.cuda.synchronize()
    clk = _Clock()
    c0 = clk.mark()
    u0 = _start(init, pyr, F, M, schedule)
    c1 = clk.mark()
    fine.begin(F, M, field=u0, lambda0=1.0)
    marks = []
    for _ in range(len(losses)):
        fine.step(F, M, 1)
        marks.append(clk.mark())
    torch.cuda.synchronize()
    t_end = clk.ms(c0, marks[k if k is not None else -1])
    return losses, k, folded, clk.ms(c0, c1), t_end, begin_loss


def evaluate(init: LearnedInit, seeds, schedule=((1, 50),), tol=1e-3, fold_frac=1e-4,
             ablation=True, train_folded_median=None, log=print):
    """Time to the plain method's final LNCC (within tol): plain coarse-to-fine
    LM from the identity vs prediction + LM refinement (`schedule`, ending
    with at most schedule[-1][1] attempts at full resolution).  With
    `ablation` the same schedule is also run from the identity (the network
    replaced by a zero field), which separates what the network contributes
    from what the schedule does.

    Each run is done twice: once reading the state after every attempt (which
    attempt first reaches the target; untimed), once timed with events after
    every attempt and no host reads; the runs are bitwise identical, so the
    time to the target is the event time at that attempt.  A learned run that
    misses the target, or folds more than the plain run's count + fold_frac N
    voxels, falls back to the plain method and is charged both (the per-seed
    gate).  With train_folded_median the summary also reports the gate a
    deployed pipeline can apply without a plain run of the same pair: the
    folded count is compared with the median count of the plain method over
    the training set (+ fold_frac N) instead."""
    shape = init.shape
    N = int(np.prod(shape))
    schedule = [tuple(st) for st in schedule]
    if schedule[-1][0] != 1:
        raise ValueError("the last refinement stage runs at full resolution")
    pyr = _lib.Pyramid(shape, FACTORS, window=WINDOW, grad_sigma=SIGMA)
    fine = pyr.level(len(FACTORS) - 1)
    coarse_iters = ITERS[:-1] + (0,)
    u = torch.empty((3,) + shape, device="cuda")
    rows = []
    last = time.time()
    for i, seed in enumerate(seeds):
        F, M, _ = phantoms_torch.brain(shape, seed=seed)
        # plain, tracked
        pyr.run(F, M, coarse_iters, lambda0=1.0, out=u)
        plain_losses = []
        for _ in range(ITERS[-1]):
            fine.step(F, M, 1)
            plain_losses.append(fine.state()["loss"])
        plain_final = plain_losses[-1]
        plain_folded = fine.folded_count()
        target = plain_final + tol
        k_plain = _first_reaching(plain_losses, target)
        # plain, timed
        torch.cuda.synchronize()
        clk = _Clock()
        c0 = clk.mark()
        pyr.run(F, M, coarse_iters, lambda0=1.0, out=u)
        marks = []
        for _ in range(ITERS[-1]):
            fine.step(F, M, 1)
            marks.append(clk.mark())
        torch.cuda.synchronize()
        t_plain = clk.ms(c0, marks[k_plain])
        t_plain_full = clk.ms(c0, marks[-1])
        # the network's field alone
        fine.begin(F, M, field=init.predict(F, M), lambda0=1.0)
        net_loss = fine.state()["loss"]
        fine.begin(F, M, lambda0=1.0)
        identity_loss = fine.state()["loss"]
        row = dict(seed=int(seed), plain_final_loss=plain_final,
                   plain_attempt_to_target=k_plain + 1, t_plain_ms=t_plain,
                   t_plain_full_ms=t_plain_full, plain_folded=int(plain_folded),
                   identity_loss=identity_loss, net_loss=net_loss)
        variants = [("learned", init)] + ([("ablation", None)] if ablation else [])
        for tag, net in variants:
            losses, k, folded, t_start, t_end, begin_loss = _refine(
                net, pyr, fine, F, M, schedule, target)
            ok = k is not None and folded <= plain_folded + fold_frac * N
            if train_folded_median is not None:
                ok_t = k is not None and folded <= train_folded_median + fold_frac * N
                row[f"t_{tag}_train_gate_ms"] = t_end if ok_t else t_end + t_plain
                row[f"{tag}_train_gate_fallback"] = not ok_t
            row.update({f"{tag}_begin_loss": begin_loss,
                        f"{tag}_final_loss": losses[-1],
                        f"{tag}_attempts": len(losses),
                        f"{tag}_attempt_to_target": (k + 1) if k is not None else None,
                        f"{tag}_folded": int(folded),
                        f"t_{tag}_start_ms": t_start,
                        f"t_{tag}_ms": t_end if ok else t_end + t_plain,
                        f"{tag}_fallback": not ok})
        rows.append(row)
        if time.time() - last > 10 or i == len(seeds) - 1:
            last = time.time()
            log(f"[eval] {i + 1}/{len(seeds)} seed {seed}: plain {row['t_plain_ms']:.1f} ms, "
                f"learned {row['t_learned_ms']:.1f} ms (full-res attempts "
                f"{row['learned_attempts']}, fallback {row['learned_fallback']})")
    tp = np.array([r["t_plain_ms"] for r in rows])
    summary = dict(seeds=len(rows), tol=tol, schedule=schedule,
                   plain_ms_median=float(np.median(tp)),
                   plain_ms_p90=float(np.percentile(tp, 90)),
                   identity_loss_median=float(np.median([r["identity_loss"] for r in rows])),
                   net_loss_median=float(np.median([r["net_loss"] for r in rows])),
                   plain_final_loss_median=float(np.median([r["plain_final_loss"]
                                                            for r in rows])))
    for tag, _ in [("learned", 0)] + ([("ablation", 0)] if ablation else []):
        tl = np.array([r[f"t_{tag}_ms"] for r in rows])
        summary.update({
            f"{tag}_ms_median": float(np.median(tl)),
            f"{tag}_ms_p90": float(np.percentile(tl, 90)),
            f"{tag}_speedup_median": float(np.median(tp) / np.median(tl)),
            f"{tag}_fallback_rate": float(np.mean([r[f"{tag}_fallback"] for r in rows])),
            f"{tag}_attempts_median": float(np.median([r[f"{tag}_attempts"] for r in rows])),
            f"{tag}_start_ms_median": float(np.median([r[f"t_{tag}_start_ms"]
                                                       for r in rows]))})
        if train_folded_median is not None:
            tt = np.array([r[f"t_{tag}_train_gate_ms"] for r in rows])
            summary.update({
                f"{tag}_train_gate_ms_median": float(np.median(tt)),
                f"{tag}_train_gate_speedup_median": float(np.median(tp) / np.median(tt)),
                f"{tag}_train_gate_fallback_rate": float(np.mean(
                    [r[f"{tag}_train_gate_fallback"] for r in rows]))})
    summary["gate"] = ("per-seed plain run (oracle gate): target = plain final loss + tol; "
                       "folded count <= plain count + fold_frac N")
    if train_folded_median is not None:
        summary["train_gate"] = ("target = plain final loss + tol; folded count <= "
                                 f"training-set median plain count ({train_folded_median:g})"
                                 " + fold_frac N")
    return summary, rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--pairs", type=int, default=2000)
    t.add_argument("--seed0", type=int, default=1000)
    t.add_argument("--epochs", type=int, default=4)
    t.add_argument("--batch", type=int, default=4)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--out", required=True)
    t.add_argument("--shape", default="160,192,224")
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--seeds", default="5000:5200")
    e.add_argument("--schedule", default="1:50",
                   help="refinement stages factor:attempts, coarse to fine, e.g. 2:20,1:40")
    e.add_argument("--out", required=True)
    e.add_argument("--shape", default="160,192,224")
    a = ap.parse_args(argv)
    shape = tuple(int(x) for x in a.shape.split(","))

    def log(msg):
        print(msg, flush=True)

    if a.cmd == "train":
        seeds = list(range(a.seed0, a.seed0 + a.pairs))
        t0 = time.time()
        data = make_training_set(seeds, shape=shape, log=log)
        t1 = time.time()
        init = LearnedInit(shape)
        hist = train(init.net, data, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log)
        t2 = time.time()
        np.save(a.out, init.params())
        meta = dict(shape=shape, pairs=a.pairs, seed0=a.seed0, epochs=a.epochs, batch=a.batch, lr=a.lr,
                    loss_per_epoch=hist, data_s=t1 - t0, train_s=t2 - t1,
                    plain_final_loss_mean=float(data["loss"].mean()),
                    plain_folded_median=float(np.median(data["folded"])))
        with open(os.path.splitext(a.out)[0] + ".json", "w") as fh:
            json.dump(meta, fh, indent=1)
        log(json.dumps(meta))
    else:
        lo, hi = (int(x) for x in a.seeds.split(":"))
        init = LearnedInit(shape, params=np.load(a.weights))
        sched = [tuple(int(v) for v in st.split(":")) for st in a.schedule.split(",")]
        meta_path = os.path.splitext(a.weights)[0] + ".json"
        train_fold = None
        if os.path.exists(meta_path):
            with open(meta_path) as fh:
                train_fold = json.load(fh).get("training", {}).get("plain_folded_median")
        summary, rows = evaluate(init, range(lo, hi), schedule=sched,
                                 train_folded_median=train_fold, log=log)
        with open(a.out, "w") as fh:
            json.dump(dict(summary=summary, rows=rows), fh, indent=1)
        log(json.dumps(summary))


if __name__ == "__main__":
    main()
