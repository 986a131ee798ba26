"""Summaries of rocprofv3 output: HBM byte counters of one kernel, and
kernel-trace durations per kernel and grid size.

    python -m paper_2603_19371_amd.pmc_summary trace --trace T.csv \\
        --workload brain160x192x224_f32_w7 --command "..." [--out F.txt] [--top 40]

    python -m paper_2603_19371_amd.pmc_summary counters \\
        --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv \\
        --copy-bytes 1073741824 --kernel k_update --grid 7864320 \\
        --name update --workload brain160x192x224_f32_w7 --command "..." \\
        [--out profiles/update__brain160x192x224_f32_w7.pmc.txt]

    python -m paper_2603_19371_amd.pmc_summary sq --csv C.csv \\
        --workload unet80x96x112 --command "..." --kernels k_conv_tile,k_wgrad \\
        --out profiles/sq__unet80x96x112.txt

Inputs are the counter-collection CSV files of four rocprofv3 --pmc runs: the
workload with FETCH_SIZE, the workload with WRITE_SIZE, and the reference copy
(paper_2603_19371_amd.calib) with each counter.  FETCH_SIZE and WRITE_SIZE
are read in KiB per dispatch; each is scaled by (bytes the copy must move) /
(counter of the copy dispatch), so that the kernel's figure is in HBM bytes.
The dispatches of the kernel are those whose name contains --kernel and
whose grid size (work-items) equals --grid.  The summary records the hash of
the kernel sources it was taken on (bench.py uses it only while it matches).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


# The sources each timed kernel is built from (the counters of a kernel stay
# valid while these files are unchanged).
KERNEL_SOURCES = {
    "update": ["k_step.hip", "update.h", "lmr_internal.h"],
    "lncc_fwd": ["k_stencil.hip", "stencil.h", "lmr_internal.h"],
    "lncc_bwd": ["k_stencil.hip", "stencil.h", "lmr_internal.h"],
    "smooth": ["k_stencil.hip", "stencil.h", "lmr_internal.h"],
    "conv_tile_level0": ["k_unet.hip", "unet_internal.h", "lmr_internal.h"],
    "wgrad_level0": ["k_unet.hip", "unet_internal.h", "lmr_internal.h"],
    "batch_attempt": ["k_batch.hip", "batch_attempt.h", "lmr_batch.h", "stencil.h",
                      "update.h", "decide.h", "lmr_internal.h"],
}


def source_files(kernel: str | None = None):
    csrc = os.path.join(HERE, "csrc")
    if kernel in KERNEL_SOURCES:
        return list(KERNEL_SOURCES[kernel])
    return sorted(n for n in os.listdir(csrc) if n.endswith((".hip", ".h", ".cpp")))


def source_sha(files=None) -> str:
    """Hash of the given library sources (default: all of them)."""
    h = hashlib.sha256()
    csrc = os.path.join(HERE, "csrc")
    for name in files if files is not None else source_files():
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _rows(path):
    with open(path, newline="") as fh:
        yield from csv.DictReader(fh)


def counter_per_dispatch(path, counter, kernel=None, grid=None):
    """Mean of `counter` over the selected dispatches (values summed over
    the counter's instances within a dispatch)."""
    per = {}
    for r in _rows(path):
        if r.get("Counter_Name") != counter:
            continue
        name = r.get("Kernel_Name", "")
        if kernel and kernel not in name:
            continue
        if grid is not None and int(float(r.get("Grid_Size", "0"))) != grid:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"no {counter} rows for kernel {kernel!r} grid {grid} in {path}")
    return statistics.mean(per.values()), len(per)


def copy_scale(path, counter, nbytes):
    """bytes / counter for the largest dispatch of the reference copy."""
    best = 0.0
    per = {}
    for r in _rows(path):
        if r.get("Counter_Name") != counter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    for v in per.values():
        best = max(best, v)
    if best <= 0:
        raise SystemExit(f"no {counter} rows in {path}")
    return nbytes / best, best


def _short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").replace("lmr::", "")
    n = n.replace("void ", "")
    n = n.split("(")[0]
    # library kernels (rocBLAS / composable_kernel) carry very long names
    return n if len(n) <= 72 else n[:64] + "...(" + str(len(n)) + ")"


def trace_summary(a):
    """Per (kernel, grid size): dispatches, mean / min / max duration."""
    per = {}
    for r in _rows(a.trace):
        grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        per.setdefault((_short(r["Kernel_Name"]), grid), []).append(d)
    total = sum(sum(v) for v in per.values())
    lines = [f"# rocprofv3 kernel trace, workload {a.workload}",
             f"# command: {a.command}",
             "# kernel | grid (work-items) | dispatches | mean us | min us | max us | "
             "share of kernel time"]
    rows = sorted(per.items(), key=lambda kv: -sum(kv[1]))
    for (k, grid), v in rows[:a.top]:
        lines.append(f"{k} | {grid} | {len(v)} | {statistics.mean(v):.2f} | {min(v):.2f} | "
                     f"{max(v):.2f} | {100 * sum(v) / total:.1f}%")
    rest = rows[a.top:]
    if rest:
        t_rest = sum(sum(v) for _, v in rest)
        lines.append(f"# {len(rest)} more (kernel, grid) rows: "
                     f"{sum(len(v) for _, v in rest)} dispatches, "
                     f"{100 * t_rest / total:.1f}% of kernel time")
    lines.append(f"# total kernel time {total * 1e-3:.2f} ms")
    out = a.out or os.path.join(ROOT, "profiles", f"kernels__{a.workload}.txt")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def sq_summary(a):
    """Per (kernel, grid): dispatches and the mean per dispatch of each
    counter of one --pmc pass; SQ_ instruction and cycle counters also per
    wave (divided by SQ_WAVES of the same dispatches)."""
    per = {}
    for r in _rows(a.csv):
        name = _short(r.get("Kernel_Name", ""))
        if a.kernels and not any(k in name for k in a.kernels.split(",")):
            continue
        grid = int(float(r.get("Grid_Size", "0")))
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        d = per.setdefault((name, grid), {}).setdefault(key, {})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    lines = [f"# rocprofv3 --pmc counters per dispatch, workload {a.workload}",
             f"# command: {a.command}",
             "# kernel | grid (work-items) | dispatches | counter = mean per dispatch "
             "(per wave)"]
    for (name, grid), disp in sorted(per.items(), key=lambda kv: (kv[0][0], -kv[0][1])):
        names = sorted({c for d in disp.values() for c in d})
        mean = {c: statistics.mean(d.get(c, 0.0) for d in disp.values()) for c in names}
        waves = mean.get("SQ_WAVES")
        cells = []
        for c in names:
            cell = f"{c}={mean[c]:.4g}"
            if waves and c != "SQ_WAVES" and c.startswith(("SQ_INSTS", "SQ_LDS", "SQ_WAIT",
                                                           "SQ_WAVE_CYCLES")):
                cell += f" ({mean[c] / waves:.1f}/wave)"
            cells.append(cell)
        lines.append(f"{name} | {grid} | {len(disp)} | " + "; ".join(cells))
    out = a.out
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    for k in ("trace", "workload", "command"):
        t.add_argument("--" + k, required=True)
    t.add_argument("--out")
    t.add_argument("--top", type=int, default=40, help="rows kept (by total time)")
    c = sub.add_parser("counters")
    for k in ("fetch", "write", "copy-fetch", "copy-write", "kernel", "name", "workload",
              "command"):
        c.add_argument("--" + k, required=True)
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--grid", type=int, required=True)
    c.add_argument("--out")
    q = sub.add_parser("sq")
    for k in ("csv", "workload", "command", "out"):
        q.add_argument("--" + k, required=True)
    q.add_argument("--kernels", default="", help="comma-separated name fragments")
    a = ap.parse_args()
    if a.cmd == "trace":
        trace_summary(a)
        return
    if a.cmd == "sq":
        sq_summary(a)
        return
    f_kib, nf = counter_per_dispatch(a.fetch, "FETCH_SIZE", a.kernel, a.grid)
    w_kib, nw = counter_per_dispatch(a.write, "WRITE_SIZE", a.kernel, a.grid)
    sf, cf = copy_scale(a.copy_fetch, "FETCH_SIZE", a.copy_bytes)
    sw, cw = copy_scale(a.copy_write, "WRITE_SIZE", a.copy_bytes)
    hbm = f_kib * sf + w_kib * sw
    out = a.out or os.path.join(ROOT, "profiles", f"{a.name}__{a.workload}.pmc.txt")
    lines = [
        f"# rocprofv3 HBM counters: kernel {a.kernel} (grid {a.grid} work-items), "
        f"workload {a.workload}",
        f"# command: {a.command}",
        f"# reference: python -m paper_2603_19371_amd.calib (copy of {a.copy_bytes} bytes "
        f"read + written)",
        f"source_files: {' '.join(source_files(a.name))}",
        f"source_sha: {source_sha(source_files(a.name))}",
        f"dispatches_fetch: {nf}",
        f"dispatches_write: {nw}",
        f"fetch_size_per_dispatch: {f_kib:.1f}",
        f"write_size_per_dispatch: {w_kib:.1f}",
        f"copy_fetch_size: {cf:.1f}",
        f"copy_write_size: {cw:.1f}",
        f"fetch_scale: {sf:.6g}",
        f"write_scale: {sw:.6g}",
        f"hbm_read_bytes_per_launch: {f_kib * sf:.0f}",
        f"hbm_write_bytes_per_launch: {w_kib * sw:.0f}",
        f"hbm_bytes_per_launch: {hbm:.0f}",
    ]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
