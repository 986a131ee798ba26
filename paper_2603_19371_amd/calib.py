"""Reference kernel for calibrating rocprofv3's HBM byte counters.

    python -m paper_2603_19371_amd.calib [--mib 1024]

Launches one plain device copy y = x + 0 of a known size (reads and writes
`mib` MiB each) after a warm-up launch, so that the FETCH_SIZE / WRITE_SIZE
counters of that dispatch can be divided by the bytes it must move: the ratio
scales the counters read for the registration kernels into HBM bytes.
"""
from __future__ import annotations

import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    a = ap.parse_args()
    n = a.mib * (1 << 20) // 4
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    torch.add(x, 0.0, out=y)   # warm-up dispatch
    torch.cuda.synchronize()
    torch.add(x, 0.0, out=y)   # the reference dispatch: reads and writes n*4 bytes
    torch.cuda.synchronize()
    print(f"copy of {n * 4} bytes done", flush=True)


if __name__ == "__main__":
    main()
