"""Tune the kernel MVM's launch table for the benchmark workloads on this GPU and write it as JSON.

Usage: python -m paper_1905_10587_amd.tune [--out PATH] [--only NAME ...] [--update]

Each entry times every kernel variant, then the two fastest with their source split (or super-tile edge)
halved and doubled, on a square product of the workload's size class (krr_autotune).  The bench loads
the table from tuned/<arch>.json beside this file when it exists.  --update starts from that table, so that
re-tuning some shapes keeps the entries of the others.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

# (name, precision, d, R, n): the working-precision and FP64 products of each workload's solve
SHAPES = [
    ("small-fp64", "fp64", 3, 1, 2000),
    ("fp32-mixed", "mixed", 8, 1, 100_000),
    ("fp32-fp64", "fp64", 8, 1, 100_000),
    ("mixed-mixed", "mixed", 4, 1, 1_000_000),
    ("mixed-fp64", "fp64", 4, 1, 1_000_000),
    ("adjoint-mixed", "mixed", 16, 1, 200_000),
    ("adjoint-fp64", "fp64", 16, 1, 200_000),
    ("block-mixed", "mixed", 6, 128, 500_000),
    ("block-fp64", "fp64", 6, 128, 500_000),
]


def table_path(arch: str) -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", f"{arch}.json")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--out", default=None)
    ap.add_argument("--only", nargs="*", default=None)
    ap.add_argument("--update", action="store_true", help="start from the committed table of this GPU")
    a = ap.parse_args(argv)
    import torch
    import paper_1905_10587_amd as krr
    krr.load()
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    out = a.out or table_path(arch)
    if a.update and os.path.exists(table_path(arch)):
        krr.autotune_load(table_path(arch))
    for name, prec, d, R, n in SHAPES:
        if a.only and name not in a.only:
            continue
        t0 = time.perf_counter()
        v = krr.autotune(d, R, prec, n=n)
        print(f"tune {name}: {prec} d={d} R={R} n={n}: variant {v} ({time.perf_counter() - t0:.1f} s)",
              file=sys.stderr, flush=True)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    krr.autotune_save(out)
    print(out)


if __name__ == "__main__":
    main()
