"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_2305_10356_amd.profiling counters <counter_collection_trace.csv> [...]
    python -m paper_2305_10356_amd.profiling source-hash

``counters`` prints, per kernel and counter, the mean value per dispatch and
the number of dispatches (rocprofv3 --pmc output converted with rocpd2csv).
``source-hash`` prints the SHA-256 of the kernel source, which a counter
summary records so that a later benchmark can tell whether the counters
still describe the kernels it runs.
"""
from __future__ import annotations

import csv
import hashlib
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "ofm_kernels.hip")


def source_hash(path: str = KERNEL_SOURCE) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def counter_means(paths):
    acc = defaultdict(lambda: [0.0, 0])
    for p in paths:
        with open(p, newline="") as f:
            for row in csv.DictReader(f):
                key = (row["Kernel_Name"], row["Counter_Name"])
                acc[key][0] += float(row["Counter_Value"])
                acc[key][1] += 1
    return {k: (v[0] / v[1], v[1]) for k, v in acc.items()}


def read_traffic(summary_path: str):
    """Per-pass traffic lines ``traffic_bytes <pass> <bytes>`` of a committed
    counter summary, valid only if its ``source_sha256`` matches the current
    kernel source; returns {} otherwise."""
    if not os.path.exists(summary_path):
        return {}
    out = {}
    sha = None
    with open(summary_path) as f:
        for line in f:
            parts = line.strip().strip("`").split()
            if len(parts) == 2 and parts[0] == "source_sha256:":
                sha = parts[1]
            if len(parts) == 3 and parts[0] == "traffic_bytes":
                out[parts[1]] = float(parts[2])
    if sha != source_hash():
        return {}
    return out


def main(argv):
    if len(argv) >= 1 and argv[0] == "source-hash":
        print(source_hash())
        return 0
    if len(argv) >= 2 and argv[0] == "counters":
        res = counter_means(argv[1:])
        for (kern, ctr), (mean, cnt) in sorted(res.items()):
            print(f"{mean:16.2f}  {cnt:5d}  {ctr:14s}  {kern[:110]}")
        return 0
    print(__doc__)
    return 1


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
