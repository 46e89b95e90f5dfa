"""Summaries of rocprofv3 output for the library's kernels.

    python -m paper_2305_10356_amd.profiling counters <counter_collection_trace.csv> [...]
    python -m paper_2305_10356_amd.profiling source-hash

``counters`` prints, per kernel and counter, the mean value per dispatch and
the number of dispatches (rocprofv3 --pmc output converted with rocpd2csv).
``source-hash`` prints the SHA-256 of the kernel source, which a counter
summary records so that a later benchmark can tell whether the counters
still describe the kernels it runs.

    python -m paper_2305_10356_amd.profiling traffic <fetch.csv> <write.csv> [<l2.csv>]

    python -m paper_2305_10356_amd.profiling mfma <mfma.csv>

``mfma`` reads SQ_INSTS_VALU_MFMA_MOPS_F64/_F32 (units of 512 flops),
SQ_VALU_MFMA_BUSY_CYCLES (summed over SIMDs) and GRBM_GUI_ACTIVE (summed over
the 8 XCDs) per dispatch and prints, per kernel, the matrix-core flops per
launch, their rate over the dispatch time and the matrix-core busy fraction
busy / (GUI_ACTIVE / 8 x 1024 SIMDs).

``traffic`` scales FETCH_SIZE and WRITE_SIZE (KiB per dispatch) by what the
same counters read for the 256 MiB device copy of ``bench.py
--copy-calibration`` and prints bytes per launch for the passes of one f1 step
(lines ``traffic_bytes <pass> <bytes>``), with the L2 hit rate when a
TCC_HIT/TCC_MISS file is given.
"""
from __future__ import annotations

import csv
import hashlib
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
# the kernels and the graph layout they read (the counters depend on both)
KERNEL_SOURCES = (os.path.join(HERE, "csrc", "ofm_kernels.hip"),
                  os.path.join(HERE, "csrc", "ofm_graph.hip"))


def source_hash(paths=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


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
    kernel and graph-layout sources (``source_hash``); returns {} otherwise."""
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


# kernel instantiation (name prefix) -> pass, for the FP32 k = 32 kernels of
# an f1 step; the last template argument of the SpMM is the gather policy
F1_PASSES = {
    "spmm_kernel<float, 32, 1, false, false, ": "spmm_x",
    "spmm_kernel<float, 32, 3, false, false, ": "spmm_v",
    "dense_kernel<float, 32, 6>": "v",
    "dense_kernel<float, 32, 7>": "update",
}
COPY_BYTES = 256 * 1024 * 1024


def _per_dispatch(path, counter):
    out = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] == counter:
                out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def traffic(fetch_csv, write_csv, l2_csv=None, passes=F1_PASSES):
    fe = _per_dispatch(fetch_csv, "FETCH_SIZE")
    wr = _per_dispatch(write_csv, "WRITE_SIZE")
    copy = [k for k in fe if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no calibration copy in the counter file (run with --copy-calibration)")
    # the calibration launches are the copies of COPY_BYTES (the largest ones)
    big_f = max(fe[copy[0]])
    big_w = max(wr[copy[0]])
    sf = COPY_BYTES / (big_f * 1024.0)
    sw = COPY_BYTES / (big_w * 1024.0)
    hits = _per_dispatch(l2_csv, "TCC_HIT_sum") if l2_csv else {}
    miss = _per_dispatch(l2_csv, "TCC_MISS_sum") if l2_csv else {}
    rows = []
    for kern in sorted(fe):
        name = next((p for key, p in passes.items() if key in kern), None)
        if name is None:
            continue
        f = sum(fe[kern]) / len(fe[kern])
        w = sum(wr.get(kern, [0.0])) / max(len(wr.get(kern, [])), 1)
        hr = None
        if kern in hits and kern in miss:
            h, m = sum(hits[kern]), sum(miss[kern])
            hr = h / (h + m) if h + m > 0 else None
        rows.append((name, kern, f, w, 1024.0 * (f * sf + w * sw), hr))
    return sf, sw, rows


def mfma(path):
    rows = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            key = (row["Kernel_Name"], row["Dispatch_Id"])
            d = rows.setdefault(key, {"ns": int(row["End_Timestamp"]) - int(row["Start_Timestamp"])})
            d[row["Counter_Name"]] = float(row["Counter_Value"])
    per = defaultdict(list)
    for (kern, _), d in rows.items():
        per[kern].append(d)
    out = []
    for kern, ds in sorted(per.items()):
        n = len(ds)
        f64 = sum(d.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) for d in ds) * 512 / n
        f32 = sum(d.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0) for d in ds) * 512 / n
        ns = sum(d["ns"] for d in ds) / n
        busy = sum(d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for d in ds) / n
        gui = sum(d.get("GRBM_GUI_ACTIVE", 0.0) for d in ds) / n
        util = busy / (gui / 8.0 * 1024.0) if gui > 0 else 0.0
        out.append((kern, n, ns, f64, f32, util))
    return out


def main(argv):
    if len(argv) >= 1 and argv[0] == "source-hash":
        print(source_hash())
        return 0
    if len(argv) >= 3 and argv[0] == "traffic":
        sf, sw, rows = traffic(argv[1], argv[2], argv[3] if len(argv) > 3 else None)
        print(f"scale: FETCH x{sf:.3f}, WRITE x{sw:.3f}")
        print("| pass | kernel | FETCH_SIZE KiB/launch | WRITE_SIZE KiB/launch "
              "| scaled bytes/launch | L2 hit rate |")
        print("|:--|:--|--:|--:|--:|--:|")
        for name, kern, f, w, b, hr in rows:
            k = kern.replace("void ofm::", "").replace("(ofm::PassArgs)", "")
            h = f"{100 * hr:.1f}%" if hr is not None else "-"
            print(f"| {name} | {k} | {f:.2f} | {w:.2f} | {b:.4g} | {h} |")
        print()
        for name, _, _, _, b, _ in rows:
            print(f"    traffic_bytes {name} {int(round(b))}")
        return 0
    if len(argv) >= 2 and argv[0] == "mfma":
        print("| kernel | launches | us/launch | F64 MFMA GFLOP | F32 MFMA GFLOP | TFLOP/s | busy |")
        print("|:--|--:|--:|--:|--:|--:|--:|")
        for kern, n, ns, f64, f32, util in mfma(argv[1]):
            if f64 + f32 == 0:
                continue
            k = kern.replace("void ofm::", "").replace("(ofm::PassArgs)", "")
            print(f"| {k} | {n} | {ns / 1e3:.1f} | {f64 / 1e9:.2f} | {f32 / 1e9:.2f} | "
                  f"{(f64 + f32) / ns / 1e3:.1f} | {100 * util:.1f}% |")
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
