#!/usr/bin/env python3
"""Benchmark of the orthogonalization-free iteration on one MI355X.

Workload: degree-corrected SBM with N = 2,000,000 nodes, k = 32 blocks,
mean degree 25, power-law (exponent 2.5) degree propensity inside blocks,
inter/intra edge ratio 0.5 (seeded, synthetic), X0 ~ N(0, 1/N).  A step is
one X update of Algorithm 2 (two SpMMs, the direction, CG, exact line
search, update; the residual every 10 steps) in FP32 with FP64 k x k
products.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "OFM iters/s + SpMM HBM GB/s (N=2M,k=32); batched vs plain time to residual 1e-4"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pass_bytes(name: str, n: int, nnz: int, k: int, esz: int, variant: str, ntiles: int,
               recur: bool = False, layout: bool = False, upper=None) -> float:
    """HBM bytes of one launch of a pass, each array moved once.  The graph
    part of an SpMM is counted as the method needs it (layout=False): the
    pattern-only CSR of an unweighted graph, 4 B per entry, row_ptr (4 B per
    row) and D^{-1/2} (one value per row in the working precision); with
    layout=True as this library stores it: packed (column, normalized weight)
    entries (8 B in FP32, 16 B in FP64), 8 B of offsets and row ids per row
    and the tile table.
    Without the recurrence the SpMM of X forms the direction in its epilogue
    (f2 with X^T A X advanced by the line search); with it, the SpMM of X runs
    on residual steps only and stores A X, the SpMM of V stores A V, the
    update also reads A X, A V and writes A X, and G is formed in a pass of
    its own from the stored A X.
    f2 at k >= 32 without the recurrence stores A V and forms X^T A V, V^T A V
    in a streaming pass ("other").
    upper = (rows, entries) of the Laplacian's upper-triangle copy, from which
    the variants without the recurrence take their products with A V (f1:
    diag(V^T A V); f2 at k <= 32: V^T A V, with X^T A V = (AX)^T V formed in
    the V pass, which then also reads the A X that the SpMM of X writes): the
    SpMM of V then reads the entries above the diagonal (pattern-only: 4 B
    each, n + 1 row offsets and D^{-1/2}; layout: packed entries, offsets and
    row ids of the copy's rows) and V."""
    B = n * k * esz
    f2 = variant in ("f2", "tri-f2")
    use_upper = (upper is not None and upper[1] > 0 and not recur and (not f2 or k <= 32))
    f2u = use_upper and f2
    if name == "spmm_v" and use_upper:
        nu, nnzu = upper
        if layout:
            return nnzu * (8 if esz == 4 else 16) + 8 * nu + 4 * ((nu + 15) // 16 + 1) + B
        return 4 * nnzu + 4 * (n + 1) + esz * n + B
    if f2u and name == "v":
        return 5 * B                             # G, V_prev, X, A X read; V write
    if f2u and name == "spmm_x":
        graph = (nnz * (8 if esz == 4 else 16) + 8 * n + 4 * (ntiles + 1) if layout
                 else 4 * nnz + 4 * (n + 1) + esz * n)
        return graph + 4 * B                     # X, G_prev read; G, A X write
    if layout:
        graph = nnz * (8 if esz == 4 else 16) + 8 * n + 4 * (ntiles + 1)
    else:
        graph = 4 * nnz + 4 * (n + 1) + esz * n
    split = f2 and not recur and k >= 32 and not f2u
    if name == "spmm_x":
        # X; without the recurrence G_prev read + G write, with it A X write
        return graph + (2 * B if recur else 3 * B)
    if name == "spmm_v":
        if split:
            return graph + 2 * B                 # V read, A V write
        # V; f2 also reads X; the recurrence writes A V
        return graph + (2 * B if f2 else B) + (B if recur else 0)
    if name == "other":
        return 3 * B if split else 0.0           # X, V, A V read
    if name == "g":
        return 4 * B                             # X, AX, G_prev read; G write
    if name == "v":
        return 4 * B                             # G, V_prev, X read; V write
    if name == "update":
        return 6 * B if recur else 3 * B         # X, V (, AX, AV) read; X (, AX) write
    return 0.0


def cpu_baseline(g, x0, k: int, variant_id: int, gpu_iters_to_tol=None, loop_iters: int = 3):
    """The FP64 oracle on the same graph and X0 (FP32-rounded) on this host:
    the Laplacian and the set-up step of Algorithm 2 (untimed), then
    ``loop_iters`` timed loop iterations; s/iteration times the device's
    iteration count to residual 1e-4 gives an extrapolated time to 1e-4."""
    import numpy as np
    from oracle import ofm_oracle as O
    try:
        import threadpoolctl
        threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    lap = O.laplacian(g.n, g.row_ptr, g.col_idx)
    x = x0.astype(np.float32).astype(np.float64)
    # the triangular variants run with the descent restart, as on the device
    opts = O.Options(variant=variant_id, restart=O.is_tri(variant_id))
    st, _ = O.init(lap, x, opts)
    t1 = time.perf_counter()
    first = None
    for i in range(loop_iters):
        st, _ = O.step(lap, st, opts)
        if i == 0:
            first = st.X
    t2 = time.perf_counter()
    cpu_baseline.first_step_x = first
    s_per_it = (t2 - t1) / loop_iters
    out = {"value": round(loop_iters / (t2 - t1), 4), "unit": "iters/s", "cores": int(threads),
           "kind": "oracle",
           "sample": (f"{loop_iters} loop iterations of Algorithm 2 (two products with A each) on "
                      f"the same graph and X0, FP64 NumPy/SciPy, {t2 - t1:.1f} s; the Laplacian "
                      f"and the set-up step ({t1 - t0:.1f} s) untimed; SciPy's CSR x dense "
                      f"product runs on 1 thread, the dense products on {threads} BLAS threads")}
    if gpu_iters_to_tol:
        out["extrapolated_time_to_1e-4_s"] = round(gpu_iters_to_tol * s_per_it, 1)
        out["extrapolated_from"] = (f"{gpu_iters_to_tol} updates (the device's count to residual "
                                    f"1e-4) x {s_per_it:.2f} s per oracle iteration: extrapolated")
    return out


def read_clocks():
    """GPU clocks as rocm-smi reports them (clocks are not pinned here)."""
    import subprocess
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True,
                           timeout=20)
        d = json.loads(r.stdout)
        card = d[sorted(d)[0]]
        return {k: v for k, v in card.items() if "clock" in k.lower()}
    except Exception:
        return None


def batched_vs_plain(variant: str, count: int = 256, plain: bool = True):
    """256 independent SBM graphs (N ~ U{1000..50000}, k ~ U{4,8,16,32}, mean
    degree ~ U[8,32], r = 0.3): wall time until every graph reaches residual
    1e-4 (checked every 10 iterations), batched FP32 (eager lockstep loop, and
    the loop replayed as HIP graphs) vs a loop of per-graph FP64 solves on the
    same GPU.  Graph set-up and allocation are outside every timed region."""
    import numpy as np
    import torch
    from paper_2305_10356_amd import graphs, ofm
    t = time.perf_counter()
    specs = graphs.batched_graph_specs(count)
    gl = [graphs.batched_graph(sp) for sp in specs]
    log(f"batched workload generated in {time.perf_counter() - t:.1f} s")
    laps = [ofm.Laplacian(g.row_ptr, g.col_idx) for g, _ in gl]
    ks = [sp["k"] for sp in specs]
    tri = variant.startswith("tri")

    def batched(graph=False, recur=False, persistent=False):
        B = ofm.Batch(laps, ks, variant=variant, precision=ofm.OFM_FP32, max_iter=3000,
                      check_every=10, tol=1e-4, restart=tri, recur=recur, graph=graph)
        if persistent:
            B.set_persistent(True)
        Xs = [torch.tensor(x0.astype(np.float32), device="cuda") for _, x0 in gl]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = B.solve(Xs)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        sched, esc = B.schedule()
        loop_ms, finish_ms = B.phases()
        rec = {"s": round(dt, 4), "converged": int(sum(s["converged"] for s in st)),
               "max_iters": int(max(s["iters"] for s in st)), "escalated_to_fp64": esc,
               "schedule": {f"k{d['k']}": f"tpw {d['tpw']}, {d['workers']} blocks/XCD"
                            for d in sched},
               "schedule_candidates_ms": {f"k{d['k']}": [round(x, 3) for x in d["ms"]]
                                          for d in sched},
               "phase_ms": {"fp32_loop": round(loop_ms, 1), "fp64_finish": round(finish_ms, 1)},
               "graph_replays": B.replays}
        if persistent:
            rec["persistent_launches"], rec["persistent_min_workers"] = B.persist_info()
        B.close()
        return rec, st

    eager, st_b = batched()
    replayed, _ = batched(graph=True)
    recur, _ = batched(recur=True)
    # one persistent launch per width group and chunk of 10 updates (f1 forms)
    persistent = batched(persistent=True)[0] if variant in ("f1", "tri-f1") else None
    st_p, t_plain = [{"converged": 0, "iters": 0}], float("nan")
    if plain:
        wss = [ofm.Workspace(lap, k, variant=variant, precision=ofm.OFM_FP64, max_iter=3000,
                             check_every=10, tol=1e-4, restart=tri) for lap, k in zip(laps, ks)]
        X64 = [torch.tensor(x0, dtype=torch.float64, device="cuda") for _, x0 in gl]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st_p = [ws.solve(X) for ws, X in zip(wss, X64)]
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        for ws in wss:
            ws.close()
    best = min(eager["s"], replayed["s"])
    return {
        "graphs": count, "sum_n": int(sum(g.n for g, _ in gl)),
        "sum_nnz": int(sum(g.nnz for g, _ in gl)),
        "batched_fp32_s": best,
        "batched_form": "graph-replayed" if replayed["s"] <= eager["s"] else "eager",
        "plain_fp64_loop_s": round(t_plain, 4),
        "speedup": round(t_plain / best, 2),
        "plain_converged": int(sum(s["converged"] for s in st_p)),
        "plain_max_iters": int(max(s["iters"] for s in st_p)),
        "eager": eager, "graph_replayed": replayed, "recur_ax": recur,
        "persistent": persistent,
        "persistent_s": persistent["s"] if persistent else None,
        "speedup_recur": round(t_plain / recur["s"], 2),
        "batched_not_converged": [
            {"graph": i, "n": gl[i][0].n, "k": ks[i], "relres": st_b[i]["relres"]}
            for i in range(count) if not st_b[i]["converged"]],
    }


def spmm_locality_ladder(g, k: int = 32, windows=(32768, 262144, None), reps: int = 20):
    """The SpMM kernel (Y = A Z, FP32) on graphs with the rows and degrees of
    the headline graph but every column folded into the first W node ids
    (col mod W, duplicates in a row merged): the gathered rows then come from
    a W x k window of Z (W = 32768: 4 MB, the L2 of one XCD; 262144: 32 MB;
    None: all of Z, 256 MB).  Same kernel, same entry count, different reuse."""
    import numpy as np
    import torch
    from paper_2305_10356_amd import ofm
    n = g.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr))
    Z = torch.randn(n, k, device="cuda")
    Y = torch.empty_like(Z)
    out = []
    for w in windows:
        if w is None:
            rp, ci = g.row_ptr, g.col_idx
        else:
            key = np.unique(rows * w + (g.col_idx.astype(np.int64) % w))
            r = key // w
            ci = (key % w).astype(np.int32)
            rp = np.zeros(n + 1, dtype=np.int64)
            np.cumsum(np.bincount(r, minlength=n), out=rp[1:])
            rp = rp.astype(np.int32)
        lap = ofm.Laplacian(rp, ci)
        for _ in range(3):
            lap.apply(Z, Y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            lap.apply(Z, Y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        nnz = int(ci.shape[0])
        out.append({"window_rows": w if w is not None else n,
                    "window_MB": round((w if w is not None else n) * k * 4 / 2**20, 1),
                    "nnz": nnz, "avg_us": round(1e3 * ms, 1),
                    "gathered_GBs": round(nnz * k * 4 / (ms * 1e-3) / 1e9, 1)})
        lap.close()
    return out


def orderings_study(g, x0, k: int, variant: str, names, steps: int = 30, gather=None):
    """The step on the headline graph stored in other node orders (graph-only
    preprocessing, no clustering): as generated (random ids), hub-first (ids by
    degree, descending) and reverse Cuthill-McKee; FP32 and the BF16 gathered
    copy.  Event-timed products with A and iterations/s per order."""
    import numpy as np
    import torch
    from paper_2305_10356_amd import graphs, ofm
    out = {}
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    for name in names:
        t0 = time.perf_counter()
        order = {"random": None, "hub-first": graphs.hub_first_order,
                 "rcm": graphs.rcm_order}[name]
        order = None if order is None else order(g)
        t_order = time.perf_counter() - t0
        gg = g if order is None else graphs.relabel(g, order)
        xx = x0 if order is None else x0[order]
        # locality of the order: share of entries within 32768 ids (a 4 MB
        # window of X rows) of their row
        if order is None:
            span = np.abs(rows - g.col_idx)
        else:
            inv = np.empty(g.n, dtype=np.int64)
            inv[order] = np.arange(g.n)
            span = np.abs(inv[rows] - inv[g.col_idx])
        near = float(np.mean(span < 32768))
        lap = ofm.Laplacian(gg.row_ptr, gg.col_idx)
        rec = {"order_s": round(t_order, 2), "entries_within_4MB_window": round(near, 4)}
        for pname, prec in (("fp32", ofm.OFM_FP32), ("bf16x", ofm.OFM_FP32_BF16X)):
            ws = ofm.Workspace(lap, k, variant=variant, precision=prec, check_every=10,
                               restart=variant.startswith("tri"),
                               gather=ofm.GATHER_DEFAULT if prec != ofm.OFM_FP32 else
                               (ofm.GATHER_AUTO if gather is None else gather))
            X = torch.as_tensor(xx, dtype=torch.float32, device="cuda").contiguous()
            ws.init(X)
            for _ in range(5):
                ws.step(X)
            ws.set_timing(["spmm_x", "spmm_v"])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(steps):
                ws.step(X)
            torch.cuda.synchronize()
            rate = steps / (time.perf_counter() - t1)
            ws.set_timing(False)
            tm = ws.timing(reset=True)
            rec[pname] = {"iters_per_s": round(rate, 1),
                          "spmm_x_us": round(1e3 * tm["spmm_x"][0] / max(tm["spmm_x"][1], 1), 1),
                          "spmm_v_us": round(1e3 * tm["spmm_v"][0] / max(tm["spmm_v"][1], 1), 1),
                          "gather": {1: "default", 2: "hot/cold"}[ws.stats()["gather"]]}
            ws.close()
            del X
        lap.close()
        out[name] = rec
        log(f"ordering {name}: {rec}")
    return out


def gather_ceiling(nrows: int = 2_000_000, S: int = 25, reps: int = 5):
    """How fast the chip serves random rows: nrows output rows each summing S
    rows of a table chosen uniformly at random (50M gathers, the entry count
    of the headline graph), for tables of 4 MB-class, 32 MB-class and 2M rows
    and rows of 64, 128 and 256 bytes (ofm_gather_rows: the gathers of the
    products with A without the sparse-matrix work)."""
    import torch
    from paper_2305_10356_amd import ofm
    out = []
    gen = torch.Generator(device="cuda")
    for rows in (32768, 262144, 2_000_000):
        gen.manual_seed(rows)
        idx = torch.randint(0, rows, (nrows * S,), generator=gen, device="cuda",
                            dtype=torch.int32)
        for rf in (16, 32, 64):
            Z = torch.zeros((rows, rf), dtype=torch.float32, device="cuda")
            Y = torch.empty((nrows, rf), dtype=torch.float32, device="cuda")
            for _ in range(2):
                ofm.gather_rows(idx, Z, S, Y)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                ofm.gather_rows(idx, Z, S, Y)
            e1.record()
            e1.synchronize()
            us = 1e3 * e0.elapsed_time(e1) / reps
            out.append({"table_rows": rows, "table_MB": round(rows * rf * 4 / 2**20, 1),
                        "row_bytes": rf * 4, "gathers": nrows * S, "avg_us": round(us, 1),
                        "G_rows_per_s": round(nrows * S / us / 1e3, 1),
                        "G_lines_per_s": round(nrows * S * max(1, rf * 4 // 128) / us / 1e3, 1)})
            log(f"gather ceiling {out[-1]}")
            del Z, Y
        del idx
    return out


def gather_ceiling_for(n: int, nnz: int, k: int, kernel_us: float, reps: int = 5):
    """The random-row rate that bounds a product with A of this size: n output
    rows each summing S = nnz / n rows (k FP32 values) drawn uniformly from an
    n-row table, timed with HIP events (ofm_gather_rows); `kernel_frac` is this
    time over the kernel's own (1.0 = the kernel gathers as fast as the memory
    system serves random rows)."""
    import torch
    from paper_2305_10356_amd import ofm
    S = max(1, round(nnz / n))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(n)
    idx = torch.randint(0, n, (n * S,), generator=gen, device="cuda", dtype=torch.int32)
    Z = torch.zeros((n, k), dtype=torch.float32, device="cuda")
    Y = torch.empty((n, k), dtype=torch.float32, device="cuda")
    for _ in range(2):
        ofm.gather_rows(idx, Z, S, Y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ofm.gather_rows(idx, Z, S, Y)
    e1.record()
    e1.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    del idx, Z, Y
    return {"gathers": n * S, "row_bytes": 4 * k, "table_rows": n, "avg_us": round(us, 1),
            "G_rows_per_s": round(n * S / us / 1e3, 1), "kernel_frac": round(us / kernel_us, 3)}


def streaming_c4(variant: str = "f1", n_final: int = 2_000_000, stages: int = 10,
                 cold_stages=(9,), recur: bool = False, check_every: int = 10,
                 grouped: bool = False, gs=None):
    """Growth stream of 10 snapshots, N = 200k .. 2M, k = 64, mean degree 20,
    r = 0.3: each stage solved to residual 1e-4 (checked every 10 iterations)
    in FP32 from the previous stage's solution (new rows N(0, 1/N_s)), with
    the loop replayed as HIP graphs.  The stages in ``cold_stages`` are also
    solved from a fresh random block for comparison.  ``grouped``: each stage's
    Laplacian is built with its rows laid out for the XCDs by the clusters of
    the previous stage (k-means on its features, timed apart as labels_s)."""
    import torch
    from paper_2305_10356_amd import graphs, ofm
    from paper_2305_10356_amd.streaming import StreamingSolver
    if gs is None:
        t = time.perf_counter()
        gs = graphs.GrowthStream(n_final=n_final, stages=stages, k=64, dbar=20, r=0.3, seed=4)
        log(f"growth stream generated in {time.perf_counter() - t:.1f} s")
    tri = variant.startswith("tri")
    warm = StreamingSolver(64, variant=variant, precision=ofm.OFM_FP32, tol=1e-4,
                           check_every=check_every, max_iter=5000, graph=True, restart=tri,
                           recur=recur, seed=4, grouped=grouped)
    stages_out = []
    for s in range(stages):
        g = gs.snapshot(s)
        rec = warm.solve_stage(g.row_ptr, g.col_idx, warm=True)
        if s in cold_stages:
            cold = StreamingSolver(64, variant=variant, precision=ofm.OFM_FP32, tol=1e-4,
                                   check_every=check_every, max_iter=5000, graph=True,
                                   restart=tri, recur=recur, seed=4)
            cold.stage = s
            rc = cold.solve_stage(g.row_ptr, g.col_idx, warm=False)
            rec["cold_iters"] = rc["iters"]
            rec["cold_solve_s"] = round(rc["solve_s"], 4)
            rec["cold_converged"] = rc["converged"]
            del cold
        for key in ("solve_s", "laplacian_s", "xinit_s", "labels_s"):
            if key in rec:
                rec[key] = round(rec[key], 4)
        log(f"stream stage {s}: {rec}")
        stages_out.append(rec)
    torch.cuda.synchronize()
    return {
        "workload": f"growth stream {stages} snapshots N={gs.bounds[0]}..{n_final} k=64 "
                    f"mean-degree 20 r=0.3, FP32, graph-replayed loop, tol 1e-4",
        "variant": variant,
        "recur_ax": recur,
        "grouped_order": grouped,
        "check_every": check_every,
        "total_solve_s": round(sum(r["solve_s"] for r in stages_out), 4),
        # end to end: the solves plus each stage's Laplacian set-up and, for the
        # grouped order, the k-means that supplies the grouping (the warm-start
        # rows drawn on the host are the same in every mode and left out)
        "total_with_setup_s": round(sum(r["solve_s"] + r.get("laplacian_s", 0.0) +
                                        r.get("labels_s", 0.0) for r in stages_out), 4),
        "all_converged": all(r["converged"] == 1 for r in stages_out),
        "stages": stages_out,
    }


def streaming_edges(variant: str = "f1", n: int = 1_000_000, k: int = 32, parts: int = 10,
                    check_every: int = 10, fixed_iters: int = 2, dbar: float = 48.0,
                    max_iter: int = 1000):
    """Edge-sampling stream: the undirected edges of an SBM (N = 1M, k = 32
    equal blocks, mean degree 48 like the paper's 1M-node streaming graphs,
    r = 0.3) dealt to ten disjoint parts, stage s the graph of parts 0..s on
    the nodes touched so far, warm-started from the previous stage (carried
    rows; new nodes N(0, 1/N_s)).  Two runs: to residual 1e-4 per stage (FP32,
    graph-replayed loop, at most max_iter updates), and the numerical results'
    setting of a fixed 2 updates per stage, with the k-means labels of each
    stage's features scored against the planted blocks (ARI)."""
    import numpy as np
    import torch
    from sklearn.metrics import adjusted_rand_score
    from paper_2305_10356_amd import graphs, ofm
    from paper_2305_10356_amd.streaming import StreamingSolver
    t = time.perf_counter()
    g = graphs.sbm_plain(graphs.equal_sizes(n, k), dbar, 0.3, np.random.default_rng([7, 1]))
    es = graphs.EdgeStream(g, parts=parts, seed=7)
    stage_graphs = [es.stage(s) for s in range(parts)]
    log(f"edge stream generated in {time.perf_counter() - t:.1f} s")
    tri = variant.startswith("tri")
    out = {"workload": f"edge-sampling stream, {parts} parts of an SBM N={n} k={k} "
                       f"mean-degree {dbar:g} r=0.3, FP32, graph-replayed loop",
           "variant": variant}
    for mode in ("tol", "fixed"):
        sol = StreamingSolver(k, variant=variant, precision=ofm.OFM_FP32,
                              tol=1e-4 if mode == "tol" else 0.0, check_every=check_every,
                              max_iter=max_iter if mode == "tol" else fixed_iters,
                              graph=mode == "tol", restart=tri, seed=7)
        recs = []
        ids_prev = None
        for s, (h, ids) in enumerate(stage_graphs):
            carry = None if ids_prev is None else graphs.EdgeStream.carry(ids_prev, ids)
            rec = sol.solve_stage(h.row_ptr, h.col_idx, warm=True, carry=carry)
            if mode == "fixed":
                u = np.random.default_rng([7, 3, s]).random(k)
                lab, _, _ = ofm.kmeans(ofm.row_normalize(sol.X), k, u, max_iter=30)
                rec["ari"] = round(float(adjusted_rand_score(h.labels, lab.cpu().numpy())), 4)
                rec["relres"] = sol_residual(sol, h)
            for key in ("solve_s", "laplacian_s", "xinit_s"):
                rec[key] = round(rec[key], 4)
            log(f"edge stream {mode} stage {s}: {rec}")
            recs.append(rec)
            ids_prev = ids
        out[mode] = {"total_solve_s": round(sum(r["solve_s"] for r in recs), 4),
                     "total_with_setup_s": round(sum(r["solve_s"] + r["laplacian_s"]
                                                     for r in recs), 4),
                     "stages": recs}
    h, _ = stage_graphs[-1]
    cold = StreamingSolver(k, variant=variant, precision=ofm.OFM_FP32, tol=1e-4,
                           check_every=check_every, max_iter=max_iter, graph=True,
                           restart=tri, seed=8)
    rc = cold.solve_stage(h.row_ptr, h.col_idx, warm=False)
    out["last_stage_cold"] = {"iters": rc["iters"], "solve_s": round(rc["solve_s"], 4),
                              "converged": rc["converged"]}
    out["tol"]["all_converged"] = all(r["converged"] == 1 for r in out["tol"]["stages"])
    torch.cuda.synchronize()
    return out


def sol_residual(sol, h):
    """Residual of the solver's current features on stage graph h."""
    from paper_2305_10356_amd import ofm
    lap = ofm.Laplacian(h.row_ptr, h.col_idx)
    ws = ofm.Workspace(lap, sol.k, variant=sol.variant, precision=sol.precision)
    r = ws.residual(sol.X)["relres"]
    ws.close()
    lap.close()
    return r


def postprocess(X, k):
    """Algorithm 1 steps 4-5 on the features X (n x k, FP32, on the device):
    row normalisation and the K-means assignment, event-timed averages over
    repeated calls on torch's current stream against their HBM bytes, and the
    whole K-means (k-means++ seeding, Lloyd to no label change or 30
    iterations) timed on the host."""
    import numpy as np
    import torch
    from paper_2305_10356_amd import ofm
    n = X.shape[0]
    Yn = ofm.row_normalize(X)
    C = Yn[torch.randperm(n, device=X.device)[:k]].contiguous()
    ofm.kmeans_assign(Yn, C)
    esz = Yn.element_size()

    def timed_us(fn, reps=10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return 1e3 * e0.elapsed_time(e1) / reps

    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, _, km_iters = ofm.kmeans(Yn, k, np.random.default_rng([7, 7]).random(k), max_iter=30)
    torch.cuda.synchronize()
    t_km = time.perf_counter() - t1
    us_norm = timed_us(lambda: ofm.row_normalize(X, Yn))
    us_asg = timed_us(lambda: ofm.kmeans_assign(Yn, C))
    b_norm = 2 * n * k * esz
    b_asg = n * k * 4 + n * 4
    return {
        "row_normalize": {"us": round(us_norm, 1), "bytes": b_norm,
                          "GB_s": round(b_norm / us_norm / 1e3, 1)},
        "kmeans_assign": {"us": round(us_asg, 1), "bytes": b_asg, "clusters": k,
                          "GB_s": round(b_asg / us_asg / 1e3, 1)},
        "kmeans_full": {"seconds": round(t_km, 4), "lloyd_iters": int(km_iters)}}


def grouped_order(row_ptr, col_idx, X, k: int, x0, variant: str, planted):
    """The same step on the Laplacian whose row order is laid out for the eight
    XCDs by the clusters of a finished solve (k-means++ and Lloyd on the
    row-normalized features), as a re-solve or the next snapshot of a stream
    would have them."""
    import numpy as np
    import torch
    from paper_2305_10356_amd import ofm
    u = np.random.default_rng([7, 7]).random(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    labels, _, km_iters = ofm.kmeans(ofm.row_normalize(X), k, u, max_iter=30)
    lab = labels.cpu().numpy()
    t1 = time.perf_counter()
    lapg = ofm.Laplacian(row_ptr, col_idx, groups=lab)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    def timed_rate(prec):
        ws = ofm.Workspace(lapg, k, variant=variant, precision=prec, check_every=10,
                           restart=variant.startswith("tri"),
                           gather=ofm.GATHER_AUTO if prec == ofm.OFM_FP32 else
                           ofm.GATHER_DEFAULT)
        Xg = torch.as_tensor(x0, dtype=torch.float32, device="cuda").contiguous()
        ws.init(Xg)
        for _ in range(5):
            ws.step(Xg)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(50):
            ws.step(Xg)
        torch.cuda.synchronize()
        rate = 50 / (time.perf_counter() - t)
        ws.set_timing(True)
        for _ in range(20):
            ws.step(Xg)
        ws.set_timing(False)
        tm = ws.timing(reset=True)
        st = ws.stats()
        ws.close()
        return rate, tm, st

    rate, tm, st = timed_rate(ofm.OFM_FP32)
    rate_b, tm_b, _ = timed_rate(ofm.OFM_FP32_BF16X)
    lapg.close()
    # share of nodes whose cluster's majority planted block is their own
    agree = 0
    for c in range(k):
        m = lab == c
        if m.any():
            agree += np.bincount(planted[m]).max()
    return {"iters_per_s": round(rate, 1),
            "pass_us": {p: round(1e3 * v[0] / v[1], 1) for p, v in tm.items() if v[1]},
            "labels_s": round(t1 - t0, 4), "lloyd_iters": int(km_iters),
            "label_purity": round(float(agree) / len(lab), 4),
            "laplacian_with_upload_s": round(t2 - t1, 3),
            "gather": {1: "default", 2: "hot/cold"}[st["gather"]],
            "bf16_gather": {"iters_per_s": round(rate_b, 1),
                            "pass_us": {p: round(1e3 * v[0] / v[1], 1)
                                        for p, v in tm_b.items() if v[1]}}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--variant", default="f1", choices=["f1", "tri-f1", "f2", "tri-f2"])
    ap.add_argument("--n", type=int, default=None, help="override N (same recipe)")
    ap.add_argument("--k", type=int, default=32, choices=[4, 8, 16, 32, 64],
                    help="override k, the width of X (same graph)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched solve (no plain loop, no 2M-node run); prints its JSON")
    ap.add_argument("--no-streaming", action="store_true")
    ap.add_argument("--recur", action="store_true",
                    help="headline loop with A X by recurrence between residual checks")
    ap.add_argument("--streaming-only", action="store_true",
                    help="run only the streaming warm-start workload; prints its JSON")
    ap.add_argument("--edge-stream-only", action="store_true",
                    help="run only the edge-sampling streaming workload; prints its JSON")
    ap.add_argument("--gather", default="auto", choices=["auto", "default", "hot-cold"],
                    help="cache policy of the SpMM row gathers of the headline loop (auto: "
                         "timed at workspace creation)")
    ap.add_argument("--grouped", action="store_true",
                    help="with --postprocess-only: also time the step on the XCD-grouped order; "
                         "with --streaming-only: group each stage by the previous one's clusters")
    ap.add_argument("--postprocess-only", action="store_true",
                    help="solve the 2M-node graph to residual 1e-4, then time only the "
                         "post-processing (row normalisation, K-means); prints its JSON")
    ap.add_argument("--details", default=os.path.join(ROOT, "gpurun_out", "bench_details.json"),
                    help="file for the per-stage and per-variant detail (empty: none)")
    ap.add_argument("--orderings", default=None,
                    help="comma-separated node orders of the headline graph to time (random, "
                         "hub-first, rcm); prints their JSON")
    ap.add_argument("--gather-ceiling", action="store_true",
                    help="time random row gathers alone (tables of 4, 32, 256 MB class; rows of "
                         "64, 128, 256 B); prints their JSON")
    ap.add_argument("--ladder", action="store_true",
                    help="also time the SpMM with the columns folded into windows of X")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported (the "
              f"row-sharded multi-GPU design is described, not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2305_10356_amd import graphs, ofm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.batched_only:
        print(json.dumps(batched_vs_plain(args.variant, plain=False)), flush=True)
        return
    if args.gather_ceiling:
        print(json.dumps({"gather_ceiling": gather_ceiling()}), flush=True)
        return
    if args.edge_stream_only:
        print(json.dumps(streaming_edges(args.variant)), flush=True)
        return
    if args.streaming_only:
        print(json.dumps(streaming_c4(args.variant, recur=args.recur, grouped=args.grouped)),
              flush=True)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    k = args.k
    log("generating graph ...")
    t = time.perf_counter()
    g, x0 = graphs.workload("dcsbm-n2m-k32", n=args.n)
    if k != x0.shape[1]:
        x0 = graphs.initial_x(g.n, k, np.random.default_rng([3, 2, k]))
    gstats = g.stats()
    log(f"graph: {gstats} in {time.perf_counter() - t:.1f} s")
    n, nnz = g.n, g.nnz
    if args.orderings:
        if args.copy_calibration:
            # a plain 256 MiB device copy: counter calibration (as below)
            src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            for _ in range(5):
                dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
        print(json.dumps({"workload": f"dcsbm N={n} k={k} (nnz={nnz}) in other node orders",
                          "orderings": orderings_study(g, x0, k, args.variant,
                                                       args.orderings.split(","),
                                                       steps=args.steps,
                                                       gather={"auto": None,
                                                               "default": ofm.GATHER_DEFAULT,
                                                               "hot-cold": ofm.GATHER_HOT_COLD}[
                                                           args.gather])}), flush=True)
        return

    torch.cuda.synchronize()
    t = time.perf_counter()
    d_rp = torch.as_tensor(g.row_ptr, dtype=torch.int32).cuda()
    d_ci = torch.as_tensor(g.col_idx, dtype=torch.int32).cuda()
    torch.cuda.synchronize()
    t_up = time.perf_counter() - t
    t = time.perf_counter()
    lap = ofm.Laplacian(d_rp, d_ci)
    torch.cuda.synchronize()
    t_lap = time.perf_counter() - t
    del d_rp, d_ci
    ntiles = (n + 15) // 16
    upper = lap.upper()
    if args.postprocess_only:
        wsp = ofm.Workspace(lap, k, variant=args.variant, precision=ofm.OFM_FP32, check_every=10,
                            tol=1e-4, max_iter=3000, restart=args.variant.startswith("tri"))
        Xp = torch.as_tensor(x0, dtype=torch.float32, device=dev).contiguous()
        stp = wsp.solve(Xp)
        out = {"workload": "dcsbm-n2m-k32 features solved to residual 1e-4 (FP32, "
                           f"{stp['iters']} updates)", "postprocess": postprocess(Xp, k)}
        if args.grouped:
            out["grouped_order"] = grouped_order(g.row_ptr, g.col_idx, Xp, k, x0, args.variant,
                                                 g.labels)
        print(json.dumps(out), flush=True)
        return

    def make(variant, precision=ofm.OFM_FP32, **kw):
        ws = ofm.Workspace(lap, k, variant=variant, precision=precision, check_every=10,
                           restart=variant.startswith("tri"), **kw)
        dt = torch.float64 if precision == ofm.OFM_FP64 else torch.float32
        X = torch.as_tensor(x0, dtype=dt, device=dev).contiguous()
        return ws, X

    if args.copy_calibration:
        # a plain device-to-device copy of known size: 256 MiB read, 256 MiB
        # written per launch; hardware byte counters are scaled by it
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---------------- headline: iterations/s of the chosen variant ----------
    gather = {"auto": ofm.GATHER_AUTO, "default": ofm.GATHER_DEFAULT,
              "hot-cold": ofm.GATHER_HOT_COLD}[args.gather]
    ws, X = make(args.variant, recur=args.recur, gather=gather)
    ws.init(X)
    for _ in range(args.warmup):
        ws.step(X)
    # per-pass breakdown: a separate run with events around every pass (the
    # events themselves cost about 2% of a step, so the timed loop below
    # brackets only the two products with A)
    breakdown_steps = 50
    torch.cuda.synchronize()
    ws.timing(reset=True)
    ws.set_timing(True)
    for _ in range(breakdown_steps):
        ws.step(X)
    ws.set_timing(False)
    per_pass = ws.timing(reset=True)
    passes = {}
    for name, (ms, cnt) in per_pass.items():
        if cnt == 0:
            continue
        avg_ms = ms / cnt
        b = pass_bytes(name, n, nnz, k, 4, args.variant, ntiles, args.recur, upper=upper)
        passes[name] = {"launches": cnt, "avg_us": round(1e3 * avg_ms, 2),
                        "ms_per_step": round(ms / breakdown_steps, 4)}
        if b > 0:
            passes[name]["alg_bytes"] = int(b)
            passes[name]["alg_GBs"] = round(b / (avg_ms * 1e-3) / 1e9, 1)
    dom = max((p for p in passes if "alg_bytes" in passes[p]), key=lambda p: per_pass[p][0])
    spmms = [p for p in ("spmm_x", "spmm_v") if p in passes]

    # the timed region: wall time for `value`, HIP events around the products
    # with A (on the stream they are launched on) for the roofline
    timed = sorted(set(spmms + [dom]))
    ws.set_timing(timed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ws.step(X)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ws.set_timing(False)
    tm = ws.timing(reset=True)
    stats = ws.stats()
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps / elapsed

    def launch_roof(p):
        ms, cnt = tm[p]
        avg = ms / cnt
        alg = pass_bytes(p, n, nnz, k, 4, args.variant, ntiles, args.recur, upper=upper)
        lay = pass_bytes(p, n, nnz, k, 4, args.variant, ntiles, args.recur, layout=True,
                         upper=upper)
        ach = alg / (avg * 1e-3) / 1e9
        return {"launches": cnt, "avg_us": round(1e3 * avg, 2), "alg_bytes_per_launch": int(alg),
                "achieved": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                "layout_bytes_per_launch": int(lay),
                "layout_GBs": round(lay / (avg * 1e-3) / 1e9, 1)}

    from paper_2305_10356_amd import profiling
    traffic = profiling.read_traffic(os.path.join(
        ROOT, "profiles", f"pmc_traffic_ofm_step_{args.variant}_dcsbm_n2m_k32_fp32.md"))
    # the counters were taken with the hot/cold gathers; another policy moves other bytes
    if args.n is not None or args.k != 32 or args.recur or stats["gather"] != ofm.GATHER_HOT_COLD:
        traffic = {}
    d = launch_roof(dom)
    roofline = {"bound": "hbm", "achieved": d["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": d["frac"], "traffic": int(traffic[dom]) if dom in traffic else None,
                "kernel": dom, "launches": d["launches"], "avg_us": d["avg_us"],
                "alg_bytes_per_launch": d["alg_bytes_per_launch"],
                "layout_bytes_per_launch": d["layout_bytes_per_launch"]}
    for p in spmms:
        r = launch_roof(p)
        r["traffic"] = int(traffic[p]) if p in traffic else None
        roofline[p] = r
    if not args.no_extras and dom == "spmm_x" and k in (16, 32, 64):
        # what the memory system allows the dominant kernel: the same number of
        # random row gathers (nnz, rows of k FP32 values from an N-row table,
        # uniform at random) with no sparse-matrix work, timed now
        roofline["gather_ceiling"] = gather_ceiling_for(n, nnz, k, d["avg_us"])
    log(f"headline {args.variant}: {value:.1f} it/s, {ms_per_step:.3f} ms/step; roofline {roofline}; "
        f"passes {passes}")

    extras = {}
    summary = {}
    iters_to_tol = None
    if not args.no_extras:
        # SpMM alone (Y = A Z), FP32
        Z = torch.randn(n, k, device=dev)
        Y = torch.empty_like(Z)
        for _ in range(3):
            lap.apply(Z, Y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        reps = 20
        for _ in range(reps):
            lap.apply(Z, Y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        b = 4 * nnz + 8 * n + 2 * n * k * 4
        extras["spmm_apply_fp32"] = {"avg_us": round(1e3 * ms, 1), "alg_bytes": b,
                                     "alg_GBs": round(b / (ms * 1e-3) / 1e9, 1)}
        del Z, Y
        if args.ladder:
            extras["spmm_locality_ladder"] = spmm_locality_ladder(g, k)
        # the other variants, and the FP64 plain form; the triangular variants
        # run with the descent restart (outside Algorithm 2, see the key names)
        for v, prec in (("tri-f1", ofm.OFM_FP32), ("f2", ofm.OFM_FP32), ("tri-f2", ofm.OFM_FP32),
                        ("f1", ofm.OFM_FP64)):
            if v == args.variant and prec == ofm.OFM_FP32:
                continue
            w2, X2 = make(v, prec)
            w2.init(X2)
            for _ in range(5):
                w2.step(X2)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(50):
                w2.step(X2)
            torch.cuda.synchronize()
            tag = "_restart" if v.startswith("tri") else ""
            key = f"{v}{tag}_{'fp32' if prec == ofm.OFM_FP32 else 'fp64'}_iters_per_s"
            extras[key] = round(50 / (time.perf_counter() - t1), 1)
            w2.close()
            del X2
        # A X by recurrence between residual checks: one product with A per update
        w6, X6 = make(args.variant, recur=True)
        w6.init(X6)
        for _ in range(9):
            w6.step(X6)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(100):
            w6.step(X6)
        torch.cuda.synchronize()
        rec_rate = 100 / (time.perf_counter() - t1)
        w6.set_timing(True)
        for _ in range(30):
            w6.step(X6)
        w6.set_timing(False)
        tm6 = w6.timing(reset=True)
        w6.close()
        w7, X7 = make(args.variant, recur=True, tol=1e-4, max_iter=3000)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st7 = w7.solve(X7)
        torch.cuda.synchronize()
        t_rec_solve = time.perf_counter() - t1
        # the two gather policies of the SpMMs, each forced, same loop
        pol = {}
        for name, gp in (("default", ofm.GATHER_DEFAULT), ("hot/cold", ofm.GATHER_HOT_COLD)):
            wg, Xg = make(args.variant, gather=gp)
            wg.init(Xg)
            for _ in range(5):
                wg.step(Xg)
            wg.set_timing(["spmm_x", "spmm_v"])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(30):
                wg.step(Xg)
            torch.cuda.synchronize()
            rate = 30 / (time.perf_counter() - t1)
            wg.set_timing(False)
            tg = wg.timing(reset=True)
            pol[name] = {"iters_per_s": round(rate, 1),
                         "spmm_x_us": round(1e3 * tg["spmm_x"][0] / max(tg["spmm_x"][1], 1), 1),
                         "spmm_v_us": round(1e3 * tg["spmm_v"][0] / max(tg["spmm_v"][1], 1), 1)}
            wg.close()
            del Xg
        extras["gather_policy"] = pol
        extras["recur_ax"] = {
            "iters_per_s": round(rec_rate, 1),
            "pass_us": {p: round(1e3 * v[0] / v[1], 1) for p, v in tm6.items() if v[1]},
            "solve_to_1e-4": {"seconds": round(t_rec_solve, 3),
                              "iters": st7["iters"], "relres": st7["relres"],
                              "converged": st7["converged"]}}
        w7.close()
        del X6, X7
        # BF16 storage of the gathered rows: iterations/s and the residual it reaches
        w4, X4 = make(args.variant, ofm.OFM_FP32_BF16X, max_iter=300)
        w4.init(X4)
        for _ in range(5):
            w4.step(X4)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(50):
            w4.step(X4)
        torch.cuda.synchronize()
        bf_rate = 50 / (time.perf_counter() - t1)
        w4.set_timing(True)
        for _ in range(20):
            w4.step(X4)
        w4.set_timing(False)
        tm4 = w4.timing(reset=True)
        w4.close()
        w5, X5 = make(args.variant, ofm.OFM_FP32_BF16X, max_iter=300)
        st5 = w5.solve(X5)
        rr5 = w5.residual(X5)["relres"]
        extras["bf16_gather"] = {
            "iters_per_s": round(bf_rate, 1),
            "spmm_x_us": round(1e3 * tm4["spmm_x"][0] / max(tm4["spmm_x"][1], 1), 1),
            "spmm_v_us": round(1e3 * tm4["spmm_v"][0] / max(tm4["spmm_v"][1], 1), 1),
            "relres_after_300": rr5, "iters": st5["iters"]}
        w5.close()
        del X4, X5
        # time to residual 1e-4 (solve from X0)
        ws3, X3 = make(args.variant, tol=1e-4, max_iter=3000)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st3 = ws3.solve(X3)
        torch.cuda.synchronize()
        extras["solve_to_1e-4"] = {"seconds": round(time.perf_counter() - t1, 3),
                                   "iters": st3["iters"], "relres": st3["relres"],
                                   "converged": st3["converged"]}
        if st3["converged"]:
            iters_to_tol = int(st3["iters"])
        summary["solve_to_1e-4_s"] = extras["solve_to_1e-4"]["seconds"]
        if not args.no_batched:
            bvp = batched_vs_plain(args.variant)
            extras["batched_vs_plain"] = bvp
            summary.update({"batched_fp32_s": bvp["batched_fp32_s"],
                            "batched_form": bvp["batched_form"],
                            "batched_persistent_s": bvp["persistent_s"],
                            "plain_fp64_loop_s": bvp["plain_fp64_loop_s"],
                            "speedup": bvp["speedup"],
                            "batched_converged": f"{bvp['eager']['converged']}/{bvp['graphs']}",
                            "plain_converged": f"{bvp['plain_converged']}/{bvp['graphs']}"})
        if not args.no_streaming:
            gs = graphs.GrowthStream(n_final=2_000_000, stages=10, k=64, dbar=20, r=0.3, seed=4)
            extras["streaming_warm_start"] = streaming_c4(args.variant, gs=gs)
            extras["streaming_warm_start_recur"] = streaming_c4(args.variant, recur=True, gs=gs)
            extras["streaming_warm_start_grouped"] = streaming_c4(args.variant, grouped=True,
                                                                  gs=gs)
            del gs
            sw = extras["streaming_warm_start"]
            summary["stream_total_s"] = sw["total_solve_s"]
            summary["stream_total_with_setup_s"] = sw["total_with_setup_s"]
            summary["stream_all_converged"] = sw["all_converged"]
            ed = streaming_edges(args.variant)
            extras["streaming_edge_sampling"] = ed
            summary["edge_stream_total_s"] = ed["tol"]["total_solve_s"]
            summary["edge_stream_all_converged"] = ed["tol"]["all_converged"]
            summary["edge_stream_2_updates_ari_last"] = ed["fixed"]["stages"][-1]["ari"]
        extras["postprocess"] = postprocess(X3, k)
        extras["grouped_order"] = grouped_order(g.row_ptr, g.col_idx, X3, k, x0, args.variant,
                                                g.labels)
        extras["laplacian_build_s"] = round(t_lap, 3)
        extras["csr_upload_s"] = round(t_up, 3)
        del X3
        for key in ("tri-f1_restart_fp32_iters_per_s", "f2_fp32_iters_per_s",
                    "tri-f2_restart_fp32_iters_per_s", "f1_fp64_iters_per_s"):
            if key in extras:
                summary[key] = extras[key]
        summary["recur_ax_iters_per_s"] = extras["recur_ax"]["iters_per_s"]

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        from oracle import ofm_oracle as O
        vid = {"f1": O.F1, "tri-f1": O.TRI_F1, "f2": O.F2, "tri-f2": O.TRI_F2}[args.variant]
        cpu = cpu_baseline(g, x0, k, vid, gpu_iters_to_tol=iters_to_tol)
        # the error of the device path against the oracle on the same first
        # two updates (set-up step + one loop iteration), per precision
        xo = cpu_baseline.first_step_x
        prec_err = {}
        for name, prec in (("fp32", ofm.OFM_FP32), ("fp64", ofm.OFM_FP64)):
            w8, X8 = make(args.variant, prec)
            if prec == ofm.OFM_FP64:
                X8.copy_(torch.as_tensor(x0.astype(np.float32).astype(np.float64)))
            w8.init(X8)
            w8.step(X8)
            xg = X8.cpu().numpy().astype(np.float64)
            prec_err[name] = float(np.abs(xg - xo).max() / np.abs(xo).max())
            w8.close()
            del X8
        cpu["device_vs_oracle_rel_err"] = prec_err

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"dcsbm N={n} k={k} mean-degree 25 power-law 2.5 r=0.5 (nnz={nnz})",
                   "variant": args.variant, "precision": "fp32 passes, fp64 k x k products",
                   "check_every": 10, "recur_ax": bool(args.recur),
                   "gather": {1: "default", 2: "hot/cold"}[stats["gather"]]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        **summary,
        "passes": passes,
        "relres_last_check": stats["relres"],
    }
    details = {"graph": gstats, "clocks": read_clocks(), "extras": extras}
    if args.details:
        os.makedirs(os.path.dirname(os.path.abspath(args.details)), exist_ok=True)
        with open(args.details, "w") as f:
            json.dump({"headline": out, **details}, f)
        out["details_file"] = os.path.relpath(args.details, ROOT)
    print(json.dumps(out), flush=True)

if __name__ == "__main__":
    main()
