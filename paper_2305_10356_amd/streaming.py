"""Warm-started solves over a stream of growing graphs.

The numerical results section (comparison on streaming graphs) feeds each
stage's computed features to the next stage as its initial point; the methods
then converge in a few iterations because the old features are already close
to the new ones.  A stage here is either a snapshot of a node-arrival growth
process (node ids are arrival order, so a snapshot is a prefix of the next
one: the previous rows stay in place and rows N(0, 1/N_s) are appended for
the new nodes) or a stage of an edge-sampling stream (the graph of the first
s+1 edge parts on the nodes touched so far: the previous rows go to the
positions ``carry`` gives and the newly touched nodes get rows N(0, 1/N_s)).

Every stage runs ``ofm_solve`` with the loop captured as HIP graphs of
check_every updates (``graph=True``); the gather policy of the products with
A is timed at the first stage with a large enough block and kept afterwards.  Host work per stage: building the
Laplacian handle and assembling the initial block; both are timed apart from
the solve.
"""
from __future__ import annotations

import math
import time
from typing import List

import numpy as np

from . import ofm


def new_rows(n_old: int, n: int, k: int, seed, dtype=np.float32) -> np.ndarray:
    """Rows n_old..n-1 of a warm start, N(0, 1/n), from a seeded stream."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n - n_old, k)) / math.sqrt(n)).astype(dtype)


class StreamingSolver:
    """Solves stage after stage, each from the previous stage's solution."""

    def __init__(self, k: int, variant="f1", precision=ofm.OFM_FP32, tol: float = 1e-4,
                 check_every: int = 10, max_iter: int = 5000, graph: bool = True,
                 restart: bool = False, recur: bool = False, seed: int = 4,
                 gather: int = ofm.GATHER_AUTO, grouped: bool = False,
                 label_iters: int = 30):
        self.k = k
        self.variant = variant
        self.precision = precision
        self.tol = tol
        self.check_every = check_every
        self.max_iter = max_iter
        self.graph = graph
        self.restart = restart
        self.recur = recur
        self.seed = seed
        # gather policy: chosen by timing at the first stage whose block is
        # large enough, then kept for the later stages
        self.gather = gather
        # grouped: after each stage, cluster its features (Algorithm 1, steps
        # 4-5) and build the next stage's Laplacian with its rows laid out for
        # the XCDs by those clusters (new nodes in no group)
        self.grouped = grouped
        self.label_iters = label_iters
        self.labels = None
        self.X = None
        self.stage = 0
        self.records: List[dict] = []

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == ofm.OFM_FP64 else torch.float32

    def initial_block(self, n: int, x_prev=None, carry=None):
        """Device block for a stage with n nodes: x_prev's rows (at positions
        ``carry``, default the first rows), new rows N(0, 1/n) elsewhere."""
        import torch
        n_old = 0 if x_prev is None else int(x_prev.shape[0])
        if n_old > n:
            raise ValueError("a stage cannot drop nodes")
        npdt = np.float64 if self.precision == ofm.OFM_FP64 else np.float32
        X = torch.empty((n, self.k), dtype=self.dtype, device="cuda")
        fresh = torch.from_numpy(new_rows(n_old, n, self.k, [self.seed, 2, self.stage], npdt))
        if carry is None:
            if n_old:
                X[:n_old].copy_(x_prev)
            if n > n_old:
                X[n_old:].copy_(fresh)
            return X
        carry = np.asarray(carry, dtype=np.int64)
        if carry.shape != (n_old,):
            raise ValueError("carry must give one position per previous row")
        new = np.ones(n, dtype=bool)
        new[carry] = False
        if n_old:
            X[torch.from_numpy(carry).cuda()] = x_prev
        if n > n_old:
            X[torch.from_numpy(np.flatnonzero(new)).cuda()] = fresh.cuda()
        return X

    def solve_stage(self, row_ptr, col_idx, warm: bool = True, carry=None) -> dict:
        """Solve the next stage.  ``warm=False`` starts from a fresh random
        block instead (the cold-start comparison); the solver's state still
        advances to this stage's solution.  ``carry``: positions in this stage
        of the previous stage's rows (default: the first rows)."""
        import torch
        n = int(row_ptr.shape[0] - 1)
        t0 = time.perf_counter()
        groups = None
        if self.grouped and self.labels is not None and warm:
            groups = np.full(n, -1, dtype=np.int32)
            if carry is None:
                groups[:self.labels.shape[0]] = self.labels
            else:
                groups[np.asarray(carry, dtype=np.int64)] = self.labels
        lap = ofm.Laplacian(row_ptr, col_idx, groups=groups)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        X = self.initial_block(n, self.X if warm else None, carry if warm else None)
        ws = ofm.Workspace(lap, self.k, variant=self.variant, precision=self.precision,
                           max_iter=self.max_iter, check_every=self.check_every,
                           tol=self.tol, graph=self.graph, restart=self.restart,
                           recur=self.recur, gather=self.gather)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st = ws.solve(X)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        rec = {
            "stage": self.stage, "n": n, "nnz": int(col_idx.shape[0]), "warm": bool(warm and
                                                                                 self.X is not None),
            "iters": int(st["iters"]), "relres": float(st["relres"]),
            "converged": int(st["converged"]), "status": int(st["status"]),
            "solve_s": t3 - t2, "laplacian_s": t1 - t0, "xinit_s": t2 - t1,
            "gather": int(st["gather"]),
        }
        if self.grouped:
            u = np.random.default_rng([self.seed, 3, self.stage]).random(self.k)
            labels, _, _ = ofm.kmeans(ofm.row_normalize(X), self.k, u, max_iter=self.label_iters)
            self.labels = labels.cpu().numpy()
            torch.cuda.synchronize()
            rec["labels_s"] = time.perf_counter() - t3
            rec["grouped_order"] = groups is not None
        if self.gather == ofm.GATHER_AUTO and n * self.k * (8 if self.precision == ofm.OFM_FP64
                                                            else 4) >= 32 << 20:
            self.gather = int(st["gather"])
        self.records.append(rec)
        self.X = X
        self.stage += 1
        ws.close()
        lap.close()
        return rec
