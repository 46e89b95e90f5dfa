"""Streaming warm starts (numerical results, comparison on streaming graphs) and
the graph-captured solve loop.

* ofm_solve with the loop replayed as HIP graphs gives bitwise the iterate,
  the residual and the iteration count of the eager loop;
* every stage of a small growth stream, warm-started from the previous
  stage, reaches the tolerance, and its limit matches the dense
  eigendecomposition of that stage's Laplacian (Theorem 1 for f1, Theorem 3
  for f2), checked with the FP64 oracle;
* warm starts need fewer iterations than cold starts from N(0, 1/N);
* a stream whose stages are built in the row order grouped by the previous
  stage's clusters converges like the plain order."""
import sys

import numpy as np
import pytest

from oracle import ofm_oracle as O
from paper_2305_10356_amd import graphs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("prec,ce,variant", [("fp64", 10, "f1"), ("fp64", 7, "tri-f2"),
                                             ("fp64", 1, "f2"), ("fp32", 10, "f1"),
                                             ("fp32", 5, "tri-f1")])
def test_graph_replay_is_bitwise_eager(lib, prec, ce, variant):
    from paper_2305_10356_amd import ofm
    g, x0 = graphs.workload("sbm-n1000-k8" if prec == "fp64" else "sbm-n50k-k32")
    k = x0.shape[1]
    lap = ofm.Laplacian(g.row_ptr, g.col_idx)
    p = ofm.OFM_FP64 if prec == "fp64" else ofm.OFM_FP32
    dt = torch.float64 if prec == "fp64" else torch.float32
    tol = 1e-7 if prec == "fp64" else 1e-4
    restart = variant.startswith("tri")
    out = []
    for graph in (False, True):
        say(f"graph={graph} {prec} ce={ce} {variant}")
        ws = ofm.Workspace(lap, k, variant=variant, precision=p, max_iter=400, check_every=ce,
                           tol=tol, restart=restart, graph=graph)
        X = torch.as_tensor(x0, dtype=dt).cuda()
        st = ws.solve(X)
        out.append((host(X), st))
        if graph:
            # a second solve replays the kept graphs from a fresh init
            X2 = torch.as_tensor(x0, dtype=dt).cuda()
            st2 = ws.solve(X2)
            assert st2 == st
            np.testing.assert_array_equal(host(X2), out[0][0])
        ws.close()
    (xe, se), (xg, sg) = out
    assert se == sg
    np.testing.assert_array_equal(xe, xg)


def test_graph_replay_hits_max_iter_exactly(lib):
    from paper_2305_10356_amd import ofm
    g, x0 = graphs.workload("sbm-n1000-k8")
    lap = ofm.Laplacian(g.row_ptr, g.col_idx)
    res = []
    for graph in (False, True):
        ws = ofm.Workspace(lap, 8, variant="f1", precision=ofm.OFM_FP64, max_iter=37,
                           check_every=10, tol=1e-30, graph=graph)
        X = torch.as_tensor(x0).cuda()
        st = ws.solve(X)
        assert st["iters"] == 37 and st["relres_iter"] == 30
        res.append(host(X))
    np.testing.assert_array_equal(res[0], res[1])


def _stream_case(variant, vid, prec, k, n_final, stages, tol, recur=False):
    from paper_2305_10356_amd import ofm
    from paper_2305_10356_amd.streaming import StreamingSolver
    gs = graphs.GrowthStream(n_final=n_final, stages=stages, k=k, dbar=20, r=0.3, seed=7)
    warm = StreamingSolver(k, variant=variant, precision=prec, tol=tol, check_every=5,
                           max_iter=4000, graph=True, recur=recur, seed=7)
    cold = StreamingSolver(k, variant=variant, precision=prec, tol=tol, check_every=5,
                           max_iter=4000, graph=True, recur=recur, seed=7)
    recs = []
    for s in range(stages):
        g = gs.snapshot(s)
        say(f"stream {variant} stage {s} n={g.n}")
        rw = warm.solve_stage(g.row_ptr, g.col_idx, warm=True)
        rc = cold.solve_stage(g.row_ptr, g.col_idx, warm=False)
        assert rw["converged"] == 1 and rc["converged"] == 1, (rw, rc)
        recs.append((g, rw, rc, host(warm.X)))
    return recs


@pytest.mark.parametrize("variant,vid", [("f1", O.F1), ("f2", O.F2)])
def test_streaming_fp64_limits_match_dense_eigh(lib, variant, vid):
    from paper_2305_10356_amd import ofm
    k = 4
    tol = 1e-6
    recs = _stream_case(variant, vid, ofm.OFM_FP64, k, 2400, 3, tol)
    for s, (g, rw, rc, X) in enumerate(recs):
        olap = O.laplacian(g.n, g.row_ptr, g.col_idx)
        r = O.relres(olap, X)
        assert r <= 1.05 * tol  # the Gram form loses ~4 digits at 1e-6
        mu, U = O.dense_eigh(olap)
        lam = mu - 2.0
        gap = mu[k] - mu[k - 1]
        assert gap > 1e-2  # the limit is well defined
        # Davis-Kahan: sin(angle(span X, U_k)) <= ||A Q - Q T||_F / gap, where
        # the Ritz residual is relres * ||T||_F for the Ritz values T
        Q, _ = np.linalg.qr(X)
        T = np.linalg.eigvalsh(Q.T @ O.apply_A(olap, Q))
        sin_f = np.linalg.norm(Q - U[:, :k] @ (U[:, :k].T @ Q))
        assert sin_f <= 1.5 * r * np.linalg.norm(T) / gap + 1e-12
        # Ritz values: second order in the residual
        np.testing.assert_allclose(T, lam[:k], atol=10 * (r * np.linalg.norm(T)) ** 2 / gap + 1e-13)
        ev = np.sort(np.linalg.eigvalsh(X.T @ X))
        # Theorem 1: X^T X -> -Lam_k (f1); Theorem 3: X^T X -> I (f2)
        target = np.sort(-lam[:k]) if vid == O.F1 else np.ones(k)
        np.testing.assert_allclose(ev, target, atol=20 * r)
        if s > 0:
            assert rw["iters"] < rc["iters"], (rw, rc)


@pytest.mark.parametrize("recur", [False, True])
def test_streaming_fp32_k64(lib, recur):
    from paper_2305_10356_amd import ofm
    recs = _stream_case("f1", O.F1, ofm.OFM_FP32, 64, 90000, 3, 1e-4, recur=recur)
    warm_iters = [rw["iters"] for _, rw, _, _ in recs[1:]]
    cold_iters = [rc["iters"] for _, _, rc, _ in recs[1:]]
    say("warm", warm_iters, "cold", cold_iters)
    assert sum(warm_iters) < sum(cold_iters)
    g, rw, _, X = recs[-1]
    olap = O.laplacian(g.n, g.row_ptr, g.col_idx)
    # the FP64 residual of the FP32 iterate agrees with the library's
    assert O.relres(olap, X) == pytest.approx(rw["relres"], rel=0.05, abs=2e-6)


def test_streaming_grouped_order_fp32(lib):
    """Each stage after the first built with its rows grouped for the XCDs by
    the previous stage's clusters: every stage converges, the residual of the
    last iterate agrees with the oracle's, and the iterations match the plain
    order's within the spread of FP32 roundings."""
    from paper_2305_10356_amd import ofm
    from paper_2305_10356_amd.streaming import StreamingSolver
    gs = graphs.GrowthStream(n_final=90000, stages=3, k=64, dbar=20, r=0.3, seed=7)
    plain = StreamingSolver(64, precision=ofm.OFM_FP32, tol=1e-4, check_every=5, max_iter=4000,
                            graph=True, seed=7)
    grp = StreamingSolver(64, precision=ofm.OFM_FP32, tol=1e-4, check_every=5, max_iter=4000,
                          graph=True, seed=7, grouped=True)
    for s in range(3):
        g = gs.snapshot(s)
        say(f"grouped stream stage {s} n={g.n}")
        rp = plain.solve_stage(g.row_ptr, g.col_idx)
        rg = grp.solve_stage(g.row_ptr, g.col_idx)
        say("plain", rp["iters"], "grouped", rg["iters"], rg["grouped_order"])
        assert rg["converged"] == 1 and rg["grouped_order"] == (s > 0)
        assert grp.labels.shape == (g.n,) and grp.labels.min() >= 0 and grp.labels.max() < 64
        assert rg["iters"] <= 2 * rp["iters"] + 20
    olap = O.laplacian(g.n, g.row_ptr, g.col_idx)
    assert O.relres(olap, host(grp.X)) == pytest.approx(rg["relres"], rel=0.05, abs=2e-6)


@pytest.mark.parametrize("variant,prec", [("f1", "fp64"), ("f2", "fp32")])
def test_edge_sampling_stream(lib, variant, prec):
    # ten disjoint edge parts of an SBM, each stage adding one (the nodes
    # touched so far; the previous rows carried to their new positions): the
    # carried rows enter the stage unchanged, and every stage from the third
    # on reaches the tolerance with the oracle's residual of the returned X
    # matching the device's
    from paper_2305_10356_amd import ofm
    from paper_2305_10356_amd.streaming import StreamingSolver
    g = graphs.sbm_plain(graphs.equal_sizes(6000, 8), 48.0, 0.15, np.random.default_rng([61, 1]))
    es = graphs.EdgeStream(g, parts=10, seed=61)
    p = ofm.OFM_FP64 if prec == "fp64" else ofm.OFM_FP32
    tol = 1e-6 if prec == "fp64" else 1e-4
    sol = StreamingSolver(8, variant=variant, precision=p, tol=tol, check_every=10,
                          max_iter=4000, graph=True, seed=61)
    ids_prev, x_prev = None, None
    for s in range(10):
        h, ids = es.stage(s)
        carry = None if ids_prev is None else graphs.EdgeStream.carry(ids_prev, ids)
        if carry is not None:
            X0 = sol.initial_block(h.n, sol.X, carry)
            np.testing.assert_array_equal(host(X0)[carry], x_prev)
        rec = sol.solve_stage(h.row_ptr, h.col_idx, warm=True, carry=carry)
        olap = O.laplacian(h.n, h.row_ptr, h.col_idx)
        x_prev = host(sol.X)
        rr = O.relres(olap, x_prev)
        say(f"edge stage {s}: n={h.n} nnz={h.nnz} iters={rec['iters']} relres={rec['relres']:.2e} "
            f"oracle={rr:.2e}")
        assert rec["status"] == 0
        if s >= 2:
            assert rec["converged"] == 1
            # below ~1e-7 the Gram form of the residual is at its rounding floor
            assert rr == pytest.approx(rec["relres"], rel=0.05, abs=1e-7 if prec == "fp64" else 2e-6)
        ids_prev = ids
    # the last stage is the whole graph: warm start from the ninth stage beats
    # a cold start
    cold = StreamingSolver(8, variant=variant, precision=p, tol=tol, check_every=10,
                           max_iter=4000, graph=True, seed=62)
    h, _ = es.stage(9)
    rc = cold.solve_stage(h.row_ptr, h.col_idx, warm=False)
    say(f"last stage warm {sol.records[-1]['iters']} vs cold {rc['iters']} updates")
    assert sol.records[-1]["iters"] < rc["iters"]
