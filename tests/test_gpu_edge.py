"""Edge cases of the method and of the tiling, through the C ABI, against the
FP64 oracle and the dense eigendecomposition:

* k = N (X square): the limits are the full decompositions of Theorems 1 and
  3, and the Ritz residual is zero for any X of full rank, so the solve is run
  for a fixed number of updates;
* a disconnected graph (A has eigenvalue -2 once per component);
* graphs smaller than one tile, and one row past a tile;
* weighted similarities;
* a step before the set-up step is refused."""
import sys

import numpy as np
import pytest

from oracle import ofm_oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def csr(n, edges, weights=None):
    u = np.array([a for a, b in edges] + [b for a, b in edges], dtype=np.int64)
    v = np.array([b for a, b in edges] + [a for a, b in edges], dtype=np.int64)
    w = None if weights is None else np.concatenate([weights, weights])
    order = np.lexsort((v, u))
    u, v = u[order], v[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, u + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return rp, v.astype(np.int32), (None if w is None else w[order])


def cycle_edges(n, off=0):
    return [(off + i, off + (i + 1) % n) for i in range(n)]


def x0_for(n, k, seed):
    return np.random.default_rng(seed).standard_normal((n, k)) / np.sqrt(n)


def run_fixed(ofm, lap, x0, variant, iters, precision=None, restart=False):
    precision = ofm.OFM_FP64 if precision is None else precision
    dt = torch.float64 if precision == ofm.OFM_FP64 else torch.float32
    ws = ofm.Workspace(lap, x0.shape[1], variant=variant, precision=precision, max_iter=iters,
                       check_every=1000000, tol=0.0, restart=restart)
    X = torch.as_tensor(x0, dtype=dt).cuda()
    st = ws.solve(X)
    assert st["iters"] == iters and st["status"] == 0, st
    return host(X)


@pytest.mark.parametrize("variant", ["f1", "f2"])
def test_k_equals_n(lib, variant):
    # an odd cycle with a chord: connected and not bipartite, so every
    # eigenvalue of A lies in [-2, 0)
    from paper_2305_10356_amd import ofm
    n = 8
    rp, ci, _ = csr(n, cycle_edges(7) + [(7, 0), (7, 3)])
    lap = ofm.Laplacian(rp, ci)
    olap = O.laplacian(n, rp, ci)
    A = O.dense_A(olap)
    assert np.linalg.eigvalsh(A).max() < -1e-3
    X = run_fixed(ofm, lap, x0_for(n, n, 3), variant, 300)
    if variant == "f1":
        # Theorem 1 with k = N: X X^T = -A
        np.testing.assert_allclose(X @ X.T, -A, atol=1e-9)
    else:
        # Theorem 3 with k = N: X^T X = I
        np.testing.assert_allclose(X.T @ X, np.eye(n), atol=1e-9)
    # the Ritz residual vanishes for every full-rank square X
    ws = ofm.Workspace(lap, n, variant=variant, precision=ofm.OFM_FP64)
    r = ws.residual(torch.as_tensor(x0_for(n, n, 4)).cuda())
    assert r["relres"] < 1e-6


def test_disconnected_graph(lib):
    # a 5-cycle and a 7-cycle: A has eigenvalue -2 twice, then the pair of the
    # 7-cycle at -2 + (1 - cos(2 pi / 7)); the fifth eigenvalue is separated
    from paper_2305_10356_amd import ofm
    n, k = 12, 4
    rp, ci, _ = csr(n, cycle_edges(5) + cycle_edges(7, 5))
    lap = ofm.Laplacian(rp, ci)
    olap = O.laplacian(n, rp, ci)
    mu, U = O.dense_eigh(olap)
    assert abs(mu[0]) < 1e-12 and abs(mu[1]) < 1e-12 and mu[4] - mu[3] > 0.1
    for variant, restart in (("f1", False), ("f2", False), ("tri-f1", True)):
        X = run_fixed(ofm, lap, x0_for(n, k, 5), variant, 400, restart=restart)
        Uk = U[:, :k]
        if variant in ("f1", "tri-f1"):
            target = (Uk * (2.0 - mu[:k])[None, :]) @ Uk.T
        else:
            target = Uk @ Uk.T
        np.testing.assert_allclose(X @ X.T, target, atol=1e-8, err_msg=variant)


@pytest.mark.parametrize("n,k", [(5, 4), (16, 8), (17, 16), (33, 32)])
def test_small_and_ragged_graphs(lib, n, k):
    from paper_2305_10356_amd import ofm
    rng = np.random.default_rng(n)
    edges = cycle_edges(n) + [(int(a), int(b)) for a, b in rng.integers(0, n, size=(2 * n, 2))
                              if a != b]
    edges = list({(min(a, b), max(a, b)) for a, b in edges})
    rp, ci, _ = csr(n, edges)
    lap = ofm.Laplacian(rp, ci)
    olap = O.laplacian(n, rp, ci)
    x0 = x0_for(n, k, n + 1)
    # one set-up step and a few loop steps, FP64 and FP32, against the oracle
    for prec, dt, tol in ((ofm.OFM_FP64, torch.float64, 1e-10), (ofm.OFM_FP32, torch.float32, 1e-4)):
        xs = x0 if dt == torch.float64 else x0.astype(np.float32).astype(np.float64)
        ws = ofm.Workspace(lap, k, variant="f2", precision=prec, check_every=1000000)
        X = torch.as_tensor(xs, dtype=dt).cuda()
        ws.init(X)
        st, _ = O.init(olap, xs, O.Options(variant=O.F2))
        for _ in range(3):
            ws.step(X)
            st, _ = O.step(olap, st, O.Options(variant=O.F2))
        err = np.abs(host(X) - st.X).max() / np.abs(st.X).max()
        say(f"n={n} k={k} prec={prec}: err {err:.2e}")
        assert err < tol


def test_weighted_graph(lib):
    from paper_2305_10356_amd import graphs, ofm
    g, x0 = graphs.workload("sbm-n1000-k8")
    rng = np.random.default_rng(77)
    # symmetric positive weights: one weight per undirected edge
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    key = np.minimum(rows, g.col_idx) * g.n + np.maximum(rows, g.col_idx)
    uniq, inv = np.unique(key, return_inverse=True)
    w = rng.uniform(0.1, 3.0, size=uniq.shape[0])[inv]
    lap = ofm.Laplacian(g.row_ptr, g.col_idx, vals=w, validate=True)
    olap = O.laplacian(g.n, g.row_ptr, g.col_idx, vals=w)
    np.testing.assert_allclose(lap.info()["degrees"], olap.d, rtol=1e-14)
    Z = rng.standard_normal((g.n, 8))
    Y = host(lap.apply(torch.as_tensor(Z).cuda()))
    np.testing.assert_allclose(Y, O.apply_A(olap, Z), rtol=0, atol=1e-13 * np.abs(Y).max())
    X = run_fixed(ofm, lap, x0, "f1", 500)
    mu, U = O.dense_eigh(olap)
    Uk = U[:, :8]
    np.testing.assert_allclose(X @ X.T, (Uk * (2.0 - mu[:8])[None, :]) @ Uk.T, atol=1e-6)


def cycle_with_loops(n, w):
    """C_n plus a self-loop of weight w at every node (stored once per row)."""
    rp, ci, _ = csr(n, cycle_edges(n))
    rows = np.repeat(np.arange(n), np.diff(rp))
    rows = np.concatenate([rows, np.arange(n)])
    cols = np.concatenate([ci, np.arange(n)])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    vals = np.where(rows == cols, w, 1.0)
    return np.cumsum(rp).astype(np.int32), cols.astype(np.int32), vals


@pytest.mark.parametrize("w", [0.5, 3.0])
@pytest.mark.parametrize("n", [11, 40])
def test_self_loops_closed_form(lib, n, w):
    # S = adjacency(C_n) + w I is (2 + w)-regular: ||A||_F^2 = n (1 + w/(2+w))^2
    # + 2n/(2+w)^2, and cos(2 pi j i / n) is an eigenvector of A with eigenvalue
    # -1 - (w + 2 cos(2 pi j / n)) / (2 + w); weights given in FP64 and in FP32
    # (0.5 and 3 are exact in both) build the same Laplacian
    from paper_2305_10356_amd import ofm
    rp, ci, vals = cycle_with_loops(n, w)
    d = 2.0 + w
    expect = n * (1.0 + w / d) ** 2 + 2.0 * n / d ** 2
    olap = O.laplacian(n, rp, ci, vals=vals)
    i = np.arange(n)
    Z = np.stack([np.cos(2 * np.pi * j * i / n) for j in range(8)], axis=1)
    lam = -1.0 - (w + 2.0 * np.cos(2 * np.pi * np.arange(8) / n)) / d
    outs = []
    for vv in (vals, vals.astype(np.float32)):
        lap = ofm.Laplacian(rp, ci, vals=vv, validate=True)
        info = lap.info()
        np.testing.assert_allclose(info["degrees"], d, rtol=1e-15)
        assert info["normA2"] == pytest.approx(expect, rel=1e-13)
        assert info["normA2"] == pytest.approx(O.norm_A_fro_sq(olap), rel=1e-13)
        Y = host(lap.apply(torch.as_tensor(Z).cuda()))
        np.testing.assert_allclose(Y, Z * lam[None, :], rtol=0, atol=1e-13)
        np.testing.assert_allclose(Y, O.apply_A(olap, Z), rtol=0, atol=1e-13)
        Y32 = host(lap.apply(torch.as_tensor(Z.astype(np.float32)).cuda()))
        np.testing.assert_allclose(Y32, O.apply_A(olap, Z.astype(np.float32).astype(np.float64)),
                                   rtol=0, atol=1e-6)
        outs.append((info["normA2"], Y))
    assert outs[0][0] == outs[1][0] and np.array_equal(outs[0][1], outs[1][1])


def test_fp32_weights_match_fp64(lib):
    # FP32 weights are widened exactly: the Laplacian equals the one built from
    # the same values in FP64, bit for bit
    from paper_2305_10356_amd import graphs, ofm
    g, _ = graphs.workload("sbm-n1000-k8")
    rng = np.random.default_rng(78)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    key = np.minimum(rows, g.col_idx) * g.n + np.maximum(rows, g.col_idx)
    uniq, inv = np.unique(key, return_inverse=True)
    w32 = rng.uniform(0.1, 3.0, size=uniq.shape[0]).astype(np.float32)[inv]
    l32 = ofm.Laplacian(g.row_ptr, g.col_idx, vals=w32, validate=True)
    l64 = ofm.Laplacian(g.row_ptr, g.col_idx, vals=w32.astype(np.float64), validate=True)
    i32, i64 = l32.info(), l64.info()
    assert np.array_equal(i32["degrees"], i64["degrees"]) and i32["normA2"] == i64["normA2"]
    Z = torch.as_tensor(rng.standard_normal((g.n, 16))).cuda()
    assert torch.equal(l32.apply(Z), l64.apply(Z))
    olap = O.laplacian(g.n, g.row_ptr, g.col_idx, vals=w32.astype(np.float64))
    assert i32["normA2"] == pytest.approx(O.norm_A_fro_sq(olap), rel=1e-12)


def test_step_before_init_is_refused(lib):
    from paper_2305_10356_amd import graphs, ofm
    g, x0 = graphs.workload("sbm-n1000-k8")
    lap = ofm.Laplacian(g.row_ptr, g.col_idx)
    ws = ofm.Workspace(lap, 8, variant="f1", precision=ofm.OFM_FP64)
    X = torch.as_tensor(x0).cuda()
    with pytest.raises(ofm.OfmError) as e:
        ws.step(X)
    assert e.value.status == -1
    # wrong dtype / shape are refused before anything is enqueued
    with pytest.raises(ValueError):
        ws.init(X.float())
    with pytest.raises(ValueError):
        ws.init(X[:, :4].contiguous())


def test_timing_mask_selects_passes(lib):
    from paper_2305_10356_amd import graphs, ofm
    g, x0 = graphs.workload("sbm-n1000-k8")
    lap = ofm.Laplacian(g.row_ptr, g.col_idx)
    ws = ofm.Workspace(lap, 8, variant="f1", precision=ofm.OFM_FP64)
    X = torch.as_tensor(x0).cuda()
    ws.init(X)
    ws.timing(reset=True)
    ws.set_timing(["spmm_x"])
    for _ in range(3):
        ws.step(X)
    ws.set_timing(False)
    t = ws.timing(reset=True)
    assert t["spmm_x"][1] == 3 and t["spmm_x"][0] > 0
    assert all(cnt == 0 for p, (ms, cnt) in t.items() if p != "spmm_x")
    ws.set_timing(True)
    ws.step(X)
    ws.set_timing(False)
    t = ws.timing(reset=True)
    assert t["spmm_x"][1] == 1 and t["v"][1] == 1 and t["update"][1] == 1


@pytest.mark.parametrize("variant,vid", [("f1", O.F1), ("tri-f1", O.TRI_F1), ("f2", O.F2),
                                         ("tri-f2", O.TRI_F2)])
def test_zero_padded_width(lib, variant, vid):
    # k = 5 run as k = 8 with three zero columns: the first five columns follow
    # the oracle's k = 5 iteration, the padding stays zero, and the residual is
    # that of the five columns
    from paper_2305_10356_amd import graphs, ofm
    g, x0 = graphs.workload("sbm-n1000-k8")
    lap = ofm.Laplacian(g.row_ptr, g.col_idx)
    olap = O.laplacian(g.n, g.row_ptr, g.col_idx)
    x5 = x0[:, :5].copy()
    xp = np.zeros((g.n, 8))
    xp[:, :5] = x5
    ws = ofm.Workspace(lap, 8, variant=variant, precision=ofm.OFM_FP64, check_every=1000000)
    X = torch.as_tensor(xp).cuda()
    ws.init(X)
    st, _ = O.init(olap, x5, O.Options(variant=vid))
    for _ in range(12):
        ws.step(X)
        st, _ = O.step(olap, st, O.Options(variant=vid))
    Xh = host(X)
    assert np.all(Xh[:, 5:] == 0.0)
    err = np.abs(Xh[:, :5] - st.X).max() / np.abs(st.X).max()
    assert err < 1e-10, err
    r = ws.residual(X)
    assert r["status"] == 0
    assert r["relres"] == pytest.approx(O.relres(olap, st.X), rel=1e-6)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("variant,recur", [("f1", False), ("f2", False), ("tri-f2", False),
                                           ("f1", True)])
def test_hot_cold_gathers_are_bitwise_default(lib, prec, variant, recur):
    """The gather policy changes only how rows are cached: the iterates, step
    scalars and residuals with the hot/cold policy equal those with the default
    policy bit for bit (power-law graph, so many columns carry the cold mark;
    residual steps included)."""
    from paper_2305_10356_amd import graphs, ofm
    g, x0 = graphs.workload("dcsbm-n2m-k32", n=30000)
    lap = ofm.Laplacian(g.row_ptr, g.col_idx)
    p = ofm.OFM_FP64 if prec == "fp64" else ofm.OFM_FP32
    dt = torch.float64 if prec == "fp64" else torch.float32
    out = []
    for gather in (ofm.GATHER_DEFAULT, ofm.GATHER_HOT_COLD):
        ws = ofm.Workspace(lap, 32, variant=variant, precision=p, check_every=4, max_iter=13,
                           tol=1e-12, recur=recur, restart=variant.startswith("tri"),
                           gather=gather)
        X = torch.as_tensor(x0, dtype=dt).cuda()
        st = ws.solve(X)
        assert st["gather"] == gather
        out.append((host(X), st["relres"], ws.step_info()["alpha"]))
        ws.close()
    say(f"hot/cold vs default {variant} {prec} recur={recur}: relres {out[0][1]:.3e}")
    np.testing.assert_array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]
    np.testing.assert_array_equal(out[0][2], out[1][2])


def test_gather_policy_choice_and_refusals(lib):
    from paper_2305_10356_amd import graphs, ofm
    g, x0 = graphs.workload("dcsbm-n2m-k32", n=30000)
    lap = ofm.Laplacian(g.row_ptr, g.col_idx)
    # a block far below the size where the policy is timed keeps the default
    ws = ofm.Workspace(lap, 32, precision=ofm.OFM_FP32, max_iter=3)
    X = torch.as_tensor(x0, dtype=torch.float32).cuda()
    assert ws.solve(X)["gather"] == ofm.GATHER_DEFAULT
    ws.close()
    with pytest.raises(ofm.OfmError) as e:
        ofm.Workspace(lap, 32, precision=ofm.OFM_FP32, gather=3)
    assert e.value.status == -1
    with pytest.raises(ofm.OfmError) as e:
        ofm.Workspace(lap, 32, precision=ofm.OFM_FP32_BF16X, gather=ofm.GATHER_HOT_COLD)
    assert e.value.status == -8
