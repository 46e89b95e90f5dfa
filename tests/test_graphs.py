"""Checks of the seeded synthetic graph generators."""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from paper_2305_10356_amd import graphs


def check_simple_symmetric_connected(g):
    n = g.n
    rp, ci = g.row_ptr.astype(np.int64), g.col_idx.astype(np.int64)
    assert rp[0] == 0 and rp[-1] == ci.shape[0]
    S = sp.csr_matrix((np.ones(ci.shape[0]), ci, rp), shape=(n, n))
    assert (S != S.T).nnz == 0
    assert S.diagonal().sum() == 0
    assert S.max() == 1.0
    for i in range(0, n, max(1, n // 50)):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)
    assert g.degrees().min() >= 1
    assert connected_components(S, directed=False)[0] == 1


def test_config1_reproducible_and_valid():
    g1, x1 = graphs.workload("sbm-n1000-k8")
    g2, x2 = graphs.workload("sbm-n1000-k8")
    assert np.array_equal(g1.col_idx, g2.col_idx) and np.array_equal(x1, x2)
    check_simple_symmetric_connected(g1)
    s = g1.stats()
    assert s["n"] == 1000 and abs(s["mean_degree"] - 16) < 1.0
    assert abs(s["realized_r"] - 0.3) < 0.05
    assert min(g1.meta["sizes"]) >= 50
    np.testing.assert_allclose(x1, np.random.default_rng(0).standard_normal((1000, 8)) / np.sqrt(1000))


def test_config2_stats():
    g, x = graphs.workload("sbm-n50k-k32")
    check_simple_symmetric_connected(g)
    s = g.stats()
    assert abs(s["mean_degree"] - 20) < 0.5 and abs(s["realized_r"] - 0.4) < 0.03
    assert x.shape == (50000, 32)


def test_dcsbm_small_heavy_tail():
    g, _ = graphs.workload("dcsbm-n2m-k32", n=64000)
    check_simple_symmetric_connected(g)
    s = g.stats()
    assert 22 < s["mean_degree"] <= 25.5
    assert abs(s["realized_r"] - 0.5) < 0.05
    assert s["max_degree"] > 5 * s["mean_degree"]


def test_node_order_hides_blocks():
    g, _ = graphs.workload("sbm-n50k-k32")
    # consecutive ids are not in the same block more often than chance
    same = np.mean(g.labels[1:] == g.labels[:-1])
    assert same < 0.1


def test_bfs_ball():
    g, _ = graphs.workload("sbm-n50k-k32")
    sub = graphs.bfs_ball_subgraph(g, 500, np.random.default_rng(9))
    assert sub.n == 500
    check_simple_symmetric_connected(sub)


def test_batched_specs():
    specs = graphs.batched_graph_specs(256)
    assert len(specs) == 256
    assert all(1000 <= s["n"] <= 50000 and s["k"] in (4, 8, 16, 32) and 8 <= s["dbar"] <= 32
               for s in specs)
    g, x = graphs.batched_graph(specs[0])
    check_simple_symmetric_connected(g)
    assert x.shape == (specs[0]["n"], specs[0]["k"])


def test_growth_stream_structure():
    gs = graphs.GrowthStream(n_final=20000, stages=4, k=16, dbar=20, r=0.3, seed=11)
    m = gs.m
    prev = None
    for s in range(gs.stages):
        g = gs.snapshot(s)
        assert g.n == gs.bounds[s]
        check_simple_symmetric_connected(g)
        rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        earlier = np.bincount(rows[g.col_idx < rows], minlength=g.n)
        # the clique, then exactly m distinct earlier neighbours per arrival
        np.testing.assert_array_equal(earlier[: m + 1], np.arange(m + 1))
        assert np.all(earlier[m + 1:] == m)
        assert g.degrees().min() >= m
        if prev is not None:
            # the previous snapshot is the subgraph induced by its node ids
            keep = (rows < prev.n) & (g.col_idx < prev.n)
            np.testing.assert_array_equal(g.col_idx[keep], prev.col_idx)
            np.testing.assert_array_equal(np.bincount(rows[keep], minlength=prev.n),
                                          prev.degrees())
        prev = g
    st = prev.stats()
    assert abs(st["mean_degree"] - 20) < 0.1
    assert abs(st["realized_r"] - 0.3) < 0.04
    # same seed, same stream
    again = graphs.GrowthStream(n_final=20000, stages=4, k=16, dbar=20, r=0.3, seed=11)
    np.testing.assert_array_equal(again.col_idx, gs.col_idx)


def test_growth_stream_arrival_order_hides_blocks():
    gs = graphs.GrowthStream(n_final=30000, stages=2, k=32, seed=3)
    counts = np.bincount(gs.labels, minlength=32)
    assert counts.min() > 0.8 * 30000 / 32
    assert np.mean(gs.labels[1:] == gs.labels[:-1]) < 0.1


def test_warm_start_rows():
    rng = np.random.default_rng(1)
    old = rng.standard_normal((100, 4))
    x = graphs.warm_start(old, 5000, 4, np.random.default_rng(2))
    np.testing.assert_array_equal(x[:100], old)
    assert abs(x[100:].var() * 5000 - 1.0) < 0.05


def test_relabel_is_an_isomorphism():
    from paper_2305_10356_amd import graphs as G
    g, _ = G.workload("sbm-n1000-k8")
    for order in (G.hub_first_order(g), G.rcm_order(g),
                  np.random.default_rng(3).permutation(g.n)):
        h = G.relabel(g, order)
        assert h.n == g.n and h.nnz == g.nnz
        inv = np.empty(g.n, dtype=np.int64)
        inv[order] = np.arange(g.n)
        # every edge (u, v) of g is the edge (inv u, inv v) of h, and back
        rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        e_g = set(zip(inv[rows].tolist(), inv[g.col_idx].tolist()))
        rows_h = np.repeat(np.arange(h.n), np.diff(h.row_ptr))
        e_h = set(zip(rows_h.tolist(), h.col_idx.tolist()))
        assert e_g == e_h
        for i in range(h.n):
            c = h.col_idx[h.row_ptr[i]:h.row_ptr[i + 1]]
            assert np.all(np.diff(c) > 0)
        assert np.array_equal(h.labels, g.labels[order])
    deg = np.diff(G.relabel(g, G.hub_first_order(g)).row_ptr)
    assert np.all(np.diff(deg) <= 0)


def test_edge_stream_stages_are_nested_partitions():
    from paper_2305_10356_amd import graphs as G
    g, _ = G.workload("sbm-n1000-k8")
    es = G.EdgeStream(g, parts=10, seed=3)
    full = set()
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    for a, b in zip(rows.tolist(), g.col_idx.tolist()):
        if a < b:
            full.add((a, b))
    prev_ids, prev_edges = None, set()
    sizes = []
    for s in range(10):
        h, ids = es.stage(s)
        assert np.all(np.diff(ids) > 0) and h.n == ids.shape[0]
        assert np.all(np.diff(h.row_ptr) >= 1)            # every node has an edge
        assert np.array_equal(h.labels, g.labels[ids])
        r = np.repeat(np.arange(h.n), np.diff(h.row_ptr))
        edges = {(int(ids[a]), int(ids[b])) for a, b in zip(r, h.col_idx) if a < b}
        assert all(np.diff(h.col_idx[h.row_ptr[i]:h.row_ptr[i + 1]]).min(initial=1) > 0
                   for i in range(h.n))
        # symmetric pattern, a subset of the graph, growing
        assert edges <= full and prev_edges <= edges
        assert len(edges) * 2 == h.nnz
        if prev_ids is not None:
            pos = G.EdgeStream.carry(prev_ids, ids)
            assert np.array_equal(ids[pos], prev_ids)
        sizes.append(len(edges) - len(prev_edges))
        prev_ids, prev_edges = ids, edges
    assert prev_edges == full
    # ten parts of about a tenth each
    assert min(sizes) > 0.06 * len(full) and max(sizes) < 0.14 * len(full)
