"""Pins of the oracle's Laplacian and shifted operator against closed forms
(Introduction, eq. (1): L = I - D^{-1/2} S D^{-1/2}, spectrum in [0, 2],
smallest eigenvalue 0; A = L - 2I)."""
import numpy as np
import pytest

from oracle import ofm_oracle as O
from paper_2305_10356_amd import graphs


def csr_from_edges(n, edges):
    rows, cols = [], []
    for a, b in edges:
        rows += [a, b]
        cols += [b, a]
    order = np.lexsort((cols, rows))
    rows = np.asarray(rows)[order]
    cols = np.asarray(cols)[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp), cols


def cycle(n):
    return csr_from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def complete(n):
    return csr_from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def cliques(c, m):
    e = []
    for b in range(c):
        e += [(b * m + i, b * m + j) for i in range(m) for j in range(i + 1, m)]
    return csr_from_edges(c * m, e)


@pytest.mark.parametrize("n", [5, 8, 13])
def test_cycle_spectrum_closed_form(n):
    lap = O.laplacian(n, *cycle(n))
    w = np.linalg.eigvalsh(O.dense_L(lap))
    expect = np.sort(1.0 - np.cos(2 * np.pi * np.arange(n) / n))
    np.testing.assert_allclose(w, expect, atol=1e-13)


def test_cycle_fourier_modes_apply_A():
    n = 12
    lap = O.laplacian(n, *cycle(n))
    i = np.arange(n)
    for j in range(n):
        u = np.cos(2 * np.pi * j * i / n)
        # 2-regular: A u = (-1 - cos(2 pi j / n)) u
        np.testing.assert_allclose(O.apply_A(lap, u[:, None])[:, 0],
                                   (-1.0 - np.cos(2 * np.pi * j / n)) * u, atol=1e-13)


@pytest.mark.parametrize("n", [3, 6, 9])
def test_complete_graph_spectrum(n):
    lap = O.laplacian(n, *complete(n))
    w = np.linalg.eigvalsh(O.dense_L(lap))
    np.testing.assert_allclose(w[0], 0.0, atol=1e-13)
    np.testing.assert_allclose(w[1:], n / (n - 1.0), atol=1e-13)


def test_disjoint_cliques_zero_multiplicity():
    lap = O.laplacian(20, *cliques(4, 5))
    w = np.linalg.eigvalsh(O.dense_L(lap))
    assert np.sum(np.abs(w) < 1e-12) == 4


def test_bipartite_top_eigenvalue_two():
    # even cycle is bipartite: lambda_max(L) = 2, i.e. A has eigenvalue 0
    lap = O.laplacian(10, *cycle(10))
    w = np.linalg.eigvalsh(O.dense_L(lap))
    np.testing.assert_allclose(w[-1], 2.0, atol=1e-13)
    lap = O.laplacian(9, *cycle(9))  # odd cycle: not bipartite
    assert np.linalg.eigvalsh(O.dense_L(lap))[-1] < 2.0 - 1e-3


def test_sbm_invariants():
    g, _ = graphs.workload("sbm-n1000-k8")
    lap = O.laplacian(g.n, g.row_ptr, g.col_idx)
    L = O.dense_L(lap)
    d = g.degrees().astype(float)
    # L D^{1/2} 1 = 0
    np.testing.assert_allclose(L @ np.sqrt(d), 0.0, atol=1e-12)
    w = np.linalg.eigvalsh(L)
    assert w[0] > -1e-12 and w[-1] < 2.0 + 1e-12
    np.testing.assert_allclose(np.trace(L), g.n, atol=1e-9)
    # A D^{1/2} 1 = -2 D^{1/2} 1 through the sparse operator
    v = np.sqrt(d)[:, None]
    np.testing.assert_allclose(O.apply_A(lap, v), -2.0 * v, atol=1e-12)


def test_regular_graph_norm_A():
    # d-regular: A = -I - S/d, ||A||_F^2 = N (1 + 1/d)
    for n in (7, 10):
        lap = O.laplacian(n, *cycle(n))
        np.testing.assert_allclose(O.norm_A_fro_sq(lap), n * 1.5, rtol=1e-14)
    lap = O.laplacian(6, *complete(6))
    np.testing.assert_allclose(O.norm_A_fro_sq(lap), 6 * (1 + 1 / 5.0), rtol=1e-14)


def test_isolated_node_rejected():
    rp, ci = cycle(5)
    rp = np.concatenate([rp, [rp[-1]]])
    with pytest.raises(O.GraphError):
        O.laplacian(6, rp, ci)


def test_weighted_degrees():
    # weights enter the degrees: a path 0-1-2 with weights 2 and 3
    rp = np.array([0, 1, 3, 4])
    ci = np.array([1, 0, 2, 1])
    vals = np.array([2.0, 2.0, 3.0, 3.0])
    lap = O.laplacian(3, rp, ci, vals)
    np.testing.assert_allclose(lap.d, [2.0, 5.0, 3.0])
    L = O.dense_L(lap)
    np.testing.assert_allclose(L[0, 1], -2.0 / np.sqrt(2.0 * 5.0))


def cycle_with_loops(n):
    """C_n plus a self-loop at every node (the diagonal entry stored once)."""
    rp, ci = cycle(n)
    rows = np.repeat(np.arange(n), np.diff(rp))
    rows = np.concatenate([rows, np.arange(n)])
    cols = np.concatenate([ci, np.arange(n)])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp), cols


@pytest.mark.parametrize("w", [1.0, 0.5, 3.0])
@pytest.mark.parametrize("n", [6, 11])
def test_self_loop_cycle_closed_forms(n, w):
    # S = adjacency(C_n) + w I is (2 + w)-regular: D = (2 + w) I,
    # A = -I - S / (2 + w), so ||A||_F^2 = n (1 + w/(2+w))^2 + 2n/(2+w)^2 and the
    # spectrum of L is 1 - (w + 2 cos(2 pi j / n)) / (2 + w)
    rp, ci = cycle_with_loops(n)
    vals = np.where(ci == np.repeat(np.arange(n), np.diff(rp)), w, 1.0)
    lap = O.laplacian(n, rp, ci, None if w == 1.0 else vals)
    d = 2.0 + w
    np.testing.assert_allclose(lap.d, d)
    expect = n * (1.0 + w / d) ** 2 + 2.0 * n / d ** 2
    np.testing.assert_allclose(O.norm_A_fro_sq(lap), expect, rtol=1e-14)
    mus = np.sort(1.0 - (w + 2.0 * np.cos(2 * np.pi * np.arange(n) / n)) / d)
    np.testing.assert_allclose(np.linalg.eigvalsh(O.dense_L(lap)), mus, atol=1e-13)
    i = np.arange(n)
    for j in range(n):
        u = np.cos(2 * np.pi * j * i / n)
        lam = -1.0 - (w + 2.0 * np.cos(2 * np.pi * j / n)) / d
        np.testing.assert_allclose(O.apply_A(lap, u[:, None])[:, 0], lam * u, atol=1e-13)
