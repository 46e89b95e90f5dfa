"""Pins of the oracle's objectives and directions (Section 2: eqs.
gradientf1, gradientg1, gradientf2, gradientg2; Theorems 1-4)."""
import numpy as np
import pytest

from oracle import ofm_oracle as O
from paper_2305_10356_amd import graphs


@pytest.fixture(scope="module")
def small():
    g, _ = graphs.workload("sbm-n1000-k8", n=120)
    lap = O.laplacian(g.n, g.row_ptr, g.col_idx)
    A = O.dense_A(lap)
    rng = np.random.default_rng(11)
    X = rng.standard_normal((g.n, 4)) * 0.3
    return lap, A, X


def fd_grad(f, X, h):
    G = np.zeros_like(X)
    for idx in np.ndindex(*X.shape):
        E = np.zeros_like(X)
        E[idx] = h
        G[idx] = (f(X + E) - f(X - E)) / (2 * h)
    return G


def test_grad_f1_finite_difference(small):
    lap, A, X = small
    AX = O.apply_A(lap, X)
    G = O.direction(O.F1, X, AX)
    G_fd = fd_grad(lambda Z: O.f1_dense(A, Z), X, 1e-5)
    np.testing.assert_allclose(G, G_fd, rtol=0, atol=1e-6 * np.abs(G).max())


def test_grad_f2_finite_difference(small):
    lap, A, X = small
    AX = O.apply_A(lap, X)
    G = O.direction(O.F2, X, AX)
    G_fd = fd_grad(lambda Z: O.f2_dense(A, Z), X, 1e-5)
    np.testing.assert_allclose(G, G_fd, rtol=0, atol=1e-6 * np.abs(G).max())


def test_objective_gram_forms_match_definitions(small):
    lap, A, X = small
    np.testing.assert_allclose(O.objective(O.F1, lap, X), O.f1_dense(A, X), rtol=1e-12)
    np.testing.assert_allclose(O.objective(O.F2, lap, X), O.f2_dense(A, X), rtol=1e-12)


def test_g1_equals_quarter_grad_when_gram_diagonal(small):
    lap, A, X = small
    Q, _ = np.linalg.qr(X)
    Xo = Q * np.array([0.3, 1.1, 0.7, 2.0])[None, :]
    AX = O.apply_A(lap, Xo)
    np.testing.assert_allclose(O.direction(O.TRI_F1, Xo, AX),
                               O.direction(O.F1, Xo, AX) / 4.0, atol=1e-12)


def test_g2_equals_half_grad_when_grams_diagonal(small):
    lap, A, X = small
    w, U = np.linalg.eigh(A)
    Xe = U[:, [0, 3, 5, 9]] * np.array([0.5, 1.2, 0.9, 1.7])[None, :]
    AX = O.apply_A(lap, Xe)
    np.testing.assert_allclose(O.direction(O.TRI_F2, Xe, AX),
                               O.direction(O.F2, Xe, AX) / 2.0, atol=1e-12)
    # and the off-diagonal case differs (the triu matters)
    AX = O.apply_A(lap, X)
    assert np.abs(O.direction(O.TRI_F2, X, AX) - O.direction(O.F2, X, AX) / 2).max() > 1e-3


@pytest.mark.parametrize("variant", [O.TRI_F1, O.TRI_F2])
def test_triangular_dependence(small, variant):
    lap, A, X = small
    AX = O.apply_A(lap, X)
    G = O.direction(variant, X, AX)
    rng = np.random.default_rng(3)
    for j in range(X.shape[1]):
        Xp = X.copy()
        Xp[:, j] += 0.1 * rng.standard_normal(X.shape[0])
        Gp = O.direction(variant, Xp, O.apply_A(lap, Xp))
        for i in range(X.shape[1]):
            diff = np.abs(Gp[:, i] - G[:, i]).max()
            if i < j:
                assert diff < 1e-14, (i, j)
            else:
                assert diff > 1e-6, (i, j)


def test_fixed_points_theorems(small):
    lap, A, X = small
    w, U = np.linalg.eigh(A)
    k = 4
    Uk, lk = U[:, :k], w[:k]
    Xf1 = Uk * np.sqrt(-lk)[None, :]
    for v in (O.F1, O.TRI_F1):
        G = O.direction(v, Xf1, O.apply_A(lap, Xf1))
        assert np.abs(G).max() < 1e-12
    # any rotation keeps a minimum of f1 (Theorem 1); not a fixed point of g1
    Q, _ = np.linalg.qr(np.random.default_rng(5).standard_normal((k, k)))
    Xr = Xf1 @ Q
    assert np.abs(O.direction(O.F1, Xr, O.apply_A(lap, Xr))).max() < 1e-12
    assert np.abs(O.direction(O.TRI_F1, Xr, O.apply_A(lap, Xr))).max() > 1e-3
    for v in (O.F2, O.TRI_F2):
        G = O.direction(v, Uk, O.apply_A(lap, Uk))
        assert np.abs(G).max() < 1e-12
    assert np.abs(O.direction(O.F2, Uk @ Q, O.apply_A(lap, Uk @ Q))).max() < 1e-12
    # minimum values: f1 = sum_{i>k} lambda_i^2, f2 = sum_{i<=k} lambda_i
    np.testing.assert_allclose(O.f1_dense(A, Xf1), np.sum(w[k:] ** 2), rtol=1e-10)
    np.testing.assert_allclose(O.f2_dense(A, Uk), np.sum(lk), rtol=1e-12)
