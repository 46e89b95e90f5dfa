"""Pins of the oracle's exact line search (Section 3.2: eqs. f1-derivative,
alphai-f1, f2-derivative, alphai-f2 and the root rules) and of the
column-wise Polak-Ribiere update of Algorithm 2."""
import json
import os

import numpy as np
import pytest

from oracle import ofm_oracle as O
from paper_2305_10356_amd import graphs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def state():
    g, _ = graphs.workload("sbm-n1000-k8", n=150)
    lap = O.laplacian(g.n, g.row_ptr, g.col_idx)
    A = O.dense_A(lap)
    rng = np.random.default_rng(21)
    X = rng.standard_normal((g.n, 5)) * 0.2
    V = rng.standard_normal((g.n, 5)) * 0.1
    return lap, A, X, V


def coeffs_for(variant, lap, X, V):
    AX = O.apply_A(lap, X)
    G = O.direction(variant, X, AX)
    M, H, C, P, E, F, vg = O._grams(lap, X, AX, V, G)
    return O.linesearch_coeffs(variant, M, H, C, P, E, F, vg)


ALPHAS = np.linspace(-1.5, 1.5, 9)


def test_f1_cubic_is_quarter_derivative_of_definition(state):
    lap, A, X, V = state
    co = coeffs_for(O.F1, lap, X, V)
    vals = [O.f1_dense(A, X + a * V) for a in ALPHAS]
    quartic = np.polyfit(ALPHAS, vals, 4)
    deriv = np.polyder(quartic)  # 4 a^3, 3 a^2, 2 a, 1 coefficients
    np.testing.assert_allclose(co, deriv / 4.0, rtol=1e-7, atol=1e-9 * np.abs(deriv).max())


def test_f2_cubic_is_derivative_of_definition(state):
    lap, A, X, V = state
    co = coeffs_for(O.F2, lap, X, V)
    vals = [O.f2_dense(A, X + a * V) for a in ALPHAS]
    deriv = np.polyder(np.polyfit(ALPHAS, vals, 4))
    np.testing.assert_allclose(co, deriv, rtol=1e-7, atol=1e-9 * np.abs(deriv).max())


@pytest.mark.parametrize("variant", [O.TRI_F1, O.TRI_F2])
def test_tri_cubic_is_column_of_direction(state, variant):
    lap, A, X, V = state
    co = coeffs_for(variant, lap, X, V)
    # [V^T g(X + a V)]_ii straight from the direction, every column moved by a
    vals = np.array([np.sum(V * O.direction(variant, X + a * V, A @ (X + a * V)), axis=0)
                     for a in ALPHAS])
    for i in range(X.shape[1]):
        fit = np.polyfit(ALPHAS, vals[:, i], 3)
        np.testing.assert_allclose(co[:, i], fit, rtol=1e-7, atol=1e-9 * np.abs(fit).max())


def test_a0_dot_equals_printed_trace_form(state):
    lap, A, X, V = state
    AX = O.apply_A(lap, X)
    M, H, C, P, E, F, vg = O._grams(lap, X, AX, V, O.direction(O.F1, X, AX))
    # printed constant term: tr(V^T A X) + tr(V^T X X^T X)
    np.testing.assert_allclose(np.sum(vg) / 4.0, np.trace(E) + np.trace(C.T @ M), rtol=1e-12)
    M, H, C, P, E, F, vg = O._grams(lap, X, AX, V, O.direction(O.F2, X, AX))
    np.testing.assert_allclose(np.sum(vg), 2 * (2 * np.trace(E.T) - np.trace(C.T @ H)
                                                - np.trace(M @ E.T)), rtol=1e-12)


def test_k1_tri_and_ofm_cubics_coincide(state):
    lap, A, X, V = state
    x, v = X[:, :1], V[:, :1]
    np.testing.assert_allclose(coeffs_for(O.TRI_F1, lap, x, v)[:, 0], coeffs_for(O.F1, lap, x, v),
                               rtol=1e-12)
    np.testing.assert_allclose(coeffs_for(O.TRI_F2, lap, x, v)[:, 0], coeffs_for(O.F2, lap, x, v) / 2,
                               rtol=1e-12)


def test_cubic_roots_against_companion_eigenvalues():
    rng = np.random.default_rng(4)
    for _ in range(300):
        c = rng.standard_normal(4) * np.exp(rng.uniform(-3, 3))
        got = sorted(r for r, _ in O.cubic_real_roots(*c))
        ref = np.roots(c)
        ref = sorted(r.real for r in ref if abs(r.imag) <= 1e-9 * max(1.0, abs(r)))
        assert len(got) == len(ref)
        np.testing.assert_allclose(got, ref, rtol=1e-8, atol=1e-10)


def test_cubic_golden_cases():
    data = json.load(open(os.path.join(GOLDEN, "cubics.json")))
    for case in data["cases"]:
        roots = sorted(r for r, _ in O.cubic_real_roots(*case["coeffs"]))
        np.testing.assert_allclose(roots, case["roots"], atol=1e-9)
        assert O.select_root(O.F1, case["coeffs"])[0] == pytest.approx(case["ofm"], abs=1e-9)
        assert O.select_root(O.TRI_F1, case["coeffs"])[0] == pytest.approx(case["tri"], abs=1e-9)


@pytest.mark.parametrize("variant,fdef", [(O.F1, O.f1_dense), (O.F2, O.f2_dense)])
def test_ofm_step_is_global_line_minimum(state, variant, fdef):
    lap, A, X, V = state
    AX = O.apply_A(lap, X)
    G = O.direction(variant, X, AX)
    for Vd in (V, -G):
        alpha, co, _ = O.step_size(variant, lap, X, AX, Vd, G)
        a = alpha[0]
        fa = fdef(A, X + a * Vd)
        grid = np.linspace(-4 * abs(a) - 1, 4 * abs(a) + 1, 801)
        fg = np.array([fdef(A, X + t * Vd) for t in grid])
        assert fa <= fg.min() + 1e-10 * abs(fg).max()


def test_beta_hand_worked():
    d = json.load(open(os.path.join(GOLDEN, "beta_hand.json")))
    G = np.array(d["G"])
    Gp = np.array(d["G_prev"])
    beta = O.pr_beta(G, Gp)
    np.testing.assert_allclose(beta, d["beta"], rtol=1e-15)
    np.testing.assert_allclose(-G + np.array(d["V_prev"]) * beta[None, :], d["V"], rtol=1e-14)
    # a zero previous column gives beta = 0
    Gp0 = Gp.copy()
    Gp0[:, 1] = 0.0
    assert O.pr_beta(G, Gp0)[1] == 0.0


def test_exact_line_search_orthogonality(state):
    # after an exact OFM step the new gradient is orthogonal to the direction
    lap, A, X, V = state
    for variant in (O.F1, O.F2):
        AX = O.apply_A(lap, X)
        G = O.direction(variant, X, AX)
        alpha, _, _ = O.step_size(variant, lap, X, AX, -G, G)
        Xn = X - alpha[0] * G
        Gn = O.direction(variant, Xn, O.apply_A(lap, Xn))
        assert abs(np.sum(G * Gn)) < 1e-9 * np.linalg.norm(G) * np.linalg.norm(Gn)
    # triangular: per column, [V^T g(X + a_i V)]_ii = 0 at the chosen a_i
    for variant in (O.TRI_F1, O.TRI_F2):
        AX = O.apply_A(lap, X)
        G = O.direction(variant, X, AX)
        alpha, _, _ = O.step_size(variant, lap, X, AX, -G, G)
        for i in range(X.shape[1]):
            Xi = X - alpha[i] * G
            gi = O.direction(variant, Xi, A @ Xi)
            assert abs(np.sum(G[:, i] * gi[:, i])) < 1e-9 * np.linalg.norm(G[:, i]) ** 2
