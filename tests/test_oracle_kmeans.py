"""Pins of the oracle's post-processing (Algorithm 1 steps 4-5) and of the
evaluation indices (numerical results section, "Evaluation metrics")."""
import numpy as np
import pytest

from oracle import ofm_oracle as O


def test_ari_nmi_against_scikit_learn():
    metrics = pytest.importorskip("sklearn.metrics")
    rng = np.random.default_rng(2)
    for _ in range(20):
        a = rng.integers(0, 5, size=300)
        b = np.where(rng.random(300) < 0.6, a, rng.integers(0, 6, size=300))
        assert O.ari(a, b) == pytest.approx(metrics.adjusted_rand_score(a, b), abs=1e-12)
        assert O.nmi(a, b) == pytest.approx(
            metrics.normalized_mutual_info_score(a, b, average_method="arithmetic"), abs=1e-12)


def test_ari_nmi_identities():
    a = np.array([0, 0, 1, 1, 2, 2])
    perm = np.array([2, 2, 0, 0, 1, 1])
    assert O.ari(a, perm) == pytest.approx(1.0)
    assert O.nmi(a, perm) == pytest.approx(1.0)


def test_row_normalize():
    X = np.array([[3.0, 4.0], [0.0, 0.0], [-1.0, 0.0]])
    np.testing.assert_allclose(O.row_normalize(X), [[0.6, 0.8], [0, 0], [-1, 0]])


def test_kmeans_assign_brute_force_and_ties():
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((50, 3))
    C = rng.standard_normal((4, 3))
    lab, d2 = O.kmeans_assign(Y, C)
    for i in range(50):
        dd = [sum((Y[i, d] - C[c, d]) ** 2 for d in range(3)) for c in range(4)]
        assert lab[i] == int(np.argmin(dd))
        assert d2[i] == pytest.approx(min(dd))
    # equidistant point goes to the lowest index
    lab, _ = O.kmeans_assign(np.array([[0.0, 0.0]]), np.array([[1.0, 0.0], [-1.0, 0.0]]))
    assert lab[0] == 0


def test_lloyd_recovers_separated_blobs():
    rng = np.random.default_rng(3)
    centers = np.eye(4) * 10
    truth = rng.integers(0, 4, size=400)
    Y = centers[truth] + 0.3 * rng.standard_normal((400, 4))
    lab, C, it = O.kmeans(Y, 4, seed=0)
    assert O.ari(lab, truth) == pytest.approx(1.0)
    assert it < 300


def test_kmeanspp_uses_given_uniforms():
    Y = np.arange(10, dtype=float)[:, None]
    C = O.kmeanspp_init(Y, 2, np.array([0.0, 0.999999]))
    assert C[0, 0] == 0.0 and C[1, 0] == 9.0
