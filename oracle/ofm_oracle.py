"""FP64 CPU oracle for orthogonalization-free spectral clustering.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the test suite, the package smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library; it is a plain, slow, obviously-correct restatement of the paper
(Pang & Yang, "Spectral clustering via orthogonalization-free methods",
arXiv 2305.10356) in NumPy/SciPy, FP64 throughout.

What it computes, and where the paper defines it
-------------------------------------------------
* Symmetric normalized Laplacian L = I - D^{-1/2} S D^{-1/2} and the shifted
  matrix A = L - 2I (Introduction, eq. (1); Algorithm 1, step 2).
* Objectives f1(X) = ||A + X X^T||_F^2 and f2(X) = tr((2I - X^T X) X^T A X)
  (Introduction, the two unconstrained problems; Section 2.1 and 2.2).
* Directions: grad f1 = 4AX + 4X X^T X (eq. gradientf1);
  g1 = AX + X triu(X^T X) (eq. gradientg1);
  grad f2 = 4AX - 2X X^T A X - 2AX X^T X (eq. gradientf2);
  g2 = 2AX - AX triu(X^T X) - X triu(X^T A X) (eq. gradientg2).
* Exact line search: the cubic coefficients of Section 3.2
  (eqs. f1-derivative, alphai-f1, f2-derivative, alphai-f2), real roots by
  Cardano's formula / the trigonometric form, and the root rules of
  Section 3.2 (one real root: it; two: the simple one; three: the one of
  least objective value).
* Algorithm 2 (orthogonalization-free framework): column-wise Polak-Ribiere
  beta, V_i = -G_i + beta_i V_i^prev, per-column or scalar step, update.
* The relative residual used as stopping test (numerical results section,
  "Evaluation metrics": Ritz pairs of A on span(X)).
* Post-processing of Algorithm 1 (steps 4-5): row normalisation, Euclidean
  K-means (assignment, Lloyd iterations, k-means++ seeding), ARI and NMI.
* Dense eigendecomposition of L for the limit checks (Theorems 1-4).

Readings taken where the paper is silent or garbled
----------------------------------------------------
* Triangular variants: the per-column cubic is [V^T g(X + a_i V)]_ii, i.e.
  column i of g with every column moved by a_i; this reproduces the printed
  coefficients exactly (eqs. alphai-f1 / alphai-f2 are written with V_i, X_i
  but contain traces and triu of k x k products).
* Triangular variants: g1, g2 are not gradients, so "least objective value"
  is undefined; with three real roots the root of smallest |a| is taken.
* First step (Algorithm 2, the update before the loop): exact line search by
  default; ``first_step="fixed"`` uses the given alpha0 (the literal reading).
* Polak-Ribiere beta as printed, no clamp, beta_i = 0 when the previous
  column norm is zero.  An optional descent restart (``restart=True``,
  beta_i := 0 when <V_i, G_i> >= 0) is a safeguard outside Algorithm 2; it is
  off by default.
* OFM-f1 cubic: the printed polynomial is (1/4) d/da f1; a0 is evaluated
  as <V, grad f1(X)>/4 (equal to tr(V^T A X) + tr(V^T X X^T X)); for the
  other variants a0 = <V, G> as well.  Roots are scale-invariant.
* Cubic solve: normalise by a3, depress, classify with a relative
  tolerance of 1e-12, two Newton polish steps on the original cubic; a3 = 0
  falls back to the quadratic / linear; no real root gives a = 0.
* Residual: relres = ||A U - U Lam||_F / ||U Lam||_F with (Lam, U) the Ritz
  pairs of A itself on span(X).
* Iterating past convergence: Algorithm 2 runs a fixed t_max.  An optional
  freeze (``freeze_eps > 0``) skips a step (every step size 0) whose direction
  satisfies ||G||_F <= freeze_eps ||X||_F, so a converged X stays put.
* A line search whose polynomial is not identically zero but has no real
  root takes step 0 and is flagged (``no_root`` in the step info).

Parity pins for every function live in tests/test_oracle_*.py.  Iterate
values of long runs have no printed worked example in the paper: they are
pinned only through the per-step pins, the limits of Theorems 1-4 and the
planted-partition recovery ("parity unpinned" for free-running trajectories).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional, Tuple

import numpy as np
import scipy.sparse as sp

F1, TRI_F1, F2, TRI_F2 = 0, 1, 2, 3
VARIANT_NAMES = {F1: "OFM-f1", TRI_F1: "TriOFM-f1", F2: "OFM-f2", TRI_F2: "TriOFM-f2"}


def is_tri(variant: int) -> bool:
    return variant in (TRI_F1, TRI_F2)


def is_f2(variant: int) -> bool:
    return variant in (F2, TRI_F2)


# ---------------------------------------------------------------------------
# Laplacian and the shifted operator  (Introduction, eq. (1); Algorithm 1)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Laplacian:
    n: int
    S: sp.csr_matrix          # similarity matrix (FP64 values, 1 for an edge)
    d: np.ndarray             # degrees D_ii = sum_j S_ij
    dinv: np.ndarray          # D^{-1/2}


class GraphError(ValueError):
    pass


def laplacian(n: int, row_ptr, col_idx, vals=None) -> Laplacian:
    """Degrees and D^{-1/2} of the similarity matrix S given in CSR form.

    S_ij = 1 for every stored (i, j) unless weights ``vals`` are given.  A node
    with zero degree has no D^{-1/2} and is rejected."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    if row_ptr.shape != (n + 1,) or row_ptr[0] != 0 or row_ptr[-1] != col_idx.shape[0]:
        raise GraphError("malformed CSR")
    if col_idx.shape[0] and (col_idx.min() < 0 or col_idx.max() >= n):
        raise GraphError("column index out of range")
    data = np.ones(col_idx.shape[0]) if vals is None else np.asarray(vals, dtype=np.float64)
    S = sp.csr_matrix((data, col_idx, row_ptr), shape=(n, n))
    d = np.asarray(S.sum(axis=1)).ravel()
    if np.any(d <= 0):
        raise GraphError("node with zero degree")
    return Laplacian(n=n, S=S, d=d, dinv=1.0 / np.sqrt(d))


def dense_L(lap: Laplacian) -> np.ndarray:
    """L = I - D^{-1/2} S D^{-1/2} as a dense matrix (small graphs only)."""
    Sd = lap.S.toarray()
    return np.eye(lap.n) - lap.dinv[:, None] * Sd * lap.dinv[None, :]


def dense_A(lap: Laplacian) -> np.ndarray:
    """A = L - 2I (dense, small graphs only)."""
    return dense_L(lap) - 2.0 * np.eye(lap.n)


def apply_A(lap: Laplacian, Z: np.ndarray) -> np.ndarray:
    """A Z = -Z - D^{-1/2} S D^{-1/2} Z."""
    Z = np.asarray(Z, dtype=np.float64)
    return -Z - lap.dinv[:, None] * (lap.S @ (lap.dinv[:, None] * Z))


def norm_A_fro_sq(lap: Laplacian) -> float:
    """||A||_F^2 = sum_ij (A_ij)^2 with A = -I - D^{-1/2} S D^{-1/2}."""
    S = lap.S.tocoo()
    w = S.data * lap.dinv[S.row] * lap.dinv[S.col]
    diag = np.zeros(lap.n)
    on = S.row == S.col
    np.add.at(diag, S.row[on], w[on])
    off = float(np.sum(w[~on] ** 2))
    return float(np.sum((1.0 + diag) ** 2)) + off


# ---------------------------------------------------------------------------
# Objectives and directions  (Sections 2.1, 2.2)
# ---------------------------------------------------------------------------

def objective(variant: int, lap: Laplacian, X: np.ndarray, AX: Optional[np.ndarray] = None) -> float:
    """f1 for the f1 variants, f2 for the f2 variants, via k x k products:
    f1 = ||A||_F^2 + 2 tr(X^T A X) + ||X^T X||_F^2,
    f2 = 2 tr(X^T A X) - tr(X^T X X^T A X)."""
    if AX is None:
        AX = apply_A(lap, X)
    M = X.T @ X
    H = X.T @ AX
    if is_f2(variant):
        return float(2.0 * np.trace(H) - np.trace(M @ H))
    return float(norm_A_fro_sq(lap) + 2.0 * np.trace(H) + np.sum(M * M))


def f1_dense(A: np.ndarray, X: np.ndarray) -> float:
    """f1 straight from its definition ||A + X X^T||_F^2 (dense A)."""
    R = A + X @ X.T
    return float(np.sum(R * R))


def f2_dense(A: np.ndarray, X: np.ndarray) -> float:
    """f2 straight from its definition tr((2I - X^T X) X^T A X) (dense A)."""
    k = X.shape[1]
    return float(np.trace((2.0 * np.eye(k) - X.T @ X) @ (X.T @ A @ X)))


def direction(variant: int, X: np.ndarray, AX: np.ndarray) -> np.ndarray:
    """G = g(X) for the four variants:
    OFM-f1   : 4 AX + 4 X (X^T X)
    TriOFM-f1: AX + X triu(X^T X)
    OFM-f2   : 4 AX - 2 X (X^T A X) - 2 AX (X^T X)
    TriOFM-f2: 2 AX - AX triu(X^T X) - X triu(X^T A X)."""
    M = X.T @ X
    if variant == F1:
        return 4.0 * AX + 4.0 * X @ M
    if variant == TRI_F1:
        return AX + X @ np.triu(M)
    H = X.T @ AX
    if variant == F2:
        return 4.0 * AX - 2.0 * X @ H - 2.0 * AX @ M
    if variant == TRI_F2:
        return 2.0 * AX - AX @ np.triu(M) - X @ np.triu(H)
    raise ValueError(variant)


# ---------------------------------------------------------------------------
# Exact line search  (Section 3.2)
# ---------------------------------------------------------------------------

def _diag_xu(Xm: np.ndarray, Ym: np.ndarray) -> np.ndarray:
    """Diagonal of Xm @ triu(Ym)."""
    return np.diag(Xm @ np.triu(Ym))


def linesearch_coeffs(variant: int, M, H, C, P, E, F, vg) -> np.ndarray:
    """Cubic coefficients (a3, a2, a1, a0) of the exact line search.

    M = X^T X, H = X^T A X, C = X^T V, P = V^T V, E = X^T A V, F = V^T A V,
    vg = per-column <V_i, G_i> with G = g(X).  OFM variants return shape (4,),
    triangular variants shape (4, k) (one cubic per column)."""
    Ct, Et = C.T, E.T
    if variant == F1:
        # (1/4) d/da f1(X + aV), eq. f1-derivative
        a3 = np.trace(P @ P)
        a2 = 3.0 * np.trace(P @ C)
        a1 = np.trace(F) + np.trace(Ct @ Ct) + np.trace(Ct @ C) + np.trace(P @ M)
        a0 = np.sum(vg) / 4.0
        return np.array([a3, a2, a1, a0])
    if variant == F2:
        # d/da f2(X + aV), eq. f2-derivative
        a3 = -4.0 * np.trace(P @ F)
        a2 = -6.0 * (np.trace(Ct @ F) + np.trace(P @ Et))
        a1 = 2.0 * (2.0 * np.trace(F) - 2.0 * np.trace(Ct @ E) - 2.0 * np.trace(Ct @ Et)
                    - np.trace(P @ H) - np.trace(M @ F))
        a0 = np.sum(vg)
        return np.array([a3, a2, a1, a0])
    if variant == TRI_F1:
        # [V^T g1(X + a_i V)]_ii, eq. alphai-f1
        a3 = _diag_xu(P, P)
        a2 = _diag_xu(P, C) + _diag_xu(P, Ct) + _diag_xu(Ct, P)
        a1 = np.diag(F) + _diag_xu(Ct, Ct) + _diag_xu(Ct, C) + _diag_xu(P, M)
        a0 = np.asarray(vg, dtype=np.float64).copy()
        return np.stack([a3, a2, a1, a0])
    if variant == TRI_F2:
        # [V^T g2(X + a_i V)]_ii, eq. alphai-f2
        a3 = -(_diag_xu(F, P) + _diag_xu(P, F))
        a2 = -(_diag_xu(Et, P) + _diag_xu(F, C) + _diag_xu(F, Ct)
               + _diag_xu(Ct, F) + _diag_xu(P, E) + _diag_xu(P, Et))
        a1 = (2.0 * np.diag(F) - _diag_xu(Et, C) - _diag_xu(Et, Ct) - _diag_xu(F, M)
              - _diag_xu(Ct, E) - _diag_xu(Ct, Et) - _diag_xu(P, H))
        a0 = np.asarray(vg, dtype=np.float64).copy()
        return np.stack([a3, a2, a1, a0])
    raise ValueError(variant)


CUBIC_TOL = 1e-12


def cubic_real_roots(a3: float, a2: float, a1: float, a0: float):
    """Real roots of a3 x^3 + a2 x^2 + a1 x + a0 with their multiplicity.

    Returns a list of (root, multiplicity).  Cardano's formula when the
    discriminant shows one real root, the trigonometric (Viete) form when it
    shows three, the closed form of the repeated root when it vanishes
    (relative tolerance 1e-12); two Newton steps polish every root.  a3 = 0
    falls back to the quadratic / linear equation."""
    a3, a2, a1, a0 = float(a3), float(a2), float(a1), float(a0)

    def poly(x):
        return ((a3 * x + a2) * x + a1) * x + a0

    def dpoly(x):
        return (3.0 * a3 * x + 2.0 * a2) * x + a1

    def polish(x):
        for _ in range(2):
            dp = dpoly(x)
            if dp == 0.0 or not math.isfinite(dp):
                break
            xn = x - poly(x) / dp
            if not math.isfinite(xn):
                break
            x = xn
        return x

    if a3 == 0.0:
        if a2 == 0.0:
            if a1 == 0.0:
                return []
            return [(-a0 / a1, 1)]
        disc = a1 * a1 - 4.0 * a2 * a0
        scale = max(a1 * a1, abs(4.0 * a2 * a0))
        if disc < -CUBIC_TOL * scale:
            return []
        if disc <= CUBIC_TOL * scale:
            return [(-a1 / (2.0 * a2), 2)]
        sq = math.sqrt(disc)
        # numerically stable pair
        qq = -0.5 * (a1 + math.copysign(sq, a1))
        r1 = qq / a2
        r2 = a0 / qq if qq != 0.0 else -a1 / a2 - r1
        return sorted([(r1, 1), (r2, 1)])
    b = a2 / a3
    c = a1 / a3
    d = a0 / a3
    # x = t - b/3 gives t^3 + p t + q = 0
    p = c - b * b / 3.0
    q = 2.0 * b * b * b / 27.0 - b * c / 3.0 + d
    shift = -b / 3.0
    D = q * q / 4.0 + p * p * p / 27.0
    scale = max(q * q / 4.0, abs(p * p * p / 27.0))
    if scale == 0.0:
        return [(polish(shift), 3)]
    if abs(D) <= CUBIC_TOL * scale:
        if p == 0.0:
            return [(polish(shift), 3)]
        simple = 3.0 * q / p + shift
        double = -3.0 * q / (2.0 * p) + shift
        return sorted([(polish(simple), 1), (double, 2)])
    if D > 0.0:
        sq = math.sqrt(D)
        u = np.cbrt(-q / 2.0 + sq)
        v = np.cbrt(-q / 2.0 - sq)
        return [(polish(float(u + v) + shift), 1)]
    # three distinct real roots (p < 0 here)
    m = 2.0 * math.sqrt(-p / 3.0)
    arg = 3.0 * q / (p * m)
    arg = min(1.0, max(-1.0, arg))
    th = math.acos(arg) / 3.0
    roots = [polish(m * math.cos(th - 2.0 * math.pi * j / 3.0) + shift) for j in range(3)]
    return sorted([(r, 1) for r in roots])


def select_root(variant: int, coeffs) -> Tuple[float, int]:
    """Step size from the cubic's real roots (Section 3.2 root rules).

    One real root: that root.  A simple and a repeated root: the simple one.
    Three real roots: the least objective value along the line for OFM
    (Phi(a) = a3 a^4/4 + a2 a^3/3 + a1 a^2/2 + a0 a, the line restriction of
    the objective up to a positive factor and a constant); the smallest |a|
    for the triangular variants.  No real root: 0.  Returns (alpha, nroots)."""
    a3, a2, a1, a0 = (float(x) for x in coeffs)
    roots = cubic_real_roots(a3, a2, a1, a0)
    if not roots:
        return 0.0, 0
    simple = [r for r, mlt in roots if mlt == 1]
    if len(roots) == 1:
        return float(roots[0][0]), 1
    if len(roots) == 2 and len(simple) == 1:
        return float(simple[0]), 2
    cands = [r for r, _ in roots]
    # ascending |a| then a: the first of equal candidates wins
    cands.sort(key=lambda x: (abs(x), x))
    if is_tri(variant):
        return float(cands[0]), len(cands)

    def phi(x):
        return ((a3 * x / 4.0 + a2 / 3.0) * x + a1 / 2.0) * x * x + a0 * x

    best = cands[0]
    best_val = phi(best)
    for x in cands[1:]:
        val = phi(x)
        if val < best_val:
            best, best_val = x, val
    return float(best), len(cands)


# ---------------------------------------------------------------------------
# Algorithm 2
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Options:
    variant: int = F1
    first_step: str = "linesearch"   # or "fixed"
    alpha0: float = 0.0
    freeze_eps: float = 0.0
    restart: bool = False            # descent restart of the CG direction


@dataclasses.dataclass
class State:
    X: np.ndarray
    V_prev: Optional[np.ndarray] = None
    G_prev: Optional[np.ndarray] = None
    t: int = 0


def _grams(lap: Laplacian, X, AX, V, G):
    AV = apply_A(lap, V)
    M = X.T @ X
    H = X.T @ AX
    C = X.T @ V
    P = V.T @ V
    E = X.T @ AV
    F = V.T @ AV
    vg = np.sum(V * G, axis=0)
    return M, H, C, P, E, F, vg


def step_size(variant: int, lap: Laplacian, X, AX, V, G) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Exact line search along V from X: returns (alpha[k], coeffs, nroots)."""
    k = X.shape[1]
    M, H, C, P, E, F, vg = _grams(lap, X, AX, V, G)
    co = linesearch_coeffs(variant, M, H, C, P, E, F, vg)
    if is_tri(variant):
        alpha = np.zeros(k)
        nr = np.zeros(k, dtype=np.int64)
        for i in range(k):
            alpha[i], nr[i] = select_root(variant, co[:, i])
        return alpha, co, nr
    a, nr = select_root(variant, co)
    return np.full(k, a), co, np.array([nr])


def _frozen(opts: Options, G, X) -> bool:
    """Stopping once converged (a project reading: Algorithm 2 runs a fixed
    t_max and says nothing about iterating past convergence).  With
    freeze_eps > 0 the step is skipped (every step size 0) when the direction
    is negligible against the iterate, ||G||_F <= freeze_eps ||X||_F; X then
    stays at its fixed point instead of drifting along the neutral orbit that
    rounding noise excites."""
    if opts.freeze_eps <= 0.0:
        return False
    return float(np.linalg.norm(G)) <= opts.freeze_eps * float(np.linalg.norm(X))


def no_root(coeffs, nroots) -> np.ndarray:
    """Per cubic: the line search found no real root although the polynomial
    is not identically zero (the step size is then 0).  A zero polynomial (a
    zero search direction) is not such a case."""
    co = np.asarray(coeffs, dtype=np.float64).reshape(4, -1)
    nr = np.asarray(nroots).reshape(-1)
    return (nr == 0) & np.any(co != 0.0, axis=0)


def init(lap: Laplacian, X0: np.ndarray, opts: Options) -> Tuple[State, Dict]:
    """Algorithm 2 before the loop: G0 = g(X0), V0 = -G0, X1 = X0 + V0 diag(alpha)."""
    X = np.array(X0, dtype=np.float64, copy=True)
    AX = apply_A(lap, X)
    G = direction(opts.variant, X, AX)
    V = -G
    k = X.shape[1]
    if opts.first_step == "fixed":
        alpha = np.full(k, float(opts.alpha0))
        co = None
    else:
        alpha, co, _ = step_size(opts.variant, lap, X, AX, V, G)
    frozen = _frozen(opts, G, X)
    if frozen:
        alpha = np.zeros(k)
    Xn = X + V * alpha[None, :]
    return State(X=Xn, V_prev=V, G_prev=G, t=1), {"alpha": alpha, "coeffs": co, "G": G, "V": V,
                                                  "frozen": frozen}


def pr_beta(G: np.ndarray, G_prev: np.ndarray) -> np.ndarray:
    """Column-wise Polak-Ribiere: sum_r (G - Gp)_ri G_ri / sum_r Gp_ri^2 (0 if the
    denominator vanishes)."""
    num = np.sum((G - G_prev) * G, axis=0)
    den = np.sum(G_prev * G_prev, axis=0)
    out = np.zeros_like(num)
    nz = den != 0.0
    out[nz] = num[nz] / den[nz]
    return out


def step(lap: Laplacian, state: State, opts: Options) -> Tuple[State, Dict]:
    """One loop iteration of Algorithm 2 from (X^t, V^{t-1}, G^{t-1})."""
    X = state.X
    AX = apply_A(lap, X)
    G = direction(opts.variant, X, AX)
    beta = pr_beta(G, state.G_prev)
    V = -G + state.V_prev * beta[None, :]
    if opts.restart:
        # optional safeguard (not part of Algorithm 2): a column whose CG
        # direction is not a descent direction, <V_i, G_i> >= 0, restarts from
        # -G_i (beta_i = 0)
        bad = np.sum(V * G, axis=0) >= 0.0
        beta = np.where(bad, 0.0, beta)
        V = -G + state.V_prev * beta[None, :]
    alpha, co, nr = step_size(opts.variant, lap, X, AX, V, G)
    frozen = _frozen(opts, G, X)
    if frozen:
        alpha = np.zeros_like(alpha)
    Xn = X + V * alpha[None, :]
    return (State(X=Xn, V_prev=V, G_prev=G, t=state.t + 1),
            {"alpha": alpha, "beta": beta, "coeffs": co, "nroots": nr, "G": G, "V": V, "AX": AX,
             "frozen": frozen, "no_root": bool(np.any(no_root(co, nr)))})


def run(lap: Laplacian, X0: np.ndarray, iters: int, opts: Options, record=None):
    """``iters`` updates of X (the first from the pre-loop step).  ``record``
    may be a set of t values whose X^t is kept; returns (X, history)."""
    hist = {"f": [], "X": {}}
    state, _ = init(lap, X0, opts)
    if record is not None and 1 in record:
        hist["X"][1] = state.X.copy()
    for _ in range(iters - 1):
        state, info = step(lap, state, opts)
        if record is not None and state.t in record:
            hist["X"][state.t] = state.X.copy()
    return state, hist


# ---------------------------------------------------------------------------
# Residual  (numerical results section, "Evaluation metrics")
# ---------------------------------------------------------------------------

def relres_gram(M: np.ndarray, H: np.ndarray, K: np.ndarray) -> float:
    """relres^2 = tr(M^{-1} K) / tr((M^{-1} H)^2) - 1 with M = X^T X,
    H = X^T A X, K = (AX)^T (AX)."""
    MiK = np.linalg.solve(M, K)
    MiH = np.linalg.solve(M, H)
    den = float(np.trace(MiH @ MiH))
    val = float(np.trace(MiK)) / den - 1.0
    return math.sqrt(max(val, 0.0))


def relres(lap: Laplacian, X: np.ndarray) -> float:
    """Residual of the Ritz pairs of A on span(X) through the k x k products."""
    AX = apply_A(lap, X)
    return relres_gram(X.T @ X, X.T @ AX, AX.T @ AX)


def relres_direct(lap: Laplacian, X: np.ndarray) -> float:
    """Same quantity through R = AX - X M^{-1} H:
    ||R M^{-1/2}||_F / ||M^{-1/2} H M^{-1/2}||_F."""
    AX = apply_A(lap, X)
    M = X.T @ X
    H = X.T @ AX
    w, Q = np.linalg.eigh(M)
    Mih = Q @ np.diag(1.0 / np.sqrt(w)) @ Q.T
    R = AX - X @ np.linalg.solve(M, H)
    return float(np.linalg.norm(R @ Mih) / np.linalg.norm(Mih @ H @ Mih))


def relres_ritz(lap: Laplacian, X: np.ndarray) -> float:
    """Same quantity the long way: orthonormalise (QR), Rayleigh-Ritz, explicit
    residual ||A U - U Lam||_F / ||U Lam||_F."""
    Q, _ = np.linalg.qr(X)
    T = Q.T @ apply_A(lap, Q)
    lam, W = np.linalg.eigh(0.5 * (T + T.T))
    U = Q @ W
    R = apply_A(lap, U) - U * lam[None, :]
    return float(np.linalg.norm(R) / np.linalg.norm(U * lam[None, :]))


def dense_eigh(lap: Laplacian):
    """Eigenvalues (ascending) and eigenvectors of the dense L."""
    return np.linalg.eigh(dense_L(lap))


# ---------------------------------------------------------------------------
# Post-processing  (Algorithm 1, steps 4-5; numerical results section)
# ---------------------------------------------------------------------------

def row_normalize(X: np.ndarray) -> np.ndarray:
    """Y_l = X_l / ||X_l||_2 (a zero row stays zero)."""
    X = np.asarray(X, dtype=np.float64)
    nr = np.sqrt(np.sum(X * X, axis=1))
    out = np.zeros_like(X)
    nz = nr > 0
    out[nz] = X[nz] / nr[nz, None]
    return out


def kmeans_dist2(Y: np.ndarray, centroids: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances, n x c, sum_d (y_d - mu_d)^2."""
    Y = np.asarray(Y, dtype=np.float64)
    Cn = np.asarray(centroids, dtype=np.float64)
    return np.stack([np.sum((Y - Cn[c][None, :]) ** 2, axis=1) for c in range(Cn.shape[0])], axis=1)


def kmeans_assign(Y: np.ndarray, centroids: np.ndarray):
    """Nearest centroid (lowest index on ties) and its squared distance."""
    D = kmeans_dist2(Y, centroids)
    lab = np.argmin(D, axis=1)
    return lab.astype(np.int32), D[np.arange(D.shape[0]), lab]


def kmeanspp_init(Y: np.ndarray, n_clusters: int, u: np.ndarray) -> np.ndarray:
    """k-means++ seeding (Arthur & Vassilvitskii 2007) driven by given uniforms
    u[0..n_clusters-1] in [0, 1): the first centre is point floor(u0 n); centre
    c is the first point whose running sum of D^2 exceeds u_c * sum D^2."""
    n = Y.shape[0]
    idx = [min(int(u[0] * n), n - 1)]
    d2 = np.sum((Y - Y[idx[0]][None, :]) ** 2, axis=1)
    for c in range(1, n_clusters):
        tot = float(np.sum(d2))
        if tot <= 0.0:
            idx.append(idx[-1])
            continue
        cs = np.cumsum(d2)
        j = int(np.searchsorted(cs, u[c] * tot, side="right"))
        j = min(j, n - 1)
        idx.append(j)
        d2 = np.minimum(d2, np.sum((Y - Y[j][None, :]) ** 2, axis=1))
    return Y[np.array(idx)].copy()


def kmeans_lloyd(Y: np.ndarray, centroids: np.ndarray, max_iter: int = 300):
    """Lloyd iterations until no label changes (or max_iter); an empty cluster
    keeps its previous centroid.  Returns (labels, centroids, iterations)."""
    Cn = np.array(centroids, dtype=np.float64, copy=True)
    lab = None
    for it in range(max_iter):
        new, _ = kmeans_assign(Y, Cn)
        if lab is not None and np.array_equal(new, lab):
            return lab, Cn, it
        lab = new
        for c in range(Cn.shape[0]):
            mem = lab == c
            if np.any(mem):
                Cn[c] = Y[mem].mean(axis=0)
    return lab, Cn, max_iter


def kmeans_uniforms(seed: int, n_clusters: int) -> np.ndarray:
    """The uniforms k-means++ consumes for one repeat (seeded)."""
    return np.random.default_rng([seed, 7]).random(n_clusters)


def kmeans(Y: np.ndarray, n_clusters: int, seed: int = 0, max_iter: int = 300):
    u = kmeans_uniforms(seed, n_clusters)
    return kmeans_lloyd(Y, kmeanspp_init(Y, n_clusters, u), max_iter)


def _contingency(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    _, ai = np.unique(a, return_inverse=True)
    _, bi = np.unique(b, return_inverse=True)
    T = np.zeros((ai.max() + 1, bi.max() + 1), dtype=np.int64)
    np.add.at(T, (ai, bi), 1)
    return T


def ari(a, b) -> float:
    """Adjusted Rand index (Hubert & Arabie 1985) from the contingency table."""
    T = _contingency(a, b)
    n = T.sum()

    def c2(x):
        x = np.asarray(x, dtype=np.float64)
        return x * (x - 1) / 2.0

    s_ij = c2(T).sum()
    s_a = c2(T.sum(axis=1)).sum()
    s_b = c2(T.sum(axis=0)).sum()
    tot = c2(n)
    exp = s_a * s_b / tot if tot > 0 else 0.0
    mx = 0.5 * (s_a + s_b)
    if mx == exp:
        return 1.0
    return float((s_ij - exp) / (mx - exp))


def nmi(a, b) -> float:
    """Normalised mutual information, 2 I(a;b) / (H(a) + H(b)) (Danon et al. 2005)."""
    T = _contingency(a, b).astype(np.float64)
    n = T.sum()
    pa = T.sum(axis=1) / n
    pb = T.sum(axis=0) / n
    pij = T / n
    nz = pij > 0
    I = float(np.sum(pij[nz] * np.log(pij[nz] / (pa[:, None] * pb[None, :])[nz])))
    Ha = -float(np.sum(pa[pa > 0] * np.log(pa[pa > 0])))
    Hb = -float(np.sum(pb[pb > 0] * np.log(pb[pb > 0])))
    if Ha + Hb == 0.0:
        return 1.0
    return 2.0 * I / (Ha + Hb)


def cluster(X: np.ndarray, n_clusters: int, repeats: int = 10, truth=None):
    """Algorithm 1 steps 4-5: row-normalise, K-means repeated with seeds
    0..repeats-1; mean ARI / NMI against ``truth`` when given."""
    Y = row_normalize(X)
    labs = [kmeans(Y, n_clusters, seed=s)[0] for s in range(repeats)]
    if truth is None:
        return labs, None, None
    return labs, float(np.mean([ari(l, truth) for l in labs])), float(np.mean([nmi(l, truth) for l in labs]))
