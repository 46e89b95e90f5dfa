"""Comparison of one device step of Algorithm 2 with the oracle's step from the
same state (teacher forcing), shared by the single-graph and batched parity
tests.

A root-choice flip (the two sides taking different real roots of the same
line-search cubic) is accepted only where rounding can decide the choice
(Section 3.2 root rules):
* both step sizes are roots of the oracle's cubic, and
* OFM variants: the line objective Phi(a) = a3 a^4/4 + a2 a^3/3 + a1 a^2/2 +
  a0 a takes the same value at both within the tie tolerance;
* triangular variants: |a| is the same for both within the tie tolerance;
* either: the cubic has a near-repeated root (its discriminant is within the
  classification tolerance of zero), so the number of real roots itself is
  decided by rounding.
X is then compared with X^t + V diag(alpha_device) using the oracle's V."""
import numpy as np

from oracle import ofm_oracle as O


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def phi(co, x):
    a3, a2, a1, a0 = (float(c) for c in co)
    return ((a3 * x / 4.0 + a2 / 3.0) * x + a1 / 2.0) * x * x + a0 * x


def phi_scale(co, x):
    a3, a2, a1, a0 = (abs(float(c)) for c in co)
    x = abs(x)
    return a3 * x ** 4 / 4.0 + a2 * x ** 3 / 3.0 + a1 * x * x / 2.0 + a0 * x


def disc_ratio(co):
    """|discriminant| / its scale, as the root classification measures it."""
    a3, a2, a1, a0 = (float(c) for c in co)
    if a3 == 0.0:
        if a2 == 0.0:
            return np.inf
        scale = max(a1 * a1, abs(4.0 * a2 * a0))
        return abs(a1 * a1 - 4.0 * a2 * a0) / scale if scale > 0 else 0.0
    b, c, d = a2 / a3, a1 / a3, a0 / a3
    p = c - b * b / 3.0
    q = 2.0 * b ** 3 / 27.0 - b * c / 3.0 + d
    D = q * q / 4.0 + p ** 3 / 27.0
    scale = max(q * q / 4.0, abs(p ** 3 / 27.0))
    return abs(D) / scale if scale > 0 else 0.0


def flip_explained(vid, co, ag, ao, fp64):
    """(ok, why) for device step size ag against oracle step size ao."""
    rtol = 1e-6 if fp64 else 1e-3
    ttol = 1e-7 if fp64 else 1e-3
    dtol = 1e-6 if fp64 else 1e-2
    for a in (ag, ao):
        scale = sum(abs(c) * abs(a) ** (3 - j) for j, c in enumerate(co))
        if abs(np.polyval(co, a)) > rtol * scale:
            return False, f"{a} is not a root"
    if disc_ratio(co) <= dtol:
        return True, "near-repeated root"
    if O.is_tri(vid):
        if abs(abs(ag) - abs(ao)) <= ttol * max(abs(ag), abs(ao)):
            return True, "|alpha| tie"
        return False, f"|alpha| differ: {ag} vs {ao}"
    sc = max(phi_scale(co, ag), phi_scale(co, ao))
    if abs(phi(co, ag) - phi(co, ao)) <= ttol * sc:
        return True, "Phi tie"
    return False, f"Phi differ: {phi(co, ag)} vs {phi(co, ao)}"


U32 = 2.0 ** -24   # unit roundoff of FP32


def condition(vid, k, info_o, G_prev):
    """||AX_i|| / min(||G_i||, ||G_prev,i||) per column (OFM variants: the
    norms over all columns): G = g(X) is formed from terms of the size of A X,
    so its relative rounding error is about u times this (u the unit roundoff
    of the arithmetic that formed it)."""
    G = info_o["G"]
    AX = info_o["AX"]
    if O.is_tri(vid):
        gn = np.linalg.norm(G, axis=0)
        gp = np.linalg.norm(G_prev, axis=0) if G_prev is not None else gn
        an = np.linalg.norm(AX, axis=0)
    else:
        gn = np.full(k, np.linalg.norm(G))
        gp = np.full(k, np.linalg.norm(G_prev) if G_prev is not None else gn[0])
        an = np.full(k, np.linalg.norm(AX))
    return an / np.maximum(np.minimum(gn, gp), 1e-300)


def scalar_tol(vid, k, info_o, G_prev, fp64):
    """Tolerance per column for alpha_i and beta_i.  FP64: 1e-8.  FP32: 1e-4,
    widened to 100 u cond_i (u = 2^-24) where the direction carries that much
    rounding (see condition)."""
    if fp64:
        return np.full(k, 1e-8)
    return np.maximum(1e-4, 100.0 * U32 * condition(vid, k, info_o, G_prev))


def compare_step(vid, k, Xh, Xnew, gi, info_o, X_oracle, fp64, say=print, G_prev=None):
    """Compare the device's X^{t+1}, alpha, beta (and, in FP64, the cubic
    coefficients) with the oracle's; asserts the step scalars against
    scalar_tol column by column.  Returns (dX, dalpha, dbeta, flips), the
    scalar errors as the largest ratio of error to tolerance, and raises
    AssertionError when a root-choice flip is not explained."""
    # scalars are compared where the data determine them: a column whose
    # direction is a small difference of large terms, ||G_i|| (or ||G_prev,i||)
    # below 1e-6 (FP64) or 1e-3 (FP32) of ||AX_i||, has alpha_i and beta_i set
    # largely by the rounding of G (its X is still compared)
    live = condition(vid, k, info_o, G_prev) <= (1e6 if fp64 else 1e3)
    ag, ao = gi["alpha"], info_o["alpha"]
    ftol = 1e-6 if fp64 else 1e-2
    flip = live & (np.abs(ag - ao) > ftol * max(np.abs(ao).max(), 1e-30))
    flips = []
    ex = rel(Xnew, X_oracle)
    if flip.any():
        cols = np.flatnonzero(flip) if O.is_tri(vid) else [0]
        for i in cols:
            co = info_o["coeffs"][:, i] if O.is_tri(vid) else info_o["coeffs"]
            ok, why = flip_explained(vid, co, ag[i], ao[i], fp64)
            assert ok, (O.VARIANT_NAMES[vid], int(i), why)
            flips.append((int(i), why))
        ex = rel(Xnew, Xh + info_o["V"] * ag[None, :])
        say(f"    root-choice flip in columns {[c for c, _ in flips]}: "
            f"{[w for _, w in flips]} (device {ag[flip]}, oracle {ao[flip]})")
        live = live & ~flip
    ea = rel(ag[live], ao[live]) if live.any() else 0.0
    eb = rel(gi["beta"][live], info_o["beta"][live]) if live.any() and "beta" in info_o else 0.0
    if live.any():
        tol = scalar_tol(vid, k, info_o, G_prev, fp64)
        da = np.abs(ag - ao) / max(np.abs(ao[live]).max(), 1e-300)
        worst_a = float((da / tol)[live].max())
        worst_b = 0.0
        if "beta" in info_o:
            bo = info_o["beta"]
            db = np.abs(gi["beta"] - bo) / max(np.abs(bo[live]).max(), 1e-300)
            worst_b = float((db / tol)[live].max())
        assert worst_a <= 1.0 and worst_b <= 1.0, ("alpha/beta beyond tolerance", ea, eb,
                                                   worst_a, worst_b)
    if fp64 and live.any():
        if O.is_tri(vid):
            assert rel(gi["coeffs"][:, live], info_o["coeffs"][:, live]) < 1e-8
        else:
            assert rel(gi["coeffs"][:, 0], info_o["coeffs"]) < 1e-8
    return ex, ea, eb, flips
