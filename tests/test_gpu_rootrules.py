"""The root rules of the exact line search (Section 3.2) as the device runs
them (ofm_select_roots calls the same device function as every step) against
the oracle's select_root: the hand-worked cubics of tests/golden/cubics.json,
cubics built from chosen real roots (one, two and three), quadratics with and
without real roots, and raw random coefficients."""
import json
import os

import numpy as np
import pytest

from oracle import ofm_oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
VARS = [("f1", O.F1), ("tri-f1", O.TRI_F1), ("f2", O.F2), ("tri-f2", O.TRI_F2)]


@pytest.fixture(scope="module")
def ofm(lib):
    from paper_2305_10356_amd import ofm as m
    return m


def test_golden_cubics(ofm):
    cases = json.load(open(os.path.join(HERE, "golden", "cubics.json")))["cases"]
    co = np.array([c["coeffs"] for c in cases], dtype=np.float64)
    for variant, key in (("f1", "ofm"), ("f2", "ofm"), ("tri-f1", "tri"), ("tri-f2", "tri")):
        al, nr = ofm.select_roots(variant, co)
        np.testing.assert_allclose(al, [c[key] for c in cases], rtol=1e-12, atol=1e-12)
        assert nr.tolist() == [len(c["roots"]) for c in cases]


def cubic_from_roots(a, r):
    r1, r2, r3 = r
    return [a, -a * (r1 + r2 + r3), a * (r1 * r2 + r1 * r3 + r2 * r3), -a * r1 * r2 * r3]


def random_cubics(seed=23, m=4000):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(m):
        kind = rng.integers(0, 4)
        a = float(np.exp(rng.uniform(-20, 20))) * (1 if rng.random() < 0.8 else -1)
        s = float(np.exp(rng.uniform(-6, 3)))
        if kind == 0:      # three distinct real roots
            r = np.sort(rng.uniform(-1, 1, size=3)) * s
            out.append(cubic_from_roots(a, r))
        elif kind == 1:    # one real root and a complex pair (x - r)(x^2 + b x + c), b^2 < 4c
            r = rng.uniform(-1, 1) * s
            b = rng.uniform(-1, 1) * s
            c = b * b / 4 + float(np.exp(rng.uniform(-4, 1))) * s * s
            out.append([a, a * (b - r), a * (c - r * b), -a * r * c])
        elif kind == 2:    # quadratic (a3 = 0), with or without real roots
            q = rng.standard_normal(3) * s
            out.append([0.0, q[0], q[1], q[2]])
        else:              # raw coefficients over many scales
            out.append(list(rng.standard_normal(4) * np.exp(rng.uniform(-10, 10, size=4))))
    return np.array(out, dtype=np.float64)


def phi(co, x):
    a3, a2, a1, a0 = co
    return ((a3 * x / 4.0 + a2 / 3.0) * x + a1 / 2.0) * x * x + a0 * x


@pytest.mark.parametrize("variant,vid", VARS)
def test_random_cubics_match_oracle(ofm, variant, vid):
    co = random_cubics()
    al, nr = ofm.select_roots(variant, co)
    ref = [O.select_root(vid, c) for c in co]
    ao = np.array([r[0] for r in ref])
    no = np.array([r[1] for r in ref])
    # the classification (number of distinct real roots) is a discrete choice
    # both sides take in FP64 with the same tolerance: identical
    assert np.array_equal(nr, no), np.flatnonzero(nr != no)[:10]
    # the chosen root: equal up to the rounding of cbrt / acos and the polish,
    # relative to the scale of the roots of that cubic
    bad = []
    for i, c in enumerate(co):
        if no[i] == 0:
            assert al[i] == 0.0
            continue
        rts = [r for r, _ in O.cubic_real_roots(*c)]
        scale = max(abs(x) for x in rts) or 1.0
        if abs(al[i] - ao[i]) > 1e-9 * scale:
            bad.append((i, al[i], ao[i]))
    if bad and not O.is_tri(vid):
        # a different choice among three real roots is only acceptable at a
        # tie of the line objective (within the rounding of Phi)
        for i, a, b in bad:
            sc = max(abs(x) for x in co[i]) * max(abs(a), abs(b), 1.0) ** 4
            assert abs(phi(co[i], a) - phi(co[i], b)) <= 1e-12 * sc, (i, co[i], a, b)
        bad = []
    assert not bad, bad[:5]
    print(f"{variant}: {len(co)} cubics, root counts {np.bincount(nr, minlength=4).tolist()}",
          flush=True)


def test_no_root_and_degenerate(ofm):
    co = np.array([
        [0.0, 1.0, 0.0, 1.0],      # x^2 + 1: no real root -> 0
        [0.0, 0.0, 0.0, 0.0],      # zero polynomial -> 0
        [0.0, 0.0, 2.0, -1.0],     # linear 2x - 1 -> 0.5
        [0.0, 1.0, -2.0, 1.0],     # (x - 1)^2 -> 1 (double)
        [1.0, 0.0, 1.0, 1.0],      # x^3 + x + 1: one real root
    ])
    for variant, vid in VARS:
        al, nr = ofm.select_roots(variant, co)
        for i, c in enumerate(co):
            a, n = O.select_root(vid, c)
            assert nr[i] == n and al[i] == pytest.approx(a, rel=1e-13, abs=1e-15), (variant, i)
        assert nr[0] == 0 and al[0] == 0.0 and nr[1] == 0 and al[1] == 0.0
        assert al[2] == 0.5 and al[3] == pytest.approx(1.0)
        assert abs(al[4] ** 3 + al[4] + 1.0) < 1e-14
