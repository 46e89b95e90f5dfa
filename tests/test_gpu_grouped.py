"""The grouped row order (ofm_build_laplacian_grouped: rows dealt to eight XCD
slots by node group) against the plain order and the FP64 oracle.

* Products with A are bitwise those of the plain order (each row is summed by
  the same lanes in the same entry order), for several groupings: the planted
  blocks, scattered ids with a fifth of the nodes in no group, a single group
  (seven empty slots) and no group at all, at k = 8, 32, 64 and in FP64.
* Iterations on a 150,000-node graph, which runs the SpMMs with one workgroup
  per tile group (over 1,024 workgroups, so the partial rows are reduced in
  more than two levels) and the residual steps on the strided grid: the k x k
  products and the iterates agree with the plain order to the rounding of the
  FP64 sums, and the residual of the grouped FP64 iterate matches the oracle's.
* An FP32 solve to 1e-4 on the grouped order, residual checked by the oracle.
* Argument errors."""
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


@pytest.fixture(scope="module")
def ofm(lib):
    from paper_2305_10356_amd import ofm as m
    return m


@pytest.fixture(scope="module")
def dc150k():
    g, _ = graphs.workload("dcsbm-n2m-k32", n=150_000)
    return g


def groupings(g, rng):
    lab = g.labels.astype(np.int32)
    mixed = rng.permutation(64).astype(np.int32)[lab]
    mixed[rng.random(g.n) < 0.2] = -1
    return {"planted": lab, "mixed": mixed, "one": np.zeros(g.n, np.int32),
            "none": np.full(g.n, -1, np.int32)}


def test_grouped_apply_is_bitwise_plain(ofm, dc150k):
    g = dc150k
    plain = ofm.Laplacian(g.row_ptr, g.col_idx)
    rng = np.random.default_rng(11)
    cases = ((32, torch.float32), (64, torch.float32), (8, torch.float32), (32, torch.float64))
    Zs = {c: torch.as_tensor(rng.standard_normal((g.n, c[0])), dtype=c[1]).cuda() for c in cases}
    ref = {c: plain.apply(Z) for c, Z in Zs.items()}
    for name, gr in groupings(g, rng).items():
        lap = ofm.Laplacian(g.row_ptr, g.col_idx, groups=gr)
        for c, Z in Zs.items():
            say(f"grouped apply: grouping {name}, k={c[0]}, {c[1]}")
            Y = lap.apply(Z)
            assert torch.equal(Y, ref[c])
        lap.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_grouped_steps_match_plain_and_oracle(ofm, dc150k, prec):
    g = dc150k
    P, dt = (ofm.OFM_FP64, torch.float64) if prec == "fp64" else (ofm.OFM_FP32, torch.float32)
    x0 = graphs.initial_x(g.n, 32, np.random.default_rng(5))
    runs = []
    for gr in (None, g.labels):
        lap = ofm.Laplacian(g.row_ptr, g.col_idx, groups=gr)
        ws = ofm.Workspace(lap, 32, variant="f1", precision=P, max_iter=10**6, check_every=3)
        X = torch.as_tensor(x0, dtype=dt).cuda()
        ws.init(X)
        for _ in range(7):
            ws.step(X)
        M = ws.product("M")
        res = ws.residual(X)
        runs.append((host(X), M, res))
        ws.close()
        lap.close()
    (x_p, m_p, r_p), (x_g, m_g, r_g) = runs
    dx = np.abs(x_g - x_p).max() / np.abs(x_p).max()
    dm = np.abs(m_g - m_p).max() / np.abs(m_p).max()
    say(f"grouped vs plain {prec}: X {dx:.2e}, X^T X {dm:.2e}, relres {r_g['relres']:.6e} / {r_p['relres']:.6e}")
    if prec == "fp64":
        assert dx < 1e-10 and dm < 1e-10
        olap = O.laplacian(g.n, g.row_ptr, g.col_idx)
        rr = O.relres(olap, x_g)
        say(f"  oracle relres of the grouped iterate {rr:.6e}")
        assert abs(r_g["relres"] - rr) <= 1e-8 * rr
    else:
        # one FP32 rounding of the step sizes apart, amplified by 8 updates
        assert dx < 1e-4 and dm < 1e-4
        assert abs(r_g["relres"] - r_p["relres"]) <= 1e-3 * r_p["relres"]


def test_grouped_fp32_solve_reaches_tolerance(ofm, dc150k):
    g = dc150k
    lap = ofm.Laplacian(g.row_ptr, g.col_idx, groups=g.labels)
    x0 = graphs.initial_x(g.n, 32, np.random.default_rng(6)).astype(np.float32)
    ws = ofm.Workspace(lap, 32, variant="f1", precision=ofm.OFM_FP32, max_iter=2000,
                       check_every=10, tol=1e-4)
    X = torch.as_tensor(x0).cuda()
    st = ws.solve(X)
    olap = O.laplacian(g.n, g.row_ptr, g.col_idx)
    rr = O.relres(olap, host(X))
    say(f"grouped FP32 solve: iters={st['iters']} relres {st['relres']:.2e}, oracle {rr:.2e}")
    assert st["converged"] == 1 and rr < 2e-4


def test_grouped_build_errors(ofm):
    g, _ = graphs.workload("sbm-n1000-k8")
    bad = g.labels.astype(np.int32).copy()
    bad[7] = g.n
    with pytest.raises(ofm.OfmError):
        ofm.Laplacian(g.row_ptr, g.col_idx, groups=bad)
    with pytest.raises(ofm.OfmError):
        ofm.Laplacian(g.row_ptr, g.col_idx, groups=g.labels, reorder=False)
    with pytest.raises(ValueError):
        ofm.Laplacian(g.row_ptr, g.col_idx, groups=g.labels[:-1])


def test_grouped_weighted_validated_small(ofm):
    """Weighted similarities, the symmetry check, and a graph smaller than one
    tile per slot (several slots empty): products with A bitwise the plain
    order's and equal to the oracle's."""
    g, _ = graphs.workload("sbm-n1000-k8")
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    a, b = np.minimum(rows, g.col_idx), np.maximum(rows, g.col_idx)
    w = 1.0 + ((a * 7919 + b * 104729) % 13) / 13.0  # symmetric by construction
    olap = O.laplacian(g.n, g.row_ptr, g.col_idx, w)
    rng = np.random.default_rng(3)
    Z = torch.as_tensor(rng.standard_normal((g.n, 8))).cuda()
    plain = ofm.Laplacian(g.row_ptr, g.col_idx, vals=w, validate=True)
    ref = plain.apply(Z)
    for gr in (g.labels, np.where(np.arange(g.n) < 40, 3, -1).astype(np.int32),
               torch.as_tensor(g.labels).cuda()):
        lap = ofm.Laplacian(g.row_ptr, g.col_idx, vals=w, validate=True, groups=gr)
        Y = lap.apply(Z)
        assert torch.equal(Y, ref)
        np.testing.assert_allclose(host(Y), O.apply_A(olap, host(Z)), rtol=0, atol=1e-13)
        lap.close()
