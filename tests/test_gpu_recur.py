"""A X by recurrence (opts.recur): A X^{t+1} = A X^t + A V^t diag(alpha^t), exact
A X at every residual evaluation.  The iteration of Algorithm 2 is the same in
exact arithmetic, so the iterates are compared with the FP64 oracle (which
forms A X^t directly) over a free-running window, the limits with the dense
eigendecomposition, and the recurred products with the oracle's."""
import sys

import numpy as np
import pytest

from oracle import ofm_oracle as O
from paper_2305_10356_amd import graphs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

VARS = [("f1", O.F1), ("tri-f1", O.TRI_F1), ("f2", O.F2), ("tri-f2", O.TRI_F2)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def sbm1k(lib):
    from paper_2305_10356_amd import ofm
    g, x0 = graphs.workload("sbm-n1000-k8")
    return g, x0, O.laplacian(g.n, g.row_ptr, g.col_idx), ofm.Laplacian(g.row_ptr, g.col_idx)


@pytest.mark.parametrize("ce", [1000000, 7])
@pytest.mark.parametrize("variant,vid", VARS)
def test_recur_free_running_window_fp64(sbm1k, variant, vid, ce):
    from paper_2305_10356_amd import ofm
    g, x0, olap, glap = sbm1k
    ws = ofm.Workspace(glap, 8, variant=variant, precision=ofm.OFM_FP64, check_every=ce,
                       recur=True)
    X = torch.as_tensor(x0).cuda()
    ws.init(X)
    st, _ = O.init(olap, x0, O.Options(variant=vid))
    for t in range(1, 20):
        ws.step(X)
        st, _ = O.step(olap, st, O.Options(variant=vid))
    err = rel(host(X), st.X)
    say(f"recur free-running {variant} ce={ce} err={err:.2e}")
    assert err < 1e-10


@pytest.mark.parametrize("variant,vid", [("f2", O.F2), ("tri-f2", O.TRI_F2)])
def test_recurred_products_match_oracle(variant, vid):
    """After updates with no residual evaluation, X^T A X is formed from the
    recurred A X; it matches the oracle's product of the same X."""
    from paper_2305_10356_amd import ofm
    g, x0 = graphs.workload("sbm-n50k-k32")
    olap = O.laplacian(g.n, g.row_ptr, g.col_idx)
    glap = ofm.Laplacian(g.row_ptr, g.col_idx)
    for prec, dt, tol in ((ofm.OFM_FP64, torch.float64, 1e-12),
                          (ofm.OFM_FP32, torch.float32, 2e-5)):
        ws = ofm.Workspace(glap, 32, variant=variant, precision=prec, check_every=1000000,
                           recur=True, restart=variant.startswith("tri"))
        X = torch.as_tensor(x0, dtype=dt).cuda()
        ws.init(X)
        for _ in range(9):
            ws.step(X)
        Xh = host(X)
        H = ws.product("H")
        Href = Xh.T @ O.apply_A(olap, Xh)
        err = rel(H, Href)
        say(f"recurred H {variant} {dt}: {err:.2e}")
        assert err < tol


@pytest.mark.parametrize("variant,vid", VARS)
def test_recur_solve_limits_fp64(sbm1k, variant, vid):
    from paper_2305_10356_amd import ofm
    g, x0, olap, glap = sbm1k
    k = 8
    mu, U = O.dense_eigh(olap)
    ws = ofm.Workspace(glap, k, variant=variant, precision=ofm.OFM_FP64, max_iter=500,
                       check_every=10, tol=1e-9, restart=O.is_tri(vid), recur=True)
    X = torch.as_tensor(x0).cuda()
    st = ws.solve(X)
    Xh = host(X)
    rr_o = O.relres(olap, Xh)
    say(f"recur solve {variant}: iters={st['iters']} relres={st['relres']:.2e} oracle={rr_o:.2e}")
    assert st["status"] == 0 and st["converged"] == 1
    assert rr_o < 1e-7
    Uk = U[:, :k]
    if vid in (O.F1, O.TRI_F1):
        target = (Uk * (2.0 - mu[:k])[None, :]) @ Uk.T
    else:
        target = Uk @ Uk.T
    np.testing.assert_allclose(Xh @ Xh.T, target, atol=1e-6)


def test_recur_fp32_sbm50k_reaches_tolerance():
    from paper_2305_10356_amd import ofm
    g, x0 = graphs.workload("sbm-n50k-k32")
    olap = O.laplacian(g.n, g.row_ptr, g.col_idx)
    glap = ofm.Laplacian(g.row_ptr, g.col_idx)
    iters = {}
    for recur in (False, True):
        ws = ofm.Workspace(glap, 32, variant="f1", precision=ofm.OFM_FP32, max_iter=2000,
                           check_every=10, tol=1e-4, recur=recur)
        X = torch.as_tensor(x0.astype(np.float32)).cuda()
        st = ws.solve(X)
        rr = O.relres(olap, host(X))
        say(f"50k-node SBM FP32 f1 recur={recur}: iters={st['iters']} relres={st['relres']:.2e} "
            f"oracle={rr:.2e}")
        assert st["converged"] == 1
        assert rr < 2e-4
        iters[recur] = st["iters"]
    assert iters[True] <= 1.3 * iters[False] + 20


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_recur_graph_replay_is_bitwise_eager(prec):
    from paper_2305_10356_amd import ofm
    g, x0 = graphs.workload("sbm-n1000-k8" if prec == "fp64" else "sbm-n50k-k32")
    glap = ofm.Laplacian(g.row_ptr, g.col_idx)
    p = ofm.OFM_FP64 if prec == "fp64" else ofm.OFM_FP32
    dt = torch.float64 if prec == "fp64" else torch.float32
    out = []
    for graph in (False, True):
        ws = ofm.Workspace(glap, x0.shape[1], variant="f2", precision=p, max_iter=300,
                           check_every=10, tol=1e-7 if prec == "fp64" else 1e-4, recur=True,
                           graph=graph)
        X = torch.as_tensor(x0, dtype=dt).cuda()
        st = ws.solve(X)
        out.append((host(X), st))
    assert out[0][1] == out[1][1]
    np.testing.assert_array_equal(out[0][0], out[1][0])
