"""The upper-triangle copy of the Laplacian and the line searches that take
their products with A V from it (Section 3.2).  The copy keeps, of every
stored pair (i, j), (j, i), the entry whose column comes later in the order of
the nodes by (degree, id).  With A symmetric and U_i = sum over row i of the
copy of w_ij V_j: the OFM-f1 and TriOFM-f1 cubics need only
diag(V^T A V) = -diag(V^T V) - 2 diag(V^T U); the f2 cubics need
V^T A V = -V^T V - (V^T U + U^T V) and X^T A V = (AX)^T V, the latter formed
in the V pass from the A X that the SpMM of X stores (k <= 32).

* its size, and the Laplacians that build none (self-loops, index order,
  the opt-out flag);
* teacher-forced steps through it against the FP64 oracle, and against the
  same step with the full product A V from the same state."""
import sys

import numpy as np
import pytest

import stepcheck
from oracle import ofm_oracle as O
from paper_2305_10356_amd import graphs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ofm(lib):
    from paper_2305_10356_amd import ofm as m
    return m


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def upper_size(rp, ci):
    """(rows with an entry in the copy, entries in the copy): entry (i, j) is
    in it when node j comes after node i by (degree, id)"""
    n = len(rp) - 1
    deg = np.diff(rp)
    rows = np.repeat(np.arange(n), deg)
    up = (deg[ci] > deg[rows]) | ((deg[ci] == deg[rows]) & (ci > rows))
    return int(np.count_nonzero(np.bincount(rows[up], minlength=n))), int(up.sum())


@pytest.fixture(scope="module")
def dcsbm20k():
    g, _ = graphs.workload("dcsbm-n2m-k32", n=20000)
    return g


def test_upper_copy_size(ofm, dcsbm20k):
    g = dcsbm20k
    lap = ofm.Laplacian(g.row_ptr, g.col_idx)
    rows, ents = lap.upper()
    say(f"upper copy: {rows} rows, {ents} entries of {len(g.col_idx)}")
    assert (rows, ents) == upper_size(g.row_ptr, g.col_idx)
    assert 2 * ents == len(g.col_idx)      # symmetric, no self-loops
    assert rows < g.n                      # the last node by (degree, id) has nothing after it
    for kw in ({"upper": False}, {"reorder": False}):
        assert ofm.Laplacian(g.row_ptr, g.col_idx, **kw).upper() == (0, 0), kw
    # the grouped order keeps the same copy, laid out in its XCD slots
    assert ofm.Laplacian(g.row_ptr, g.col_idx, groups=g.labels).upper() == (rows, ents)
    # one self-loop: no copy (the identity above needs w_ii = 0)
    n = 6
    ent = sorted([(i, (i + 1) % n) for i in range(n)] + [((i + 1) % n, i) for i in range(n)]
                 + [(2, 2)])
    rp = np.zeros(n + 1, dtype=np.int32)
    for a, _ in ent:
        rp[a + 1] += 1
    rp = np.cumsum(rp).astype(np.int32)
    ci = np.array([b for _, b in ent], dtype=np.int32)
    assert ofm.Laplacian(rp, ci).upper() == (0, 0)


F1_VARS = [("f1", O.F1), ("tri-f1", O.TRI_F1)]
ALL_VARS = F1_VARS + [("f2", O.F2), ("tri-f2", O.TRI_F2)]


def teacher_forced_pair(ofm, g, x0, variant, vid, precision, checkpoints, tol, restart):
    """Steps of a workspace on the Laplacian with the upper copy, each checked
    against the oracle's step from the same state and against a workspace on
    the Laplacian without it, set to that state."""
    dt = torch.float64 if precision == ofm.OFM_FP64 else torch.float32
    fp64 = precision == ofm.OFM_FP64
    k = x0.shape[1]
    olap = O.laplacian(g.n, g.row_ptr, g.col_idx)
    lu = ofm.Laplacian(g.row_ptr, g.col_idx)
    lf = ofm.Laplacian(g.row_ptr, g.col_idx, upper=False)
    assert lu.upper()[1] > 0 and lf.upper() == (0, 0)
    opts = O.Options(variant=vid, restart=restart)
    wu = ofm.Workspace(lu, k, variant=variant, precision=precision, restart=restart,
                       check_every=1000000)
    wf = ofm.Workspace(lf, k, variant=variant, precision=precision, restart=restart,
                       check_every=1000000)
    x0 = x0.astype(np.float32) if not fp64 else x0
    Xu, Xf = dev(x0, dt), dev(x0, dt)
    X0h = host(Xu)
    wu.init(Xu)
    wf.init(Xf)
    st_o, info_o = O.init(olap, X0h, opts)
    assert stepcheck.rel(host(Xu), st_o.X) < tol
    assert stepcheck.rel(host(Xu), host(Xf)) < (1e-12 if fp64 else 1e-5)
    flips = []
    for t in range(1, max(checkpoints) + 1):
        if t not in checkpoints:
            wu.step(Xu)
            continue
        Xh = host(Xu)
        Vp, Gp = wu.get_state()
        state = O.State(X=Xh, V_prev=host(Vp), G_prev=host(Gp), t=t)
        st_o, info_o = O.step(olap, state, opts)
        # the full-product workspace from the same state
        Xf = Xu.clone()
        wf.set_state(Xf, Vp.clone(), Gp.clone(), t)
        wu.step(Xu)
        wf.step(Xf)
        gu, gf = wu.step_info(), wf.step_info()
        ex, ea, eb, fl = stepcheck.compare_step(vid, k, Xh, host(Xu), gu, info_o, st_o.X, fp64,
                                                say=say, G_prev=state.G_prev)
        flips += [(t, c, why) for c, why in fl]
        # coefficients of the two device forms: the same cubics up to the
        # rounding of the quadratic forms
        du = stepcheck.rel(gu["coeffs"], gf["coeffs"])
        say(f"  {variant} t={t} dX={ex:.2e} dalpha={ea:.2e} coeffs upper/full {du:.2e}")
        assert ex < tol, (variant, t, "X")
        assert du < (1e-12 if fp64 else 1e-4), (variant, t, "coefficients upper vs full")
        if not fl:
            assert stepcheck.rel(host(Xu), host(Xf)) < (1e-12 if fp64 else 1e-4)
    assert len(flips) <= 2, flips


@pytest.mark.parametrize("variant,vid", ALL_VARS)
@pytest.mark.parametrize("k", [8, 32])
def test_teacher_forced_upper_fp64(ofm, dcsbm20k, variant, vid, k):
    g = dcsbm20k
    x0 = graphs.initial_x(g.n, k, np.random.default_rng([21, k]))
    say(f"teacher-forced FP64 upper copy, 20k-node DC-SBM, k={k} {variant}")
    teacher_forced_pair(ofm, g, x0, variant, vid, ofm.OFM_FP64, {1, 2, 5, 12, 30}, 1e-10,
                        restart=O.is_tri(vid))


@pytest.mark.parametrize("variant,vid", ALL_VARS)
@pytest.mark.parametrize("k", [4, 16, 32, 64])
def test_teacher_forced_upper_fp32(ofm, dcsbm20k, variant, vid, k):
    g = dcsbm20k
    x0 = graphs.initial_x(g.n, k, np.random.default_rng([22, k]))
    say(f"teacher-forced FP32 upper copy, 20k-node DC-SBM, k={k} {variant}")
    teacher_forced_pair(ofm, g, x0, variant, vid, ofm.OFM_FP32, {1, 2, 5, 12}, 1e-4,
                        restart=O.is_tri(vid))


def test_upper_small_graphs(ofm):
    # a 70-node clique (equal degrees: the copy keeps the later ids, so node 0
    # keeps 69 entries, a row processed a wavefront at a time), 80 nodes hung
    # on five clique nodes (entries toward the clique) and the last node by
    # (degree, id) with nothing in the copy
    n = 150
    edges = {(a, b) for a in range(70) for b in range(a + 1, 70)}
    edges |= {(65 + i % 5, i) for i in range(70, n)}
    # and some leaf-leaf edges, which break the clique's symmetry
    rng = np.random.default_rng(5)
    edges |= {(int(min(a, b)), int(max(a, b))) for a, b in rng.integers(70, n, size=(60, 2))
              if a != b}
    ent = sorted(list(edges) + [(b, a) for a, b in edges])
    rp = np.zeros(n + 1, dtype=np.int32)
    for a, _ in ent:
        rp[a + 1] += 1
    rp = np.cumsum(rp).astype(np.int32)
    ci = np.array([b for _, b in ent], dtype=np.int32)
    g = graphs.Graph(n=n, row_ptr=rp, col_idx=ci, labels=np.zeros(n, dtype=np.int32), meta={})
    lap = ofm.Laplacian(rp, ci)
    rows, ents = upper_size(rp, ci)
    assert lap.upper() == (rows, ents) and rows == n - 1
    deg = np.diff(rp)
    r = np.repeat(np.arange(n), deg)
    up = (deg[ci] > deg[r]) | ((deg[ci] == deg[r]) & (ci > r))
    assert np.bincount(r[up], minlength=n).max() >= 64
    for variant, vid in ALL_VARS:
        x0 = graphs.initial_x(n, 8, np.random.default_rng(6))
        teacher_forced_pair(ofm, g, x0, variant, vid, ofm.OFM_FP64, {1, 3, 10}, 1e-10,
                            restart=O.is_tri(vid))


@pytest.mark.parametrize("variant,vid", ALL_VARS)
def test_teacher_forced_upper_grouped(ofm, dcsbm20k, variant, vid):
    # the copy in the grouped order (planted blocks as groups, XCD slots)
    # against the oracle and the full product on a plain Laplacian
    g = dcsbm20k
    k = 16
    x0 = graphs.initial_x(g.n, k, np.random.default_rng([23, k]))
    olap = O.laplacian(g.n, g.row_ptr, g.col_idx)
    lg = ofm.Laplacian(g.row_ptr, g.col_idx, groups=g.labels)
    lf = ofm.Laplacian(g.row_ptr, g.col_idx, upper=False)
    restart = O.is_tri(vid)
    opts = O.Options(variant=vid, restart=restart)
    wg = ofm.Workspace(lg, k, variant=variant, precision=ofm.OFM_FP32, restart=restart,
                       check_every=1000000)
    wf = ofm.Workspace(lf, k, variant=variant, precision=ofm.OFM_FP32, restart=restart,
                       check_every=1000000)
    X = dev(x0.astype(np.float32), torch.float32)
    wg.init(X)
    for t in range(1, 8):
        Xh = host(X)
        Vp, Gp = wg.get_state()
        state = O.State(X=Xh, V_prev=host(Vp), G_prev=host(Gp), t=t)
        st_o, info_o = O.step(olap, state, opts)
        Xf = X.clone()
        wf.set_state(Xf, Vp.clone(), Gp.clone(), t)
        wg.step(X)
        wf.step(Xf)
        gg, gf = wg.step_info(), wf.step_info()
        ex, ea, eb, fl = stepcheck.compare_step(vid, k, Xh, host(X), gg, info_o, st_o.X, False,
                                                say=say, G_prev=state.G_prev)
        assert ex < 1e-4, (variant, t, ex)
        assert stepcheck.rel(gg["coeffs"], gf["coeffs"]) < 1e-4, (variant, t)
