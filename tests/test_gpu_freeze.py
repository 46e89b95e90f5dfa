"""Stopping once converged (ofm_opts.freeze_eps; Algorithm 2 itself runs a
fixed number of steps): a step whose direction is negligible against the
iterate, ||G||_F <= eps ||X||_F, takes step size 0 in every column.  Checked
step by step against the oracle's decision from the same state (teacher
forcing), and the frozen iterate stays bit for bit where it is."""
import numpy as np
import pytest

from oracle import ofm_oracle as O
from paper_2305_10356_amd import graphs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("variant,vid,prec,eps", [
    ("f1", O.F1, "fp64", 1e-7), ("f2", O.F2, "fp64", 1e-7),
    ("tri-f1", O.TRI_F1, "fp64", 1e-7), ("f1", O.F1, "fp32", 1e-4)])
def test_freeze_decision_matches_oracle(lib, variant, vid, prec, eps):
    from paper_2305_10356_amd import ofm
    g, x0 = graphs.workload("sbm-n1000-k8")
    olap = O.laplacian(g.n, g.row_ptr, g.col_idx)
    p = ofm.OFM_FP64 if prec == "fp64" else ofm.OFM_FP32
    dt = torch.float64 if prec == "fp64" else torch.float32
    restart = O.is_tri(vid)
    ws = ofm.Workspace(ofm.Laplacian(g.row_ptr, g.col_idx), 8, variant=variant, precision=p,
                       check_every=1000000, freeze_eps=eps, restart=restart)
    X = torch.as_tensor(x0.astype(np.float32) if p == ofm.OFM_FP32 else x0, dtype=dt).cuda()
    opts = O.Options(variant=vid, freeze_eps=eps, restart=restart)
    ws.init(X)
    frozen_at, ties = None, 0
    for t in range(1, 700):
        Xh = host(X)
        Vp, Gp = ws.get_state()
        _, info = O.step(olap, O.State(X=Xh, V_prev=host(Vp), G_prev=host(Gp), t=t), opts)
        ws.step(X)
        alpha = ws.step_info()["alpha"]
        G = host(ws.get_state()[1])        # the direction of this step
        ratio = np.linalg.norm(G) / np.linalg.norm(Xh)
        gpu_frozen = bool(np.all(alpha == 0.0))
        if abs(ratio / eps - 1.0) < 1e-3:  # too close to the threshold to call
            ties += 1
        else:
            assert gpu_frozen == (ratio <= eps), (t, ratio)
            assert gpu_frozen == info["frozen"], (t, ratio, info["frozen"])
        if gpu_frozen:
            assert np.array_equal(host(X), Xh), t
            frozen_at = t if frozen_at is None else frozen_at
    print(f"{variant} {prec}: frozen from step {frozen_at}, near-threshold steps {ties}",
          flush=True)
    assert frozen_at is not None
    assert O.relres(olap, host(X)) < (1e-5 if prec == "fp64" else 1e-2)


def test_freeze_off_keeps_moving(lib):
    # eps = 0 never freezes: the converged FP64 OFM-f1 iterate keeps taking
    # nonzero steps along the neutral orbit (rounding noise)
    from paper_2305_10356_amd import ofm
    g, x0 = graphs.workload("sbm-n1000-k8")
    ws = ofm.Workspace(ofm.Laplacian(g.row_ptr, g.col_idx), 8, variant="f1",
                       precision=ofm.OFM_FP64, check_every=1000000)
    X = torch.as_tensor(x0).cuda()
    ws.init(X)
    for _ in range(400):
        ws.step(X)
    assert np.any(ws.step_info()["alpha"] != 0.0)


def test_freeze_eps_refused_when_negative(lib):
    from paper_2305_10356_amd import ofm
    g, _ = graphs.workload("sbm-n1000-k8")
    lap = ofm.Laplacian(g.row_ptr, g.col_idx)
    with pytest.raises(ofm.OfmError) as e:
        ofm.Workspace(lap, 8, freeze_eps=-1.0)
    assert e.value.status == -1
