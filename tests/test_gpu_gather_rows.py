"""ofm_gather_rows (the measurement of random row gathers that bench.py
--gather-ceiling times) sums the indexed rows: against a plain gather-sum."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("rf", [16, 32, 64])
def test_gather_rows_sums_the_indexed_rows(lib, rf):
    from paper_2305_10356_amd import ofm
    rng = np.random.default_rng(rf)
    rows, nrows, S = 5000, 3001, 7
    Z = rng.standard_normal((rows, rf)).astype(np.float32)
    idx = rng.integers(0, rows, size=nrows * S).astype(np.int32)
    Y = ofm.gather_rows(torch.as_tensor(idx).cuda(), torch.as_tensor(Z).cuda(), S)
    torch.cuda.synchronize()
    ref = Z[idx].reshape(nrows, S, rf).astype(np.float64).sum(axis=1)
    np.testing.assert_allclose(Y.cpu().numpy(), ref, rtol=0, atol=1e-5)
