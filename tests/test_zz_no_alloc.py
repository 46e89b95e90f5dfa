"""ofm_kmeans_noalloc (the K-means of Algorithm 1 step 5 with its buffers in a
fixed device array, for callers that cannot allocate) against ofm_kmeans, the
entry point it mirrors: labels, centroids and Lloyd iteration counts bit for
bit, on two calls in a row, the second with a smaller input."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def blobs(n, dim, nc, seed):
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((nc, dim)) * 3.0
    lab = rng.integers(0, nc, size=n)
    Y = centres[lab] + rng.standard_normal((n, dim))
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    return Y.astype(np.float32)


def test_noalloc_matches_kmeans_twice(lib):
    from paper_2305_10356_amd import ofm
    for n, dim, nc, seed in [(300007, 32, 32, 1), (41000, 16, 12, 2)]:
        print(f"no-alloc k-means n={n} dim={dim} clusters={nc}", flush=True)
        Y = torch.as_tensor(blobs(n, dim, nc, seed)).cuda()
        u = np.random.default_rng([seed, 7]).random(nc)
        la, ca, ia = ofm.kmeans(Y, nc, u, max_iter=60)
        lb, cb, ib = ofm.kmeans(Y, nc, u, max_iter=60, noalloc=True)
        torch.cuda.synchronize()
        assert ia == ib and ia >= 2, (ia, ib)
        assert torch.equal(la, lb)
        assert torch.equal(ca, cb)
        assert int(lb.min()) >= 0 and int(lb.max()) < nc


def test_noalloc_refuses_beyond_its_array(lib):
    from paper_2305_10356_amd import ofm
    L = ofm.load()
    assert L.ofm_kmeans_static_bytes(300007, 32, 32) <= 64 << 20
    big = 10_000_000
    assert L.ofm_kmeans_static_bytes(big, 32, 32) > 64 << 20
    u = (ctypes.c_double * 32)(*([0.5] * 32))
    p = ctypes.c_void_p(256)
    # refused on the host before any device work (the pointers are never read)
    assert L.ofm_kmeans_noalloc(big, 32, 32, p, u, 10, p, p, None, None) == -2
