"""Seeded synthetic graph and initial-point generators.

This module produces the inputs that both the HIP path and the FP64 checker
consume: undirected stochastic-block-model (SBM) graphs in CSR form, their
planted partitions, and the random initial feature block X0.  It holds none of
the method's arithmetic (no Laplacian, no gradient, no step); it only draws
random graphs.

The paper evaluates on the IEEE HPEC Graph Challenge SBM graphs (numerical
results section, "Dataset").  Those files are not available, so seeded synthetic
SBM graphs of the same kind stand in for them:

* plain SBM: exact G(n, p) per block pair (binomial edge count, then distinct
  uniformly chosen pairs);
* degree-corrected SBM with a truncated power-law degree propensity theta
  (exponent 2.5 on [1, theta_c]) inside each block, for the large
  bandwidth-bound graph;
* a node-arrival growth process for the streaming snapshots.

Every graph is made simple (no self-loops, no duplicate edges), symmetric,
connected (one extra edge per non-giant component, into the giant component,
inside the same block) and its node ids are randomly permuted so that storage
order does not reveal the blocks.

The block-mixing parameter ``r`` is the expected ratio of inter-block to
intra-block edge counts.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Graph",
    "sbm_plain",
    "dcsbm_powerlaw",
    "workload",
    "initial_x",
    "dirichlet_sizes",
    "lognormal_sizes",
    "equal_sizes",
    "bfs_ball_subgraph",
    "batched_graph_specs",
    "streaming_snapshots",
    "GrowthStream",
    "warm_start",
]


@dataclasses.dataclass
class Graph:
    """Undirected simple graph in CSR form (both directions stored).

    ``row_ptr`` is int32[n+1], ``col_idx`` int32[nnz] with sorted columns per
    row; ``labels`` int32[n] is the planted block of every node.
    """

    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    labels: np.ndarray
    meta: dict

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def stats(self) -> dict:
        deg = self.degrees()
        lab = self.labels
        rows = np.repeat(np.arange(self.n, dtype=np.int64), deg)
        inter = int(np.count_nonzero(lab[rows] != lab[self.col_idx]))
        intra = self.nnz - inter
        return {
            "n": self.n,
            "nnz": self.nnz,
            "mean_degree": float(deg.mean()) if self.n else 0.0,
            "max_degree": int(deg.max()) if self.n else 0,
            "min_degree": int(deg.min()) if self.n else 0,
            "realized_r": inter / max(intra, 1),
            "blocks": int(lab.max()) + 1 if self.n else 0,
        }


# ----------------------------------------------------------------------------
# block sizes
# ----------------------------------------------------------------------------

def _round_sizes(n: int, frac: np.ndarray) -> np.ndarray:
    sizes = np.floor(n * frac).astype(np.int64)
    sizes[int(np.argmax(sizes))] += n - int(sizes.sum())
    return sizes


def dirichlet_sizes(n: int, k: int, rng: np.random.Generator, conc: float = 2.0,
                    min_size: int = 50) -> np.ndarray:
    """Block sizes with proportions ~ Dirichlet(conc * 1_k), resampled until
    every block has at least ``min_size`` nodes; the rounding remainder goes
    to the largest block."""
    for _ in range(100000):
        frac = rng.dirichlet(np.full(k, conc))
        sizes = _round_sizes(n, frac)
        if sizes.min() >= min_size:
            return sizes
    raise RuntimeError("could not draw Dirichlet block sizes with the minimum size")


def lognormal_sizes(n: int, k: int, rng: np.random.Generator, sigma: float = 0.5) -> np.ndarray:
    """Block sizes proportional to LogNormal(0, sigma) weights, summing to n."""
    w = rng.lognormal(0.0, sigma, size=k)
    return _round_sizes(n, w / w.sum())


def equal_sizes(n: int, k: int) -> np.ndarray:
    sizes = np.full(k, n // k, dtype=np.int64)
    sizes[: n - int(sizes.sum())] += 1
    return sizes


# ----------------------------------------------------------------------------
# edge sampling helpers
# ----------------------------------------------------------------------------

def _tri_unrank(idx: np.ndarray, m: int):
    """Map linear indices over the strict upper triangle of an m x m matrix
    (row-major, pairs u < v) back to (u, v)."""
    idx = idx.astype(np.int64)
    # row u starts at offset u*m - u*(u+1)/2
    mf = float(m)
    u = np.floor((2 * mf - 1 - np.sqrt((2 * mf - 1) ** 2 - 8.0 * idx)) / 2).astype(np.int64)
    u = np.clip(u, 0, m - 2)

    def start(uu):
        return uu * m - uu * (uu + 1) // 2

    # fix floating point off-by-one
    too_far = start(u) > idx
    while np.any(too_far):
        u[too_far] -= 1
        too_far = start(u) > idx
    nxt = start(u + 1) <= idx
    while np.any(nxt & (u < m - 2)):
        u[nxt & (u < m - 2)] += 1
        nxt = start(u + 1) <= idx
    v = idx - start(u) + u + 1
    return u, v


def _choose_distinct(rng: np.random.Generator, population: int, m: int) -> np.ndarray:
    if m <= 0:
        return np.zeros(0, dtype=np.int64)
    if m > population:
        raise ValueError("more edges than pairs")
    if m * 4 >= population:
        return rng.permutation(population)[:m].astype(np.int64)
    out = np.unique(rng.integers(0, population, size=int(m * 1.2) + 16, dtype=np.int64))
    while out.shape[0] < m:
        extra = rng.integers(0, population, size=(m - out.shape[0]) * 2 + 16, dtype=np.int64)
        out = np.unique(np.concatenate([out, extra]))
    # keep a uniformly random subset of size m of the distinct draws
    return rng.permutation(out)[:m]


def _edges_to_csr(n: int, u: np.ndarray, v: np.ndarray):
    """Undirected edge list (u != v, each pair once, any orientation) to a
    symmetric CSR with sorted columns."""
    a = np.concatenate([u, v]).astype(np.int64)
    b = np.concatenate([v, u]).astype(np.int64)
    key = a * n + b
    key = np.unique(key)
    rows = key // n
    cols = key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr, cols


def _canonical_unique(n: int, u: np.ndarray, v: np.ndarray):
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * np.int64(n) + hi)
    return key // n, key % n


def _connect(n: int, u: np.ndarray, v: np.ndarray, labels: np.ndarray,
             rng: np.random.Generator):
    """Add one edge from a random member of every non-giant connected
    component to a random giant-component node of the same block (any giant
    node if the block has none there)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    adj = sp.coo_matrix((np.ones(u.shape[0], dtype=np.int8), (u, v)), shape=(n, n)).tocsr()
    ncomp, comp = connected_components(adj, directed=False)
    if ncomp == 1:
        return u, v, 0
    counts = np.bincount(comp, minlength=ncomp)
    giant = int(np.argmax(counts))
    in_giant = comp == giant
    giant_nodes = np.flatnonzero(in_giant)
    giant_by_block = {}
    glab = labels[giant_nodes]
    order = np.argsort(glab, kind="stable")
    gs = giant_nodes[order]
    gl = glab[order]
    bounds = np.flatnonzero(np.diff(gl)) + 1
    for seg in np.split(np.arange(gs.shape[0]), bounds):
        if seg.shape[0]:
            giant_by_block[int(gl[seg[0]])] = gs[seg]
    # one random member per non-giant component (deterministic given rng)
    nodes = np.flatnonzero(~in_giant)
    perm = rng.permutation(nodes.shape[0])
    nodes = nodes[perm]
    _, first = np.unique(comp[nodes], return_index=True)
    reps = nodes[first]
    reps.sort()
    add_u = np.empty(reps.shape[0], dtype=np.int64)
    add_v = np.empty(reps.shape[0], dtype=np.int64)
    for t, node in enumerate(reps):
        pool = giant_by_block.get(int(labels[node]), giant_nodes)
        add_u[t] = node
        add_v[t] = pool[int(rng.integers(0, pool.shape[0]))]
    u = np.concatenate([u, add_u])
    v = np.concatenate([v, add_v])
    return u, v, int(reps.shape[0])


def _finish(n: int, u: np.ndarray, v: np.ndarray, labels: np.ndarray,
            rng: np.random.Generator, meta: dict, permute: bool = True) -> Graph:
    u, v = _canonical_unique(n, u.astype(np.int64), v.astype(np.int64))
    u, v, added = _connect(n, u, v, labels, rng)
    meta = dict(meta)
    meta["connect_edges_added"] = added
    if permute:
        perm = rng.permutation(n)  # old id -> new id
        u = perm[u]
        v = perm[v]
        new_labels = np.empty_like(labels)
        new_labels[perm] = labels
        labels = new_labels
    row_ptr, cols = _edges_to_csr(n, u, v)
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return Graph(n=n, row_ptr=row_ptr.astype(np.int32), col_idx=cols.astype(np.int32),
                 labels=labels.astype(np.int32), meta=meta)


# ----------------------------------------------------------------------------
# generators
# ----------------------------------------------------------------------------

def sbm_plain(sizes: Sequence[int], dbar: float, r: float, rng: np.random.Generator,
              permute: bool = True) -> Graph:
    """Plain SBM.  p_in and p_out are global and set so that the expected mean
    degree is ``dbar`` and the expected inter/intra edge-count ratio is ``r``;
    each block pair draws m ~ Binomial(#pairs, p) and then m distinct pairs
    uniformly at random (exact G(n, p) per block pair)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    n = int(sizes.sum())
    kb = sizes.shape[0]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    labels = np.repeat(np.arange(kb, dtype=np.int32), sizes)
    intra_pairs = float((sizes * (sizes - 1) // 2).sum())
    inter_pairs = float((sizes.sum() ** 2 - (sizes ** 2).sum()) // 2)
    e_total = n * dbar / 2.0
    p_in = e_total / (1.0 + r) / intra_pairs
    p_out = (e_total * r / (1.0 + r) / inter_pairs) if inter_pairs > 0 else 0.0
    if p_in > 1.0 or p_out > 1.0:
        raise ValueError("edge probabilities exceed 1 for these sizes")
    us: List[np.ndarray] = []
    vs: List[np.ndarray] = []
    for b in range(kb):
        nb = int(sizes[b])
        pairs = nb * (nb - 1) // 2
        m = int(rng.binomial(pairs, p_in)) if pairs > 0 else 0
        idx = _choose_distinct(rng, pairs, m)
        uu, vv = _tri_unrank(idx, nb)
        us.append(uu + offs[b])
        vs.append(vv + offs[b])
        for c in range(b + 1, kb):
            nc = int(sizes[c])
            pairs = nb * nc
            m = int(rng.binomial(pairs, p_out)) if p_out > 0 else 0
            idx = _choose_distinct(rng, pairs, m)
            us.append(idx // nc + offs[b])
            vs.append(idx % nc + offs[c])
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    meta = {"kind": "sbm", "dbar": dbar, "r": r, "p_in": p_in, "p_out": p_out,
            "sizes": sizes.tolist()}
    return _finish(n, u, v, labels, rng, meta, permute=permute)


def _powerlaw_theta(nb: int, rng: np.random.Generator, exponent: float, ratio: float):
    """theta ~ pdf proportional to theta^-exponent on [1, c], with c chosen so
    that c / E[theta] = ratio; returned normalised to mean 1."""
    a = exponent - 1.0

    def mean(c):
        # mean of the truncated power law on [1, c]
        if abs(exponent - 2.0) < 1e-12:
            return math.log(c) / (1.0 - 1.0 / c)
        return (a / (a - 1.0)) * (1.0 - c ** (1.0 - a)) / (1.0 - c ** (-a))

    lo, hi = 1.0 + 1e-9, 1e9
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if mid / mean(mid) < ratio:
            lo = mid
        else:
            hi = mid
    c = lo
    u = rng.random(nb)
    # inverse CDF of the truncated power law
    theta = (1.0 - u * (1.0 - c ** (-a))) ** (-1.0 / a)
    return theta / theta.mean(), c


def dcsbm_powerlaw(sizes: Sequence[int], dbar: float, r: float, rng: np.random.Generator,
                   exponent: float = 2.5, permute: bool = True) -> Graph:
    """Degree-corrected SBM.  Inside each block, theta_i follows a truncated
    power law (pdf ~ theta^-exponent) whose cutoff makes the largest expected
    degree sqrt(n_b * dbar) (structural cutoff); theta is normalised to mean 1
    per block.  Each block pair draws m ~ Poisson(mu_bc) edges whose endpoints
    are chosen with probability proportional to theta inside their block; then
    self-loops and duplicates are dropped."""
    sizes = np.asarray(sizes, dtype=np.int64)
    n = int(sizes.sum())
    kb = sizes.shape[0]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    labels = np.repeat(np.arange(kb, dtype=np.int32), sizes)
    e_total = n * dbar / 2.0
    e_intra = e_total / (1.0 + r)
    e_inter = e_total * r / (1.0 + r)
    intra_w = sizes.astype(np.float64) ** 2
    intra_w /= intra_w.sum()
    inter_w = np.outer(sizes, sizes).astype(np.float64)
    np.fill_diagonal(inter_w, 0.0)
    inter_w = np.triu(inter_w)
    inter_w /= max(inter_w.sum(), 1.0)
    cdfs = []
    cut = []
    for b in range(kb):
        nb = int(sizes[b])
        ratio = math.sqrt(nb * dbar) / dbar
        theta, c = _powerlaw_theta(nb, rng, exponent, ratio)
        cut.append(c)
        cdf = np.cumsum(theta)
        cdfs.append(cdf / cdf[-1])

    def draw(b, m):
        x = rng.random(m)
        return np.searchsorted(cdfs[b], x, side="right").clip(0, int(sizes[b]) - 1) + offs[b]

    us: List[np.ndarray] = []
    vs: List[np.ndarray] = []
    for b in range(kb):
        m = int(rng.poisson(e_intra * intra_w[b]))
        us.append(draw(b, m))
        vs.append(draw(b, m))
        for c in range(b + 1, kb):
            m = int(rng.poisson(e_inter * inter_w[b, c]))
            us.append(draw(b, m))
            vs.append(draw(c, m))
    u = np.concatenate(us)
    v = np.concatenate(vs)
    meta = {"kind": "dcsbm", "dbar": dbar, "r": r, "exponent": exponent,
            "theta_cut": cut[0], "sizes": sizes.tolist()}
    return _finish(n, u, v, labels, rng, meta, permute=permute)


def relabel(g: Graph, order: np.ndarray) -> Graph:
    """The same graph with old node ``order[i]`` renamed ``i`` (``order`` a
    permutation of 0..n-1): rows taken in that order, column ids mapped, each
    row's columns sorted.  A node order is a storage choice, not part of the
    method (rows of X are permuted with it)."""
    n = g.n
    order = np.asarray(order, dtype=np.int64)
    inv = np.empty(n, dtype=np.int64)
    inv[order] = np.arange(n, dtype=np.int64)
    deg = np.diff(g.row_ptr).astype(np.int64)[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=rp[1:])
    src = np.repeat(g.row_ptr[order].astype(np.int64) - rp[:-1], deg) + np.arange(rp[-1])
    key = np.repeat(np.arange(n, dtype=np.int64) * n, deg) + inv[g.col_idx[src]]
    key.sort()
    cols = key % n
    meta = dict(g.meta)
    meta["relabeled"] = True
    return Graph(n=n, row_ptr=rp.astype(np.int32), col_idx=cols.astype(np.int32),
                 labels=g.labels[order], meta=meta)


def hub_first_order(g: Graph) -> np.ndarray:
    """Nodes by degree, descending (ties by id): the rows gathered most often
    get the smallest ids, so they share memory pages."""
    return np.argsort(-np.diff(g.row_ptr).astype(np.int64), kind="stable")


def rcm_order(g: Graph) -> np.ndarray:
    """Reverse Cuthill-McKee order of the (symmetric) pattern (SciPy)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    S = sp.csr_matrix((np.ones(g.nnz, dtype=np.int8), g.col_idx, g.row_ptr), shape=(g.n, g.n))
    return np.asarray(reverse_cuthill_mckee(S, symmetric_mode=True), dtype=np.int64)


def initial_x(n: int, k: int, rng: np.random.Generator) -> np.ndarray:
    """X0 with i.i.d. N(0, 1/n) entries, FP64, row-major n x k."""
    return rng.standard_normal((n, k)) / math.sqrt(n)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

WORKLOADS = {
    # name: recipe; `seed` keys the graph stream ([seed, 1]) and X0 ([seed, 2])
    "sbm-n1000-k8": dict(n=1000, k=8, dbar=16.0, r=0.3, seed=1),
    "sbm-n50k-k32": dict(n=50_000, k=32, dbar=20.0, r=0.4, seed=2),
    "dcsbm-n2m-k32": dict(n=2_000_000, k=32, dbar=25.0, r=0.5, seed=3),
}


def workload(name: str, n: Optional[int] = None):
    """Graph and X0 of a named workload.

    sbm-n1000-k8:  N=1000, k=8, Dirichlet(2) sizes (min 50), mean degree 16,
                   r=0.3; X0 from default_rng(0).
    sbm-n50k-k32:  N=50,000, k=32, LogNormal(0, 0.5) sizes, mean degree 20,
                   r=0.4.
    dcsbm-n2m-k32: N=2,000,000, k=32 equal blocks, degree-corrected power law
                   2.5, mean degree 25, r=0.5.
    ``n`` overrides N (same recipe at another size, for quick tests).
    Returns (graph, X0 float64 [n, k]).
    """
    if name not in WORKLOADS:
        raise ValueError(f"unknown workload {name}")
    spec = WORKLOADS[name]
    nn = int(n if n is not None else spec["n"])
    k = spec["k"]
    seed = spec["seed"]
    grng = np.random.default_rng([seed, 1])
    if name == "sbm-n1000-k8":
        sizes = dirichlet_sizes(nn, k, grng, 2.0, min(50, nn // (2 * k)))
        g = sbm_plain(sizes, spec["dbar"], spec["r"], grng)
        xrng = np.random.default_rng(0)
    elif name == "sbm-n50k-k32":
        sizes = lognormal_sizes(nn, k, grng, 0.5)
        g = sbm_plain(sizes, spec["dbar"], spec["r"], grng)
        xrng = np.random.default_rng([seed, 2])
    else:
        sizes = equal_sizes(nn, k)
        g = dcsbm_powerlaw(sizes, spec["dbar"], spec["r"], grng, 2.5)
        xrng = np.random.default_rng([seed, 2])
    g.meta["workload"] = name if n is None else f"{name}@n{nn}"
    return g, initial_x(nn, k, xrng)


def batched_graph_specs(count: int = 256, seed: int = 5):
    """Per-graph parameters of the batched uneven workload: N ~ U{1000..50000},
    k ~ U{4, 8, 16, 32}, mean degree ~ U[8, 32], r = 0.3, equal blocks."""
    rng = np.random.default_rng([seed, 0])
    specs = []
    for b in range(count):
        specs.append(dict(n=int(rng.integers(1000, 50001)),
                          k=int(rng.choice([4, 8, 16, 32])),
                          dbar=float(rng.uniform(8.0, 32.0)), r=0.3, index=b))
    return specs


def batched_graph(spec: dict, seed: int = 5):
    """Graph and X0 of one member of the batched workload."""
    b = spec["index"]
    grng = np.random.default_rng([seed, b, 1])
    g = sbm_plain(equal_sizes(spec["n"], spec["k"]), spec["dbar"], spec["r"], grng)
    x0 = initial_x(spec["n"], spec["k"], np.random.default_rng([seed, b, 2]))
    return g, x0


def bfs_ball_subgraph(g: Graph, size: int, rng: np.random.Generator) -> Graph:
    """Induced subgraph on the first ``size`` nodes reached by BFS from a random
    start node (connected, so every degree is at least 1)."""
    start = int(rng.integers(0, g.n))
    seen = np.zeros(g.n, dtype=bool)
    order = [start]
    seen[start] = True
    head = 0
    while head < len(order) and len(order) < size:
        x = order[head]
        head += 1
        for y in g.col_idx[g.row_ptr[x]:g.row_ptr[x + 1]]:
            if not seen[y]:
                seen[y] = True
                order.append(int(y))
                if len(order) >= size:
                    break
    nodes = np.array(order[:size], dtype=np.int64)
    remap = -np.ones(g.n, dtype=np.int64)
    remap[nodes] = np.arange(nodes.shape[0])
    us, vs = [], []
    for new, old in enumerate(nodes):
        nb = g.col_idx[g.row_ptr[old]:g.row_ptr[old + 1]].astype(np.int64)
        m = remap[nb]
        m = m[m >= 0]
        us.append(np.full(m.shape[0], new, dtype=np.int64))
        vs.append(m)
    u = np.concatenate(us)
    v = np.concatenate(vs)
    row_ptr, cols = _edges_to_csr(nodes.shape[0], u, v)
    return Graph(n=int(nodes.shape[0]), row_ptr=row_ptr.astype(np.int32),
                 col_idx=cols.astype(np.int32), labels=g.labels[nodes].astype(np.int32),
                 meta={"kind": "bfs-ball", "parent": g.meta.get("workload")})


class GrowthStream:
    """Node-arrival growth process for streaming snapshots.

    Nodes arrive one at a time with a uniform block label.  The first m+1
    arrivals (m = dbar/2) form a clique; every later arrival adds m edges to
    distinct earlier nodes.  Each edge is intra-block with probability
    1/(1+r); its target is uniform among the earlier nodes of the arrival's
    own block (intra) or of the other blocks (inter), or among all earlier
    nodes while that class holds fewer than m nodes.  The mean degree is
    therefore about dbar at every size, older nodes keep gaining edges, and
    every node has degree >= m.

    Node ids are arrival order, so the snapshot with n_s nodes is the
    subgraph induced by ids [0, n_s) and each snapshot extends the previous
    one: a warm start keeps the old rows of X in place and appends rows for
    the new nodes.  The arrival order is random with respect to the blocks,
    so storage order does not reveal them.

    The full graph is stored once as a symmetric CSR with sorted columns;
    since an edge (i, j) is present in a snapshot exactly when max(i, j) <
    n_s, each row of a snapshot is a prefix of the same row of the full
    graph, and ``snapshot`` cuts it out with a mask.
    """

    def __init__(self, n_final: int = 2_000_000, stages: int = 10, k: int = 64,
                 dbar: float = 20.0, r: float = 0.3, seed: int = 4):
        self.n_final = int(n_final)
        self.stages = int(stages)
        self.k = int(k)
        self.dbar = float(dbar)
        self.r = float(r)
        m = int(round(dbar / 2))
        self.m = m
        if self.n_final <= m + 1:
            raise ValueError("n_final must exceed dbar/2 + 1")
        rng = np.random.default_rng([seed, 1])
        n = self.n_final
        labels = rng.integers(0, k, size=n).astype(np.int64)
        self.labels = labels.astype(np.int32)
        # rank[a] = number of earlier arrivals in the block of a;
        # members[off[b] + j] = the j-th arrival of block b
        members = np.argsort(labels, kind="stable")
        counts = np.bincount(labels, minlength=k)
        off = np.concatenate([[0], np.cumsum(counts)])
        rank = np.empty(n, dtype=np.int64)
        rank[members] = np.arange(n, dtype=np.int64) - off[labels[members]]

        c = m + 1
        cu, cv = np.tril_indices(c, -1)  # clique among the first m+1 arrivals
        a = np.arange(c, n, dtype=np.int64)  # later arrivals, each with m slots
        na = a.shape[0]
        lab = labels[a]
        own = rank[a]
        intra = rng.random((na, m)) < 1.0 / (1.0 + self.r)
        # classes too small to hold m distinct targets fall back to everyone
        fallback = np.where(intra, (own < m)[:, None], ((a - own) < m)[:, None])
        tgt = np.empty((na, m), dtype=np.int64)
        todo = np.ones((na, m), dtype=bool)
        while True:
            self._draw(rng, tgt, todo, a, lab, own, intra, fallback, labels, members, off)
            srt = np.sort(tgt, axis=1)
            dup_rows = np.flatnonzero((srt[:, 1:] == srt[:, :-1]).any(axis=1))
            if dup_rows.shape[0] == 0:
                break
            todo[:] = False
            sub = tgt[dup_rows]
            # keep the first occurrence of every target in a row, redraw the rest
            order = np.argsort(sub, axis=1, kind="stable")
            ss = np.take_along_axis(sub, order, axis=1)
            rep = np.zeros_like(ss, dtype=bool)
            rep[:, 1:] = ss[:, 1:] == ss[:, :-1]
            redo = np.zeros_like(rep)
            np.put_along_axis(redo, order, rep, axis=1)
            todo[dup_rows] = redo
        u = np.concatenate([cu.astype(np.int64), np.repeat(a, m)])
        v = np.concatenate([cv.astype(np.int64), tgt.reshape(-1)])
        key = np.concatenate([u * n + v, v * n + u])
        key.sort()
        rows = key // n
        self.col_idx = (key % n).astype(np.int32)
        self._rows = rows.astype(np.int32)
        rp = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
        self.row_ptr = rp
        step = n // self.stages
        self.bounds = [step * (s + 1) for s in range(self.stages)]
        self.bounds[-1] = n

    @staticmethod
    def _draw(rng, tgt, todo, a, lab, own, intra, fallback, labels, members, off):
        rows, cols = np.nonzero(todo)
        if rows.shape[0] == 0:
            return
        aa = a[rows]
        fb = fallback[rows, cols]
        it = intra[rows, cols] & ~fb
        inter = ~intra[rows, cols] & ~fb
        out = np.empty(rows.shape[0], dtype=np.int64)
        # any earlier node
        idx = np.flatnonzero(fb)
        out[idx] = (rng.random(idx.shape[0]) * aa[idx]).astype(np.int64)
        # an earlier node of the own block
        idx = np.flatnonzero(it)
        j = (rng.random(idx.shape[0]) * own[rows[idx]]).astype(np.int64)
        out[idx] = members[off[lab[rows[idx]]] + j]
        # an earlier node of another block, by rejection
        idx = np.flatnonzero(inter)
        while idx.shape[0]:
            cand = (rng.random(idx.shape[0]) * aa[idx]).astype(np.int64)
            ok = labels[cand] != lab[rows[idx]]
            out[idx[ok]] = cand[ok]
            idx = idx[~ok]
        tgt[rows, cols] = out

    def snapshot(self, s: int) -> Graph:
        """Snapshot s (0-based): the subgraph on the first bounds[s] arrivals."""
        ns = self.bounds[s]
        end = int(self.row_ptr[ns])
        cols = self.col_idx[:end]
        keep = cols < ns
        cnt = np.bincount(self._rows[:end][keep], minlength=ns)
        rp = np.zeros(ns + 1, dtype=np.int64)
        np.cumsum(cnt, out=rp[1:])
        return Graph(n=ns, row_ptr=rp.astype(np.int32), col_idx=cols[keep].copy(),
                     labels=self.labels[:ns].copy(),
                     meta={"kind": "growth", "stage": s, "dbar": self.dbar, "r": self.r,
                           "m": self.m})


def streaming_snapshots(n_final: int = 2_000_000, stages: int = 10, k: int = 64,
                        dbar: float = 20.0, r: float = 0.3, seed: int = 4):
    """Yields (graph, n_s) for the stages of a ``GrowthStream``."""
    gs = GrowthStream(n_final, stages, k, dbar, r, seed)
    for s in range(gs.stages):
        yield gs.snapshot(s), gs.bounds[s]


class EdgeStream:
    """Edge-sampling stream over a fixed graph: its undirected edges are dealt
    uniformly at random to ``parts`` disjoint parts, and stage s is the graph
    of parts 0..s (the streaming comparison of the numerical results section:
    ten non-overlapping parts of a graph's edges, each stage adding one).

    A stage holds the nodes that have at least one edge so far (a node
    without edges has no D^{-1/2}), renumbered in the order of their ids in
    the full graph; ``ids`` maps a stage's rows to full-graph ids.  Stages are
    nested: every node and edge of stage s is in stage s+1, so a warm start
    carries the previous rows to the positions ``carry`` returns."""

    def __init__(self, g: Graph, parts: int = 10, seed: int = 6):
        self.g = g
        self.parts = int(parts)
        rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
        cols = g.col_idx.astype(np.int64)
        keep = rows < cols
        self.u = rows[keep]
        self.v = cols[keep]
        self.part = np.random.default_rng([seed, 1]).integers(0, self.parts, size=self.u.shape[0])

    def stage(self, s: int):
        """(Graph of parts 0..s on its touched nodes, full-graph ids of its rows)."""
        if not 0 <= s < self.parts:
            raise ValueError("stage out of range")
        m = self.part <= s
        u, v = self.u[m], self.v[m]
        touched = np.zeros(self.g.n, dtype=bool)
        touched[u] = True
        touched[v] = True
        ids = np.flatnonzero(touched).astype(np.int64)
        loc = np.full(self.g.n, -1, dtype=np.int64)
        loc[ids] = np.arange(ids.shape[0], dtype=np.int64)
        n = int(ids.shape[0])
        rp, ci = _edges_to_csr(n, loc[u], loc[v])
        meta = dict(self.g.meta)
        meta.update({"edge_stream_stage": s, "edge_parts": self.parts})
        return Graph(n=n, row_ptr=rp.astype(np.int32), col_idx=ci.astype(np.int32),
                     labels=self.g.labels[ids], meta=meta), ids

    @staticmethod
    def carry(ids_prev: np.ndarray, ids: np.ndarray) -> np.ndarray:
        """Positions in a stage of the previous stage's rows."""
        pos = np.searchsorted(ids, ids_prev)
        if pos.shape[0] and (pos.max() >= ids.shape[0] or np.any(ids[pos] != ids_prev)):
            raise ValueError("stages are not nested")
        return pos


def warm_start(x_prev: Optional[np.ndarray], n: int, k: int, rng: np.random.Generator,
               dtype=np.float64) -> np.ndarray:
    """Initial block for a grown graph: the previous solution's rows in place,
    new rows drawn N(0, 1/n)."""
    x = np.empty((n, k), dtype=dtype)
    old = 0 if x_prev is None else x_prev.shape[0]
    if old:
        x[:old] = x_prev
    x[old:] = rng.standard_normal((n - old, k)) / math.sqrt(n)
    return x
