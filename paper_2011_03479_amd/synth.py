"""Seeded synthetic inputs: graphs shaped like the paper's workloads and initial embeddings.

This module holds no part of the method's arithmetic.  It draws graphs and starting
coordinates only, so that the GPU path and the CPU oracle can be fed identical inputs.

Every generator uses numpy's PCG64 (``numpy.random.default_rng``).  Vertex ids are
randomly permuted after generation so that tiles of consecutive ids do not line up with
blocks or hubs (the paper renames vertices randomly before hashing, Sec. III-C; here the
renaming only de-correlates structure from the id order).

Graphs are returned as symmetric CSR: ``row_ptr`` int64[n+1], ``col_idx`` int32[2m],
every undirected edge stored in both directions, rows sorted ascending, no self-loops, no
duplicates (the problem statement of Sec. II-A: undirected, unweighted, unlabeled edges).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col_idx: np.ndarray  # int32[nnz]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def edges_upper(self) -> np.ndarray:
        """(m, 2) int64 array of the undirected edges with i < j, sorted."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        cols = self.col_idx.astype(np.int64)
        keep = rows < cols
        return np.stack([rows[keep], cols[keep]], axis=1)


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray, name: str = "", meta=None) -> Graph:
    """Symmetric sorted CSR from an undirected edge list (self-loops and repeats dropped)."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = np.unique(a * n + b)
    a = key // n
    b = key % n
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    order = np.argsort(src * n + dst, kind="stable")
    src, dst = src[order], dst[order]
    counts = np.bincount(src, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr, col_idx=dst.astype(np.int32), name=name, meta=dict(meta or {}))


def _permute(n: int, u: np.ndarray, v: np.ndarray, rng) -> tuple[np.ndarray, np.ndarray]:
    perm = rng.permutation(n).astype(np.int64)
    return perm[u], perm[v]


def bernoulli_positions(total: int, p: float, rng) -> np.ndarray:
    """Sorted positions in [0, total), each kept independently with probability p.

    Geometric skipping (Batagelj and Brandes, Phys. Rev. E 71, 036113, 2005): the gap
    between successive kept positions is geometric with parameter p.
    """
    if total <= 0 or p <= 0.0:
        return np.zeros(0, dtype=np.int64)
    if p >= 1.0:
        return np.arange(total, dtype=np.int64)
    out = []
    pos = -1
    expect = max(16, int(total * p * 1.1) + 64)
    while True:
        gaps = rng.geometric(p, size=expect).astype(np.int64)
        cand = pos + np.cumsum(gaps)
        inside = cand < total
        out.append(cand[inside])
        if not inside.all():
            break
        pos = int(cand[-1])
    return np.concatenate(out)


def _upper_index_to_pair(n: int, L: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Row-major linear index over {(i, j): 0 <= i < j < n} -> (i, j)."""
    L = L.astype(np.int64)
    # row i starts at s(i) = i*(2n - i - 1)/2
    nf = float(n)
    i = np.floor((2 * nf - 1 - np.sqrt((2 * nf - 1) ** 2 - 8.0 * L)) / 2).astype(np.int64)
    i = np.clip(i, 0, n - 2)

    def start(ii):
        return ii * (2 * n - ii - 1) // 2

    # integer fix-up of the floating-point row estimate
    for _ in range(3):
        too_big = start(i) > L
        i = np.where(too_big, i - 1, i)
        nxt = start(i + 1) <= L
        i = np.where(nxt, i + 1, i)
    j = L - start(i) + i + 1
    return i, j


def erdos_renyi(n: int, mean_degree: float, seed: int, permute: bool = True) -> Graph:
    """G(n, p) with p = mean_degree / (n - 1), over the upper triangle."""
    rng = np.random.default_rng(seed)
    p = mean_degree / (n - 1)
    N = n * (n - 1) // 2
    pos = bernoulli_positions(N, p, rng)
    u, v = _upper_index_to_pair(n, pos)
    if permute:
        u, v = _permute(n, u, v, rng)
    return csr_from_edges(n, u, v, name=f"er_n{n}_k{mean_degree:g}_s{seed}",
                          meta=dict(kind="er", p=p, seed=seed, expected_m=p * N))


def chung_lu_weights(n: int, mean_degree: float, gamma: float) -> np.ndarray:
    """Expected degrees w_i ~ (i+1)^(-1/(gamma-1)), capped at sqrt(sum w), mean rescaled."""
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (gamma - 1.0))
    for _ in range(5):
        w *= mean_degree / w.mean()
        w = np.minimum(w, math.sqrt(w.sum()))
    w *= mean_degree / w.mean()
    return w


def _chung_lu_pairs(w_sorted: np.ndarray, rng) -> tuple[np.ndarray, np.ndarray]:
    """Edges with P[(u,v)] = min(1, w_u w_v / S) for u < v, weights sorted descending.

    Miller and Hagberg, "Efficient generation of networks with given expected degrees"
    (WAW 2011): per row u, skip geometrically under the current bound p and accept with
    q/p, where q is the true probability at the landing column.  All rows advance
    together (vectorised over u); the distribution is the one of the sequential method.
    """
    n = w_sorted.shape[0]
    S = w_sorted.sum()
    u = np.arange(n - 1, dtype=np.int64)
    v = u + 1
    p = np.minimum(w_sorted[u] * w_sorted[v] / S, 1.0)
    active = p > 0
    eu, ev = [], []
    while True:
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        pu = p[idx]
        r = rng.random(idx.size)
        with np.errstate(divide="ignore", invalid="ignore"):
            skip = np.where(pu < 1.0, np.floor(np.log(r) / np.log1p(-pu)), 0.0)
        skip = np.minimum(np.nan_to_num(skip, nan=float(n), posinf=float(n)), float(n))
        vv = v[idx] + skip.astype(np.int64)
        inside = vv < n
        idx_in = idx[inside]
        vv_in = vv[inside]
        q = np.minimum(w_sorted[u[idx_in]] * w_sorted[vv_in] / S, 1.0)
        r2 = rng.random(idx_in.size)
        acc = r2 < q / p[idx_in]
        eu.append(u[idx_in][acc])
        ev.append(vv_in[acc])
        p[idx_in] = q
        v[idx_in] = vv_in + 1
        active[idx[~inside]] = False
        active[idx_in[(vv_in + 1 >= n) | (q <= 0)]] = False
    if eu:
        return np.concatenate(eu), np.concatenate(ev)
    return np.zeros(0, np.int64), np.zeros(0, np.int64)


def chung_lu(n: int, mean_degree: float, gamma: float, seed: int, permute: bool = True) -> Graph:
    rng = np.random.default_rng(seed)
    w = chung_lu_weights(n, mean_degree, gamma)  # already descending
    u, v = _chung_lu_pairs(w, rng)
    if permute:
        u, v = _permute(n, u, v, rng)
    return csr_from_edges(n, u, v, name=f"cl_n{n}_k{mean_degree:g}_g{gamma:g}_s{seed}",
                          meta=dict(kind="chung_lu", gamma=gamma, seed=seed,
                                    expected_m=float(w.sum() / 2)))


def sbm(blocks: int, block_size: int, p_in: float, p_out: float, seed: int,
        permute: bool = True) -> Graph:
    """Stochastic block model with equal blocks (geometric skipping per block pair)."""
    rng = np.random.default_rng(seed)
    B = block_size
    n = blocks * B
    us, vs = [], []
    for a in range(blocks):
        pos = bernoulli_positions(B * (B - 1) // 2, p_in, rng)
        i, j = _upper_index_to_pair(B, pos)
        us.append(i + a * B)
        vs.append(j + a * B)
    for a in range(blocks):
        for b in range(a + 1, blocks):
            pos = bernoulli_positions(B * B, p_out, rng)
            us.append(a * B + pos // B)
            vs.append(b * B + pos % B)
    u = np.concatenate(us)
    v = np.concatenate(vs)
    if permute:
        u, v = _permute(n, u, v, rng)
    pin = blocks * B * (B - 1) / 2
    pout = blocks * (blocks - 1) / 2 * B * B
    return csr_from_edges(n, u, v, name=f"sbm_{blocks}x{B}_s{seed}",
                          meta=dict(kind="sbm", p_in=p_in, p_out=p_out, seed=seed,
                                    expected_m=pin * p_in + pout * p_out))


def init_embedding(n: int, d: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """i.i.d. N(0, scale^2) drawn in float64, returned rounded to float32 (row-major n x d)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, d)) * scale).astype(np.float32)


# --------------------------------------------------------------------------------------
# Workloads.  Graph seed s, initial-embedding seed 1000 + s.
# --------------------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    graph: Graph
    d: int
    X0: np.ndarray  # float32 (n, d)
    iters: int
    eta: float
    precision: str  # "fp32" | "bf16"
    mu: float = 1.5
    sigma: float = 1.0

    @property
    def pairs_per_iter(self) -> int:
        n = self.graph.n
        return n * (n - 1) // 2


def step_size(n: int) -> float:
    """Fixed gradient step 0.1 / (n - 1) (the workloads only say "fixed step size")."""
    return 0.1 / (n - 1)


def workload(name: str) -> Workload:
    """The workloads: er1k, cl3400, sbm100k, cl1m (and its bf16 and d = 2 variants)."""
    if name == "er1k":  # Erdos-Renyi n=1000, mean degree 10, d=2, 100 iterations
        g = erdos_renyi(1000, 10.0, seed=1)
        return Workload(name, g, 2, init_embedding(1000, 2, 1001), 100, step_size(1000), "fp32")
    if name == "cl3400":  # Chung-Lu n=3400, ~19,000 edges, gamma 2.5, d=2, 1000 iterations
        g = chung_lu(3400, 2 * 19000 / 3400, 2.5, seed=2)
        return Workload(name, g, 2, init_embedding(3400, 2, 1002), 1000, step_size(3400), "fp32")
    if name == "sbm100k":  # SBM 50 x 2000, p_in 2e-3, p_out 2e-5, d=128, bf16 Gram, 20 iterations
        g = sbm(50, 2000, 2e-3, 2e-5, seed=3)
        return Workload(name, g, 128, init_embedding(g.n, 128, 1003), 20, step_size(g.n), "bf16")
    if name == "sbm100k_fp32":  # the SBM workload with every pair in FP32 (the other side of FP32 vs BF16)
        g = sbm(50, 2000, 2e-3, 2e-5, seed=3)
        return Workload(name, g, 128, init_embedding(g.n, 128, 1003), 20, step_size(g.n), "fp32")
    if name == "sbm100k_t9":  # the same graph from a contracted start: X0 ~ N(0, (mu / sqrt(2d))^2),
        # so that the typical distance is about mu and nearly every pair is near
        g = sbm(50, 2000, 2e-3, 2e-5, seed=3)
        return Workload(name, g, 128, init_embedding(g.n, 128, 1003, scale=1.5 / math.sqrt(2 * 128)), 20,
                        step_size(g.n), "bf16")
    if name in ("cl1m", "cl1m_bf16", "cl1m_d2"):  # Chung-Lu n=1e6, mean 20, gamma 2.3, d=16, 5 iterations
        g = chung_lu(1_000_000, 20.0, 2.3, seed=4)
        prec = "bf16" if name.endswith("bf16") else "fp32"
        d = 2 if name.endswith("d2") else 16   # d2: the drawing dimension on the large graph
        return Workload(name, g, d, init_embedding(g.n, d, 1004), 5, step_size(g.n), prec)
    raise KeyError(name)


@dataclass
class Job:
    job_id: int
    arrival_s: float
    graph: Graph
    d: int
    X0: np.ndarray
    iters: int
    eta: float
    precision: str


def serving_stream(num_jobs: int, rate_per_s: float, seed: int = 5, n_min: int = 500,
                   n_max: int = 50_000, iters: int = 200, dims=(2, 16, 128)) -> list[Job]:
    """Poisson stream of embedding requests (the serving mix).

    n log-uniform in [n_min, n_max]; Erdos-Renyi or Chung-Lu (gamma 2.5) with mean degree
    U[8, 30]; d uniform over ``dims``; bf16 Gram for d >= 64, fp32 otherwise.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for k in range(num_jobs):
        t += rng.exponential(1.0 / rate_per_s)
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        kdeg = float(rng.uniform(8.0, 30.0))
        gseed = int(rng.integers(1 << 30))
        if rng.random() < 0.5:
            g = erdos_renyi(n, kdeg, seed=gseed)
        else:
            g = chung_lu(n, kdeg, 2.5, seed=gseed)
        d = int(dims[int(rng.integers(len(dims)))])
        X0 = init_embedding(n, d, 1000 + gseed)
        jobs.append(Job(k, t, g, d, X0, iters, step_size(n), "bf16" if d >= 64 else "fp32"))
    return jobs
