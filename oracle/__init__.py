"""FP64 CPU oracle for the all-pairs GEMPE loss and gradient (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline leg
of the benchmark, never by the library.  The arithmetic lives in ``gempe_oracle.c`` (plain
C, double precision, brute force over all pairs); this module compiles it with gcc and
marshals numpy arrays.  It imports nothing from the GPU package.

Functions follow Sec. II-B (s+/-, dl+/-, Eq. 2) and Sec. II-C (Eqs. 3-5) of the paper;
see the header comment of ``gempe_oracle.c`` for the exact definitions and readings.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gempe_oracle.c")
_LIB = os.path.join(_HERE, "libgempe_oracle.so")
_lib = None

LN2 = float(np.log(2.0))


def compile_source(src: str, out: str) -> str:
    """gcc -O2 -fopenmp build of an oracle source file into a shared library (IEEE math)."""
    tmp = out + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle (always when force=True, else only if the source is newer)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB)
    return _LIB


def source_path() -> str:
    return _SRC


def _bind(path: str):
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_pair.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                dp, dp, dp]
    lib.oracle_pair.restype = None
    lib.oracle_rows.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64p, i32p, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int, i64p, dp, dp, dp, i64p, dp, dp, dp]
    lib.oracle_rows.restype = None
    lib.oracle_loss_grad.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64p, i32p, ctypes.c_double,
                                     ctypes.c_double, dp, dp, i64p, dp, dp]
    lib.oracle_loss_grad.restype = None
    lib.oracle_loss_grad_shard.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64p, i32p, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_double), dp, ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_loss_grad_shard.restype = None
    lib.oracle_rows_shard.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64p, i32p, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, i64p, dp]
    lib.oracle_rows_shard.restype = None
    u64p = ctypes.POINTER(ctypes.c_uint64)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.oracle_histogram.argtypes = [ctypes.c_int, ctypes.c_int, fp, i64p, i32p, ctypes.c_int, ctypes.c_float,
                                     u64p, u64p]
    lib.oracle_histogram.restype = None
    lib.oracle_sigma_hist.argtypes = [ctypes.c_int, ctypes.c_double, u64p, u64p, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.oracle_sigma_hist.restype = ctypes.c_double
    lib.oracle_sigma_exact.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64p, i32p, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int]
    lib.oracle_sigma_exact.restype = ctypes.c_double
    lib.oracle_sample_pairs.argtypes = [ctypes.c_int, i64p, i32p, ctypes.c_uint64, ctypes.c_int, i32p]
    lib.oracle_sample_pairs.restype = None
    lib.oracle_sampled_step.argtypes = [ctypes.c_int, ctypes.c_int, dp, i64p, i32p, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_uint64, ctypes.c_int, dp, dp, i32p]
    lib.oracle_sampled_step.restype = None
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _bind(_LIB)
    return _lib


def use_library(path):
    """Point this module at another build of the oracle source (None: the default build).

    Used by the tests that plant a mistake in a copy of the oracle source and check that
    the pins catch it.
    """
    global _lib
    _lib = None if path is None else _bind(path)


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(t: int) -> None:
    _load().oracle_set_num_threads(int(t))


def pair(delta: float, is_edge: bool, mu: float = 1.5, sigma: float = 1.0):
    """(dl, d dl/d delta, d^2 dl/d delta^2) of one vertex pair, dl in bits."""
    lib = _load()
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib.oracle_pair(float(delta), int(bool(is_edge)), float(mu), float(sigma),
                    ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


def _graph_arrays(row_ptr, col_idx):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    return rp, ci


def loss_grad(X, row_ptr, col_idx, mu: float = 1.5, sigma: float = 1.0, want_grad=True,
              want_row_loss=False, want_abs_slope=False):
    """DL (bits), gradient (n x d), edge hits, optional per-vertex row loss and
    A_i = sum_j |d dl_ij / d delta| (the magnitude of the terms that cancel in g_i); FP64."""
    lib = _load()
    Xd = np.ascontiguousarray(X, dtype=np.float64)
    n, d = Xd.shape
    rp, ci = _graph_arrays(row_ptr, col_idx)
    loss = ctypes.c_double()
    hits = ctypes.c_int64()
    G = np.zeros((n, d), dtype=np.float64) if want_grad else None
    RL = np.zeros(n, dtype=np.float64) if want_row_loss else None
    AS = np.zeros(n, dtype=np.float64) if want_abs_slope else None
    lib.oracle_loss_grad(n, d, _ptr(Xd, ctypes.c_double), _ptr(rp, ctypes.c_int64),
                         _ptr(ci, ctypes.c_int32), float(mu), float(sigma), ctypes.byref(loss),
                         _ptr(G, ctypes.c_double), ctypes.byref(hits), _ptr(RL, ctypes.c_double),
                         _ptr(AS, ctypes.c_double))
    out = {"loss": loss.value, "edge_hits": hits.value}
    if want_grad:
        out["grad"] = G
    if want_row_loss:
        out["row_loss"] = RL
    if want_abs_slope:
        out["abs_slope"] = AS
    return out


def loss_grad_shard(X, row_ptr, col_idx, strip_rows: int, nshards: int, shard: int, mu: float = 1.5,
                    sigma: float = 1.0):
    """One shard of the pair sum (strips of strip_rows rows, strip q paired with S-1-q, pair p
    owned by shard p mod nshards): {"loss", "grad", "edge_hits"} over the shard's pairs; FP64."""
    lib = _load()
    Xd = np.ascontiguousarray(X, dtype=np.float64)
    n, d = Xd.shape
    rp, ci = _graph_arrays(row_ptr, col_idx)
    loss = ctypes.c_double()
    hits = ctypes.c_int64()
    G = np.zeros((n, d), dtype=np.float64)
    lib.oracle_loss_grad_shard(n, d, _ptr(Xd, ctypes.c_double), _ptr(rp, ctypes.c_int64), _ptr(ci, ctypes.c_int32),
                               float(mu), float(sigma), int(strip_rows), int(nshards), int(shard),
                               ctypes.byref(loss), _ptr(G, ctypes.c_double), ctypes.byref(hits))
    return {"loss": loss.value, "grad": G, "edge_hits": hits.value}


def rows_shard(X, row_ptr, col_idx, rows_idx, strip_rows: int, nshards: int, shard: int, mu: float = 1.5,
               sigma: float = 1.0):
    """Gradient rows (r x d) of one shard (see loss_grad_shard) for a subset of rows; FP64."""
    lib = _load()
    Xd = np.ascontiguousarray(X, dtype=np.float64)
    n, d = Xd.shape
    rp, ci = _graph_arrays(row_ptr, col_idx)
    ri = np.ascontiguousarray(rows_idx, dtype=np.int64)
    G = np.zeros((ri.shape[0], d))
    lib.oracle_rows_shard(n, d, _ptr(Xd, ctypes.c_double), _ptr(rp, ctypes.c_int64), _ptr(ci, ctypes.c_int32),
                          float(mu), float(sigma), int(strip_rows), int(nshards), int(shard), int(ri.shape[0]),
                          _ptr(ri, ctypes.c_int64), _ptr(G, ctypes.c_double))
    return G


def rows(X, row_ptr, col_idx, rows_idx, mu: float = 1.5, sigma: float = 1.0, wm=False):
    """Per-row quantities for a subset of rows, each row against all n vertices.

    Returns grad (r x d), row_loss (r), upper_loss (r), upper_hits (r), abs_slope (r) and,
    with wm=True, z (r) and y (r x d) of Eq. 5.
    """
    lib = _load()
    Xd = np.ascontiguousarray(X, dtype=np.float64)
    n, d = Xd.shape
    rp, ci = _graph_arrays(row_ptr, col_idx)
    ri = np.ascontiguousarray(rows_idx, dtype=np.int64)
    r = ri.shape[0]
    G = np.zeros((r, d))
    L = np.zeros(r)
    U = np.zeros(r)
    H = np.zeros(r, dtype=np.int64)
    Z = np.zeros(r) if wm else None
    Y = np.zeros((r, d)) if wm else None
    AS = np.zeros(r)
    lib.oracle_rows(n, d, _ptr(Xd, ctypes.c_double), _ptr(rp, ctypes.c_int64), _ptr(ci, ctypes.c_int32),
                    float(mu), float(sigma), r, _ptr(ri, ctypes.c_int64), _ptr(G, ctypes.c_double),
                    _ptr(L, ctypes.c_double), _ptr(U, ctypes.c_double), _ptr(H, ctypes.c_int64),
                    _ptr(Z, ctypes.c_double), _ptr(Y, ctypes.c_double), _ptr(AS, ctypes.c_double))
    out = {"grad": G, "row_loss": L, "upper_loss": U, "upper_hits": H, "abs_slope": AS}
    if wm:
        out["z"] = Z
        out["y"] = Y
    return out


def gd_trajectory(X0, row_ptr, col_idx, iters: int, eta: float, mu: float = 1.5,
                  sigma: float = 1.0):
    """Fixed-step gradient descent X <- X - eta * G(X) in FP64.

    Returns (loss history of length iters + 1, final X).  loss[k] is DL at X_k.
    """
    X = np.array(X0, dtype=np.float64)
    hist = []
    for k in range(iters + 1):
        r = loss_grad(X, row_ptr, col_idx, mu, sigma)
        hist.append(r["loss"])
        if k < iters:
            X = X - eta * r["grad"]
    return np.array(hist), X


def wm_update(X, row_ptr, col_idx, mu: float = 1.5, sigma: float = 1.0):
    """One weighted-majorization step (Eq. 5): x_i <- y_i / z_i for every vertex."""
    n = np.asarray(X).shape[0]
    r = rows(X, row_ptr, col_idx, np.arange(n), mu, sigma, wm=True)
    return r["y"] / r["z"][:, None], r


def wm_trajectory(X0, row_ptr, col_idx, iters: int, mu: float = 1.5, sigma: float = 1.0):
    """Weighted-majorization iterations at fixed mu, sigma (Sec. II-C: parabola parameters for
    every pair, then Eq. 5 for every vertex), FP64.  Returns (loss history, final X)."""
    X = np.array(X0, dtype=np.float64)
    hist = []
    for k in range(iters + 1):
        hist.append(loss_grad(X, row_ptr, col_idx, mu, sigma, want_grad=False)["loss"])
        if k < iters:
            X, _ = wm_update(X, row_ptr, col_idx, mu, sigma)
    return np.array(hist), X


# ------------------------------------------------------------------------------------
# slope optimisation (Sec. III-F)
# ------------------------------------------------------------------------------------

SIGMA_LO, SIGMA_HI, SIGMA_ITERS = 1e-3, 1e3, 200


def histogram(X32, row_ptr, col_idx, nbins: int, r2_max: float):
    """(all-pair counts, edge counts) per squared-distance bin, from single-precision X."""
    lib = _load()
    Xf = np.ascontiguousarray(X32, dtype=np.float32)
    n, d = Xf.shape
    rp, ci = _graph_arrays(row_ptr, col_idx)
    ha = np.zeros(nbins, dtype=np.uint64)
    he = np.zeros(nbins, dtype=np.uint64)
    inv_w = np.float32(nbins / r2_max)
    lib.oracle_histogram(n, d, Xf.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _ptr(rp, ctypes.c_int64),
                         _ptr(ci, ctypes.c_int32), int(nbins), float(inv_w),
                         ha.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                         he.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return ha, he


def sigma_from_histogram(hist_all, hist_edge, r2_max: float, mu: float = 1.5, lo=SIGMA_LO, hi=SIGMA_HI,
                         iters=SIGMA_ITERS) -> float:
    lib = _load()
    ha = np.ascontiguousarray(hist_all, dtype=np.uint64)
    he = np.ascontiguousarray(hist_edge, dtype=np.uint64)
    return float(lib.oracle_sigma_hist(int(ha.size), float(r2_max), ha.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                       he.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), float(mu), float(lo),
                                       float(hi), int(iters)))


def sigma_exact(X, row_ptr, col_idx, mu: float = 1.5, lo=SIGMA_LO, hi=SIGMA_HI, iters=SIGMA_ITERS) -> float:
    """The sigma where d DL / d sigma = 0 over every pair (FP64, no histogram)."""
    lib = _load()
    Xd = np.ascontiguousarray(X, dtype=np.float64)
    n, d = Xd.shape
    rp, ci = _graph_arrays(row_ptr, col_idx)
    return float(lib.oracle_sigma_exact(n, d, _ptr(Xd, ctypes.c_double), _ptr(rp, ctypes.c_int64),
                                        _ptr(ci, ctypes.c_int32), float(mu), float(lo), float(hi), int(iters)))


# ------------------------------------------------------------------------------------
# negative sampling (Sec. III-C)
# ------------------------------------------------------------------------------------

def sample_pairs(row_ptr, col_idx, n: int, seed: int, max_tries: int = 32):
    """int32[2 nnz]: the sampled non-neighbours of both ends of every entry with i < j."""
    lib = _load()
    rp, ci = _graph_arrays(row_ptr, col_idx)
    out = np.empty(2 * max(int(rp[-1]), 1), dtype=np.int32)
    lib.oracle_sample_pairs(int(n), _ptr(rp, ctypes.c_int64), _ptr(ci, ctypes.c_int32), ctypes.c_uint64(seed),
                            int(max_tries), _ptr(out, ctypes.c_int32))
    return out[:2 * int(rp[-1])]


def sampled_step(X, row_ptr, col_idx, seed: int, max_tries: int = 32, mu: float = 1.5, sigma: float = 1.0):
    """One negative-sampled weighted-majorization step: (X_new, dl over the pairs used, samples)."""
    lib = _load()
    Xd = np.ascontiguousarray(X, dtype=np.float64)
    n, d = Xd.shape
    rp, ci = _graph_arrays(row_ptr, col_idx)
    Xn = np.empty_like(Xd)
    loss = ctypes.c_double()
    smp = np.empty(2 * max(int(rp[-1]), 1), dtype=np.int32)
    lib.oracle_sampled_step(n, d, _ptr(Xd, ctypes.c_double), _ptr(rp, ctypes.c_int64), _ptr(ci, ctypes.c_int32),
                            float(mu), float(sigma), ctypes.c_uint64(seed), int(max_tries),
                            _ptr(Xn, ctypes.c_double), ctypes.byref(loss), _ptr(smp, ctypes.c_int32))
    return Xn, loss.value, smp[:2 * int(rp[-1])]
