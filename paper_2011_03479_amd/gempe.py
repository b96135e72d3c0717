"""ctypes binding of libgempe.so (include/gempe.h), argument marshalling only.

Every call here forwards to the HIP library; nothing is computed in Python.  PyTorch is
used for device memory (tensors' data pointers) and streams (torch's current stream).
If the library has not been built the first call raises GempeLibraryMissing: there is no
fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgempe.so")

GEMPE_OK = 0
GEMPE_ERR_ARG = -1
GEMPE_ERR_GRAPH = -2
GEMPE_ERR_NOMEM = -3
GEMPE_ERR_HIP = -4
GEMPE_ERR_NUMERIC = -5
GEMPE_ERR_UNSUPPORTED = -6
GEMPE_ERR_TIMEOUT = -7

GEMPE_FP32 = 0
GEMPE_BF16_GRAM = 1

GEMPE_F_NONE = 0
GEMPE_F_REVERSE_TILES = 1  # FP32 sweeps take their tiles in reverse order

# Every symbol include/gempe.h declares (checked by the tests).
ABI_SYMBOLS = (
    "gempe_params_default",
    "gempe_graph_workspace_bytes",
    "gempe_graph_create",
    "gempe_graph_destroy",
    "gempe_graph_num_vertices",
    "gempe_graph_num_edges",
    "gempe_has_edge",
    "gempe_workspace_bytes",
    "gempe_loss_grad",
    "gempe_loss_grad_noalloc_bytes",
    "gempe_loss_grad_noalloc",
    "gempe_loss_grad_shard",
    "gempe_shard_rows",
    "gempe_step",
    "gempe_embed",
    "gempe_timing_enable",
    "gempe_timing_read",
    "gempe_status_string",
    "gempe_last_error",
    "gempe_wm_terms",
    "gempe_wm_step",
    "gempe_embed_wm",
    "gempe_histogram_workspace_bytes",
    "gempe_distance_histogram",
    "gempe_r2_bound",
    "gempe_sigma_fit",
    "gempe_embed_wm_sigma",
    "gempe_sampled_workspace_bytes",
    "gempe_sampled_step",
    "gempe_embed_sampled",
    "gempe_job_footprint",
    "gempe_server_create",
    "gempe_server_submit",
    "gempe_server_query",
    "gempe_server_wait",
    "gempe_server_get_stats",
    "gempe_server_destroy",
)

GEMPE_JOB_QUEUED = 0
GEMPE_JOB_RUNNING = 1
GEMPE_JOB_DONE = 2
GEMPE_JOB_FAILED = 3


class GempeLibraryMissing(RuntimeError):
    pass


class GempeError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"gempe status {status}: {message}")
        self.status = status


class gempe_params(ctypes.Structure):
    _fields_ = [
        ("mu", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("near_k", ctypes.c_double),
        ("flags", ctypes.c_uint32),
        ("reserved1", ctypes.c_uint32),
    ]


class gempe_job_desc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("d", ctypes.c_int32),
        ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p),
        ("col_idx", ctypes.c_void_p),
        ("X0", ctypes.c_void_p),
        ("iters", ctypes.c_int32),
        ("eta", ctypes.c_float),
        ("params", gempe_params),
        ("release_s", ctypes.c_double),
        ("X_out", ctypes.c_void_p),
        ("loss_hist", ctypes.c_void_p),
    ]


class gempe_job_info(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("batched", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("release_s", ctypes.c_double),
        ("admit_s", ctypes.c_double),
        ("done_s", ctypes.c_double),
        ("footprint", ctypes.c_uint64),
    ]


class gempe_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "admitted", "done", "failed", "rejected", "ticks",
                                              "peak_bytes", "max_concurrent", "budget_bytes")] + \
               [("pairs", ctypes.c_double)]


_lib = None


def load(path: str | None = None):
    """Loads libgempe.so (once) and declares the ABI's signatures."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise GempeLibraryMissing(
            f"{p} is not built; run `python -m paper_2011_03479_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(p)
    vp = ctypes.c_void_p
    st = ctypes.c_int
    P = ctypes.POINTER(gempe_params)
    lib.gempe_params_default.argtypes = [P]
    lib.gempe_params_default.restype = None
    lib.gempe_graph_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64]
    lib.gempe_graph_workspace_bytes.restype = ctypes.c_size_t
    lib.gempe_graph_create.argtypes = [ctypes.c_int32, ctypes.c_int64, vp, vp, vp, ctypes.c_size_t, vp,
                                       ctypes.POINTER(vp)]
    lib.gempe_graph_create.restype = st
    lib.gempe_graph_destroy.argtypes = [vp]
    lib.gempe_graph_destroy.restype = st
    lib.gempe_graph_num_vertices.argtypes = [vp]
    lib.gempe_graph_num_vertices.restype = ctypes.c_int32
    lib.gempe_graph_num_edges.argtypes = [vp]
    lib.gempe_graph_num_edges.restype = ctypes.c_int64
    lib.gempe_has_edge.argtypes = [vp, ctypes.c_int64, vp, vp, vp, vp]
    lib.gempe_has_edge.restype = st
    lib.gempe_workspace_bytes.argtypes = [vp, ctypes.c_int32, P]
    lib.gempe_workspace_bytes.restype = ctypes.c_size_t
    lib.gempe_loss_grad.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, P, vp]
    lib.gempe_loss_grad.restype = st
    lib.gempe_loss_grad_noalloc_bytes.argtypes = [vp, ctypes.c_int32, P]
    lib.gempe_loss_grad_noalloc_bytes.restype = ctypes.c_size_t
    lib.gempe_loss_grad_noalloc.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, P, vp]
    lib.gempe_loss_grad_noalloc.restype = st
    lib.gempe_loss_grad_shard.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int32, vp,
                                          ctypes.c_size_t, P, vp]
    lib.gempe_loss_grad_shard.restype = st
    lib.gempe_shard_rows.argtypes = [vp, ctypes.c_int32, P]
    lib.gempe_shard_rows.restype = ctypes.c_int64
    lib.gempe_step.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_float, vp, vp, ctypes.c_size_t, P, vp]
    lib.gempe_step.restype = st
    lib.gempe_embed.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_float, vp, vp,
                                ctypes.c_size_t, P, vp]
    lib.gempe_embed.restype = st
    lib.gempe_timing_enable.argtypes = [ctypes.c_int32]
    lib.gempe_timing_enable.restype = st
    lib.gempe_timing_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    lib.gempe_timing_read.restype = st
    lib.gempe_status_string.argtypes = [st]
    lib.gempe_status_string.restype = ctypes.c_char_p
    lib.gempe_last_error.argtypes = []
    lib.gempe_last_error.restype = ctypes.c_char_p
    lib.gempe_wm_terms.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, vp, ctypes.c_size_t, P, vp]
    lib.gempe_wm_terms.restype = st
    lib.gempe_wm_step.argtypes = [vp, ctypes.c_int32, vp, vp, vp, ctypes.c_size_t, P, vp]
    lib.gempe_wm_step.restype = st
    lib.gempe_embed_wm.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, vp, vp, ctypes.c_size_t, P, vp]
    lib.gempe_embed_wm.restype = st
    lib.gempe_histogram_workspace_bytes.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    lib.gempe_histogram_workspace_bytes.restype = ctypes.c_size_t
    lib.gempe_distance_histogram.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_float, vp, vp, vp,
                                             ctypes.c_size_t, vp]
    lib.gempe_distance_histogram.restype = st
    lib.gempe_r2_bound.argtypes = [vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_float), vp, ctypes.c_size_t, vp]
    lib.gempe_r2_bound.restype = st
    lib.gempe_sigma_fit.argtypes = [ctypes.c_int32, ctypes.c_float, vp, vp, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    lib.gempe_sigma_fit.restype = st
    lib.gempe_embed_wm_sigma.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_double), vp, vp, ctypes.c_size_t, P, vp]
    lib.gempe_embed_wm_sigma.restype = st
    lib.gempe_sampled_workspace_bytes.argtypes = [vp, ctypes.c_int32]
    lib.gempe_sampled_workspace_bytes.restype = ctypes.c_size_t
    lib.gempe_sampled_step.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_uint64, ctypes.c_int32, vp, vp, vp,
                                       ctypes.c_size_t, P, vp]
    lib.gempe_sampled_step.restype = st
    lib.gempe_embed_sampled.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, vp,
                                        vp, ctypes.c_size_t, P, vp]
    lib.gempe_embed_sampled.restype = st
    lib.gempe_job_footprint.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P]
    lib.gempe_job_footprint.restype = ctypes.c_size_t
    lib.gempe_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(vp)]
    lib.gempe_server_create.restype = st
    lib.gempe_server_submit.argtypes = [vp, ctypes.POINTER(gempe_job_desc), ctypes.POINTER(ctypes.c_int64)]
    lib.gempe_server_submit.restype = st
    lib.gempe_server_query.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(gempe_job_info)]
    lib.gempe_server_query.restype = st
    lib.gempe_server_wait.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(gempe_job_info)]
    lib.gempe_server_wait.restype = st
    lib.gempe_server_get_stats.argtypes = [vp, ctypes.POINTER(gempe_server_stats)]
    lib.gempe_server_get_stats.restype = st
    lib.gempe_server_destroy.argtypes = [vp]
    lib.gempe_server_destroy.restype = st
    if path is None:
        _lib = lib
    return lib


def _check(status: int):
    if status != GEMPE_OK:
        lib = load()
        raise GempeError(status, lib.gempe_last_error().decode())


def params_default(**over) -> gempe_params:
    p = gempe_params()
    load().gempe_params_default(ctypes.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


GEMPE_TK_SWEEP = 0
GEMPE_TK_GRAM = 1
GEMPE_TK_EXACT = 2
GEMPE_TK_EDGES = 3
GEMPE_TK_FULL = 4


def timing_enable(on: bool = True):
    """Brackets the library's kernel launches with HIP events (gempe_timing_enable)."""
    _check(load().gempe_timing_enable(1 if on else 0))


def timing_read(kclass: int) -> tuple[int, float]:
    """(launches, total milliseconds) recorded for one kernel class since the last read."""
    nl = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(load().gempe_timing_read(int(kclass), ctypes.byref(nl), ctypes.byref(ms)))
    return int(nl.value), float(ms.value)


def status_string(s: int) -> str:
    return load().gempe_status_string(int(s)).decode()


def last_error() -> str:
    return load().gempe_last_error().decode()


# ------------------------------------------------------------------------------------
# torch marshalling
# ------------------------------------------------------------------------------------

def _torch():
    import torch

    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# Live handles, closed at interpreter exit before the HIP runtime shuts down (a handle
# released during module teardown could otherwise reach the runtime after its own
# finalisation has begun).
_live = weakref.WeakSet()


@atexit.register
def _close_live_handles():
    for h in list(_live):
        try:
            h.close()
        except Exception:
            pass


class Graph:
    """Owns a gempe_graph handle built from CSR arrays (numpy or CUDA tensors), and the
    device workspace (a torch uint8 tensor) that holds the graph."""

    def __init__(self, n: int, row_ptr, col_idx, device="cuda", stream=None):
        torch = _torch()
        lib = load()
        self.handle = None
        rp = torch.as_tensor(np.asarray(row_ptr, dtype=np.int64) if not torch.is_tensor(row_ptr) else row_ptr,
                             dtype=torch.int64, device=device).contiguous()
        ci = torch.as_tensor(np.asarray(col_idx, dtype=np.int32) if not torch.is_tensor(col_idx) else col_idx,
                             dtype=torch.int32, device=device).contiguous()
        if ci.numel() == 0:
            ci = torch.zeros(1, dtype=torch.int32, device=device)
            nnz = 0
        else:
            nnz = int(ci.numel())
        nbytes = int(lib.gempe_graph_workspace_bytes(int(n), nnz))
        self.mem = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(lib.gempe_graph_create(int(n), nnz, _ptr(rp), _ptr(ci), _ptr(self.mem), nbytes, _stream(stream),
                                      ctypes.byref(h)))
        self.handle = h
        self.n = int(n)
        self.nnz = nnz
        _live.add(self)

    @property
    def m(self) -> int:
        return int(load().gempe_graph_num_edges(self.handle))

    def num_vertices(self) -> int:
        return int(load().gempe_graph_num_vertices(self.handle))

    def close(self):
        """Releases the handle (no device call) and drops the reference to its memory;
        torch reuses that memory only after the work queued on its stream."""
        if getattr(self, "handle", None) is not None and self.handle.value:
            _check(load().gempe_graph_destroy(self.handle))
            self.handle = None
        self.mem = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def graph_create(n, row_ptr, col_idx, stream=None) -> Graph:
    return Graph(n, row_ptr, col_idx, stream=stream)


def has_edge(g: Graph, qi, qj, stream=None):
    torch = _torch()
    qi = torch.as_tensor(qi, dtype=torch.int32, device="cuda").contiguous()
    qj = torch.as_tensor(qj, dtype=torch.int32, device="cuda").contiguous()
    out = torch.empty(qi.numel(), dtype=torch.uint8, device="cuda")
    _check(load().gempe_has_edge(g.handle, int(qi.numel()), _ptr(qi), _ptr(qj), _ptr(out), _stream(stream)))
    return out


def workspace_bytes(g: Graph, d: int, params: gempe_params | None = None) -> int:
    p = params or params_default()
    nbytes = int(load().gempe_workspace_bytes(g.handle, int(d), ctypes.byref(p)))
    if nbytes == 0:
        raise GempeError(GEMPE_ERR_ARG, last_error())
    return nbytes


def workspace(g: Graph, d: int, params: gempe_params | None = None):
    """A torch uint8 CUDA tensor of workspace_bytes (torch allocations are 256-B aligned)."""
    torch = _torch()
    return torch.empty(workspace_bytes(g, d, params), dtype=torch.uint8, device="cuda")


@dataclass
class LossGrad:
    loss: "object"        # float64[1] tensor
    grad: "object"        # float32[n, d] tensor or None
    edge_hits: "object"   # int64[1] tensor or None
    row_loss: "object"    # float32[n] tensor or None


def loss_grad(g: Graph, X, ws=None, params=None, want_grad=True, want_hits=True, want_row_loss=False,
              stream=None, out: LossGrad | None = None) -> LossGrad:
    torch = _torch()
    n, d = X.shape
    p = params or params_default()
    if ws is None:
        ws = workspace(g, d, p)
    if out is None:
        out = LossGrad(
            loss=torch.empty(1, dtype=torch.float64, device="cuda"),
            grad=torch.empty((n, d), dtype=torch.float32, device="cuda") if want_grad else None,
            edge_hits=torch.empty(1, dtype=torch.int64, device="cuda") if want_hits else None,
            row_loss=torch.empty(n, dtype=torch.float32, device="cuda") if want_row_loss else None,
        )
    _check(load().gempe_loss_grad(g.handle, int(d), _ptr(X), _ptr(out.grad), _ptr(out.loss), _ptr(out.edge_hits),
                                  _ptr(out.row_loss), _ptr(ws), int(ws.numel()), ctypes.byref(p), _stream(stream)))
    return out


NOALLOC_SCRATCH_BYTES = 32 << 20  # GEMPE_NOALLOC_SCRATCH_BYTES


def loss_grad_noalloc_bytes(g: Graph, d: int, params=None) -> int:
    p = params or params_default()
    return int(load().gempe_loss_grad_noalloc_bytes(g.handle, int(d), ctypes.byref(p)))


def loss_grad_noalloc(g: Graph, X, params=None, want_hits=True, want_row_loss=False, stream=None,
                      out: LossGrad | None = None) -> LossGrad:
    """gempe_loss_grad_noalloc: the loss and gradient with the library's static scratch
    (no workspace); outputs are allocated here unless `out` is given."""
    torch = _torch()
    n, d = X.shape
    p = params or params_default()
    if out is None:
        out = LossGrad(
            loss=torch.empty(1, dtype=torch.float64, device="cuda"),
            grad=torch.empty((n, d), dtype=torch.float32, device="cuda"),
            edge_hits=torch.empty(1, dtype=torch.int64, device="cuda") if want_hits else None,
            row_loss=torch.empty(n, dtype=torch.float32, device="cuda") if want_row_loss else None,
        )
    _check(load().gempe_loss_grad_noalloc(g.handle, int(d), _ptr(X), _ptr(out.grad), _ptr(out.loss),
                                          _ptr(out.edge_hits), _ptr(out.row_loss), ctypes.byref(p),
                                          _stream(stream)))
    return out


def shard_rows(g: Graph, d: int, params=None) -> int:
    """Strip height of the shard split (gempe_shard_rows)."""
    p = params or params_default()
    return int(load().gempe_shard_rows(g.handle, int(d), ctypes.byref(p)))


def loss_grad_shard(g: Graph, X, shard: int, nshards: int, ws=None, params=None, want_grad=True, stream=None):
    """One shard's share of the loss, gradient and edge hits (gempe_loss_grad_shard)."""
    torch = _torch()
    n, d = X.shape
    p = params or params_default()
    if ws is None:
        ws = workspace(g, d, p)
    out = LossGrad(
        loss=torch.empty(1, dtype=torch.float64, device="cuda"),
        grad=torch.empty((n, d), dtype=torch.float32, device="cuda") if want_grad else None,
        edge_hits=torch.empty(1, dtype=torch.int64, device="cuda"),
        row_loss=None,
    )
    _check(load().gempe_loss_grad_shard(g.handle, int(d), _ptr(X), _ptr(out.grad), _ptr(out.loss),
                                        _ptr(out.edge_hits), int(shard), int(nshards), _ptr(ws), int(ws.numel()),
                                        ctypes.byref(p), _stream(stream)))
    return out


def step(g: Graph, X, eta: float, ws=None, params=None, loss_before=None, stream=None):
    n, d = X.shape
    p = params or params_default()
    if ws is None:
        ws = workspace(g, d, p)
    _check(load().gempe_step(g.handle, int(d), _ptr(X), float(eta), _ptr(loss_before), _ptr(ws), int(ws.numel()),
                             ctypes.byref(p), _stream(stream)))
    return X


def embed(g: Graph, X, iters: int, eta: float, ws=None, params=None, loss_hist=None, stream=None):
    n, d = X.shape
    p = params or params_default()
    if ws is None:
        ws = workspace(g, d, p)
    _check(load().gempe_embed(g.handle, int(d), _ptr(X), int(iters), float(eta), _ptr(loss_hist), _ptr(ws),
                              int(ws.numel()), ctypes.byref(p), _stream(stream)))
    return X


# ------------------------------------------------------------------------------------
# weighted majorization
# ------------------------------------------------------------------------------------

def wm_terms(g: Graph, X, ws=None, params=None, want_grad=True, stream=None):
    """(loss float64[1], grad float32[n, d] or None, z float32[n]) at X."""
    torch = _torch()
    n, d = X.shape
    p = params or params_default()
    if ws is None:
        ws = workspace(g, d, p)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty((n, d), dtype=torch.float32, device="cuda") if want_grad else None
    z = torch.empty(n, dtype=torch.float32, device="cuda")
    _check(load().gempe_wm_terms(g.handle, int(d), _ptr(X), _ptr(grad), _ptr(z), _ptr(loss), _ptr(ws),
                                 int(ws.numel()), ctypes.byref(p), _stream(stream)))
    return loss, grad, z


def wm_step(g: Graph, X, ws=None, params=None, loss_before=None, stream=None):
    n, d = X.shape
    p = params or params_default()
    if ws is None:
        ws = workspace(g, d, p)
    _check(load().gempe_wm_step(g.handle, int(d), _ptr(X), _ptr(loss_before), _ptr(ws), int(ws.numel()),
                                ctypes.byref(p), _stream(stream)))
    return X


def embed_wm(g: Graph, X, iters: int, ws=None, params=None, loss_hist=None, stream=None):
    n, d = X.shape
    p = params or params_default()
    if ws is None:
        ws = workspace(g, d, p)
    _check(load().gempe_embed_wm(g.handle, int(d), _ptr(X), int(iters), _ptr(loss_hist), _ptr(ws),
                                 int(ws.numel()), ctypes.byref(p), _stream(stream)))
    return X


# ------------------------------------------------------------------------------------
# slope optimisation
# ------------------------------------------------------------------------------------

def histogram_workspace(g: Graph, d: int, nbins: int):
    torch = _torch()
    nbytes = int(load().gempe_histogram_workspace_bytes(g.handle, int(d), int(nbins)))
    if nbytes == 0:
        raise GempeError(GEMPE_ERR_ARG, "histogram_workspace_bytes: invalid arguments")
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def r2_bound(g: Graph, X, ws=None, stream=None) -> float:
    torch = _torch()
    n, d = X.shape
    if ws is None:
        ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    out = ctypes.c_float()
    _check(load().gempe_r2_bound(g.handle, int(d), _ptr(X), ctypes.byref(out), _ptr(ws), int(ws.numel()),
                                 _stream(stream)))
    return float(out.value)


def distance_histogram(g: Graph, X, nbins: int, r2_max: float, ws=None, stream=None):
    """(hist_all, hist_edge) as int64 CUDA tensors (the uint64 counts, which fit)."""
    torch = _torch()
    n, d = X.shape
    if ws is None:
        ws = histogram_workspace(g, d, nbins)
    ha = torch.empty(nbins, dtype=torch.int64, device="cuda")
    he = torch.empty(nbins, dtype=torch.int64, device="cuda")
    _check(load().gempe_distance_histogram(g.handle, int(d), _ptr(X), int(nbins), float(r2_max), _ptr(ha), _ptr(he),
                                           _ptr(ws), int(ws.numel()), _stream(stream)))
    return ha, he


def sigma_fit(hist_all, hist_edge, r2_max: float, mu: float = 1.5, sigma_lo: float = 1e-3,
              sigma_hi: float = 1e3) -> float:
    ha = np.ascontiguousarray(hist_all, dtype=np.uint64)
    he = np.ascontiguousarray(hist_edge, dtype=np.uint64)
    out = ctypes.c_double()
    _check(load().gempe_sigma_fit(int(ha.size), float(r2_max), ha.ctypes.data, he.ctypes.data, float(mu),
                                  float(sigma_lo), float(sigma_hi), ctypes.byref(out)))
    return float(out.value)


def embed_wm_sigma(g: Graph, X, iters: int, sigma: float, sigma_every: int = 1, nbins: int = 4096, params=None,
                   loss_hist=None, stream=None) -> float:
    """Weighted majorization with the slope refitted every sigma_every steps; returns the last slope."""
    torch = _torch()
    n, d = X.shape
    p = params or params_default()
    nbytes = workspace_bytes(g, d, p) + int(load().gempe_histogram_workspace_bytes(g.handle, int(d), int(nbins)))
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = ctypes.c_double(float(sigma))
    _check(load().gempe_embed_wm_sigma(g.handle, int(d), _ptr(X), int(iters), int(sigma_every), int(nbins),
                                       ctypes.byref(s), _ptr(loss_hist), _ptr(ws), int(ws.numel()), ctypes.byref(p),
                                       _stream(stream)))
    return float(s.value)


# ------------------------------------------------------------------------------------
# negative sampling
# ------------------------------------------------------------------------------------

def sampled_workspace(g: Graph, d: int):
    torch = _torch()
    nbytes = int(load().gempe_sampled_workspace_bytes(g.handle, int(d)))
    if nbytes == 0:
        raise GempeError(GEMPE_ERR_ARG, "sampled_workspace_bytes: invalid arguments")
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def sampled_step(g: Graph, X, seed: int, max_tries: int = 32, ws=None, params=None, want_samples=False,
                 stream=None):
    """One negative-sampled WM step in place; returns (loss float64[1], samples int32[2 nnz] or None)."""
    torch = _torch()
    n, d = X.shape
    p = params or params_default()
    if ws is None:
        ws = sampled_workspace(g, d)
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    smp = torch.empty(max(2 * g.nnz, 1), dtype=torch.int32, device="cuda") if want_samples else None
    _check(load().gempe_sampled_step(g.handle, int(d), _ptr(X), ctypes.c_uint64(int(seed)), int(max_tries), _ptr(smp),
                                     _ptr(loss), _ptr(ws), int(ws.numel()), ctypes.byref(p), _stream(stream)))
    return loss, (smp[:2 * g.nnz] if smp is not None else None)


def embed_sampled(g: Graph, X, iters: int, seed: int, max_tries: int = 32, ws=None, params=None, loss_hist=None,
                  stream=None):
    n, d = X.shape
    p = params or params_default()
    if ws is None:
        ws = sampled_workspace(g, d)
    _check(load().gempe_embed_sampled(g.handle, int(d), _ptr(X), int(iters), ctypes.c_uint64(int(seed)),
                                      int(max_tries), _ptr(loss_hist), _ptr(ws), int(ws.numel()), ctypes.byref(p),
                                      _stream(stream)))
    return X


# ------------------------------------------------------------------------------------
# serving
# ------------------------------------------------------------------------------------

def job_footprint(n: int, nnz: int, d: int, iters: int, params: gempe_params | None = None) -> int:
    p = params or params_default()
    return int(load().gempe_job_footprint(int(n), int(nnz), int(d), int(iters), ctypes.byref(p)))


@dataclass
class JobInfo:
    state: int
    status: int
    batched: bool
    release_s: float
    admit_s: float
    done_s: float
    footprint: int

    @property
    def latency_s(self) -> float:
        return self.done_s - self.release_s


def _info(i: gempe_job_info) -> JobInfo:
    return JobInfo(int(i.state), int(i.status), bool(i.batched), float(i.release_s), float(i.admit_s),
                   float(i.done_s), int(i.footprint))


class Server:
    """A gempe_server handle.  Inputs are numpy arrays on the host; results are written by
    the library into numpy arrays this object keeps per job until `result` is called."""

    def __init__(self, budget_bytes: int, max_jobs: int = 256):
        self.handle = None
        h = ctypes.c_void_p()
        _check(load().gempe_server_create(int(budget_bytes), int(max_jobs), ctypes.byref(h)))
        self.handle = h
        self._out = {}
        _live.add(self)

    def submit(self, n, row_ptr, col_idx, X0, iters: int, eta: float, params=None, release_s: float = 0.0,
               want_hist: bool = True) -> int:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        x0 = np.ascontiguousarray(X0, dtype=np.float32)
        d = int(x0.shape[1])
        X_out = np.empty_like(x0)
        hist = np.empty(int(iters) + 1, dtype=np.float64) if want_hist else None
        desc = gempe_job_desc()
        desc.n = int(n)
        desc.d = d
        desc.nnz = int(ci.size)
        desc.row_ptr = rp.ctypes.data
        desc.col_idx = ci.ctypes.data if ci.size else None
        desc.X0 = x0.ctypes.data
        desc.iters = int(iters)
        desc.eta = float(eta)
        desc.params = params or params_default()
        desc.release_s = float(release_s)
        desc.X_out = X_out.ctypes.data
        desc.loss_hist = hist.ctypes.data if hist is not None else None
        jid = ctypes.c_int64()
        _check(load().gempe_server_submit(self.handle, ctypes.byref(desc), ctypes.byref(jid)))
        self._out[int(jid.value)] = (X_out, hist)
        return int(jid.value)

    def query(self, job_id: int) -> JobInfo:
        i = gempe_job_info()
        _check(load().gempe_server_query(self.handle, int(job_id), ctypes.byref(i)))
        return _info(i)

    def wait(self, job_id: int = -1, timeout_s: float = -1.0) -> JobInfo | None:
        i = gempe_job_info()
        _check(load().gempe_server_wait(self.handle, int(job_id), float(timeout_s), ctypes.byref(i)))
        return _info(i) if job_id >= 0 else None

    def result(self, job_id: int):
        """(final coordinates, loss history) of a finished job."""
        return self._out[int(job_id)]

    def stats(self) -> dict:
        s = gempe_server_stats()
        _check(load().gempe_server_get_stats(self.handle, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in gempe_server_stats._fields_}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _check(load().gempe_server_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
