"""The d = 16 sweep on the matrix cores (plain loss-and-gradient evaluations from n = 8192
on): whole-graph parity against the FP64 oracle on ragged sizes, near pairs (the exact
path), coincident points, the reversed tile order, an all-edge block, and the 1M-vertex
workload at X0 on sampled rows."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import (assert_grad_close, assert_loss_close, check_rows_plain, note, require_gpu, to_dev)
from paper_2011_03479_amd import gempe, synth

pytestmark = pytest.mark.gpu


def _plain(G, X, params=None):
    r = gempe.loss_grad(G, to_dev(X), params=params)
    torch.cuda.synchronize()
    return float(r.loss.item()), r.grad.double().cpu().numpy(), int(r.edge_hits.item())


def _full(g, X, what):
    require_gpu()
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    loss, grad, hits = _plain(G, X)
    ref = oracle.loss_grad(X, g.row_ptr, g.col_idx, want_abs_slope=True)
    assert hits == g.m == ref["edge_hits"], what
    assert_loss_close(loss, ref["loss"], what=what)
    assert_grad_close(grad, ref["grad"], ref["abs_slope"], what=what)
    G.close()
    return loss, ref


@pytest.mark.parametrize("n,kind", [(8192, "cl"), (8229, "er"), (12043, "cl"), (9000, "sbm")])
def test_mfma16_whole_graph(n, kind):
    """Ragged n (a last strip and column block partly past n), several graph kinds, X ~ N(0, 1)."""
    if kind == "cl":
        g = synth.chung_lu(n, 12.0, 2.3, seed=n)
    elif kind == "er":
        g = synth.erdos_renyi(n, 10.0, seed=n)
    else:
        g = synth.sbm(9, n // 9, 5e-3, 5e-5, seed=n)
    X = synth.init_embedding(g.n, 16, seed=n + 16)
    note(f"mfma16 whole graph n={g.n} {kind} m={g.m}")
    _full(g, X, f"mfma16 n{g.n} {kind}")


def test_mfma16_near_pairs_clusters():
    """Tight clusters away from the origin: every pair inside a cluster is near (its squared
    distance is far below kappa (|x_i|^2 + |x_j|^2)) and takes the exact path; pairs across
    clusters stay on the Gram."""
    from test_gpu_bf16 import clusters

    n = 8300
    X, lab = clusters(n, 16, 40, spread=0.1, sep=3.0, seed=7)
    rng = np.random.default_rng(3)
    u = rng.integers(0, n, 3 * n)
    members = [np.nonzero(lab == k)[0] for k in range(40)]
    same = np.array([rng.choice(members[lab[a]]) for a in u[:2 * n]])
    g = synth.csr_from_edges(n, u, np.concatenate([same, rng.integers(0, n, n)]))
    note(f"mfma16 clusters n={n} m={g.m}")
    _full(g, X, "mfma16 clusters")


def test_mfma16_translated_embedding():
    """Every coordinate offset by 40: all pairs are near relative to their norms, so the
    whole sweep runs the exact path; the result meets the FP32 bound (translation invariance
    of DL and G is the oracle's, pinned on the CPU)."""
    n = 8250
    g = synth.chung_lu(n, 10.0, 2.5, seed=11)
    X = (synth.init_embedding(n, 16, seed=12).astype(np.float64) + 40.0).astype(np.float32)
    note("mfma16 translated embedding")
    _full(g, X, "mfma16 translated")


def test_mfma16_coincident_points():
    """All points equal: every pair has delta = 0 (near), dl+(0) per edge and dl-(0) per
    non-edge, gradient 0."""
    n = 8200
    g = synth.erdos_renyi(n, 6.0, seed=13)
    X = np.full((n, 16), 0.75, dtype=np.float32)
    note("mfma16 coincident points")
    loss, ref = _full(g, X, "mfma16 coincident")
    N = n * (n - 1) // 2
    closed = g.m * oracle.pair(0.0, True)[0] + (N - g.m) * oracle.pair(0.0, False)[0]
    assert abs(loss - closed) <= 1e-5 * closed


def test_mfma16_reversed_tile_order():
    n = 9100
    g = synth.chung_lu(n, 10.0, 2.5, seed=17)
    X = synth.init_embedding(n, 16, seed=18)
    note("mfma16 reversed tile order")
    require_gpu()
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    fwd = _plain(G, X)
    rev = _plain(G, X, params=gempe.params_default(flags=gempe.GEMPE_F_REVERSE_TILES))
    assert rev[0] == fwd[0], (rev[0], fwd[0])
    A = oracle.loss_grad(X, g.row_ptr, g.col_idx, want_abs_slope=True)["abs_slope"]
    assert_grad_close(rev[1], fwd[1], A, rtol=1e-5, what="mfma16 reversed")
    G.close()


def test_mfma16_dense_block():
    """A clique on 70 vertices spanning two column blocks plus sparse edges: edges inside the
    diagonal and off-diagonal blocks, at contracted distances (edges near mu)."""
    n = 8256
    rng = np.random.default_rng(19)
    cl = np.arange(30, 100)
    uu, vv = np.meshgrid(cl, cl)
    keep = uu < vv
    u = np.concatenate([uu[keep], rng.integers(0, n, 2 * n)])
    v = np.concatenate([vv[keep], rng.integers(0, n, 2 * n)])
    g = synth.csr_from_edges(n, u, v)
    X = synth.init_embedding(n, 16, seed=20)
    X[cl] = synth.init_embedding(70, 16, seed=21, scale=0.2)
    note(f"mfma16 dense block m={g.m}")
    _full(g, X, "mfma16 dense block")


def test_mfma16_cl1m_sampled_rows():
    """The 1M-vertex workload at X0, plain evaluation: sampled gradient rows (hubs included)
    against the oracle; the loss against the evaluation with row losses."""
    require_gpu()
    w = synth.workload("cl1m")
    g = w.graph
    rng = np.random.default_rng(2)
    hubs = np.argsort(-np.diff(g.row_ptr))[:6]
    rows = np.unique(np.concatenate([rng.choice(g.n, 60, replace=False), hubs, [0, g.n - 1]]))
    note(f"mfma16 cl1m sampled rows, m={g.m}")
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    check_rows_plain(g, G, w.X0, rows, what="mfma16 cl1m")
    G.close()


@pytest.mark.parametrize("n,d", [(4100, 32), (4500, 64), (4160, 128)])
def test_mfma_wide_whole_graph(n, d):
    """d = 32, 64, 128 on the matrix cores (n >= 4096): whole-graph parity, ragged n."""
    g = synth.chung_lu(n, 10.0, 2.4, seed=n + d)
    X = synth.init_embedding(n, d, seed=3 * n + d)
    note(f"mfma wide whole graph n={n} d={d} m={g.m}")
    _full(g, X, f"mfma wide n{n} d{d}")


@pytest.mark.parametrize("d", [32, 128])
def test_mfma_wide_near_pairs(d):
    """Clusters away from the origin (near pairs on the exact path) and, at d = 32, a
    translated embedding (every pair near)."""
    from test_gpu_bf16 import clusters

    n = 4200
    X, lab = clusters(n, d, 30, spread=0.1, sep=3.0, seed=d)
    rng = np.random.default_rng(d)
    u = rng.integers(0, n, 3 * n)
    members = [np.nonzero(lab == k)[0] for k in range(30)]
    same = np.array([rng.choice(members[lab[a]]) for a in u[:2 * n]])
    g = synth.csr_from_edges(n, u, np.concatenate([same, rng.integers(0, n, n)]))
    note(f"mfma wide clusters d={d}")
    _full(g, X, f"mfma wide clusters d{d}")
    if d == 32:
        Xt = (synth.init_embedding(n, d, seed=5).astype(np.float64) + 30.0).astype(np.float32)
        note("mfma wide translated d=32")
        _full(g, Xt, "mfma wide translated d32")


def test_mfma_wide_reversed_tile_order():
    n, d = 4400, 64
    g = synth.chung_lu(n, 10.0, 2.5, seed=23)
    X = synth.init_embedding(n, d, seed=24)
    note("mfma wide reversed tile order")
    require_gpu()
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    fwd = _plain(G, X)
    rev = _plain(G, X, params=gempe.params_default(flags=gempe.GEMPE_F_REVERSE_TILES))
    assert rev[0] == fwd[0], (rev[0], fwd[0])
    A = oracle.loss_grad(X, g.row_ptr, g.col_idx, want_abs_slope=True)["abs_slope"]
    assert_grad_close(rev[1], fwd[1], A, rtol=1e-5, what="mfma wide reversed")
    G.close()
