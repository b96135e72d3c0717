"""BF16 MFMA Gram screen (precision GEMPE_BF16_GRAM) against the FP64 oracle."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from gpu_util import (BF16_FLUSH_GRAD, BF16_GRAD_RTOL, BF16_LOSS_RTOL, assert_grad_close, check_full, check_rows,
                      gpu_loss_grad, note, require_gpu,
                      to_dev)
from paper_2011_03479_amd import gempe, synth

pytestmark = pytest.mark.gpu

BF16 = dict(precision=1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()
    oracle.build(force=False)


def clusters(n, d, k, spread, sep, seed):
    """k cluster centres `sep` apart (pairwise far), points N(0, spread^2) around them."""
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((k, d)) * sep
    lab = rng.integers(0, k, n)
    return (centres[lab] + rng.standard_normal((n, d)) * spread).astype(np.float32), lab


@pytest.mark.parametrize("n,d", [(700, 64), (257, 16), (130, 128), (1000, 48)])
def test_bf16_all_near_equals_fp32_bound(n, d):
    """Contracted embedding (typical delta ~ mu): every tile is flagged, the exact FP32
    pass covers everything, so the FP32 bound holds."""
    g = synth.erdos_renyi(n, 8.0, seed=n + d)
    X = synth.init_embedding(n, d, seed=5 * n + d, scale=1.5 / np.sqrt(2 * d))
    note(f"bf16 all-near n={n} d={d}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    check_full(g, G, X, params=gempe.params_default(**BF16), what=f"bf16 near n{n} d{d}")


@pytest.mark.parametrize("n,d", [(3000, 128), (1200, 64), (333, 32)])
def test_bf16_far_init(n, d):
    """N(0,1) init: all non-edge pairs far, only edges matter."""
    g = synth.sbm(6, n // 6, 0.02, 0.001, seed=n)
    n = g.n
    X = synth.init_embedding(n, d, seed=n + 7)
    note(f"bf16 far n={n} d={d}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    check_full(g, G, X, params=gempe.params_default(**BF16), what=f"bf16 far n{n} d{d}",
               loss_rtol=BF16_LOSS_RTOL, grad_rtol=BF16_GRAD_RTOL, grad_atol=(n - 1) * BF16_FLUSH_GRAD)


@pytest.mark.parametrize("n,d", [(1500, 64), (900, 128)])
def test_bf16_clusters_mixed(n, d):
    """Tight clusters far apart: within-cluster tiles are flagged, cross-cluster pairs flushed."""
    X, lab = clusters(n, d, 6, spread=0.12, sep=4.0, seed=n)
    # edges mostly inside clusters
    rng = np.random.default_rng(n)
    u = rng.integers(0, n, 8 * n)
    v = np.where(rng.random(8 * n) < 0.9, u, rng.integers(0, n, 8 * n))
    same = np.array([rng.choice(np.nonzero(lab == lab[a])[0]) for a in u[:4 * n]])
    uu = np.concatenate([u[:4 * n], u[4 * n:]])
    vv = np.concatenate([same, v[4 * n:]])
    g = synth.csr_from_edges(n, uu, vv)
    note(f"bf16 clusters n={n} d={d} m={g.m}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    got, ref = check_full(g, G, X, params=gempe.params_default(**BF16), what=f"bf16 clusters n{n} d{d}",
                          loss_rtol=BF16_LOSS_RTOL, grad_rtol=BF16_GRAD_RTOL, grad_atol=(n - 1) * BF16_FLUSH_GRAD)
    # the flushed pairs are negligible: the result is in fact FP32-accurate
    assert abs(got["loss"] - ref["loss"]) <= 1e-5 * ref["loss"]


def test_bf16_embed_trajectory():
    n, d, iters = 1024, 64, 3
    g = synth.chung_lu(n, 10.0, 2.5, seed=3)
    X0 = synth.init_embedding(n, d, seed=9, scale=0.2)
    eta = 0.1 / (n - 1)
    note("bf16 embed n=1024 d=64 iters=3")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    p = gempe.params_default(**BF16)
    ws = gempe.workspace(G, d, p)
    X = to_dev(X0)
    hist = torch.empty(iters + 1, dtype=torch.float64, device="cuda")
    gempe.embed(G, X, iters, eta, ws=ws, params=p, loss_hist=hist)
    ref_hist, X_ref = oracle.gd_trajectory(X0, g.row_ptr, g.col_idx, iters, eta)
    assert np.allclose(hist.cpu().numpy(), ref_hist, rtol=BF16_LOSS_RTOL, atol=0)
    xg = X.double().cpu().numpy()
    assert np.max(np.linalg.norm(xg - X_ref, axis=1)) <= 1e-3 * np.max(np.linalg.norm(X_ref, axis=1))


def test_sbm100k_sampled_rows():
    """The representation-learning workload at full size (n = 100,000, d = 128, SBM 50 x
    2,000): sampled rows against the oracle, every edge counted once."""
    w = synth.workload("sbm100k")
    g = w.graph
    rng = np.random.default_rng(0)
    hubs = np.argsort(-np.diff(g.row_ptr))[:8]
    rows = np.unique(np.concatenate([rng.choice(g.n, 150, replace=False), hubs, [0, g.n - 1]]))
    note(f"sbm100k sampled rows, m={g.m}")
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    check_rows(g, G, w.X0, rows, params=gempe.params_default(**BF16), what="sbm100k",
               loss_rtol=BF16_LOSS_RTOL, grad_rtol=BF16_GRAD_RTOL, grad_atol=(g.n - 1) * BF16_FLUSH_GRAD)


@pytest.mark.parametrize("n,d", [(40000, 32), (33000, 128)])
def test_bf16_tall_strips_clusters(n, d):
    """n >= 32,768 selects the 512-row screen strips (the last strip partly past n); tight
    clusters make most flagged tiles sparse.  Sampled rows against the oracle."""
    X, lab = clusters(n, d, 40, spread=0.1, sep=3.0, seed=n + d)
    rng = np.random.default_rng(n)
    u = rng.integers(0, n, 3 * n)
    members = [np.nonzero(lab == k)[0] for k in range(40)]
    same = np.array([rng.choice(members[lab[a]]) for a in u[:2 * n]])
    vv = np.concatenate([same, rng.integers(0, n, n)])
    g = synth.csr_from_edges(n, u, vv)
    rows = np.unique(np.concatenate([rng.choice(n, 100, replace=False), [0, n - 1]]))
    note(f"bf16 tall strips n={n} d={d} m={g.m}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    check_rows(g, G, X, rows, params=gempe.params_default(**BF16), what=f"bf16 tall n{n} d{d}",
               loss_rtol=BF16_LOSS_RTOL, grad_rtol=BF16_GRAD_RTOL, grad_atol=(n - 1) * BF16_FLUSH_GRAD)


def test_bf16_d16_near_edges_cancel():
    """BF16 at d = 16: a 16-vertex clique packed into a ball of radius 0.03 at the origin
    (every pair an edge close in tau, dl+ ~ 0.1 bit, dl- ~ 3.9 bits) plus far vertices.  A
    pass of the sweep adds each edge's non-edge term and the edge pass subtracts it; with the
    same pair function (the table at d = 16) they agree to the rounding of the squared
    distance (bit for bit for the exact near pairs), leaving the FP32 rounding of dl+ - dl-
    (~2e-7 relative of 3.9 bits per pair), well inside 5e-6 of the loss.  A non-edge term
    from the other pair function (the table's fit error, up to 5e-6 relative) moved the loss
    by 4.4e-4."""
    n = 300
    rng = np.random.default_rng(41)
    X = rng.standard_normal((n, 16)) * 3.0
    X[:16] = rng.standard_normal((16, 16)) * (0.03 / 4.0)
    X = X.astype(np.float32)
    cl = np.arange(16)
    uu, vv = np.meshgrid(cl, cl)
    keep = uu < vv
    g = synth.csr_from_edges(n, uu[keep], vv[keep])
    note("bf16 d16 near clique")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    got = gpu_loss_grad(G, X, params=gempe.params_default(**BF16))
    ref = oracle.loss_grad(X, g.row_ptr, g.col_idx, want_abs_slope=True)
    assert got["edge_hits"] == g.m == 120
    # the clique's own pairs carry the loss that matters here: compare its share
    ref_far = oracle.loss_grad(X[16:], synth.csr_from_edges(n - 16, np.zeros(0, np.int64),
                                                            np.zeros(0, np.int64)).row_ptr,
                               np.zeros(0, np.int32), want_grad=False)["loss"]
    clique_gpu = got["loss"] - ref_far
    clique_ref = ref["loss"] - ref_far
    assert abs(clique_gpu - clique_ref) <= 5e-6 * ref["loss"], (clique_gpu, clique_ref, ref["loss"])
    # the stated BF16 gradient bound (the far vertices' pairs are all flushed, < 2e-18 each)
    assert_grad_close(got["grad"], ref["grad"], ref["abs_slope"], rtol=BF16_GRAD_RTOL, what="bf16 d16 near clique",
                      atol=(n - 1) * BF16_FLUSH_GRAD)
    # the clique's vertices, whose pairs are all near edges, meet the FP32 bound
    assert_grad_close(got["grad"][:16], ref["grad"][:16], ref["abs_slope"][:16], what="bf16 d16 clique vertices")


@pytest.mark.parametrize("n,d,kind", [(9000, 16, "spread"), (8300, 16, "clusters"), (4500, 32, "contracted"),
                                       (4200, 64, "contracted"), (4300, 64, "clusters"), (4150, 128, "contracted")])
def test_bf16_full_sweep_route(n, d, kind):
    """BF16 from n = 8,192 (d = 16) or 4,096 (d = 32, 64, 128) on.  When more than half of
    the tiles are flagged (d = 16 from X ~ N(0, 1), any d from a contracted start) the sparse
    pass hands the evaluation to the full matrix-core sweep (every pair exact in FP32; the
    dense list pass exits).  Tight far-apart clusters: most tiles unflagged, the list route.
    All against the whole-graph oracle; the exact pass's launch count shows the route was
    planned (the sparse pass and the list in the exact class, the full sweep in its own)."""
    if kind == "spread":
        g = synth.chung_lu(n, 10.0, 2.4, seed=n)
        X = synth.init_embedding(n, d, seed=n + 1)
    elif kind == "contracted":
        g = synth.chung_lu(n, 10.0, 2.4, seed=n)
        X = synth.init_embedding(n, d, seed=n + 1, scale=1.5 / np.sqrt(2 * d))
    else:
        X, lab = clusters(n, d, 40, spread=0.1, sep=4.0, seed=n)
        order = np.argsort(lab, kind="stable")  # vertices by cluster: far tiles off the diagonal
        X, lab = X[order], lab[order]
        rng = np.random.default_rng(n)
        u = rng.integers(0, n, 3 * n)
        members = [np.nonzero(lab == k)[0] for k in range(40)]
        same = np.array([rng.choice(members[lab[a]]) for a in u])
        g = synth.csr_from_edges(n, u, same)
    note(f"bf16 full-sweep route n={n} d={d} {kind} m={g.m}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    gempe.timing_enable(True)
    gempe.timing_read(gempe.GEMPE_TK_EXACT)
    gempe.timing_read(gempe.GEMPE_TK_FULL)
    got = gpu_loss_grad(G, X, params=gempe.params_default(**BF16))
    nl, _ = gempe.timing_read(gempe.GEMPE_TK_EXACT)
    nf, _ = gempe.timing_read(gempe.GEMPE_TK_FULL)
    gempe.timing_enable(False)
    assert (nl, nf) == (2, 1), (nl, nf)
    ref = oracle.loss_grad(X, g.row_ptr, g.col_idx, want_abs_slope=True)
    assert got["edge_hits"] == g.m == ref["edge_hits"]
    what = f"bf16 route n{n} d{d} {kind}"
    if kind != "clusters":
        # every pair exact in FP32: the FP32 bounds hold
        assert abs(got["loss"] - ref["loss"]) <= 1e-5 * ref["loss"], (what, got["loss"], ref["loss"])
        assert_grad_close(got["grad"], ref["grad"], ref["abs_slope"], what=what)
    else:
        assert abs(got["loss"] - ref["loss"]) <= BF16_LOSS_RTOL * ref["loss"], (what, got["loss"], ref["loss"])
        assert_grad_close(got["grad"], ref["grad"], ref["abs_slope"], rtol=BF16_GRAD_RTOL, what=what,
                          atol=(n - 1) * BF16_FLUSH_GRAD)
    G.close()


def test_bf16_route_sample_alternating():
    """At d = 16 a plain BF16 evaluation that may take the full matrix-core route screens a
    sample of its tiles first and skips the screen when most of the sample is flagged.  One
    graph and one workspace, evaluated from a spread start (the sample is dense: no screen,
    the full sweep) and from tight far-apart clusters (the sample is sparse: the screen and
    the list route) in turn, so each evaluation starts from the other route's leftover
    flags, list, counts and loss slots; every one against the whole-graph oracle, and the
    repeats' losses bit for bit equal to the first ones (fixed-order loss sums)."""
    n, d = 8300, 16
    Xc, lab = clusters(n, d, 40, spread=0.1, sep=4.0, seed=7)
    order = np.argsort(lab, kind="stable")
    Xc, lab = Xc[order], lab[order]
    rng = np.random.default_rng(8)
    u = rng.integers(0, n, 3 * n)
    members = [np.nonzero(lab == k)[0] for k in range(40)]
    same = np.array([rng.choice(members[lab[a]]) for a in u])
    g = synth.csr_from_edges(n, u, same)
    Xs = synth.init_embedding(n, d, seed=9)
    note(f"bf16 route sample alternating n={n} d={d} m={g.m}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    params = gempe.params_default(**BF16)
    ws = gempe.workspace(G, d, params)
    refs = {"spread": oracle.loss_grad(Xs, g.row_ptr, g.col_idx, want_abs_slope=True),
            "clusters": oracle.loss_grad(Xc, g.row_ptr, g.col_idx, want_abs_slope=True)}
    first = {}
    for kind in ("clusters", "spread", "clusters", "spread", "spread", "clusters"):
        X = Xs if kind == "spread" else Xc
        r = gempe.loss_grad(G, to_dev(X), ws=ws, params=params)
        torch.cuda.synchronize()
        loss, grad = float(r.loss.item()), r.grad.double().cpu().numpy()
        # the route the sample chose: the workspace opens with the library's counter block,
        # whose bytes 40..47 hold the sample's flagged and sampled sub-tile counts
        flagged, sampled = (int(v) for v in ws[40:48].cpu().view(torch.int32))
        assert sampled > 0 and (2 * flagged > sampled) == (kind == "spread"), (kind, flagged, sampled)
        ref = refs[kind]
        assert int(r.edge_hits.item()) == g.m == ref["edge_hits"]
        what = f"route sample {kind}"
        if kind == "spread":  # every pair exact in FP32
            assert abs(loss - ref["loss"]) <= 1e-5 * ref["loss"], (what, loss, ref["loss"])
            assert_grad_close(grad, ref["grad"], ref["abs_slope"], what=what)
        else:
            assert abs(loss - ref["loss"]) <= BF16_LOSS_RTOL * ref["loss"], (what, loss, ref["loss"])
            assert_grad_close(grad, ref["grad"], ref["abs_slope"], rtol=BF16_GRAD_RTOL, what=what,
                              atol=(n - 1) * BF16_FLUSH_GRAD)
        if kind in first:
            assert loss == first[kind], (what, loss, first[kind])
        first.setdefault(kind, loss)
    G.close()


@pytest.mark.parametrize("n,d,kind", [(9000, 16, "spread"), (8300, 16, "clusters"), (4200, 64, "contracted"),
                                       (4300, 64, "clusters")])
def test_bf16_reversed_tile_order(n, d, kind):
    """The BF16 path with its tiles taken in reverse order (GEMPE_F_REVERSE_TILES), on the
    full matrix-core route (spread at d = 16 through the route sample, contracted at d = 64)
    and on the list route (clusters): the loss is a fixed-order sum of per-item or per-list
    slots, so it is bit for bit the forward run's; the gradient (atomics) agrees to rounding."""
    if kind == "clusters":
        X, lab = clusters(n, d, 40, spread=0.1, sep=4.0, seed=n)
        order = np.argsort(lab, kind="stable")
        X, lab = X[order], lab[order]
        rng = np.random.default_rng(n)
        u = rng.integers(0, n, 3 * n)
        members = [np.nonzero(lab == k)[0] for k in range(40)]
        g = synth.csr_from_edges(n, u, np.array([rng.choice(members[lab[a]]) for a in u]))
    else:
        g = synth.chung_lu(n, 10.0, 2.4, seed=n)
        scale = 1.5 / np.sqrt(2 * d) if kind == "contracted" else 1.0
        X = synth.init_embedding(n, d, seed=n + 1, scale=scale)
    note(f"bf16 reversed tile order n={n} d={d} {kind}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    fwd = gpu_loss_grad(G, X, params=gempe.params_default(**BF16))
    rev = gpu_loss_grad(G, X, params=gempe.params_default(flags=gempe.GEMPE_F_REVERSE_TILES, **BF16))
    assert rev["loss"] == fwd["loss"], (rev["loss"], fwd["loss"])
    assert rev["edge_hits"] == fwd["edge_hits"] == g.m
    A = np.abs(fwd["grad"]).sum(axis=1) + 1e-30
    assert_grad_close(rev["grad"], fwd["grad"], A, rtol=1e-5, what=f"bf16 reversed n{n} d{d} {kind}")
    G.close()
