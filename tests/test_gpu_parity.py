"""GPU parity of the FP32 all-pairs path against the FP64 oracle, through the C ABI."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_util import (assert_grad_close, assert_loss_close, check_full, check_rows, gpu_loss_grad, note,
                      require_gpu, to_dev)
from paper_2011_03479_amd import gempe, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()
    oracle.build(force=False)


def make_graph(n, kind, seed):
    if kind == "empty":
        return synth.csr_from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64))
    if kind == "complete":
        i, j = np.triu_indices(n, 1)
        return synth.csr_from_edges(n, i, j)
    if kind == "star":
        return synth.csr_from_edges(n, np.zeros(n - 1, np.int64), np.arange(1, n))
    if kind == "cl":
        return synth.chung_lu(n, min(10.0, (n - 1) / 2), 2.5, seed=seed)
    return synth.erdos_renyi(n, min(6.0, (n - 1) / 2), seed=seed)


SHAPES = [
    (2, 2, "er"), (3, 1, "complete"), (5, 3, "er"), (63, 2, "er"), (64, 2, "star"), (65, 2, "er"),
    (129, 4, "cl"), (200, 5, "er"), (300, 8, "er"), (257, 13, "cl"), (300, 16, "er"), (130, 17, "er"),
    (200, 32, "cl"), (150, 64, "er"), (100, 100, "er"), (130, 128, "er"), (700, 2, "empty"),
    (1000, 16, "cl"), (2500, 2, "cl"), (97, 2, "complete"),
]


@pytest.mark.parametrize("n,d,kind", SHAPES, ids=[f"n{n}_d{d}_{k}" for n, d, k in SHAPES])
def test_parity_shapes(n, d, kind):
    g = make_graph(n, kind, seed=n * 31 + d)
    X = synth.init_embedding(n, d, seed=7 + n + d)
    note(f"parity n={n} d={d} graph={kind} m={g.m}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    check_full(g, G, X, what=f"n{n} d{d} {kind}")


def test_er1k_at_init():
    w = synth.workload("er1k")
    note("parity er1k (n=1000, d=2) at X0")
    G = gempe.Graph(w.graph.n, w.graph.row_ptr, w.graph.col_idx)
    check_full(w.graph, G, w.X0, what="er1k")


def test_cl3400_at_init():
    w = synth.workload("cl3400")
    note("parity cl3400 (n=3400, d=2) at X0")
    G = gempe.Graph(w.graph.n, w.graph.row_ptr, w.graph.col_idx)
    check_full(w.graph, G, w.X0, what="cl3400")


@pytest.mark.parametrize("mu,sigma,scale", [(2.0, 0.5, 1.0), (0.7, 1.7, 1.0), (1.5, 1.0, 20.0),
                                            (1.5, 1.0, 1e-3)])
def test_parameters_and_regimes(mu, sigma, scale):
    """Non-default mu/sigma, far edges (log-domain tail), contracted (all-near) points."""
    n, d = 400, 3
    g = synth.erdos_renyi(n, 8.0, seed=5)
    X = (synth.init_embedding(n, d, 99).astype(np.float64) * scale).astype(np.float32)
    p = gempe.params_default(mu=mu, sigma=sigma)
    note(f"parity mu={mu} sigma={sigma} scale={scale}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    check_full(g, G, X, mu=mu, sigma=sigma, params=p, what=f"mu{mu} s{sigma} x{scale}")


# The sweeps tabulate the non-edge term for tau >= -8 only.  With sigma < mu / 8 a close
# non-edge pair falls below the table and is evaluated in closed form behind a per-pair
# test; with the default slope every non-edge lies inside the table and the sweeps drop
# that test.  Both forms, on the small-n and the multi-wave tile plans and in the fused
# iteration.
def _below_table_pairs(X, mu, sigma):
    """Pairs i < j closer than mu - 8 sigma (counted on the CPU, in FP64)."""
    Xd = X.astype(np.float64)
    r2 = np.sum((Xd[:, None, :] - Xd[None, :, :]) ** 2, axis=-1)
    return int(np.count_nonzero(np.triu(np.sqrt(r2) < mu - 8.0 * sigma, 1)))


@pytest.mark.parametrize("n,d,scale", [(400, 2, 1.0), (300, 16, 0.05), (600, 8, 0.08)])
def test_below_table_pairs(n, d, scale):
    mu, sigma = 1.5, 0.15
    g = synth.erdos_renyi(n, 8.0, seed=n + d)
    X = (synth.init_embedding(n, d, 21 + d).astype(np.float64) * scale).astype(np.float32)
    below = _below_table_pairs(X, mu, sigma)
    assert below > 100, below
    note(f"below-table parity n={n} d={d} pairs below the table: {below}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    check_full(g, G, X, mu=mu, sigma=sigma, params=gempe.params_default(mu=mu, sigma=sigma),
               what=f"below-table n{n} d{d}")


@pytest.mark.parametrize("sigma", [1.0, 0.15])
def test_multiwave_plan_both_table_forms(sigma):
    """n = 40,000 at d = 16 selects tiles of 2 rows per lane and 4 waves; contracted points
    put most non-edges near, and below the table when sigma = 0.15."""
    mu, n, d = 1.5, 40000, 16
    g = synth.chung_lu(n, 12.0, 2.3, seed=77)
    X = (synth.init_embedding(n, d, seed=78).astype(np.float64) * 0.05).astype(np.float32)
    rng = np.random.default_rng(79)
    rows = np.unique(np.concatenate([rng.choice(n, 60, replace=False), np.argsort(-np.diff(g.row_ptr))[:4]]))
    if sigma < mu / 8:
        assert _below_table_pairs(X[:400], mu, sigma) > 100
    note(f"multi-wave plan n={n} d={d} sigma={sigma}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    check_rows(g, G, X, rows, mu=mu, sigma=sigma, params=gempe.params_default(mu=mu, sigma=sigma),
               what=f"n{n} d{d} sigma{sigma}")


def test_fused_iteration_below_table():
    mu, sigma, n, d, iters = 1.5, 0.15, 1000, 2, 4
    g = synth.chung_lu(n, 8.0, 2.5, seed=31)
    X0 = synth.init_embedding(n, d, seed=32)
    assert _below_table_pairs(X0, mu, sigma) > 100
    eta = 0.01 / (n - 1)
    p = gempe.params_default(mu=mu, sigma=sigma)
    note(f"fused iteration below the table n={n} iters={iters}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    Xa = to_dev(X0)
    h = torch.empty(iters + 1, dtype=torch.float64, device="cuda")
    gempe.embed(G, Xa, iters, eta, params=p, loss_hist=h)
    torch.cuda.synchronize()
    ref_hist, X_ref = oracle.gd_trajectory(X0, g.row_ptr, g.col_idx, iters, eta, mu=mu, sigma=sigma)
    assert np.allclose(h.cpu().numpy(), ref_hist, rtol=1e-5, atol=0)
    xa = Xa.double().cpu().numpy()
    assert np.max(np.linalg.norm(xa - X_ref, axis=1)) <= 1e-4 * np.max(np.linalg.norm(X_ref, axis=1))


def test_two_vertices_and_coincident_points():
    note("two vertices / coincident points")
    X = np.array([[0.0, 0.0], [3.0, 4.0]], dtype=np.float32)
    for edges in ([(0, 1)], []):
        g = synth.csr_from_edges(2, np.array([e[0] for e in edges], np.int64), np.array([e[1] for e in edges], np.int64))
        G = gempe.Graph(2, g.row_ptr, g.col_idx)
        got = gpu_loss_grad(G, X)
        dl, d1, _ = oracle.pair(5.0, bool(edges))
        assert_loss_close(got["loss"], dl, what="two vertices")
        g1 = d1 * (X[0] - X[1]) / 5.0
        assert np.allclose(got["grad"][0], g1, rtol=1e-5) and np.allclose(got["grad"][1], -g1, rtol=1e-5)
    g = synth.erdos_renyi(50, 6.0, seed=3)
    X = np.full((50, 4), 0.25, dtype=np.float32)
    G = gempe.Graph(50, g.row_ptr, g.col_idx)
    got = gpu_loss_grad(G, X)
    N = 50 * 49 // 2
    ref = g.m * oracle.pair(0.0, True)[0] + (N - g.m) * oracle.pair(0.0, False)[0]
    assert_loss_close(got["loss"], ref, what="coincident")
    assert np.all(got["grad"] == 0.0)


def test_has_edge_bit_exact():
    g = synth.chung_lu(3000, 12.0, 2.3, seed=17)
    note(f"has_edge n=3000 m={g.m}")
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    E = g.edges_upper()
    rng = np.random.default_rng(0)
    qi = np.concatenate([E[:, 0], E[:, 1], rng.integers(0, g.n, 20000), [-1, 0, 5, 3000, 7]])
    qj = np.concatenate([E[:, 1], E[:, 0], rng.integers(0, g.n, 20000), [0, -1, 5, 1, 3000]])
    got = gempe.has_edge(G, qi, qj).cpu().numpy()
    Es = set(map(tuple, E.tolist()))
    ref = np.array([(min(a, b), max(a, b)) in Es for a, b in zip(qi.tolist(), qj.tolist())], dtype=np.uint8)
    assert np.array_equal(got, ref)


def _bad_csr(kind):
    n = 6
    edges = [(0, 1), (1, 2), (2, 3), (4, 5)]
    g = synth.csr_from_edges(n, np.array([e[0] for e in edges]), np.array([e[1] for e in edges]))
    rp, ci = g.row_ptr.copy(), g.col_idx.copy()
    if kind == "self_loop":
        ci[0] = 0
    elif kind == "unsorted":  # row 1 holds (0, 2): swap
        a, b = rp[1], rp[2]
        ci[a:b] = ci[a:b][::-1]
    elif kind == "asymmetric":  # redirect (4, 5) to (4, 3): (3, 4) is absent
        ci[rp[4]] = 3
    elif kind == "duplicate":  # row 2 holds (1, 3) -> (1, 1)
        ci[rp[2] + 1] = 1
    elif kind == "out_of_range":
        ci[-1] = 17
    elif kind == "row_ptr":
        rp[3] = rp[4] + 1
    return n, rp, ci


@pytest.mark.parametrize("kind", ["self_loop", "unsorted", "asymmetric", "duplicate", "out_of_range", "row_ptr"])
def test_invalid_graph_rejected(kind):
    note(f"invalid graph: {kind}")
    n, rp, ci = _bad_csr(kind)
    with pytest.raises(gempe.GempeError) as e:
        gempe.Graph(n, rp, ci)
    assert e.value.status == gempe.GEMPE_ERR_GRAPH


def test_loss_is_deterministic_and_grad_stable():
    w = synth.workload("er1k")
    G = gempe.Graph(w.graph.n, w.graph.row_ptr, w.graph.col_idx)
    note("determinism er1k x5")
    outs = [gpu_loss_grad(G, w.X0) for _ in range(5)]
    assert len({o["loss"] for o in outs}) == 1, "loss must be bitwise reproducible"
    # the gradient's cross-tile FP32 atomics add in a run-dependent order: runs agree to
    # the gradient bound, not bitwise
    A = oracle.loss_grad(w.X0, w.graph.row_ptr, w.graph.col_idx, want_abs_slope=True)["abs_slope"]
    for o in outs[1:]:
        assert_grad_close(o["grad"], outs[0]["grad"], A, rtol=1e-5, what="run-to-run")


@pytest.mark.parametrize("n,d", [(2500, 2), (1000, 16), (700, 32), (3000, 4)])
def test_reversed_tile_order(n, d):
    """Schedule perturbation: the sweep takes its tiles in reverse order (GEMPE_F_REVERSE_TILES).
    Each tile keeps its loss-partial slot and the FP64 sum runs in slot order, so the loss is
    bitwise unchanged; the gradient differs only by the order of its FP32 atomic additions."""
    g = synth.chung_lu(n, min(10.0, (n - 1) / 3), 2.5, seed=5 * n + d)
    X = synth.init_embedding(n, d, seed=n + 3 * d)
    note(f"reversed tile order n={n} d={d}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    fwd = gpu_loss_grad(G, X)
    rev = gpu_loss_grad(G, X, params=gempe.params_default(flags=gempe.GEMPE_F_REVERSE_TILES))
    assert rev["loss"] == fwd["loss"], (rev["loss"], fwd["loss"])
    assert rev["edge_hits"] == fwd["edge_hits"] == g.m
    A = oracle.loss_grad(X, g.row_ptr, g.col_idx, want_abs_slope=True)["abs_slope"]
    assert_grad_close(rev["grad"], fwd["grad"], A, rtol=1e-5, what=f"reversed n{n} d{d}")


def test_reversed_tile_order_fused_iteration():
    """The fused gradient-descent iteration with its tiles in reverse order: the loss of the
    start point is bitwise the same, the trajectory equal within the FP32 reassociation of the
    gradient's atomic additions."""
    n, d, iters = 3400, 2, 6
    w = synth.workload("cl3400")
    note(f"reversed tile order, fused iteration n={n} d={d} iters={iters}")
    G = gempe.Graph(n, w.graph.row_ptr, w.graph.col_idx)
    runs = []
    for flags in (gempe.GEMPE_F_NONE, gempe.GEMPE_F_REVERSE_TILES):
        X = to_dev(w.X0)
        hist = torch.zeros(iters + 1, dtype=torch.float64, device="cuda")
        gempe.embed(G, X, iters, w.eta, params=gempe.params_default(flags=flags), loss_hist=hist)
        torch.cuda.synchronize()
        runs.append((X.double().cpu().numpy(), hist.cpu().numpy()))
    (xf, hf), (xr, hr) = runs
    assert hr[0] == hf[0], (hr[0], hf[0])
    np.testing.assert_allclose(hr, hf, rtol=1e-6)
    assert np.max(np.abs(xr - xf)) <= 1e-5 * np.max(np.abs(xf))


def test_workspace_and_argument_errors():
    g = synth.erdos_renyi(100, 5.0, seed=2)
    G = gempe.Graph(100, g.row_ptr, g.col_idx)
    X = to_dev(synth.init_embedding(100, 2, 3))
    ws = gempe.workspace(G, 2)
    small = ws[: ws.numel() // 2]
    note("workspace/argument errors")
    with pytest.raises(gempe.GempeError) as e:
        gempe.loss_grad(G, X, ws=small)
    assert e.value.status == gempe.GEMPE_ERR_NOMEM
    with pytest.raises(gempe.GempeError) as e:
        gempe.step(G, X, eta=-1.0, ws=ws)
    assert e.value.status == gempe.GEMPE_ERR_ARG
    with pytest.raises(gempe.GempeError) as e:
        gempe.loss_grad(G, to_dev(np.zeros((100, 129), np.float32)))
    assert e.value.status == gempe.GEMPE_ERR_ARG
    bad = X.clone()
    bad[3, 0] = float("nan")
    hist = torch.empty(3, dtype=torch.float64, device="cuda")
    with pytest.raises(gempe.GempeError) as e:
        gempe.embed(G, bad, iters=2, eta=1e-3, ws=ws, loss_hist=hist)
    assert e.value.status == gempe.GEMPE_ERR_NUMERIC
    # without a loss history the fused iteration (n <= 23,000, d <= 16) still reduces and
    # checks every sweep's loss, and the per-evaluation path (d = 32) its scratch loss
    note("NaN without a loss history: fused (d = 2) and per-evaluation (d = 32) paths")
    for d in (2, 32):
        Gd = gempe.Graph(100, g.row_ptr, g.col_idx)
        wsd = gempe.workspace(Gd, d)
        Xd = to_dev(synth.init_embedding(100, d, 4))
        Xd[7, d - 1] = float("nan")
        for iters in (1, 3):
            with pytest.raises(gempe.GempeError) as e:
                gempe.embed(Gd, Xd.clone(), iters=iters, eta=1e-3, ws=wsd)
            assert e.value.status == gempe.GEMPE_ERR_NUMERIC, (d, iters)
        # and a finite run on the same workspace reports no error afterwards
        gempe.embed(Gd, to_dev(synth.init_embedding(100, d, 4)), iters=3, eta=1e-3, ws=wsd)
        Gd.close()


def test_er1k_trajectory():
    """100 fixed-step iterations: every iterate re-anchored against the oracle, the loss
    history of gempe_embed against the step loop, final coordinates against the FP64
    trajectory."""
    w = synth.workload("er1k")
    g = w.graph
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    ws = gempe.workspace(G, w.d)
    X = to_dev(w.X0)
    loss_before = torch.empty(1, dtype=torch.float64, device="cuda")
    losses = []
    note("trajectory er1k: 100 steps")
    for k in range(w.iters + 1):
        Xk = X.cpu().numpy()
        if k in (0, 50, 100):
            check_full(g, G, Xk, row_loss=False, what=f"er1k iter {k}")
        if k == w.iters:
            break
        gempe.step(G, X, w.eta, ws=ws, loss_before=loss_before)
        torch.cuda.synchronize()
        lb = float(loss_before.item())
        ref = oracle.loss_grad(Xk, g.row_ptr, g.col_idx, want_grad=False)["loss"]
        assert_loss_close(lb, ref, what=f"er1k loss iter {k}")
        losses.append(lb)
    X_gpu = X.cpu().numpy().astype(np.float64)
    # gempe_embed from X0 reproduces the step loop's loss history
    X2 = to_dev(w.X0)
    hist = torch.empty(w.iters + 1, dtype=torch.float64, device="cuda")
    gempe.embed(G, X2, w.iters, w.eta, ws=ws, loss_hist=hist)
    h = hist.cpu().numpy()
    assert np.allclose(h[:-1], np.array(losses), rtol=1e-6, atol=0)
    assert np.all(np.diff(h) < 0), "loss must decrease monotonically at this step size"
    ref_hist, X_ref = oracle.gd_trajectory(w.X0, g.row_ptr, g.col_idx, w.iters, w.eta)
    assert np.allclose(h, ref_hist, rtol=1e-5, atol=0)
    scale = np.max(np.linalg.norm(X_ref, axis=1))
    for Xg in (X_gpu, X2.cpu().numpy().astype(np.float64)):
        dev = np.max(np.linalg.norm(Xg - X_ref, axis=1))
        assert dev <= 1e-4 * scale, dev / scale


@pytest.mark.parametrize("n,d", [(70000, 2), (20000, 16), (40000, 16), (5000, 8)])
def test_large_sampled_rows(n, d):
    """Sizes that select the multi-wave / multi-row tile plans; oracle on sampled rows."""
    g = synth.chung_lu(n, 12.0, 2.3, seed=n + d)
    X = synth.init_embedding(n, d, seed=3 * n + d)
    rng = np.random.default_rng(n)
    hubs = np.argsort(-np.diff(g.row_ptr))[:8]
    rows = np.unique(np.concatenate([rng.choice(n, 120, replace=False), hubs, [0, n - 1]]))
    note(f"sampled rows n={n} d={d} m={g.m}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    check_rows(g, G, X, rows, what=f"n{n} d{d}")


def test_pair_function_accuracy():
    """Single-pair values over a dense distance grid (edge and non-edge): the FP32 pair
    function against the FP64 oracle.  Bound: 2e-6 relative, plus the FP32 rounding of the
    exponent of exp(-tau^2/2) (two roundings of tau^2 log2(e)/2, each eps relative, i.e.
    an exponent error of about eps tau^2 nats): 1.2e-7 tau^2."""
    note("pair function grid")
    deltas = np.concatenate([np.linspace(0.0, 12.0, 97), [15.0, 20.0, 30.0, 45.0, 60.0]]).astype(np.float32)
    for edge in (True, False):
        g = synth.csr_from_edges(2, np.array([0] if edge else [], np.int64), np.array([1] if edge else [], np.int64))
        G = gempe.Graph(2, g.row_ptr, g.col_idx)
        for dlt in deltas:
            X = np.array([[0.0, 0.0], [dlt, 0.0]], dtype=np.float32)
            got = gpu_loss_grad(G, X)
            dl, d1, _ = oracle.pair(float(dlt), edge)
            tau = (float(dlt) - 1.5) * (-1.0 if edge else 1.0)
            rtol = 2e-6 + 1.2e-7 * tau * tau
            assert abs(got["loss"] - dl) <= rtol * abs(dl) + 1e-37, (edge, float(dlt), got["loss"], dl)
            gx = -d1 if dlt > 0 else 0.0
            assert abs(got["grad"][0, 0] - gx) <= rtol * abs(gx) + 1e-37, (edge, float(dlt), got["grad"][0, 0], gx)
            assert got["grad"][0, 1] == 0.0


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_cl1m_sampled_rows(prec):
    """The large all-pairs workload at full size (Chung-Lu n = 1,000,000, mean degree 20,
    exponent 2.3, d = 16): sampled rows (including the hubs) against the oracle."""
    from gpu_util import BF16_FLUSH_GRAD, BF16_GRAD_RTOL, BF16_LOSS_RTOL

    w = synth.workload("cl1m" if prec == "fp32" else "cl1m_bf16")
    g = w.graph
    rng = np.random.default_rng(1)
    hubs = np.argsort(-np.diff(g.row_ptr))[:6]
    rows = np.unique(np.concatenate([rng.choice(g.n, 60, replace=False), hubs, [0, g.n - 1]]))
    note(f"cl1m {prec} sampled rows, m={g.m}")
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    if prec == "fp32":
        check_rows(g, G, w.X0, rows, what="cl1m fp32")
    else:
        check_rows(g, G, w.X0, rows, params=gempe.params_default(precision=1), what="cl1m bf16",
                   loss_rtol=BF16_LOSS_RTOL, grad_rtol=BF16_GRAD_RTOL, grad_atol=(g.n - 1) * BF16_FLUSH_GRAD)
