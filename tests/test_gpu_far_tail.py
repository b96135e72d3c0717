"""Far non-edges whose dl lies below FP32's smallest normal (2^-126, tau beyond about 13).

A vertex placed far from a N(0, 1) cloud, with no edges, owes its whole gradient to such
pairs when its nearest pair is at tau = 13.05, and a part of it at tau = 12.9.  The hardware
exp2 returns 0 below 2^-126; the pair functions evaluate it on a range where the result is
normal and scale back, so these rows must meet the ordinary FP32 bound.  Every FP32 sweep is
covered: the VALU sweeps at d = 8, 16 (table) and 128 (closed form), the per-vertex-extras
sweep, and the matrix-core sweeps at d = 16, 64, 128.

The construction is pinned on the CPU against scipy's normal tail (independent of the
oracle): every pair of the far vertex has dl < 2^-126 at tau = 13.05, and the oracle's
gradient row equals the sum of the pair gradients written from Sec. II-B (dl = -log2 Phi).
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_grad_close, assert_loss_close, note, require_gpu, to_dev
from paper_2011_03479_amd import gempe, synth

MU, SIGMA = 1.5, 1.0
FLT_MIN = 2.0 ** -126


def far_embedding(n, d, seed, tau_min):
    """N(0, 1) rows, then row 0 moved along a random direction until its nearest row is at
    delta = mu + tau_min sigma (bisection on the float32-rounded position)."""
    X = synth.init_embedding(n, d, seed).astype(np.float64)
    rng = np.random.default_rng(seed + 7)
    e = rng.standard_normal(d)
    e /= np.linalg.norm(e)
    target = MU + tau_min * SIGMA
    lo, hi = 0.0, 1000.0
    for _ in range(200):
        t = 0.5 * (lo + hi)
        x0 = (t * e).astype(np.float32).astype(np.float64)
        if np.min(np.linalg.norm(X[1:] - x0, axis=1)) < target:
            lo = t
        else:
            hi = t
    X[0] = hi * e
    return X.astype(np.float32)


def far_graph(n, seed):
    """Random edges among vertices 1..n-1 (vertex 0 has none)."""
    rng = np.random.default_rng(seed)
    u = rng.integers(1, n, 4 * n)
    v = rng.integers(1, n, 4 * n)
    return synth.csr_from_edges(n, u, v)


def test_far_vertex_construction_pinned():
    """Not a GPU test: scipy's normal tail puts every pair of the far vertex below 2^-126 at
    tau = 13.05, and the oracle's row equals the pair sum d dl/d delta (x_0 - x_j)/delta with
    d dl/d delta = -phi(tau) / (sigma Phi(tau) ln 2) (the non-edge cost -log2 Phi(tau))."""
    from scipy.stats import norm

    n, d = 700, 16
    X = far_embedding(n, d, 27, 13.05)
    g = far_graph(n, 28)
    df = X[0].astype(np.float64) - X[1:].astype(np.float64)
    delta = np.linalg.norm(df, axis=1)
    tau = (delta - MU) / SIGMA
    assert abs(tau.min() - 13.05) < 1e-5
    dl = -np.log1p(-norm.sf(tau)) / np.log(2.0)
    assert np.all(dl < FLT_MIN) and np.all(dl > 0.0)
    slope = -norm.pdf(tau) / (SIGMA * norm.cdf(tau) * np.log(2.0))
    want = np.sum((slope / delta)[:, None] * df, axis=0)
    ref = oracle.rows(X, g.row_ptr, g.col_idx, np.array([0]), MU, SIGMA)
    assert np.linalg.norm(ref["grad"][0] - want) <= 1e-10 * np.linalg.norm(want)
    assert np.linalg.norm(want) > 4 * FLT_MIN  # the row itself is above FP32's smallest normal


CASES = [
    # (n, d, extras): VALU sweeps below the matrix-core sizes, then the matrix-core sweeps
    (700, 8, False),
    (700, 16, False),
    (700, 128, False),
    (2000, 16, True),
    (8200, 16, False),
    (4160, 64, False),
    (4160, 128, False),
]


@pytest.mark.gpu
@pytest.mark.parametrize("tau_min", [13.05, 12.9])
@pytest.mark.parametrize("n,d,extras", CASES)
def test_far_vertex_rows(n, d, extras, tau_min):
    require_gpu()
    X = far_embedding(n, d, 11 + d, tau_min)
    g = far_graph(n, 12 + d)
    note(f"far vertex n={n} d={d} extras={extras} tau_min={tau_min}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    Xd = to_dev(X)
    r = gempe.loss_grad(G, Xd, want_row_loss=extras)
    torch.cuda.synchronize()
    grad = r.grad.double().cpu().numpy()
    ref = oracle.loss_grad(X, g.row_ptr, g.col_idx, MU, SIGMA, want_abs_slope=True)
    what = f"far vertex n{n} d{d} tau {tau_min}"
    assert int(r.edge_hits.item()) == g.m == ref["edge_hits"], what
    assert_loss_close(float(r.loss.item()), ref["loss"], what=what)
    assert np.linalg.norm(ref["grad"][0]) > 4 * FLT_MIN
    assert_grad_close(grad, ref["grad"], ref["abs_slope"], what=what)
    if extras:
        rl = r.row_loss.double().cpu().numpy()
        assert abs(0.5 * rl.sum() - float(r.loss.item())) <= 1e-5 * float(r.loss.item()), what
    G.close()
