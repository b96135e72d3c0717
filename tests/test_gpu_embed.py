"""gempe_embed (one fused launch per iteration for small n) against the step-by-step path and the
FP64 oracle trajectory."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from gpu_util import note, require_gpu, to_dev
from paper_2011_03479_amd import gempe, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()
    oracle.build(force=False)


CASES = [
    (100, 2, 1, True), (100, 2, 1, False), (257, 3, 2, True), (257, 3, 3, False), (1000, 16, 4, True),
    (650, 8, 5, False), (130, 1, 6, True), (70, 2, 0, True), (3400, 2, 7, True), (2000, 5, 2, False),
    # longer runs: the gradient ring (three slots) and the iterate ping-pong through many cycles
    (1000, 2, 40, True), (1500, 8, 13, True), (700, 16, 25, False),
]


@pytest.mark.parametrize("n,d,iters,hist", CASES, ids=[f"n{c[0]}_d{c[1]}_it{c[2]}_h{int(c[3])}" for c in CASES])
def test_embed_matches_steps_and_oracle(n, d, iters, hist):
    g = synth.chung_lu(n, min(10.0, (n - 1) / 3), 2.5, seed=n + d)
    X0 = synth.init_embedding(n, d, seed=11 * n + d)
    eta = 0.1 / (n - 1)
    note(f"embed n={n} d={d} iters={iters} hist={hist}")
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    ws = gempe.workspace(G, d)
    Xa = to_dev(X0)
    h = torch.full((iters + 1,), float("nan"), dtype=torch.float64, device="cuda") if hist else None
    gempe.embed(G, Xa, iters, eta, ws=ws, loss_hist=h)
    # step-by-step reference on the same device
    Xb = to_dev(X0)
    lb = torch.empty(1, dtype=torch.float64, device="cuda")
    losses = []
    for _ in range(iters):
        gempe.step(G, Xb, eta, ws=ws, loss_before=lb)
        torch.cuda.synchronize()
        losses.append(float(lb.item()))
    final = gempe.loss_grad(G, Xb, ws=ws)
    torch.cuda.synchronize()
    losses.append(float(final.loss.item()))
    xa = Xa.double().cpu().numpy()
    xb = Xb.double().cpu().numpy()
    scale = max(1.0, float(np.abs(xb).max()))
    assert np.max(np.abs(xa - xb)) <= 1e-5 * scale
    ref_hist, X_ref = oracle.gd_trajectory(X0, g.row_ptr, g.col_idx, iters, eta)
    assert np.max(np.linalg.norm(xa - X_ref, axis=1)) <= 1e-4 * np.max(np.linalg.norm(X_ref, axis=1))
    if hist:
        hh = h.cpu().numpy()
        assert np.all(np.isfinite(hh))
        assert np.allclose(hh, np.array(losses), rtol=1e-6, atol=0)
        assert np.allclose(hh, ref_hist, rtol=1e-5, atol=0)


def test_embed_resume_equals_one_run():
    """embed(2k) = embed(k) + embed(k) (checkpoint / resume of the coordinates)."""
    w = synth.workload("er1k")
    g = w.graph
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    ws = gempe.workspace(G, w.d)
    note("embed resume er1k 2x25 vs 50")
    Xa = to_dev(w.X0)
    gempe.embed(G, Xa, 50, w.eta, ws=ws)
    Xb = to_dev(w.X0)
    gempe.embed(G, Xb, 25, w.eta, ws=ws)
    gempe.embed(G, Xb, 25, w.eta, ws=ws)
    torch.cuda.synchronize()
    a = Xa.double().cpu().numpy()
    b = Xb.double().cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-5 * np.abs(a).max()
