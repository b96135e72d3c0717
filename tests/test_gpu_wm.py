"""Weighted majorization (Sec. II-C, Eqs. 3-5) through the C ABI against the FP64 oracle.

z_i = sum_j w_ij is a sum of positive terms, so its tolerance is relative: 1e-5 (FP32; each
w carries <= ~1e-6 relative error: the table's 2.6e-7 slope error amplified by at most
R / (R + tau) <= 4.4 at tau = -mu/sigma, or the closed form's ~1e-6), plus, for the BF16
screen, (n - 1) 7e-18 for the flushed far pairs.  The update x - g/(2z) is checked per vertex
against the oracle's y_i / z_i, re-anchored at the GPU's X, to the bound that follows from the
gradient and z tolerances."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from gpu_util import GRAD_FLOOR, GRAD_RTOL, LOSS_RTOL, assert_grad_close, note, require_gpu, to_dev
from paper_2011_03479_amd import gempe, synth

pytestmark = pytest.mark.gpu

Z_RTOL = 1e-5
BF16_Z_FLUSH = 7e-18


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()
    oracle.build(force=False)


def graph_of(kind, n, seed):
    if kind == "er":
        return synth.erdos_renyi(n, min(10.0, (n - 1) / 3), seed=seed)
    if kind == "cl":
        return synth.chung_lu(n, min(12.0, (n - 1) / 3), 2.5, seed=seed)
    if kind == "sbm":
        return synth.sbm(4, n // 4, 0.05, 0.002, seed=seed)
    raise KeyError(kind)


def check_terms(g, X, params=None, z_atol=0.0, loss_rtol=LOSS_RTOL, grad_rtol=GRAD_RTOL, grad_atol=0.0):
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    loss, grad, z = gempe.wm_terms(G, to_dev(X), params=params)
    torch.cuda.synchronize()
    rows = np.arange(g.n)
    ref = oracle.rows(X.astype(np.float64), g.row_ptr, g.col_idx, rows, wm=True)
    full = oracle.loss_grad(X.astype(np.float64), g.row_ptr, g.col_idx, want_grad=False)
    assert abs(float(loss.item()) - full["loss"]) <= loss_rtol * full["loss"]
    assert_grad_close(grad.double().cpu().numpy(), ref["grad"], ref["abs_slope"], rtol=grad_rtol, atol=grad_atol)
    zg = z.double().cpu().numpy()
    err = np.abs(zg - ref["z"])
    bound = Z_RTOL * ref["z"] + z_atol
    assert np.all(ref["z"] > 0)
    assert np.all(err <= bound), f"z: worst {np.max(err / bound):.3f} of the bound at vertex {int(np.argmax(err / bound))}"
    return ref


SHAPES = [("er", 300, 2), ("cl", 1000, 2), ("cl", 700, 3), ("sbm", 800, 8), ("er", 1500, 16), ("cl", 520, 32),
          ("er", 400, 100), ("sbm", 640, 128)]


@pytest.mark.parametrize("kind,n,d", SHAPES, ids=[f"{k}_n{n}_d{d}" for k, n, d in SHAPES])
def test_wm_terms(kind, n, d):
    note(f"wm_terms {kind} n={n} d={d}")
    g = graph_of(kind, n, seed=n + d)
    X = synth.init_embedding(n, d, seed=3 * n + d)
    check_terms(g, X)


@pytest.mark.parametrize("scale", [0.05, 6.0, 25.0])
def test_wm_terms_regimes(scale):
    """Coincident-ish, spread and far embeddings: far edges have tau << 0, where R + tau
    cancels unless the Mills-ratio form is used."""
    g = graph_of("cl", 600, seed=7)
    X = synth.init_embedding(600, 2, seed=8, scale=scale)
    note(f"wm_terms regime scale={scale}")
    check_terms(g, X)


def test_wm_terms_bf16():
    g = graph_of("sbm", 2048, seed=9)
    X = synth.init_embedding(g.n, 64, seed=10, scale=0.2)
    note("wm_terms bf16 n=2048 d=64")
    check_terms(g, X, gempe.params_default(precision=gempe.GEMPE_BF16_GRAM), z_atol=(g.n - 1) * BF16_Z_FLUSH,
                loss_rtol=1e-4, grad_rtol=1e-3, grad_atol=(g.n - 1) * 2e-18)


@pytest.mark.parametrize("kind,n,d", [("er", 300, 2), ("cl", 900, 16), ("er", 500, 32)])
def test_wm_step_reanchored(kind, n, d):
    """Three Eq. 5 steps, each compared with the oracle's y_i / z_i from the same X."""
    g = graph_of(kind, n, seed=2 * n + d)
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    ws = gempe.workspace(G, d)
    X = to_dev(synth.init_embedding(n, d, seed=5 * n + d))
    for it in range(3):
        x0 = X.double().cpu().numpy()
        lb = torch.empty(1, dtype=torch.float64, device="cuda")
        gempe.wm_step(G, X, ws=ws, loss_before=lb)
        torch.cuda.synchronize()
        x1 = X.double().cpu().numpy()
        xr, ref = oracle.wm_update(x0, g.row_ptr, g.col_idx)
        full = oracle.loss_grad(x0, g.row_ptr, g.col_idx, want_grad=False)
        assert abs(float(lb.item()) - full["loss"]) <= LOSS_RTOL * full["loss"]
        step = xr - x0
        gnorm = np.linalg.norm(ref["grad"], axis=1)
        bound = (GRAD_RTOL * np.maximum(gnorm, GRAD_FLOOR * ref["abs_slope"]) / (2 * ref["z"])
                 + 2 * Z_RTOL * np.linalg.norm(step, axis=1) + 4e-7 * np.linalg.norm(x0, axis=1) + 1e-30)
        err = np.linalg.norm(x1 - xr, axis=1)
        note(f"wm step {it}: worst {np.max(err / bound):.3f} of the bound, mean |step| {np.mean(np.linalg.norm(step, axis=1)):.3e}")
        assert np.all(err <= bound)


def test_embed_wm_matches_steps_and_oracle():
    n, d, iters = 400, 2, 12
    g = graph_of("er", n, seed=77)
    X0 = synth.init_embedding(n, d, seed=78)
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    ws = gempe.workspace(G, d)
    Xa = to_dev(X0)
    h = torch.full((iters + 1,), float("nan"), dtype=torch.float64, device="cuda")
    gempe.embed_wm(G, Xa, iters, ws=ws, loss_hist=h)
    Xb = to_dev(X0)
    losses = []
    for _ in range(iters):
        lb = torch.empty(1, dtype=torch.float64, device="cuda")
        gempe.wm_step(G, Xb, ws=ws, loss_before=lb)
        torch.cuda.synchronize()
        losses.append(float(lb.item()))
    hh = h.cpu().numpy()
    assert np.all(np.isfinite(hh))
    assert np.allclose(hh[:iters], np.array(losses), rtol=1e-5, atol=0)
    ref_hist, X_ref = oracle.wm_trajectory(X0, g.row_ptr, g.col_idx, iters)
    note(f"embed_wm: loss {hh[0]:.6e} -> {hh[-1]:.6e} (oracle {ref_hist[-1]:.6e})")
    assert np.allclose(hh, ref_hist, rtol=1e-4, atol=0)
    assert hh[-1] < hh[0]
