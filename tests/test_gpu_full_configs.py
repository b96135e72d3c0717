"""The full-size workloads after their iterations, against the FP64 oracle.

  - the SBM workload (n = 100,000, d = 128, BF16 Gram): 20 gradient-descent iterations;
    loss and per-vertex gradient on a 2,000-vertex subsample at iterations 0 and 20 (the
    oracle evaluates those rows against all n vertices at the GPU's iterate), and the
    full-size coding cost at X0 against one full oracle evaluation (stored by
    tests/golden/gen_full_loss.py, which calls only the oracle);
  - the same graph from the contracted start (X0 ~ N(0, (mu / sqrt(2d))^2): nearly every
    pair near, the exact pass covers almost all tiles): full-size loss against the stored
    oracle value, and the 2,000-vertex subsample;
  - the 1M-vertex Chung-Lu workload (d = 16), FP32 and BF16 Gram: sampled rows (the hubs
    included) after its 5 iterations.
The tolerances are the FP32 and BF16 bounds of gpu_util.
"""
import json
import os

import numpy as np
import pytest
import torch

from gpu_util import (BF16_FLUSH_GRAD, BF16_GRAD_RTOL, BF16_LOSS_RTOL, LOSS_RTOL, check_rows, check_rows_plain,
                      note, require_gpu, to_dev)
from paper_2011_03479_amd import gempe, synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_loss.json")


def _golden(w):
    import hashlib

    rec = json.load(open(GOLDEN))[w.name]
    h = hashlib.sha256()
    for a in (w.graph.row_ptr, w.graph.col_idx, w.X0):
        h.update(np.ascontiguousarray(a).tobytes())
    assert h.hexdigest() == rec["fingerprint"], f"{w.name}: inputs differ from those of the stored oracle value"
    assert rec["m"] == w.graph.m and rec["edge_hits"] == w.graph.m
    return rec


def _bf16_rows(g, G, X, rows, what):
    return check_rows(g, G, X, rows, params=gempe.params_default(precision=gempe.GEMPE_BF16_GRAM), what=what,
                      loss_rtol=BF16_LOSS_RTOL, grad_rtol=BF16_GRAD_RTOL, grad_atol=(g.n - 1) * BF16_FLUSH_GRAD)


def _subsample(g, k, seed):
    rng = np.random.default_rng(seed)
    hubs = np.argsort(-np.diff(g.row_ptr))[:8]
    return np.unique(np.concatenate([rng.choice(g.n, k, replace=False), hubs, [0, g.n - 1]]))


def test_sbm100k_twenty_iterations():
    require_gpu()
    w = synth.workload("sbm100k")
    g = w.graph
    rec = _golden(w)
    rows = _subsample(g, 2000, 20)
    note(f"sbm100k: {w.iters} BF16 iterations, {rows.size} sampled rows at iterations 0 and {w.iters}")
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    p = gempe.params_default(precision=gempe.GEMPE_BF16_GRAM)
    ws = gempe.workspace(G, w.d, p)
    X = to_dev(w.X0)
    hist = torch.empty(w.iters + 1, dtype=torch.float64, device="cuda")
    gempe.embed(G, X, w.iters, w.eta, ws=ws, params=p, loss_hist=hist)
    h = hist.cpu().numpy()
    # the whole-graph loss at X0 against one full FP64 evaluation (the flushed far pairs add
    # < 2e-19 bits each, so it meets the FP32 bound too)
    assert abs(h[0] - rec["loss_bits"]) <= LOSS_RTOL * rec["loss_bits"], (h[0], rec["loss_bits"])
    assert np.all(np.isfinite(h)), h
    X20 = X.cpu().numpy()
    _bf16_rows(g, G, w.X0, rows, "sbm100k iteration 0")
    got, _ = _bf16_rows(g, G, X20, rows, f"sbm100k iteration {w.iters}")
    # the evaluation at the final iterate agrees with the run's own history entry
    assert abs(got["loss"] - h[-1]) <= 1e-9 * h[-1], (got["loss"], h[-1])
    G.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_sbm100k_full_loss(prec):
    """Whole-graph loss at X0 against the stored full oracle evaluation, in FP32 (every pair
    exact) and with the BF16 screen."""
    require_gpu()
    w = synth.workload("sbm100k")
    rec = _golden(w)
    note(f"sbm100k full loss {prec}")
    G = gempe.Graph(w.graph.n, w.graph.row_ptr, w.graph.col_idx)
    p = gempe.params_default(precision=gempe.GEMPE_BF16_GRAM if prec == "bf16" else gempe.GEMPE_FP32)
    r = gempe.loss_grad(G, to_dev(w.X0), params=p, want_grad=False)
    assert int(r.edge_hits.item()) == w.graph.m
    loss = float(r.loss.item())
    assert abs(loss - rec["loss_bits"]) <= LOSS_RTOL * rec["loss_bits"], (loss, rec["loss_bits"])
    G.close()


def test_sbm100k_contracted_start():
    """T9: X0 ~ N(0, (mu / sqrt(2d))^2) on the SBM graph, BF16 screen: almost every tile is
    flagged and recomputed exactly.  Whole-graph loss against the stored oracle value and a
    2,000-vertex subsample of rows."""
    require_gpu()
    w = synth.workload("sbm100k_t9")
    g = w.graph
    rec = _golden(w)
    rows = _subsample(g, 2000, 9)
    note(f"sbm100k contracted start: full loss and {rows.size} sampled rows")
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    got, _ = _bf16_rows(g, G, w.X0, rows, "sbm100k contracted")
    assert abs(got["loss"] - rec["loss_bits"]) <= BF16_LOSS_RTOL * rec["loss_bits"], (got["loss"], rec["loss_bits"])
    G.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_cl1m_after_iterations(prec):
    """The 1M-vertex workload after its 5 iterations: sampled rows (hubs included) at the
    GPU's final iterate against the oracle, FP32 and BF16 bounds."""
    require_gpu()
    w = synth.workload("cl1m")
    g = w.graph
    rows = _subsample(g, 60, 5)
    note(f"cl1m {prec}: {w.iters} iterations, then {rows.size} sampled rows")
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    p = gempe.params_default(precision=gempe.GEMPE_BF16_GRAM if prec == "bf16" else gempe.GEMPE_FP32)
    ws = gempe.workspace(G, w.d, p)
    X = to_dev(w.X0)
    hist = torch.empty(w.iters + 1, dtype=torch.float64, device="cuda")
    gempe.embed(G, X, w.iters, w.eta, ws=ws, params=p, loss_hist=hist)
    h = hist.cpu().numpy()
    assert np.all(np.isfinite(h)), h
    del ws
    X5 = X.cpu().numpy()
    if prec == "fp32":
        # the plain evaluation (the sweep gradient descent runs) and the one with row losses
        loss, _ = check_rows_plain(g, G, X5, rows, what="cl1m fp32 after 5 iterations")
    else:
        got, _ = _bf16_rows(g, G, X5, rows, "cl1m bf16 after 5 iterations")
        loss = got["loss"]
    # the run's own history entry for the final iterate, within the FP32 bound
    assert abs(loss - h[-1]) <= LOSS_RTOL * h[-1], (loss, h[-1])
    G.close()
