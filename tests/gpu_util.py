"""Helpers for the GPU parity tests: run the HIP path through the C ABI, compare with the
FP64 oracle.

Tolerances (FP32 path):
  loss:      |DL - DL*| <= 1e-5 DL*
  gradient:  per vertex, |g_i - g_i*| <= 1e-4 max(|g_i*|, 1e-2 A_i),
             A_i = sum_j |d dl_ij / d delta| (the size of the terms that cancel in g_i)
"""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
from paper_2011_03479_amd import gempe

LOSS_RTOL = 1e-5
GRAD_RTOL = 1e-4
GRAD_FLOOR = 1e-2
# BF16 Gram screen: the stated looser bound (the flushed far pairs themselves are below
# 2e-19 bits each; the bound leaves room for the screen's conservative choices)
BF16_LOSS_RTOL = 1e-4
BF16_GRAD_RTOL = 1e-3
# a flushed non-edge (delta >= mu + 9 sigma) has |d dl / d delta| <= R(9)/ln2 < 2e-18, so
# the flush moves |g_i| by at most (n - 1) 2e-18: the absolute part of the BF16 bound
BF16_FLUSH_GRAD = 2e-18


def note(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def require_gpu():
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    gempe.load()


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def gpu_loss_grad(G, X, params=None, row_loss=False):
    Xd = to_dev(X)
    r = gempe.loss_grad(G, Xd, params=params, want_row_loss=row_loss)
    torch.cuda.synchronize()
    out = {
        "loss": float(r.loss.item()),
        "grad": r.grad.double().cpu().numpy(),
        "edge_hits": int(r.edge_hits.item()),
    }
    if row_loss:
        out["row_loss"] = r.row_loss.double().cpu().numpy()
    return out


def grad_errors(g, ref, A, rtol=GRAD_RTOL, floor=GRAD_FLOOR, atol=0.0):
    err = np.linalg.norm(g - ref, axis=1)
    bound = rtol * np.maximum(np.linalg.norm(ref, axis=1), floor * A) + atol
    return err, bound


def assert_grad_close(g, ref, A, rtol=GRAD_RTOL, floor=GRAD_FLOOR, what="", atol=0.0):
    err, bound = grad_errors(g, ref, A, rtol, floor, atol)
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, (f"{what}: {bad.size} vertices over the gradient bound; worst ratio "
                           f"{float(np.max(err / np.maximum(bound, 1e-300))):.3g} at vertex {int(bad[0])}")


def assert_loss_close(loss, ref, rtol=LOSS_RTOL, what=""):
    assert abs(loss - ref) <= rtol * abs(ref), f"{what}: loss {loss!r} vs oracle {ref!r} (rel {abs(loss-ref)/abs(ref):.3g})"


def check_full(graph, G, X, mu=1.5, sigma=1.0, params=None, row_loss=True, what="", loss_rtol=LOSS_RTOL,
               grad_rtol=GRAD_RTOL, grad_atol=0.0):
    """Whole-graph parity: loss, every vertex's gradient, edge hits, row losses."""
    got = gpu_loss_grad(G, X, params=params, row_loss=row_loss)
    ref = oracle.loss_grad(X, graph.row_ptr, graph.col_idx, mu, sigma, want_row_loss=True, want_abs_slope=True)
    assert got["edge_hits"] == graph.m == ref["edge_hits"], (what, got["edge_hits"], graph.m)
    assert_loss_close(got["loss"], ref["loss"], rtol=loss_rtol, what=what)
    assert_grad_close(got["grad"], ref["grad"], ref["abs_slope"], rtol=grad_rtol, what=what, atol=grad_atol)
    if row_loss:
        rl = got["row_loss"]
        assert np.all(np.abs(rl - ref["row_loss"]) <= loss_rtol * np.abs(ref["row_loss"]) + 1e-6), what
    return got, ref


def check_rows(graph, G, X, rows, mu=1.5, sigma=1.0, params=None, what="", loss_rtol=LOSS_RTOL,
               grad_rtol=GRAD_RTOL, grad_atol=0.0):
    """Sampled-row parity for sizes the oracle cannot sweep whole."""
    got = gpu_loss_grad(G, X, params=params, row_loss=True)
    ref = oracle.rows(X, graph.row_ptr, graph.col_idx, rows, mu, sigma)
    assert got["edge_hits"] == graph.m, (what, got["edge_hits"], graph.m)
    assert_grad_close(got["grad"][rows], ref["grad"], ref["abs_slope"], rtol=grad_rtol, what=what,
                      atol=grad_atol)
    rl = got["row_loss"][rows]
    assert np.all(np.abs(rl - ref["row_loss"]) <= loss_rtol * np.abs(ref["row_loss"]) + 1e-6), what
    # the loss is half the sum of the row losses (self-consistency at full size)
    half = 0.5 * float(np.sum(got["row_loss"]))
    assert abs(half - got["loss"]) <= 1e-5 * got["loss"], (what, half, got["loss"])
    return got, ref


def check_rows_plain(graph, G, X, rows, mu=1.5, sigma=1.0, params=None, what="", loss_rtol=LOSS_RTOL,
                     grad_rtol=GRAD_RTOL, grad_atol=0.0):
    """Sampled-row parity of a plain loss-and-gradient evaluation (no per-vertex extras, the
    call the gradient-descent loop makes): the sampled gradient rows against the oracle, and
    the loss against the evaluation that also returns the row losses, whose rows are checked
    against the oracle and whose halved sum is its loss."""
    Xd = to_dev(X)
    r = gempe.loss_grad(G, Xd, params=params)
    torch.cuda.synchronize()
    loss, grad = float(r.loss.item()), r.grad.double().cpu().numpy()
    assert int(r.edge_hits.item()) == graph.m, (what, int(r.edge_hits.item()), graph.m)
    ref = oracle.rows(X, graph.row_ptr, graph.col_idx, rows, mu, sigma)
    assert_grad_close(grad[rows], ref["grad"], ref["abs_slope"], rtol=grad_rtol, what=what, atol=grad_atol)
    full, _ = check_rows(graph, G, X, rows, mu, sigma, params, what + " (with row losses)", loss_rtol, grad_rtol,
                         grad_atol)
    assert abs(loss - full["loss"]) <= loss_rtol * abs(full["loss"]), (what, loss, full["loss"])
    return loss, grad
