"""One device's share of the all-pairs sweep (gempe_loss_grad_shard) against the FP64 oracle's
shard of the pair sum, and the shards against the whole."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from gpu_util import GRAD_FLOOR, GRAD_RTOL, LOSS_RTOL, assert_grad_close, assert_loss_close, note, require_gpu, to_dev
from paper_2011_03479_amd import gempe, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()
    oracle.build(force=False)


SHAPES = [(1500, 2), (1000, 16), (700, 40), (3000, 8), (129, 3)]


@pytest.mark.parametrize("n,d", SHAPES, ids=[f"n{n}_d{d}" for n, d in SHAPES])
def test_shards_match_oracle_and_sum_to_whole(n, d):
    g = synth.chung_lu(n, min(10.0, (n - 1) / 3), 2.5, seed=n + 3 * d)
    X0 = synth.init_embedding(n, d, seed=7 * n + d)
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    ws = gempe.workspace(G, d)
    X = to_dev(X0)
    T = gempe.shard_rows(G, d)
    assert T % 64 == 0 and T > 0
    full = gempe.loss_grad(G, X, ws=ws)
    torch.cuda.synchronize()
    ref_full = oracle.loss_grad(X0, g.row_ptr, g.col_idx, want_abs_slope=True)
    A = ref_full["abs_slope"]
    for nsh in (1, 2, 3, 8):
        note(f"shard n={n} d={d} T={T} nshards={nsh}")
        tot_loss, tot_hits, tot_grad = 0.0, 0, np.zeros((n, d))
        for s in range(nsh):
            r = gempe.loss_grad_shard(G, X, s, nsh, ws=ws)
            torch.cuda.synchronize()
            ref = oracle.loss_grad_shard(X0, g.row_ptr, g.col_idx, T, nsh, s)
            loss, hits, grad = float(r.loss.item()), int(r.edge_hits.item()), r.grad.double().cpu().numpy()
            assert hits == ref["edge_hits"], (s, hits, ref["edge_hits"])
            if ref["loss"] > 0:
                assert_loss_close(loss, ref["loss"], what=f"shard {s}/{nsh}")
            else:
                assert loss == 0.0
            # a shard's gradient cancels less than the whole: the whole's term scale is the floor
            assert_grad_close(grad, ref["grad"], A, what=f"shard {s}/{nsh}")
            tot_loss += loss
            tot_hits += hits
            tot_grad += grad
        assert tot_hits == g.m
        assert abs(tot_loss - float(full.loss.item())) <= LOSS_RTOL * ref_full["loss"]
        assert_grad_close(tot_grad, full.grad.double().cpu().numpy(), A, what=f"sum of {nsh} shards")


def test_shard_arguments():
    g = synth.erdos_renyi(200, 5.0, seed=1)
    G = gempe.Graph(200, g.row_ptr, g.col_idx)
    X = to_dev(synth.init_embedding(200, 2, seed=2))
    for s, nsh in ((-1, 2), (2, 2), (0, 0)):
        with pytest.raises(gempe.GempeError):
            gempe.loss_grad_shard(G, X, s, nsh)
    with pytest.raises(gempe.GempeError):
        gempe.loss_grad_shard(G, to_dev(synth.init_embedding(200, 16, seed=2)), 0, 2,
                              params=gempe.params_default(precision=gempe.GEMPE_BF16_GRAM))
    # more shards than strip pairs: the extra shards own nothing
    r = gempe.loss_grad_shard(G, X, 7, 8)
    torch.cuda.synchronize()
    assert float(r.loss.item()) == 0.0 and int(r.edge_hits.item()) == 0
    assert float(r.grad.abs().max().item()) == 0.0


def test_shard_at_full_size():
    """One of eight shards of the 1M-vertex Chung-Lu graph at d = 16 (one GPU's share of that
    sweep at its real shape): sampled rows against the oracle's shard, and the time of the
    shard against the whole evaluation."""
    w = synth.workload("cl1m")
    g = w.graph
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    ws = gempe.workspace(G, w.d)
    X = to_dev(w.X0)
    T = gempe.shard_rows(G, w.d)
    rng = np.random.default_rng(5)
    hubs = np.argsort(-np.diff(g.row_ptr))[:4]
    rows = np.unique(np.concatenate([rng.choice(g.n, 40, replace=False), hubs, [0, g.n - 1]]))
    note(f"cl1m shard 3 of 8, T={T}")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    r = gempe.loss_grad_shard(G, X, 3, 8, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    t_shard = e0.elapsed_time(e1)
    ref = oracle.rows_shard(w.X0, g.row_ptr, g.col_idx, rows, T, 8, 3)
    ref_a = oracle.rows(w.X0, g.row_ptr, g.col_idx, rows)["abs_slope"]
    assert_grad_close(r.grad.double().cpu().numpy()[rows], ref, ref_a, what="cl1m shard 3/8")
    e0.record()
    full = gempe.loss_grad(G, X, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    t_full = e0.elapsed_time(e1)
    note(f"cl1m: shard 3/8 {t_shard:.1f} ms, whole {t_full:.1f} ms")
    assert float(r.loss.item()) < float(full.loss.item())
    assert t_shard < 0.25 * t_full
