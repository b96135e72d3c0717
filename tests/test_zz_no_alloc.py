"""gempe_loss_grad_noalloc (the entry point for callers that cannot allocate) against
gempe_loss_grad, through the C ABI: two calls in a row on one device, the second with a
smaller problem (fewer vertices and a different dimension, so a different tile plan and
partial count over the static scratch the first call left behind), each checked against
gempe_loss_grad on the same input and against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import (assert_grad_close, assert_loss_close, note, require_gpu, to_dev)
from paper_2011_03479_amd import gempe, synth

pytestmark = pytest.mark.gpu


def _pair_of_calls(graph, d, seed, row_loss):
    G = gempe.Graph(graph.n, graph.row_ptr, graph.col_idx)
    X0 = synth.init_embedding(graph.n, d, seed)
    X = to_dev(X0)
    assert gempe.loss_grad_noalloc_bytes(G, d) <= gempe.NOALLOC_SCRATCH_BYTES
    ref = gempe.loss_grad(G, X, want_row_loss=row_loss)
    got = gempe.loss_grad_noalloc(G, X, want_row_loss=row_loss)
    torch.cuda.synchronize()
    orc = oracle.loss_grad(X0, graph.row_ptr, graph.col_idx, want_row_loss=True, want_abs_slope=True)
    what = f"noalloc n={graph.n} d={d}"
    # the same kernels and the same fixed-order FP64 reduction: the loss is bitwise equal
    assert float(got.loss.item()) == float(ref.loss.item()), what
    assert int(got.edge_hits.item()) == int(ref.edge_hits.item()) == graph.m, what
    assert_loss_close(float(got.loss.item()), orc["loss"], what=what)
    g_got = got.grad.double().cpu().numpy()
    assert_grad_close(g_got, ref.grad.double().cpu().numpy(), orc["abs_slope"], what=what + " vs loss_grad")
    assert_grad_close(g_got, orc["grad"], orc["abs_slope"], what=what + " vs oracle")
    if row_loss:
        rl = got.row_loss.double().cpu().numpy()
        assert np.all(np.abs(rl - orc["row_loss"]) <= 1e-5 * np.abs(orc["row_loss"]) + 1e-6), what
    G.close()


def test_noalloc_two_calls_second_smaller():
    require_gpu()
    note("noalloc: n=6000 d=16 Chung-Lu, then n=1500 d=3 Erdos-Renyi")
    _pair_of_calls(synth.chung_lu(6000, 12.0, 2.5, seed=21), 16, 2021, row_loss=True)
    _pair_of_calls(synth.erdos_renyi(1500, 9.0, seed=22), 3, 2022, row_loss=False)


def test_noalloc_rejects_oversized_and_bf16():
    require_gpu()
    note("noalloc: host-side rejections")
    n = 300_000
    u = np.arange(n - 1, dtype=np.int64)
    g = synth.csr_from_edges(n, u, u + 1)
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    X = torch.zeros((n, 32), dtype=torch.float32, device="cuda")
    assert gempe.loss_grad_noalloc_bytes(G, 32) > gempe.NOALLOC_SCRATCH_BYTES
    with pytest.raises(gempe.GempeError) as e:
        gempe.loss_grad_noalloc(G, X)
    assert e.value.status == gempe.GEMPE_ERR_NOMEM
    with pytest.raises(gempe.GempeError) as e:
        gempe.loss_grad_noalloc(G, X, params=gempe.params_default(precision=gempe.GEMPE_BF16_GRAM))
    assert e.value.status == gempe.GEMPE_ERR_UNSUPPORTED
    G.close()
