"""Negative-sampled weighted majorization (Sec. III-C) through the C ABI against the oracle.

The sampled vertices are integers decided by the same single-precision mapping and an exact
membership test on both sides, so they are compared bit-exactly.  The step itself is FP32 on
the device and FP64 in the oracle; per vertex the update x - g/(2z) is held to the bound that
the gradient tolerance (1e-4 with the 1e-2 A conditioning floor) and the z tolerance (1e-5)
imply, as for the all-pairs weighted-majorization step."""
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


GRAPHS = {
    "er2000": lambda: synth.erdos_renyi(2000, 12.0, seed=1),
    "cl3400": lambda: synth.chung_lu(3400, 11.2, 2.5, seed=2),
    "star": lambda: synth.csr_from_edges(300, np.zeros(250, np.int64), np.arange(1, 251, dtype=np.int64)),
    "dense": lambda: synth.erdos_renyi(40, 35.0, seed=3),
    "complete": lambda: synth.csr_from_edges(12, *[a.astype(np.int64) for a in np.triu_indices(12, 1)]),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
@pytest.mark.parametrize("seed,tries", [(1, 32), (2 ** 40 + 7, 4)])
def test_samples_bit_exact(name, seed, tries):
    g = GRAPHS[name]()
    X = synth.init_embedding(g.n, 2, seed=5)
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    _, smp = gempe.sampled_step(G, to_dev(X), seed, tries, want_samples=True)
    torch.cuda.synchronize()
    got = smp.cpu().numpy()
    ref = oracle.sample_pairs(g.row_ptr, g.col_idx, g.n, seed, tries)
    note(f"samples {name} seed={seed} tries={tries}: {int(np.sum(ref >= 0))} drawn, {int(np.sum(ref == -1))} empty")
    assert np.array_equal(got, ref), f"{int(np.sum(got != ref))} samples differ"
    if name == "complete":
        assert np.all(got == -1)


def sampled_terms(X, g, smp):
    """Per vertex: g^P, z^P and A^P = sum |d dl/d delta| over the pairs used (oracle pair function)."""
    n, d = X.shape
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    pairs = []
    for e in range(g.nnz):
        i, j = int(rows[e]), int(g.col_idx[e])
        if i < j:
            pairs.append((i, j, True))
            for side, v in ((0, i), (1, j)):
                if smp[2 * e + side] >= 0:
                    pairs.append((v, int(smp[2 * e + side]), False))
    Gv = np.zeros((n, d))
    Z = np.zeros(n)
    A = np.zeros(n)
    for a, b, edge in pairs:
        diff = X[a] - X[b]
        delta = float(np.linalg.norm(diff))
        _, d1, d2 = oracle.pair(delta, edge)
        c = d1 / delta if delta > 0 else 0.0
        Gv[a] += c * diff
        Gv[b] -= c * diff
        Z[a] += d2 / 2
        Z[b] += d2 / 2
        A[a] += abs(d1)
        A[b] += abs(d1)
    return Gv, Z, A


@pytest.mark.parametrize("name,d", [("er2000", 2), ("cl3400", 16), ("dense", 3), ("star", 32)])
def test_sampled_step_against_oracle(name, d):
    g = GRAPHS[name]()
    X0 = synth.init_embedding(g.n, d, seed=9)
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    X = to_dev(X0)
    loss, smp = gempe.sampled_step(G, X, 31337, 32, want_samples=True)
    torch.cuda.synchronize()
    x1 = X.double().cpu().numpy()
    x0 = X0.astype(np.float64)
    xr, lr, sr = oracle.sampled_step(x0, g.row_ptr, g.col_idx, 31337, 32)
    assert np.array_equal(smp.cpu().numpy(), sr)
    assert abs(float(loss.item()) - lr) <= 1e-5 * abs(lr)
    Gv, Z, A = sampled_terms(x0, g, sr)
    step = xr - x0
    zs = np.where(Z > 0, Z, 1.0)
    bound = (1e-4 * np.maximum(np.linalg.norm(Gv, axis=1), 1e-2 * A) / (2 * zs)
             + 2e-5 * np.linalg.norm(step, axis=1) + 4e-7 * np.linalg.norm(x0, axis=1) + 1e-30)
    err = np.linalg.norm(x1 - xr, axis=1)
    note(f"sampled step {name} d={d}: worst {np.max(err / bound):.3f} of the bound")
    assert np.all(err <= bound)


def test_embed_sampled_trajectory():
    g = GRAPHS["er2000"]()
    X0 = synth.init_embedding(g.n, 2, seed=13)
    iters, seed = 6, 4242
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    X = to_dev(X0)
    h = torch.empty(iters, dtype=torch.float64, device="cuda")
    gempe.embed_sampled(G, X, iters, seed, 32, loss_hist=h)
    xo = X0.astype(np.float64)
    hist = []
    for k in range(iters):
        xo, l, _ = oracle.sampled_step(xo, g.row_ptr, g.col_idx, seed + 2 * g.nnz * k, 32)
        hist.append(l)
    hh = h.cpu().numpy()
    note(f"embed_sampled: sampled loss {hh[0]:.6e} -> {hh[-1]:.6e} (oracle {hist[-1]:.6e})")
    assert np.allclose(hh, np.array(hist), rtol=1e-4, atol=0)
    assert np.max(np.abs(X.double().cpu().numpy() - xo)) <= 1e-3 * np.abs(xo).max()


def test_samples_valid_at_scale():
    """A 100,000-vertex power-law graph: every sample is a non-neighbour of its vertex and not
    the vertex itself (checked through the library's exact membership query)."""
    g = synth.chung_lu(100_000, 20.0, 2.3, seed=17)
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    X = to_dev(synth.init_embedding(g.n, 16, seed=18))
    _, smp = gempe.sampled_step(G, X, 99, 32, want_samples=True)
    rows = torch.as_tensor(np.repeat(np.arange(g.n, dtype=np.int32), np.diff(g.row_ptr)), device="cuda")
    cols = torch.as_tensor(g.col_idx, device="cuda")
    s = smp.view(-1, 2)
    upper = rows < cols
    for side, v in ((0, rows), (1, cols)):
        c = s[:, side]
        ok = upper & (c >= 0)
        assert bool(torch.all((c[ok] != v[ok]) & (c[ok] < g.n)))
        hit = gempe.has_edge(G, v[ok], c[ok])
        torch.cuda.synchronize()
        assert int(hit.sum().item()) == 0
        assert bool(torch.all(c[~upper] == -1))
    drawn = int((s[upper] >= 0).sum().item())
    note(f"scale: {drawn} of {2 * g.m} samples drawn")
    assert drawn >= 2 * g.m - 10
