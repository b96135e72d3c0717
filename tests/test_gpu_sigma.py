"""Slope optimisation (Sec. III-F) through the C ABI: distance histograms bit-exact against
the oracle (integer counts from the same single-precision bin decision), the histogram
bisection against the oracle's, the histogram slope against the exact all-pairs slope, and
weighted majorization with the slope refitted against the oracle's composition."""
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


def clustered(blocks, size, d, seed, spread=3.0, noise=0.6, p_in=0.3, p_out=0.01):
    g = synth.sbm(blocks, size, p_in, p_out, seed=seed, permute=False)
    rng = np.random.default_rng(seed + 1)
    centres = spread * rng.standard_normal((blocks, d))
    X = centres[np.repeat(np.arange(blocks), size)] + noise * rng.standard_normal((blocks * size, d))
    return g, X.astype(np.float32)


def gpu_hist(g, X32, nbins, r2_max):
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    ha, he = gempe.distance_histogram(G, to_dev(X32), nbins, r2_max)
    torch.cuda.synchronize()
    return ha.cpu().numpy().astype(np.uint64), he.cpu().numpy().astype(np.uint64)


SHAPES = [(1, 300, 257), (2, 1000, 4096), (3, 700, 4096), (5, 450, 1000), (16, 1300, 16384), (17, 333, 4096),
          (32, 600, 2048), (100, 260, 4096), (128, 520, 8192)]


@pytest.mark.parametrize("d,n,nbins", SHAPES, ids=[f"d{d}_n{n}_b{b}" for d, n, b in SHAPES])
def test_histogram_bit_exact(d, n, nbins):
    g = synth.chung_lu(n, min(10.0, (n - 1) / 3), 2.5, seed=n + d)
    X = synth.init_embedding(n, d, seed=7 * n + d)
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    r2_max = gempe.r2_bound(G, to_dev(X))
    note(f"histogram d={d} n={n} nbins={nbins} r2_max={r2_max:.4g}")
    diffs = X.astype(np.float64)[:, None, :] - X.astype(np.float64)[None, :, :] if n <= 1300 and d <= 16 else None
    if diffs is not None:
        assert np.max(np.sum(diffs ** 2, axis=2)) <= r2_max
    ha, he = gpu_hist(g, X, nbins, r2_max)
    ra, re = oracle.histogram(X, g.row_ptr, g.col_idx, nbins, r2_max)
    assert int(ha.sum()) == n * (n - 1) // 2 and int(he.sum()) == g.m
    assert np.array_equal(ha, ra), f"all-pair counts differ in {int(np.sum(ha != ra))} bins"
    assert np.array_equal(he, re), f"edge counts differ in {int(np.sum(he != re))} bins"


def test_histogram_edge_cases():
    """Coincident points (every pair in bin 0), a graph without edges, the largest bin count."""
    n = 200
    g = synth.erdos_renyi(n, 0.0, seed=1)
    X = np.zeros((n, 2), np.float32)
    ha, he = gpu_hist(g, X, 16384, 1.0)
    assert int(ha[0]) == n * (n - 1) // 2 and int(ha[1:].sum()) == 0 and int(he.sum()) == 0
    g2 = synth.erdos_renyi(n, 5.0, seed=2)
    X2 = synth.init_embedding(n, 2, seed=3)
    ha, he = gpu_hist(g2, X2, 2, 1e-3)   # almost every pair clamps into the last bin
    ra, re = oracle.histogram(X2, g2.row_ptr, g2.col_idx, 2, 1e-3)
    assert np.array_equal(ha, ra) and np.array_equal(he, re)


@pytest.mark.parametrize("d", [2, 16, 64])
def test_sigma_fit(d):
    g, X = clustered(5, 80, d, seed=11 + d)
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    r2_max = gempe.r2_bound(G, to_dev(X))
    ha, he = gpu_hist(g, X, 16384, r2_max)
    s_gpu = gempe.sigma_fit(ha, he, r2_max, 1.5)
    s_orc = oracle.sigma_from_histogram(ha, he, r2_max, 1.5)
    s_exact = oracle.sigma_exact(X.astype(np.float64), g.row_ptr, g.col_idx, 1.5)
    note(f"sigma d={d}: library {s_gpu:.10f} oracle(hist) {s_orc:.10f} exact {s_exact:.10f}")
    assert 1e-3 < s_exact < 1e3
    assert abs(s_gpu / s_orc - 1) <= 1e-10
    # the histogram's own approximation (bins uniform in the squared distance, evaluated at the
    # bin centre): 16,384 bins put the slope within 5e-4 of the exact all-pairs slope here
    assert abs(s_gpu / s_exact - 1) <= 5e-4


def test_sigma_fit_host_checks():
    ha = np.array([5, 5], np.uint64)
    he = np.array([6, 0], np.uint64)
    with pytest.raises(gempe.GempeError):
        gempe.sigma_fit(ha, he, 1.0)           # more edges than pairs in a bin
    with pytest.raises(gempe.GempeError):
        gempe.sigma_fit(ha, np.zeros(2, np.uint64), 1.0, sigma_lo=2.0, sigma_hi=1.0)


def test_embed_wm_sigma_against_oracle():
    """WM with the slope refitted every two steps; the oracle composes its own WM update, its
    own histogram of the single-precision coordinates and its own bisection."""
    g, X0 = clustered(4, 60, 2, seed=21, spread=2.0, noise=1.0)
    iters, every, nbins = 8, 2, 4096
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    X = to_dev(X0)
    h = torch.empty(iters + 1, dtype=torch.float64, device="cuda")
    s_final = gempe.embed_wm_sigma(G, X, iters, 1.0, sigma_every=every, nbins=nbins, loss_hist=h)
    hh = h.cpu().numpy()
    # oracle composition
    Xo = X0.astype(np.float64)
    sigma = 1.0
    hist = []
    for k in range(iters + 1):
        hist.append(oracle.loss_grad(Xo, g.row_ptr, g.col_idx, 1.5, sigma, want_grad=False)["loss"])
        if k == iters:
            break
        Xo, _ = oracle.wm_update(Xo, g.row_ptr, g.col_idx, 1.5, sigma)
        if (k + 1) % every == 0:
            X32 = Xo.astype(np.float32)
            box = X32.max(0).astype(np.float64) - X32.min(0).astype(np.float64)
            r2_max = float(np.float32(np.sum(box * box) * (1 + 1e-5) + 1e-30))
            ra, re = oracle.histogram(X32, g.row_ptr, g.col_idx, nbins, r2_max)
            sigma = oracle.sigma_from_histogram(ra, re, r2_max, 1.5)
    note(f"embed_wm_sigma: sigma {s_final:.6f} (oracle {sigma:.6f}), loss {hh[0]:.6e} -> {hh[-1]:.6e} "
         f"(oracle {hist[-1]:.6e})")
    assert abs(s_final / sigma - 1) <= 1e-4
    assert np.allclose(hh, np.array(hist), rtol=1e-4, atol=0)
    assert np.allclose(X.double().cpu().numpy(), Xo, rtol=0, atol=1e-3 * np.abs(Xo).max())
