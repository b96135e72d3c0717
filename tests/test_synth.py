"""Seeded generators: well-formed CSR, realised edge counts near expectation, determinism."""
import numpy as np
import pytest

from paper_2011_03479_amd import synth


def check_csr(g):
    n = g.n
    rp, ci = g.row_ptr, g.col_idx
    assert rp.dtype == np.int64 and ci.dtype == np.int32
    assert rp[0] == 0 and rp[-1] == ci.shape[0] and np.all(np.diff(rp) >= 0)
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.all((ci >= 0) & (ci < n))
    assert not np.any(rows == ci), "self-loop"
    # strictly increasing within rows (sorted, no duplicates)
    same_row = rows[1:] == rows[:-1]
    assert np.all(ci[1:][same_row] > ci[:-1][same_row])
    # symmetric
    fwd = rows.astype(np.int64) * n + ci
    bwd = ci.astype(np.int64) * n + rows
    assert np.array_equal(np.sort(fwd), np.sort(bwd))


@pytest.mark.parametrize("make", [
    lambda: synth.erdos_renyi(1000, 10.0, seed=1),
    lambda: synth.erdos_renyi(5000, 8.0, seed=9),
    lambda: synth.chung_lu(3400, 2 * 19000 / 3400, 2.5, seed=2),
    lambda: synth.sbm(10, 300, 2e-2, 2e-4, seed=3),
])
def test_generator_csr_and_edge_count(make):
    g = make()
    check_csr(g)
    em = g.meta["expected_m"]
    # realised m within 5 sd of its expectation (sum of independent Bernoullis: var <= mean)
    assert abs(g.m - em) <= 5 * np.sqrt(em) + 5 * 0.02 * em * (g.meta["kind"] == "chung_lu")


def test_generators_are_seeded():
    a = synth.chung_lu(2000, 10.0, 2.3, seed=4)
    b = synth.chung_lu(2000, 10.0, 2.3, seed=4)
    c = synth.chung_lu(2000, 10.0, 2.3, seed=5)
    assert np.array_equal(a.col_idx, b.col_idx) and np.array_equal(a.row_ptr, b.row_ptr)
    assert not (a.m == c.m and np.array_equal(a.col_idx, c.col_idx))
    x = synth.init_embedding(100, 3, 7)
    assert x.dtype == np.float32 and np.array_equal(x, synth.init_embedding(100, 3, 7))


def test_upper_index_mapping_bijective():
    n = 37
    L = np.arange(n * (n - 1) // 2)
    i, j = synth._upper_index_to_pair(n, L)
    assert np.all(i < j) and np.all(j < n)
    assert len(set(zip(i.tolist(), j.tolist()))) == L.size


def test_workload_shapes():
    w = synth.workload("er1k")
    assert w.graph.n == 1000 and w.d == 2 and w.iters == 100 and w.X0.shape == (1000, 2)
    w2 = synth.workload("cl3400")
    assert w2.graph.n == 3400 and abs(w2.graph.m - 19000) < 600 and w2.iters == 1000


def test_serving_stream_shape():
    jobs = synth.serving_stream(6, rate_per_s=10.0, seed=5, n_min=500, n_max=2000, iters=3)
    assert len(jobs) == 6
    assert all(500 <= j.graph.n <= 2000 for j in jobs)
    assert all(j.d in (2, 16, 128) for j in jobs)
    assert all(b.arrival_s > a.arrival_s for a, b in zip(jobs, jobs[1:]))
    for j in jobs:
        check_csr(j.graph)
