"""Serving loop with continuous batching, through the C ABI.

Each job's result in the mix equals the same job run alone through gempe_embed (within the
trajectory tolerance: the runs differ only in the order of FP32 atomic additions);
admission under a budget that holds one or two jobs at a time; a job over the whole budget
is rejected; a job with a non-finite input or an invalid graph fails alone; sampled jobs
of the mix against the FP64 oracle trajectory."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from gpu_util import note, require_gpu, to_dev
from paper_2011_03479_amd import gempe, synth

pytestmark = pytest.mark.gpu

X_RTOL = 1e-4       # final coordinates: max_i |x_i - x_i'| <= 1e-4 max_i |x_i'|
HIST_RTOL = 1e-5    # loss history, entry by entry


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()
    oracle.build(force=False)


def make_job(n, d, seed, iters, kind="cl"):
    deg = min(12.0, (n - 1) / 3)
    g = synth.chung_lu(n, deg, 2.5, seed=seed) if kind == "cl" else synth.erdos_renyi(n, deg, seed=seed)
    X0 = synth.init_embedding(n, d, seed=1000 + seed)
    prec = gempe.GEMPE_BF16_GRAM if d >= 64 else gempe.GEMPE_FP32
    return dict(g=g, d=d, X0=X0, iters=iters, eta=0.1 / (n - 1), prec=prec)


def run_alone(job):
    g = job["g"]
    p = gempe.params_default(precision=job["prec"])
    G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
    X = to_dev(job["X0"])
    h = torch.empty(job["iters"] + 1, dtype=torch.float64, device="cuda")
    gempe.embed(G, X, job["iters"], job["eta"], params=p, loss_hist=h)
    torch.cuda.synchronize()
    return X.double().cpu().numpy(), h.cpu().numpy()


def submit(srv, job, release_s=0.0):
    g = job["g"]
    return srv.submit(g.n, g.row_ptr, g.col_idx, job["X0"], job["iters"], job["eta"],
                      params=gempe.params_default(precision=job["prec"]), release_s=release_s)


def assert_same(job, X, h, Xr, hr, what):
    scale = max(1.0, float(np.abs(Xr).max()))
    errx = float(np.max(np.abs(X.astype(np.float64) - Xr)))
    assert errx <= X_RTOL * scale, f"{what}: final X differs by {errx:.3e} (scale {scale:.3g})"
    assert np.all(np.isfinite(h)), what
    rel = float(np.max(np.abs(h - hr) / np.abs(hr)))
    assert rel <= HIST_RTOL, f"{what}: loss history differs by {rel:.3e} relative"


MIX = [  # (n, d, seed, kind): batched (d <= 16, small n), solo FP32 (large n or d > 16), solo BF16
    (300, 2, 11, "cl"), (3400, 2, 12, "cl"), (1200, 16, 13, "er"), (700, 3, 14, "er"),
    (2500, 8, 15, "cl"), (30000, 2, 16, "er"), (1500, 32, 17, "cl"), (900, 128, 18, "cl"),
    (5000, 16, 19, "cl"), (450, 1, 20, "er"), (2000, 64, 21, "er"), (6000, 4, 22, "cl"),
]


def test_mix_equals_alone():
    iters = 60
    jobs = [make_job(n, d, s, iters, k) for (n, d, s, k) in MIX]
    alone = []
    for (n, d, s, k), job in zip(MIX, jobs):
        note(f"serve: alone n={n} d={d} seed={s}")
        alone.append(run_alone(job))
    note("serve: mix of 12 jobs, staggered arrivals")
    with gempe.Server(4 << 30) as srv:
        # six at once (the 30,000-vertex job runs for tens of ms), six arriving while they run
        ids = [submit(srv, job, release_s=0.0 if q < 6 else 0.001 * (q - 5)) for q, job in enumerate(jobs)]
        srv.wait(-1, timeout_s=90.0)
        st = srv.stats()
        infos = [srv.query(i) for i in ids]
        for (n, d, s, k), job, jid, info, (Xr, hr) in zip(MIX, jobs, ids, infos, alone):
            assert info.state == gempe.GEMPE_JOB_DONE, (n, d, info, gempe.last_error())
            X, h = srv.result(jid)
            assert_same(job, X, h, Xr, hr, f"n={n} d={d}")
            assert info.batched == (d <= 16 and n <= 23000)
            assert info.release_s <= info.admit_s <= info.done_s
    note(f"serve: stats {st}")
    assert st["done"] == len(MIX) and st["failed"] == 0 and st["rejected"] == 0
    assert st["max_concurrent"] >= 4          # the jobs overlapped on the device
    assert st["ticks"] >= iters + 1           # batched jobs shared launches
    assert st["ticks"] < sum(j["iters"] + 1 for j, (n, d, s, k) in zip(jobs, MIX) if d <= 16 and n <= 23000)
    assert st["peak_bytes"] <= st["budget_bytes"]


def test_admission_under_small_budget():
    iters = 30
    spec = [(2000, 2, 31), (3000, 16, 32), (1000, 2, 33), (2500, 8, 34), (800, 128, 35), (4000, 2, 36)]
    jobs = [make_job(n, d, s, iters) for (n, d, s) in spec]
    fps = [gempe.job_footprint(j["g"].n, j["g"].nnz, j["d"], iters, gempe.params_default(precision=j["prec"]))
           for j in jobs]
    budget = int(max(fps) * 1.3)   # at most one large job (and a small one) at a time
    note(f"serve: admission budget={budget} footprints={fps}")
    big = make_job(20000, 16, 37, iters)
    with gempe.Server(budget) as srv:
        with pytest.raises(gempe.GempeError) as ex:
            submit(srv, big)
        assert ex.value.status == gempe.GEMPE_ERR_NOMEM
        ids = [submit(srv, j) for j in jobs]
        srv.wait(-1, timeout_s=90.0)
        st = srv.stats()
        for (n, d, s), job, jid in zip(spec, jobs, ids):
            info = srv.query(jid)
            assert info.state == gempe.GEMPE_JOB_DONE, (n, d, gempe.last_error())
            X, h = srv.result(jid)
            Xr, hr = run_alone(job)
            assert_same(job, X, h, Xr, hr, f"n={n} d={d}")
    assert st["rejected"] == 1 and st["done"] == len(spec)
    assert st["peak_bytes"] <= budget
    assert st["max_concurrent"] < len(spec)  # the budget bound admission


def test_failures_stay_with_their_job():
    iters = 20
    good = [make_job(1000, 2, 41, iters), make_job(1500, 16, 42, iters), make_job(600, 32, 43, iters)]
    nan_job = make_job(800, 2, 44, iters)
    nan_job["X0"] = nan_job["X0"].copy()
    nan_job["X0"][17, 1] = np.nan
    bad = make_job(500, 2, 45, iters)
    g = bad["g"]
    rp, ci = g.row_ptr.copy(), g.col_idx.copy()
    # drop the mirror of one edge: (i, j) present without (j, i) -> invalid graph
    i = int(np.argmax(np.diff(rp) > 0))
    ci[rp[i]] = (ci[rp[i]] + 1) % g.n if (ci[rp[i]] + 1) % g.n != i else (ci[rp[i]] + 2) % g.n
    note("serve: NaN job, invalid-graph job and three good jobs")
    with gempe.Server(1 << 30) as srv:
        ids = [submit(srv, j) for j in good]
        nid = submit(srv, nan_job)
        bid = srv.submit(g.n, rp, ci, bad["X0"], iters, bad["eta"])
        srv.wait(-1, timeout_s=60.0)
        ninfo, binfo = srv.query(nid), srv.query(bid)
        assert ninfo.state == gempe.GEMPE_JOB_FAILED and ninfo.status == gempe.GEMPE_ERR_NUMERIC
        assert binfo.state == gempe.GEMPE_JOB_FAILED and binfo.status == gempe.GEMPE_ERR_GRAPH
        for job, jid in zip(good, ids):
            assert srv.query(jid).state == gempe.GEMPE_JOB_DONE
            X, h = srv.result(jid)
            Xr, hr = run_alone(job)
            assert_same(job, X, h, Xr, hr, f"good n={job['g'].n}")
        st = srv.stats()
    assert st["failed"] == 2 and st["done"] == 3


def test_sampled_jobs_against_oracle():
    """Two jobs of a mix against the FP64 oracle's gradient-descent trajectory."""
    iters = 40
    jobs = [make_job(300, 2, 51, iters), make_job(400, 16, 52, iters, "er"), make_job(5000, 2, 53, iters)]
    with gempe.Server(1 << 30) as srv:
        ids = [submit(srv, j, release_s=0.001 * q) for q, j in enumerate(jobs)]
        srv.wait(-1, timeout_s=60.0)
        for job, jid in list(zip(jobs, ids))[:2]:
            assert srv.query(jid).state == gempe.GEMPE_JOB_DONE
            X, h = srv.result(jid)
            g = job["g"]
            note(f"serve: oracle trajectory n={g.n} d={job['d']}")
            ref_hist, X_ref = oracle.gd_trajectory(job["X0"], g.row_ptr, g.col_idx, iters, job["eta"])
            assert np.allclose(h, ref_hist, rtol=1e-5, atol=0)
            err = np.max(np.linalg.norm(X.astype(np.float64) - X_ref, axis=1))
            assert err <= 1e-4 * np.max(np.linalg.norm(X_ref, axis=1))


def test_wait_timeout_and_destroy_with_work_pending():
    job = make_job(30000, 2, 61, 400, "er")
    srv = gempe.Server(2 << 30)
    jid = submit(srv, job)
    with pytest.raises(gempe.GempeError) as ex:
        srv.wait(jid, timeout_s=0.0)
    assert ex.value.status == gempe.GEMPE_ERR_TIMEOUT
    late = submit(srv, make_job(500, 2, 62, 10), release_s=3600.0)
    srv.close()  # the scheduler stops; unfinished jobs are not reported as done
    assert srv.handle is None
    del late
