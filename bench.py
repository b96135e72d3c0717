"""Benchmark: all-pairs GEMPE gradient iterations on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cl1m]

A step is one full iteration of the hot path: the all-pairs sweep (loss and gradient of
every unordered vertex pair), the exact edge correction, the FP64 loss reduction with its
finite check, and the update X <- X - eta G.  The default workload is the large all-pairs
sweep: a Chung-Lu power-law graph with n = 1,000,000 vertices, mean degree 20 and degree
exponent 2.3 (about 1e7 edges), d = 16, FP32; the same graph with the BF16 MFMA Gram screen
is measured in the same run under `variants`, and the other workloads (the drawing-sized
graph at d = 2, the SBM at d = 128 in BF16 and in FP32) under `extras`.  Prints one JSON line with
pairs/s (unordered pairs x iterations / time), the roofline figures of the dominant
kernel, timed with HIP events on the stream it runs on, the FP64 CPU oracle timed on the
host on a bounded sample of rows, and the serving mix.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3    # MI355X dense FP32 vector (AMD published)
PEAK_BF16_TFLOPS = 2516.6   # MI355X dense BF16 MFMA (AMD published, without sparsity)
# the stated parity bounds: per-vertex gradient error relative to max(|g*|, 1e-2 A_i), loss
FP32_GRAD, FP32_LOSS = 1e-4, 1e-5
BF16_GRAD, BF16_LOSS = 1e-3, 1e-4


def flops_per_pair(d: int) -> int:
    """Algorithmic FP32 operations per unordered pair: 3d for the squared distance, 4d for
    the two gradient contributions, 31 for the pair function (square root, -log Phi and
    phi/Phi, glue arithmetic).  7d + 31, i.e. 45 at d = 2 and 143 at d = 16."""
    return 7 * d + 31


def traffic_path(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed PMC summary, or None
    when there is none or the kernel's sources changed since the counters were taken."""
    import hashlib

    path = traffic_path(workload)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel") != kernel or rec.get("workload") != workload:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return rec


TRAFFIC_SOURCES = ["paper_2011_03479_amd/csrc/sweep.hip", "paper_2011_03479_amd/csrc/sweep_mfma.hip",
                   "paper_2011_03479_amd/csrc/pairfn.h", "paper_2011_03479_amd/csrc/ltab_stage.h",
                   "paper_2011_03479_amd/csrc/ltab.h", "paper_2011_03479_amd/csrc/erfcx_coef.h",
                   "paper_2011_03479_amd/csrc/millsq_coef.h", "paper_2011_03479_amd/csrc/tiles.h",
                   "paper_2011_03479_amd/csrc/internal.h"]


# the BF16 screen's record hashes its own sources
SCREEN_SOURCES = ["paper_2011_03479_amd/csrc/gram.hip", "paper_2011_03479_amd/csrc/internal.h",
                  "paper_2011_03479_amd/csrc/ltab_stage.h", "paper_2011_03479_amd/csrc/pairfn.h",
                  "paper_2011_03479_amd/csrc/tiles.h"]


def sources_of(kernel: str):
    return SCREEN_SOURCES if "k_gram_screen" in kernel else TRAFFIC_SOURCES


def record_traffic(outdir: str, kernel: str, workload: str, copy_bytes: int):
    """Writes profiles/traffic_<workload>.json from four rocprofv3 --pmc runs under
    `outdir` (pmc_fetch, pmc_write: FETCH_SIZE / WRITE_SIZE of the bench; pmc_copy_fetch,
    pmc_copy_write: the same counters over the --copy-probe copy of `copy_bytes` bytes).
    Each counter is the median over the kernel's dispatches; the copy fixes the factor that
    turns it into bytes (the copy reads and writes copy_bytes)."""
    import csv
    import hashlib
    import statistics

    def median_kib(sub, name):
        path = os.path.join(outdir, sub, "run_counter_collection.csv")
        vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path)) if r["Kernel_Name"].removeprefix("void ").split("(")[0] == name]
        if not vals:
            raise SystemExit(f"no dispatch of {name} in {path}")
        return statistics.median(vals), len(vals)

    fetch, nk = median_kib("pmc_fetch", kernel)
    write, _ = median_kib("pmc_write", kernel)
    cfetch, _ = median_kib("pmc_copy_fetch", "__amd_rocclr_copyBuffer")
    cwrite, _ = median_kib("pmc_copy_write", "__amd_rocclr_copyBuffer")
    ff = copy_bytes / 1024.0 / cfetch
    wf = copy_bytes / 1024.0 / cwrite
    h = hashlib.sha256()
    for f in sources_of(kernel):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    rec = {"kernel": kernel, "workload": workload, "sources": sources_of(kernel),
           "source_sha256": h.hexdigest(), "dispatches": nk,
           "fetch_size_kib_per_launch": fetch, "write_size_kib_per_launch": write,
           "copy_probe_bytes": copy_bytes, "copy_fetch_size_kib": cfetch, "copy_write_size_kib": cwrite,
           "fetch_factor": ff, "write_factor": wf,
           "fetch_bytes_per_launch": fetch * 1024 * ff, "write_bytes_per_launch": write * 1024 * wf,
           "traffic_bytes_per_launch": fetch * 1024 * ff + write * 1024 * wf}
    out = traffic_path(workload)
    json.dump(rec, open(out, "w"), indent=1)
    print(json.dumps(rec))


def serving_bench(num_jobs: int, load: float, budget_gib: float, oracle_every: int):
    """The serving mix: Poisson stream of `num_jobs` embedding requests (n log-uniform in
    [500, 50000], ER or Chung-Lu with mean degree U[8, 30], d in {2, 16, 128}, 200
    iterations, BF16 Gram for d >= 64).  Pass 1 releases every job at once and measures the
    capacity (jobs/s); pass 2 replays the stream's arrival times scaled to load x capacity
    and reports throughput and the latency (arrival -> result on the host) percentiles."""
    import numpy as np

    from paper_2011_03479_amd import gempe, synth

    t0 = time.perf_counter()
    jobs = synth.serving_stream(num_jobs, 1.0)   # arrival times for rate 1 / s, rescaled below
    gen_s = time.perf_counter() - t0
    pairs = [j.graph.n * (j.graph.n - 1) // 2 * j.iters for j in jobs]
    budget = int(budget_gib * (1 << 30))

    def params(j):
        return gempe.params_default(precision=gempe.GEMPE_BF16_GRAM if j.precision == "bf16" else gempe.GEMPE_FP32)

    def run(release):
        with gempe.Server(budget, max_jobs=256) as srv:
            ids = [srv.submit(j.graph.n, j.graph.row_ptr, j.graph.col_idx, j.X0, j.iters, j.eta, params=params(j),
                              release_s=r) for j, r in zip(jobs, release)]
            srv.wait(-1)
            infos = [srv.query(i) for i in ids]
            st = srv.stats()
            res = [srv.result(i) for i in ids]
        return infos, st, res

    # warm-up: a few small jobs of each kind (module load, first launches)
    with gempe.Server(1 << 30) as srv:
        for d in (2, 16, 128):
            g = synth.erdos_renyi(600, 10.0, seed=d)
            srv.submit(g.n, g.row_ptr, g.col_idx, synth.init_embedding(g.n, d, seed=d), 20, 0.1 / 599,
                       params=gempe.params_default(precision=gempe.GEMPE_BF16_GRAM if d >= 64 else gempe.GEMPE_FP32))
        srv.wait(-1)

    infos, st1, _ = run([0.0] * num_jobs)
    assert all(i.state == gempe.GEMPE_JOB_DONE for i in infos), gempe.last_error()
    makespan = max(i.done_s for i in infos) - min(i.release_s for i in infos)
    capacity = num_jobs / makespan
    rate = load * capacity
    start = 0.05  # leave the submissions time to complete before the first arrival
    release = [start + j.arrival_s / rate for j in jobs]
    infos, st2, res = run(release)
    assert all(i.state == gempe.GEMPE_JOB_DONE for i in infos), gempe.last_error()
    lat = np.array([i.done_s - i.release_s for i in infos])
    span = max(i.done_s for i in infos) - min(i.release_s for i in infos)

    # per-class latency: batched (shared per-iteration launches) and solo jobs by precision
    def cls(j, info):
        return "batched" if info.batched else ("solo_bf16" if j.precision == "bf16" else "solo_fp32")
    classes = {}
    for j, info, l in zip(jobs, infos, lat):
        classes.setdefault(cls(j, info), []).append((l, j.graph.n, j.d, info.admit_s - info.release_s,
                                                     info.done_s - info.admit_s))

    def pct(v, i, q):
        return float(np.percentile([x[i] for x in v], q))
    # latency = wait for admission (release -> admit) + service on the device (admit -> done)
    per_class = {c: {"jobs": len(v), "p50_s": pct(v, 0, 50), "p99_s": pct(v, 0, 99),
                     "wait_p50_s": pct(v, 3, 50), "wait_p99_s": pct(v, 3, 99),
                     "service_p50_s": pct(v, 4, 50), "service_p99_s": pct(v, 4, 99),
                     "n_max": int(max(x[1] for x in v)), "d": sorted({x[2] for x in v})} for c, v in classes.items()}

    # every oracle_every-th job (10 %) against the FP64 oracle at the job's final X: the loss of
    # the run's history, per-vertex gradient and row loss on sampled rows (each against all n
    # vertices); the final X against the oracle's own trajectory where n is small enough, else
    # against the same job run alone on the GPU (same arithmetic, up to the order of FP32
    # atomic additions)
    import torch

    import oracle

    oracle.build(force=False)
    checks = []
    for k in range(0, num_jobs, oracle_every):
        j = jobs[k]
        X, hist = res[k]
        g = j.graph
        p = params(j)
        bf16 = j.precision == "bf16"
        G = gempe.Graph(g.n, g.row_ptr, g.col_idx)
        r = gempe.loss_grad(G, torch.as_tensor(X, device="cuda"), params=p, want_row_loss=True)
        torch.cuda.synchronize()
        rows = np.unique(np.random.default_rng(k).choice(g.n, min(g.n, 48), replace=False)).astype(np.int64)
        ref = oracle.rows(X.astype(np.float64), g.row_ptr, g.col_idx, rows, 1.5, 1.0)
        gg = r.grad.double().cpu().numpy()[rows]
        rl = r.row_loss.double().cpu().numpy()[rows]
        gerr = float(np.max(np.linalg.norm(gg - ref["grad"], axis=1) /
                            np.maximum(np.linalg.norm(ref["grad"], axis=1), 1e-2 * ref["abs_slope"])))
        rlerr = float(np.max(np.abs(rl - ref["row_loss"]) / np.abs(ref["row_loss"])))
        # the run's last history entry against the evaluation at its final X
        herr = abs(float(hist[-1]) - float(r.loss.item())) / abs(float(r.loss.item()))
        if g.n * (g.n - 1) / 2 * j.iters * max(j.d, 8) <= 2e10:  # a few seconds of host work
            _, X_ref = oracle.gd_trajectory(j.X0.astype(np.float64), g.row_ptr, g.col_idx, j.iters, j.eta)
            xkind = "oracle trajectory"
        else:
            Xa = torch.as_tensor(j.X0, device="cuda")
            gempe.embed(G, Xa, j.iters, j.eta, params=p)
            X_ref = Xa.double().cpu().numpy()
            xkind = "alone on the GPU"
        xerr = float(np.max(np.linalg.norm(X.astype(np.float64) - X_ref, axis=1)) /
                     np.max(np.linalg.norm(X_ref, axis=1)))
        G.close()
        checks.append({"job": k, "n": g.n, "d": j.d, "precision": j.precision, "grad_err_rel_bound": gerr,
                       "row_loss_err": rlerr, "hist_vs_final_eval": herr, "x_err": xerr, "x_against": xkind})
    gb, lb = (BF16_GRAD, BF16_LOSS), (FP32_GRAD, FP32_LOSS)
    ok = all(c["grad_err_rel_bound"] <= (gb if c["precision"] == "bf16" else lb)[0] and
             c["row_loss_err"] <= (gb if c["precision"] == "bf16" else lb)[1] and
             c["x_err"] <= (1e-3 if c["precision"] == "bf16" else 1e-4) for c in checks)
    return {
        "jobs": num_jobs,
        "iters_per_job": jobs[0].iters,
        "load": load,
        "capacity_jobs_per_s": capacity,
        "capacity_pairs_per_s": sum(pairs) / makespan,
        "rate_jobs_per_s": rate,
        "throughput_jobs_per_s": num_jobs / span,
        "throughput_pairs_per_s": sum(pairs) / span,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_max_s": float(lat.max()),
        "latency_per_class": per_class,
        "batched_jobs": int(sum(i.batched for i in infos)),
        "max_concurrent": int(st2["max_concurrent"]),
        "ticks": int(st2["ticks"]),
        "peak_bytes": int(st2["peak_bytes"]),
        "budget_bytes": int(st2["budget_bytes"]),
        "oracle_checked_jobs": len(checks),
        "oracle_checks_within_bounds": ok,
        "oracle_worst": {key: max(c[key] for c in checks) for key in
                         ("grad_err_rel_bound", "row_loss_err", "hist_vs_final_eval", "x_err")} if checks else None,
        "oracle_checks": checks,
        "generate_s": gen_s,
    }


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def gd_run(w, steps: int, warmup: int):
    """`steps` gradient-descent iterations of workload `w` from its X0 after `warmup`
    untimed ones, with the library's kernel timing on during the timed region.  Returns the
    HIP-event time of the whole region and the per-class kernel times."""
    import torch

    from paper_2011_03479_amd import gempe

    g = w.graph
    n, d = g.n, w.d
    stream = torch.cuda.current_stream()
    params = gempe.params_default(precision=gempe.GEMPE_BF16_GRAM if w.precision == "bf16" else gempe.GEMPE_FP32)
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    ws = gempe.workspace(G, d, params)
    X0 = torch.as_tensor(w.X0, device="cuda")
    X = X0.clone()
    if warmup > 0:
        # on the buffers of the timed run, as a training loop reuses its own
        gempe.embed(G, X, warmup, w.eta, ws=ws, params=params)
        X.copy_(X0)
    torch.cuda.synchronize()
    for c in range(5):  # drop anything recorded before the timed region
        gempe.timing_read(c)
    gempe.timing_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    gempe.embed(G, X, steps, w.eta, ws=ws, params=params)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gempe.timing_enable(False)
    ms = ev0.elapsed_time(ev1)
    kern = {}
    for c, name in ((gempe.GEMPE_TK_SWEEP, "sweep"), (gempe.GEMPE_TK_GRAM, "gram_screen"),
                    (gempe.GEMPE_TK_EXACT, "exact_near"), (gempe.GEMPE_TK_EDGES, "edges"),
                    (gempe.GEMPE_TK_FULL, "full_sweep")):
        nl, kms = gempe.timing_read(c)
        if nl:
            kern[name] = {"launches": nl, "ms_total": kms, "ms_per_launch": kms / nl}
    # the loss of the final iterate (one more evaluation, outside the timed region)
    out = gempe.LossGrad(torch.empty(1, dtype=torch.float64, device="cuda"), None, None, None)
    gempe.loss_grad(G, X, ws=ws, params=params, out=out)
    torch.cuda.synchronize()
    final_loss = float(out.loss.item())
    G.close()
    del ws, X, X0
    torch.cuda.empty_cache()
    N = n * (n - 1) // 2
    return {"ms": ms, "wall_s": wall, "kernels": kern, "final_loss_bits": final_loss,
            "value": N * steps / (ms / 1e3), "N": N}


def roofline_of(w, r, steps: int):
    """Roofline object of the dominant kernel: the FP32 sweep (7d + 31 flops per pair,
    against the FP32 peak) or, on the BF16 path, the Gram screen (2d MFMA flops per pair,
    against the BF16 peak) or, when it took longer, the full FP32 matrix-core sweep that
    evaluates every pair once more than half of the tiles are flagged (a launch that found
    fewer returns at once: it is taken as having run only when it also took at least the
    time every pair needs at the FP32 peak); its per-launch time from the HIP events
    bracketing its launches."""
    d, N = w.d, r["N"]
    if w.precision == "bf16":
        k = r["kernels"].get("gram_screen")
        fpp, peak, bound, name = 2 * d, PEAK_BF16_TFLOPS, "mfma", "k_gram_screen (BF16 MFMA Gram screen)"
        kf = r["kernels"].get("full_sweep")
        ran = kf and kf["ms_per_launch"] * 1e-3 >= flops_per_pair(d) * N / (PEAK_FP32_TFLOPS * 1e12)
        if ran and (not k or kf["ms_total"] > k["ms_total"]):
            kern = "k_sweep_mfma16<true>" if d == 16 else f"k_sweep_mfma_wide<{d}, true>"
            k, fpp, peak = kf, flops_per_pair(d), PEAK_FP32_TFLOPS
            name = f"{kern} (BF16 path, most tiles flagged: every pair in FP32 on the matrix cores)"
    else:
        k = r["kernels"].get("sweep")
        fpp, peak, bound = flops_per_pair(d), PEAK_FP32_TFLOPS, "alu"
        fused = w.graph.n <= 23000 and d <= 16
        name = "k_iter (fused iteration: sweep, edge pass, update)" if fused else "k_sweep_small / k_sweep_wide"
        if (d == 16 and w.graph.n >= 8192 and not fused) or (d in (32, 64, 128) and w.graph.n >= 4096):
            # the squared distance and both gradient sides on FP32 MFMA (6d flops per pair),
            # the pair function on the vector ALUs; FP32 matrix and vector peaks are the same
            kern = "k_sweep_mfma16<false>" if d == 16 else f"k_sweep_mfma_wide<{d}, false>"
            name, bound = f"{kern} (FP32 MFMA Gram and gradient products, VALU pair function)", "mfma"
    if not k:
        return None
    kms = k["ms_per_launch"]
    achieved = fpp * N / (kms / 1e3) / 1e12
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": None, "kernel": name, "kernel_ms": kms, "kernel_launches": k["launches"],
            "flops_per_pair": fpp, "timing": "HIP events around the kernel's launches on its stream"}


def attach_traffic(roof, kernel: str, workload: str):
    tr = measured_traffic(kernel, workload)
    if roof is None or tr is None:
        return
    roof["traffic"] = tr["traffic_bytes_per_launch"]
    roof["traffic_detail"] = {
        "unit": "bytes per launch", "kernel": kernel, "fetch": tr["fetch_bytes_per_launch"],
        "write": tr["write_bytes_per_launch"], "fetch_factor": tr["fetch_factor"], "write_factor": tr["write_factor"],
        "source": f"profiles/traffic_{workload}.json (rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-calibrated)"}


def traffic_kernel_of(w):
    """The symbol of the workload's dominant kernel, as rocprofv3 names it (the key of its
    traffic record), or None.  On the BF16 path that is the screen (rocprofv3 reports its
    name mangled), whose record is attached only while the screen is the roofline's kernel."""
    d, n = w.d, w.graph.n
    if w.precision == "bf16":
        rw = 8 if (n + 511) // 512 >= 64 else 2
        return f"_ZN5gempe13k_gram_screenILi{d}ELi{rw}EEEvPKDF16bPKfS4_iiixfPhiiPKiPi"
    if n <= 23000 and d <= 16:
        return f"gempe::k_iter<{d if d <= 4 else (8 if d <= 8 else 16)}>"
    if d == 16 and n >= 8192:
        return "gempe::k_sweep_mfma16<false>"
    if d in (32, 64, 128) and n >= 4096:
        return f"gempe::k_sweep_mfma_wide<{d}, false>"
    return None


def summary(w, r, steps: int, warmup: int):
    roof = roofline_of(w, r, steps)
    kern = traffic_kernel_of(w)
    if kern is not None and roof is not None and ("k_gram_screen" in kern) == roof["kernel"].startswith("k_gram_screen"):
        attach_traffic(roof, kern, w.name)
    d = {"workload": w.name, "n": w.graph.n, "m": w.graph.m, "d": w.d, "precision": w.precision,
         "steps": steps, "warmup": warmup, "pairs_per_iter": r["N"], "value": r["value"], "unit": "pairs/s",
         "ms_per_step": r["ms"] / steps, "kernels": r["kernels"], "final_loss_bits": r["final_loss_bits"],
         "roofline": roof}
    return d


def cpu_baseline(w, seconds: float):
    """The FP64 oracle on the host on whole rows of the workload: each sampled row i is
    evaluated against all n vertices (its loss and gradient), in batches of 500 seeded
    random rows until `seconds` have passed.  A row does n - 1 ordered pair evaluations,
    half of the work the full oracle spends per unordered pair, so the unordered-pair rate
    is rows (n - 1) / 2 / time; one full iteration is extrapolated from it."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    g = w.graph
    n = g.n
    X = w.X0.astype(np.float64)
    rng = np.random.default_rng(7)
    rows = 0
    t0 = time.perf_counter()
    while True:
        idx = np.sort(rng.choice(n, size=min(500, n), replace=False)).astype(np.int64)
        oracle.rows(X, g.row_ptr, g.col_idx, idx, w.mu, w.sigma)
        rows += idx.size
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    rate = rows * (n - 1) / 2.0 / el
    N = n * (n - 1) // 2
    return {"value": rate, "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"{rows} random rows of {w.name} at X0, each against all {n} vertices (loss and gradient "
                      f"of the row; FP64 brute force, OpenMP over rows), {el:.1f} s; counted as rows (n-1)/2 "
                      f"unordered pairs",
            "extrapolated_s_per_iter": N / rate}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cl1m")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-mix pass")
    ap.add_argument("--no-extras", action="store_true", help="skip the BF16 variant and the other workloads")
    ap.add_argument("--variant-steps", type=int, default=5, help="timed iterations of the BF16 variant")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes 20 times (the reference "
                         "kernel that calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--record-traffic", default=None, metavar="DIR",
                    help="only write profiles/traffic_<workload>.json from the rocprofv3 --pmc runs under "
                         "DIR (no GPU needed); --traffic-kernel names the kernel")
    ap.add_argument("--traffic-kernel", default="gempe::k_sweep_mfma16<false>")
    ap.add_argument("--serve-jobs", type=int, default=200)
    ap.add_argument("--serve-load", type=float, default=0.8)
    ap.add_argument("--serve-budget-gib", type=float, default=32.0)
    args = ap.parse_args()
    if args.record_traffic:
        record_traffic(args.record_traffic, args.traffic_kernel, args.workload, 268435456)
        return
    if args.copy_probe:
        import torch

        torch.cuda.set_device(0)
        src = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(20):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "launches": 20}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1 (the sweep's "
                                   "sharding over several GPUs, gempe_loss_grad_shard, is measured per "
                                   "device, not as a multi-GPU run)"}))
        sys.exit(2)

    import torch

    from paper_2011_03479_amd import synth

    torch.cuda.set_device(0)
    t_gen = time.perf_counter()
    w = synth.workload(args.workload)
    gen_s = time.perf_counter() - t_gen
    steps = args.steps if args.steps is not None else w.iters
    print(f"# {w.name}: n={w.graph.n} m={w.graph.m} d={w.d} generated in {gen_s:.1f} s; "
          f"{args.warmup} + {steps} iterations", file=sys.stderr, flush=True)
    r = gd_run(w, steps, args.warmup)
    main_sum = summary(w, r, steps, args.warmup)
    roof = main_sum["roofline"]
    result = {
        "metric": "vertex-pairs/s per full-gradient iteration (FP32; BF16-MFMA Gram variant under variants)",
        "value": r["value"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"] / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.precision == "fp32" else "bf16+f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.graph.n, "m": w.graph.m, "d": w.d, "iters": steps,
                   "pairs_per_iter": r["N"], "eta": w.eta, "mu": w.mu, "sigma": w.sigma,
                   "precision": w.precision, "graph": "Chung-Lu power law, mean degree 20, exponent 2.3"
                   if w.name.startswith("cl1m") else w.name},
        "roofline": roof,
        "kernels": r["kernels"],
        "wall_s": r["wall_s"],
        "final_loss_bits": r["final_loss_bits"],
    }
    print(f"# {w.name}: {r['ms'] / steps:.3f} ms/iteration, {r['value']:.4g} pairs/s", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        print(f"# cpu baseline: {result['cpu_baseline']['value']:.4g} pairs/s", file=sys.stderr, flush=True)
    if not args.no_extras:
        if w.name == "cl1m":
            wb = synth.Workload("cl1m_bf16", w.graph, w.d, w.X0, w.iters, w.eta, "bf16")
            rb = gd_run(wb, args.variant_steps, 1)
            result["variants"] = {"cl1m_bf16": summary(wb, rb, args.variant_steps, 1)}
            print(f"# cl1m_bf16: {rb['ms'] / args.variant_steps:.3f} ms/iteration", file=sys.stderr, flush=True)
        del w
        result["extras"] = {}
        for name, st, wu in (("cl3400", 1000, 20), ("sbm100k", 20, 2), ("sbm100k_fp32", 3, 1)):
            we = synth.workload(name)
            re_ = gd_run(we, st, wu)
            result["extras"][name] = summary(we, re_, st, wu)
            print(f"# {name}: {re_['ms'] / st:.4f} ms/iteration", file=sys.stderr, flush=True)
    if not args.no_serve:
        result["serving"] = serving_bench(args.serve_jobs, args.serve_load, args.serve_budget_gib, 10)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
