"""Benchmark: all-pairs GEMPE gradient iterations on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cl3400]

A step is one full iteration of the hot path: the all-pairs FP32 sweep (loss and gradient
of every unordered vertex pair), the exact edge correction, the FP64 loss reduction and
the update X <- X - eta G.  The default workload is the drawing-sized Chung-Lu graph
(n = 3,400, about 19,000 edges, degree exponent 2.5, d = 2, 1,000 iterations).  Prints
one JSON line with pairs/s (unordered pairs x iterations / time), the roofline figures of
the dominant kernel and the FP64 CPU oracle timed on the host on a bounded sample.
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


def flops_per_pair(d: int) -> int:
    """Algorithmic FP32 operations per unordered pair: 3d for the squared distance, 4d for
    the two gradient contributions, 31 for the pair function (square root, -log Phi and
    phi/Phi, glue arithmetic).  7d + 31, i.e. 45 at d = 2 and 143 at d = 16."""
    return 7 * d + 31


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed PMC summary, or None
    when there is none or the kernel's sources changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_iter_cl3400_traffic.json")
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


TRAFFIC_SOURCES = ["paper_2011_03479_amd/csrc/sweep.hip", "paper_2011_03479_amd/csrc/pairfn.h",
                   "paper_2011_03479_amd/csrc/ltab.h", "paper_2011_03479_amd/csrc/erfcx_coef.h",
                   "paper_2011_03479_amd/csrc/millsq_coef.h", "paper_2011_03479_amd/csrc/tiles.h",
                   "paper_2011_03479_amd/csrc/internal.h"]


def record_traffic(outdir: str, kernel: str, workload: str, copy_bytes: int):
    """Writes profiles/k_iter_cl3400_traffic.json from four rocprofv3 --pmc runs under
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
    for f in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    rec = {"kernel": kernel, "workload": workload, "sources": TRAFFIC_SOURCES,
           "source_sha256": h.hexdigest(), "dispatches": nk,
           "fetch_size_kib_per_launch": fetch, "write_size_kib_per_launch": write,
           "copy_probe_bytes": copy_bytes, "copy_fetch_size_kib": cfetch, "copy_write_size_kib": cwrite,
           "fetch_factor": ff, "write_factor": wf,
           "fetch_bytes_per_launch": fetch * 1024 * ff, "write_bytes_per_launch": write * 1024 * wf,
           "traffic_bytes_per_launch": fetch * 1024 * ff + write * 1024 * wf}
    out = os.path.join(ROOT, "profiles", "k_iter_cl3400_traffic.json")
    json.dump(rec, open(out, "w"), indent=1)
    print(json.dumps(rec))


def serving_bench(num_jobs: int, load: float, budget_gib: float, oracle_every: int, oracle_max_n: int):
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

    # error against the FP64 oracle on sampled jobs: DL at each sampled job's final X
    import oracle

    oracle.build(force=False)
    errs = []
    sampled = [k for k in range(0, num_jobs, oracle_every) if jobs[k].graph.n <= oracle_max_n]
    for k in sampled:
        j = jobs[k]
        X, hist = res[k]
        ref = oracle.loss_grad(X.astype(np.float64), j.graph.row_ptr, j.graph.col_idx, 1.5, 1.0, want_grad=False)
        errs.append((j.precision, abs(float(hist[-1]) - ref["loss"]) / abs(ref["loss"])))
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
        "batched_jobs": int(sum(i.batched for i in infos)),
        "max_concurrent": int(st2["max_concurrent"]),
        "ticks": int(st2["ticks"]),
        "peak_bytes": int(st2["peak_bytes"]),
        "budget_bytes": int(st2["budget_bytes"]),
        "oracle_sampled_jobs": len(sampled),
        "oracle_max_rel_loss_err_fp32": max([e for p, e in errs if p == "fp32"], default=None),
        "oracle_max_rel_loss_err_bf16": max([e for p, e in errs if p == "bf16"], default=None),
        "generate_s": gen_s,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cl3400")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-mix pass")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes 20 times (the reference "
                         "kernel that calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--record-traffic", default=None, metavar="DIR",
                    help="only write the k_iter traffic record from the rocprofv3 --pmc runs under DIR "
                         "(no GPU needed)")
    ap.add_argument("--serve-jobs", type=int, default=200)
    ap.add_argument("--serve-load", type=float, default=0.8)
    ap.add_argument("--serve-budget-gib", type=float, default=32.0)
    args = ap.parse_args()
    if args.record_traffic:
        record_traffic(args.record_traffic, "gempe::k_iter<2>", "cl3400", 268435456)
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
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(the multi-GPU sharding is described in DESIGN.md, not built)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2011_03479_amd import gempe, synth

    w = synth.workload(args.workload)
    steps = args.steps if args.steps is not None else w.iters
    g = w.graph
    n, d = g.n, w.d
    N = n * (n - 1) // 2
    torch.cuda.set_device(0)
    G = gempe.Graph(n, g.row_ptr, g.col_idx)
    params = gempe.params_default(precision=gempe.GEMPE_BF16_GRAM if w.precision == "bf16" else gempe.GEMPE_FP32)
    ws = gempe.workspace(G, d, params)
    X0 = torch.as_tensor(w.X0, device="cuda")
    stream = torch.cuda.current_stream()

    # warm-up
    X = X0.clone()
    if args.warmup > 0:
        gempe.embed(G, X, args.warmup, w.eta, ws=ws, params=params)
    torch.cuda.synchronize()

    # timed region: exactly `steps` iterations from X0
    X = X0.clone()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    gempe.embed(G, X, steps, w.eta, ws=ws, params=params)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    value = N * steps / (ms / 1e3)

    # Dominant kernel.  Small n: the fused iteration kernel (one launch per step, so the
    # timed region above is `steps` back-to-back launches of it plus two tiny kernels);
    # large n: the sweep launched inside each step.  Its average duration is bounded by the
    # per-step time measured with HIP events on the stream the kernels run on.
    k_ms = ms / steps
    if w.precision == "bf16":
        # MFMA-bound screen: 2d BF16 MFMA flops per pair for the Gram term
        fpp, peak, bound = 2 * d, PEAK_BF16_TFLOPS, "mfma"
        plan_kernel = "k_gram_screen (BF16 MFMA Gram screen; kernel_ms is the whole step, an upper bound)"
    else:
        fpp, peak, bound = flops_per_pair(d), PEAK_FP32_TFLOPS, "alu"
        plan_kernel = "k_iter (fused iteration: all-pairs sweep, exact edge pass, update)" if n <= 23000 and d <= 16 \
            else "k_sweep_small / k_sweep_wide (per step, with the edge pass and update)"
    achieved = fpp * N / (k_ms / 1e3) / 1e12

    result = {
        "metric": "vertex-pairs/s per full-gradient iteration",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.precision == "fp32" else "bf16+f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "m": g.m, "d": d, "iters": steps,
                   "pairs_per_iter": N, "eta": w.eta, "mu": w.mu, "sigma": w.sigma,
                   "precision": w.precision},
        "roofline": {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": plan_kernel, "kernel_ms": k_ms, "flops_per_pair": fpp},
        "wall_s": wall,
        "final_loss_bits": None,
    }
    tr = measured_traffic("gempe::k_iter<2>", w.name) if plan_kernel.startswith("k_iter") and d == 2 else None
    if tr is not None:
        result["roofline"]["traffic"] = tr["traffic_bytes_per_launch"]
        result["roofline"]["traffic_detail"] = {
            "unit": "bytes per launch", "fetch": tr["fetch_bytes_per_launch"], "write": tr["write_bytes_per_launch"],
            "fetch_factor": tr["fetch_factor"], "write_factor": tr["write_factor"],
            "source": "profiles/k_iter_cl3400_traffic.json (rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-calibrated)"}
    hist = torch.empty(1, dtype=torch.float64, device="cuda")
    gempe.loss_grad(G, X, ws=ws, params=params, out=gempe.LossGrad(hist, None, None, None))
    torch.cuda.synchronize()
    result["final_loss_bits"] = float(hist.item())

    if not args.no_cpu_baseline:
        import oracle

        oracle.build(force=False)
        Xc = w.X0.astype(np.float64)
        t0 = time.perf_counter()
        its = 0
        while True:
            oracle.loss_grad(Xc, g.row_ptr, g.col_idx, w.mu, w.sigma)
            its += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        result["cpu_baseline"] = {
            "value": N * its / el, "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{its} full loss+gradient evaluations of {w.name} at X0 (FP64 brute force over all "
                      f"ordered pairs, OpenMP over rows), {el:.1f} s",
        }
    if not args.no_serve:
        result["serving"] = serving_bench(args.serve_jobs, args.serve_load, args.serve_budget_gib, 10, 6000)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
