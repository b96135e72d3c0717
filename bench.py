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

PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 vector (AMD published)


def flops_per_pair(d: int) -> int:
    """Algorithmic FP32 operations per unordered pair ("Roofline").

    distance sum_k (x_ik - x_jk)^2: 3d - 1; delta = sqrt: 1; tau = (delta - mu)/sigma: 2;
    dl and dl' from Phi: erfc, exp, log and one division + 4 arithmetic: 8; coefficient
    dl'/delta and its sign/scale: 2; gradient cc (x_i - x_j), row add, column add: 3d;
    loss accumulation: 1.  Total 6d + 13.
    """
    return 6 * d + 13


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cl3400")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
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

    # dominant kernel: one loss/gradient evaluation (sweep + edge pass + reduction),
    # timed with HIP events on the stream it is launched on
    reps = max(10, min(200, int(0.5e3 / max(ms / steps, 1e-3))))
    out = gempe.loss_grad(G, X0, ws=ws, params=params)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        gempe.loss_grad(G, X0, ws=ws, params=params, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    k_ms = e0.elapsed_time(e1) / reps
    fl = flops_per_pair(d) * N
    achieved = fl / (k_ms / 1e3) / 1e12

    result = {
        "metric": "vertex-pairs/s per full-gradient iteration (FP32, all pairs)",
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
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "loss_grad (sweep + edge pass + FP64 reduction)",
                     "kernel_ms": k_ms, "flops_per_pair": flops_per_pair(d)},
        "wall_s": wall,
        "final_loss_bits": None,
    }
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
    print(json.dumps(result))


if __name__ == "__main__":
    main()
