"""Writes full_loss.json: the FP64 oracle's coding cost DL (Eq. 2 at mu = 1.5, sigma = 1,
summed over every unordered pair) of the full-size SBM workload (n = 100,000 in 50 blocks
of 2,000, p_in = 2e-3, p_out = 2e-5, d = 128) at two seeded starting points: X0 ~ N(0, 1)
and the contracted X0 ~ N(0, (mu / sqrt(2d))^2) where nearly every pair is near.  Each is
about 5e9 pair evaluations (several minutes on a few host cores), too long to run inside a
GPU test, so the values are stored.  Calls only the oracle and the seeded input
generators; a fingerprint of each input lets the tests detect a changed generator.

    python tests/golden/gen_full_loss.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2011_03479_amd import synth  # noqa: E402


def fingerprint(w) -> str:
    h = hashlib.sha256()
    for a in (w.graph.row_ptr, w.graph.col_idx, w.X0):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    oracle.build(force=False)
    out = {}
    for name in ("sbm100k", "sbm100k_t9"):
        w = synth.workload(name)
        t0 = time.perf_counter()
        r = oracle.loss_grad(w.X0.astype(np.float64), w.graph.row_ptr, w.graph.col_idx, w.mu, w.sigma,
                             want_grad=False)
        el = time.perf_counter() - t0
        out[name] = {"n": w.graph.n, "m": w.graph.m, "d": w.d, "mu": w.mu, "sigma": w.sigma,
                     "fingerprint": fingerprint(w), "loss_bits": r["loss"], "edge_hits": r["edge_hits"],
                     "oracle_seconds": el, "oracle_threads": oracle.num_threads()}
        print(name, out[name], flush=True)
    json.dump(out, open(os.path.join(HERE, "full_loss.json"), "w"), indent=1)


if __name__ == "__main__":
    main()
