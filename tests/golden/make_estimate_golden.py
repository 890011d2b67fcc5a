"""Write the oracle's whole estimates for sampled instances of the batched
workloads into ``estimates_oracle.json`` (the expected values of
``tests/test_gpu_estimate_golden.py``).

Calls only ``oracle/`` (the dense FP64 estimator with its default parameters)
on inputs from ``paper_1705_06073_amd.synth`` (seeded generators, no method
arithmetic).  Cases:

  * the 256 x N=4096 batch (K ~ Poisson(40), separation 1/N, alpha ~ CN(0,1),
    SNR ~ U[0,30] dB, grid 8N): instances 0, 77, 191, 255;
  * the uneven batch (N log-uniform on [128, 16384], K ~ Poisson(N/64),
    SNR ~ U[5,30] dB, grid 2^round(log2 8N)): instances 2, 8, 19, 29
    (N = 1255, 3704, 2699, 5757; the dense oracle is affordable up to a few
    thousand samples).

With --incomplete, the incomplete-data oracle (oracle/incomplete.py) on the
runtime experiment's incomplete workload (N = 4096, M = 3072 rows of the
identity, K = 15, separation 2/N, the paper's alpha, 20 dB): instances 0..3,
into ``estimates_incomplete_oracle.json`` (the expected values of
``tests/test_gpu_incomplete_golden.py``).

Beside K, theta, alpha, gamma, beta, zeta and the objective, each case keeps
the smallest decision margins the oracle met (relative distance between the
two sides of a comparison that took a discrete decision), the input to the
ambiguity rule of the parity test.

    python tests/golden/make_estimate_golden.py [--jobs 4] [--incomplete]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "estimates_oracle.json")
OUT_INCOMPLETE = os.path.join(HERE, "estimates_incomplete_oracle.json")

Z_SITES = ("criterion", "gamma_hat", "delta_L", "ratio", "distance", "deactivate", "terminate")

CASES = [("n4096", i) for i in (0, 77, 191, 255)] + [("uneven", i) for i in (2, 8, 19, 29)]
CASES_INCOMPLETE = [("incomplete_n4096", i) for i in range(4)]


def _instance(kind, i):
    from paper_1705_06073_amd import synth
    if kind == "incomplete_n4096":
        return synth.workload_incomplete_n4096(i)
    return synth.workload_n4096(i) if kind == "n4096" else synth.workload_uneven(i)


def _z_changes(trace):
    """Outer iterations in which the active set changed (activation or deactivation)."""
    its, it = [], 1
    for rec in trace:
        if rec[0] == "iter":
            it = rec[1] + 1
        elif (rec[0] == "exact" and rec[3]) or (rec[0] == "approx" and rec[3] > 0) \
                or rec[0] == "deact":
            its.append(rec[1] if rec[0] == "deact" else it)
    return its


def solve(case):
    kind, i = case
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    from threadpoolctl import threadpool_limits

    from oracle import incomplete
    from oracle.estimator import Params, estimate
    inst = _instance(kind, i)
    with threadpool_limits(int(os.environ.get("SFLS_GOLDEN_THREADS", "2"))):
        t0 = time.perf_counter()
        if inst.idx is None:
            r = estimate(inst.y, Params())
        else:
            r = incomplete.estimate(inst.y.astype("complex128"), inst.idx, inst.N, inst.phi,
                                    Params())
        dt = time.perf_counter() - t0
    zc = _z_changes(r.trace)
    last_z = int(max(zc)) if zc else 0

    def top(sel, k=6):
        ms = sorted((m for m in r.margins if sel(m)), key=lambda m: m[3])[:k]
        return [[m[0], m[1], int(m[2]), float(m[3])] for m in ms]

    return {
        "workload": kind, "instance": i, "N": inst.N, "M": inst.M, "K_true": inst.K,
        "K": r.K, "theta": [float(x) for x in r.theta],
        "alpha_re": [float(x) for x in r.alpha.real], "alpha_im": [float(x) for x in r.alpha.imag],
        "gamma": [float(x) for x in r.gamma], "beta": float(r.beta), "zeta": float(r.zeta),
        "objective": float(r.objective), "iterations": int(r.iterations),
        "evaluations": int(r.evaluations), "status": int(r.status),
        "last_z_change_iteration": last_z,
        # decisions that choose the active set or end the outer loop
        "margins_z": top(lambda m: m[0] == "fp64" and m[1] in Z_SITES),
        # rankings of grid points (argmin, local minima), taken in the grid's precision
        "margins_grid": top(lambda m: m[0] == "grid"),
        # decisions of the continuous path up to the last change of the active set
        "margins_path": top(lambda m: m[0] == "fp64" and m[1] not in Z_SITES and m[2] <= last_z),
        "oracle_seconds": round(dt, 1),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--incomplete", action="store_true")
    a = ap.parse_args()
    with ProcessPoolExecutor(a.jobs) as ex:
        res = list(ex.map(solve, CASES_INCOMPLETE if a.incomplete else CASES))
    for r in res:
        print(f"{r['workload']}[{r['instance']}] N={r['N']} K={r['K']} (true {r['K_true']}) "
              f"evals={r['evaluations']} {r['oracle_seconds']} s", flush=True)
    if a.incomplete:
        doc = {"source": "oracle.incomplete.estimate (dense FP64, default Params) on "
                         "paper_1705_06073_amd.synth.workload_incomplete_n4096",
               "cases": res}
    else:
        doc = {"source": "oracle.estimator.estimate (dense FP64, default Params) on "
                         "paper_1705_06073_amd.synth.workload_n4096 / workload_uneven",
               "cases": res}
    out = OUT_INCOMPLETE if a.incomplete else OUT
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {out}")


if __name__ == "__main__":
    main()
