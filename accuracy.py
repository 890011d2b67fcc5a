#!/usr/bin/env python3
"""Accuracy experiments of Sec. VI on the GPU estimator (Superfast LSE only;
the comparison algorithms are not part of this library).

  snr       Fig. snr: N = M = 128, K = 10, separation 2/N, alpha = a + 0.2 e^{j arg a}
            (a ~ CN, std 0.8), SNR -5 .. 30 dB; block success rate, component
            success rate, NMSE, and the NMSE of least squares with the true
            frequencies (Oracle).
  pairsep   Fig. pairsep: N = 128, 5 pairs (K = 10) with intra-pair separation
            0.2/N .. 1.75/N, pairs at least 2/N apart, SNR 20 dB.
  phasetran Fig. phasetran: block success rate over pair separation x K/N (pairs
            as in pairsep, as many as give K/N closest to the target), N = 128,
            SNR 20 dB.
  mton      Fig. MtoN: incomplete data, M/N = 0.2 .. 1 rows of the identity
            (first and last sample kept), N = 128, K = 10, 20 dB, by
            sfls_estimate_incomplete (the semifast method of Sec. IV).

Every trial of a figure is one instance of a single sfls_estimate batch.  The
metrics (Sec. VI-A): a block success is the right model order with every
matched frequency within 0.5/N; the component success rate counts estimates
and true components with a partner within 0.5/N; NMSE = ||h_est - h||^2 / ||h||^2
averaged over trials.

    python accuracy.py --figure snr --trials 500 [--precision fp64|mixed]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SNRS = (-5.0, 0.0, 3.0, 6.0, 9.0, 12.0, 15.0, 20.0, 25.0, 30.0)
SEPS = (0.2, 0.4, 0.55, 0.7, 0.85, 1.0, 1.25, 1.5, 1.75)
MTON = (0.2, 0.3, 0.4, 0.5, 0.6, 0.8, 1.0)
RATIOS = (0.05, 0.1, 0.15, 0.2, 0.25, 0.3)


def summarise(insts, results, N):
    import numpy as np
    from tests import metrics
    bs = [metrics.block_success(i.theta, r.theta, N) for i, r in zip(insts, results)]
    cs = [metrics.component_success_rate(i.theta, r.theta, N) for i, r in zip(insts, results)]
    ns = [metrics.nmse(i.theta, i.alpha, r.theta, r.alpha, N) for i, r in zip(insts, results)]
    ls = [metrics.oracle_ls_nmse(i) for i in insts]
    return {"trials": len(insts), "bsr": float(np.mean(bs)), "csr": float(np.mean(cs)),
            "nmse_db": 10 * math.log10(float(np.mean(ns))),
            "oracle_ls_nmse_db": 10 * math.log10(float(np.mean(ls))),
            "K_mean": float(np.mean([r.K for r in results])),
            "status_ok": int(sum(r.status == 0 for r in results))}


def run(ctx, points, make, params):
    """One batch over every (point, trial); returns {point: summary}."""
    import paper_1705_06073_amd as sf
    insts = [make(p, t) for p, t in points]
    t0 = time.perf_counter()
    if insts and insts[0].idx is not None:
        res = sf.estimate_batch_incomplete(ctx, [(i.N, i.idx, i.phi, i.y) for i in insts], params)
    else:
        res = sf.estimate_batch(ctx, [i.y for i in insts], params)
    dt = time.perf_counter() - t0
    out = {}
    keys = sorted({p for p, _ in points})
    for k in keys:
        idx = [j for j, (p, _) in enumerate(points) if p == k]
        out[k] = summarise([insts[j] for j in idx], [res[j] for j in idx], insts[idx[0]].N)
    return out, dt, len(insts)


def figure_snr(ctx, trials, params, snrs=SNRS):
    from paper_1705_06073_amd import synth
    pts = [(s, t) for s in snrs for t in range(trials)]
    return run(ctx, pts, lambda s, t: synth.workload_paper_snr(t, s), params)


def figure_pairsep(ctx, trials, params, seps=SEPS):
    from paper_1705_06073_amd import synth
    pts = [(s, t) for s in seps for t in range(trials)]
    return run(ctx, pts, lambda s, t: synth.workload_paper_pairs(t, s), params)


def figure_mton(ctx, trials, params, ratios=MTON):
    from paper_1705_06073_amd import synth
    pts = [(r, t) for r in ratios for t in range(trials)]
    return run(ctx, pts, lambda r, t: synth.workload_paper_mton(t, r), params)


def figure_phasetran(ctx, trials, params, seps=SEPS, ratios=RATIOS, N=128):
    from paper_1705_06073_amd import synth
    pts = [((s, r), t) for s in seps for r in ratios for t in range(trials)]

    def make(p, t):
        s, r = p
        npairs = max(1, int(round(r * N / 2)))
        return synth.workload_paper_pairs(t + 100000 * int(round(r * 100)), s, N=N, npairs=npairs)
    return run(ctx, pts, make, params)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--figure", choices=["snr", "pairsep", "phasetran", "mton"], default="snr")
    ap.add_argument("--trials", type=int, default=500)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--param", action="append", default=[],
                    help="estimator parameter override name=value (sfls_params field)")
    a = ap.parse_args()
    import paper_1705_06073_amd as sf
    ctx = sf.Context(0)
    over = {}
    for kv in a.param:
        k, v = kv.split("=", 1)
        over[k] = float(v) if "." in v or "e" in v else int(v)
    params = sf.default_params(precision=sf.SFLS_MIXED if a.precision == "mixed" else sf.SFLS_FP64,
                               **over)
    fn = {"snr": figure_snr, "pairsep": figure_pairsep, "phasetran": figure_phasetran,
          "mton": figure_mton}[a.figure]
    out, dt, count = fn(ctx, a.trials, params)
    ctx.close()
    print(json.dumps({"figure": a.figure, "trials": a.trials, "precision": a.precision,
                      "params": over,
                      "instances": count, "gpu_seconds": dt,
                      "points": {str(k): v for k, v in out.items()}}), flush=True)


if __name__ == "__main__":
    main()
