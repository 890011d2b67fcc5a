#!/usr/bin/env python3
"""Throughput benchmark: estimation solves/sec at N=4096 on one MI355X.

A step is one batch of 256 full solves (every evaluation: covariance column,
superfast factorisation, grid stage, active-set vectors and the device-side
driver) of synthetic signals with N=4096, K~Poisson(40), minimum separation
1/N, alpha~CN(0,1), SNR~U[0,30] dB, grid L=8N=32768, FP64 recursion and FP32
grid FFTs.  Inputs are resident in HBM before timing starts.

`value`: batched throughput, each step one sfls_estimate call that solves its
batch of 256 to completion (so a step lasts as long as its slowest instance);
latency is each solve's completion within its batch.  Also reported: the same
batches streamed through a 256-slot server (continuous batching: a slot freed
by a finished solve takes the next instance at the following round), the plain
FP64 method launched one instance at a time over the 256 instances, the
roofline position of the dominant kernel (from HIP events the library records
on its stream) with its HBM reading and counter traffic, per-kernel HBM and
FP64 fractions, the idle share of a round, and the CPU oracle timed on a
bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
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

METRIC = "estimation solves/sec at N=4096 (batched vs plain FP64); p50/p99 latency"
FP64_PEAK = 78.6e12   # MI355X dense FP64 vector, FLOP/s
HBM_PEAK = 8.0e12     # B/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(B):
    import numpy as np
    from paper_1705_06073_amd import synth
    insts = [synth.workload_n4096(i) for i in range(B)]
    return insts, np


def cpu_baseline(insts, per_solve_active, per_solve_grid, L_mult=8.0):
    """Time the oracle on a bounded sample of the workload: one evaluation with
    the grid stage and two without, at the first instance's true state, then
    scale by the evaluations a solve takes (counted on the GPU run)."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import numerics as nm
    from oracle.estimator import OracleEstimator, Params

    inst = insts[0]
    th, ga, be = inst.theta, np.abs(inst.alpha) ** 2, inst.beta
    est = OracleEstimator(inst.y, Params(L_mult=L_mult))
    t0 = time.perf_counter()
    ev = nm.Evaluation(inst.y, th, ga, be)
    est._exact_activation_round(ev, th, ga, min(0.5, len(th) / inst.N))  # grid stage
    t_grid = time.perf_counter() - t0
    t1 = time.perf_counter()
    for _ in range(2):
        nm.Evaluation(inst.y, th, ga, be)
    t_active = (time.perf_counter() - t1) / 2
    t_solve = per_solve_grid * t_grid + per_solve_active * t_active
    info = threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] or [1])
    blas = sorted({f"{i.get('internal_api')} {i.get('version')}" for i in info
                   if i.get("user_api") == "blas"})
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        nproc = os.cpu_count()
    return {
        "value": 1.0 / t_solve,
        "unit": "solves/s",
        "cores": int(threads),
        "host": {"nproc": nproc, "cpu_model": model, "blas": blas},
        "kind": "oracle",
        "sample": (f"dense FP64 oracle on instance 0 (N={inst.N}, K={inst.K}): one grid "
                   f"evaluation {t_grid:.2f} s, active evaluations {t_active:.2f} s each; "
                   f"per solve {per_solve_grid:.1f} grid + {per_solve_active:.1f} active "
                   f"evaluations (mean over the GPU batch) -> {t_solve:.1f} s/solve"),
    }


SERVE_CLASSES = ((1024, 512), (4096, 256), (16384, 256), (65536, 256))
SERVE_HBM = (2 << 30, 4 << 30, 8 << 30, 32 << 30)
SERVE_POOL = {256: 64, 1024: 64, 4096: 32, 16384: 16, 65536: 8}


def cpu_full_solves(insts, count, L_mult=8.0):
    """Whole oracle solves of the first `count` instances (minutes each at
    N=4096): per-solve median and the times, for the record beside the bounded
    sample of cpu_baseline."""
    import numpy as np
    from oracle.estimator import Params, estimate

    times, evals = [], []
    for inst in insts[:count]:
        t0 = time.perf_counter()
        r = estimate(inst.y, Params(L_mult=L_mult))
        times.append(time.perf_counter() - t0)
        evals.append(r.evaluations)
        log(f"oracle solve: N={inst.N} K={r.K} evaluations={r.evaluations} {times[-1]:.1f} s")
    med = float(np.median(times))
    return {"value": 1.0 / med, "unit": "solves/s", "median_s": med, "times_s": times,
            "evaluations": evals, "instances": count}


def serve_leg(rate, seconds, prec, single_n=None):
    """The serving stream: Poisson arrivals at `rate`/s for `seconds`, N from
    {256, 1024, 4096, 16384, 65536} (weights .3/.3/.2/.15/.05), K~Poisson(N/64),
    SNR~U[5,30] dB, complex64 input, one server per size class on its own
    stream.  Signals come from a seeded pool per N (request i of size N uses
    pool entry i mod pool size); every request is a full solve."""
    import numpy as np
    import torch
    import paper_1705_06073_amd as sf
    from paper_1705_06073_amd import serving, synth

    if single_n:
        arrivals, sizes = synth.serving_stream(rate, seconds, sizes=[single_n])
        pool_sizes = {single_n: 256}
        classes, hbm = ((single_n, 256),), (4 << 30,)
    else:
        arrivals, sizes = synth.serving_stream(rate, seconds)
        pool_sizes, classes, hbm = SERVE_POOL, SERVE_CLASSES, SERVE_HBM
    log(f"serving: {len(arrivals)} requests over {seconds:.0f} s; building the signal pool")
    pool, addr_of = [], {}
    o = 0
    for N, cnt in pool_sizes.items():
        for j in range(cnt):
            inst = synth.workload_serving_signal(N, j)
            pool.append(inst.y.astype(np.complex64))
            addr_of[(N, j)] = o
            o += N
    y = torch.from_numpy(np.concatenate(pool).view(np.float32).copy()).to("cuda:0")
    base = y.data_ptr()
    count = {N: 0 for N in pool_sizes}
    ptrs = np.zeros(len(arrivals), np.int64)
    for i, N in enumerate(sizes):
        N = int(N)
        ptrs[i] = base + 8 * addr_of[(N, count[N] % pool_sizes[N])]
        count[N] += 1
    ctx = sf.Context(0)
    params = sf.default_params(precision=prec)
    lanes = serving.default_lanes(ctx, params, size_classes=classes, hbm_bytes=hbm)
    lane_of = [serving.lane_index(classes, int(n)) for n in sizes]
    # warm the kernels of every lane once (one request each, not timed)
    for N in pool_sizes:
        li = serving.lane_index(classes, N)
        lanes[li].submit(base + 8 * addr_of[(N, 0)], N, 0)
    for s in lanes:
        while s.stats()["in_flight"]:
            s.step()
        s.poll()
    torch.cuda.synchronize()
    log("serving: stream starts")
    res, lat, st = serving.run_stream(lanes, lane_of, arrivals, sizes, lambda i: int(ptrs[i]),
                                      log=log)
    summ = serving.summarize(lat, sizes, arrivals, st["wall_s"])
    statuses = np.array([r.status for r in res])
    summ.update({
        "rate_per_s": rate, "seconds": seconds, "wall_s": st["wall_s"],
        "max_backlog": st["max_backlog"],
        "lanes": [{"max_n": mx, "slots": sl, "rounds": ls["rounds"],
                   "hbm_reserved_GiB": ls["bytes_reserved"] / 2**30}
                  for (mx, sl), ls in zip(classes, st["lanes"])],
        "status_counts": {int(k): int(v) for k, v in zip(*np.unique(statuses, return_counts=True))},
        "evals_mean": float(np.mean([r.evaluations for r in res])),
        "precision": "mixed" if prec == sf.SFLS_MIXED else "fp64",
        "input": "complex64, device-resident signal pool " + str(pool_sizes),
    })
    for s in lanes:
        s.close()
    ctx.close()
    return summ


UNEVEN_CLASSES = ((1024, 1024), (4096, 1024), (16384, 1024))
UNEVEN_HBM = (4 << 30, 16 << 30, 64 << 30)


def uneven_leg(prec, count=2048):
    """The uneven batch: `count` instances with N log-uniform on [128, 16384],
    K ~ Poisson(N/64), SNR ~ U[5,30] dB, complex128, grid 8N; solved (a) by one
    sfls_estimate call for the whole batch and (b) by continuous batching
    through one server per size class (every instance admitted at t = 0)."""
    import numpy as np
    import torch
    import paper_1705_06073_amd as sf
    from paper_1705_06073_amd import serving, synth

    log(f"uneven batch: generating {count} instances")
    insts = [synth.workload_uneven(i, blocked=True) for i in range(count)]
    n = np.array([i.N for i in insts], np.int64)
    off = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)
    y = torch.from_numpy(np.concatenate([i.y.astype(np.complex128) for i in insts])
                         .view(np.float64).copy()).to("cuda:0")
    ctx = sf.Context(0)
    params = sf.default_params(precision=prec)
    out = {}
    # (a) one call
    B = count
    kcap = n.copy()  # K_max = N, as the servers' default capacity
    koff = np.concatenate([[0], np.cumsum(kcap)[:-1]]).astype(np.int64)
    KT = int(kcap.sum())
    f64 = dict(dtype=torch.float64, device="cuda:0")
    i32 = dict(dtype=torch.int32, device="cuda:0")
    o = dict(K=torch.zeros(B, dtype=torch.int64, device="cuda:0"), theta=torch.zeros(KT, **f64),
             alpha=torch.zeros(2 * KT, **f64), gamma=torch.zeros(KT, **f64),
             beta=torch.zeros(B, **f64), zeta=torch.zeros(B, **f64),
             objective=torch.zeros(B, **f64), iters=torch.zeros(B, **i32),
             evals=torch.zeros(B, **i32), status=torch.zeros(B, **i32))
    stream = torch.cuda.current_stream()

    def call():
        sf.sfls_estimate(ctx, n, off, y, sf.SFLS_C128, params, kcap, koff, o["K"], o["theta"],
                         o["alpha"], o["gamma"], o["beta"], o["zeta"], o["objective"],
                         o["iters"], o["evals"], o["status"], stream=stream)
        torch.cuda.synchronize()

    call()  # warm-up
    t = time.perf_counter()
    call()
    ta = time.perf_counter() - t
    run, _ = ctx.last_run()
    st = o["status"].cpu().numpy()
    Ka = o["K"].cpu().numpy()
    out["one_call"] = {"value": B / ta, "unit": "solves/s", "seconds": ta, "rounds": run["rounds"],
                       "evals_mean": run["evals"] / B,
                       "status_counts": {int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))}}
    log(f"uneven batch, one call: {B / ta:.1f} solves/s ({run['rounds']} rounds)")
    # (b) size-class servers
    lanes = serving.default_lanes(ctx, params, size_classes=UNEVEN_CLASSES, hbm_bytes=UNEVEN_HBM,
                                  ydtype=sf.SFLS_C128)
    lane_of = [serving.lane_index(UNEVEN_CLASSES, int(v)) for v in n]
    base = y.data_ptr()
    arrivals = np.zeros(B)
    res, lat, stt = serving.run_stream(lanes, lane_of, arrivals, n, lambda i: base + 16 * int(off[i]))
    tb = stt["wall_s"]
    Kb = np.array([r.K for r in res])
    out["size_class_servers"] = {
        "value": B / tb, "unit": "solves/s", "seconds": tb,
        "lanes": [{"max_n": mx, "slots": sl, "rounds": ls["rounds"]}
                  for (mx, sl), ls in zip(UNEVEN_CLASSES, stt["lanes"])],
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p99": float(np.percentile(lat, 99) * 1e3)}}
    log(f"uneven batch, size-class servers: {B / tb:.1f} solves/s")
    out["workload"] = (f"{B} instances, N log-uniform on [128, 16384] (mean {n.mean():.0f}), "
                       "K ~ Poisson(N/64), separation 1/N, alpha ~ CN(0,1), SNR ~ U[5,30] dB, "
                       "complex128, grid 8N")
    out["K_equal_between_the_two"] = int(np.sum(Ka == Kb))
    for s in lanes:
        s.close()
    ctx.close()
    return out


def incomplete_leg(steps, warmup, prec, B=256):
    """Incomplete data by the semifast method (Sec. IV): B instances of the
    runtime experiment's incomplete workload (N = 4096, M = 3072 rows of the
    identity, K = 15, 20 dB, complex64), one sfls_estimate_incomplete call per
    step timed end to end; then one more call with every kernel timed."""
    import numpy as np
    import torch
    import paper_1705_06073_amd as sf
    from paper_1705_06073_amd import synth
    dev = torch.device("cuda", 0)
    insts = [synth.workload_incomplete_n4096(i) for i in range(B)]
    ctx = sf.Context(0)
    n, m, moff, idx, phid, ydev, ydt = sf.pack_incomplete(ctx, [(i.N, i.idx, i.phi, i.y)
                                                               for i in insts])
    kc = np.full(B, sf.SFLS_SF_MAX_K, np.int64)
    koff = np.concatenate([[0], np.cumsum(kc)[:-1]]).astype(np.int64)
    KT = int(kc.sum())
    f64 = dict(dtype=torch.float64, device=dev)
    i32 = dict(dtype=torch.int32, device=dev)
    out = dict(K=torch.zeros(B, dtype=torch.int64, device=dev), theta=torch.zeros(KT, **f64),
               alpha=torch.zeros(2 * KT, **f64), gamma=torch.zeros(KT, **f64),
               beta=torch.zeros(B, **f64), zeta=torch.zeros(B, **f64),
               objective=torch.zeros(B, **f64), iters=torch.zeros(B, **i32),
               evals=torch.zeros(B, **i32), status=torch.zeros(B, **i32))
    params = sf.default_params(precision=prec)
    stream = torch.cuda.current_stream()

    def call():
        sf.sfls_estimate_incomplete(ctx, n, m, moff, idx, phid, ydev, ydt, params, kc, koff,
                                    out["K"], out["theta"], out["alpha"], out["gamma"],
                                    out["beta"], out["zeta"], out["objective"], out["iters"],
                                    out["evals"], out["status"], stream=stream)

    for w in range(warmup):
        t = time.perf_counter()
        call()
        torch.cuda.synchronize()
        log(f"incomplete warmup {w + 1}/{warmup}: {time.perf_counter() - t:.3f} s")
    times, rounds = [], 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in range(steps):
        ts = time.perf_counter()
        call()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        run, _ = ctx.last_run()
        rounds += run["rounds"]
        log(f"incomplete step {s_ + 1}/{steps}: {times[-1]:.3f} s, rounds={run['rounds']}")
    elapsed = time.perf_counter() - t0
    Kh = out["K"].cpu().numpy()
    st = out["status"].cpu().numpy()
    evs = out["evals"].cpu().numpy()
    # one more call with every kernel timed, outside the timed region
    ctx.reset_stats()
    ctx.set_timing(1)
    torch.cuda.synchronize()
    tk0 = time.perf_counter()
    call()
    torch.cuda.synchronize()
    tk = time.perf_counter() - tk0
    ctx.set_timing(False)
    kst = ctx.kernel_stats()
    ksum = sum(v["seconds"] for v in kst.values())
    names = {"factor": "semifast evaluation (Gram sums, K x K Cholesky, residual)",
             "omega": "semifast grid inputs (Phi^H C^-1 y, columns U, omega_s by FFT)",
             "active": "semifast candidates (direct sums)", "grid": "grid q^G, s^G, Delta L",
             "select": "grid selection", "driver": "driver"}
    kernels = {}
    for k, v in kst.items():
        if v["launches"] == 0:
            continue
        e = {"stage": names.get(k, k), "launches": v["launches"], "ms_total": 1e3 * v["seconds"],
             "share": v["seconds"] / max(1e-30, ksum)}
        if v["flops"] > 0 and v["seconds"] > 0:
            e["fp64_TFLOPs"] = v["flops"] / v["seconds"] / 1e12
            e["fp64_frac"] = v["flops"] / v["seconds"] / FP64_PEAK
        if v["bytes"] > 0 and v["seconds"] > 0:
            e["hbm_GBps"] = v["bytes"] / v["seconds"] / 1e9
            e["hbm_frac"] = v["bytes"] / v["seconds"] / HBM_PEAK
        kernels[k] = e
    ctx.close()
    value = steps * B / elapsed
    return {"value": value, "unit": "solves/s",
            "workload": f"{B} instances, N=4096, M=3072 observed rows of the identity (first and "
                        "last sample kept), K=15, separation 2/N, alpha = a + 0.2 e^(j arg a), "
                        "20 dB, complex64 input; FP64 evaluation, "
                        + ("FP32" if prec == sf.SFLS_MIXED else "FP64") + " grid",
            "ms_per_step": 1e3 * elapsed / steps, "steps": steps,
            "rounds_per_batch": rounds / steps, "K_mean": float(np.mean(Kh)),
            "evals_mean": float(np.mean(evs)), "evals_max": int(evs.max()),
            "status_counts": {int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))},
            "kernels": kernels,
            "round_idle_frac": max(0.0, 1.0 - ksum / float(np.median(times))),
            "round_idle_frac_event_timed": max(0.0, 1.0 - ksum / tk),
            "paper_context": {"seconds_per_solve": 0.930,
                              "hardware": "MATLAB, one thread, 2011 MacBook Pro (Fig. runtime_N, "
                                          "incomplete data, N = 4096)",
                              "solves_per_s": 1.0 / 0.930}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--plain", type=int, default=256,
                    help="instances for the plain FP64 one-per-launch baseline (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-solves", type=int, default=0,
                    help="also time this many whole oracle solves of the batch (minutes each)")
    ap.add_argument("--nufft", choices=["auto", "off", "on"], default="auto",
                    help="off-grid Fourier sums by direct sums or NUFFT (default: per instance)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only copy this many bytes device to device (the calibration copy "
                         "for the HBM counters) and exit")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--factor", choices=["auto", "levinson", "schur"], default="auto",
                    help="generator recursion (auto: superfast Schur from N=256 on)")
    ap.add_argument("--slots", type=int, default=256,
                    help="server slots of the continuous-batching leg (instances on the device)")
    ap.add_argument("--servers", type=int, default=1,
                    help="servers (each on its own stream) sharing the continuous-batching leg")
    ap.add_argument("--schur-lds", type=int, default=4096,
                    help="largest superfast-recursion transform kept in LDS (256..4096)")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="also run the serving stream for this many seconds of arrivals "
                         "(60 for the full stream)")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve4096-seconds", type=float, default=3.0,
                    help="serving stream of N=4096 requests beside the default legs (0: skip)")
    ap.add_argument("--serve4096-rate", type=float, default=2000.0)
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving stream and print its summary")
    ap.add_argument("--incomplete-steps", type=int, default=3,
                    help="steps of the incomplete-data (semifast) leg; 0 skips it")
    ap.add_argument("--incomplete-only", action="store_true",
                    help="run only the incomplete-data leg and print its JSON")
    ap.add_argument("--uneven", action="store_true",
                    help="run only the uneven batch (2048 instances, N in [128, 16384])")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the uneven batch leg of the default run")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU: the estimator's instances are independent, so a "
              f"multi-GPU run is N copies of this one (got --gpus {args.gpus}, "
              f"WORLD_SIZE={world}); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.serve_only or args.serve_seconds > 0:
        # one hardware queue per server stream (HIP's default is 4 per process)
        os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")
    import numpy as np
    import torch
    import paper_1705_06073_amd as sf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    if args.copy_bytes > 0:
        src = torch.ones(args.copy_bytes, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "copies": 3}))
        return
    if args.incomplete_only:
        prec = sf.SFLS_MIXED if args.precision == "mixed" else sf.SFLS_FP64
        print(json.dumps({"incomplete": incomplete_leg(max(1, args.incomplete_steps),
                                                       args.warmup, prec)}), flush=True)
        return
    if args.uneven:
        prec = sf.SFLS_MIXED if args.precision == "mixed" else sf.SFLS_FP64
        print(json.dumps({"uneven": uneven_leg(prec)}), flush=True)
        return
    if args.serve_only:
        prec = sf.SFLS_MIXED if args.precision == "mixed" else sf.SFLS_FP64
        print(json.dumps({"serving": serve_leg(args.serve_rate, args.serve_seconds or 10.0,
                                               prec)}), flush=True)
        return
    log(f"generating {args.batch} instances (N=4096)")
    insts, _ = make_workload(args.batch)
    B = len(insts)
    n = np.array([i.N for i in insts], np.int64)
    off = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)
    kcap = np.full(B, 256, np.int64)
    koff = np.concatenate([[0], np.cumsum(kcap)[:-1]]).astype(np.int64)
    yflat = np.concatenate([i.y.astype(np.complex128) for i in insts])
    y = torch.from_numpy(yflat.view(np.float64).copy()).to(dev)
    KT = int(kcap.sum())
    f64 = dict(dtype=torch.float64, device=dev)
    i32 = dict(dtype=torch.int32, device=dev)
    out = dict(K=torch.zeros(B, dtype=torch.int64, device=dev), theta=torch.zeros(KT, **f64),
               alpha=torch.zeros(2 * KT, **f64), gamma=torch.zeros(KT, **f64),
               beta=torch.zeros(B, **f64), zeta=torch.zeros(B, **f64),
               objective=torch.zeros(B, **f64), iters=torch.zeros(B, **i32),
               evals=torch.zeros(B, **i32), status=torch.zeros(B, **i32))
    prec = sf.SFLS_MIXED if args.precision == "mixed" else sf.SFLS_FP64
    params = sf.default_params(precision=prec)
    ctx = sf.Context(0)
    ctx.set_factor({"auto": sf.SFLS_FACTOR_AUTO, "levinson": sf.SFLS_FACTOR_LEVINSON,
                    "schur": sf.SFLS_FACTOR_SCHUR}[args.factor])
    ctx.set_nufft({"auto": sf.SFLS_NUFFT_AUTO, "off": sf.SFLS_NUFFT_OFF,
                   "on": sf.SFLS_NUFFT_ON}[args.nufft])
    ctx.set_schur_lds(args.schur_lds)
    stream = torch.cuda.current_stream()

    def run_batch():
        sf.sfls_estimate(ctx, n, off, y, sf.SFLS_C128, params, kcap, koff, out["K"],
                         out["theta"], out["alpha"], out["gamma"], out["beta"], out["zeta"],
                         out["objective"], out["iters"], out["evals"], out["status"],
                         stream=stream)

    # --- continuous batching (the reported value): the steps' batches stream
    # through a server with one slot per instance of a batch; a slot freed by
    # a finished solve takes the next instance for the next round, so no
    # round waits for the slowest instance of its batch.
    streams = [stream] + [torch.cuda.Stream() for _ in range(args.servers - 1)]
    srvs = [sf.Server(ctx, max_n=4096, max_slots=args.slots, ydtype=sf.SFLS_C128,
                      hbm_bytes=(4 << 30) * max(1, args.slots // 256), params=params, stream=s)
            for s in streams]
    yaddr = np.array([y.data_ptr() + 16 * int(o) for o in off], dtype=np.uint64)
    n_np = np.asarray(n, dtype=np.int64)

    def admit(srv, nxt, total):
        # queued instances into the slots the last round freed, in one call
        idx = np.arange(nxt, min(total, nxt + args.slots), dtype=np.int64)
        if len(idx) == 0:
            return nxt
        return nxt + srv.submit_many(yaddr[idx % B], n_np[idx % B], idx.astype(np.uint64))

    def run_stream(nsteps):
        # when a round completes, the slots its finished solves freed take the
        # next instances at once (they join the next round, which starts right
        # after); results are collected while that round runs
        total = nsteps * B
        nxt, got = 0, []
        for srv in srvs:
            nxt = admit(srv, nxt, total)
            srv.launch()
        while len(got) < total:
            for srv in srvs:
                if len(srvs) > 1:
                    ready, _ = srv.wait(block=False)
                    if not ready:
                        continue
                else:
                    srv.wait()
                nxt = admit(srv, nxt, total)
                srv.launch()
                got += srv.poll()
        return got

    # --- the batched measurement (value): one sfls_estimate call per step of
    # 256 instances, timed end to end, so each step waits for its slowest
    # instance; the timed legs bracket only the recursion with events (the
    # roofline's kernel), since an event between two kernels idles the device
    for w in range(args.warmup):
        t = time.perf_counter()
        run_batch()
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup} (one call per batch): {time.perf_counter() - t:.3f} s")
    ctx.reset_stats()
    ctx.set_timing(2)
    lat, step_s, rounds_b = [], [], 0
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    for s_ in range(args.steps):
        ts = time.perf_counter()
        run_batch()
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - ts)
        run, timeline = ctx.last_run()
        rounds_b += run["rounds"]
        ev = out["evals"].cpu().numpy()
        lat.extend(timeline[np.clip(ev, 0, len(timeline) - 1)].tolist())
        log(f"step {s_ + 1}/{args.steps}: {step_s[-1]:.3f} s, rounds={run['rounds']}, "
            f"evals={run['evals']} (grid {run['grid_evals']})")
    torch.cuda.synchronize()
    elapsed_b = time.perf_counter() - tb0
    kst = ctx.kernel_stats()
    run, _ = ctx.last_run()
    st = out["status"].cpu().numpy()
    Kh = out["K"].cpu().numpy()
    its = out["iters"].cpu().numpy()
    evs = out["evals"].cpu().numpy()
    solves = args.steps * B
    value = solves / elapsed_b

    # --- continuous batching (secondary): the same batches stream through a
    # server with one slot per instance of a batch; a slot freed by a finished
    # solve takes the next instance for the next round
    for w in range(args.warmup):
        t = time.perf_counter()
        run_stream(1)
        log(f"warmup {w + 1}/{args.warmup} (continuous): {time.perf_counter() - t:.3f} s")
    r0 = sum(s.stats()["rounds"] for s in srvs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    served = run_stream(args.steps)
    torch.cuda.synchronize()
    elapsed_c = time.perf_counter() - t0
    rounds_c = sum(s.stats()["rounds"] for s in srvs) - r0
    lat_c = np.array([r.t_done - r.t_submit for r in served])
    log(f"continuous: {solves} solves in {elapsed_c:.3f} s over {rounds_c} rounds")
    for r in served:
        assert r.status in (sf.SFLS_OK, sf.SFLS_NOTCONV), r.status
    for s in srvs:
        s.close()
    ctx.set_timing(False)
    # every step solves the same batch: each served solve of instance b has
    # the model order the batch call found for b
    same_K = int(sum(int(r.K == Kh[r.tag % B]) for r in served))

    # --- per-kernel breakdown: one more call of the batch, outside the timed
    # region, with every kernel bracketed by events
    ctx.reset_stats()
    ctx.set_timing(1)
    torch.cuda.synchronize()
    tk0 = time.perf_counter()
    run_batch()
    torch.cuda.synchronize()
    tk = time.perf_counter() - tk0
    ctx.set_timing(False)
    kst_all = ctx.kernel_stats()
    run_k, _ = ctx.last_run()
    ksum = sum(x["seconds"] for x in kst_all.values())
    kernels = {}
    for k, v in kst_all.items():
        e = {"launches": v["launches"], "ms_total": 1e3 * v["seconds"],
             "share": v["seconds"] / max(1e-30, ksum)}
        if v["bytes"] > 0 and v["seconds"] > 0:
            e["hbm_GBps"] = v["bytes"] / v["seconds"] / 1e9
            e["hbm_frac"] = v["bytes"] / v["seconds"] / HBM_PEAK
        if v["flops"] > 0 and v["seconds"] > 0:
            e["fp64_TFLOPs"] = v["flops"] / v["seconds"] / 1e12
            e["fp64_frac"] = v["flops"] / v["seconds"] / FP64_PEAK
        kernels[k] = e
    rounds_k = max(1, run_k["rounds"])
    t_med = float(np.median(step_s))
    idle = {"round_ms": 1e3 * t_med / rounds_k, "kernels_ms_per_round": 1e3 * ksum / rounds_k,
            "idle_frac": max(0.0, 1.0 - ksum / t_med),
            "idle_frac_event_timed": max(0.0, 1.0 - ksum / tk),
            "definition": "1 - (sum of the kernel event durations of one batch call with every "
                          "kernel timed) / (median wall time of the timed, untimed-kernel calls "
                          "of the same batch); idle_frac_event_timed divides by the wall time of "
                          "the event-timed call itself, whose events add gaps of their own"}

    # dominant kernel and its roofline position
    dom = max(kst.items(), key=lambda kv: kv[1]["seconds"])
    name, ks = dom
    algo = "levinson" if args.factor == "levinson" else "schur"  # AUTO: Schur from N=256 on
    launches = max(1, ks["launches"])
    traffic = None
    if name == "factor" and algo == "schur" and B == 256:
        # HBM bytes per launch from the committed counter summary of this
        # workload (None once the kernel's sources have changed)
        from paper_1705_06073_amd import pmc
        traffic = pmc.traffic_bytes(os.path.join(ROOT, "profiles",
                                                 "k_schur_n4096_b256_traffic.md"), "k_schur")
    hbm_alg = ks["bytes"] / launches
    hbm_read = {"bound": "hbm", "achieved": ks["bytes"] / ks["seconds"] / 1e9,
                "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": ks["bytes"] / ks["seconds"] / HBM_PEAK,
                "algorithmic_per_launch": hbm_alg,
                "traffic_over_algorithmic": (traffic / hbm_alg) if traffic and hbm_alg else None}
    if ks["flops"] > 0:
        achieved = ks["flops"] / ks["seconds"]
        roof = {"bound": "alu", "kernel": name + (f" ({algo})" if name == "factor" else ""),
                "achieved": achieved / 1e12, "peak": FP64_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": achieved / FP64_PEAK, "traffic": traffic,
                "avg_launch_ms": 1e3 * ks["seconds"] / launches,
                "algorithmic_per_launch": ks["flops"] / launches,
                "hbm_reading": hbm_read}
    else:
        roof = dict(hbm_read, kernel=name, traffic=traffic,
                    avg_launch_ms=1e3 * ks["seconds"] / launches)

    # plain FP64, one instance per launch, no batching
    plain = None
    if args.plain > 0:
        pp = sf.default_params(precision=sf.SFLS_FP64)
        nb = min(args.plain, B)
        times = []
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for b in range(nb):
            tb = time.perf_counter()
            sf.sfls_estimate(ctx, n[b:b + 1], np.zeros(1, np.int64), y[2 * off[b]:2 * (off[b] + n[b])],
                             sf.SFLS_C128, pp, kcap[b:b + 1], np.zeros(1, np.int64), out["K"],
                             out["theta"], out["alpha"], out["gamma"], out["beta"], out["zeta"],
                             out["objective"], out["iters"], out["evals"], out["status"],
                             stream=stream)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - tb)
            if (b + 1) % 64 == 0:
                log(f"plain FP64: {b + 1}/{nb}")
        tp = time.perf_counter() - tp0
        plain = {"value": nb / tp, "unit": "solves/s", "instances": nb,
                 "latency_ms": {"p50": 1e3 * float(np.percentile(times, 50)),
                                "p99": 1e3 * float(np.percentile(times, 99))}}
        log(f"plain FP64: {nb} solves in {tp:.2f} s")

    serve = None
    if args.serve_seconds > 0:
        serve = serve_leg(args.serve_rate, args.serve_seconds, prec)
    serve4096 = None
    if args.serve4096_seconds > 0:
        serve4096 = serve_leg(args.serve4096_rate, args.serve4096_seconds, prec, single_n=4096)

    incomplete = None
    if args.incomplete_steps > 0:
        incomplete = incomplete_leg(args.incomplete_steps, args.warmup, prec)
    uneven = None
    if not args.no_uneven:
        uneven = uneven_leg(prec)

    cpu = None
    if not args.no_cpu_baseline:
        g_per = run["grid_evals"] / B
        a_per = (run["evals"] - run["grid_evals"]) / B
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(insts, a_per, g_per)
        if args.cpu_solves > 0:
            cpu["whole_solves"] = cpu_full_solves(insts, args.cpu_solves)

    lat = np.array(lat)
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed_b / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32grid" if prec == sf.SFLS_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": "256 independent instances, N=4096, K~Poisson(40), separation "
                               "1/N, alpha~CN(0,1), SNR~U[0,30] dB, grid L=8N=32768; FP64 "
                               "recursion, " + ("FP32" if prec == sf.SFLS_MIXED else "FP64")
                               + " grid; a step is one sfls_estimate call solving a batch of "
                               "256 to completion",
                   "batch": B, "N": 4096, "L": 32768,
                   "precision": "mixed" if prec == sf.SFLS_MIXED else "fp64",
                   "factor": args.factor, "nufft": args.nufft},
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                       "p99": 1e3 * float(np.percentile(lat, 99)),
                       "definition": "completion of each solve within its batch (from the start "
                                     "of the call)"},
        "batch_median": {"value": B / float(np.median(step_s)), "unit": "solves/s",
                         "ms": 1e3 * float(np.median(step_s)),
                         "definition": "256 / median wall time of one batch call"},
        "rounds_per_batch": rounds_b / args.steps,
        "continuous": {"value": solves / elapsed_c, "unit": "solves/s",
                       "ms_per_step": 1e3 * elapsed_c / args.steps,
                       "latency_ms": {"p50": 1e3 * float(np.percentile(lat_c, 50)),
                                      "p99": 1e3 * float(np.percentile(lat_c, 99)),
                                      "definition": "admission to completion"},
                       "rounds": rounds_c, "slots": args.slots, "servers": args.servers,
                       "solves": solves, "schur_lds_transform": args.schur_lds,
                       "solves_with_K_of_the_batch_call": same_K,
                       "definition": "the same batches streamed through a 256-slot server"},
        "plain_fp64": plain,
        "per_solve": {"evals_mean": run["evals"] / B, "grid_evals_mean": run["grid_evals"] / B,
                      "evals_p50": float(np.percentile(evs, 50)),
                      "evals_p99": float(np.percentile(evs, 99)), "evals_max": int(evs.max()),
                      "rounds": run["rounds"], "iters_mean": float(np.mean(its)),
                      "iters_p50": float(np.percentile(its, 50)), "iters_max": int(its.max()),
                      "K_mean": float(np.mean(Kh)),
                      "status_counts": {int(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))}},
        "roofline": roof,
        "kernels": kernels,
        "kernels_source": ("one more sfls_estimate call of the batch (256 solves) with every "
                           "kernel timed, outside the timed region; ms_total per call"),
        "round_idle": idle,
        "cpu_baseline": cpu,
        "serving": serve,
        "serving_n4096": serve4096,
        "incomplete": incomplete,
        "uneven": uneven,
    }
    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
