"""Request loop of the estimation server: requests arrive over time, are
admitted into servers (one per size class, each on its own stream) as slots
and pool memory free up, and every server runs evaluation rounds while others
do, so the device interleaves their kernels.

All estimation work runs in the library's kernels (sfls_server_*); this loop
only decides when to submit, launch and collect.
"""
from __future__ import annotations

import collections
import sys
import time

import numpy as np

from . import Server


def run_stream(lanes, lane_of, arrivals, sizes, ptr_of, progress_every: float = 5.0,
               log=None):
    """Serve requests i = 0..R-1 arriving at arrivals[i] seconds (ascending)
    with length sizes[i]; request i goes to lanes[lane_of[i]] with its signal
    at device address ptr_of(i).  Returns (results, latency_s, stats), where
    latency is completion minus arrival on the host clock."""
    R = len(arrivals)
    queues = [collections.deque() for _ in lanes]
    lat = np.full(R, np.nan)
    results = [None] * R
    max_backlog = 0
    done = 0
    i = 0
    t0 = time.perf_counter()
    next_report = progress_every
    while done < R:
        now = time.perf_counter() - t0
        while i < R and arrivals[i] <= now:
            queues[lane_of[i]].append(i)
            i += 1
        backlog = sum(len(q) for q in queues)
        max_backlog = max(max_backlog, backlog)
        progressed = False
        for li, srv in enumerate(lanes):
            fin = 0
            if srv.in_flight:
                ready, fin = srv.wait(block=False)
                if ready:
                    progressed = True
            # admission: when a round has completed, the slots it freed take
            # queued requests before the next round starts (they join it);
            # while a round runs, arrivals are admitted for the round after
            q = queues[li]
            while q and srv.submit(ptr_of(q[0]), int(sizes[q[0]]), q[0]):
                q.popleft()
            if not srv.in_flight:
                srv.launch()
            # results are collected while the next round runs
            if fin:
                tc = time.perf_counter() - t0
                for r in srv.poll():
                    lat[r.tag] = tc - arrivals[r.tag]
                    results[r.tag] = r
                    done += 1
        if not any(s.in_flight for s in lanes):
            if i < R:
                time.sleep(max(0.0, arrivals[i] - (time.perf_counter() - t0)))
            continue
        if not progressed:
            time.sleep(0)  # yield; a timed sleep would add its granularity to every round
        if log is not None and now >= next_report:
            log(f"serving t={now:.1f}s arrived={i} done={done} backlog={backlog}")
            next_report += progress_every
    wall = time.perf_counter() - t0
    stats = dict(wall_s=wall, max_backlog=max_backlog,
                 lanes=[s.stats() for s in lanes])
    return results, lat, stats


def summarize(lat, sizes, arrivals, wall_s):
    out = dict(requests=int(len(lat)),
               offered_per_s=float(len(lat) / max(arrivals[-1], 1e-9)) if len(lat) else 0.0,
               achieved_per_s=float(len(lat) / wall_s) if wall_s > 0 else 0.0,
               latency_ms=dict(p50=float(np.percentile(lat, 50) * 1e3),
                               p99=float(np.percentile(lat, 99) * 1e3)),
               by_n={})
    for n in sorted(set(int(v) for v in sizes)):
        m = sizes == n
        out["by_n"][str(n)] = dict(count=int(m.sum()),
                                   p50_ms=float(np.percentile(lat[m], 50) * 1e3),
                                   p99_ms=float(np.percentile(lat[m], 99) * 1e3))
    return out


def default_lanes(ctx, params, size_classes=((1024, 1024), (4096, 512), (65536, 256)),
                  hbm_bytes=(4 << 30, 8 << 30, 48 << 30), ydtype=None):
    """One server per size class: (max_n, max_slots) each with its own stream."""
    import torch
    from . import SFLS_C64
    lanes = []
    for (mx, slots), hb in zip(size_classes, hbm_bytes):
        st = torch.cuda.Stream(device=ctx.device)
        lanes.append(Server(ctx, max_n=mx, max_slots=slots,
                            ydtype=SFLS_C64 if ydtype is None else ydtype, hbm_bytes=hb,
                            params=params, stream=st))
        lanes[-1]._torch_stream = st
    return lanes


def lane_index(size_classes, n):
    for li, (mx, _) in enumerate(size_classes):
        if n <= mx:
            return li
    raise ValueError(f"no lane takes n = {n}")


if __name__ == "__main__":
    sys.exit("use bench.py --serve")
