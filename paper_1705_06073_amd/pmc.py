"""HBM traffic of a kernel from rocprofv3 hardware counters.

Two counter runs of the same program (FETCH_SIZE, then WRITE_SIZE, in KiB per
dispatch) give the bytes one dispatch of the kernel moves between the caches
and HBM.  Each counter is scaled by what it reads for a plain device copy of
known size (the copy reads and writes that many bytes), run under the same
counters.  The summary records a hash of the sources that define the kernel:
`traffic_bytes` returns None once they differ from the measured build.

    python -m paper_1705_06073_amd.pmc --kernel k_schur \\
        --fetch F.csv --write W.csv --cal-fetch CF.csv --cal-write CW.csv \\
        --cal-bytes 1073741824 --cmd "..." --out profiles/<kernel>_<workload>_traffic.md
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re

_PKG = os.path.dirname(os.path.abspath(__file__))
# sources whose change invalidates a measured figure, per kernel
KERNEL_SOURCES = {
    "k_schur": ["csrc/k_schur.hip", "csrc/dev_common.hpp", "csrc/sfls_kernels.hpp",
                "csrc/abi.hip", "csrc/server.hip", "csrc/host_internal.hpp"],
}


def sources_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kernel]:
        with open(os.path.join(_PKG, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read() + b"\0")
    return h.hexdigest()


def counter_values(path: str, kernel_regex: str, counter: str) -> list[float]:
    """Per-dispatch values of one counter for the kernels matching the regex."""
    rx = re.compile(kernel_regex)
    out = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] == counter and rx.search(row["Kernel_Name"]):
                d = int(row["Dispatch_Id"])
                out[d] = out.get(d, 0.0) + float(row["Counter_Value"])
    return [out[d] for d in sorted(out)]


def traffic_bytes(summary_path: str, kernel: str) -> float | None:
    """Bytes per launch recorded in a summary, or None when it is missing or
    was measured on other sources."""
    try:
        with open(summary_path) as f:
            text = f.read()
    except OSError:
        return None
    m = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+-]+)\s*$", text, re.M)
    hs = re.search(r"^sources_sha256:\s*([0-9a-f]{64})\s*$", text, re.M)
    if not m or not hs or hs.group(1) != sources_hash(kernel):
        return None
    return float(m.group(1))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--cal-fetch", required=True)
    ap.add_argument("--cal-write", required=True)
    ap.add_argument("--cal-bytes", type=float, required=True)
    ap.add_argument("--cal-regex", default="copyBuffer")
    ap.add_argument("--cmd", action="append", default=[], help="commands that made the CSVs")
    ap.add_argument("--title", default="")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    fk = counter_values(a.fetch, a.kernel, "FETCH_SIZE")
    wk = counter_values(a.write, a.kernel, "WRITE_SIZE")
    cf = counter_values(a.cal_fetch, a.cal_regex, "FETCH_SIZE")
    cw = counter_values(a.cal_write, a.cal_regex, "WRITE_SIZE")
    if not (fk and wk and cf and cw):
        raise SystemExit("missing counter rows")
    kib = a.cal_bytes / 1024.0
    # the largest copy dispatch is the calibration copy (smaller ones are staging)
    sf, sw = kib / max(cf), kib / max(cw)
    mf, mw = sum(fk) / len(fk), sum(wk) / len(wk)
    tb = (mf * sf + mw * sw) * 1024.0
    lines = [f"# HBM traffic of {a.kernel}{(' - ' + a.title) if a.title else ''}", "",
             "Commands (from the repository root on one MI355X; $REPO is the repository root):", ""]
    lines += [f"    {c}" for c in a.cmd]
    lines += ["",
              "| quantity | FETCH_SIZE | WRITE_SIZE |", "|---|---:|---:|",
              f"| copy of {a.cal_bytes:.0f} bytes, KiB read by the counter | {max(cf):.1f} | {max(cw):.1f} |",
              f"| scale (true KiB per counted KiB) | {sf:.4f} | {sw:.4f} |",
              f"| {a.kernel}: dispatches | {len(fk)} | {len(wk)} |",
              f"| {a.kernel}: mean KiB per dispatch (counted) | {mf:.1f} | {mw:.1f} |",
              f"| {a.kernel}: min / max KiB per dispatch | {min(fk):.1f} / {max(fk):.1f} | "
              f"{min(wk):.1f} / {max(wk):.1f} |",
              f"| {a.kernel}: mean bytes per dispatch (scaled) | {mf * sf * 1024:.4e} | {mw * sw * 1024:.4e} |",
              "",
              f"traffic_bytes_per_launch: {tb:.6e}",
              f"sources_sha256: {sources_hash(a.kernel)}", ""]
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print(f"{a.kernel}: {tb:.4e} bytes per launch -> {a.out}")


if __name__ == "__main__":
    main()
