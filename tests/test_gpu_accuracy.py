"""The GPU estimator reproduces the Superfast LSE curves of the paper's
accuracy experiments (Sec. VI) at the paper's 500 trials per point:
Fig. snr (N = 128, K = 10, SNR -5 .. 30 dB) and Fig. pairsep (5 pairs with
separation 0.2/N .. 1.75/N at 20 dB), and the Semifast LSE curves of Fig. MtoN
(incomplete data, M/N = 0.4 .. 1; below 0.4 the oracle itself activates more
spurious components than the figure shows, and those points are printed, not
compared).  Expected values: the figures' plot data
(tests/golden/fig_snr_n128_k10.txt, tests/golden/fig_pairsep_n128_k10.txt,
tests/golden/fig_mton_n128_k10.txt).

Our trials are other random draws than the paper's, so each rate is compared
within three standard errors of the difference of two 500-trial estimates
(plus 0.01), CSR within 0.01, NMSE within 1 dB; the least-squares NMSE with
the true frequencies (the figures' Oracle curve) pins the generator within
0.3 dB.  Where the paper's BSR is 0 (-5 dB: no estimate recovers the model)
only the BSR is compared; the CSR and NMSE there average estimates of noise
and are printed, not compared."""
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import accuracy  # noqa: E402
import paper_1705_06073_amd as sf  # noqa: E402

TRIALS = 500
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    rows = {}
    for line in open(os.path.join(GOLD, name)):
        if line.startswith("#") or not line.strip():
            continue
        x, bsr, csr, nmse, ls = map(float, line.split())
        rows[x] = dict(bsr=bsr, csr=csr, nmse=nmse, ls=ls)
    return rows


@pytest.fixture(scope="module")
def ctx():
    c = sf.Context(0)
    yield c
    c.close()


def compare(ref, got, label, skip=()):
    bad = []
    for x, r in sorted(ref.items()):
        g = got[x]
        p = 0.5 * (r["bsr"] + g["bsr"])
        tol = 3.0 * math.sqrt(max(p * (1 - p), 0.0) * 2.0 / TRIALS) + 0.01
        line = (f"[{label}] {x:>6}: BSR {g['bsr']:.3f} (paper {r['bsr']:.3f}, tol {tol:.3f})  "
                f"CSR {g['csr']:.4f} ({r['csr']:.4f})  NMSE {g['nmse_db']:.2f} dB "
                f"({r['nmse']:.2f})  LS {g['oracle_ls_nmse_db']:.2f} ({r['ls']:.2f})")
        print(line + (" (printed only)" if x in skip else ""), flush=True)
        if x in skip:
            continue
        if abs(g["bsr"] - r["bsr"]) > tol:
            bad.append(("bsr", x, g["bsr"], r["bsr"]))
        if r["bsr"] > 0.0:
            if abs(g["csr"] - r["csr"]) > 0.01:
                bad.append(("csr", x, g["csr"], r["csr"]))
            if abs(g["nmse_db"] - r["nmse"]) > 1.0:
                bad.append(("nmse", x, g["nmse_db"], r["nmse"]))
        if abs(g["oracle_ls_nmse_db"] - r["ls"]) > 0.3:
            bad.append(("ls", x, g["oracle_ls_nmse_db"], r["ls"]))
    assert not bad, bad


def test_fig_snr_500_trials(ctx):
    out, dt, count = accuracy.figure_snr(ctx, TRIALS, sf.default_params())
    print(f"[snr] {count} solves in {dt:.2f} s", flush=True)
    compare(load("fig_snr_n128_k10.txt"), out, "snr")


def test_fig_pairsep_500_trials(ctx):
    out, dt, count = accuracy.figure_pairsep(ctx, TRIALS, sf.default_params())
    print(f"[pairsep] {count} solves in {dt:.2f} s", flush=True)
    compare(load("fig_pairsep_n128_k10.txt"), out, "pairsep")


def test_fig_mton_500_trials(ctx):
    out, dt, count = accuracy.figure_mton(ctx, TRIALS, sf.default_params())
    print(f"[mton] {count} solves in {dt:.2f} s", flush=True)
    compare(load("fig_mton_n128_k10.txt"), out, "mton", skip=(0.2, 0.3))
