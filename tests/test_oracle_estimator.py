"""Pins of the oracle estimator (no GPU): block-descent invariant, noiseless
recovery, the generator's SNR definition, and the paper's accuracy figures."""
import math

import numpy as np
import pytest

from oracle.estimator import Params, estimate
from paper_1705_06073_amd import synth
from tests import metrics

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden",
                                    "fig_snr_n128_k10.txt")


def load_fig_snr():
    rows = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        snr, bsr, csr, nmse, ls = map(float, line.split())
        rows[snr] = dict(bsr=bsr, csr=csr, nmse=nmse, ls=ls)
    return rows


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_every_exact_block_update_does_not_increase_the_objective(seed):
    """Each block update (exact activation, zeta, beta, L-BFGS step, deactivation) never
    increases the objective (Sec. II-C; Appendix A lemmas).  The approximate activation
    sweep of Sec. II-F activates several components judged against one C and is exempt."""
    inst = synth.workload_paper_snr(seed, 9.0, N=48, K=4)
    res = estimate(inst.y, Params(), check_blocks=True)
    blocks = [t for t in res.trace if t[0] == "block"]
    assert blocks, "no block updates recorded"
    names = {b[1] for b in blocks}
    assert {"zeta", "beta", "lbfgs"} <= names
    for _, name, fb, fa in blocks:
        if name == "approx":
            continue
        assert fa <= fb + 1e-9 * max(1.0, abs(fb)), (name, fb, fa)


def test_exact_activation_only_also_monotone():
    inst = synth.workload_n64(3)
    res = estimate(inst.y, Params(L_mult=4.0, approx_max_iters=0), check_blocks=True)
    acts = [t for t in res.trace if t[0] == "block" and t[1] == "activate"]
    assert len(acts) >= 1
    for _, name, fb, fa in (t for t in res.trace if t[0] == "block"):
        assert fa <= fb + 1e-9 * max(1.0, abs(fb)), (name, fb, fa)


@pytest.mark.parametrize("snr_db", [60.0, 80.0])
def test_noiseless_recovery(snr_db):
    """At very high SNR the estimator returns the true model order and frequencies."""
    inst = synth.make_instance(np.random.Generator(np.random.PCG64(99)), 64, 4, 2.0 / 64,
                               "paper", snr_db)
    res = estimate(inst.y, Params(L_mult=4.0))
    assert res.K == inst.K
    r, c = metrics.match(inst.theta, res.theta)
    err = np.max(synth.wrap_distance(inst.theta[r], res.theta[c]))
    # frequency CRB scales like sqrt(6/(N^3 SNR))/(2 pi); allow a wide margin
    crb = math.sqrt(6.0 / (64 ** 3 * 10 ** (snr_db / 10))) / (2 * math.pi)
    assert err < 50 * crb + 1e-12, (err, crb)
    assert abs(res.beta - inst.beta) < 0.5 * inst.beta + 1e-12


def test_zero_signal():
    """y = 0 has no noise floor to estimate: K = 0, beta = 0, no evaluation."""
    res = estimate(np.zeros(32, np.complex128))
    assert res.K == 0 and res.beta == 0.0 and res.evaluations == 0


def test_generator_snr_matches_oracle_ls_nmse():
    """Oracle-LS NMSE equals K/(N SNR) in expectation (Fig. snr dash-dotted curve:
    -31.0045 dB at 20 dB for N=128, K=10): pins the SNR definition of the generator."""
    fig = load_fig_snr()
    vals = [metrics.oracle_ls_nmse(synth.workload_paper_snr(i, 20.0)) for i in range(300)]
    db = 10 * math.log10(np.mean(vals))
    assert abs(db - fig[20.0]["ls"]) < 0.35, db
    assert abs(db - 10 * math.log10(10 / (128 * 100))) < 0.35


@pytest.mark.parametrize("snr_db,trials", [(20.0, 60), (12.0, 60)])
def test_accuracy_reproduces_fig_snr(snr_db, trials):
    """Statistical reproduction of the Superfast LSE curves of Fig. snr (N=128, K=10):
    BSR within 3 standard errors (floor 0.05), NMSE within 1.5 dB, CSR within 0.02."""
    ref = load_fig_snr()[snr_db]
    bs, cs, ns = [], [], []
    for i in range(trials):
        inst = synth.workload_paper_snr(i, snr_db)
        res = estimate(inst.y)
        bs.append(metrics.block_success(inst.theta, res.theta, inst.N))
        cs.append(metrics.component_success_rate(inst.theta, res.theta, inst.N))
        ns.append(metrics.nmse(inst.theta, inst.alpha, res.theta, res.alpha, inst.N))
    bsr = float(np.mean(bs))
    se = max(0.05, 3 * math.sqrt(ref["bsr"] * (1 - ref["bsr"]) / trials))
    assert abs(bsr - ref["bsr"]) <= se, (bsr, ref["bsr"])
    assert abs(float(np.mean(cs)) - ref["csr"]) <= 0.02
    nm_db = 10 * math.log10(float(np.mean(ns)))
    assert abs(nm_db - ref["nmse"]) <= 1.5, (nm_db, ref["nmse"])
