"""GPU parity of the full estimator (sfls_estimate, all steps in device kernels)
against the oracle estimator on the small workloads, plus batch properties."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1705_06073_amd as sf  # noqa: E402
from oracle.estimator import Params, estimate  # noqa: E402
from paper_1705_06073_amd import synth  # noqa: E402
from tests import metrics  # noqa: E402

# Frequencies after the final polish agree within 1e-9/N (FP64 path).
THETA_TOL = 1e-9


@pytest.fixture(scope="module")
def ctx():
    c = sf.Context(0)
    yield c
    c.close()


def compare(inst, g, o, label):
    N = inst.N
    print(f"[{label}] N={N} K_true={inst.K} gpu K={g.K} it={g.iterations} ev={g.evaluations} "
          f"st={g.status} | oracle K={o.K} it={o.iterations} ev={o.evaluations} st={o.status}",
          flush=True)
    assert g.status in (sf.SFLS_OK, sf.SFLS_NOTCONV)
    assert g.K == o.K, (g.K, o.K)
    if g.K:
        d = metrics.wrap_distance(g.theta, o.theta)
        print(f"   max |dtheta| N = {np.max(d) * N:.3e}", flush=True)
        assert np.max(d) < THETA_TOL / N, np.max(d) * N
        assert np.allclose(g.gamma, o.gamma, rtol=1e-6, atol=1e-12)
        assert np.allclose(g.alpha, o.alpha, rtol=1e-6, atol=1e-9)
    assert abs(g.beta - o.beta) <= 1e-8 * o.beta
    assert abs(g.objective - o.objective) <= 1e-8 * max(1.0, abs(o.objective))


@pytest.mark.parametrize("seed", range(4))
def test_n64_fp64_matches_oracle(ctx, seed):
    """N=64, K=3, separation 1/N, SNR 20 dB, grid 4N, FP64 throughout."""
    inst = synth.workload_n64(seed)
    p = sf.default_params(L_mult=4.0, precision=sf.SFLS_FP64)
    g = sf.estimate_batch(ctx, [inst.y], p)[0]
    o = estimate(inst.y, Params(L_mult=4.0))
    compare(inst, g, o, f"n64 seed {seed}")


@pytest.mark.parametrize("prec", [sf.SFLS_FP64, sf.SFLS_MIXED])
def test_n1024_matches_oracle(ctx, prec):
    """N=1024, K=20, c64 input, 20 dB amplitude range, SNR 15 dB, grid 8N."""
    inst = synth.workload_n1024(0)
    p = sf.default_params(precision=prec)
    g = sf.estimate_batch(ctx, [inst.y], p)[0]
    o = estimate(inst.y.astype(np.complex128), Params())
    compare(inst, g, o, f"n1024 prec {prec}")


def test_exact_activation_only(ctx):
    inst = synth.workload_n64(5)
    p = sf.default_params(L_mult=4.0, approx_max_iters=0)
    g = sf.estimate_batch(ctx, [inst.y], p)[0]
    o = estimate(inst.y, Params(L_mult=4.0, approx_max_iters=0))
    compare(inst, g, o, "n64 exact-only")


def test_zero_signal_and_capacity(ctx):
    y0 = np.zeros(64, np.complex128)
    r = sf.estimate_batch(ctx, [y0])[0]
    assert r.K == 0 and r.beta == 0.0 and r.status == sf.SFLS_OK
    inst = synth.workload_n64(1)
    r = sf.estimate_batch(ctx, [inst.y], sf.default_params(L_mult=4.0), kcap=1)[0]
    assert r.K <= 1 and r.status == sf.SFLS_ECAPACITY


def test_batch_results_equal_single_runs(ctx):
    """Each instance's result is the same alone and inside a ragged batch (bitwise)."""
    insts = [synth.workload_n64(0), synth.workload_paper_snr(3, 15.0),
             synth.workload_n64(2), synth.workload_paper_snr(4, 20.0, N=200, K=6)]
    ys = [i.y.astype(np.complex128) for i in insts]
    p = sf.default_params()
    batch = sf.estimate_batch(ctx, ys, p)
    for y, rb in zip(ys, batch):
        rs = sf.estimate_batch(ctx, [y], p)[0]
        assert rb.K == rs.K and rb.iterations == rs.iterations
        assert np.array_equal(rb.theta, rs.theta) and rb.beta == rs.beta


def test_uneven_batch_results_equal_single_runs(ctx):
    """A batch of uneven N in the superfast range runs its instances longest
    first; each instance's result is still bitwise the one it gets alone."""
    ns = [300, 2000, 512, 5000, 260, 2000]
    insts = [synth.workload_paper_snr(10 + i, 15.0, N=n, K=max(2, n // 100))
             for i, n in enumerate(ns)]
    ys = [i.y.astype(np.complex128) for i in insts]
    p = sf.default_params(precision=sf.SFLS_MIXED)
    batch = sf.estimate_batch(ctx, ys, p)
    for k, (y, rb) in enumerate(zip(ys, batch)):
        rs = sf.estimate_batch(ctx, [y], p)[0]
        print(f"instance {k}: N={len(y)} K={rb.K} evals={rb.evaluations}", flush=True)
        assert rb.status == rs.status and rb.K == rs.K and rb.iterations == rs.iterations
        assert np.array_equal(rb.theta, rs.theta) and np.array_equal(rb.alpha, rs.alpha)
        assert rb.beta == rs.beta and rb.objective == rs.objective


def test_paper_snr_workload_statistics(ctx):
    """The GPU estimator reproduces the Fig. snr Superfast LSE block success rate at
    20 dB (0.998 over 500 trials in the paper) on a 64-trial batch."""
    insts = [synth.workload_paper_snr(i, 20.0) for i in range(64)]
    res = sf.estimate_batch(ctx, [i.y for i in insts], sf.default_params())
    bsr = np.mean([metrics.block_success(i.theta, r.theta, i.N) for i, r in zip(insts, res)])
    assert bsr >= 0.93, bsr


def test_iteration_cap_reports_notconv(ctx):
    """max_outer = 1: the outer loop ends after one iteration without meeting
    the termination test of Sec. II-E, so both sides report NOTCONV; the
    estimate is still refined and returned, and equals the oracle's."""
    inst = synth.workload_n64(3)
    p = sf.default_params(L_mult=4.0, max_outer=1)
    g = sf.estimate_batch(ctx, [inst.y], p)[0]
    o = estimate(inst.y, Params(L_mult=4.0, max_outer=1))
    assert o.status == 1 and o.iterations == 1
    assert g.status == sf.SFLS_NOTCONV and g.iterations == 1
    compare(inst, g, o, "n64 max_outer=1")
