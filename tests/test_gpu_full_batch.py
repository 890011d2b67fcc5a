"""GPU checks at the full batched workload: 256 instances of N=4096,
K ~ Poisson(40), separation 1/N, alpha ~ CN(0,1), SNR ~ U[0,30] dB, grid 8N,
in one batched launch as the throughput benchmark runs it.  Every instance is
checked for properties that hold at any size; sampled instances are checked
against the dense oracle, which is affordable one instance at a time."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1705_06073_amd as sf  # noqa: E402
from oracle import numerics as nm  # noqa: E402
from paper_1705_06073_amd import synth  # noqa: E402
from tests.gpu_helpers import DEV, c2d, d2c, f64d, ragged, relerr, zeros_c  # noqa: E402

B = 256
N = 4096
EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def ctx():
    c = sf.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def workload():
    return [synth.workload_n4096(i) for i in range(B)]


def kappa(inst):
    """Bound on cond(C) at the true state: 1 + N sum(gamma) / beta."""
    return 1.0 + inst.N * float(np.sum(np.abs(inst.alpha) ** 2)) / inst.beta


def test_factor_full_batch(ctx, workload):
    """a1 + a3 (superfast Schur with refinement) for the 256 true states in one
    launch: pivots positive and rho_{N-1} = 1 everywhere; generator, pivots and
    ln|C| of sampled instances against the Cholesky factor.  The tolerance
    follows the error growth of a stable Toeplitz solver, cond(C) * eps."""
    ns = [N] * B
    n, off = ragged(ns)
    K = np.array([inst.K for inst in workload], np.int64)
    koff = np.concatenate([[0], np.cumsum(K)[:-1]]).astype(np.int64)
    th = f64d(np.concatenate([inst.theta for inst in workload] + [np.zeros(1)]))
    ga = f64d(np.concatenate([np.abs(inst.alpha) ** 2 for inst in workload] + [np.zeros(1)]))
    be = f64d([inst.beta for inst in workload])
    c = zeros_c(n.sum())
    sf.sfls_toeplitz_column(ctx, n, off, K, koff, th, ga, be, c)
    rho = zeros_c(n.sum())
    delta = torch.zeros(int(n.sum()), dtype=torch.float64, device=DEV)
    logdet = torch.zeros(B, dtype=torch.float64, device=DEV)
    status = torch.zeros(B, dtype=torch.int32, device=DEV)
    failed = torch.zeros(B, dtype=torch.int64, device=DEV)
    print(f"[full factor] B={B} N={N}", flush=True)
    sf.sfls_factor(ctx, n, off, c, rho, delta, logdet, status, failed)
    torch.cuda.synchronize()
    st, fl = status.cpu().numpy(), failed.cpu().numpy()
    assert (st == 0).all() and (fl == -1).all()
    rg, dg, lg = d2c(rho), delta.cpu().numpy(), logdet.cpu().numpy()
    assert (dg > 0).all() and np.isfinite(lg).all()
    assert np.max(np.abs(rg[off + N - 1] - 1.0)) < 1e-12
    cg = d2c(c)
    for b in (0, 77, 191, 255):
        inst = workload[b]
        tol = max(1e-12, 100.0 * kappa(inst) * EPS)
        col = nm.toeplitz_column(inst.theta, np.abs(inst.alpha) ** 2, inst.beta, N)
        sl = slice(off[b], off[b] + N)
        assert relerr(cg[sl], col) < 1e-13, b
        F = nm.DenseFactor(nm.dense_from_column(col))
        r_ref, _ = F.generator()
        er, ed = relerr(rg[sl], r_ref), relerr(dg[sl], F.delta)
        el = abs(lg[b] - F.logdet) / max(1.0, abs(F.logdet))
        print(f"   b={b} K={inst.K} kappa={kappa(inst):.2e} tol={tol:.1e} rho {er:.2e} "
              f"delta {ed:.2e} logdet {el:.2e}", flush=True)
        assert er < tol and ed < tol and el < max(1e-9, tol), b


def test_estimate_full_batch(ctx, workload):
    """sfls_estimate on the whole batch (FP64 recursion, FP32 grid) in one call.
    All instances: a valid status, theta sorted in [0, 1), gamma > 0, beta > 0,
    a finite objective.  Sampled instances (and the one that needed the most
    evaluations): the dense oracle evaluated at the returned point reproduces
    the returned objective and alpha = gamma * A^H C^{-1} y."""
    p = sf.default_params(precision=sf.SFLS_MIXED)
    print(f"[full estimate] B={B} N={N}", flush=True)
    res = sf.estimate_batch(ctx, [inst.y for inst in workload], p, kcap=256)
    for b, r in enumerate(res):
        assert r.status in (sf.SFLS_OK, sf.SFLS_NOTCONV), (b, r.status)
        assert 0 < r.K <= 256 and r.evaluations >= 1, b
        assert np.all(r.theta >= 0.0) and np.all(r.theta < 1.0) and np.all(np.diff(r.theta) >= 0)
        assert np.all(r.gamma > 0.0) and r.beta > 0.0 and math.isfinite(r.objective), b
    worst = int(np.argmax([r.evaluations for r in res]))
    print(f"   evaluations: mean {np.mean([r.evaluations for r in res]):.1f}, "
          f"max {res[worst].evaluations} (instance {worst})", flush=True)
    for b in sorted({0, 100, 200, worst}):
        inst, r = workload[b], res[b]
        ev = nm.Evaluation(inst.y, r.theta, r.gamma, r.beta)
        fo = ev.f(r.K, r.zeta)
        ef = abs(r.objective - fo) / max(1.0, abs(fo))
        a_ref = r.gamma * ev.act["q"]
        ea = np.max(np.abs(r.alpha - a_ref) / (1e-6 * np.abs(a_ref) + 1e-9))
        print(f"   b={b} K={r.K} (true {inst.K}) ev={r.evaluations} objective rel {ef:.2e} "
              f"alpha err/tol {ea:.2e}", flush=True)
        assert ef <= 1e-8, b
        assert ea <= 1.0, b
