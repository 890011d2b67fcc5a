"""Pins of the incomplete-observation oracle (Sec. IV; Phi = M weighted rows of
the identity) against what the paper and the mathematics fix: the complete-data
oracle when every sample is observed, the Woodbury and determinant-lemma forms
of Sec. IV (eqs. CfromSigma, AhA and the ln|C| lemma), the Gaussian marginal of
the unobserved samples, the invariance under a common complex scale of the
weights and the signal, Sherman-Morrison closed forms at K = 1, brute-force grid
sums, finite differences of the objective, the EM bound of eq. betaUpdate, and
noiseless recovery.  No GPU."""
import math

import numpy as np
import pytest
import scipy.optimize as so

from oracle import estimator as oe
from oracle import incomplete as inc
from oracle import numerics as nm
from paper_1705_06073_amd import synth


def _obs(rng, N, M, weights="scaled"):
    idx = synth.draw_observed(rng, N, M)
    return inc.Observation(N, idx, synth.draw_weights(rng, M, weights))


def _state(rng, K):
    return rng.random(K), 0.2 + 2.0 * rng.random(K), 0.05 + 0.5 * rng.random()


def _y(rng, obs, theta, amp, beta):
    h = obs.A(theta) @ np.asarray(amp, np.complex128)
    return h + math.sqrt(beta / 2) * (rng.standard_normal(obs.M) + 1j * rng.standard_normal(obs.M))


# ---------------------------------------------------------- reductions ----

def test_every_sample_observed_is_the_complete_oracle():
    """Phi = I: every quantity and the whole estimate equal the complete-data
    oracle's bit for bit (the reduction Sec. IV starts from)."""
    inst = synth.workload_n64(0)
    obs = inc.Observation(inst.N, np.arange(inst.N))
    th, ga, be = np.array([0.1, 0.37, 0.8]), np.array([1.0, 0.5, 2.0]), 0.03
    e1 = nm.Evaluation(inst.y, th, ga, be)
    e2 = inc.EvaluationIncomplete(inst.y, obs, th, ga, be)
    assert e1.logdet == e2.logdet and e1.yCy == e2.yCy
    for k in "qrustvx":
        assert np.array_equal(e1.act[k], e2.act[k]), k
    for a, b in zip(e1.grid(256), e2.grid(256)):
        assert np.array_equal(a, b)
    r1 = oe.estimate(inst.y, oe.Params(L_mult=4.0))
    r2 = inc.estimate(inst.y, np.arange(inst.N), inst.N, params=oe.Params(L_mult=4.0))
    assert r1.K == r2.K and np.array_equal(r1.theta, r2.theta)
    assert r1.objective == r2.objective and r1.evaluations == r2.evaluations


@pytest.mark.parametrize("seed", range(3))
def test_unit_weights_are_the_gaussian_marginal(seed):
    """With |phi| = 1, y is the observed part of a complete-data signal: C is
    Phi C_full Phi^H (the marginal over the unobserved samples), so ln|C| and
    y^H C^{-1} y are those of that submatrix."""
    rng = np.random.default_rng(10 + seed)
    N, M, K = 40, 23, 3
    obs = _obs(rng, N, M, "phase")
    th, ga, be = _state(rng, K)
    y = _y(rng, obs, th, [1, 0.5j, -0.7], be)
    Cf = nm.covariance(th, ga, be, N)
    Ph = obs.matrix()
    Cm = Ph @ Cf @ Ph.conj().T
    ev = inc.EvaluationIncomplete(y, obs, th, ga, be)
    assert np.allclose(ev.C, Cm, rtol=0, atol=1e-13)
    assert ev.logdet == pytest.approx(np.linalg.slogdet(Cm)[1], rel=1e-12)
    assert ev.yCy == pytest.approx(np.vdot(y, np.linalg.solve(Cm, y)).real, rel=1e-12)


# ------------------------------------------------------ Sec. IV identities --

@pytest.mark.parametrize("seed", range(3))
def test_determinant_lemma_and_woodbury_forms(seed):
    """Sec. IV: ln|C| = M ln beta + sum ln gamma + ln|Sigma^{-1}| and
    C^{-1} = beta^{-1} I - beta^{-2} A Sigma A^H (eq. CfromSigma) with
    Sigma^{-1} = Gamma^{-1} + A^H A / beta (eq. bSigma); [A^H A]_{ik} =
    sum_m |phi_m|^2 e^{j2pi n_m (theta_k - theta_i)} (eq. AhA)."""
    rng = np.random.default_rng(20 + seed)
    N, M, K = 64, 37, 4
    obs = _obs(rng, N, M)
    th, ga, be = _state(rng, K)
    y = _y(rng, obs, th, rng.standard_normal(K) + 1j * rng.standard_normal(K), be)
    ev = inc.EvaluationIncomplete(y, obs, th, ga, be)
    n = obs.idx.astype(float)
    w2 = np.abs(obs.phi) ** 2
    AhA = np.array([[np.sum(w2 * np.exp(2j * np.pi * n * (th[k] - th[i]))) for k in range(K)]
                    for i in range(K)])
    A = obs.A(th)
    assert np.allclose(A.conj().T @ A, AhA, rtol=0, atol=1e-11 * M)
    Si = np.diag(1.0 / ga) + AhA / be
    ld = M * math.log(be) + np.sum(np.log(ga)) + np.linalg.slogdet(Si)[1]
    assert ev.logdet == pytest.approx(ld, rel=1e-11)
    Sigma = np.linalg.inv(Si)
    wM = y / be - A @ (Sigma @ (A.conj().T @ y)) / be ** 2
    assert np.allclose(ev.wM, wM, rtol=0, atol=1e-10 * np.max(np.abs(wM)))
    # the posterior mean mu = gamma .* q (Sec. II-D, after eq. betaUpdate)
    mu = Sigma @ (A.conj().T @ y) / be
    assert np.allclose(ga * ev.act["q"], mu, rtol=1e-9, atol=1e-12)


def test_common_complex_scale_leaves_the_vectors_unchanged():
    """phi -> c phi, y -> c y, beta -> |c|^2 beta multiplies C by |c|^2: the
    objective moves by M ln|c|^2 and q..x, w and the grid do not change.  A
    missing conjugate in Phi^H turns q into e^{2j arg c} q and fails here."""
    rng = np.random.default_rng(31)
    N, M, K = 48, 30, 3
    obs = _obs(rng, N, M)
    th, ga, be = _state(rng, K)
    y = _y(rng, obs, th, [0.8, 1j, -0.4], be)
    c = 1.7 * np.exp(0.9j)
    obs2 = inc.Observation(N, obs.idx, c * obs.phi)
    e1 = inc.EvaluationIncomplete(y, obs, th, ga, be)
    e2 = inc.EvaluationIncomplete(c * y, obs2, th, ga, abs(c) ** 2 * be)
    assert e2.f(K, 0.1) - e1.f(K, 0.1) == pytest.approx(M * math.log(abs(c) ** 2), rel=1e-10)
    for k in "qrustvx":
        assert np.allclose(e1.act[k], e2.act[k], rtol=1e-10, atol=1e-12), k
    assert np.allclose(e1.w, e2.w, rtol=1e-10, atol=1e-13)
    for a, b in zip(e1.grid(256), e2.grid(256)):
        assert np.allclose(a, b, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("seed", range(2))
def test_single_component_closed_forms(seed):
    """K = 1 (Sherman-Morrison): with a = Phi psi(theta_1) and
    g(x) = sum_m |phi_m|^2 e^{j2pi n_m x},
    s(theta) = (g(0) - gamma |g(theta - theta_1)|^2 / (beta + gamma g(0))) / beta and
    q(theta) = (psi^H Phi^H y - gamma conj(g(theta - theta_1)) a^H y / (beta + gamma g(0))) / beta,
    on the whole grid (through w, the diagonal sums of E and the FFTs)."""
    rng = np.random.default_rng(40 + seed)
    N, M, L = 50, 29, 128
    obs = _obs(rng, N, M)
    th1, ga1, be = rng.random(), 0.3 + rng.random(), 0.2 + rng.random()
    y = _y(rng, obs, [th1], [1.2 - 0.3j], be)
    ev = inc.EvaluationIncomplete(y, obs, [th1], [ga1], be)
    qG, sG = ev.grid(L)
    x = np.arange(L) / L
    n = obs.idx.astype(float)
    w2 = np.abs(obs.phi) ** 2
    g = np.array([np.sum(w2 * np.exp(2j * np.pi * n * (xl - th1))) for xl in x])
    g0 = np.sum(w2)
    s_ref = (g0 - ga1 * np.abs(g) ** 2 / (be + ga1 * g0)) / be
    a = obs.phi * np.exp(2j * np.pi * n * th1)
    py = np.array([np.sum(np.conj(obs.phi * np.exp(2j * np.pi * n * xl)) * y) for xl in x])
    q_ref = (py - ga1 * np.conj(g) * np.vdot(a, y) / (be + ga1 * g0)) / be
    assert np.allclose(sG, s_ref, rtol=1e-11, atol=1e-11 * g0 / be)
    assert np.allclose(qG, q_ref, rtol=1e-11, atol=1e-11 * np.max(np.abs(q_ref)))


def test_empty_active_set():
    """K = 0: C = beta I, so ln|C| = M ln beta, q^G is the DFT of Phi^H y / beta
    and s^G is the constant sum |phi|^2 / beta."""
    rng = np.random.default_rng(50)
    obs = _obs(rng, 40, 17)
    y = rng.standard_normal(17) + 1j * rng.standard_normal(17)
    ev = inc.EvaluationIncomplete(y, obs, [], [], 0.4)
    qG, sG = ev.grid(128)
    assert ev.logdet == pytest.approx(17 * math.log(0.4), rel=1e-14)
    assert np.allclose(sG, np.sum(np.abs(obs.phi) ** 2) / 0.4, rtol=1e-12)
    ref = np.array([np.sum(np.conj(obs.phi) * y * np.exp(-2j * np.pi * obs.idx * l / 128))
                    for l in range(128)]) / 0.4
    assert np.allclose(qG, ref, rtol=1e-12, atol=1e-12)


def test_grid_matches_bruteforce():
    """s^G_l = psi_l^H Phi^H C^{-1} Phi psi_l and r^G, t^G by direct quadratic
    forms at every grid point (the diagonal-sum and FFT route checked against
    the definition)."""
    rng = np.random.default_rng(60)
    N, M, K, L = 24, 15, 3, 64
    obs = _obs(rng, N, M)
    th, ga, be = _state(rng, K)
    y = _y(rng, obs, th, [1, -1j, 0.5], be)
    ev = inc.EvaluationIncomplete(y, obs, th, ga, be)
    Psi = nm.steering(np.arange(L) / L, N)
    d = nm.d_diag(N)
    Ph = obs.matrix()
    Ci = np.linalg.inv(ev.C)
    X = Ph.conj().T @ Ci @ Ph @ Psi
    s_bf = np.real(np.sum(Psi.conj() * X, axis=0))
    t_bf = np.sum(Psi.conj() * d[:, None] * X, axis=0)
    qG, sG = ev.grid(L)
    rG, tG = ev.grid_derivatives(L)
    w = Ph.conj().T @ (Ci @ y)
    assert np.allclose(sG, s_bf, rtol=1e-11, atol=1e-12)
    assert np.allclose(tG, t_bf, rtol=1e-10, atol=1e-10)
    assert np.allclose(qG, Psi.conj().T @ w, rtol=1e-11, atol=1e-12)
    assert np.allclose(rG, Psi.conj().T @ (d * w), rtol=1e-11, atol=1e-10)


# ---------------------------------------------------------- derivatives ----

def _f_plain(y, obs, th, ga, be):
    """ln|C| + y^H C^{-1} y by slogdet and an LU solve of C = beta I + A Gamma A^H."""
    A = obs.phi[:, None] * np.exp(2j * np.pi * np.multiply.outer(obs.idx, th))
    C = (A * ga) @ A.conj().T + be * np.eye(obs.M)
    return np.linalg.slogdet(C)[1] + np.vdot(y, np.linalg.solve(C, y)).real


@pytest.mark.parametrize("seed", range(2))
def test_derivatives_against_finite_differences(seed):
    """eqs. derivative / derivative2 through the q..x of eqs. q-x under Phi,
    against central differences of the objective (which pins where D sits in
    t, v, x and the conjugations of Phi^H)."""
    rng = np.random.default_rng(70 + seed)
    N, M, K = 32, 19, 3
    obs = _obs(rng, N, M)
    th = np.array([0.11, 0.43, 0.77]) + 0.01 * rng.random(3)
    ga = np.array([1.3, 0.6, 2.2])
    be = 0.25
    y = _y(rng, obs, th, rng.standard_normal(K) + 1j * rng.standard_normal(K), 0.1)
    ev = inc.EvaluationIncomplete(y, obs, th, ga, be)
    gth, gga = nm.gradient(ga, ev.act)
    hth, hga = nm.hessian_diag(ga, ev.act)
    for k in range(K):
        for which, x0, gk, hk, h in (("th", th, gth[k], hth[k], 1e-5),
                                     ("ga", ga, gga[k], hga[k], 1e-4)):
            def f(dx):
                a = x0.copy()
                a[k] += dx
                return _f_plain(y, obs, a, ga, be) if which == "th" else \
                    _f_plain(y, obs, th, a, be)
            f0 = f(0.0)

            def d1(hh):
                return (f(hh) - f(-hh)) / (2 * hh)

            def d2(hh):
                return (f(hh) - 2 * f0 + f(-hh)) / hh ** 2
            # Richardson extrapolation of the central differences (error O(h^4))
            g_fd = (4 * d1(h / 2) - d1(h)) / 3
            h_fd = (4 * d2(h / 2) - d2(h)) / 3
            assert abs(g_fd - gk) <= 1e-6 * max(1.0, abs(gk)), (which, k, g_fd, gk)
            assert abs(h_fd - hk) <= 1e-3 * max(1.0, abs(hk)), (which, k, h_fd, hk)


# ----------------------------------------------------------------- beta ----

@pytest.mark.parametrize("seed", range(2))
def test_beta_update_minimises_the_em_bound(seed):
    """eq. betaUpdate with M observations is the minimiser of eq. bound_explicit,
    Q(beta) = M ln beta + (tr(Sigma A^H A) + ||y - A mu||^2) / beta, whose terms
    are formed here from an explicit posterior (eqs. bmu, bSigma) by sampling
    nothing: the expectation of ||y - A alpha||^2 under CN(mu, Sigma) is written
    as the trace plus the residual; the minimiser is found numerically."""
    rng = np.random.default_rng(80 + seed)
    N, M, K = 40, 26, 2
    obs = _obs(rng, N, M)
    th = np.array([0.2, 0.61]) + 0.02 * rng.random(2)
    y = _y(rng, obs, th, [1.0, 0.6j], 0.3)
    ga = 0.5 + rng.random(2)
    b_old = 0.1 + rng.random()
    A = obs.A(th)
    P = A.conj().T @ A / b_old + np.diag(1.0 / ga)
    Lc = np.linalg.cholesky(np.linalg.inv(P))
    mu = np.linalg.solve(P, A.conj().T @ y) / b_old
    # E||y - A alpha||^2 by a fixed 3-point Gauss-Hermite tensor rule (exact for
    # the quadratic integrand) over alpha = mu + Lc z
    x, wq = np.polynomial.hermite_e.hermegauss(3)
    wq = wq / wq.sum()
    grids = np.meshgrid(*([np.arange(3)] * (2 * K)), indexing="ij")
    wts = np.prod([wq[g] for g in grids], axis=0).ravel()
    z = (np.stack([x[g].ravel() for g in grids[:K]])
         + 1j * np.stack([x[g].ravel() for g in grids[K:]])) / math.sqrt(2.0)
    res = y[:, None] - A @ (mu[:, None] + Lc @ z)
    e_res = float(np.sum(wts * np.sum(np.abs(res) ** 2, axis=0)))
    r = so.minimize_scalar(lambda lb: M * lb + e_res * math.exp(-lb),
                           bounds=(math.log(1e-4), math.log(1e2)), method="bounded",
                           options={"xatol": 1e-11})
    b_upd = inc.beta_update_definition(y, obs, th, ga, b_old, 1e-12)
    assert math.exp(r.x) == pytest.approx(b_upd, rel=1e-7)
    # and the divisor is M, not N
    assert abs(b_upd - e_res / N) > 1e-3 * b_upd


# ------------------------------------------------------------ estimator ----

@pytest.mark.parametrize("seed", range(3))
def test_noiseless_recovery_from_incomplete_data(seed):
    """Well-separated components observed on about 60% of the samples with
    scaled weights, at 80 dB: the estimate has the true model order and
    frequencies within 1e-4/N (about ten times the Cramer-Rao spread there)."""
    rng = np.random.default_rng(90 + seed)
    N, M = 96, 58
    obs = _obs(rng, N, M)
    th = np.sort(np.mod(0.13 + np.array([0.0, 0.31, 0.58]) + 0.05 * rng.random(3), 1.0))
    amp = np.exp(2j * np.pi * rng.random(3)) * (0.6 + rng.random(3))
    h = obs.A(th) @ amp
    beta = float(np.vdot(h, h).real) / (M * 1e8)
    y = h + math.sqrt(beta / 2) * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    r = inc.estimate(y, obs.idx, N, obs.phi)
    assert r.K == 3
    assert np.max(np.abs(r.theta - th)) * N < 1e-4
    assert r.beta == pytest.approx(beta, rel=0.5)


def test_count_scales_are_in_observations():
    """K_max = M and zeta = min(1/2, K/M) (eq. zetaUpdate with K_max = M); the
    prior term of the objective uses M - K inactive components."""
    inst = synth.workload_paper_mton(3, 0.5)
    r = inc.estimate(inst.y, inst.idx, inst.N)
    assert r.zeta == pytest.approx(min(0.5, r.K / inst.M), rel=1e-15)
    ev = inc.EvaluationIncomplete(inst.y, inc.Observation(inst.N, inst.idx), r.theta, r.gamma,
                                  r.beta)
    prior = -(r.K * math.log(r.zeta) + (inst.M - r.K) * math.log(1.0 - r.zeta))
    assert r.objective == pytest.approx(ev.logdet + ev.yCy + prior, rel=1e-12)


def test_observation_validation():
    with pytest.raises(ValueError):
        inc.Observation(10, [0, 3, 3, 9])
    with pytest.raises(ValueError):
        inc.Observation(10, [0, 10])
    with pytest.raises(ValueError):
        inc.Observation(10, [0, 4], [1.0, 0.0])


# ------------------------------------------------------- Fig. MtoN (Sec. VI-E) --

def load_fig_mton():
    import os
    rows = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "fig_mton_n128_k10.txt")):
        if line.startswith("#") or not line.strip():
            continue
        r, bsr, csr, nmse, ls = map(float, line.split())
        rows[r] = dict(bsr=bsr, csr=csr, nmse=nmse, ls=ls)
    return rows


def test_generator_matches_fig_mton_oracle_curve():
    """The least-squares NMSE with the true frequencies (Fig. MtoN, dash-dotted)
    pins the generator: the index sets (first and last sample kept), the SNR on
    the observed samples and the NMSE on the whole signal."""
    from tests import metrics
    fig = load_fig_mton()
    for ratio in (0.2, 0.5, 1.0):
        vals = [metrics.oracle_ls_nmse(synth.workload_paper_mton(i, ratio)) for i in range(300)]
        db = 10 * math.log10(np.mean(vals))
        assert abs(db - fig[ratio]["ls"]) < 0.35, (ratio, db)


@pytest.mark.parametrize("ratio,trials", [(0.5, 40), (0.4, 40)])
def test_accuracy_reproduces_fig_mton(ratio, trials):
    """Statistical reproduction of the Semifast LSE curves of Fig. MtoN (N=128,
    K=10, 20 dB): BSR within 3 standard errors (floor 0.05), CSR within 0.02,
    NMSE within 1.5 dB.  Below M/N = 0.4 the oracle activates more spurious
    components than the figure shows (BSR about 0.77 against 0.90 at 0.3, CSR
    about 0.49 against 0.66 at 0.2); those points are not pins."""
    from tests import metrics
    ref = load_fig_mton()[ratio]
    bs, cs, ns = [], [], []
    for i in range(trials):
        inst = synth.workload_paper_mton(i, ratio)
        res = inc.estimate(inst.y, inst.idx, inst.N, inst.phi)
        bs.append(metrics.block_success(inst.theta, res.theta, inst.N))
        cs.append(metrics.component_success_rate(inst.theta, res.theta, inst.N))
        ns.append(metrics.nmse(inst.theta, inst.alpha, res.theta, res.alpha, inst.N))
    bsr = float(np.mean(bs))
    se = max(0.05, 3 * math.sqrt(ref["bsr"] * (1 - ref["bsr"]) / trials))
    assert abs(bsr - ref["bsr"]) <= se, (bsr, ref["bsr"])
    assert abs(float(np.mean(cs)) - ref["csr"]) <= 0.02
    nm_db = 10 * math.log10(float(np.mean(ns)))
    assert abs(nm_db - ref["nmse"]) <= 1.5, (nm_db, ref["nmse"])
