"""Pins of the dense oracle numerics against closed forms, brute force and
independent identities (no GPU).  Each test names what fixes the value."""
import math

import numpy as np
import pytest
import scipy.optimize as so

from oracle import numerics as nm


def rand_state(rng, N, K, beta=0.3):
    theta = rng.random(K)
    gamma = 0.2 + rng.random(K) * 2.0
    return theta, gamma, beta


def rand_y(rng, N):
    return (rng.standard_normal(N) + 1j * rng.standard_normal(N)) / math.sqrt(2)


# ---------------------------------------------------------------- factor ----

@pytest.mark.parametrize("N,K", [(1, 1), (2, 1), (5, 2), (16, 3), (40, 6)])
def test_gohberg_semencul_reconstructs_inverse(N, K):
    """C^{-1} = delta_{N-1}^{-1}(T1^H T1 - T0 T0^H) with [T0]_{ik} = rho_{i-k-1},
    [T1]_{ik} = rho_{N-1+i-k} (Sec. III, eq. gohberg-semencul), against numpy's inverse."""
    rng = np.random.default_rng(N * 100 + K)
    th, ga, be = rand_state(rng, N, K)
    C = nm.covariance(th, ga, be, N)
    rho, dN = nm.DenseFactor(C).generator()

    def r(i):
        return rho[i] if 0 <= i <= N - 1 else 0.0

    T0 = np.array([[r(i - k - 1) for k in range(N)] for i in range(N)], dtype=complex)
    T1 = np.array([[r(N - 1 + i - k) for k in range(N)] for i in range(N)], dtype=complex)
    Ci = (T1.conj().T @ T1 - T0 @ T0.conj().T) / dN
    ref = np.linalg.inv(C)
    assert np.max(np.abs(Ci - ref)) <= 1e-10 * np.max(np.abs(ref))
    assert abs(rho[-1] - 1.0) < 1e-14
    # rho = delta_{N-1} C^{-1} e_{N-1}
    assert np.allclose(rho, dN * ref[:, -1], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("N,K", [(3, 1), (12, 2), (33, 4)])
def test_pivots_are_ratios_of_leading_minors(N, K):
    """delta_n = det C_{n+1} / det C_n (LDL^H pivots), ln|C| = sum ln delta (Sec. III-A)."""
    rng = np.random.default_rng(7 + N)
    th, ga, be = rand_state(rng, N, K)
    C = nm.covariance(th, ga, be, N)
    F = nm.DenseFactor(C)
    ld = [0.0] + [np.linalg.slogdet(C[:m, :m])[1] for m in range(1, N + 1)]
    ref = np.exp(np.diff(ld))
    assert np.allclose(F.delta, ref, rtol=1e-10)
    assert abs(F.logdet - np.linalg.slogdet(C)[1]) < 1e-9 * max(1.0, abs(F.logdet))


def test_covariance_column_matches_dense_toeplitz():
    """C is Hermitian Toeplitz (Sec. III): rebuilding it from its first column is exact."""
    rng = np.random.default_rng(3)
    th, ga, be = rand_state(rng, 20, 4)
    C = nm.covariance(th, ga, be, 20)
    c = nm.toeplitz_column(th, ga, be, 20)
    assert np.allclose(C, nm.dense_from_column(c), atol=1e-12)
    assert np.allclose(C[:, 0], c, atol=1e-13)


def test_empty_active_set_closed_forms():
    """K = 0: C = beta I, so rho = e_{N-1}, delta = beta, q^G = FFT(y)/beta, s^G = N/beta."""
    rng = np.random.default_rng(11)
    N, L, beta = 24, 64, 0.7
    y = rand_y(rng, N)
    ev = nm.Evaluation(y, [], [], beta)
    rho, dN = ev.F.generator()
    e = np.zeros(N)
    e[-1] = 1
    assert np.allclose(rho, e, atol=1e-15) and abs(dN - beta) < 1e-14
    assert np.allclose(ev.F.delta, beta)
    qG, sG = ev.grid(L)
    ref = np.array([np.sum(y * np.exp(-2j * np.pi * np.arange(N) * l / L)) for l in range(L)]) / beta
    assert np.allclose(qG, ref, atol=1e-12)
    assert np.allclose(sG, N / beta, rtol=1e-13)


def test_single_component_closed_forms():
    """K = 1 by Sherman-Morrison: delta_n = beta(beta+(n+1)gamma)/(beta+n gamma);
    rho_i = -gamma e^{j2pi(i-N+1)theta}/(beta+(N-1)gamma), i < N-1;
    s^G(theta) = N/beta - gamma |D_N(theta-theta1)|^2 / (beta(beta+N gamma))."""
    N, L, th1, g, b = 32, 128, 0.2137, 1.7, 0.4
    ev = nm.Evaluation(np.ones(N), [th1], [g], b)
    n = np.arange(N)
    assert np.allclose(ev.F.delta, b * (b + (n + 1) * g) / (b + n * g), rtol=1e-12)
    rho, dN = ev.F.generator()
    ref = -g * np.exp(2j * np.pi * (n - N + 1) * th1) / (b + (N - 1) * g)
    ref[-1] = 1.0
    assert np.allclose(rho, ref, atol=1e-13)
    _, sG = ev.grid(L)
    grid = np.arange(L) / L
    DN = np.array([np.sum(np.exp(2j * np.pi * n * (t - th1))) for t in grid])
    assert np.allclose(sG, N / b - g * np.abs(DN) ** 2 / (b * (b + N * g)), rtol=1e-11)


# ----------------------------------------------------------------- omegas ---

def app_b_omegas(rho, dN):
    """Appendix B closed forms (c_s, c_t, c_v with the garbled 'M' read as N, c_x)."""
    N = len(rho)
    out = {k: np.zeros(2 * N - 1, complex) for k in "stvx"}
    qb = np.arange(N, dtype=float)
    for i in range(-(N - 1), N):
        rq = rho
        rqi = np.array([rho[q + i] if 0 <= q + i < N else 0.0 for q in range(N)])
        prod = rq * np.conj(rqi)
        cs = 2 - N + i + 2 * qb
        ct = -qb * (qb + i) + i * (N - (3 + i) / 2) + qb ** 2 + (N - 1) * (qb - (N - 2) / 2)
        cv = (qb * (qb + i) ** 2 + (3 * qb - 2 * N * qb - qb ** 2) * (qb + i) + 2 / 3 * qb ** 3
              + (N - 1) * qb ** 2 + (N ** 2 - 3 * N + 7 / 3) * qb + 1.5 * (i - N) ** 2
              + (i ** 3 - N ** 3) / 3 + (13 / 6 - N * i) * (i - N) + 1)
        cx = ((qb ** 2 + 2 * qb - N * qb) * (qb + i) - qb ** 3 / 3 + (N ** 2 - 3 * N + 7 / 3) * qb
              - i ** 3 / 6 + (3 * N ** 2 - 9 * N + 7) / 6 * i - N ** 3 / 3 + 1.5 * N ** 2
              - 13 / 6 * N + 1)
        j = i + N - 1
        out["s"][j] = np.sum(cs * prod) / dN
        out["t"][j] = 2 * np.pi * np.sum(ct * prod) / dN
        out["v"][j] = 4 * np.pi ** 2 * np.sum(cv * prod) / dN
        out["x"][j] = 4 * np.pi ** 2 * np.sum(cx * prod) / dN
    return out


@pytest.mark.parametrize("N,K", [(2, 1), (9, 2), (24, 4)])
def test_diagonal_sums_match_appendix_b(N, K):
    """Dense diagonal sums of C^{-1}, DC^{-1}, D^2C^{-1}, DC^{-1}D (eqs. omega_*) equal the
    Appendix-B polynomials applied to the Gohberg-Semencul generator, for every lag
    i = -(N-1)..N-1 (the garbled 'M' in c_v read as N)."""
    rng = np.random.default_rng(50 + N)
    th, ga, be = rand_state(rng, N, K)
    F = nm.DenseFactor(nm.covariance(th, ga, be, N))
    om = dict(zip("stvx", nm.omegas(F)))
    ref = app_b_omegas(*F.generator())
    for k in "stvx":
        assert np.max(np.abs(om[k] - ref[k])) <= 1e-9 * np.max(np.abs(om[k])), k
    # omega_s is Hermitian in the lag (C^{-1} is Hermitian)
    assert np.allclose(om["s"][::-1], np.conj(om["s"]), atol=1e-12 * np.max(np.abs(om["s"])))


def test_omega_v_is_not_hermitian_in_the_lag():
    """Reading of Appendix B: the stated omega_v(-i) = omega_v(i)^* does not hold for the
    diagonal sums of D^2 C^{-1} as defined (eq. omega_v), while the c_v polynomial itself is
    valid for negative lags too; v_k therefore uses omega_v over all lags.  Here N = 2, K = 1:
    omega_v(1) = 0 (only row 0, weight 0) but omega_v(-1) = (2pi)^2 [C^{-1}]_{1,0} != 0."""
    F = nm.DenseFactor(nm.covariance([0.3], [1.0], 0.5, 2))
    om_v = nm.omegas(F)[2]
    assert abs(om_v[2]) < 1e-14
    assert abs(om_v[0] - (2 * np.pi) ** 2 * F.inverse()[1, 0]) < 1e-12
    assert abs(om_v[0]) > 1.0


def test_grid_matches_bruteforce():
    """q^G and s^G via FFT equal direct psi^H C^{-1} y and psi^H C^{-1} psi on the grid."""
    rng = np.random.default_rng(5)
    N, L = 12, 48
    th, ga, be = rand_state(rng, N, 3)
    y = rand_y(rng, N)
    ev = nm.Evaluation(y, th, ga, be)
    qG, sG = ev.grid(L)
    Psi = nm.steering(np.arange(L) / L, N)
    assert np.allclose(qG, Psi.conj().T @ ev.w, atol=1e-12)
    assert np.allclose(sG, nm.grid_s_bruteforce(ev.F, L), rtol=1e-12)
    # s at an off-grid point from the diagonal sums (eq. sFourier) vs the quadratic form
    t0 = 0.3127
    p = nm.steering([t0], N)[:, 0]
    assert abs(nm.s_at(ev.omega[0], [t0])[0] - np.vdot(p, ev.F.solve(p)).real) < 1e-11


def test_grid_derivatives_match_bruteforce():
    """r^G and t^G via FFTs equal the direct products psi^H D C^{-1} y and
    psi^H D C^{-1} psi on the grid (numpy inverse), including an odd L not
    tied to N; t^G is complex and differs from its conjugate-symmetric part."""
    rng = np.random.default_rng(15)
    for N, L in ((12, 48), (9, 17)):
        th, ga, be = rand_state(rng, N, 3)
        y = rand_y(rng, N)
        ev = nm.Evaluation(y, th, ga, be)
        rG, tG = ev.grid_derivatives(L)
        Psi = nm.steering(np.arange(L) / L, N)
        D = np.diag(nm.d_diag(N))
        Ci = np.linalg.inv(ev.C)
        assert np.allclose(rG, Psi.conj().T @ D @ Ci @ y, rtol=1e-12, atol=1e-11)
        t_ref = np.sum(Psi.conj() * (D @ Ci @ Psi), axis=0)
        assert np.allclose(tG, t_ref, rtol=1e-12, atol=1e-10)
        assert np.max(np.abs(tG.imag)) > 1e-3 * np.max(np.abs(tG))
        # at the grid points that are active frequencies, r and t are eqs. r and t
        Kg = nm.active_vectors(ev.F, ev.w, np.arange(L)[:3] / L)
        assert np.allclose(rG[:3], Kg["r"], atol=1e-10) and np.allclose(tG[:3], Kg["t"], atol=1e-10)


def test_active_vectors_match_definitions_via_inverse():
    """q..x against the plain matrix products with numpy's inverse (eqs. q-x)."""
    rng = np.random.default_rng(9)
    N = 20
    th, ga, be = rand_state(rng, N, 3)
    y = rand_y(rng, N)
    ev = nm.Evaluation(y, th, ga, be)
    Ci = np.linalg.inv(ev.C)
    P = nm.steering(th, N)
    D = np.diag(nm.d_diag(N))
    ref = dict(q=P.conj().T @ Ci @ y, r=P.conj().T @ D @ Ci @ y, u=P.conj().T @ D @ D @ Ci @ y,
               s=np.diag(P.conj().T @ Ci @ P), t=np.diag(P.conj().T @ D @ Ci @ P),
               v=np.diag(P.conj().T @ D @ D @ Ci @ P), x=np.diag(P.conj().T @ D @ Ci @ D @ P))
    for k in "qrustvx":
        assert np.allclose(ev.act[k], ref[k], rtol=1e-9, atol=1e-9 * np.max(np.abs(ref[k]))), k
    # and the diagonal-sum route for s, t, v, x at the active frequencies (eq. sFourier)
    N2 = np.arange(-(N - 1), N)
    E = np.exp(2j * np.pi * np.outer(N2, th))
    for k, om in zip("stvx", ev.omega):
        assert np.allclose(om @ E, ref[k], rtol=1e-9, atol=1e-9 * np.max(np.abs(ref[k]))), k


# ------------------------------------------------------------ derivatives ---

def f_plain(y, th, ga, be):
    C = nm.covariance(th, ga, be, len(y))
    return np.linalg.slogdet(C)[1] + np.vdot(y, np.linalg.solve(C, y)).real


@pytest.mark.parametrize("seed", [0, 1])
def test_derivatives_against_finite_differences(seed):
    """eqs. derivative / derivative2 against central differences of ln|C| + y^H C^{-1} y
    (slogdet + LU solve, not the Cholesky route)."""
    rng = np.random.default_rng(seed)
    N, K = 16, 3
    th = np.array([0.11, 0.43, 0.77]) + 0.01 * rng.random(3)
    ga = np.array([1.3, 0.6, 2.2])
    be = 0.25
    y = nm.steering(th, N) @ (rng.standard_normal(K) + 1j * rng.standard_normal(K)) + 0.3 * rand_y(rng, N)
    ev = nm.Evaluation(y, th, ga, be)
    gth, gga = nm.gradient(ga, ev.act)
    hth, hga = nm.hessian_diag(ga, ev.act)
    for k in range(K):
        for which, x0, gk, hk, h in (("th", th, gth[k], hth[k], 1e-5), ("ga", ga, gga[k], hga[k], 1e-4)):
            def f(dx):
                a = x0.copy()
                a[k] += dx
                return f_plain(y, a, ga, be) if which == "th" else f_plain(y, th, a, be)
            f0, fp, fm = f(0.0), f(h), f(-h)
            g_fd = (fp - fm) / (2 * h)
            h_fd = (fp - 2 * f0 + fm) / h ** 2
            assert abs(g_fd - gk) <= 1e-6 * max(1.0, abs(gk)), (which, k, g_fd, gk)
            assert abs(h_fd - hk) <= 1e-3 * max(1.0, abs(hk)), (which, k, h_fd, hk)


# --------------------------------------------------------------- woodbury ---

def test_woodbury_shortcuts():
    """mu = gamma . q, tr(Sigma A^H A) = beta sum gamma s (Sec. II-D after eq. betaUpdate),
    q~_k = q/(1-gamma s), s~_k = s/(1-gamma s) (after eq. deactivate),
    ||y - A mu||^2 = beta^2 ||C^{-1} y||^2 (since y - A Gamma A^H C^{-1} y = beta C^{-1} y)."""
    rng = np.random.default_rng(21)
    N = 18
    th, ga, be = rand_state(rng, N, 4)
    y = rand_y(rng, N)
    ev = nm.Evaluation(y, th, ga, be)
    A = nm.steering(th, N)
    AhA = A.conj().T @ A
    Sigma = np.linalg.inv(AhA / be + np.diag(1 / ga))
    mu = Sigma @ A.conj().T @ y / be
    q, s = ev.act["q"], ev.act["s"].real
    assert np.allclose(mu, ga * q, atol=1e-11)
    assert abs(np.trace(Sigma @ AhA).real - be * np.sum(ga * s)) < 1e-10
    res = y - A @ mu
    assert abs(np.vdot(res, res).real - be ** 2 * np.vdot(ev.w, ev.w).real) < 1e-10
    for k in range(4):
        keep = [j for j in range(4) if j != k]
        ev_k = nm.Evaluation(y, th[keep], ga[keep], be)
        p = A[:, k]
        qt_ref = np.vdot(p, ev_k.w)
        st_ref = np.vdot(p, ev_k.F.solve(p)).real
        qt, st = nm.loo_qs(q[k], s[k], ga[k])
        assert abs(qt - qt_ref) < 1e-10 and abs(st - st_ref) < 1e-10


def test_gamma_hat_minimises_single_component_objective():
    """eq. activate_gamma is the minimiser over gamma >= 0 of
    -|q|^2/(gamma^{-1}+s) + ln(1 + gamma s) (eq. singlecomp in gamma)."""
    for q, s in [(3.0 + 1j, 2.0), (0.5, 2.0), (10.0, 0.3), (1.2, 1.0)]:
        f = lambda g: -abs(q) ** 2 * g / (1 + g * s) + math.log1p(g * s)
        res = so.minimize_scalar(f, bounds=(0.0, 1e4), method="bounded",
                                 options={"xatol": 1e-12})
        gh = float(nm.gamma_hat(q, s))
        best = min([(f(0.0), 0.0), (res.fun, res.x)])
        assert abs(gh - best[1]) < 1e-5 * max(1.0, gh), (q, s, gh, best)


def test_zeta_update_is_the_constrained_minimiser():
    """eq. zetaUpdate: min(1/2, K/N) minimises the prior term over [0, 1/2]."""
    for K, N in [(0, 50), (3, 50), (20, 50), (40, 50)]:
        zs = np.linspace(0.0, 0.5, 50001)
        vals = [nm.prior_term(K, N, z) if (z > 0 or K == 0) else math.inf for z in zs]
        zbest = zs[int(np.argmin(vals))]
        assert abs(zbest - min(0.5, K / N)) < 2e-5


def test_delta_L_and_criterion_relations():
    """Delta L < 0 is eq. activate_derived; tau > 0 only tightens it (eq. activate_criterion).
    With gbar = gamma_hat the objective change is ln(kappa (1-zeta)/zeta) - (kappa - 1)."""
    rng = np.random.default_rng(4)
    for _ in range(200):
        q = complex(*rng.standard_normal(2) * 4)
        s = float(rng.random() * 3 + 0.05)
        gb = float(rng.random() * 5 + 1e-3)
        z = float(rng.random() * 0.49 + 0.005)
        dl = float(nm.delta_L(q, s, gb, z))
        assert bool(nm.activation_criterion(q, s, gb, z, 0.0)) == (dl < 0)
        if bool(nm.activation_criterion(q, s, gb, z, 5.0)):
            assert dl < 0
        gh = float(nm.gamma_hat(q, s))
        if gh > 0:
            kap = abs(q) ** 2 / s
            assert abs(float(nm.delta_L(q, s, gh, z)) - (math.log(kap * (1 - z) / z) - (kap - 1))) < 1e-9


def test_beta_update_does_not_increase_objective():
    """EM bound (eqs. bound, bound_explicit): the beta update never increases ln|C| + y^H C^{-1} y."""
    rng = np.random.default_rng(8)
    for trial in range(5):
        N = 24
        th, ga, be = rand_state(rng, N, 3, beta=0.05 + rng.random())
        y = rand_y(rng, N) + nm.steering(th, N) @ rng.standard_normal(3)
        f0 = f_plain(y, th, ga, be)
        b1 = nm.beta_update_definition(y, th, ga, be, 1e-12)
        assert f_plain(y, th, ga, b1) <= f0 + 1e-10
