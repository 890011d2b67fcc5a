"""Pins of the MMV oracle (Sec. V; no GPU): each quantity against its definition
from dense linear algebra, finite differences or a numeric minimiser, the
reduction to the single-vector oracle at G = 1, and the estimator's block
descent and recovery."""
import math

import numpy as np
import pytest
import scipy.optimize as so

from oracle import estimator as oe
from oracle import mmv
from oracle import numerics as nm
from paper_1705_06073_amd import synth
from tests import metrics
from tests.test_oracle_pins import _em_bound_by_quadrature


def _signals(rng, G, N, theta, beta):
    A = nm.steering(theta, N)
    K = len(theta)
    al = (rng.standard_normal((G, K)) + 1j * rng.standard_normal((G, K))) / math.sqrt(2)
    w = (rng.standard_normal((G, N)) + 1j * rng.standard_normal((G, N))) * math.sqrt(beta / 2)
    return al @ A.T + w


def _state(seed, G=3, N=24):
    rng = np.random.default_rng(seed)
    theta = np.array([0.13, 0.42, 0.77]) + 0.01 * rng.random(3)
    Y = _signals(rng, G, N, theta, 0.2)
    gamma = 0.5 + rng.random(3)
    beta = 0.1 + 0.2 * rng.random()
    return rng, Y, theta, gamma, beta


def _dense_objective(Y, theta, gamma, beta, zeta):
    """-sum_g ln CN(y_g; 0, C) - prior, dropping G N ln pi (Sec. V), with C formed
    from its definition and numpy's slogdet and solve."""
    N = Y.shape[1]
    C = beta * np.eye(N) + (nm.steering(theta, N) * gamma) @ nm.steering(theta, N).conj().T
    ld = np.linalg.slogdet(C)[1]
    quad = sum(np.vdot(y, np.linalg.solve(C, y)).real for y in Y)
    K = len(theta)
    prior = -(K * math.log(zeta) + (N - K) * math.log(1 - zeta))
    return Y.shape[0] * ld + quad + prior


@pytest.mark.parametrize("seed", range(3))
def test_single_vector_case_is_the_smv_oracle_bitwise(seed):
    """G = 1: the MMV estimator takes the single-vector estimator's steps and
    returns its result bit for bit."""
    inst = synth.workload_n64(seed)
    a = oe.estimate(inst.y, oe.Params(L_mult=4.0))
    b = mmv.estimate(inst.y[None, :], oe.Params(L_mult=4.0))
    assert a.K == b.K and a.evaluations == b.evaluations and a.iterations == b.iterations
    assert np.array_equal(a.theta, b.theta) and np.array_equal(a.gamma, b.gamma)
    assert np.array_equal(a.alpha, b.alpha[0]) and a.beta == b.beta
    assert a.objective == b.objective


def test_objective_is_the_sum_of_the_vectors_likelihoods():
    _, Y, th, ga, be = _state(1)
    ev = mmv.EvaluationMMV(Y, th, ga, be)
    assert ev.f(3, 0.1) == pytest.approx(_dense_objective(Y, th, ga, be, 0.1), rel=1e-12)


@pytest.mark.parametrize("seed", range(2))
def test_derivatives_match_finite_differences(seed):
    """The summed eqs. derivative / derivative2 against central differences of
    the dense MMV objective, in theta and gamma."""
    _, Y, th, ga, be = _state(10 + seed)
    ev = mmv.EvaluationMMV(Y, th, ga, be)
    gth, gga = mmv.gradient(ga, ev.per_vector)
    hth, hga = mmv.hessian_diag(ga, ev.per_vector)
    f = lambda t, g: _dense_objective(Y, t, g, be, 0.1)  # noqa: E731
    f0 = f(th, ga)
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        h = 1e-6
        ft_p, ft_m = f(th + h * e, ga), f(th - h * e, ga)
        assert gth[k] == pytest.approx((ft_p - ft_m) / (2 * h), rel=1e-5, abs=1e-6)
        h2 = 1e-4
        d2 = (f(th + h2 * e, ga) - 2 * f0 + f(th - h2 * e, ga)) / h2 ** 2
        assert hth[k] == pytest.approx(d2, rel=2e-4)
        hg = 1e-6 * ga[k]
        assert gga[k] == pytest.approx((f(th, ga + hg * e) - f(th, ga - hg * e)) / (2 * hg),
                                       rel=1e-5, abs=1e-6)
        hg2 = 1e-3 * ga[k]
        d2g = (f(th, ga + hg2 * e) - 2 * f0 + f(th, ga - hg2 * e)) / hg2 ** 2
        assert hga[k] == pytest.approx(d2g, rel=1e-4)


@pytest.mark.parametrize("seed", range(3))
def test_delta_L_is_the_dense_objective_change_of_an_added_component(seed):
    """Adding a component at theta_new with variance gamma changes the dense
    objective by the z_k = 1 term of eq. singlecomp-mmv (q, s at theta_new)."""
    rng, Y, th, ga, be = _state(20 + seed)
    ev = mmv.EvaluationMMV(Y, th, ga, be)
    t_new = 0.6 + 0.05 * rng.random()
    zeta = 0.1
    q = np.array([nm.q_at(w, [t_new])[0] for w in ev.w])
    s = float(nm.s_at(ev.omega[0], [t_new])[0])
    for g_new in (0.05, 0.7, 3.0):
        d = (_dense_objective(Y, np.append(th, t_new), np.append(ga, g_new), be, zeta)
             - _dense_objective(Y, th, ga, be, zeta))
        # the prior term changes by ln((1-zeta)/zeta) when one more component is active
        dl = float(mmv.delta_L(mmv.sum_q2(q), s, g_new, zeta, 3))
        assert dl == pytest.approx(d, rel=1e-9, abs=1e-9)


def test_gamma_hat_is_the_minimiser_of_the_single_component_term():
    rng = np.random.default_rng(3)
    for _ in range(5):
        G = int(rng.integers(2, 6))
        s = 0.5 + rng.random()
        Q = G * s * (1.5 + 3 * rng.random())        # Qbar / s > 1
        h = lambda g: G * math.log1p(g * s) - Q * g / (1 + g * s)  # noqa: E731
        r = so.minimize_scalar(h, bounds=(1e-9, 1e3), method="bounded",
                               options={"xatol": 1e-12})
        assert float(mmv.gamma_hat(Q, s, G)) == pytest.approx(r.x, rel=1e-6)
    assert float(mmv.gamma_hat(0.9 * 4 * 2.0, 2.0, 4)) == 0.0  # Qbar / s < 1


def test_criterion_without_tau_is_delta_L_below_zero():
    """Reading M1 with tau = 0 is the sign of Delta L_MMV at the average gamma."""
    rng = np.random.default_rng(4)
    for _ in range(200):
        G = int(rng.integers(1, 6))
        s, gb, zeta = 0.2 + rng.random(), 0.05 + rng.random(), 0.02 + 0.4 * rng.random()
        Q = G * s * 4 * rng.random()
        dl = float(mmv.delta_L(Q, s, gb, zeta, G))
        if abs(dl) < 1e-9:
            continue
        assert mmv.activation_criterion(Q, s, gb, zeta, 0.0, G) == (dl < 0)
    # tau raises the threshold on the averaged SNR by exactly tau
    s, gb, zeta, G = 0.7, 0.3, 0.1, 3
    rhs0 = mmv.criterion_rhs(s, gb, zeta, 0.0, G)
    assert mmv.criterion_rhs(s, gb, zeta, 5.0, G) == pytest.approx(rhs0 + 5.0, rel=1e-15)


@pytest.mark.parametrize("seed", range(3))
def test_deactivation_margin_is_the_dense_objective_difference(seed):
    """margin_k = L(z_k = 1) - L(z_k = 0) from dense evaluations, both signs."""
    rng = np.random.default_rng(600 + seed)
    G, N = 3, 40
    true_th = np.array([0.11, 0.37, 0.71])
    Y = _signals(rng, G, N, true_th, 0.05)
    spur = np.array([0.52, 0.9]) + 0.01 * rng.random(2)
    th = np.concatenate([true_th + 1e-3 * rng.standard_normal(3), spur])
    ga = np.concatenate([0.5 + rng.random(3), 0.01 + 0.02 * rng.random(2)])
    be, zeta = 0.05, 5.0 / N
    ev = mmv.EvaluationMMV(Y, th, ga, be)
    marg = mmv.deactivation_margin(ev.act["q"], ev.act["s"].real, ga, zeta, G)
    f_all = _dense_objective(Y, th, ga, be, zeta)
    signs = set()
    for k in range(len(th)):
        keep = np.arange(len(th)) != k
        diff = f_all - _dense_objective(Y, th[keep], ga[keep], be, zeta)
        assert marg[k] == pytest.approx(diff, rel=1e-8, abs=1e-9 * abs(f_all))
        signs.add(np.sign(diff))
    assert signs == {-1.0, 1.0}


@pytest.mark.parametrize("seed", range(2))
def test_beta_update_is_the_minimiser_of_the_summed_em_bound(seed):
    """The MMV beta minimises sum_g of the EM bound of eq. bound_explicit, each
    expectation by quadrature over its vector's posterior."""
    rng = np.random.default_rng(910 + seed)
    G, N = 3, 16
    theta = np.array([0.2, 0.61]) + 0.02 * rng.random(2)
    Y = _signals(rng, G, N, theta, 0.3)
    gamma = 0.5 + rng.random(2)
    beta_old = 0.1 + rng.random()
    b_upd = mmv.beta_update_definition(Y, theta, gamma, beta_old, 1e-12)
    bound = lambda lb: float(sum(_em_bound_by_quadrature(y, theta, gamma, beta_old,  # noqa: E731
                                                         math.exp(lb))[0] for y in Y))
    r = so.minimize_scalar(bound, bounds=(math.log(1e-4), math.log(1e2)), method="bounded",
                           options={"xatol": 1e-10})
    assert math.exp(r.x) == pytest.approx(b_upd, rel=1e-6)


@pytest.mark.parametrize("seed", range(2))
def test_block_updates_do_not_increase_the_objective(seed):
    rng = np.random.default_rng(700 + seed)
    th = synth.draw_frequencies(rng, 4, 2.0 / 48)
    Y = _signals(rng, 3, 48, th, 0.05)
    res = mmv.estimate(Y, oe.Params(), check_blocks=True)
    blocks = [t for t in res.trace if t[0] == "block"]
    assert {"zeta", "beta", "lbfgs"} <= {b[1] for b in blocks}
    for _, name, fb, fa in blocks:
        if name == "approx":
            continue
        assert fa <= fb + 1e-9 * max(1.0, abs(fb)), (name, fb, fa)


def test_noiseless_recovery_and_shapes():
    rng = np.random.default_rng(77)
    th = synth.draw_frequencies(rng, 4, 2.0 / 64)
    Y = _signals(rng, 4, 64, th, 1e-7)
    res = mmv.estimate(Y, oe.Params(L_mult=4.0))
    assert res.K == 4 and res.alpha.shape == (4, 4)
    r, c = metrics.match(th, res.theta)
    assert np.max(synth.wrap_distance(th[r], res.theta[c])) < 1e-5


def test_more_vectors_resolve_more_at_low_snr():
    """Sec. V motivation: with the same frequencies seen in G = 4 vectors the
    model order and frequencies are recovered more often than from one vector
    (N = 48, K = 4, 3 dB, 16 trials)."""
    wins = [0, 0]
    for t in range(16):
        rng = np.random.default_rng(800 + t)
        th = synth.draw_frequencies(rng, 4, 2.0 / 48)
        A = nm.steering(th, 48)
        al = (rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))) / math.sqrt(2)
        H = al @ A.T
        beta = float(np.mean(np.sum(np.abs(H) ** 2, axis=1))) / (48 * 10 ** 0.3)
        Y = H + (rng.standard_normal((4, 48)) + 1j * rng.standard_normal((4, 48))) * math.sqrt(beta / 2)
        for i, Yg in enumerate((Y[:1], Y)):
            res = mmv.estimate(Yg)
            wins[i] += metrics.block_success(th, res.theta, 48)
    assert wins[1] > wins[0], wins
