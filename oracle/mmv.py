"""Multiple measurement vectors (Sec. V): G observation vectors y^(g) that
share the frequencies, the component variances gamma, the noise variance beta
and the activation probability zeta.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The covariance C = beta I + Psi Gamma Psi^H is the one of the single-vector
model (Sec. II-B), so every quantity that depends on C alone (ln|C|, s, t, v,
x, the diagonal sums) is computed once; every quantity that depends on y
(w = C^{-1} y, q, r, u, q^G, y^H C^{-1} y) is computed per vector.  The
formulas, each from its definition:

  objective    L_MMV = G ln|C| + sum_g y_g^H C^{-1} y_g - prior   (Sec. V)
  derivatives  the sums over g of eqs. derivative / derivative2 with y -> y_g
  single comp. L(z_k, theta_k, gamma_k) = z_k ( G ln(1 + gamma s~)
               - sum_g |q~_g|^2 / (gamma^{-1} + s~) + ln((1-zeta)/zeta) )
               (eq. singlecomp-mmv), hence
  gamma_hat    (Qbar - s) / s^2 when Qbar / s > 1, Qbar = sum_g |q_g|^2 / G
               (its minimiser over gamma),
  Delta L      G ln(1 + gb s) + ln((1-zeta)/zeta) - sum_g |q_g|^2 / (gb^{-1} + s)
               (the single-component term at gamma = the average gb; with no
               active component, gamma = gamma_hat(theta) per point),
  deactivate   when the z_k = 1 term is positive (eq. deactivate's reading),
  beta         max(eps, tr(Sigma A^H A) / M + sum_g ||y_g - A mu_g||^2 / (G M))
               with Sigma, mu_g from eqs. bSigma, bmu (the MMV beta of Sec. V).

Readings where Sec. V leaves details to the reader ("follow straightforwardly"):

  M1  activation criterion: the analogue of eq. activate_criterion on the
      per-vector average, Qbar/s > (1 + 1/(gb s)) (ln(1 + gb s)
      + ln((1-zeta)/zeta)/G) + tau, i.e. Delta L_MMV / G < 0 written for
      kappa = Qbar/s (the component's SNR averaged over the vectors) with the
      same threshold adjustment tau; G = 1 gives eq. activate_criterion.
  M2  the scales of the stopping rules (Sec. II-E) and of the initial beta
      follow the objective, which is a sum of G single-vector objectives:
      |L_i - L_{i-1}| < G N tol, squared Newton decrement < G N tol,
      beta_0 = 0.01 sum_g ||y_g||^2 / (G N), eps_beta likewise.
  M3  amplitudes: alpha^(g) = gamma .* q^(g) (eq. bmu per vector).

With G = 1 every function reduces to its single-vector counterpart in
``numerics`` term by term, and the estimator takes the same steps.
"""
from __future__ import annotations

import math

import numpy as np

from . import numerics as nm
from .estimator import OracleEstimator, Params, Result


class EvaluationMMV:
    """All quantities of one evaluation at (theta, gamma, beta) for the
    observation matrix Y (G x N)."""

    def __init__(self, Y, theta, gamma, beta: float):
        self.Y = np.atleast_2d(np.asarray(Y, dtype=np.complex128))
        self.G, self.N = self.Y.shape
        self.theta = np.array(theta, dtype=np.float64)
        self.gamma = np.array(gamma, dtype=np.float64)
        self.beta = float(beta)
        self.C = nm.covariance(self.theta, self.gamma, self.beta, self.N)
        self.F = nm.DenseFactor(self.C)
        self.w = np.stack([self.F.solve(y) for y in self.Y])           # G x N
        self.yCy = float(sum(np.vdot(y, w).real for y, w in zip(self.Y, self.w)))
        self.logdet = self.F.logdet
        K = len(self.theta)
        if K:
            per = [nm.active_vectors(self.F, w, self.theta) for w in self.w]
            self.act = {k: np.stack([a[k] for a in per]) for k in "qru"}
            self.act.update({k: per[0][k] for k in "stvx"})
            self.per_vector = per
        else:
            z = np.zeros((self.G, 0), np.complex128)
            self.act = {"q": z, "r": z, "u": z}
            self.act.update({k: np.zeros(0, np.complex128) for k in "stvx"})
            self.per_vector = [{k: np.zeros(0, np.complex128) for k in "qrustvx"}] * self.G
        self._om = None

    @property
    def omega(self):
        if self._om is None:
            self._om = nm.omegas(self.F)
        return self._om

    def grid(self, L: int):
        """(q^G of every vector, G x L; s^G, L) on the grid l/L (Sec. III-D)."""
        return np.stack([nm.grid_q(w, L) for w in self.w]), nm.grid_s(self.omega[0], L)

    def f(self, K: int, zeta: float) -> float:
        """L_MMV (Sec. V, additive constant dropped)."""
        return self.G * self.logdet + self.yCy + nm.prior_term(K, self.N, zeta)


def gradient(gamma, per_vector):
    """Sum over g of eq. derivative with y -> y_g (Sec. V)."""
    parts = [nm.gradient(gamma, a) for a in per_vector]
    return sum(p[0] for p in parts), sum(p[1] for p in parts)


def hessian_diag(gamma, per_vector):
    """Sum over g of eq. derivative2 with y -> y_g (Sec. V)."""
    parts = [nm.hessian_diag(gamma, a) for a in per_vector]
    return sum(p[0] for p in parts), sum(p[1] for p in parts)


def sum_q2(q):
    """sum_g |q_g|^2 over the first axis (vectors)."""
    return np.sum(np.abs(np.asarray(q)) ** 2, axis=0)


def gamma_hat(Q, s, G: int):
    """Minimiser of eq. singlecomp-mmv over gamma: (Q/G - s)/s^2 if Q/(G s) > 1, else 0."""
    Qb = np.asarray(Q, dtype=np.float64) / G
    s = np.asarray(s, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(Qb / s > 1.0, (Qb - s) / (s * s), 0.0)


def delta_L(Q, s, gbar, zeta, G: int):
    """G ln(1 + gb s) + ln((1-zeta)/zeta) - Q / (gb^{-1} + s): the z_k = 1 term of
    eq. singlecomp-mmv at gamma = gb (with s~, q~ = s, q at an inactive point).
    Written as ln((1 + gb s)(1-zeta)/zeta) + (G-1) ln(1 + gb s) so that G = 1
    is eq. delta_L operation by operation."""
    Q = np.asarray(Q, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    gbar = np.asarray(gbar, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        lg = np.log((1.0 + gbar * s) * ((1.0 - zeta) / zeta)) + (G - 1) * np.log1p(gbar * s)
        quad = np.where(gbar > 0, Q / (1.0 / np.where(gbar > 0, gbar, 1.0) + s), 0.0)
        return lg - quad


def criterion_rhs(s, gbar, zeta, tau, G: int):
    """Right-hand side of reading M1, (1 + 1/(gb s)) (ln(1 + gb s) + ln((1-zeta)/zeta)/G)
    + tau, written as (1 + 1/(gb s)) (ln((1 + gb s)(1-zeta)/zeta) + (G-1) ln(1 + gb s)) / G
    + tau (G = 1: eq. activate_criterion operation by operation)."""
    lg = math.log((1.0 + gbar * s) * ((1.0 - zeta) / zeta)) + (G - 1) * math.log1p(gbar * s)
    return (1.0 + 1.0 / (gbar * s)) * (lg / G) + tau


def activation_criterion(Q, s, gbar, zeta, tau, G: int) -> bool:
    """Reading M1 of the MMV activation criterion: Qbar / s > criterion_rhs."""
    if not (s > 0 and gbar > 0 and 0 < zeta < 1):
        return False
    return bool((Q / G) / s > criterion_rhs(s, gbar, zeta, tau, G))


def deactivation_margin(q, s, gamma, zeta, G: int):
    """ln((1-zeta)/zeta) - [sum_g |q~_g|^2/(gamma^{-1}+s~) - G ln(1+gamma s~)]:
    the z_k = 1 term of eq. singlecomp-mmv at the current gamma_k; > 0 means the
    component lowers the objective when removed.  q: G x K.  gamma_k = 0: +inf."""
    gamma = np.asarray(gamma, dtype=np.float64)
    out = np.full(gamma.shape, np.inf)
    pos = gamma > 0
    if np.any(pos):
        s = np.asarray(s, dtype=np.float64)[pos]
        g = gamma[pos]
        den = 1.0 - g * s
        qt2 = sum_q2(np.asarray(q)[:, pos] / den)            # sum_g |q~_g|^2 (Woodbury)
        st = s / den
        lhs = qt2 / (1.0 / g + st) - G * np.log1p(g * st)
        thr = math.log((1.0 - zeta) / zeta) if zeta > 0 else math.inf
        out[pos] = thr - lhs
    return out


def beta_update_definition(Y, theta, gamma, beta_old: float, eps_beta: float) -> float:
    """MMV beta of Sec. V from its definition (Sigma and mu_g by eqs. bSigma, bmu)."""
    Y = np.atleast_2d(Y)
    G, N = Y.shape
    if len(theta) == 0:
        return max(eps_beta, sum(float(np.vdot(y, y).real) for y in Y) / (G * N))
    A = nm.steering(theta, N)
    AhA = A.conj().T @ A
    Sigma = np.linalg.inv(AhA / beta_old + np.diag(1.0 / np.asarray(gamma, dtype=np.float64)))
    tr = float(np.trace(Sigma @ AhA).real)
    res = 0.0
    for y in Y:
        mu = Sigma @ (A.conj().T @ y) / beta_old
        r = y - A @ mu
        res += float(np.vdot(r, r).real)
    # tr/N + res/(G N), as one quotient
    return max(eps_beta, (G * tr + res) / (G * N))


class OracleEstimatorMMV(OracleEstimator):
    """The estimator of Sec. II-C/E on the MMV objective: the block-coordinate
    descent, the approximate activation scheme, L-BFGS and the final refinement
    of the single-vector oracle, with the observation-dependent steps of
    Sec. V."""

    def __init__(self, Y, params: Params | None = None, check_blocks: bool = False):
        super().__init__(np.atleast_2d(np.asarray(Y, dtype=np.complex128)), params, check_blocks)
        self.G = self.y.shape[0]

    def _new_eval(self, theta, gamma, beta):
        return EvaluationMMV(self.y, theta, gamma, beta)

    def _energy(self) -> float:
        return sum(float(np.vdot(y, y).real) for y in self.y) / self.G   # reading M2

    def _q_at(self, ev, theta):
        return np.stack([nm.q_at(w, theta) for w in ev.w])            # G x len(theta)

    def _qq(self, q) -> float:
        return float(sum_q2(q)) / self.G                               # Qbar

    def _criterion(self, q, s, gb, zeta, tau) -> bool:
        return activation_criterion(float(sum_q2(q)), s, gb, zeta, tau, self.G)

    def _criterion_rhs(self, s, gb, zeta, tau):
        return criterion_rhs(s, gb, zeta, tau, self.G)

    def _decision_quantities(self, q, s, gamma, zeta):
        Q = float(sum_q2(q))
        gh = float(gamma_hat(Q, s, self.G))
        gb = self._gbar(gamma)
        if gb is None:       # empty active set: per-theta optimum (reading R4)
            gb = gh
        return gb, gh, float(delta_L(Q, s, gb, zeta, self.G))

    def _grid_delta_L(self, ev, gamma, zeta):
        qG, sG = ev.grid(self.L)
        Q = sum_q2(qG)
        gb = self._gbar(gamma)
        gbv = gamma_hat(Q, sG, self.G) if gb is None else np.full(self.L, gb)
        return qG, sG, delta_L(Q, sG, gbv, zeta, self.G)

    def _grad_hess(self, ev, gamma):
        gth, gga = gradient(gamma, ev.per_vector)
        hth, hga = hessian_diag(gamma, ev.per_vector)
        return gth, gga, hth, hga

    def _beta_update(self, theta, gamma, beta, eps_beta) -> float:
        return beta_update_definition(self.y, theta, gamma, beta, eps_beta)

    def _deact_margins(self, ev, gamma, zeta):
        return deactivation_margin(ev.act["q"], ev.act["s"].real, gamma, zeta, self.G)

    def _alpha(self, ev, gamma):
        return gamma[None, :] * ev.act["q"]                            # reading M3


def estimate(Y, params: Params | None = None, check_blocks: bool = False) -> Result:
    """MMV estimate of Y (G x N); Result.alpha is G x K."""
    return OracleEstimatorMMV(Y, params, check_blocks).run()
