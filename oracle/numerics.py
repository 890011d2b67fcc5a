"""Dense FP64 numerics of one evaluation of the estimator's objective.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Conventions (0-indexed): psi(theta)_n = exp(j 2 pi n theta), n = 0..N-1;
D = diag(2 pi n); the grid is theta^G_l = l / L, l = 0..L-1.

Every quantity is formed from its definition:

* C = beta I + Psi(theta) diag(gamma) Psi(theta)^H        (Sec. II-B, eq. py)
* C = L_c L_c^H (Cholesky);  delta_i = |[L_c]_ii|^2 are the pivots of the
  unit-lower LDL^H factorisation, ln|C| = sum_i ln delta_i   (Sec. III-A)
* rho, delta_{N-1} of the Gohberg-Semencul formula: C x = e_{N-1},
  delta_{N-1} = 1 / x_{N-1}, rho = x / x_{N-1}, so rho_{N-1} = 1
  (Sec. III, eq. gohberg-semencul: the last column of C^{-1} is
  delta_{N-1}^{-1} times [T_1^H T_1 - T_0 T_0^H] e_{N-1} = rho / delta_{N-1})
* w = C^{-1} y, y^H C^{-1} y                               (Sec. III-A)
* q, r, u, s, t, v, x                                       (Sec. II-D, eqs. q-x)
* omega_s, omega_t, omega_v, omega_x as diagonal sums        (Sec. III-C, eqs. omega_s-omega_x)
* q^G = Psi^H(theta^G) w, s^G = diag(Psi^H C^{-1} Psi)       (Sec. III-D)
* derivatives                                               (Sec. II-D, eqs. derivative, derivative2)
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

TWO_PI = 2.0 * math.pi


def phase_frac(n, theta):
    """(n * theta) mod 1, reduced in extended precision, returned as float64."""
    n = np.asarray(n, dtype=np.longdouble)
    th = np.asarray(theta, dtype=np.longdouble)
    p = np.multiply.outer(n, th)
    return np.asarray(p - np.floor(p), dtype=np.float64)


def steering(theta, N: int) -> np.ndarray:
    """Psi(theta): N x K matrix with [Psi]_{n,k} = exp(j 2 pi n theta_k) (Sec. II-A)."""
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    return np.exp(2j * math.pi * phase_frac(np.arange(N), theta))


def d_diag(N: int) -> np.ndarray:
    """Diagonal of D = diag(0, 2pi, 4pi, ..., 2pi(N-1)) (Sec. II-D)."""
    return TWO_PI * np.arange(N, dtype=np.float64)


def covariance(theta, gamma, beta: float, N: int) -> np.ndarray:
    """C = beta I + Psi Gamma Psi^H, formed densely (Sec. II-B, eq. py)."""
    Psi = steering(theta, N)
    gamma = np.asarray(gamma, dtype=np.float64)
    C = (Psi * gamma[None, :]) @ Psi.conj().T
    C[np.diag_indices(N)] += beta
    return C


def toeplitz_column(theta, gamma, beta: float, N: int) -> np.ndarray:
    """First column of C: c_i = [C]_{i,0} = beta [i=0] + sum_k gamma_k e^{j2pi i theta_k}.

    Read off eq. py with psi_0 = 1 (Sec. II-B; Toeplitz structure, Sec. III).
    """
    Psi = steering(theta, N)
    c = Psi @ np.asarray(gamma, dtype=np.float64).astype(np.complex128)
    c[0] += beta
    return c


def dense_from_column(c: np.ndarray) -> np.ndarray:
    """Hermitian Toeplitz matrix with first column c: C_{m,n} = c_{m-n}, c_{-i} = conj(c_i)."""
    c = np.asarray(c, dtype=np.complex128)
    return sla.toeplitz(c, c.conj())


class DenseFactor:
    """Cholesky-based factor quantities of a Hermitian positive-definite C."""

    def __init__(self, C: np.ndarray):
        self.C = np.asarray(C, dtype=np.complex128)
        self.N = self.C.shape[0]
        self.Lc = sla.cholesky(self.C, lower=True)
        self._cho = (self.Lc, True)
        self._inv = None

    # -- Sec. III-A: C = L B L^H with unit-lower L; B = diag(delta) -----------
    @property
    def delta(self) -> np.ndarray:
        return np.abs(np.diag(self.Lc)) ** 2

    @property
    def logdet(self) -> float:
        return float(np.sum(np.log(self.delta)))

    # -- Sec. III, eq. gohberg-semencul: generator (rho, delta_{N-1}) -------------
    def generator(self):
        e = np.zeros(self.N, dtype=np.complex128)
        e[-1] = 1.0
        x = sla.cho_solve(self._cho, e)
        xl = x[-1].real
        return x / xl, 1.0 / xl

    def solve(self, b):
        return sla.cho_solve(self._cho, np.asarray(b, dtype=np.complex128))

    def inverse(self) -> np.ndarray:
        if self._inv is None:
            self._inv = self.solve(np.eye(self.N, dtype=np.complex128))
        return self._inv


def diagonal_sums(M: np.ndarray) -> np.ndarray:
    """omega(i) = sum_q M[q, q+i] for i = -(N-1)..N-1; entry i is at index i+N-1.

    The definition of eqs. omega_s / omega_t / omega_v / omega_x (Sec. III-C)
    with M = C^{-1}, D C^{-1}, D^2 C^{-1}, D C^{-1} D.
    """
    N = M.shape[0]
    return np.array([np.trace(M, offset=i) for i in range(-(N - 1), N)], dtype=np.complex128)


def omegas(F: DenseFactor):
    """(omega_s, omega_t, omega_v, omega_x), each of length 2N-1, index i+N-1."""
    Ci = F.inverse()
    d = d_diag(F.N)
    return (diagonal_sums(Ci),
            diagonal_sums(d[:, None] * Ci),
            diagonal_sums((d ** 2)[:, None] * Ci),
            diagonal_sums(d[:, None] * Ci * d[None, :]))


def active_vectors(F: DenseFactor, w: np.ndarray, theta) -> dict:
    """q, r, u, s, t, v, x at the active frequencies (Sec. II-D, eqs. q-x)."""
    N = F.N
    Psi = steering(theta, N)
    d = d_diag(N)
    X = F.solve(Psi)                    # C^{-1} Psi
    XD = F.solve(d[:, None] * Psi)      # C^{-1} D Psi
    Pc = Psi.conj()
    return dict(
        q=Psi.conj().T @ w,
        r=Psi.conj().T @ (d * w),
        u=Psi.conj().T @ (d * d * w),
        s=np.sum(Pc * X, axis=0),
        t=np.sum(Pc * d[:, None] * X, axis=0),
        v=np.sum(Pc * (d * d)[:, None] * X, axis=0),
        x=np.sum(Pc * d[:, None] * XD, axis=0),
    )


def q_at(w: np.ndarray, theta) -> np.ndarray:
    """q(theta) = psi(theta)^H w (eq. q with Phi = I)."""
    return steering(theta, len(w)).conj().T @ w


def s_at(omega_s: np.ndarray, theta) -> np.ndarray:
    """s(theta) = sum_i omega_s(i) e^{j2pi i theta} (eq. sFourier); real for Hermitian omega_s."""
    N = (len(omega_s) + 1) // 2
    i = np.arange(-(N - 1), N)
    th = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    E = np.exp(2j * math.pi * phase_frac(i, th))   # (2N-1) x K
    return (omega_s @ E).real


def grid_q(w: np.ndarray, L: int) -> np.ndarray:
    """q^G_l = sum_n w_n e^{-j2pi n l / L}: a length-L DFT of zero-padded w (Sec. III-D)."""
    assert L >= len(w)
    return np.fft.fft(w, n=L)


def grid_s(omega_s: np.ndarray, L: int) -> np.ndarray:
    """s^G_l = sum_i omega_s(i) e^{+j2pi i l / L} (eq. sFourier on the grid, Sec. III-D)."""
    N = (len(omega_s) + 1) // 2
    assert L >= 2 * N - 1, "grid shorter than 2N-1 aliases the diagonal sums"
    buf = np.zeros(L, dtype=np.complex128)
    idx = np.arange(-(N - 1), N) % L
    buf[idx] = omega_s
    return (L * np.fft.ifft(buf)).real


def grid_r(w: np.ndarray, L: int) -> np.ndarray:
    """r^G_l = psi(l/L)^H D C^{-1} y = sum_n 2 pi n w_n e^{-j2pi n l / L}: the grid
    form of eq. r (Sec. III-D; the theta-derivative of q^G up to the factor -j)."""
    assert L >= len(w)
    return np.fft.fft(d_diag(len(w)) * w, n=L)


def grid_t(omega_t: np.ndarray, L: int) -> np.ndarray:
    """t^G_l = psi(l/L)^H D C^{-1} psi(l/L) = sum_i omega_t(i) e^{+j2pi i l / L}
    (eq. t through the diagonal sums of D C^{-1}, Sec. III-C/D); complex, since
    omega_t is not Hermitian in the lag."""
    N = (len(omega_t) + 1) // 2
    assert L >= 2 * N - 1, "grid shorter than 2N-1 aliases the diagonal sums"
    buf = np.zeros(L, dtype=np.complex128)
    buf[np.arange(-(N - 1), N) % L] = omega_t
    return L * np.fft.ifft(buf)


def grid_s_bruteforce(F: DenseFactor, L: int) -> np.ndarray:
    """s^G_l = psi(l/L)^H C^{-1} psi(l/L) by direct quadratic forms (tiny N only)."""
    Psi = steering(np.arange(L) / L, F.N)
    Ci = F.inverse()
    return np.real(np.sum(Psi.conj() * (Ci @ Psi), axis=0))


# ---------------------------------------------------------------------------
# Objective and derivatives (Sec. II-B eq. obj; Sec. II-D eqs. derivative,
# derivative2).
# ---------------------------------------------------------------------------

def xlogy(a: float, b: float) -> float:
    return 0.0 if a == 0 else a * math.log(b)


def prior_term(K: int, N: int, zeta: float) -> float:
    """-sum_k (z_k ln zeta + (1 - z_k) ln(1 - zeta)) with K_max = N and 0 ln 0 = 0."""
    return -(xlogy(K, zeta) + xlogy(N - K, 1.0 - zeta))


def objective(logdet: float, yCy: float, K: int, N: int, zeta: float) -> float:
    """L = ln|C| + y^H C^{-1} y - prior (eq. obj, additive constant dropped)."""
    return logdet + yCy + prior_term(K, N, zeta)


def gradient(gamma, a: dict):
    """dL/dtheta_k = 2 gamma_k Im{t_k - q_k^* r_k};  dL/dgamma_k = s_k - |q_k|^2."""
    g = np.asarray(gamma, dtype=np.float64)
    q, r, s, t = a["q"], a["r"], a["s"].real, a["t"]
    return 2.0 * g * np.imag(t - q.conj() * r), s - np.abs(q) ** 2


def hessian_diag(gamma, a: dict):
    """Second derivatives on the diagonal (eq. derivative2, as printed)."""
    g = np.asarray(gamma, dtype=np.float64)
    q, r, u, s, t, v, x = (a[k] for k in "qrustvx")
    s = s.real
    inner = (x - v + g * (t * t - x * s)
             + g * (x * np.abs(q) ** 2 + s * np.abs(r) ** 2 - 2.0 * t * r * q.conj())
             + (u * q.conj() - np.abs(r) ** 2))
    return 2.0 * g * np.real(inner), 2.0 * s * np.abs(q) ** 2 - s * s


# ---------------------------------------------------------------------------
# Activation / deactivation quantities (Sec. II-D, eqs. singlecomp - activate_criterion)
# ---------------------------------------------------------------------------

def delta_L(q, s, gbar, zeta):
    """Delta L(theta) = ln((1 + gbar s)(1 - zeta)/zeta) - |q|^2 / (gbar^{-1} + s) (eq. delta_L)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.asarray(q)
        s = np.asarray(s, dtype=np.float64)
        gbar = np.asarray(gbar, dtype=np.float64)
        lg = np.log((1.0 + gbar * s) * ((1.0 - zeta) / zeta))
        quad = np.where(gbar > 0, np.abs(q) ** 2 / (1.0 / np.where(gbar > 0, gbar, 1.0) + s), 0.0)
        return lg - quad


def gamma_hat(q, s):
    """Minimiser of the single-component objective in gamma (eq. activate_gamma)."""
    q = np.asarray(q)
    s = np.asarray(s, dtype=np.float64)
    q2 = np.abs(q) ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(q2 / s > 1.0, (q2 - s) / (s * s), 0.0)


def activation_criterion(q, s, gbar, zeta, tau):
    """|q|^2/s > (1 + 1/(gbar s)) ln((1 + gbar s)(1-zeta)/zeta) + tau (eq. activate_criterion;
    tau = 0 gives eq. activate_derived)."""
    q = np.asarray(q)
    s = np.asarray(s, dtype=np.float64)
    gbar = np.asarray(gbar, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        kappa = np.abs(q) ** 2 / s
        rhs = (1.0 + 1.0 / (gbar * s)) * np.log((1.0 + gbar * s) * ((1.0 - zeta) / zeta)) + tau
        res = kappa > rhs
    return np.where(np.isnan(rhs), False, res)


def loo_qs(q, s, gamma):
    """q_{~k}, s_{~k} at theta_k from q_k, s_k by Woodbury (Sec. II-D, after eq. deactivate)."""
    den = 1.0 - np.asarray(gamma) * np.asarray(s, dtype=np.float64)
    return np.asarray(q) / den, np.asarray(s, dtype=np.float64) / den


def deactivation_margin(q, s, gamma, zeta):
    """ln((1-zeta)/zeta) - [ |q~|^2/(gamma^{-1}+s~) - ln(1+gamma s~) ]; > 0 means
    eq. deactivate holds.  A component with gamma <= 0 gets +inf."""
    gamma = np.asarray(gamma, dtype=np.float64)
    out = np.full(gamma.shape, np.inf)
    pos = gamma > 0
    if np.any(pos):
        qt, st = loo_qs(np.asarray(q)[pos], np.asarray(s)[pos], gamma[pos])
        g = gamma[pos]
        lhs = np.abs(qt) ** 2 / (1.0 / g + st) - np.log1p(g * st)
        with np.errstate(divide="ignore"):
            thr = math.log((1.0 - zeta) / zeta) if zeta > 0 else math.inf
        out[pos] = thr - lhs
    return out


def beta_update_definition(y, theta, gamma, beta_old: float, eps_beta: float) -> float:
    """beta = max(eps, (tr(Sigma A^H A) + ||y - A mu||^2)/M) with mu, Sigma from
    eqs. bmu / bSigma at beta_old (Sec. II-D, eq. betaUpdate), by the definition."""
    N = len(y)
    if len(theta) == 0:
        return max(eps_beta, float(np.vdot(y, y).real) / N)
    A = steering(theta, N)
    AhA = A.conj().T @ A
    Sigma = np.linalg.inv(AhA / beta_old + np.diag(1.0 / np.asarray(gamma, dtype=np.float64)))
    mu = Sigma @ (A.conj().T @ y) / beta_old
    tr = float(np.trace(Sigma @ AhA).real)
    res = y - A @ mu
    return max(eps_beta, (tr + float(np.vdot(res, res).real)) / N)


class Evaluation:
    """All quantities of one evaluation at (theta, gamma, beta) for observation y."""

    def __init__(self, y, theta, gamma, beta: float):
        self.y = np.asarray(y, dtype=np.complex128)
        self.N = len(self.y)
        self.theta = np.array(theta, dtype=np.float64)
        self.gamma = np.array(gamma, dtype=np.float64)
        self.beta = float(beta)
        self.C = covariance(self.theta, self.gamma, self.beta, self.N)
        self.F = DenseFactor(self.C)
        self.w = self.F.solve(self.y)
        self.yCy = float(np.vdot(self.y, self.w).real)
        self.logdet = self.F.logdet
        self.act = active_vectors(self.F, self.w, self.theta) if len(self.theta) else \
            {k: np.zeros(0, np.complex128) for k in "qrustvx"}
        self._om = None

    @property
    def omega(self):
        if self._om is None:
            self._om = omegas(self.F)
        return self._om

    def grid(self, L: int):
        return grid_q(self.w, L), grid_s(self.omega[0], L)

    def grid_derivatives(self, L: int):
        """(r^G, t^G) on the grid l/L (Sec. III-D)."""
        return grid_r(self.w, L), grid_t(self.omega[1], L)

    def f(self, K: int, zeta: float) -> float:
        return objective(self.logdet, self.yCy, K, self.N, zeta)
