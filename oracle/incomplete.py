"""Incomplete observations (Sec. IV): the observation y in C^M is y =
Phi Psi(theta) alpha + w with Phi made of M rows of an N x N diagonal matrix
(a subsampling and scaling matrix; the footnote of Sec. IV).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The observation operator is given by the observed sample indices n_m
(0-indexed, strictly increasing in [0, N)) and the nonzero weights phi_m, so
that Phi[m, n_m] = phi_m is the only nonzero entry of row m.  With
A(theta) = Phi Psi(theta) (Sec. II-A) every quantity is formed from its
definition, densely, in FP64:

* C = beta I_M + A diag(gamma) A^H (M x M)              (Sec. II-B, eq. py)
* ln|C| by a Cholesky factor of C, w_M = C^{-1} y, y^H C^{-1} y
* the N-space vector w = Phi^H C^{-1} y, so that eqs. q, r, u read
  q = Psi^H w, r = Psi^H D w, u = Psi^H D^2 w
* the N x N matrix E = Phi^H C^{-1} Phi, so that eqs. s, t, v, x read
  s = diag(Psi^H E Psi), t = diag(Psi^H D E Psi), v = diag(Psi^H D^2 E Psi),
  x = diag(Psi^H D E D Psi)
* q^G = Psi^H(theta^G) w and s^G = diag(Psi^H(theta^G) E Psi(theta^G)): the
  grid forms of Sec. III-D applied to w and to the diagonal sums of E
* the objective (eq. obj) with K_max = M (the footnote of Sec. II-A)
* the beta update (eq. betaUpdate) with A = Phi Psi and the divisor M.

None of the Woodbury / determinant-lemma forms by which Sec. IV computes these
quantities is used here; the tests check those identities against this
module instead.  With every sample observed and unit weights each quantity is
the complete-data one of ``numerics`` operation by operation.
"""
from __future__ import annotations

import numpy as np

from . import numerics as nm
from .estimator import OracleEstimator, Params, Result


class Observation:
    """Observed indices n_m and weights phi_m of Phi (footnote of Sec. IV)."""

    def __init__(self, N: int, idx, phi=None):
        self.N = int(N)
        self.idx = np.asarray(idx, dtype=np.int64)
        if self.idx.ndim != 1 or len(self.idx) == 0:
            raise ValueError("idx must be a non-empty 1-D index list")
        if np.any(np.diff(self.idx) <= 0) or self.idx[0] < 0 or self.idx[-1] >= self.N:
            raise ValueError("idx must be strictly increasing in [0, N)")
        self.M = len(self.idx)
        self.phi = (np.ones(self.M, np.complex128) if phi is None
                    else np.asarray(phi, dtype=np.complex128))
        if self.phi.shape != (self.M,) or np.any(self.phi == 0):
            raise ValueError("phi must hold M nonzero weights")

    def matrix(self) -> np.ndarray:
        """Phi as a dense M x N matrix."""
        P = np.zeros((self.M, self.N), np.complex128)
        P[np.arange(self.M), self.idx] = self.phi
        return P

    def A(self, theta) -> np.ndarray:
        """A(theta) = Phi Psi(theta) (M x K)."""
        return self.phi[:, None] * nm.steering(theta, self.N)[self.idx]

    def adjoint(self, v) -> np.ndarray:
        """Phi^H v: the N-vector with conj(phi_m) v_m at n_m and zeros elsewhere."""
        out = np.zeros(self.N, np.complex128)
        out[self.idx] = self.phi.conj() * np.asarray(v, dtype=np.complex128)
        return out


def covariance(obs: Observation, theta, gamma, beta: float) -> np.ndarray:
    """C = beta I_M + A Gamma A^H with A = Phi Psi (Sec. II-B, eq. py)."""
    A = obs.A(theta)
    C = (A * np.asarray(gamma, dtype=np.float64)[None, :]) @ A.conj().T
    C[np.diag_indices(obs.M)] += beta
    return C


def e_matrix(obs: Observation, F: nm.DenseFactor) -> np.ndarray:
    """E = Phi^H C^{-1} Phi (N x N), zero outside the observed rows and columns:
    [E]_{n_a, n_b} = conj(phi_a) [C^{-1}]_{ab} phi_b (each entry of the product
    has the one term of the observed pair)."""
    E = np.zeros((obs.N, obs.N), np.complex128)
    E[np.ix_(obs.idx, obs.idx)] = (obs.phi.conj()[:, None] * F.inverse()) * obs.phi[None, :]
    return E


def adjoint_rows(obs: Observation, V: np.ndarray) -> np.ndarray:
    """Phi^H V for an M x K matrix V (N x K, zero outside the observed rows)."""
    out = np.zeros((obs.N, V.shape[1]), np.complex128)
    out[obs.idx] = obs.phi.conj()[:, None] * V
    return out


def active_vectors(obs: Observation, F: nm.DenseFactor, w: np.ndarray, theta) -> dict:
    """q, r, u, s, t, v, x at the active frequencies (eqs. q-x with Phi)."""
    N = obs.N
    Psi = nm.steering(theta, N)
    d = nm.d_diag(N)
    X = adjoint_rows(obs, F.solve(obs.phi[:, None] * Psi[obs.idx]))   # Phi^H C^{-1} Phi Psi
    XD = adjoint_rows(obs, F.solve(obs.phi[:, None] * (d[:, None] * Psi)[obs.idx]))
    Pc = Psi.conj()
    return dict(
        q=Pc.T @ w,
        r=Pc.T @ (d * w),
        u=Pc.T @ (d * d * w),
        s=np.sum(Pc * X, axis=0),
        t=np.sum(Pc * d[:, None] * X, axis=0),
        v=np.sum(Pc * (d * d)[:, None] * X, axis=0),
        x=np.sum(Pc * d[:, None] * XD, axis=0),
    )


def omegas(obs: Observation, E: np.ndarray):
    """Diagonal sums of E, D E, D^2 E and D E D (eqs. omega_s-omega_x with
    C^{-1} replaced by E = Phi^H C^{-1} Phi), index i + N - 1."""
    d = nm.d_diag(obs.N)
    return (nm.diagonal_sums(E),
            nm.diagonal_sums(d[:, None] * E),
            nm.diagonal_sums((d ** 2)[:, None] * E),
            nm.diagonal_sums(d[:, None] * E * d[None, :]))


def beta_update_definition(y, obs: Observation, theta, gamma, beta_old: float,
                           eps_beta: float) -> float:
    """beta = max(eps, (tr(Sigma A^H A) + ||y - A mu||^2) / M), A = Phi Psi, with
    mu, Sigma from eqs. bmu / bSigma at beta_old (eq. betaUpdate)."""
    y = np.asarray(y, dtype=np.complex128)
    M = obs.M
    if len(theta) == 0:
        return max(eps_beta, float(np.vdot(y, y).real) / M)
    A = obs.A(theta)
    AhA = A.conj().T @ A
    Sigma = np.linalg.inv(AhA / beta_old + np.diag(1.0 / np.asarray(gamma, dtype=np.float64)))
    mu = Sigma @ (A.conj().T @ y) / beta_old
    tr = float(np.trace(Sigma @ AhA).real)
    res = y - A @ mu
    return max(eps_beta, (tr + float(np.vdot(res, res).real)) / M)


class EvaluationIncomplete:
    """All quantities of one evaluation at (theta, gamma, beta) for the
    observation y of `obs`.  ``w`` is the N-space vector Phi^H C^{-1} y (what
    eqs. q, r, u and the grid q^G transform); ``wM`` is C^{-1} y itself."""

    def __init__(self, y, obs: Observation, theta, gamma, beta: float):
        self.y = np.asarray(y, dtype=np.complex128)
        self.obs = obs
        self.N, self.M = obs.N, obs.M
        self.theta = np.array(theta, dtype=np.float64)
        self.gamma = np.array(gamma, dtype=np.float64)
        self.beta = float(beta)
        self.C = covariance(obs, self.theta, self.gamma, self.beta)
        self.F = nm.DenseFactor(self.C)
        self.wM = self.F.solve(self.y)
        self.yCy = float(np.vdot(self.y, self.wM).real)
        self.logdet = self.F.logdet
        self.w = obs.adjoint(self.wM)
        self._E = None
        self.act = active_vectors(obs, self.F, self.w, self.theta) if len(self.theta) else \
            {k: np.zeros(0, np.complex128) for k in "qrustvx"}
        self._om = None

    @property
    def E(self) -> np.ndarray:
        """Phi^H C^{-1} Phi (formed on first use)."""
        if self._E is None:
            self._E = e_matrix(self.obs, self.F)
        return self._E

    @property
    def omega(self):
        if self._om is None:
            self._om = omegas(self.obs, self.E)
        return self._om

    def grid(self, L: int):
        return nm.grid_q(self.w, L), nm.grid_s(self.omega[0], L)

    def grid_derivatives(self, L: int):
        return nm.grid_r(self.w, L), nm.grid_t(self.omega[1], L)

    def f(self, K: int, zeta: float) -> float:
        """eq. obj with K_max = M."""
        return nm.objective(self.logdet, self.yCy, K, self.M, zeta)


class OracleEstimatorIncomplete(OracleEstimator):
    """The estimator of Sec. II-C/E on incomplete observations: the same
    block-coordinate descent, activation schemes, L-BFGS and final refinement,
    with C, q..x and the grid from their definitions under Phi, and the count
    scales of Sec. II-E (the initial beta, eps_beta, the stopping rules, K_max,
    eq. zetaUpdate) in the number of observations M."""

    def __init__(self, y, obs: Observation, params: Params | None = None,
                 check_blocks: bool = False):
        super().__init__(y, params, check_blocks)
        if self.y.shape != (obs.M,):
            raise ValueError("y must hold one entry per observed index")
        self.obs = obs
        self.N, self.M = obs.N, obs.M
        self.L = self.p.grid_size(self.N)
        self.kcap = self.M if self.p.kcap <= 0 else min(self.p.kcap, self.M)

    def _new_eval(self, theta, gamma, beta):
        return EvaluationIncomplete(self.y, self.obs, theta, gamma, beta)

    def _beta_update(self, theta, gamma, beta, eps_beta) -> float:
        return beta_update_definition(self.y, self.obs, theta, gamma, beta, eps_beta)


def estimate(y, idx, N: int, phi=None, params: Params | None = None,
             check_blocks: bool = False) -> Result:
    """Estimate from the samples y observed at indices idx (weights phi, default 1)
    of a length-N signal."""
    return OracleEstimatorIncomplete(y, Observation(N, idx, phi), params, check_blocks).run()
