"""Superfast-LSE estimator driver on top of the dense oracle numerics.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows the block-coordinate descent of Sec. II-C/E step by step:

  1. activation (Sec. II-D "Component Activation"; the approximate scheme of
     Sec. II-F for the first iterations),
  2. zeta update (eq. zetaUpdate),
  3. beta update (eq. betaUpdate, mu and Sigma by eqs. bmu / bSigma),
  4. up to 5 x { one L-BFGS step on (theta, gamma) with a diagonal-Hessian
     initialisation (Sec. II-D), deactivation by eq. deactivate },
  stop when the objective changes by less than M * 1e-7 between iterations
  (M observations; M = N for complete data),

followed by a final Newton-type polish of (theta, gamma) with z, beta, zeta
held fixed (:meth:`OracleEstimator._polish`).  The paper leaves several points
open; each reading taken here is a field of :class:`Params`.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import numerics as nm


@dataclass
class Params:
    L_mult: float = 8.0          # L = 2^round(log2(L_mult N)) (footnote, Sec. II-F)
    tau: float = 5.0             # eq. activate_criterion
    lbfgs_J: int = 10            # L-BFGS memory (Sec. II-D)
    max_inner: int = 5           # step 4 repetitions (Sec. II-E)
    max_outer: int = 200
    tol_obj: float = 1e-7        # |L_i - L_{i-1}| < M tol_obj (Sec. II-E)
    tol_newton: float = 1e-8     # squared Newton decrement < M tol_newton (Sec. II-E)
    eps_beta_rel: float = 1e-10  # eps_beta = eps_beta_rel ||y||^2 / M
    eps_L: float = 2.220446049250313e-16
    approx_max_iters: int = 10   # iterations that may use the approximate scheme
    approx_use_tau: bool = False  # Sec. II-F cites eq. activate_derived (no tau)
    approx_ratio: float = 5.0    # Delta L <= Delta L_min / 5
    approx_min_dist: float = 0.05  # wrap distance >= 0.05 / N
    ls_c1: float = 1e-4
    ls_max: int = 30
    curv_eps: float = 1e-12
    polish_max_iters: int = 30
    polish_tol: float = 1e-12    # polish converged when max |dtheta| < polish_tol / N
    polish_ftol: float = 1e-13   # rounding level of the objective, relative to 1 + |f|
    kcap: int = 0                # 0: K_max = M

    def grid_size(self, N: int) -> int:
        return int(2 ** int(round(math.log2(self.L_mult * N))))


STATUS_OK = 0
STATUS_NOTCONV = 1
STATUS_ECAPACITY = -5


@dataclass
class Result:
    K: int
    theta: np.ndarray
    alpha: np.ndarray
    gamma: np.ndarray
    beta: float
    zeta: float
    objective: float
    iterations: int
    evaluations: int
    status: int
    trace: list = field(default_factory=list)
    margins: list = field(default_factory=list)


class _Memory:
    """L-BFGS curvature pairs (Nocedal & Wright, Alg. 7.4) with a diagonal H0."""

    def __init__(self, J: int):
        self.J = J
        self.S: list[np.ndarray] = []
        self.Y: list[np.ndarray] = []

    def reset(self):
        self.S.clear()
        self.Y.clear()

    def push(self, s, y, eps):
        sy = float(np.dot(s, y))
        if sy > eps * float(np.linalg.norm(s)) * float(np.linalg.norm(y)):
            self.S.append(s.copy())
            self.Y.append(y.copy())
            if len(self.S) > self.J:
                self.S.pop(0)
                self.Y.pop(0)

    def direction(self, g, h):
        qv = g.copy()
        alphas = []
        for s, y in zip(reversed(self.S), reversed(self.Y)):
            rho = 1.0 / float(np.dot(y, s))
            a = rho * float(np.dot(s, qv))
            alphas.append((a, rho))
            qv = qv - a * y
        r = qv / h
        for (s, y), (a, rho) in zip(zip(self.S, self.Y), reversed(alphas)):
            b = rho * float(np.dot(y, r))
            r = r + (a - b) * s
        return -r


class OracleEstimator:
    def __init__(self, y, params: Params | None = None, check_blocks: bool = False):
        self.check_blocks = check_blocks
        self.y = np.asarray(y, dtype=np.complex128)
        self.N = self.y.shape[-1]
        # observations per vector (Sec. II-A: y has M entries; M = N for
        # complete data).  The count scales of Sec. II-E (the initial beta,
        # the stopping rules, K_max = M, eq. zetaUpdate) are in M; the
        # frequency scales (grid, distances, the polish's tolerance) in N.
        self.M = self.N
        self.G = 1              # observation vectors (Sec. V); 1 = the SMV model
        self.p = params or Params()
        self.L = self.p.grid_size(self.N)
        self.kcap = self.M if self.p.kcap <= 0 else min(self.p.kcap, self.M)
        self.n_evals = 0
        self.cap_hit = False
        self.trace: list = []
        # (kind, site, outer iteration, relative margin) of every comparison that
        # takes a discrete decision of the trajectory; a record only, it
        # changes nothing that is computed
        self.margins: list = []
        self._it = 0

    def _margin(self, kind, site, a, b, scale=None):
        """Record how far a decision's two compared values are apart, relative
        to their magnitude (or to `scale`).  Kinds: 'grid' (a ranking of grid
        points, taken in the grid's precision), 'fp64' (every other decision);
        `site` names the test."""
        a, b = float(a), float(b)
        den = scale if scale is not None else max(abs(a), abs(b))
        if not (math.isfinite(a) and math.isfinite(b)) or den == 0.0:
            return
        self.margins.append((kind, site, self._it, abs(a - b) / den))

    # ------------------------------------------------------------------
    def _block(self, name, before, after):
        """Debug aid: objective before/after a block update (each a tuple
        (theta, gamma, beta, zeta)); recorded only with check_blocks."""
        if not self.check_blocks:
            return
        fb, fa = (self._new_eval(t, g, b).f(len(t), z) for (t, g, b, z) in (before, after))
        self.trace.append(("block", name, fb, fa))

    # -- the steps that depend on the observation (the MMV model of Sec. V
    #    overrides them; everything else is shared) ---------------------------
    def _new_eval(self, theta, gamma, beta):
        return nm.Evaluation(self.y, theta, gamma, beta)

    def _energy(self) -> float:
        """||y||^2 (initial beta and the beta floor, Sec. II-E)."""
        return float(np.vdot(self.y, self.y).real)

    def _q_at(self, ev, theta):
        return nm.q_at(ev.w, theta)

    def _qq(self, q) -> float:
        """|q|^2 of one point (the left-hand side of eq. activate_criterion times s)."""
        return abs(q) ** 2

    def _criterion(self, q, s, gb, zeta, tau) -> bool:
        return bool(nm.activation_criterion(q, s, gb, zeta, tau))

    def _grad_hess(self, ev, gamma):
        gth, gga = nm.gradient(gamma, ev.act)
        hth, hga = nm.hessian_diag(gamma, ev.act)
        return gth, gga, hth, hga

    def _beta_update(self, theta, gamma, beta, eps_beta) -> float:
        return nm.beta_update_definition(self.y, theta, gamma, beta, eps_beta)

    def _deact_margins(self, ev, gamma, zeta):
        return nm.deactivation_margin(ev.act["q"], ev.act["s"].real, gamma, zeta)

    def _alpha(self, ev, gamma):
        return gamma * ev.act["q"]

    def evaluate(self, theta, gamma, beta) -> nm.Evaluation:
        self.n_evals += 1
        return self._new_eval(theta, gamma, beta)

    def _derivs(self, ev: nm.Evaluation, gamma):
        gth, gga, hth, hga = self._grad_hess(ev, gamma)
        N = self.N
        hth = np.where(hth > 0, hth, (50.0 * N) ** 2)
        safe_g = np.where(gamma > 0, gamma, 1.0)
        hga = np.where(hga > 0, hga, safe_g ** -2.0)
        return np.concatenate([gth, gga]), np.concatenate([hth, hga])

    def _gbar(self, gamma):
        return float(np.mean(gamma)) if len(gamma) else None

    def _decision_quantities(self, q, s, gamma, zeta):
        """(gbar used, gamma_hat, Delta L) at one point."""
        gh = float(nm.gamma_hat(q, s))
        gb = self._gbar(gamma)
        if gb is None:       # empty active set: per-theta optimum (reading R4)
            gb = gh
        dl = float(nm.delta_L(q, s, gb, zeta))
        return gb, gh, dl

    def _grid_delta_L(self, ev: nm.Evaluation, gamma, zeta):
        qG, sG = ev.grid(self.L)
        gb = self._gbar(gamma)
        if gb is None:
            gbv = nm.gamma_hat(qG, sG)
        else:
            gbv = np.full(self.L, gb)
        return qG, sG, nm.delta_L(qG, sG, gbv, zeta)

    # ------------------------------------------------------------------
    def _exact_activation_round(self, ev, theta, gamma, zeta):
        """One pass of step 1: argmin of Delta L on the grid, accept or stop."""
        p = self.p
        qG, sG, dl = self._grid_delta_L(ev, gamma, zeta)
        l = int(np.argmin(dl))                       # lowest index on ties
        th = l / self.L
        q = self._q_at(ev, [th])[..., 0]
        q = complex(q) if q.ndim == 0 else q
        s = float(nm.s_at(ev.omega[0], [th])[0])
        gb, gh, dlv = self._decision_quantities(q, s, gamma, zeta)
        ok = (gh > 0 and zeta > 0
              and self._criterion(q, s, gb, zeta, p.tau) and dlv < -p.eps_L)
        self._record_grid_argmin(dl)
        self._record_activation(q, s, gb, zeta, p.tau, dlv)
        self.trace.append(("exact", l, dlv, ok))
        if ok and len(theta) >= self.kcap:
            self.cap_hit = True
            return None
        if ok:
            return th, gh
        return None

    def _record_grid_argmin(self, dl):
        dlf = dl[np.isfinite(dl)]
        if len(dlf) > 1:
            two = np.partition(dlf, 1)[:2]
            self._margin("grid", "argmin", two[0], two[1], float(np.max(np.abs(dlf))))

    def _record_activation(self, q, s, gb, zeta, tau, dlv):
        if not (zeta > 0 and s > 0 and gb > 0):
            return
        kappa = self._qq(q) / s
        lg = math.log((1.0 + gb * s) * ((1.0 - zeta) / zeta))
        rhs = self._criterion_rhs(s, gb, zeta, tau)
        self._margin("fp64", "criterion", kappa, rhs)
        self._margin("fp64", "gamma_hat", kappa, 1.0)               # gamma_hat > 0
        self._margin("fp64", "delta_L", dlv, -self.p.eps_L, 1.0 + abs(lg))

    def _criterion_rhs(self, s, gb, zeta, tau):
        return (1.0 + 1.0 / (gb * s)) * math.log((1.0 + gb * s) * ((1.0 - zeta) / zeta)) + tau

    def _approx_activation(self, ev, theta, gamma, zeta):
        """Approximate scheme of Sec. II-F: all local minima of Delta L passing 4 filters."""
        p = self.p
        N, L = self.N, self.L
        qG, sG, dl = self._grid_delta_L(ev, gamma, zeta)
        lmin = int(np.argmin(dl))
        locmin = local_minima(dl)
        th_all = np.concatenate([[lmin / L], locmin / L])
        q_all = self._q_at(ev, th_all)
        s_all = nm.s_at(ev.omega[0], th_all)
        _, _, dl_min = self._decision_quantities(q_all[..., 0], s_all[0], gamma, zeta)
        tau = p.tau if p.approx_use_tau else 0.0
        dls, ghs, oks = [], [], []
        for j in range(len(locmin)):
            q, s = q_all[..., j + 1], s_all[j + 1]
            gb, gh, dlv = self._decision_quantities(q, s, gamma, zeta)
            dls.append(dlv)
            ghs.append(gh)
            oks.append(gh > 0 and zeta > 0 and self._criterion(q, s, gb, zeta, tau))
        new_th, new_g, cap = approx_select(dl_min, locmin, dls, ghs, oks, theta, N, L,
                                           p.approx_ratio, p.approx_min_dist,
                                           self.kcap - len(theta))
        self._record_grid_argmin(dl)
        big = float(np.max(np.abs(dl[np.isfinite(dl)]))) if np.any(np.isfinite(dl)) else 1.0
        for j, l in enumerate(locmin):
            q, s = q_all[..., j + 1], float(s_all[j + 1].real)
            gb, _, _ = self._decision_quantities(q, s, gamma, zeta)
            if dls[j] <= 0.5 * dl_min / p.approx_ratio or oks[j]:
                # local-minimum tests of the grid points that could be chosen
                self._margin("grid", "local_min", dl[l], min(dl[(l - 1) % L], dl[(l + 1) % L]), big)
                self._record_activation(q, s, gb, zeta, tau, dls[j])
                self._margin("fp64", "ratio", dls[j], dl_min / p.approx_ratio)
        for th in new_th:
            others = np.concatenate([np.asarray(theta, np.float64),
                                     np.asarray([t for t in new_th if t != th], np.float64)])
            if len(others):
                self._margin("fp64", "distance", float(np.min(nm_wrap(th, others))) * N, p.approx_min_dist)
        self.cap_hit = self.cap_hit or cap
        self.trace.append(("approx", len(locmin), int(sum(oks)), len(new_th)))
        return new_th, new_g

    # ------------------------------------------------------------------
    @staticmethod
    def _step_limit(gamma, dga):
        """Largest step keeping every gamma >= 0, and the first k that reaches it."""
        neg = dga < 0
        if not np.any(neg):
            return math.inf, -1
        ratios = np.where(neg, gamma / np.where(neg, -dga, 1.0), math.inf)
        kstar = int(np.argmin(ratios))
        return float(ratios[kstar]), kstar

    def _line_search(self, ev, theta, gamma, beta, K, zeta, g, d):
        """Backtracking Armijo search of an inner L-BFGS step (Sec. II-D; gamma kept >= 0)."""
        p = self.p
        f0 = ev.f(K, zeta)
        gd = float(np.dot(g, d))
        dth, dga = d[:K], d[K:]
        amax, kstar = self._step_limit(gamma, dga)
        alpha = min(1.0, amax)
        resolution = p.polish_ftol * (1.0 + abs(f0))
        for trial in range(p.ls_max):
            # the search gives up once the decrease it requires is below the
            # rounding level of the objective (the test would decide nothing)
            if trial > 0:
                self._margin("fp64", "ls_resolution", p.ls_c1 * alpha * abs(gd), resolution)
            if trial > 0 and p.ls_c1 * alpha * abs(gd) < resolution:
                return None
            th_t = np.mod(theta + alpha * dth, 1.0)
            ga_t = np.maximum(gamma + alpha * dga, 0.0)
            if alpha == amax and kstar >= 0:
                ga_t[kstar] = 0.0
            ev_t = self.evaluate(th_t, ga_t, beta)
            f_t = ev_t.f(K, zeta)
            self._margin("fp64", "armijo", f_t, f0 + p.ls_c1 * alpha * gd, 1.0 + abs(f0))
            if f_t <= f0 + p.ls_c1 * alpha * gd:
                return ev_t, th_t, ga_t, alpha
            alpha *= 0.5
        return None

    def _polish(self, cur, theta, gamma, beta, zeta):
        """Final Newton-type refinement of (theta, gamma) with z, beta, zeta fixed.

        The paper stops on the objective change (Sec. II-E), which leaves the
        frequencies determined only to the objective's flatness; this
        refinement drives them to a stationary point of eq. obj so that the
        result no longer depends on the trajectory.  Each step is the L-BFGS
        direction d (memory reset at the start, diagonal Hessian as H0); a
        trial point is accepted when it satisfies the Armijo condition, or,
        once the objective change is within its rounding level
        (polish_ftol (1 + |f|)), when it lowers the diagonal Newton decrement
        nu = sum_i g_i^2 / h_i (there the objective no longer resolves the
        step, the gradient still does).  The first trial is alpha = 1 (or half
        the step that zeroes a gamma), halved on rejection.  The refinement
        has converged when an accepted step moves no frequency by
        polish_tol / N, or when the trial step has been shortened below that
        without being accepted (the point is then left unchanged).
        """
        p, N = self.p, self.N
        mem = _Memory(p.lbfgs_J)
        tol = p.polish_tol / N
        for _pit in range(p.polish_max_iters):
            K = len(theta)
            if K == 0:
                break
            g, h = self._derivs(cur, gamma)
            d = self._direction(mem, g, h)
            nu0 = float(np.sum(g * g / h))
            f0 = cur.f(K, zeta)
            gd = float(np.dot(g, d))
            dth, dga = d[:K], d[K:]
            amax, _ = self._step_limit(gamma, dga)
            alpha = 1.0 if amax > 1.0 else 0.5 * amax
            dth_max = float(np.max(np.abs(dth)))
            slack = p.polish_ftol * (1.0 + abs(f0))
            acc = None
            for trial in range(p.ls_max):
                if trial > 0 and alpha * dth_max < tol:
                    break
                th_t = np.mod(theta + alpha * dth, 1.0)
                ga_t = np.maximum(gamma + alpha * dga, 0.0)
                ev_t = self.evaluate(th_t, ga_t, beta)
                f_t = ev_t.f(K, zeta)
                g_t, h_t = self._derivs(ev_t, ga_t)
                if f_t <= f0 + p.ls_c1 * alpha * gd or \
                        (f_t <= f0 + slack and float(np.sum(g_t * g_t / h_t)) < nu0):
                    acc = (ev_t, th_t, ga_t, g_t)
                    break
                alpha *= 0.5
            if acc is None:
                self.trace.append(("polish_stop", _pit, alpha * dth_max * N))
                break
            ev_t, th_t, ga_t, g_t = acc
            mem.push(alpha * d, g_t - g, p.curv_eps)
            theta, gamma, cur = th_t, ga_t, ev_t
            if alpha * dth_max < tol:
                break
        return cur, theta, gamma

    def _direction(self, mem, g, h):
        d = mem.direction(g, h)
        if not np.all(np.isfinite(d)) or float(np.dot(g, d)) >= 0.0:
            mem.reset()
            d = -g / h
        return d

    # ------------------------------------------------------------------
    def run(self) -> Result:
        p, M, G = self.p, self.M, self.G
        yy = self._energy()
        if yy == 0.0:
            return Result(0, np.zeros(0), np.zeros(0, np.complex128), np.zeros(0), 0.0, 0.0,
                          -math.inf, 0, 0, STATUS_OK)
        beta = 0.01 * yy / M                      # initialisation (Sec. II-E)
        zeta = 0.2
        eps_beta = p.eps_beta_rel * yy / M
        theta = np.zeros(0)
        gamma = np.zeros(0)
        approx_on = p.approx_max_iters > 0
        L_prev = math.inf
        mem = _Memory(p.lbfgs_J)
        z_changed = True
        cur = None
        it = 0
        converged = False

        def ensure(ev):
            return ev if ev is not None else self.evaluate(theta, gamma, beta)

        for it in range(1, p.max_outer + 1):
            self._it = it
            # ---- step 1: activation ------------------------------------
            run_exact = True
            if approx_on and it <= p.approx_max_iters:
                cur = ensure(cur)
                new_th, new_g = self._approx_activation(cur, theta, gamma, zeta)
                if new_th:
                    self._block("approx", (theta, gamma, beta, zeta),
                                (np.concatenate([theta, new_th]), np.concatenate([gamma, new_g]),
                                 beta, zeta))
                    theta = np.concatenate([theta, new_th])
                    gamma = np.concatenate([gamma, new_g])
                    cur = None
                    z_changed = True
                    run_exact = False
                else:
                    approx_on = False
            if run_exact:
                while True:
                    cur = ensure(cur)
                    got = self._exact_activation_round(cur, theta, gamma, zeta)
                    if got is None:
                        break
                    self._block("activate", (theta, gamma, beta, zeta),
                                (np.append(theta, got[0]), np.append(gamma, got[1]), beta, zeta))
                    theta = np.append(theta, got[0])
                    gamma = np.append(gamma, got[1])
                    cur = None
                    z_changed = True
            K = len(theta)
            # ---- step 2: zeta ------------------------------------------
            self._block("zeta", (theta, gamma, beta, zeta), (theta, gamma, beta, min(0.5, K / M)))
            zeta = min(0.5, K / M)
            # ---- step 3: beta (EM bound) ----------------------------------
            beta_new = self._beta_update(theta, gamma, beta, eps_beta)
            self._block("beta", (theta, gamma, beta, zeta), (theta, gamma, beta_new, zeta))
            if beta_new != beta:
                beta = beta_new
                cur = None
            # ---- step 4: L-BFGS + deactivation ---------------------------
            if z_changed:
                mem.reset()
                z_changed = False
            for _inner in range(p.max_inner):
                K = len(theta)
                if K == 0:
                    break
                cur = ensure(cur)
                g, h = self._derivs(cur, gamma)
                d = self._direction(mem, g, h)
                lam2 = -float(np.dot(g, d))
                ls = self._line_search(cur, theta, gamma, beta, K, zeta, g, d)
                if ls is None:
                    self.trace.append(("ls_fail", it))
                    break
                ev_t, th_t, ga_t, alpha = ls
                g_t, _ = self._derivs(ev_t, ga_t)
                mem.push(alpha * d, g_t - g, p.curv_eps)
                self._block("lbfgs", (theta, gamma, beta, zeta), (th_t, ga_t, beta, zeta))
                theta, gamma, cur = th_t, ga_t, ev_t
                # 4b: deactivation, one component at a time (largest margin first)
                while len(theta) > 0:
                    marg = self._deact_margins(cur, gamma, zeta)
                    k = int(np.argmax(marg))
                    if math.isfinite(marg[k]):
                        self._margin("fp64", "deactivate", marg[k], 0.0,
                                     max(1.0, abs(math.log((1.0 - zeta) / zeta))))
                    if not marg[k] > 0:
                        break
                    self.trace.append(("deact", it, float(theta[k])))
                    self._block("deact", (theta, gamma, beta, zeta),
                                (np.delete(theta, k), np.delete(gamma, k), beta, zeta))
                    theta = np.delete(theta, k)
                    gamma = np.delete(gamma, k)
                    mem.reset()
                    cur = ensure(None)
                self._margin("fp64", "decrement", lam2, G * M * p.tol_newton)
                if lam2 < G * M * p.tol_newton:
                    break
            # ---- termination ---------------------------------------------
            K = len(theta)
            cur = ensure(cur)
            L_cur = cur.f(K, zeta)
            self.trace.append(("iter", it, K, L_cur, beta))
            if math.isfinite(L_prev):
                self._margin("fp64", "terminate", abs(L_cur - L_prev), G * M * p.tol_obj,
                             1.0 + abs(L_cur))
            if abs(L_cur - L_prev) < G * M * p.tol_obj:
                converged = True
                break
            L_prev = L_cur

        # ---- final polish of (theta, gamma) with z, beta, zeta fixed ---------
        cur, theta, gamma = self._polish(ensure(cur), theta, gamma, beta, zeta)

        K = len(theta)
        alpha_hat = self._alpha(cur, gamma) if K else np.zeros((self.G, 0)[-self.y.ndim:],
                                                                np.complex128)
        order = np.argsort(theta, kind="stable")
        status = STATUS_OK if converged else STATUS_NOTCONV
        if self.cap_hit:
            status = STATUS_ECAPACITY
        return Result(K, theta[order], alpha_hat[..., order], gamma[order], beta, zeta,
                      cur.f(K, zeta), it, self.n_evals, status, self.trace, self.margins)


def nm_wrap(x, arr):
    """Wrap-around distance on the unit circle between x and each entry of arr."""
    a = np.abs(np.asarray(arr, dtype=np.float64) - x) % 1.0
    return np.minimum(a, 1.0 - a)


def local_minima(dl) -> np.ndarray:
    """Grid indices l with dl[l] <= dl[l-1] and dl[l] <= dl[l+1], indices taken
    cyclically (the grid covers the unit circle; Sec. II-F)."""
    dl = np.asarray(dl)
    return np.nonzero((dl <= np.roll(dl, 1)) & (dl <= np.roll(dl, -1)))[0]


def approx_select(dl_min, cand_l, cand_dl, cand_gh, cand_ok, theta_active, N, L,
                  ratio=5.0, min_dist=0.05, room=None):
    """The filters of the approximate activation scheme (Sec. II-F) on the local
    minima of one grid sweep.

    dl_min          Delta L at the grid argmin (FP64 re-evaluation)
    cand_l          grid indices of the local minima
    cand_dl, cand_gh Delta L and gamma_hat at each (FP64)
    cand_ok         gamma_hat > 0, zeta > 0 and the activation criterion hold
    theta_active    frequencies active before the sweep
    room            components that may still be added (None: unlimited)

    A candidate qualifies when cand_ok holds and its Delta L <= dl_min / ratio.
    Qualifying candidates are taken by ascending (Delta L, grid index) and each
    is added unless its wrap distance to an active frequency, or to one already
    added in this sweep, is below min_dist / N.  Returns (thetas, gammas,
    capacity_hit)."""
    quals = sorted((float(d), int(l), float(g)) for d, l, g, ok in
                   zip(cand_dl, cand_l, cand_gh, cand_ok) if ok and d <= dl_min / ratio)
    new_th, new_g = [], []
    cap = False
    for dlv, l, gh in quals:
        if room is not None and len(new_th) >= room:
            cap = True
            break
        th = l / L
        others = np.concatenate([np.asarray(theta_active, dtype=np.float64),
                                 np.asarray(new_th, dtype=np.float64)])
        if len(others) == 0 or float(np.min(nm_wrap(th, others))) >= min_dist / N:
            new_th.append(th)
            new_g.append(gh)
    return new_th, new_g, cap


def estimate(y, params: Params | None = None, check_blocks: bool = False) -> Result:
    return OracleEstimator(y, params, check_blocks).run()
