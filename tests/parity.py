"""Matching rules for whole estimates (test tooling, no GPU needed).

A HIP estimate matches the oracle's when the model order is identical, the
frequencies agree within 1e-9/N after matching them one to one by the
smallest squared wrap distances (Hungarian), and the component variances,
amplitudes, noise variance and objective agree at relative tolerances that
follow from the frequencies' agreement.

A result that differs is *ambiguous* rather than failed when the oracle's
trajectory took a decision whose two compared sides were closer than the
rounding by which the two implementations may differ:

  * decisions that choose the active set (activation criterion, gamma_hat > 0,
    Delta L < -eps_L, the approximate scheme's Delta L_min ratio and distance
    filters, deactivation) or end the outer loop: relative margin below 1e-9;
  * decisions of the continuous path (Armijo tests, the line search's
    resolution test, the squared Newton decrement) taken up to the last change
    of the active set: below 1e-9 (later ones only move the point inside the
    final refinement's basin, which converges to the same stationary point);
  * rankings of grid points (the argmin and the local minima of Delta L):
    below 1e-9 when the grid is FP64, below 1e-4 when it is FP32 (the FP32
    grid objective's own tolerance, norm-wise relative).

The margins are those the oracle records while it runs (``Result.margins``,
stored by ``tests/golden/make_estimate_golden.py`` for the large cases).

A difference confined to the continuous parameters (same model order) is also
ambiguous when the objective cannot tell the two points apart: evaluated by
the oracle at the HIP point, the objective equals the oracle's own within
10 x its rounding level (1e-13 (1 + |L|), the level at which the final
refinement stops judging steps by the objective), and the decrease a Newton
step from there predicts (half the diagonal Newton decrement) is within the
same 10 x.  This is the flat valley of nearly coincident components (pairs
closer than 1/N), where the refinement of either side stops at a different
point of a set on which FP64 cannot separate the objective's values.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from tests import metrics

THETA_TOL = 1e-9       # frequencies: |dtheta| < THETA_TOL / N
GAMMA_RTOL = 1e-6      # relative to the largest gamma of the instance
ALPHA_RTOL = 1e-6      # relative to the largest |alpha| of the instance
BETA_RTOL = 1e-8
OBJ_RTOL = 1e-8        # relative to max(1, |objective|)
FP64_AMBIG = 1e-9
F_RESOLUTION = 1e-13   # rounding level of the objective, relative to 1 + |L|
GRID_AMBIG_FP64 = 1e-9
GRID_AMBIG_FP32 = 1e-4

Z_SITES = ("criterion", "gamma_hat", "delta_L", "ratio", "distance", "deactivate", "terminate")


@dataclass
class Verdict:
    kind: str                 # "match", "ambiguous" or "mismatch"
    detail: str
    margin: float | None = None
    site: str | None = None


def theta_error(theta_ref, theta_got):
    """(largest wrap distance between matched frequencies, (ref index, got
    index) of the matching); (inf, None) if the counts differ."""
    a, b = np.asarray(theta_ref, np.float64), np.asarray(theta_got, np.float64)
    if len(a) != len(b):
        return np.inf, None
    if len(a) == 0:
        return 0.0, (np.zeros(0, int), np.zeros(0, int))
    r, c = metrics.match(a, b)
    return float(np.max(metrics.wrap_distance(a[r], b[c]))), (r, c)


def margins_of(ref: dict):
    """(site, margin) triples of the oracle's decisions in the three classes."""
    return ref.get("margins_z", []), ref.get("margins_grid", []), ref.get("margins_path", [])


def near_tie(ref: dict, grid_fp32: bool):
    """The closest decision of the oracle's trajectory within the ambiguity
    thresholds, as (site, margin), or None."""
    mz, mg, mp = margins_of(ref)
    thr_g = GRID_AMBIG_FP32 if grid_fp32 else GRID_AMBIG_FP64
    cands = [(m[1], m[3], m[3] / FP64_AMBIG) for m in mz + mp if m[3] < FP64_AMBIG]
    cands += [(m[1], m[3], m[3] / thr_g) for m in mg if m[3] < thr_g]
    if not cands:
        return None
    site, margin, _ = min(cands, key=lambda c: c[2])
    return site, margin


def judge(ref: dict, got, N: int, grid_fp32: bool, flat=None) -> Verdict:
    """Compare a HIP estimate `got` (attributes K, theta, alpha, gamma, beta,
    objective) with the oracle's `ref` (a dict with the same keys, alpha split
    into alpha_re / alpha_im, plus the margin lists).  `flat` (optional):
    got -> (objective, diagonal Newton decrement) of the oracle at got's point,
    for the flat-objective rule above."""
    problems = []
    if got.K != ref["K"]:
        problems.append(f"K {got.K} != {ref['K']}")
    else:
        K = got.K
        if K:
            te, (r, c) = theta_error(ref["theta"], got.theta)
            if not te < THETA_TOL / N:
                problems.append(f"max|dtheta|*N = {te * N:.3e}")
            g_ref = np.asarray(ref["gamma"])[r]
            a_ref = (np.asarray(ref["alpha_re"]) + 1j * np.asarray(ref["alpha_im"]))[r]
            g_got, a_got = np.asarray(got.gamma)[c], np.asarray(got.alpha)[c]
            eg = np.max(np.abs(g_got - g_ref)) / np.max(np.abs(g_ref))
            ea = np.max(np.abs(a_got - a_ref)) / np.max(np.abs(a_ref))
            if not eg < GAMMA_RTOL:
                problems.append(f"gamma rel {eg:.2e}")
            if not ea < ALPHA_RTOL:
                problems.append(f"alpha rel {ea:.2e}")
        eb = abs(got.beta - ref["beta"]) / abs(ref["beta"])
        eo = abs(got.objective - ref["objective"]) / max(1.0, abs(ref["objective"]))
        if not eb < BETA_RTOL:
            problems.append(f"beta rel {eb:.2e}")
        if not eo < OBJ_RTOL:
            problems.append(f"objective rel {eo:.2e}")
    if not problems:
        return Verdict("match", "")
    tie = near_tie(ref, grid_fp32)
    if tie is not None:
        return Verdict("ambiguous", "; ".join(problems), tie[1], tie[0])
    if flat is not None and got.K == ref["K"]:
        f_got, nu_got = flat(got)
        res = F_RESOLUTION * (1.0 + abs(ref["objective"]))
        df = abs(f_got - ref["objective"])
        detail = "; ".join(problems) + f"; oracle at the HIP point: |dL| = {df:.2e}, nu = {nu_got:.2e}"
        if df <= 10.0 * res and 0.5 * nu_got <= 10.0 * res:
            return Verdict("ambiguous", detail, df / (1.0 + abs(ref["objective"])),
                           "flat_objective")
        return Verdict("mismatch", detail)
    return Verdict("mismatch", "; ".join(problems))


def oracle_flat(y, params=None):
    """The `flat` callable of judge for observation y: the oracle's objective and
    diagonal Newton decrement (sum g_i^2 / h_i, the refinement's measure) at a
    HIP estimate's point."""
    import numpy as np
    from oracle.estimator import OracleEstimator, Params

    def f(got):
        est = OracleEstimator(np.asarray(y, np.complex128), params or Params())
        th, ga = np.asarray(got.theta, np.float64), np.asarray(got.gamma, np.float64)
        ev = est.evaluate(th, ga, got.beta)
        g, h = est._derivs(ev, ga)
        return ev.f(len(th), got.zeta), float(np.sum(g * g / h))
    return f


def oracle_flat_incomplete(y, obs, params=None):
    """oracle_flat for incomplete observations (obs: oracle.incomplete.Observation)."""
    import numpy as np
    from oracle.estimator import Params
    from oracle.incomplete import OracleEstimatorIncomplete

    def f(got):
        est = OracleEstimatorIncomplete(np.asarray(y, np.complex128), obs, params or Params())
        th, ga = np.asarray(got.theta, np.float64), np.asarray(got.gamma, np.float64)
        ev = est.evaluate(th, ga, got.beta)
        g, h = est._derivs(ev, ga)
        return ev.f(len(th), got.zeta), float(np.sum(g * g / h))
    return f


def last_z_change(trace) -> int:
    """Last outer iteration in which the oracle's active set changed (an
    activation or a deactivation), from its trace; 0 if it never did."""
    last, it = 0, 1
    for rec in trace:
        if rec[0] == "iter":
            it = rec[1] + 1
        elif rec[0] == "deact":
            last = max(last, rec[1])
        elif (rec[0] == "exact" and rec[3]) or (rec[0] == "approx" and rec[3] > 0):
            last = max(last, it)
    return last


def result_dict(r) -> dict:
    """An oracle Result as the dict `judge` takes (margins classified as the
    golden file stores them)."""
    ms = r.margins
    last_z = last_z_change(r.trace)
    mz = [m for m in ms if m[0] == "fp64" and m[1] in Z_SITES]
    mg = [m for m in ms if m[0] == "grid"]
    mp = [m for m in ms if m[0] == "fp64" and m[1] not in Z_SITES and m[2] <= last_z]
    return {"K": r.K, "theta": list(r.theta), "gamma": list(r.gamma),
            "alpha_re": list(np.real(r.alpha)), "alpha_im": list(np.imag(r.alpha)),
            "beta": r.beta, "objective": r.objective,
            "margins_z": [list(m) for m in mz], "margins_grid": [list(m) for m in mg],
            "margins_path": [list(m) for m in mp]}
