"""Host checks of the whole-estimate matching rules (tests/parity.py): the
classification into match / ambiguous / mismatch, on oracle results."""
from types import SimpleNamespace

import numpy as np
import pytest

from oracle.estimator import Params, estimate
from paper_1705_06073_amd import synth
from tests import parity


@pytest.fixture(scope="module")
def ref():
    inst = synth.workload_n64(0)
    r = estimate(inst.y, Params(L_mult=4.0))
    return inst, r, parity.result_dict(r)


def as_got(r, **kw):
    d = dict(K=r.K, theta=np.array(r.theta), alpha=np.array(r.alpha), gamma=np.array(r.gamma),
             beta=r.beta, objective=r.objective)
    d.update(kw)
    return SimpleNamespace(**d)


def test_identical_results_match(ref):
    inst, r, d = ref
    assert parity.judge(d, as_got(r), inst.N, False).kind == "match"


def test_order_and_wrap_do_not_matter(ref):
    """Frequencies are matched one to one by wrap distance (Hungarian), so a
    permuted output, or one whose frequency wrapped across 0, still matches."""
    inst, r, d = ref
    perm = np.arange(r.K)[::-1]
    th = np.array(r.theta)[perm]
    th[0] = th[0] - 1.0 if th[0] > 0.5 else th[0]   # same point on the circle
    th = np.mod(th, 1.0)
    got = as_got(r, theta=th, alpha=np.array(r.alpha)[perm], gamma=np.array(r.gamma)[perm])
    assert parity.judge(d, got, inst.N, False).kind == "match"


def test_frequency_outside_tolerance_is_a_mismatch(ref):
    inst, r, d = ref
    th = np.array(r.theta)
    th[1] += 3e-9 / inst.N
    d_far = dict(d, margins_z=[], margins_grid=[], margins_path=[])
    v = parity.judge(d_far, as_got(r, theta=th), inst.N, False)
    assert v.kind == "mismatch" and "dtheta" in v.detail
    th[1] -= 2.5e-9 / inst.N          # 0.5e-9/N away: inside the rule
    assert parity.judge(d_far, as_got(r, theta=th), inst.N, False).kind == "match"


def test_model_order_difference_is_a_mismatch_without_a_near_tie(ref):
    inst, r, d = ref
    got = as_got(r, K=r.K - 1, theta=np.array(r.theta)[1:], alpha=np.array(r.alpha)[1:],
                 gamma=np.array(r.gamma)[1:])
    d_far = dict(d, margins_z=[["fp64", "criterion", 2, 1e-3]], margins_grid=[],
                 margins_path=[])
    assert parity.judge(d_far, got, inst.N, True).kind == "mismatch"
    d_tie = dict(d_far, margins_z=[["fp64", "criterion", 2, 3e-11]])
    v = parity.judge(d_tie, got, inst.N, True)
    assert v.kind == "ambiguous" and v.site == "criterion" and v.margin == 3e-11


def test_grid_rank_threshold_follows_the_grid_precision(ref):
    """A near tie of two grid points at 5e-5 (relative) excuses a difference
    when the grid was FP32, not when it was FP64."""
    inst, r, d = ref
    got = as_got(r, beta=r.beta * (1 + 1e-6))
    d_g = dict(d, margins_z=[], margins_path=[], margins_grid=[["grid", "argmin", 1, 5e-5]])
    assert parity.judge(d_g, got, inst.N, True).kind == "ambiguous"
    assert parity.judge(d_g, got, inst.N, False).kind == "mismatch"


def test_oracle_records_margins_of_each_decision_class(ref):
    """The oracle's run records margins of activation decisions, grid rankings
    and the line search, and the last active-set change is inside the run."""
    inst, r, d = ref
    sites = {m[1] for m in r.margins}
    assert {"criterion", "argmin", "armijo", "terminate"} <= sites
    assert all(m[3] >= 0 for m in r.margins)
    lz = parity.last_z_change(r.trace)
    assert 1 <= lz <= r.iterations
    assert all(m[2] <= lz for m in d["margins_path"])


def test_flat_objective_rule(ref):
    """A frequency difference is ambiguous when the oracle at the HIP point has
    the same objective within its rounding level and no resolvable Newton step;
    otherwise (a larger objective, or a gradient left) it is a mismatch."""
    inst, r, d = ref
    th = np.array(r.theta)
    th[0] += 5e-9 / inst.N
    d_far = dict(d, margins_z=[], margins_grid=[], margins_path=[])
    got = as_got(r, theta=th, zeta=r.zeta)
    f0 = r.objective
    v = parity.judge(d_far, got, inst.N, False, flat=lambda g: (f0 + 1e-14 * abs(f0), 1e-20))
    assert v.kind == "ambiguous" and v.site == "flat_objective"
    v = parity.judge(d_far, got, inst.N, False, flat=lambda g: (f0 + 1e-9 * abs(f0), 1e-20))
    assert v.kind == "mismatch"
    v = parity.judge(d_far, got, inst.N, False, flat=lambda g: (f0, 1e-6))
    assert v.kind == "mismatch"
    # the oracle's own evaluation at a genuinely displaced point is not flat
    th[0] += 1e-3 / inst.N
    assert parity.judge(d_far, as_got(r, theta=th, zeta=r.zeta), inst.N, False,
                        flat=parity.oracle_flat(inst.y, oe_params())).kind == "mismatch"


def oe_params():
    from oracle.estimator import Params
    return Params(L_mult=4.0)
