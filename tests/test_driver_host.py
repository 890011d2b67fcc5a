"""The device driver's control flow (a9), compiled for the host and fed by
oracle evaluations, reproduces the oracle estimator's result: same model
order, frequencies, amplitudes, noise variance and objective.  Its
evaluation count exceeds the oracle's by the evaluations the beta update of
Sec. II-D takes (the oracle evaluates that update from its definition
without counting it), at most one per outer iteration."""
import shutil

import numpy as np
import pytest

from oracle import estimator as oe
from paper_1705_06073_amd import synth

if shutil.which("g++") is None:  # pragma: no cover
    pytest.skip("g++ not available", allow_module_level=True)

from tests import host_driver as hd  # noqa: E402


def _instances():
    rng = np.random.default_rng(4242)
    out = []
    for N, K, snr in [(64, 3, 20.0), (96, 4, 10.0), (128, 5, 30.0), (200, 6, 15.0)]:
        out.append(synth.make_instance(rng, N, K, 1.0 / N, "cn", snr))
    return out


@pytest.mark.parametrize("idx", range(4))
def test_host_driver_matches_oracle(idx):
    inst = _instances()[idx]
    o = oe.estimate(inst.y)
    r = hd.HostDriver(inst.y).run()
    assert r["status"] == o.status
    assert r["K"] == o.K
    assert r["iterations"] == o.iterations
    np.testing.assert_allclose(r["theta"], o.theta, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["gamma"], o.gamma, rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(r["alpha"], o.alpha, rtol=1e-9, atol=1e-12)
    assert r["beta"] == pytest.approx(o.beta, rel=1e-9)
    assert r["zeta"] == pytest.approx(o.zeta, rel=1e-12)
    assert r["objective"] == pytest.approx(o.objective, rel=1e-10, abs=1e-9)
    assert o.evaluations <= r["evaluations"] <= o.evaluations + o.iterations + 1, \
        (o.evaluations, o.iterations, r["evaluations"])


def test_host_driver_zero_signal():
    r = hd.HostDriver(np.zeros(32, np.complex128)).run()
    assert r["K"] == 0 and r["beta"] == 0.0 and r["evaluations"] == 0


def test_host_driver_approximate_off_matches_oracle():
    inst = _instances()[2]
    p = oe.Params(approx_max_iters=0)
    o = oe.estimate(inst.y, p)
    r = hd.HostDriver(inst.y, p).run()
    assert r["K"] == o.K
    np.testing.assert_allclose(r["theta"], o.theta, rtol=0, atol=1e-12)


REQ_EVAL, REQ_GRID = 1, 2


@pytest.mark.parametrize("idx", range(4))
def test_grid_sweeps_at_the_evaluated_point_fit_the_evaluating_round(idx):
    """The device round runs a first driver pass over the requests without a
    grid sweep, then the grid stage and a second pass.  A grid sweep at an
    unchanged point (a request with the grid bit and no evaluation) is always
    asked for by a step that consumed an evaluation alone, so the first pass
    makes it and the same round serves it: rounds = the requests that carry
    an evaluation (one fewer per outer iteration than one request per round)."""
    inst = _instances()[idx]
    drv = hd.HostDriver(inst.y)
    r = drv.run()
    seq = drv.req_seq
    grid_only = [(a, b) for a, b in seq if (b & REQ_GRID) and not (b & REQ_EVAL)]
    for consumed, made in grid_only:
        assert consumed & REQ_EVAL and not consumed & REQ_GRID, (consumed, made)
    requests = [b for _, b in seq if b]
    with_eval = [b for b in requests if b & REQ_EVAL]
    assert len(grid_only) == len(requests) - len(with_eval)
    assert len(grid_only) >= 1 and r["iterations"] >= 1


def test_host_driver_iteration_cap_matches_oracle():
    """max_outer = 1 (the iteration cap of the outer loop): status NOTCONV,
    one iteration, and the refined estimate equals the oracle's."""
    inst = _instances()[1]
    p = oe.Params(max_outer=1)
    o = oe.estimate(inst.y, p)
    r = hd.HostDriver(inst.y, p).run()
    assert o.status == oe.STATUS_NOTCONV and r["status"] == o.status
    assert r["iterations"] == o.iterations == 1 and r["K"] == o.K
    np.testing.assert_allclose(r["theta"], o.theta, rtol=0, atol=1e-12)


def _mmv_instance(seed, G, N=64, K=3, snr_db=10.0):
    rng = np.random.default_rng(seed)
    th = synth.draw_frequencies(rng, K, 2.0 / N)
    A = np.exp(2j * np.pi * np.outer(np.arange(N), th))
    al = (rng.standard_normal((G, K)) + 1j * rng.standard_normal((G, K))) / np.sqrt(2)
    H = al @ A.T
    beta = float(np.mean(np.sum(np.abs(H) ** 2, axis=1))) / (N * 10 ** (snr_db / 10))
    W = (rng.standard_normal((G, N)) + 1j * rng.standard_normal((G, N))) * np.sqrt(beta / 2)
    return H + W


@pytest.mark.parametrize("seed,G", [(1, 2), (2, 3), (3, 4)])
def test_host_driver_mmv_matches_mmv_oracle(seed, G):
    """The device driver's control flow with G observation vectors (Sec. V),
    fed by the MMV oracle's evaluations, reproduces the MMV oracle estimator."""
    from oracle import mmv
    Y = _mmv_instance(seed, G)
    o = mmv.estimate(Y)
    r = hd.HostDriver(Y).run()
    assert r["status"] == o.status and r["K"] == o.K and r["iterations"] == o.iterations
    np.testing.assert_allclose(r["theta"], o.theta, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["gamma"], o.gamma, rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(r["alpha"], o.alpha, rtol=1e-9, atol=1e-12)
    assert r["beta"] == pytest.approx(o.beta, rel=1e-9)
    assert r["objective"] == pytest.approx(o.objective, rel=1e-10, abs=1e-9)


def test_host_driver_one_vector_as_mmv_is_the_single_vector_run():
    """G = 1 given as a 1 x N observation matrix: the same steps and result, bit
    for bit, as the single-vector run."""
    inst = _instances()[1]
    a = hd.HostDriver(inst.y).run()
    b = hd.HostDriver(inst.y[None, :]).run()
    assert a["K"] == b["K"] and a["evaluations"] == b["evaluations"]
    assert np.array_equal(a["theta"], b["theta"]) and np.array_equal(a["alpha"], b["alpha"][0])
    assert a["beta"] == b["beta"] and a["objective"] == b["objective"]


def _lane_instances():
    """Signals whose runs take line searches limited by a gamma reaching zero
    (weak components drawn next to strong ones, low SNR) besides ordinary ones."""
    rng = np.random.default_rng(777)
    out = list(_instances())
    for N, K, snr in [(80, 6, 5.0), (150, 9, 8.0), (120, 12, 3.0)]:
        out.append(synth.make_instance(rng, N, K, 1.0 / N, "logamp20", snr))
    # at 0 dB: draws 1, 4 and 5 of this sequence each take one line search
    # whose first step is cut short by a gamma reaching zero
    rng = np.random.default_rng(5)
    low = [synth.make_instance(rng, 64, 8, 1.0 / 64, "logamp20", 0.0) for _ in range(6)]
    out += [low[1], low[4], low[5]]
    return out


@pytest.mark.parametrize("idx", range(10))
def test_lanes_in_lockstep_hold_the_same_state(idx):
    """The driver run as the device runs it, 8 lanes in lockstep: after every
    step all lanes hold bitwise the same scalar state (a decision taken from a
    lane's own partial value instead of the team's would split them), and the
    result is the oracle's."""
    inst = _lane_instances()[idx]
    o = oe.estimate(inst.y)
    h = hd.HostDriver(inst.y)
    r = h.run(lanes=8)
    assert all(d == 0 for d in h.lane_diffs), [i for i, d in enumerate(h.lane_diffs) if d]
    assert r["K"] == o.K
    np.testing.assert_allclose(r["theta"], o.theta, rtol=0, atol=1e-10)


@pytest.mark.parametrize("seed", range(3))
def test_host_driver_incomplete_matches_incomplete_oracle(seed):
    """Incomplete observations (Sec. IV): the driver with its count scales in M
    (initial beta, stopping rules, K_max, zeta) fed by the incomplete-data
    oracle reproduces that oracle's estimator."""
    from oracle import incomplete as inc
    inst = synth.workload_incomplete_small(seed)
    obs = inc.Observation(inst.N, inst.idx, inst.phi)
    o = inc.OracleEstimatorIncomplete(inst.y, obs).run()
    r = hd.HostDriver(inst.y, obs=obs).run()
    assert r["status"] == o.status and r["K"] == o.K and r["iterations"] == o.iterations
    np.testing.assert_allclose(r["theta"], o.theta, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["gamma"], o.gamma, rtol=1e-9, atol=1e-14)
    assert r["beta"] == pytest.approx(o.beta, rel=1e-9)
    assert r["zeta"] == pytest.approx(o.zeta, rel=1e-12)
    assert r["objective"] == pytest.approx(o.objective, rel=1e-10, abs=1e-9)


@pytest.mark.parametrize("idx", range(10))
def test_shadow_trials_change_steps_not_results(idx):
    """Speculative line-search trials (a shadow slot evaluated beside each
    trial at half its step, served from the oracle): every output
    is bitwise the result without shadows, the driver takes one step fewer for
    each shadow it used, and 8 lanes in lockstep still hold one state."""
    inst = _lane_instances()[idx]
    plain = hd.HostDriver(inst.y)
    r0 = plain.run(lanes=8)
    spec = hd.HostDriver(inst.y, shadow=True)
    r1 = spec.run(lanes=8)
    assert all(d == 0 for d in spec.lane_diffs)
    for k in ("K", "beta", "zeta", "objective", "iterations", "evaluations", "status"):
        assert r1[k] == r0[k], k
    for k in ("theta", "gamma", "alpha"):
        assert np.array_equal(r1[k], r0[k]), k
    assert len(spec.req_seq) <= len(plain.req_seq)


def _refinement_instances():
    """Two signals whose final refinements reject trials (draws 8 and 11 of
    this sequence; the others accept every first trial)."""
    rng = np.random.default_rng(2024)
    out = []
    for t in range(12):
        N = int(rng.choice([64, 96, 128, 160]))
        K = int(rng.integers(2, 10))
        snr = float(rng.uniform(0, 30))
        inst = synth.make_instance(rng, N, K, 1.0 / N, "cn", snr)
        if t in (8, 11):
            out.append(inst)
    return out


@pytest.mark.parametrize("idx", range(2))
def test_shadow_trials_save_steps(idx):
    """Where the refinement rejects trials, a rejection continues with the
    shadow in the same step: fewer steps, bitwise the same result (8 lanes in
    lockstep, one state)."""
    inst = _refinement_instances()[idx]
    plain = hd.HostDriver(inst.y)
    r0 = plain.run(lanes=8)
    spec = hd.HostDriver(inst.y, shadow=True)
    r1 = spec.run(lanes=8)
    assert all(d == 0 for d in spec.lane_diffs)
    assert len(spec.req_seq) < len(plain.req_seq) - 2
    for k in ("K", "beta", "zeta", "objective", "iterations", "evaluations", "status"):
        assert r1[k] == r0[k], k
    for k in ("theta", "gamma", "alpha"):
        assert np.array_equal(r1[k], r0[k]), k
