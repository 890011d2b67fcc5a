"""Speculative line-search trials (sfls_set_speculation): every output of
sfls_estimate is bitwise the same with shadows on and off; only the number of
rounds changes."""
import numpy as np
import pytest

import paper_1705_06073_amd as sf
from paper_1705_06073_amd import synth

pytestmark = pytest.mark.gpu


def _run(ctx, ys, spec, precision):
    ctx.set_speculation(spec)
    res = sf.estimate_batch(ctx, ys, sf.default_params(precision=precision))
    run, _ = ctx.last_run()
    return res, run["rounds"]


def _same(ra, rb):
    assert len(ra) == len(rb)
    for a, b in zip(ra, rb):
        assert a.K == b.K and a.status == b.status
        assert a.iterations == b.iterations and a.evaluations == b.evaluations
        assert a.beta == b.beta and a.zeta == b.zeta and a.objective == b.objective
        assert np.array_equal(a.theta, b.theta)
        assert np.array_equal(a.gamma, b.gamma)
        assert np.array_equal(a.alpha, b.alpha)


@pytest.mark.parametrize("precision", [sf.SFLS_MIXED, sf.SFLS_FP64])
def test_speculation_bitwise_batched_n4096(precision):
    """The batched workload (256 x N = 4096): the same outputs bit for bit,
    in fewer rounds (the slowest instances' refinements reject trials)."""
    ctx = sf.Context(0)
    ys = [synth.workload_n4096(i).y for i in range(256)]
    r_off, n_off = _run(ctx, ys, False, precision)
    r_on, n_on = _run(ctx, ys, True, precision)
    print(f"rounds without / with shadows: {n_off} / {n_on}", flush=True)
    _same(r_on, r_off)
    assert n_on < n_off
    ctx.close()


def test_speculation_bitwise_uneven():
    """A batch of uneven sizes (dispatched longest first, shadows included):
    the same outputs bit for bit."""
    ctx = sf.Context(0)
    insts = [synth.workload_uneven(i) for i in range(160)]
    ys = [i.y for i in insts if i.N <= 2048][:48]
    r_off, n_off = _run(ctx, ys, False, sf.SFLS_MIXED)
    r_on, n_on = _run(ctx, ys, True, sf.SFLS_MIXED)
    _same(r_on, r_off)
    assert n_on <= n_off
    ctx.close()


def test_budget_context_does_not_speculate():
    """A context created with an HBM budget runs without shadows (the rounds
    of speculation off) and gives the same outputs bit for bit."""
    ys = [synth.workload_n4096(i).y for i in range(24)]
    free = sf.Context(0)
    r_off, n_off = _run(free, ys, False, sf.SFLS_MIXED)
    r_on, n_on = _run(free, ys, True, sf.SFLS_MIXED)
    free.close()
    capped = sf.Context(0, hbm_budget=8 << 30)
    r_cap, n_cap = _run(capped, ys, True, sf.SFLS_MIXED)
    capped.close()
    print(f"rounds off / on / budgeted: {n_off} / {n_on} / {n_cap}", flush=True)
    _same(r_cap, r_off)
    _same(r_on, r_off)
    assert n_cap == n_off
