"""GPU parity of each step of the evaluation path against the dense oracle,
called through the C ABI (a1 generator, a2 factor, a4 apply, a5 diagonal
sums, a6/a7 grid, a8 active vectors).  Inputs are seeded random states
(theta, gamma, beta) and observations at ragged sizes that span several tiles
and a ragged tail."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1705_06073_amd as sf  # noqa: E402
from oracle import numerics as nm  # noqa: E402
from tests.gpu_helpers import DEV, c2d, c64d, d2c, f64d, ragged, relerr, zeros_c  # noqa: E402

# FP64 path tolerance (normwise relative): the factorisation error grows like
# cond(C) * eps with cond(C) <= 1 + N max(gamma)/beta ~ 1e5 for these states.
TOL64 = 1e-9


@pytest.fixture(scope="module")
def ctx():
    c = sf.Context(0)
    yield c
    c.close()


def make_states(ns, seed, kmax=5):
    rng = np.random.default_rng(seed)
    out = []
    for N in ns:
        K = int(rng.integers(0, kmax + 1))
        th = rng.random(K)
        ga = 0.2 + 2.0 * rng.random(K)
        be = 0.05 + rng.random()
        y = nm.steering(th, N) @ (rng.standard_normal(K) + 1j * rng.standard_normal(K)) \
            + math.sqrt(be / 2) * (rng.standard_normal(N) + 1j * rng.standard_normal(N))
        out.append((th, ga, be, y))
    return out


def gpu_factor(ctx, ns, cols, algo=None):
    if algo is not None:
        ctx.set_factor(algo)
    n, off = ragged(ns)
    c = c2d(np.concatenate(cols))
    rho = zeros_c(n.sum())
    delta = torch.zeros(int(n.sum()), dtype=torch.float64, device=DEV)
    logdet = torch.zeros(len(ns), dtype=torch.float64, device=DEV)
    status = torch.zeros(len(ns), dtype=torch.int32, device=DEV)
    failed = torch.zeros(len(ns), dtype=torch.int64, device=DEV)
    try:
        sf.sfls_factor(ctx, n, off, c, rho, delta, logdet, status, failed)
    finally:
        if algo is not None:
            ctx.set_factor(sf.SFLS_FACTOR_AUTO)
    torch.cuda.synchronize()
    return n, off, rho, delta, logdet, status.cpu().numpy(), failed.cpu().numpy()


SIZES = [[1, 2, 3, 17, 64], [65, 100, 255, 256, 257], [1000, 1024], [2047, 4096]]
ALGOS = {"levinson": sf.SFLS_FACTOR_LEVINSON, "schur": sf.SFLS_FACTOR_SCHUR}


@pytest.mark.parametrize("algo", list(ALGOS))
@pytest.mark.parametrize("ns", SIZES)
def test_toeplitz_column_and_factor(ctx, ns, algo):
    """a1 against the first column of the dense C; a2 (Levinson) and a3 (superfast
    Schur) against the Cholesky-based generator, pivots and ln|C|."""
    print(f"[factor] sizes={ns} algo={algo}", flush=True)
    st = make_states(ns, seed=sum(ns))
    n, off = ragged(ns)
    K = np.array([len(s[0]) for s in st], np.int64)
    koff = np.concatenate([[0], np.cumsum(K)[:-1]]).astype(np.int64)
    th = f64d(np.concatenate([s[0] for s in st] + [np.zeros(1)]))
    ga = f64d(np.concatenate([s[1] for s in st] + [np.zeros(1)]))
    be = f64d([s[2] for s in st])
    c = zeros_c(n.sum())
    sf.sfls_toeplitz_column(ctx, n, off, K, koff, th, ga, be, c)
    torch.cuda.synchronize()
    cg = d2c(c)
    cols = []
    for b, (t, g, bb, _) in enumerate(st):
        ref = nm.toeplitz_column(t, g, bb, ns[b])
        assert relerr(cg[off[b]:off[b] + ns[b]], ref) < 1e-13, b
        cols.append(ref)
    _, _, rho, delta, logdet, status, failed = gpu_factor(ctx, ns, cols, ALGOS[algo])
    assert (status == 0).all() and (failed == -1).all()
    rg, dg, lg = d2c(rho), delta.cpu().numpy(), logdet.cpu().numpy()
    for b, (t, g, bb, _) in enumerate(st):
        F = nm.DenseFactor(nm.dense_from_column(cols[b]))
        r_ref, dN = F.generator()
        sl = slice(off[b], off[b] + ns[b])
        assert relerr(rg[sl], r_ref) < TOL64, (b, relerr(rg[sl], r_ref))
        assert relerr(dg[sl], F.delta) < TOL64
        assert abs(lg[b] - F.logdet) < TOL64 * max(1.0, abs(F.logdet))
        assert abs(rg[sl][-1] - 1.0) < 1e-12


@pytest.mark.parametrize("algo", list(ALGOS))
def test_factor_closed_forms(ctx, algo):
    """K = 0: rho = e_{N-1}, delta = beta exactly; K = 1: Sherman-Morrison pivots."""
    N, b0, g, th1 = 300, 0.7, 1.3, 0.271
    cols = [np.r_[b0, np.zeros(N - 1)].astype(complex), nm.toeplitz_column([th1], [g], b0, N)]
    n, off, rho, delta, logdet, status, _ = gpu_factor(ctx, [N, N], cols, ALGOS[algo])
    rg, dg = d2c(rho), delta.cpu().numpy()
    e = np.zeros(N)
    e[-1] = 1
    assert np.max(np.abs(rg[:N] - e)) < 1e-13 and np.max(np.abs(dg[:N] - b0)) < 1e-13
    k = np.arange(N)
    assert relerr(dg[N:], b0 * (b0 + (k + 1) * g) / (b0 + k * g)) < 1e-12


@pytest.mark.parametrize("algo", list(ALGOS))
def test_factor_reports_not_positive_definite(ctx, algo):
    """c = [1, 2, 0, ...] is indefinite: delta_1 = 1 - 4 < 0 at step 1."""
    col = np.zeros(300, complex)
    col[0], col[1] = 1.0, 2.0
    _, _, _, _, logdet, status, failed = gpu_factor(ctx, [300], [col], ALGOS[algo])
    assert status[0] == sf.SFLS_ENOTPD and failed[0] == 1
    assert np.isnan(logdet.cpu().numpy()[0])


def test_factor_rejects_bad_sizes(ctx):
    with pytest.raises(sf.SflsError) as e:
        gpu_factor(ctx, [sf.SFLS_MAX_N + 1], [np.ones(sf.SFLS_MAX_N + 1, complex)])
    assert e.value.status == sf.SFLS_EUNSUPPORTED
    with pytest.raises(sf.SflsError) as e:
        sf.sfls_factor(ctx, [0], [0], None, None, None, None, None, None)
    assert e.value.status == sf.SFLS_EINVAL


def factor_states(ctx, st, ns):
    cols = [nm.toeplitz_column(t, g, b, N) for (t, g, b, _), N in zip(st, ns)]
    return gpu_factor(ctx, ns, cols)


@pytest.mark.parametrize("ns", [[5, 64, 100], [1000, 1024, 2048], [4096]])
@pytest.mark.parametrize("ydt", ["c128", "c64"])
def test_gs_apply(ctx, ns, ydt):
    print(f"[apply] sizes={ns} {ydt}", flush=True)
    st = make_states(ns, seed=7 + sum(ns))
    n, off, rho, delta, *_ = factor_states(ctx, st, ns)
    ys = [s[3] for s in st]
    if ydt == "c64":
        ys = [y.astype(np.complex64) for y in ys]
        yd, dt = c64d(np.concatenate(ys)), sf.SFLS_C64
    else:
        yd, dt = c2d(np.concatenate(ys)), sf.SFLS_C128
    w = zeros_c(n.sum())
    yCy = torch.zeros(len(ns), dtype=torch.float64, device=DEV)
    ww = torch.zeros(len(ns), dtype=torch.float64, device=DEV)
    sf.sfls_gs_apply(ctx, n, off, yd, dt, rho, delta, w, yCy, ww)
    torch.cuda.synchronize()
    wg = d2c(w)
    for b, (t, g, bb, _) in enumerate(st):
        ev = nm.Evaluation(ys[b].astype(np.complex128), t, g, bb)
        sl = slice(off[b], off[b] + ns[b])
        assert relerr(wg[sl], ev.w) < TOL64, (b, relerr(wg[sl], ev.w))
        assert abs(yCy.cpu().numpy()[b] - ev.yCy) < TOL64 * abs(ev.yCy)
        assert abs(ww.cpu().numpy()[b] - np.vdot(ev.w, ev.w).real) < TOL64 * np.vdot(ev.w, ev.w).real


@pytest.mark.parametrize("ns", [[2, 9, 24], [64, 200, 512]])
def test_omega(ctx, ns):
    print(f"[omega] sizes={ns}", flush=True)
    st = make_states(ns, seed=11 + sum(ns))
    n, off, rho, delta, *_ = factor_states(ctx, st, ns)
    oo = np.concatenate([[0], np.cumsum(2 * n - 1)[:-1]]).astype(np.int64)
    tot = int((2 * n - 1).sum())
    outs = [zeros_c(tot) for _ in range(4)]
    sf.sfls_omega(ctx, n, off, oo, rho, delta, *outs)
    torch.cuda.synchronize()
    og = [d2c(o) for o in outs]
    for b, (t, g, bb, _) in enumerate(st):
        F = nm.DenseFactor(nm.covariance(t, g, bb, ns[b]))
        ref = nm.omegas(F)
        sl = slice(oo[b], oo[b] + 2 * ns[b] - 1)
        for k in range(4):
            assert relerr(og[k][sl], ref[k]) < TOL64, (b, "stvx"[k], relerr(og[k][sl], ref[k]))


@pytest.mark.parametrize("ns,Lm", [([64], 4), ([64, 100, 1000], 8), ([1024], 8), ([4096], 8)])
def test_grid(ctx, ns, Lm):
    print(f"[grid] sizes={ns} L={Lm}N", flush=True)
    st = make_states(ns, seed=13 + sum(ns))
    n, off, rho, delta, *_ = factor_states(ctx, st, ns)
    Ls = np.array([2 ** int(round(math.log2(Lm * N))) for N in ns], np.int64)
    goff = np.concatenate([[0], np.cumsum(Ls)[:-1]]).astype(np.int64)
    yd = c2d(np.concatenate([s[3] for s in st]))
    gb_host = np.array([np.mean(s[1]) if len(s[1]) else -1.0 for s in st])
    gb, zeta = f64d(gb_host), f64d(np.full(len(ns), 0.1))
    ev = [nm.Evaluation(s[3], s[0], s[1], s[2]) for s in st]
    for prec in (sf.SFLS_FP64, sf.SFLS_MIXED):
        tot = int(Ls.sum())
        fdt = torch.float64 if prec == sf.SFLS_FP64 else torch.float32
        qG = torch.zeros(2 * tot, dtype=fdt, device=DEV)
        sG = torch.zeros(tot, dtype=fdt, device=DEV)
        dL = torch.zeros(tot, dtype=fdt, device=DEV)
        rG = torch.zeros(2 * tot, dtype=fdt, device=DEV)
        tG = torch.zeros(2 * tot, dtype=fdt, device=DEV)
        am = torch.zeros(len(ns), dtype=torch.int64, device=DEV)
        av = torch.zeros(len(ns), dtype=torch.float64, device=DEV)
        sf.sfls_grid_eval(ctx, n, off, yd, sf.SFLS_C128, rho, delta, Ls, goff, gb, zeta, qG, sG,
                          dL, am, av, precision=prec, rG=rG, tG=tG)
        torch.cuda.synchronize()
        qh = qG.cpu().numpy().astype(np.float64).view(np.complex128)
        rh = rG.cpu().numpy().astype(np.float64).view(np.complex128)
        th_ = tG.cpu().numpy().astype(np.float64).view(np.complex128)
        sh, dh = sG.cpu().numpy().astype(np.float64), dL.cpu().numpy().astype(np.float64)
        tol = TOL64 if prec == sf.SFLS_FP64 else 1e-4
        for b in range(len(ns)):
            L = int(Ls[b])
            q_ref, s_ref = ev[b].grid(L)
            r_ref, t_ref = ev[b].grid_derivatives(L)
            sl = slice(goff[b], goff[b] + L)
            assert relerr(rh[sl], r_ref) < tol, (b, prec, "r", relerr(rh[sl], r_ref))
            assert relerr(th_[sl], t_ref) < tol, (b, prec, "t", relerr(th_[sl], t_ref))
            gbv = nm.gamma_hat(q_ref, s_ref) if gb_host[b] <= 0 else np.full(L, gb_host[b])
            d_ref = nm.delta_L(q_ref, s_ref, gbv, 0.1)
            sl = slice(goff[b], goff[b] + L)
            assert relerr(qh[sl], q_ref) < tol, (b, prec, relerr(qh[sl], q_ref))
            assert relerr(sh[sl], s_ref) < tol, (b, prec, relerr(sh[sl], s_ref))
            assert relerr(dh[sl], d_ref) < tol, (b, prec, relerr(dh[sl], d_ref))
            if prec == sf.SFLS_FP64:
                assert am.cpu().numpy()[b] == int(np.argmin(d_ref))
            else:  # FP32 ranks: the pick must be within FP32 noise of the true minimum
                pick = int(am.cpu().numpy()[b])
                assert d_ref[pick] - d_ref.min() <= 1e-4 * np.max(np.abs(d_ref))


def test_context_hbm_budget():
    """A context's workspace stays within the budget given at creation: a batch
    that would need more is refused with ENOMEM (nothing enqueued), a smaller
    one runs, and a context without a cap runs the large one."""
    ns = [4096] * 64
    st = make_states(ns[:1], seed=5) * 64
    cols = np.concatenate([nm.toeplitz_column(t, g, b, N) for (t, g, b, _), N in zip(st, ns)])
    n, off = ragged(ns)
    small = sf.Context(0, hbm_budget=8 << 20)
    try:
        out = [zeros_c(n.sum()), torch.zeros(int(n.sum()), dtype=torch.float64, device=DEV),
               torch.zeros(64, dtype=torch.float64, device=DEV),
               torch.zeros(64, dtype=torch.int32, device=DEV),
               torch.zeros(64, dtype=torch.int64, device=DEV)]
        with pytest.raises(sf.SflsError) as e:
            sf.sfls_factor(small, n, off, c2d(cols), *out)
        assert e.value.status == sf.SFLS_ENOMEM
        n1, off1 = ragged(ns[:1])
        sf.sfls_factor(small, n1, off1, c2d(cols[:4096]), *[o[:2 * 4096] if i == 0 else
                                                           (o[:4096] if i == 1 else o[:1])
                                                           for i, o in enumerate(out)])
        torch.cuda.synchronize()
        assert int(out[3][0].cpu()) == 0
    finally:
        small.close()


def test_grid_out_mask(ctx):
    """Only the outputs named in out_mask are written (the others' buffers stay
    untouched), r^G alone needs no diagonal sums, a named NULL output and an
    unknown bit are rejected on the host."""
    ns = [300]
    st = make_states(ns, seed=71)
    n, off, rho, delta, *_ = factor_states(ctx, st, ns)
    L = np.array([4096], np.int64)
    goff = np.zeros(1, np.int64)
    yd = c2d(st[0][3])
    gb, zeta = f64d([np.mean(st[0][1])]), f64d([0.1])
    ev = nm.Evaluation(st[0][3], st[0][0], st[0][1], st[0][2])
    r_ref, _ = ev.grid_derivatives(4096)
    sentinel = 12345.0
    rG = torch.full((2 * 4096,), sentinel, dtype=torch.float64, device=DEV)
    tG = torch.full((2 * 4096,), sentinel, dtype=torch.float64, device=DEV)
    qG = torch.full((2 * 4096,), sentinel, dtype=torch.float64, device=DEV)
    sf.sfls_grid_eval(ctx, n, off, yd, sf.SFLS_C128, rho, delta, L, goff, None, None, qG=qG,
                      rG=rG, tG=tG, out_mask=sf.SFLS_GRID_R)
    torch.cuda.synchronize()
    assert relerr(d2c(rG), r_ref) < TOL64
    assert (tG.cpu().numpy() == sentinel).all() and (qG.cpu().numpy() == sentinel).all()
    for mask, kw in ((sf.SFLS_GRID_T, {}), (sf.SFLS_GRID_DL, dict(tG=tG)), (64, dict(rG=rG))):
        with pytest.raises(sf.SflsError) as e:
            sf.sfls_grid_eval(ctx, n, off, yd, sf.SFLS_C128, rho, delta, L, goff, gb, zeta,
                              out_mask=mask, **kw)
        assert e.value.status == sf.SFLS_EINVAL


@pytest.mark.parametrize("ns", [[64, 100], [1024], [4096]])
def test_active_vectors(ctx, ns):
    print(f"[active] sizes={ns}", flush=True)
    st = make_states(ns, seed=17 + sum(ns), kmax=6)
    n, off, rho, delta, *_ = factor_states(ctx, st, ns)
    yd = c2d(np.concatenate([s[3] for s in st]))
    w = zeros_c(n.sum())
    sf.sfls_gs_apply(ctx, n, off, yd, sf.SFLS_C128, rho, delta, w)
    rng = np.random.default_rng(5)
    thq = [np.concatenate([s[0], rng.random(3)]) for s in st]  # active + off-grid points
    K = np.array([len(t) for t in thq], np.int64)
    koff = np.concatenate([[0], np.cumsum(K)[:-1]]).astype(np.int64)
    outs = [zeros_c(K.sum()) for _ in range(7)]
    sf.sfls_active_eval(ctx, n, off, w, rho, delta, K, koff, f64d(np.concatenate(thq)), *outs)
    torch.cuda.synchronize()
    og = [d2c(o) for o in outs]
    for b, (t, g, bb, y) in enumerate(st):
        ev = nm.Evaluation(y, t, g, bb)
        ref = nm.active_vectors(ev.F, ev.w, thq[b])
        sl = slice(koff[b], koff[b] + K[b])
        for i, name in enumerate("qrustvx"):
            assert relerr(og[i][sl], ref[name]) < TOL64, (b, name, relerr(og[i][sl], ref[name]))


@pytest.mark.parametrize("lds_f", [256, 1024])
def test_factor_with_lower_lds_transform_limit(ctx, lds_f):
    """a3 with the recursion's larger merges moved from LDS to device scratch:
    the same generator, pivots and ln|C| as the dense oracle."""
    ns = [300, 1000, 2048, 4096, 4500]
    print(f"[factor lds {lds_f}] sizes={ns}", flush=True)
    st = make_states(ns, seed=77 + lds_f)
    cols = [nm.toeplitz_column(t, g, b, N) for (t, g, b, _), N in zip(st, ns)]
    ctx.set_schur_lds(lds_f)
    try:
        n, off, rho, delta, logdet, status, failed = gpu_factor(ctx, ns, cols, sf.SFLS_FACTOR_SCHUR)
    finally:
        ctx.set_schur_lds(4096)
    assert (status == 0).all() and (failed == -1).all()
    rg, dg, lg = d2c(rho), delta.cpu().numpy(), logdet.cpu().numpy()
    for b in range(len(ns)):
        F = nm.DenseFactor(nm.dense_from_column(cols[b]))
        r_ref, _ = F.generator()
        sl = slice(off[b], off[b] + ns[b])
        assert relerr(rg[sl], r_ref) < TOL64, (b, relerr(rg[sl], r_ref))
        assert relerr(dg[sl], F.delta) < TOL64
        assert abs(lg[b] - F.logdet) < TOL64 * max(1.0, abs(F.logdet))


def test_lds_transform_limit_rejects_bad_values(ctx):
    for bad in (128, 3000, 8192):
        with pytest.raises(sf.SflsError):
            ctx.set_schur_lds(bad)


def test_timing_modes(ctx):
    """Mode 2 brackets only the recursion with events, mode 1 every kernel of a
    round; the timed figures change nothing in the results; other modes are
    rejected."""
    from paper_1705_06073_amd import synth
    ys = [synth.workload_paper_snr(20 + i, 15.0, N=n, K=4).y.astype(np.complex128)
          for i, n in enumerate((300, 700))]
    p = sf.default_params(precision=sf.SFLS_MIXED)
    try:
        ctx.reset_stats()
        ctx.set_timing(2)
        a = sf.estimate_batch(ctx, ys, p)
        k2 = ctx.kernel_stats()
        ctx.reset_stats()
        ctx.set_timing(1)
        b = sf.estimate_batch(ctx, ys, p)
        k1 = ctx.kernel_stats()
    finally:
        ctx.set_timing(False)
    assert k2["factor"]["seconds"] > 0 and k2["factor"]["launches"] > 0
    assert all(v["seconds"] == 0 and v["launches"] == 0 for k, v in k2.items() if k != "factor")
    for k in ("factor", "gs_apply", "omega", "grid", "select", "active", "driver"):
        assert k1[k]["seconds"] > 0 and k1[k]["launches"] > 0, k
    assert k1["factor"]["launches"] == k2["factor"]["launches"]
    for x, y in zip(a, b):
        assert x.K == y.K and np.array_equal(x.theta, y.theta) and x.beta == y.beta
    with pytest.raises(sf.SflsError):
        ctx.set_timing(3)
