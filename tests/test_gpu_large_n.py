"""GPU parity at sizes whose transforms do not fit one CU's LDS: superfast merges
above 4096 points, Gohberg-Semencul apply / omega / refinement with P = 2N > 8192,
and grids whose M-point sub-FFTs fold the inputs (N > 4096 in FP64, N > 8192 in
FP32), up to N = 16384 of the uneven batched workload.  Dense-oracle comparisons
at N = 4500 (P = 16384, root merge of 8192 points, folded FP64 grid); at
N = 16384 properties that hold at any size: Toeplitz residuals by FFT products,
ln|C| by the determinant lemma, K = 1 closed forms, Woodbury forms of the
objective at the estimator's result."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1705_06073_amd as sf  # noqa: E402
from oracle import numerics as nm  # noqa: E402
from paper_1705_06073_amd import synth  # noqa: E402
from tests.gpu_helpers import DEV, c2d, d2c, f64d, ragged, relerr, zeros_c  # noqa: E402

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def ctx():
    c = sf.Context(0)
    yield c
    c.close()


def states(ns, seed, kmax=6):
    rng = np.random.default_rng(seed)
    out = []
    for N in ns:
        K = int(rng.integers(1, kmax + 1))
        th = rng.random(K)
        ga = 0.2 + 2.0 * rng.random(K)
        be = 0.05 + rng.random()
        y = nm.steering(th, N) @ (rng.standard_normal(K) + 1j * rng.standard_normal(K)) \
            + math.sqrt(be / 2) * (rng.standard_normal(N) + 1j * rng.standard_normal(N))
        out.append((th, ga, be, y))
    return out


def kappa(th, ga, be, N):
    return 1.0 + N * float(np.sum(ga)) / be


def toeplitz_mv(c, x):
    """C x for the Hermitian Toeplitz C with first column c, by a 2N circulant."""
    N = len(c)
    col = np.concatenate([c, [0.0], np.conj(c[:0:-1])])
    return np.fft.ifft(np.fft.fft(col) * np.fft.fft(x, 2 * N))[:N]


def lemma_logdet(th, ga, be, N):
    """ln|beta I + Psi Gamma Psi^H| = N ln beta + ln det(I + G^1/2 Psi^H Psi G^1/2 / beta)."""
    Ps = nm.steering(th, N)
    g = np.sqrt(ga)
    M = np.eye(len(th)) + (g[:, None] * (Ps.conj().T @ Ps) * g[None, :]) / be
    return N * math.log(be) + float(np.linalg.slogdet(M)[1])


def gpu_factor(ctx, ns, cols):
    n, off = ragged(ns)
    rho = zeros_c(n.sum())
    delta = torch.zeros(int(n.sum()), dtype=torch.float64, device=DEV)
    logdet = torch.zeros(len(ns), dtype=torch.float64, device=DEV)
    status = torch.zeros(len(ns), dtype=torch.int32, device=DEV)
    failed = torch.zeros(len(ns), dtype=torch.int64, device=DEV)
    sf.sfls_factor(ctx, n, off, c2d(np.concatenate(cols)), rho, delta, logdet, status, failed)
    torch.cuda.synchronize()
    assert (status.cpu().numpy() == 0).all()
    return n, off, rho, delta, logdet.cpu().numpy()


def test_factor_large_dense(ctx):
    """Superfast recursion with a root merge of 8192 points and refinement with
    P = 16384, in a ragged batch with a small instance, against the Cholesky
    generator, pivots and ln|C|."""
    ns = [4500, 300, 4097]
    st = states(ns, 101)
    cols = [nm.toeplitz_column(t, g, b, N) for (t, g, b, _), N in zip(st, ns)]
    print(f"[large factor] sizes={ns}", flush=True)
    n, off, rho, delta, lg = gpu_factor(ctx, ns, cols)
    rg, dg = d2c(rho), delta.cpu().numpy()
    for b, (t, g, bb, _) in enumerate(st):
        N = ns[b]
        F = nm.DenseFactor(nm.dense_from_column(cols[b]))
        r_ref, _ = F.generator()
        sl = slice(off[b], off[b] + N)
        tol = max(1e-12, 100.0 * kappa(t, g, bb, N) * EPS)
        er, ed = relerr(rg[sl], r_ref), relerr(dg[sl], F.delta)
        el = abs(lg[b] - F.logdet) / max(1.0, abs(F.logdet))
        print(f"   N={N} tol={tol:.1e} rho {er:.2e} delta {ed:.2e} logdet {el:.2e}", flush=True)
        assert er < tol and ed < tol and el < max(1e-9, tol)


def test_factor_n16384_properties(ctx):
    """N = 16384 (root merge 16384, level-1 merges 8192) and 9000: C rho =
    delta_{N-1} e_{N-1} to a small normwise backward error, rho_{N-1} = 1,
    positive pivots, ln|C| = sum ln delta_i against the determinant lemma."""
    ns = [16384, 9000]
    st = states(ns, 202, kmax=20)
    cols = [nm.toeplitz_column(t, g, b, N) for (t, g, b, _), N in zip(st, ns)]
    print(f"[large factor] sizes={ns}", flush=True)
    n, off, rho, delta, lg = gpu_factor(ctx, ns, cols)
    rg, dg = d2c(rho), delta.cpu().numpy()
    for b, (t, g, bb, _) in enumerate(st):
        N = ns[b]
        r = rg[off[b]:off[b] + N]
        d = dg[off[b]:off[b] + N]
        e = np.zeros(N, complex)
        e[-1] = d[-1]
        normC = 2.0 * np.sum(np.abs(cols[b]))
        eta = np.max(np.abs(toeplitz_mv(cols[b], r) - e)) / (normC * np.max(np.abs(r)) + d[-1])
        ll = lemma_logdet(t, g, bb, N)
        el = abs(lg[b] - ll) / max(1.0, abs(ll))
        print(f"   N={N} K={len(t)} backward error {eta:.2e} logdet vs lemma {el:.2e}", flush=True)
        assert abs(r[-1] - 1.0) < 1e-12 and (d > 0).all()
        assert eta < 1e-12
        assert el < 1e-9


def test_gs_apply_and_omega_large(ctx):
    """P = 16384 and 32768 transforms on device scratch: w = C^{-1} y against
    the dense solve at N = 4500 and by its residual at N = 16384; the diagonal
    sums omega against dense sums of C^{-1} at N = 4500."""
    ns = [4500, 16384]
    st = states(ns, 303)
    cols = [nm.toeplitz_column(t, g, b, N) for (t, g, b, _), N in zip(st, ns)]
    n, off, rho, delta, _ = gpu_factor(ctx, ns, cols)
    yd = c2d(np.concatenate([s[3] for s in st]))
    w = zeros_c(n.sum())
    yCy = torch.zeros(len(ns), dtype=torch.float64, device=DEV)
    print(f"[large apply] sizes={ns}", flush=True)
    sf.sfls_gs_apply(ctx, n, off, yd, sf.SFLS_C128, rho, delta, w, yCy)
    torch.cuda.synchronize()
    wg, yc = d2c(w), yCy.cpu().numpy()
    t, g, bb, y = st[0]
    ev = nm.Evaluation(y, t, g, bb)
    tol = max(1e-12, 100.0 * kappa(t, g, bb, ns[0]) * EPS)
    ew = relerr(wg[:ns[0]], ev.w)
    print(f"   N={ns[0]} w {ew:.2e} (tol {tol:.1e})", flush=True)
    assert ew < tol and abs(yc[0] - ev.yCy) < tol * abs(ev.yCy)
    N = ns[1]
    t, g, bb, y = st[1]
    w1 = wg[off[1]:off[1] + N]
    normC = 2.0 * np.sum(np.abs(cols[1]))
    eta = np.max(np.abs(toeplitz_mv(cols[1], w1) - y)) / (normC * np.max(np.abs(w1)) + np.max(np.abs(y)))
    print(f"   N={N} backward error of w {eta:.2e}", flush=True)
    assert eta < 1e-12 and abs(yc[1] - np.vdot(y, w1).real) < 1e-10 * abs(yc[1])
    # omega at N = 4500
    n1, off1 = ragged(ns[:1])
    oo = np.zeros(1, np.int64)
    outs = [zeros_c(2 * ns[0] - 1) for _ in range(4)]
    sf.sfls_omega(ctx, n1, off1, oo, rho, delta, *outs)
    torch.cuda.synchronize()
    ref = nm.omegas(ev.F)
    for k in range(4):
        eo = relerr(d2c(outs[k]), ref[k])
        print(f"   omega_{'stvx'[k]} {eo:.2e}", flush=True)
        assert eo < tol


def k1_closed_forms(th1, ga, be, N, L, y):
    """K = 1: generator, pivots, w, q^G and s^G in closed form (Sherman-Morrison)."""
    psi = nm.steering([th1], N)[:, 0]    # exact reduction of n th1 mod 1
    den = be + N * ga
    x = -ga * psi * np.conj(psi[-1]) / den
    x[-1] += 1.0
    x /= be
    rho = x / x[-1].real
    k = np.arange(N)
    delta = be * (be + (k + 1) * ga) / (be + k * ga)
    w = (y - ga * psi * np.vdot(psi, y) / den) / be
    qG = np.fft.fft(w, L)
    d = th1 - np.arange(L) / L
    sd = np.sin(np.pi * d)
    with np.errstate(divide="ignore", invalid="ignore"):
        D2 = np.where(np.abs(sd) < 1e-300, float(N * N), (np.sin(np.pi * N * d) / sd) ** 2)
    sG = (N - ga * D2 / den) / be
    return rho, delta, qG, sG


def test_grid_folded(ctx):
    """Grids whose sub-FFTs fold the inputs: N = 16384, K = 1 against the
    closed forms (FP64 sub-FFTs of 4096 points fold 4 samples each, FP32 of
    8192 points 2); N = 4500 against the dense oracle (FP64 folds 2)."""
    N, th1, ga, be = 16384, 0.3141592653589793, 0.8, 0.3
    rng = np.random.default_rng(9)
    y = math.sqrt(ga) * np.exp(2j * np.pi * np.mod(np.arange(N) * th1, 1.0)) \
        + math.sqrt(be / 2) * (rng.standard_normal(N) + 1j * rng.standard_normal(N))
    L = 8 * N
    rho_c, delta_c, q_ref, s_ref = k1_closed_forms(th1, ga, be, N, L, y)
    cases = [(N, L, y, c2d(rho_c), f64d(delta_c), q_ref, s_ref, 0.7, 0.01)]
    ns2 = [4500]
    st = states(ns2, 404)
    t, g, bb, y2 = st[0]
    ev = nm.Evaluation(y2, t, g, bb)
    F = ev.F
    r2, _ = F.generator()
    L2 = 2 ** int(round(math.log2(8 * ns2[0])))
    q2, s2 = ev.grid(L2)
    cases.append((ns2[0], L2, y2, c2d(r2), f64d(F.delta), q2, s2, float(np.mean(g)), 0.05))
    for (Nc, Lc, yc, rd, dd, qr, sr, gbv, zeta) in cases:
        n, off = ragged([Nc])
        for prec in (sf.SFLS_FP64, sf.SFLS_MIXED):
            fdt = torch.float64 if prec == sf.SFLS_FP64 else torch.float32
            qG = torch.zeros(2 * Lc, dtype=fdt, device=DEV)
            sG = torch.zeros(Lc, dtype=fdt, device=DEV)
            dL = torch.zeros(Lc, dtype=fdt, device=DEV)
            am = torch.zeros(1, dtype=torch.int64, device=DEV)
            av = torch.zeros(1, dtype=torch.float64, device=DEV)
            rG = torch.zeros(2 * Lc, dtype=fdt, device=DEV)
            tG = torch.zeros(2 * Lc, dtype=fdt, device=DEV)
            print(f"[grid folded] N={Nc} L={Lc} prec={prec}", flush=True)
            sf.sfls_grid_eval(ctx, n, off, c2d(yc), sf.SFLS_C128, rd, dd,
                              np.array([Lc], np.int64), np.zeros(1, np.int64),
                              f64d([gbv]), f64d([zeta]), qG, sG, dL, am, av, precision=prec,
                              rG=rG, tG=tG)
            torch.cuda.synchronize()
            if Nc == 4500:   # theta-derivative arrays of the folded grid against the oracle
                r_ref, t_ref = ev.grid_derivatives(Lc)
                tol_d = 1e-9 if prec == sf.SFLS_FP64 else 1e-4
                er = relerr(rG.cpu().numpy().astype(np.float64).view(np.complex128), r_ref)
                et = relerr(tG.cpu().numpy().astype(np.float64).view(np.complex128), t_ref)
                print(f"   r {er:.2e} t {et:.2e}", flush=True)
                assert er < tol_d and et < tol_d
            qh = qG.cpu().numpy().astype(np.float64).view(np.complex128)
            sh, dh = sG.cpu().numpy().astype(np.float64), dL.cpu().numpy().astype(np.float64)
            d_ref = nm.delta_L(qr, sr, np.full(Lc, gbv), zeta)
            tol = 1e-9 if prec == sf.SFLS_FP64 else 1e-4
            eq, es, ed = relerr(qh, qr), relerr(sh, sr), relerr(dh, d_ref)
            print(f"   q {eq:.2e} s {es:.2e} dL {ed:.2e}", flush=True)
            assert eq < tol and es < tol and ed < tol


def woodbury_objective(y, th, ga, be, zeta):
    """ln|C| (lemma), y^H C^{-1} y and q = Psi^H C^{-1} y by the Woodbury identity."""
    N = len(y)
    Ps = nm.steering(th, N)
    G = Ps.conj().T @ Ps
    u = Ps.conj().T @ y
    Mw = np.diag(be / ga) + G
    v = np.linalg.solve(Mw, u)
    yCy = (np.vdot(y, y).real - np.vdot(u, v).real) / be
    q = (u - G @ v) / be
    ld = lemma_logdet(th, ga, be, N)
    return nm.objective(ld, yCy, len(th), N, zeta), q


def test_estimate_uneven_batch(ctx):
    """sfls_estimate on instances of the uneven workload (N log-uniform on
    [128, 16384], K ~ Poisson(N/64), SNR ~ U[5,30] dB) including N > 8192, in
    one ragged batch: valid outputs everywhere; at sampled instances the
    objective and alpha at the returned point agree with the dense oracle
    (N <= 2048) or with the Woodbury forms (largest N)."""
    idx = list(range(24))
    insts = [synth.workload_uneven(i) for i in idx]
    big = max(range(len(insts)), key=lambda i: insts[i].N)
    print(f"[uneven] N = {[i.N for i in insts]}", flush=True)
    assert insts[big].N > 8192
    res = sf.estimate_batch(ctx, [i.y for i in insts], sf.default_params(precision=sf.SFLS_MIXED))
    for b, r in enumerate(res):
        assert r.status in (sf.SFLS_OK, sf.SFLS_NOTCONV), (b, r.status)
        assert np.all((r.theta >= 0) & (r.theta < 1)) and np.all(np.diff(r.theta) >= 0)
        assert np.all(r.gamma > 0) and r.beta > 0 and math.isfinite(r.objective)
    small = [b for b in range(len(insts)) if insts[b].N <= 2048 and res[b].K > 0][:3]
    for b in small + [big]:
        inst, r = insts[b], res[b]
        if insts[b].N <= 2048:
            ev = nm.Evaluation(inst.y, r.theta, r.gamma, r.beta)
            fo, q = ev.f(r.K, r.zeta), ev.act["q"]
        else:
            fo, q = woodbury_objective(inst.y.astype(np.complex128), r.theta, r.gamma, r.beta, r.zeta)
        ef = abs(r.objective - fo) / max(1.0, abs(fo))
        a_ref = r.gamma * q
        ea = np.max(np.abs(r.alpha - a_ref) / (1e-6 * np.abs(a_ref) + 1e-9))
        print(f"   b={b} N={inst.N} K={r.K} (true {inst.K}) ev={r.evaluations} objective rel "
              f"{ef:.2e} alpha err/tol {ea:.2e}", flush=True)
        assert ef <= 1e-8 and ea <= 1.0


def k1_omegas(th1, ga, be, N):
    """K = 1 diagonal sums of C^{-1}, D C^{-1}, D^2 C^{-1} and D C^{-1} D in
    closed form: [C^{-1}]_{q,q+i} = (delta_{i0} - ga e^{-j2 pi i th1} / (be + N ga)) / be
    summed over the q of lag i with power sums of q (exact in FP64 here)."""
    i = np.arange(-(N - 1), N, dtype=np.float64)
    lo = np.maximum(0.0, -i)                 # first q of lag i
    hi = np.minimum(N - 1.0, N - 1.0 - i)    # last q
    def psum(m, a, b):                       # sum_{q=a}^{b} q^m
        def P(x):                            # sum_{q=0}^{x-1} q^m
            return (x, x * (x - 1) / 2, (x - 1) * x * (2 * x - 1) / 6)[m]
        return P(b + 1) - P(a)
    S0, S1, S2 = psum(0, lo, hi), psum(1, lo, hi), psum(2, lo, hi)
    ph = np.exp(-2j * np.pi * nm.phase_frac(i, [th1])[:, 0])
    c = ga / (be + N * ga)
    z = (i == 0).astype(np.float64)
    tp = 2 * np.pi
    om_s = (z * S0 - c * ph * S0) / be
    om_t = tp * (z * S1 - c * ph * S1) / be
    om_v = tp ** 2 * (z * S2 - c * ph * S2) / be
    om_x = tp ** 2 * (z * S2 - c * ph * (S2 + i * S1)) / be
    return om_s, om_t, om_v, om_x


@pytest.mark.parametrize("N", [32768, 65536])
def test_k1_chain_largest_sizes(ctx, N):
    """Every step entry point at the largest sizes, chained as an evaluation
    runs them (covariance column, superfast factorisation with refinement,
    Gohberg-Semencul apply, diagonal sums, grid in FP64 and FP32), for K = 1
    where each result has a closed form (Sherman-Morrison; Dirichlet kernel
    for s^G; power sums for the diagonal sums)."""
    th1, ga, be = 0.2718281828459045, 0.8, 0.3
    rng = np.random.default_rng(N)
    y = math.sqrt(ga) * np.exp(2j * np.pi * np.mod(np.arange(N) * th1, 1.0)) \
        + math.sqrt(be / 2) * (rng.standard_normal(N) + 1j * rng.standard_normal(N))
    L = 8 * N
    rho_c, delta_c, q_ref, s_ref = k1_closed_forms(th1, ga, be, N, L, y)
    tol = max(1e-12, 100.0 * kappa([th1], [ga], be, N) * EPS)
    n, off = ragged([N])
    c = zeros_c(N)
    print(f"[k1 chain] N={N} L={L} tol={tol:.1e}", flush=True)
    sf.sfls_toeplitz_column(ctx, n, off, np.array([1]), np.zeros(1, np.int64), f64d([th1]),
                            f64d([ga]), f64d([be]), c)
    torch.cuda.synchronize()
    col_ref = ga * nm.steering([th1], N)[:, 0]   # exact reduction of i th1 mod 1
    col_ref[0] += be
    ec = relerr(d2c(c), col_ref)
    n, off, rho, delta, lg = gpu_factor(ctx, [N], [d2c(c)])
    er, ed = relerr(d2c(rho), rho_c), relerr(delta.cpu().numpy(), delta_c)
    ld_ref = N * math.log(be) + math.log1p(N * ga / be)
    el = abs(lg[0] - ld_ref) / abs(ld_ref)
    print(f"   column {ec:.2e} rho {er:.2e} delta {ed:.2e} logdet {el:.2e}", flush=True)
    # ln|C| = sum of N logs of pivots, each carrying the pivots' relative error
    # (2e-12 at N = 65536): N * 1e-15 relative
    assert ec < 1e-13 and er < tol and ed < tol and el < max(1e-12, N * 1e-15)
    # Gohberg-Semencul apply: w = C^{-1} y (Sherman-Morrison)
    psi = nm.steering([th1], N)[:, 0]
    w_ref = (y - ga * psi * np.vdot(psi, y) / (be + N * ga)) / be
    w = zeros_c(N)
    yCy = torch.zeros(1, dtype=torch.float64, device=DEV)
    sf.sfls_gs_apply(ctx, n, off, c2d(y), sf.SFLS_C128, rho, delta, w, yCy)
    torch.cuda.synchronize()
    ew = relerr(d2c(w), w_ref)
    ey = abs(float(yCy.cpu()[0]) - np.vdot(y, w_ref).real) / np.vdot(y, w_ref).real
    print(f"   w {ew:.2e} yCy {ey:.2e}", flush=True)
    assert ew < tol and ey < tol
    # diagonal sums
    outs = [zeros_c(2 * N - 1) for _ in range(4)]
    sf.sfls_omega(ctx, n, off, np.zeros(1, np.int64), rho, delta, *outs)
    torch.cuda.synchronize()
    for k, ref in enumerate(k1_omegas(th1, ga, be, N)):
        eo = relerr(d2c(outs[k]), ref)
        print(f"   omega_{'stvx'[k]} {eo:.2e}", flush=True)
        assert eo < tol
    # grid: q^G, s^G, r^G, t^G, Delta L and the argmin, FP64 and FP32; r^G and
    # t^G are length-L transforms of the closed forms D w and omega_t
    gbv, zeta = 0.7, 0.01
    r_ref = np.fft.fft(2 * np.pi * np.arange(N) * w_ref, L)
    tb = np.zeros(L, complex)
    tb[np.arange(-(N - 1), N) % L] = k1_omegas(th1, ga, be, N)[1]
    t_ref = L * np.fft.ifft(tb)
    d_ref = nm.delta_L(q_ref, s_ref, np.full(L, gbv), zeta)
    for prec in (sf.SFLS_FP64, sf.SFLS_MIXED):
        fdt = torch.float64 if prec == sf.SFLS_FP64 else torch.float32
        qG = torch.zeros(2 * L, dtype=fdt, device=DEV)
        sG = torch.zeros(L, dtype=fdt, device=DEV)
        dL = torch.zeros(L, dtype=fdt, device=DEV)
        am = torch.zeros(1, dtype=torch.int64, device=DEV)
        av = torch.zeros(1, dtype=torch.float64, device=DEV)
        rG = torch.zeros(2 * L, dtype=fdt, device=DEV)
        tG = torch.zeros(2 * L, dtype=fdt, device=DEV)
        sf.sfls_grid_eval(ctx, n, off, c2d(y), sf.SFLS_C128, rho, delta, np.array([L], np.int64),
                          np.zeros(1, np.int64), f64d([gbv]), f64d([zeta]), qG, sG, dL, am, av,
                          precision=prec, rG=rG, tG=tG)
        torch.cuda.synchronize()
        er = relerr(rG.cpu().numpy().astype(np.float64).view(np.complex128), r_ref)
        et = relerr(tG.cpu().numpy().astype(np.float64).view(np.complex128), t_ref)
        qh = qG.cpu().numpy().astype(np.float64).view(np.complex128)
        sh, dh = sG.cpu().numpy().astype(np.float64), dL.cpu().numpy().astype(np.float64)
        gtol = 1e-9 if prec == sf.SFLS_FP64 else 1e-4
        eq, es, ed2 = relerr(qh, q_ref), relerr(sh, s_ref), relerr(dh, d_ref)
        print(f"   grid prec={prec}: q {eq:.2e} s {es:.2e} dL {ed2:.2e} r {er:.2e} t {et:.2e} "
              f"argmin {int(am.cpu()[0])} (ref {int(np.argmin(d_ref))})", flush=True)
        assert eq < gtol and es < gtol and ed2 < gtol and er < gtol and et < gtol
        if prec == sf.SFLS_FP64:
            assert int(am.cpu()[0]) == int(np.argmin(d_ref))


@pytest.mark.parametrize("N", [32768, 65536])
def test_factor_and_apply_largest_sizes(ctx, N):
    """K = 20 at the largest sizes: C rho = delta_{N-1} e_{N-1} and C w = y to a
    small normwise backward error (FFT Toeplitz products), rho_{N-1} = 1,
    positive pivots, ln|C| against the determinant lemma."""
    st = states([N], 505 + N, kmax=20)
    t, g, bb, y = st[0]
    col = nm.toeplitz_column(t, g, bb, N)
    print(f"[largest factor] N={N} K={len(t)}", flush=True)
    n, off, rho, delta, lg = gpu_factor(ctx, [N], [col])
    r, d = d2c(rho), delta.cpu().numpy()
    e = np.zeros(N, complex)
    e[-1] = d[-1]
    normC = 2.0 * np.sum(np.abs(col))
    eta = np.max(np.abs(toeplitz_mv(col, r) - e)) / (normC * np.max(np.abs(r)) + d[-1])
    ll = lemma_logdet(t, g, bb, N)
    el = abs(lg[0] - ll) / max(1.0, abs(ll))
    w = zeros_c(N)
    sf.sfls_gs_apply(ctx, n, off, c2d(y), sf.SFLS_C128, rho, delta, w)
    torch.cuda.synchronize()
    w1 = d2c(w)
    etw = np.max(np.abs(toeplitz_mv(col, w1) - y)) / (normC * np.max(np.abs(w1)) + np.max(np.abs(y)))
    print(f"   backward error rho {eta:.2e} w {etw:.2e} logdet vs lemma {el:.2e}", flush=True)
    assert abs(r[-1] - 1.0) < 1e-12 and (d > 0).all()
    assert eta < 1e-12 and etw < 1e-12 and el < 1e-9
