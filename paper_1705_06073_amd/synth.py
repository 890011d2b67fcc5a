"""Seeded synthetic signals for the line-spectral-estimation workloads.

This module only draws inputs: frequencies, coefficients, noise and the
observation y = sum_k alpha_k Phi psi(theta_k) + w of the signal model (Sec. II,
eq. "model"): the complete-data case Phi = I, and incomplete observations
(Sec. IV) where Phi keeps M of the N samples, each scaled by a weight.  It holds none of the estimator's
arithmetic, so the CPU oracle and the HIP path can both consume its output.

Conventions
-----------
* psi(theta)_n = exp(j 2 pi n theta), n = 0..N-1 (the paper's 1-indexed
  exp(j2pi(n-1)theta) shifted to 0-indexing).
* Frequencies are drawn sequentially, each uniform on the part of [0,1) whose
  wrap-around distance to every earlier frequency exceeds ``sep``
  (Sec. VI-A; the wrap-around distance is the one of the footnote in Sec. II-F).
* SNR is ||Phi Psi alpha||^2 / (M beta) of the realised signal (Sec. VI-A;
  M = N for complete data); an instance with K = 0 gets beta = 1.
* Incomplete observations: the observed indices include the first and the
  last sample, the other M - 2 are drawn uniformly without replacement
  (Sec. VI-E); the weights are 1 (rows of the identity) unless a workload
  states otherwise.
* Seeds: 1705060730 + 1_000_000 * config + instance, PCG64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1705060730


def seed_for(config: int, instance: int) -> int:
    return SEED_BASE + 1_000_000 * int(config) + int(instance)


def wrap_distance(x, y):
    """d(x, y) = min(|x - y|, 1 - |x - y|) on [0, 1)."""
    a = np.abs(np.asarray(x, dtype=np.float64) - np.asarray(y, dtype=np.float64))
    a = np.mod(a, 1.0)
    return np.minimum(a, 1.0 - a)


def _wrap1(x: float, y: float) -> float:
    a = abs(x - y) % 1.0
    return min(a, 1.0 - a)


def draw_frequencies(rng: np.random.Generator, K: int, sep: float,
                     max_tries: int = 10_000) -> np.ndarray:
    """Sequential rejection sampling with minimum wrap-around separation.

    A candidate is compared with its two circular neighbours among the
    accepted frequencies (kept sorted): with separations of at least `sep`,
    every other accepted point is farther than these, so the decision is the
    one of a test against all of them."""
    import bisect
    while True:
        th: list[float] = []
        srt: list[float] = []
        ok = True
        for _ in range(K):
            for _try in range(max_tries):
                cand = rng.random()
                if srt:
                    j = bisect.bisect_left(srt, cand)
                    near = (srt[j % len(srt)], srt[j - 1])
                    if not all(_wrap1(cand, t) > sep for t in near):
                        continue
                th.append(cand)
                bisect.insort(srt, cand)
                break
            else:
                ok = False
                break
        if ok:
            return np.array(th, dtype=np.float64)


def draw_alpha(rng: np.random.Generator, K: int, kind: str) -> np.ndarray:
    """Coefficient distributions of the workloads.

    * ``cn``: alpha ~ CN(0, 1).
    * ``paper``: a ~ CN with standard deviation 0.8, alpha = a + 0.2 e^{j arg a}
      (Sec. VI-A), so |alpha| >= 0.2.
    * ``logamp20``: |alpha| = 10^{-U(0,1)} (20 dB power range), uniform phase.
    """
    if kind == "cn":
        return (rng.standard_normal(K) + 1j * rng.standard_normal(K)) / math.sqrt(2.0)
    if kind == "paper":
        a = 0.8 * (rng.standard_normal(K) + 1j * rng.standard_normal(K)) / math.sqrt(2.0)
        return a + 0.2 * np.exp(1j * np.angle(a))
    if kind == "logamp20":
        mag = 10.0 ** (-rng.random(K))
        ph = 2.0 * math.pi * rng.random(K)
        return mag * np.exp(1j * ph)
    raise ValueError(f"unknown alpha kind {kind!r}")


def clean_signal(theta: np.ndarray, alpha: np.ndarray, N: int) -> np.ndarray:
    """h = Psi(theta) alpha, built term by term in FP64."""
    n = np.arange(N, dtype=np.float64)
    h = np.zeros(N, dtype=np.complex128)
    for th, al in zip(theta, alpha):
        # exact reduction of n*theta mod 1 keeps the phase accurate at large N
        ph = np.mod(n * th, 1.0)
        h += al * np.exp(2j * math.pi * ph)
    return h


def clean_signal_blocked(theta: np.ndarray, alpha: np.ndarray, N: int, blk: int = 256) -> np.ndarray:
    """h = Psi(theta) alpha with e^{j2pi n theta} formed as the product of
    e^{j2pi a blk theta} and e^{j2pi b theta} (n = a blk + b, both phases
    reduced mod 1): equal to clean_signal up to the rounding of the phases
    (about N times the unit roundoff), with N/blk + blk instead of N
    exponentials per component, for long signals with many components."""
    nb = -(-N // blk)
    a = np.arange(nb, dtype=np.float64) * blk
    b = np.arange(blk, dtype=np.float64)
    h = np.zeros(nb * blk, dtype=np.complex128)
    for th, al in zip(theta, alpha):
        hi = np.exp(2j * math.pi * np.mod(a * th, 1.0))
        lo = al * np.exp(2j * math.pi * np.mod(b * th, 1.0))
        h += np.outer(hi, lo).ravel()
    return h[:N]


@dataclass
class Instance:
    N: int
    K: int
    theta: np.ndarray
    alpha: np.ndarray
    beta: float
    snr_db: float
    y: np.ndarray           # complex128 or complex64, as the workload states
    seed: int = 0
    meta: dict = field(default_factory=dict)
    # incomplete observations (Sec. IV): y holds the M samples at the
    # strictly increasing indices idx, weighted by phi (None: all N samples)
    idx: np.ndarray | None = None
    phi: np.ndarray | None = None

    @property
    def M(self) -> int:
        return self.N if self.idx is None else len(self.idx)


def make_instance(rng: np.random.Generator, N: int, K: int, sep: float,
                  alpha_kind: str, snr_db: float, dtype=np.complex128,
                  seed: int = 0, blocked: bool = False) -> Instance:
    theta = draw_frequencies(rng, K, sep) if K > 0 else np.zeros(0)
    alpha = draw_alpha(rng, K, alpha_kind) if K > 0 else np.zeros(0, np.complex128)
    h = clean_signal_blocked(theta, alpha, N) if blocked else clean_signal(theta, alpha, N)
    if K > 0 and math.isfinite(snr_db):
        beta = float(np.vdot(h, h).real / (N * 10.0 ** (snr_db / 10.0)))
    elif K > 0:
        beta = 0.0
    else:
        beta = 1.0
    w = math.sqrt(beta / 2.0) * (rng.standard_normal(N) + 1j * rng.standard_normal(N))
    y = (h + w).astype(dtype)
    return Instance(N=N, K=K, theta=theta, alpha=alpha, beta=beta, snr_db=snr_db,
                    y=y, seed=seed)


def draw_observed(rng: np.random.Generator, N: int, M: int) -> np.ndarray:
    """Observed sample indices: 0 and N-1, and M-2 others drawn uniformly
    without replacement from 1..N-2 (Sec. VI-E), in increasing order."""
    if not 2 <= M <= N:
        raise ValueError("need 2 <= M <= N")
    inner = rng.choice(np.arange(1, N - 1), size=M - 2, replace=False)
    return np.sort(np.concatenate([[0, N - 1], inner]).astype(np.int64))


def draw_weights(rng: np.random.Generator, M: int, kind: str) -> np.ndarray:
    """Weights phi_m of Phi: ``ones`` (rows of the identity, Sec. VI-E),
    ``phase`` (unit modulus, uniform phase), ``scaled`` (modulus log-uniform on
    [0.5, 2], uniform phase)."""
    if kind == "ones":
        return np.ones(M, np.complex128)
    ph = np.exp(2j * math.pi * rng.random(M))
    if kind == "phase":
        return ph
    if kind == "scaled":
        return ph * 2.0 ** (2.0 * rng.random(M) - 1.0)
    raise ValueError(f"unknown weight kind {kind!r}")


def make_incomplete_instance(rng: np.random.Generator, N: int, M: int, K: int, sep: float,
                             alpha_kind: str, snr_db: float, dtype=np.complex128,
                             seed: int = 0, weights: str = "ones") -> Instance:
    """y = Phi Psi(theta) alpha + w with Phi of M weighted rows of the identity."""
    theta = draw_frequencies(rng, K, sep) if K > 0 else np.zeros(0)
    alpha = draw_alpha(rng, K, alpha_kind) if K > 0 else np.zeros(0, np.complex128)
    idx = draw_observed(rng, N, M)
    phi = draw_weights(rng, M, weights)
    h = phi * clean_signal(theta, alpha, N)[idx]
    if K > 0 and math.isfinite(snr_db):
        beta = float(np.vdot(h, h).real / (M * 10.0 ** (snr_db / 10.0)))
    elif K > 0:
        beta = 0.0
    else:
        beta = 1.0
    w = math.sqrt(beta / 2.0) * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    return Instance(N=N, K=K, theta=theta, alpha=alpha, beta=beta, snr_db=snr_db,
                    y=(h + w).astype(dtype), seed=seed, idx=idx, phi=phi,
                    meta={"weights": weights})


# ---------------------------------------------------------------------------
# The workloads.  Config numbering: 0 = small single instance (N=64),
# 1 = single instance N=1024, 2 = batch of 256 at N=4096, 3 = uneven batch,
# 4 = serving stream.
# ---------------------------------------------------------------------------

def workload_n64(instance: int = 0) -> Instance:
    """N=64, K=3, separation 1/N, alpha ~ CN(0,1), SNR 20 dB, complex128."""
    s = seed_for(0, instance)
    rng = np.random.Generator(np.random.PCG64(s))
    return make_instance(rng, 64, 3, 1.0 / 64, "cn", 20.0, np.complex128, s)


def workload_n1024(instance: int = 0) -> Instance:
    """N=1024, K=20, separation 2/N, |alpha| over 20 dB, SNR 15 dB, complex64."""
    s = seed_for(1, instance)
    rng = np.random.Generator(np.random.PCG64(s))
    return make_instance(rng, 1024, 20, 2.0 / 1024, "logamp20", 15.0, np.complex64, s)


def workload_n4096(instance: int) -> Instance:
    """N=4096, K ~ Poisson(40), separation 1/N, alpha ~ CN(0,1), SNR ~ U[0,30] dB."""
    s = seed_for(2, instance)
    rng = np.random.Generator(np.random.PCG64(s))
    K = int(rng.poisson(40))
    snr = float(rng.uniform(0.0, 30.0))
    return make_instance(rng, 4096, K, 1.0 / 4096, "cn", snr, np.complex128, s)


def workload_uneven(instance: int, blocked: bool = False) -> Instance:
    """N log-uniform on [128, 16384], K ~ Poisson(N/64), SNR ~ U[5,30] dB
    (blocked: the phase-split synthesis, for many long signals)."""
    s = seed_for(3, instance)
    rng = np.random.Generator(np.random.PCG64(s))
    N = int(round(math.exp(rng.uniform(math.log(128), math.log(16384)))))
    K = int(rng.poisson(N / 64.0))
    snr = float(rng.uniform(5.0, 30.0))
    return make_instance(rng, N, K, 1.0 / N, "cn", snr, np.complex128, s, blocked=blocked)


SERVING_SIZES = (256, 1024, 4096, 16384, 65536)
SERVING_WEIGHTS = (0.3, 0.3, 0.2, 0.15, 0.05)


def workload_serving_signal(N: int, instance: int) -> Instance:
    """A serving request of length N: K ~ Poisson(N/64), separation 1/N,
    alpha ~ CN(0,1), SNR ~ U[5,30] dB, complex64."""
    s = seed_for(4, instance) + 100_000 * int(math.log2(N))
    rng = np.random.Generator(np.random.PCG64(s))
    K = int(rng.poisson(N / 64.0))
    snr = float(rng.uniform(5.0, 30.0))
    return make_instance(rng, N, K, 1.0 / N, "cn", snr, np.complex64, s, blocked=True)


def serving_stream(rate: float, duration: float, seed_instance: int = 0, sizes=None,
                   weights=None):
    """Arrival times (s, ascending) of a Poisson process of `rate` requests/s
    over `duration` seconds and each request's N drawn from SERVING_SIZES with
    SERVING_WEIGHTS (or from `sizes`, uniformly unless `weights` are given)."""
    rng = np.random.Generator(np.random.PCG64(seed_for(4, seed_instance)))
    n_exp = int(rate * duration * 1.2 + 100)
    t = np.cumsum(rng.exponential(1.0 / rate, n_exp))
    t = t[t < duration]
    sz = SERVING_SIZES if sizes is None else sizes
    wt = (SERVING_WEIGHTS if sizes is None else [1.0 / len(sz)] * len(sz)) if weights is None \
        else weights
    n = rng.choice(np.array(sz, np.int64), size=len(t), p=np.array(wt, dtype=float))
    return t, n


def workload_paper_snr(instance: int, snr_db: float, N: int = 128, K: int = 10) -> Instance:
    """The accuracy-vs-SNR experiment: N=128, K=10, separation 2/N, paper's alpha."""
    s = seed_for(7, instance) + int(round(snr_db * 1000))
    rng = np.random.Generator(np.random.PCG64(s))
    return make_instance(rng, N, K, 2.0 / N, "paper", snr_db, np.complex128, s)


def draw_pairs(rng: np.random.Generator, npairs: int, pair_sep: float, sep: float,
               max_tries: int = 10_000) -> np.ndarray:
    """Frequencies in `npairs` pairs {t, t + pair_sep}: the pairs' positions t
    are drawn one after another, uniformly among the positions whose two
    frequencies are farther than `sep` (wrap distance) from every frequency of
    the pairs drawn before (the placement of Sec. VI-A applied to pairs)."""
    while True:
        th: list[float] = []
        for _ in range(npairs):
            for _try in range(max_tries):
                t = rng.random()
                pair = (t, (t + pair_sep) % 1.0)
                if all(_wrap1(p, q) > sep for p in pair for q in th):
                    th.extend(pair)
                    break
            else:
                break
        if len(th) == 2 * npairs:
            return np.array(th, dtype=np.float64)


def workload_paper_pairs(instance: int, pair_sep_n: float, N: int = 128, npairs: int = 5,
                         snr_db: float = 20.0) -> Instance:
    """The super-resolution experiment: N=128, 5 pairs (K=10) whose members are
    pair_sep_n / N apart, pairs at least 2/N apart, paper's alpha, 20 dB."""
    s = seed_for(8, instance) + int(round(pair_sep_n * 1000)) * 1000
    rng = np.random.Generator(np.random.PCG64(s))
    theta = draw_pairs(rng, npairs, pair_sep_n / N, 2.0 / N)
    K = len(theta)
    alpha = draw_alpha(rng, K, "paper")
    h = clean_signal(theta, alpha, N)
    beta = float(np.vdot(h, h).real / (N * 10.0 ** (snr_db / 10.0)))
    w = math.sqrt(beta / 2.0) * (rng.standard_normal(N) + 1j * rng.standard_normal(N))
    return Instance(N=N, K=K, theta=theta, alpha=alpha, beta=beta, snr_db=snr_db, y=h + w,
                    seed=s, meta={"pair_sep_n": pair_sep_n})


def workload_paper_mton(instance: int, ratio: float, N: int = 128, K: int = 10,
                        snr_db: float = 20.0) -> Instance:
    """The incomplete-data experiment (Fig. MtoN): N=128, K=10, separation 2/N,
    paper's alpha, 20 dB, M = round(ratio N) rows of the identity."""
    s = seed_for(9, instance) + int(round(ratio * 1000)) * 1000
    rng = np.random.Generator(np.random.PCG64(s))
    M = int(round(ratio * N))
    return make_incomplete_instance(rng, N, M, K, 2.0 / N, "paper", snr_db, np.complex128, s)


def workload_incomplete_n4096(instance: int) -> Instance:
    """Incomplete data at the runtime experiment's size (Fig. runtime_N, right):
    N=4096, M=3072 rows of the identity, K=15, separation 2/N, paper's alpha,
    20 dB, complex64."""
    s = seed_for(10, instance)
    rng = np.random.Generator(np.random.PCG64(s))
    return make_incomplete_instance(rng, 4096, 3072, 15, 2.0 / 4096, "paper", 20.0,
                                    np.complex64, s)


def workload_incomplete_small(instance: int, weights: str = "scaled") -> Instance:
    """Small incomplete instances for parity: N uniform on [48, 320], M/N
    uniform on [0.3, 0.9], K uniform on 1..6, separation 2/N, alpha ~ CN(0,1),
    SNR uniform on [5, 30] dB, weighted rows (``weights``)."""
    s = seed_for(11, instance)
    rng = np.random.Generator(np.random.PCG64(s))
    N = int(rng.integers(48, 321))
    M = max(4, int(round(float(rng.uniform(0.3, 0.9)) * N)))
    K = int(rng.integers(1, 7))
    snr = float(rng.uniform(5.0, 30.0))
    return make_incomplete_instance(rng, N, M, K, 2.0 / N, "cn", snr, np.complex128, s,
                                    weights=weights)


def pack_batch(instances, dtype=np.complex128):
    """Concatenate y of a ragged batch; returns (y_flat, n, off)."""
    n = np.array([inst.N for inst in instances], dtype=np.int64)
    off = np.zeros(len(instances), dtype=np.int64)
    if len(instances) > 1:
        off[1:] = np.cumsum(n)[:-1]
    y = np.concatenate([inst.y.astype(dtype) for inst in instances]) if instances else \
        np.zeros(0, dtype)
    return y, n, off
