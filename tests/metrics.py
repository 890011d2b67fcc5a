"""Accuracy metrics of Sec. VI-A (test tooling): wrap-around distance, Hungarian
matching minimising the squared distances, BSR / CSR / NMSE."""
import numpy as np
from scipy.optimize import linear_sum_assignment

from paper_1705_06073_amd.synth import clean_signal, wrap_distance


def match(theta_true, theta_est):
    """Optimal assignment of estimates to true frequencies (squared wrap distance)."""
    if len(theta_true) == 0 or len(theta_est) == 0:
        return np.zeros(0, int), np.zeros(0, int)
    d = wrap_distance(np.asarray(theta_true)[:, None], np.asarray(theta_est)[None, :])
    return linear_sum_assignment(d ** 2)


def block_success(theta_true, theta_est, N):
    """Correct model order and max matched distance < 0.5/N."""
    if len(theta_true) != len(theta_est):
        return False
    if len(theta_true) == 0:
        return True
    r, c = match(theta_true, theta_est)
    return bool(np.max(wrap_distance(np.asarray(theta_true)[r], np.asarray(theta_est)[c])) < 0.5 / N)


def component_success_rate(theta_true, theta_est, N):
    K, Kh = len(theta_true), len(theta_est)
    if K + Kh == 0:
        return 1.0
    tt, te = np.asarray(theta_true), np.asarray(theta_est)
    a = sum(bool(np.min(wrap_distance(x, tt)) < 0.5 / N) for x in te) if K else 0
    b = sum(bool(np.min(wrap_distance(x, te)) < 0.5 / N) for x in tt) if Kh else 0
    return (a + b) / (Kh + K)


def nmse(theta_true, alpha_true, theta_est, alpha_est, N):
    h = clean_signal(np.asarray(theta_true), np.asarray(alpha_true), N)
    he = clean_signal(np.asarray(theta_est), np.asarray(alpha_est), N)
    return float(np.vdot(he - h, he - h).real / np.vdot(h, h).real)


def oracle_ls_nmse(inst):
    """Least squares for alpha with the true frequencies (the "Oracle" curve of
    Figs. snr and MtoN): A = Phi Psi(theta) on the observed samples, the NMSE
    taken on the whole length-N signal."""
    n = np.arange(inst.N) if inst.idx is None else inst.idx
    A = np.exp(2j * np.pi * np.outer(n, inst.theta))
    if inst.idx is not None:
        A = inst.phi[:, None] * A
    a, *_ = np.linalg.lstsq(A, inst.y.astype(np.complex128), rcond=None)
    return nmse(inst.theta, inst.alpha, inst.theta, a, inst.N)
