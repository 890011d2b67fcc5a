"""Host build of the device driver's state machine, fed by oracle evaluations.

The estimator's control flow (csrc/driver.hpp, run on the GPU one thread per
instance) is compiled for the host with g++ and driven here: every evaluation
it requests is computed by the dense oracle (oracle.numerics), and the grid
candidates are chosen from the oracle's exact Delta L on the grid, the way the
selection kernel does.  This checks the control flow against the oracle's
estimator without a GPU (test infrastructure only)."""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import tempfile

import numpy as np

from oracle import estimator as oe
from oracle import incomplete as inc
from oracle import mmv
from oracle import numerics as nm

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1705_06073_amd", "csrc")
_lib = None


def lib():
    global _lib
    if _lib is None:
        out = os.path.join(tempfile.mkdtemp(prefix="sfls_drv_"), "driver_host.so")
        subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-pthread", f"-I{CSRC}",
                        os.path.join(HERE, "host", "driver_host.cpp"), "-o", out],
                       check=True, capture_output=True)
        _lib = ctypes.CDLL(out)
    return _lib


class DrvParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("tau", "tol_obj", "tol_newton", "eps_beta_rel", "eps_L", "approx_ratio",
                 "approx_min_dist", "ls_c1", "curv_eps", "polish_tol", "polish_ftol")] + \
               [(n, ctypes.c_int32) for n in
                ("J", "max_inner", "max_outer", "approx_max_iters", "approx_use_tau", "ls_max",
                 "polish_max_iters", "cand_cap")]


class DrvState(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("phase", "it", "inner", "pit", "ls_trial", "K", "approx_on", "z_changed",
                 "cur_valid", "converged", "cap_hit", "polish", "mem_n", "mem_head", "kstar",
                 "status", "nevals", "done", "saved", "pad_")] + \
               [(n, ctypes.c_double) for n in
                ("beta", "zeta", "eps_beta", "yy", "L_prev", "f_cur", "lam2", "alpha", "amax",
                 "gd", "nu0")]


_PTRS = ["th", "ga", "th_e", "ga_e", "K_e", "beta_e", "req", "gbar_e", "zeta_e", "g", "d", "Sm",
         "Ym", "rhom", "am", "gt", "q_save", "ev_q", "ev_r", "ev_u", "ev_s", "ev_t", "ev_v", "ev_x",
         "logdet", "yCy", "ww", "lev_status", "cand", "ncand", "cand_q", "cand_s", "cbuf_dl",
         "cbuf_gh", "cbuf_l", "out_K", "out_theta", "out_alpha", "out_gamma", "out_beta",
         "out_zeta", "out_obj", "out_iters", "out_evals", "out_status",
         "sh_th_e", "sh_ga_e", "sh_K_e", "sh_beta_e", "sh_gbar_e", "sh_zeta_e", "sh_req",
         "sh_wish", "sh_ev_q", "sh_ev_r", "sh_ev_u", "sh_ev_s", "sh_ev_t", "sh_ev_v", "sh_ev_x",
         "sh_logdet", "sh_yCy", "sh_ww", "sh_lev_status"]


class DrvArrays(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("L", ctypes.c_int), ("kcap", ctypes.c_int),
                ("Mo", ctypes.c_int), ("G", ctypes.c_int), ("vk", ctypes.c_int64), ("vc", ctypes.c_int64),
                ("vo", ctypes.c_int64)] + \
               [(n, ctypes.c_void_p) for n in _PTRS]


REQ_EVAL, REQ_GRID, REQ_APPROX = 1, 2, 4


class HostDriver:
    """One instance: arrays in numpy, evaluations from the oracle.  y is one
    vector, or G x N for the multiple-vector model (evaluations from the MMV
    oracle); with ``obs`` (an oracle.incomplete.Observation) y holds the
    observed samples (evaluations from the incomplete-data oracle)."""

    def __init__(self, y, params: oe.Params | None = None, kcap: int | None = None,
                 cand_cap: int = 256, obs=None, shadow: bool = False):
        self.p = p = params or oe.Params()
        self.y = np.asarray(y, np.complex128)
        self.obs = obs
        self.mmv = self.y.ndim == 2
        G = self.G = self.y.shape[0] if self.mmv else 1
        N = self.N = self.y.shape[-1] if obs is None else obs.N
        M = self.M = self.y.shape[-1]
        self.L = p.grid_size(N)
        kc = self.kcap = min(kcap or M, M)
        J = p.lbfgs_J
        self.cand_cap = cand_cap
        f64 = lambda n: np.zeros(max(1, n), np.float64)  # noqa: E731
        i32 = lambda n: np.zeros(max(1, n), np.int32)  # noqa: E731
        a = self.a = {
            "th": f64(kc), "ga": f64(kc), "th_e": f64(kc), "ga_e": f64(kc), "K_e": i32(1),
            "beta_e": f64(1), "req": i32(1), "gbar_e": f64(1), "zeta_e": f64(1),
            "g": f64(2 * kc), "d": f64(2 * kc), "Sm": f64(J * 2 * kc), "Ym": f64(J * 2 * kc),
            "rhom": f64(J), "am": f64(J), "gt": f64(2 * kc), "q_save": f64(2 * G * kc),
            **{f"ev_{q}": f64(2 * G * kc) for q in "qru"},
            **{f"ev_{q}": f64(2 * kc) for q in "stvx"},
            "logdet": f64(1), "yCy": f64(1), "ww": f64(1), "lev_status": i32(1),
            "cand": i32(cand_cap + 1), "ncand": i32(1), "cand_q": f64(2 * G * (cand_cap + 1)),
            "cand_s": f64(cand_cap + 1), "cbuf_dl": f64(cand_cap + 1),
            "cbuf_gh": f64(cand_cap + 1), "cbuf_l": i32(cand_cap + 1),
            "out_K": np.zeros(1, np.int64), "out_theta": f64(kc), "out_alpha": f64(2 * G * kc),
            "out_gamma": f64(kc), "out_beta": f64(1), "out_zeta": f64(1), "out_obj": f64(1),
            "out_iters": i32(1), "out_evals": i32(1), "out_status": i32(1)}
        # shadow slot of the speculative line-search trials (complete data,
        # one vector): every wish is granted and served from the oracle
        self.shadow = shadow and obs is None and not self.mmv
        if self.shadow:
            a.update({"sh_th_e": f64(kc), "sh_ga_e": f64(kc), "sh_K_e": i32(1),
                      "sh_beta_e": f64(1), "sh_gbar_e": f64(1), "sh_zeta_e": f64(1),
                      "sh_req": i32(1), "sh_wish": i32(1),
                      **{f"sh_ev_{q}": f64(2 * kc) for q in "qrustvx"},
                      "sh_logdet": f64(1), "sh_yCy": f64(1), "sh_ww": f64(1),
                      "sh_lev_status": i32(1)})
        self.vk, self.vc = 2 * kc, 2 * (cand_cap + 1)
        self.arr = DrvArrays(N, self.L, kc, M, G, self.vk, self.vc, self.vk,
                             *[a[n].ctypes.data if n in a else None for n in _PTRS])
        self.shadow_served = 0
        self.prm = DrvParams(p.tau, p.tol_obj, p.tol_newton, p.eps_beta_rel, p.eps_L,
                             p.approx_ratio, p.approx_min_dist, p.ls_c1, p.curv_eps,
                             p.polish_tol, p.polish_ftol, J, p.max_inner, p.max_outer,
                             p.approx_max_iters, int(p.approx_use_tau), p.ls_max,
                             p.polish_max_iters, cand_cap)
        self.st = DrvState()
        self.st.phase = 0
        self.st.yy = (sum(float(np.vdot(v, v).real) for v in self.y) / G if self.mmv
                      else float(np.vdot(self.y, self.y).real))
        self.requests: list[tuple] = []
        self.phases: list[tuple] = []
        self.last = None

    def _evaluate(self):
        """Serve the request: an evaluation at the requested point (REQ_EVAL), and
        the grid stage on the last evaluation (REQ_GRID)."""
        a = self.a
        K = int(a["K_e"][0])
        th, ga, beta = a["th_e"][:K].copy(), a["ga_e"][:K].copy(), float(a["beta_e"][0])
        bits = int(a["req"][0])
        self.requests.append((bits, K, th, ga, beta))
        st = self.st
        self.phases.append((st.phase, st.it, st.inner, st.pit, st.polish, st.ls_trial))
        if bits & REQ_EVAL and self.mmv:
            ev = self.last = mmv.EvaluationMMV(self.y, th, ga, beta)
            a["logdet"][0] = ev.logdet
            a["yCy"][0] = ev.yCy
            a["ww"][0] = sum(float(np.vdot(w, w).real) for w in ev.w)
            for q in "qru":
                for g in range(self.G):
                    v = np.asarray(ev.act[q][g], np.complex128)
                    a[f"ev_{q}"][g * self.vk:g * self.vk + 2 * K] = v.view(np.float64)
            for q in "stvx":
                a[f"ev_{q}"][:2 * K] = np.asarray(ev.act[q], np.complex128).view(np.float64)
            a["lev_status"][0] = 0
        elif bits & REQ_EVAL:
            ev = self.last = (nm.Evaluation(self.y, th, ga, beta) if self.obs is None else
                              inc.EvaluationIncomplete(self.y, self.obs, th, ga, beta))
            a["logdet"][0] = ev.logdet
            a["yCy"][0] = ev.yCy
            wm = ev.w if self.obs is None else ev.wM     # ||C^{-1} y||^2 in the M samples
            a["ww"][0] = float(np.vdot(wm, wm).real)
            for q in "qrustvx":
                v = np.asarray(ev.act[q], np.complex128)
                a[f"ev_{q}"][:2 * K] = v.view(np.float64)
            a["lev_status"][0] = 0
        ev = self.last
        if bits & REQ_GRID:
            zeta, gb = float(a["zeta_e"][0]), float(a["gbar_e"][0])
            qG, sG = ev.grid(self.L)
            if self.mmv:
                Q = mmv.sum_q2(qG)
                gbv = mmv.gamma_hat(Q, sG, self.G) if gb <= 0 else np.full(self.L, gb)
                dl = mmv.delta_L(Q, sG, gbv, zeta, self.G)
            else:
                gbv = nm.gamma_hat(qG, sG) if gb <= 0 else np.full(self.L, gb)
                dl = nm.delta_L(qG, sG, gbv, zeta)
            dl = np.where(np.isnan(dl), np.inf, dl)
            lmin = int(np.argmin(dl))
            cands = [lmin]
            if bits & REQ_APPROX:
                loc = np.nonzero((dl <= np.roll(dl, 1)) & (dl <= np.roll(dl, -1)))[0]
                thr = dl[lmin] / self.p.approx_ratio + 1e-9 * abs(dl[lmin])
                keep = [int(l) for l in loc if dl[l] <= thr]
                keep.sort(key=lambda l: (dl[l], l))
                cands += keep[:self.cand_cap]
            ths = np.array(cands, np.float64) / self.L
            sc = nm.s_at(ev.omega[0], ths).real
            n = len(cands)
            a["cand"][:n] = cands
            a["ncand"][0] = n
            for g, w in enumerate(ev.w if self.mmv else [ev.w]):
                qc = np.asarray(nm.q_at(w, ths), np.complex128)
                a["cand_q"][g * self.vc:g * self.vc + 2 * n] = qc.view(np.float64)
            a["cand_s"][:n] = sc

    def _grant_shadow(self):
        """A wish of the last step becomes a shadow evaluation for the next
        (the device grants it while compute units are free)."""
        a = self.a
        a["sh_req"][0] = 0
        if not a["sh_wish"][0]:
            return
        a["sh_wish"][0] = 0
        K = int(a["sh_K_e"][0])
        th, ga = a["sh_th_e"][:K].copy(), a["sh_ga_e"][:K].copy()
        ev = nm.Evaluation(self.y, th, ga, float(a["sh_beta_e"][0]))
        a["sh_logdet"][0] = ev.logdet
        a["sh_yCy"][0] = ev.yCy
        a["sh_ww"][0] = float(np.vdot(ev.w, ev.w).real)
        for q in "qrustvx":
            a[f"sh_ev_{q}"][:2 * K] = np.asarray(ev.act[q], np.complex128).view(np.float64)
        a["sh_lev_status"][0] = 0
        a["sh_req"][0] = REQ_EVAL
        self.shadow_served += 1

    def run(self, max_steps=100000, lanes: int = 0):
        """Step the driver to completion.  lanes > 0 runs each step with that
        many lanes in lockstep and records, per step, how many lanes ended in a
        state different from lane 0's (``self.lane_diffs``)."""
        L = lib()
        self.lane_diffs = []
        sizes = (ctypes.c_int * 3)()
        L.drv_sizes(sizes)
        assert tuple(sizes) == (ctypes.sizeof(DrvParams), ctypes.sizeof(DrvState),
                                ctypes.sizeof(DrvArrays)), "driver structs out of sync"
        # (request the step consumed, request it made), per step
        self.req_seq = []
        prev = 0
        for _ in range(max_steps):
            if lanes > 0:
                self.lane_diffs.append(L.drv_step_lanes(
                    ctypes.byref(self.prm), ctypes.byref(self.st), ctypes.byref(self.arr), lanes))
            else:
                L.drv_step(ctypes.byref(self.prm), ctypes.byref(self.st), ctypes.byref(self.arr))
            req = int(self.a["req"][0]) if not self.st.done else 0
            self.req_seq.append((prev, req))
            prev = req
            if self.st.done:
                break
            if self.a["req"][0]:
                self._evaluate()
            if self.shadow:
                self._grant_shadow()
        a = self.a
        K = int(a["out_K"][0])
        oa = a["out_alpha"]
        alpha = (np.stack([oa[g * self.vk:g * self.vk + 2 * K].view(np.complex128)
                           for g in range(self.G)]) if self.mmv
                 else oa[:2 * K].view(np.complex128).copy())
        return dict(K=K, theta=a["out_theta"][:K].copy(), gamma=a["out_gamma"][:K].copy(),
                    alpha=alpha,
                    beta=float(a["out_beta"][0]), zeta=float(a["out_zeta"][0]),
                    objective=float(a["out_obj"][0]), iterations=int(a["out_iters"][0]),
                    evaluations=int(a["out_evals"][0]), status=int(a["out_status"][0]))
