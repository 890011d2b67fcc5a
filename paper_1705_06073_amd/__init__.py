"""Superfast line spectral estimation on MI355X (gfx950).

Thin ctypes binding of the C ABI declared in ``include/sfls.h``.  Every
function here only marshals arguments: device buffers are torch tensors on
the GPU (``data_ptr()``), sizes and offsets are host int64 arrays, and the
work is enqueued on torch's current stream.  All arithmetic runs in the HIP
kernels of ``lib/libsfls.so``; if that library is missing the binding raises
instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libsfls.so")

SFLS_OK, SFLS_NOTCONV = 0, 1
SFLS_EINVAL, SFLS_ENOMEM, SFLS_EDEVICE, SFLS_ENOTPD, SFLS_ECAPACITY, SFLS_EUNSUPPORTED = \
    -1, -2, -3, -4, -5, -6
SFLS_EAGAIN = -7
SFLS_FP64, SFLS_MIXED = 0, 1
SFLS_C64, SFLS_C128 = 0, 1
SFLS_MAX_N = 65536
SFLS_GRID_Q, SFLS_GRID_S, SFLS_GRID_R, SFLS_GRID_T, SFLS_GRID_DL, SFLS_GRID_ARGMIN = \
    1, 2, 4, 8, 16, 32

EXPORTS = ["sfls_params_default", "sfls_create", "sfls_destroy", "sfls_strerror",
           "sfls_last_error", "sfls_version", "sfls_toeplitz_column", "sfls_factor",
           "sfls_gs_apply", "sfls_gs_apply_noalloc", "sfls_omega", "sfls_grid_eval", "sfls_active_eval", "sfls_estimate",
           "sfls_estimate_mmv", "sfls_incomplete_eval", "sfls_estimate_incomplete",
           "sfls_set_timing", "sfls_reset_stats", "sfls_kernel_stats", "sfls_last_run",
           "sfls_set_factor", "sfls_set_nufft", "sfls_set_schur_lds", "sfls_set_speculation", "sfls_server_config_default",
           "sfls_server_create", "sfls_server_destroy", "sfls_server_footprint",
           "sfls_server_submit", "sfls_server_submit_many", "sfls_server_launch",
           "sfls_server_wait", "sfls_server_step", "sfls_server_poll", "sfls_server_get_stats"]
SFLS_FACTOR_AUTO, SFLS_FACTOR_LEVINSON, SFLS_FACTOR_SCHUR = 0, 1, 2
SFLS_SF_MAX_K = 64  # largest model order of the semifast (incomplete-data) evaluation
SFLS_NUFFT_AUTO, SFLS_NUFFT_OFF, SFLS_NUFFT_ON = 0, 1, 2


class SflsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"sfls status {status}: {msg}")
        self.status = status


class sfls_params(ctypes.Structure):
    _fields_ = [
        ("L_mult", ctypes.c_double), ("tau", ctypes.c_double),
        ("lbfgs_J", ctypes.c_int32), ("max_inner", ctypes.c_int32),
        ("max_outer", ctypes.c_int32), ("approx_max_iters", ctypes.c_int32),
        ("approx_use_tau", ctypes.c_int32), ("ls_max", ctypes.c_int32),
        ("polish_max_iters", ctypes.c_int32), ("cand_cap", ctypes.c_int32),
        ("tol_obj", ctypes.c_double), ("tol_newton", ctypes.c_double),
        ("eps_beta_rel", ctypes.c_double), ("eps_L", ctypes.c_double),
        ("approx_ratio", ctypes.c_double), ("approx_min_dist", ctypes.c_double),
        ("ls_c1", ctypes.c_double), ("curv_eps", ctypes.c_double),
        ("polish_tol", ctypes.c_double), ("polish_ftol", ctypes.c_double),
        ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class sfls_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64),
                ("seconds", ctypes.c_double), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class sfls_run_stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("evals", ctypes.c_int64),
                ("grid_evals", ctypes.c_int64), ("wall_seconds", ctypes.c_double)]


class sfls_server_config(ctypes.Structure):
    _fields_ = [("max_n", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("ydtype", ctypes.c_int32), ("hbm_bytes", ctypes.c_uint64),
                ("kcap_shift", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class sfls_result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("n", ctypes.c_int64), ("K", ctypes.c_int64),
                ("comp_off", ctypes.c_int64), ("beta", ctypes.c_double),
                ("zeta", ctypes.c_double), ("objective", ctypes.c_double),
                ("iters", ctypes.c_int32), ("evals", ctypes.c_int32),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_done", ctypes.c_double)]


class sfls_server_stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("in_flight", ctypes.c_int64),
                ("units_used", ctypes.c_int64), ("units_total", ctypes.c_int64),
                ("bytes_per_unit", ctypes.c_uint64), ("bytes_reserved", ctypes.c_uint64),
                ("gpu_seconds", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)


def lib() -> ctypes.CDLL:
    """Load libsfls.so (built by ``python -m paper_1705_06073_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -m paper_1705_06073_amd.build); there is no fallback")
    # torch ships its own HIP runtime under the same soname; load it first so
    # that the process has one runtime whichever module is imported first.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, st = ctypes.c_int32, ctypes.c_int64, ctypes.c_int
    L.sfls_params_default.argtypes = [ctypes.POINTER(sfls_params)]
    L.sfls_params_default.restype = None
    L.sfls_create.argtypes = [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_size_t]
    L.sfls_create.restype = st
    L.sfls_destroy.argtypes = [_P]
    L.sfls_destroy.restype = st
    L.sfls_strerror.argtypes = [st]
    L.sfls_strerror.restype = ctypes.c_char_p
    L.sfls_last_error.argtypes = [_P]
    L.sfls_last_error.restype = ctypes.c_char_p
    L.sfls_version.argtypes = []
    L.sfls_version.restype = ctypes.c_char_p
    L.sfls_toeplitz_column.argtypes = [_P, i64, _I64P, _I64P, _I64P, _I64P, _P, _P, _P, _P, _P]
    L.sfls_toeplitz_column.restype = st
    L.sfls_factor.argtypes = [_P, i64, _I64P, _I64P, _P, _P, _P, _P, _P, _P, _P]
    L.sfls_factor.restype = st
    L.sfls_gs_apply.argtypes = [_P, i64, _I64P, _I64P, _P, i32, _P, _P, _P, _P, _P, _P]
    L.sfls_gs_apply.restype = st
    L.sfls_gs_apply_noalloc.argtypes = [_P, i64, _I64P, _I64P, _P, i32, _P, _P, _P, _P, _P, _P]
    L.sfls_gs_apply_noalloc.restype = st
    L.sfls_omega.argtypes = [_P, i64, _I64P, _I64P, _I64P, _P, _P, _P, _P, _P, _P, _P]
    L.sfls_omega.restype = st
    L.sfls_grid_eval.argtypes = [_P, i64, _I64P, _I64P, _P, i32, _P, _P, _I64P, _I64P, _P, _P,
                                 ctypes.c_uint32, _P, _P, _P, _P, _P, _P, _P, i32, _P]
    L.sfls_grid_eval.restype = st
    L.sfls_active_eval.argtypes = [_P, i64, _I64P, _I64P, _P, _P, _P, _I64P, _I64P, _P,
                                   _P, _P, _P, _P, _P, _P, _P, _P]
    L.sfls_active_eval.restype = st
    L.sfls_estimate.argtypes = [_P, i64, _I64P, _I64P, _P, i32, ctypes.POINTER(sfls_params),
                                _I64P, _I64P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.sfls_estimate.restype = st
    L.sfls_estimate_mmv.argtypes = [_P, i64, _I64P, _I64P, i32, _P, i64, i32,
                                    ctypes.POINTER(sfls_params), _I64P, _I64P, _P, _P, _P, i64,
                                    _P, _P, _P, _P, _P, _P, _P, _P]
    L.sfls_estimate_mmv.restype = st
    L.sfls_incomplete_eval.argtypes = [_P, i64, _I64P, _I64P, _I64P, _P, _P, _P, i32, _I64P,
                                       _I64P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                       _P, _I64P, _I64P, _P, _P, _P, _I64P, _I64P, _P, _P, _P, _P]
    L.sfls_incomplete_eval.restype = st
    L.sfls_estimate_incomplete.argtypes = [_P, i64, _I64P, _I64P, _I64P, _P, _P, _P, i32,
                                           ctypes.POINTER(sfls_params), _I64P, _I64P, _P, _P,
                                           _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.sfls_estimate_incomplete.restype = st
    L.sfls_set_factor.argtypes = [_P, i32]
    L.sfls_set_factor.restype = st
    L.sfls_set_nufft.argtypes = [_P, i32]
    L.sfls_set_nufft.restype = st
    L.sfls_set_speculation.argtypes = [_P, i32]
    L.sfls_set_speculation.restype = st
    L.sfls_set_schur_lds.argtypes = [_P, i32]
    L.sfls_set_schur_lds.restype = st
    L.sfls_set_timing.argtypes = [_P, i32]
    L.sfls_set_timing.restype = st
    L.sfls_reset_stats.argtypes = [_P]
    L.sfls_reset_stats.restype = None
    L.sfls_kernel_stats.argtypes = [_P, ctypes.POINTER(sfls_kernel_stat), i32]
    L.sfls_kernel_stats.restype = i32
    L.sfls_last_run.argtypes = [_P, ctypes.POINTER(sfls_run_stats), ctypes.POINTER(ctypes.c_double),
                                i64, _I64P]
    L.sfls_last_run.restype = st
    u64 = ctypes.c_uint64
    _I32P = ctypes.POINTER(ctypes.c_int32)
    L.sfls_server_config_default.argtypes = [ctypes.POINTER(sfls_server_config)]
    L.sfls_server_config_default.restype = None
    L.sfls_server_create.argtypes = [_P, ctypes.POINTER(sfls_server_config),
                                     ctypes.POINTER(sfls_params), ctypes.POINTER(_P)]
    L.sfls_server_create.restype = st
    L.sfls_server_destroy.argtypes = [_P]
    L.sfls_server_destroy.restype = st
    L.sfls_server_footprint.argtypes = [_P, i64, ctypes.POINTER(u64)]
    L.sfls_server_footprint.restype = st
    L.sfls_server_submit.argtypes = [_P, _P, i64, u64]
    L.sfls_server_submit.restype = st
    L.sfls_server_submit_many.argtypes = [_P, ctypes.c_int32, _P, _P, _P,
                                          ctypes.POINTER(ctypes.c_int32)]
    L.sfls_server_submit_many.restype = st
    L.sfls_server_launch.argtypes = [_P]
    L.sfls_server_launch.restype = st
    L.sfls_server_wait.argtypes = [_P, i32, _I32P, _I32P]
    L.sfls_server_wait.restype = st
    L.sfls_server_step.argtypes = [_P, _I32P]
    L.sfls_server_step.restype = st
    L.sfls_server_poll.argtypes = [_P, ctypes.POINTER(sfls_result), i32, _P, _P, _P, i64, _I32P]
    L.sfls_server_poll.restype = st
    L.sfls_server_get_stats.argtypes = [_P, ctypes.POINTER(sfls_server_stats)]
    L.sfls_server_get_stats.restype = st
    _lib = L
    return L


def default_params(**overrides) -> sfls_params:
    p = sfls_params()
    lib().sfls_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


# ------------------------------------------------------------------ helpers --

def _i64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _hp(a: np.ndarray):
    return a.ctypes.data_as(_I64P)


def _dp(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device buffers must be GPU tensors")
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """Owns one sfls_ctx on a HIP device (hbm_budget: workspace cap in bytes, 0 = none)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        import weakref
        self._h = _P()
        self._servers = weakref.WeakSet()  # servers on this context: closed before it
        st = lib().sfls_create(ctypes.byref(self._h), int(device), int(hbm_budget))
        if st != SFLS_OK:
            raise SflsError(st, lib().sfls_strerror(st).decode())
        self.device = device

    @property
    def handle(self):
        return self._h

    def check(self, st: int):
        if st != SFLS_OK:
            msg = lib().sfls_last_error(self._h).decode() or lib().sfls_strerror(st).decode()
            raise SflsError(st, msg)

    def set_factor(self, algo: int):
        self.check(lib().sfls_set_factor(self._h, int(algo)))

    def set_nufft(self, mode: int):
        self.check(lib().sfls_set_nufft(self._h, int(mode)))

    def set_speculation(self, enable: bool = True):
        self.check(lib().sfls_set_speculation(self._h, 1 if enable else 0))

    def set_schur_lds(self, max_f: int):
        self.check(lib().sfls_set_schur_lds(self._h, int(max_f)))

    def set_timing(self, mode=True):
        """True / 1: time every kernel of a round; 2: the recursion only; False / 0: off."""
        self.check(lib().sfls_set_timing(self._h, int(mode)))

    def reset_stats(self):
        lib().sfls_reset_stats(self._h)

    def kernel_stats(self) -> dict:
        arr = (sfls_kernel_stat * 32)()
        n = lib().sfls_kernel_stats(self._h, arr, 32)
        return {arr[i].name.decode(): dict(launches=arr[i].launches, seconds=arr[i].seconds,
                                           flops=arr[i].flops, bytes=arr[i].bytes)
                for i in range(min(n, 32))}

    def last_run(self):
        st = sfls_run_stats()
        nt = ctypes.c_int64(0)
        self.check(lib().sfls_last_run(self._h, ctypes.byref(st), None, 0, ctypes.byref(nt)))
        buf = (ctypes.c_double * max(1, nt.value))()
        self.check(lib().sfls_last_run(self._h, ctypes.byref(st), buf, nt.value,
                                       ctypes.byref(nt)))
        return dict(rounds=st.rounds, evals=st.evals, grid_evals=st.grid_evals,
                    wall_seconds=st.wall_seconds), np.array(buf[:nt.value])

    def close(self):
        if self._h:
            for s in list(self._servers):
                s.close()
            lib().sfls_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------- C-ABI mirrors ------

def sfls_toeplitz_column(ctx: Context, n, off, K, koff, theta, gamma, beta, c, stream=None):
    n, off, K, koff = _i64(n), _i64(off), _i64(K), _i64(koff)
    ctx.check(lib().sfls_toeplitz_column(ctx.handle, len(n), _hp(n), _hp(off), _hp(K), _hp(koff),
                                         _dp(theta), _dp(gamma), _dp(beta), _dp(c),
                                         _stream(stream)))


def sfls_factor(ctx: Context, n, off, c, rho, delta, logdet, status, failed_step, stream=None):
    n, off = _i64(n), _i64(off)
    ctx.check(lib().sfls_factor(ctx.handle, len(n), _hp(n), _hp(off), _dp(c), _dp(rho),
                                _dp(delta), _dp(logdet), _dp(status), _dp(failed_step),
                                _stream(stream)))


def sfls_gs_apply(ctx: Context, n, off, y, ydtype, rho, delta, w, yCy=None, ww=None, stream=None):
    n, off = _i64(n), _i64(off)
    ctx.check(lib().sfls_gs_apply(ctx.handle, len(n), _hp(n), _hp(off), _dp(y), int(ydtype),
                                  _dp(rho), _dp(delta), _dp(w), _dp(yCy), _dp(ww),
                                  _stream(stream)))


def sfls_gs_apply_noalloc(ctx: Context, n, off, y, ydtype, rho, delta, w, yCy=None, ww=None,
                          stream=None):
    n, off = _i64(n), _i64(off)
    ctx.check(lib().sfls_gs_apply_noalloc(ctx.handle, len(n), _hp(n), _hp(off), _dp(y),
                                          int(ydtype), _dp(rho), _dp(delta), _dp(w), _dp(yCy),
                                          _dp(ww), _stream(stream)))


SFLS_NOALLOC_SCRATCH_BYTES = 64 << 20


def sfls_omega(ctx: Context, n, off, oout, rho, delta, omega_s=None, omega_t=None, omega_v=None,
               omega_x=None, stream=None):
    n, off, oout = _i64(n), _i64(off), _i64(oout)
    ctx.check(lib().sfls_omega(ctx.handle, len(n), _hp(n), _hp(off), _hp(oout), _dp(rho),
                               _dp(delta), _dp(omega_s), _dp(omega_t), _dp(omega_v),
                               _dp(omega_x), _stream(stream)))


def sfls_grid_eval(ctx: Context, n, off, y, ydtype, rho, delta, L, goff, gamma_bar, zeta,
                   qG=None, sG=None, dL=None, argmin=None, argmin_val=None,
                   precision=SFLS_FP64, stream=None, rG=None, tG=None, out_mask=None):
    """out_mask None: every output given (not None) is requested."""
    n, off, L, goff = _i64(n), _i64(off), _i64(L), _i64(goff)
    if out_mask is None:
        out_mask = ((SFLS_GRID_Q if qG is not None else 0) | (SFLS_GRID_S if sG is not None else 0)
                    | (SFLS_GRID_R if rG is not None else 0) | (SFLS_GRID_T if tG is not None else 0)
                    | (SFLS_GRID_DL if dL is not None else 0)
                    | (SFLS_GRID_ARGMIN if argmin is not None or argmin_val is not None else 0))
    ctx.check(lib().sfls_grid_eval(ctx.handle, len(n), _hp(n), _hp(off), _dp(y), int(ydtype),
                                   _dp(rho), _dp(delta), _hp(L), _hp(goff), _dp(gamma_bar),
                                   _dp(zeta), int(out_mask), _dp(qG), _dp(sG), _dp(rG), _dp(tG),
                                   _dp(dL), _dp(argmin), _dp(argmin_val), int(precision),
                                   _stream(stream)))


def sfls_active_eval(ctx: Context, n, off, w, rho, delta, K, koff, theta, q=None, r=None, u=None,
                     s=None, t=None, v=None, x=None, stream=None):
    n, off, K, koff = _i64(n), _i64(off), _i64(K), _i64(koff)
    ctx.check(lib().sfls_active_eval(ctx.handle, len(n), _hp(n), _hp(off), _dp(w), _dp(rho),
                                     _dp(delta), _hp(K), _hp(koff), _dp(theta), _dp(q), _dp(r),
                                     _dp(u), _dp(s), _dp(t), _dp(v), _dp(x), _stream(stream)))


def sfls_estimate(ctx: Context, n, off, y, ydtype, params, kcap, koff, K, theta, alpha, gamma,
                  beta, zeta, objective, iters, evals, status, stream=None):
    n, off, kcap, koff = _i64(n), _i64(off), _i64(kcap), _i64(koff)
    pp = ctypes.byref(params) if params is not None else None
    ctx.check(lib().sfls_estimate(ctx.handle, len(n), _hp(n), _hp(off), _dp(y), int(ydtype), pp,
                                  _hp(kcap), _hp(koff), _dp(K), _dp(theta), _dp(alpha),
                                  _dp(gamma), _dp(beta), _dp(zeta), _dp(objective), _dp(iters),
                                  _dp(evals), _dp(status), _stream(stream)))


def sfls_estimate_mmv(ctx: Context, n, off, G, y, ystride, ydtype, params, kcap, koff, K, theta,
                      alpha, alpha_stride, gamma, beta, zeta, objective, iters, evals, status,
                      stream=None):
    n, off, kcap, koff = _i64(n), _i64(off), _i64(kcap), _i64(koff)
    pp = ctypes.byref(params) if params is not None else None
    ctx.check(lib().sfls_estimate_mmv(ctx.handle, len(n), _hp(n), _hp(off), int(G), _dp(y),
                                      int(ystride), int(ydtype), pp, _hp(kcap), _hp(koff), _dp(K),
                                      _dp(theta), _dp(alpha), int(alpha_stride), _dp(gamma),
                                      _dp(beta), _dp(zeta), _dp(objective), _dp(iters),
                                      _dp(evals), _dp(status), _stream(stream)))


def sfls_incomplete_eval(ctx: Context, n, m, moff, idx, phi, y, ydtype, K, koff, theta, gamma,
                         beta, logdet=None, yCy=None, ww=None, q=None, r=None, u=None, s=None,
                         t=None, v=None, x=None, L=None, goff=None, qG=None, sG=None, cand=None,
                         ncand=None, coff=None, cq=None, cs=None, status=None, stream=None):
    n, m, moff, K, koff = _i64(n), _i64(m), _i64(moff), _i64(K), _i64(koff)
    Lh = _i64(L) if L is not None else None
    gh = _i64(goff) if goff is not None else None
    nch = _i64(ncand) if ncand is not None else None
    ch = _i64(coff) if coff is not None else None
    ctx.check(lib().sfls_incomplete_eval(
        ctx.handle, len(n), _hp(n), _hp(m), _hp(moff), _dp(idx), _dp(phi), _dp(y), int(ydtype),
        _hp(K), _hp(koff), _dp(theta), _dp(gamma), _dp(beta), _dp(logdet), _dp(yCy), _dp(ww),
        _dp(q), _dp(r), _dp(u), _dp(s), _dp(t), _dp(v), _dp(x),
        _hp(Lh) if Lh is not None else None, _hp(gh) if gh is not None else None, _dp(qG), _dp(sG),
        _dp(cand), _hp(nch) if nch is not None else None, _hp(ch) if ch is not None else None,
        _dp(cq), _dp(cs), _dp(status), _stream(stream)))


def sfls_estimate_incomplete(ctx: Context, n, m, moff, idx, phi, y, ydtype, params, kcap, koff, K,
                             theta, alpha, gamma, beta, zeta, objective, iters, evals, status,
                             stream=None):
    n, m, moff, kcap, koff = _i64(n), _i64(m), _i64(moff), _i64(kcap), _i64(koff)
    pp = ctypes.byref(params) if params is not None else None
    ctx.check(lib().sfls_estimate_incomplete(
        ctx.handle, len(n), _hp(n), _hp(m), _hp(moff), _dp(idx), _dp(phi), _dp(y), int(ydtype), pp,
        _hp(kcap), _hp(koff), _dp(K), _dp(theta), _dp(alpha), _dp(gamma), _dp(beta), _dp(zeta),
        _dp(objective), _dp(iters), _dp(evals), _dp(status), _stream(stream)))


# ------------------------------------------------- batch conveniences -------

@dataclass
class EstimateResult:
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


def estimate_batch(ctx: Context, ys, params: sfls_params | None = None, kcap: int | None = None,
                   ydtype=None, stream=None, sync: bool = True):
    """Run sfls_estimate on a list of 1-D complex arrays; returns EstimateResult per instance."""
    import torch
    dev = torch.device("cuda", ctx.device)
    if ydtype is None:
        ydtype = SFLS_C64 if all(np.asarray(y).dtype == np.complex64 for y in ys) else SFLS_C128
    npdt = np.complex64 if ydtype == SFLS_C64 else np.complex128
    n = np.array([len(y) for y in ys], np.int64)
    off = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)
    kc = np.array([min(int(k), int(m)) for k, m in zip(
        [kcap if kcap else m for m in n], n)], np.int64)
    koff = np.concatenate([[0], np.cumsum(kc)[:-1]]).astype(np.int64)
    yflat = np.concatenate([np.asarray(y, npdt) for y in ys])
    ydev = torch.from_numpy(yflat.view(np.float32 if ydtype == SFLS_C64 else np.float64)).to(dev)
    B, KT = len(ys), int(kc.sum())
    f64 = dict(dtype=torch.float64, device=dev)
    i32 = dict(dtype=torch.int32, device=dev)
    out = dict(K=torch.zeros(B, dtype=torch.int64, device=dev), theta=torch.zeros(KT, **f64),
               alpha=torch.zeros(2 * KT, **f64), gamma=torch.zeros(KT, **f64),
               beta=torch.zeros(B, **f64), zeta=torch.zeros(B, **f64),
               objective=torch.zeros(B, **f64), iters=torch.zeros(B, **i32),
               evals=torch.zeros(B, **i32), status=torch.zeros(B, **i32))
    sfls_estimate(ctx, n, off, ydev, ydtype, params, kc, koff, out["K"], out["theta"],
                  out["alpha"], out["gamma"], out["beta"], out["zeta"], out["objective"],
                  out["iters"], out["evals"], out["status"], stream=stream)
    if not sync:
        return out
    torch.cuda.synchronize(dev)
    h = {k: v.cpu().numpy() for k, v in out.items()}
    alpha = h["alpha"].view(np.complex128)
    res = []
    for b in range(B):
        k = int(h["K"][b])
        o = int(koff[b])
        res.append(EstimateResult(K=k, theta=h["theta"][o:o + k].copy(),
                                  alpha=alpha[o:o + k].copy(), gamma=h["gamma"][o:o + k].copy(),
                                  beta=float(h["beta"][b]), zeta=float(h["zeta"][b]),
                                  objective=float(h["objective"][b]),
                                  iterations=int(h["iters"][b]), evaluations=int(h["evals"][b]),
                                  status=int(h["status"][b])))
    return res


def pack_incomplete(ctx: Context, obs, ydtype=None):
    """Device arrays of a batch of incomplete observations: obs is a list of
    (N, idx, phi, y) with idx the observed indices, phi their weights (None:
    unit weights for the whole batch only when every phi is None) and y the
    observed samples.  Returns (n, m, moff, idx_dev, phi_dev or None, y_dev,
    ydtype)."""
    import torch
    dev = torch.device("cuda", ctx.device)
    if ydtype is None:
        ydtype = SFLS_C64 if all(np.asarray(o[3]).dtype == np.complex64 for o in obs) else SFLS_C128
    npdt = np.complex64 if ydtype == SFLS_C64 else np.complex128
    n = np.array([int(o[0]) for o in obs], np.int64)
    m = np.array([len(o[1]) for o in obs], np.int64)
    moff = np.concatenate([[0], np.cumsum(m)[:-1]]).astype(np.int64)
    idx = torch.from_numpy(np.concatenate([np.asarray(o[1], np.int32) for o in obs])).to(dev)
    yflat = np.concatenate([np.asarray(o[3], npdt) for o in obs])
    ydev = torch.from_numpy(yflat.view(np.float32 if ydtype == SFLS_C64 else np.float64)).to(dev)
    phid = None
    if any(o[2] is not None for o in obs):
        ph = np.concatenate([np.ones(len(o[1]), np.complex128) if o[2] is None
                             else np.asarray(o[2], np.complex128) for o in obs])
        phid = torch.from_numpy(ph.view(np.float64)).to(dev)
    return n, m, moff, idx, phid, ydev, ydtype


def estimate_batch_incomplete(ctx: Context, obs, params: sfls_params | None = None,
                              kcap: int | None = None, ydtype=None, stream=None):
    """sfls_estimate_incomplete on a list of (N, idx, phi, y); returns
    EstimateResult per instance."""
    import torch
    dev = torch.device("cuda", ctx.device)
    n, m, moff, idx, phid, ydev, ydtype = pack_incomplete(ctx, obs, ydtype)
    kc = np.array([min(int(kcap) if kcap else int(mm), int(mm), SFLS_SF_MAX_K) for mm in m],
                  np.int64)
    koff = np.concatenate([[0], np.cumsum(kc)[:-1]]).astype(np.int64)
    B, KT = len(obs), int(kc.sum())
    f64 = dict(dtype=torch.float64, device=dev)
    i32 = dict(dtype=torch.int32, device=dev)
    out = dict(K=torch.zeros(B, dtype=torch.int64, device=dev), theta=torch.zeros(KT, **f64),
               alpha=torch.zeros(2 * KT, **f64), gamma=torch.zeros(KT, **f64),
               beta=torch.zeros(B, **f64), zeta=torch.zeros(B, **f64),
               objective=torch.zeros(B, **f64), iters=torch.zeros(B, **i32),
               evals=torch.zeros(B, **i32), status=torch.zeros(B, **i32))
    sfls_estimate_incomplete(ctx, n, m, moff, idx, phid, ydev, ydtype, params, kc, koff, out["K"],
                             out["theta"], out["alpha"], out["gamma"], out["beta"], out["zeta"],
                             out["objective"], out["iters"], out["evals"], out["status"],
                             stream=stream)
    torch.cuda.synchronize(dev)
    h = {k: v.cpu().numpy() for k, v in out.items()}
    alpha = h["alpha"].view(np.complex128)
    res = []
    for b in range(B):
        k = int(h["K"][b])
        o = int(koff[b])
        res.append(EstimateResult(K=k, theta=h["theta"][o:o + k].copy(),
                                  alpha=alpha[o:o + k].copy(), gamma=h["gamma"][o:o + k].copy(),
                                  beta=float(h["beta"][b]), zeta=float(h["zeta"][b]),
                                  objective=float(h["objective"][b]),
                                  iterations=int(h["iters"][b]), evaluations=int(h["evals"][b]),
                                  status=int(h["status"][b])))
    return res


def estimate_batch_mmv(ctx: Context, Ys, params: sfls_params | None = None,
                       kcap: int | None = None, ydtype=None, stream=None):
    """sfls_estimate_mmv on a list of G x n complex arrays (one G for all);
    returns EstimateResult per instance with alpha of shape G x K."""
    import torch
    dev = torch.device("cuda", ctx.device)
    Ys = [np.atleast_2d(np.asarray(Y)) for Y in Ys]
    G = Ys[0].shape[0]
    assert all(Y.shape[0] == G for Y in Ys), "one G per call"
    if ydtype is None:
        ydtype = SFLS_C64 if all(Y.dtype == np.complex64 for Y in Ys) else SFLS_C128
    npdt = np.complex64 if ydtype == SFLS_C64 else np.complex128
    n = np.array([Y.shape[1] for Y in Ys], np.int64)
    off = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)
    ystride = int(n.sum())
    kc = np.array([min(int(kcap) if kcap else int(m), int(m)) for m in n], np.int64)
    koff = np.concatenate([[0], np.cumsum(kc)[:-1]]).astype(np.int64)
    KT = int(kc.sum())
    yflat = np.concatenate([Y.astype(npdt) for Y in Ys], axis=1)       # G x sum n
    ydev = torch.from_numpy(np.ascontiguousarray(yflat).view(
        np.float32 if ydtype == SFLS_C64 else np.float64).ravel().copy()).to(dev)
    B = len(Ys)
    f64 = dict(dtype=torch.float64, device=dev)
    i32 = dict(dtype=torch.int32, device=dev)
    out = dict(K=torch.zeros(B, dtype=torch.int64, device=dev), theta=torch.zeros(KT, **f64),
               alpha=torch.zeros(2 * G * KT, **f64), gamma=torch.zeros(KT, **f64),
               beta=torch.zeros(B, **f64), zeta=torch.zeros(B, **f64),
               objective=torch.zeros(B, **f64), iters=torch.zeros(B, **i32),
               evals=torch.zeros(B, **i32), status=torch.zeros(B, **i32))
    sfls_estimate_mmv(ctx, n, off, G, ydev, ystride, ydtype, params, kc, koff, out["K"],
                      out["theta"], out["alpha"], KT, out["gamma"], out["beta"], out["zeta"],
                      out["objective"], out["iters"], out["evals"], out["status"], stream=stream)
    torch.cuda.synchronize(dev)
    h = {k: v.cpu().numpy() for k, v in out.items()}
    alpha = h["alpha"].view(np.complex128).reshape(G, KT)
    res = []
    for b in range(B):
        k, o = int(h["K"][b]), int(koff[b])
        res.append(EstimateResult(K=k, theta=h["theta"][o:o + k].copy(),
                                  alpha=alpha[:, o:o + k].copy(), gamma=h["gamma"][o:o + k].copy(),
                                  beta=float(h["beta"][b]), zeta=float(h["zeta"][b]),
                                  objective=float(h["objective"][b]),
                                  iterations=int(h["iters"][b]), evaluations=int(h["evals"][b]),
                                  status=int(h["status"][b])))
    return res


# ------------------------------------------------------------- serving ------

@dataclass
class ServedResult:
    tag: int
    n: int
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
    t_submit: float
    t_done: float


class Server:
    """Continuous-batching estimation server (sfls_server_* of the C ABI).

    Requests are admitted with submit() (False when the server has no free slot
    or pool memory for it now), rounds run with step() or launch()/wait(), and
    finished results are collected with poll()."""

    def __init__(self, ctx: Context, max_n: int = SFLS_MAX_N, max_slots: int = 1024,
                 ydtype: int = SFLS_C64, hbm_bytes: int = 8 << 30, kcap_shift: int = 0,
                 params: sfls_params | None = None, stream=None):
        cfg = sfls_server_config()
        lib().sfls_server_config_default(ctypes.byref(cfg))
        cfg.max_n, cfg.max_slots, cfg.ydtype = int(max_n), int(max_slots), int(ydtype)
        cfg.hbm_bytes, cfg.kcap_shift = int(hbm_bytes), int(kcap_shift)
        cfg.stream = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        self.ctx = ctx
        self.ydtype = int(ydtype)
        self._h = _P()
        pp = ctypes.byref(params) if params is not None else None
        ctx.check(lib().sfls_server_create(ctx.handle, ctypes.byref(cfg), pp,
                                           ctypes.byref(self._h)))
        ctx._servers.add(self)
        self._res = (sfls_result * 4096)()
        self._cap = 1 << 16
        self._th = np.zeros(self._cap)
        self._ga = np.zeros(self._cap)
        self._al = np.zeros(2 * self._cap)
        self.in_flight = False

    def footprint(self, n: int) -> int:
        b = ctypes.c_uint64(0)
        self.ctx.check(lib().sfls_server_footprint(self._h, int(n), ctypes.byref(b)))
        return int(b.value)

    def submit(self, y, n: int, tag: int) -> bool:
        """y: GPU tensor (interleaved re/im of the server's dtype), or an
        address: device memory is read by the next round (keep it unchanged
        until the next wait()/step() returns), host memory is copied now."""
        ptr = ctypes.c_void_p(y if isinstance(y, int) else y.data_ptr())
        st = lib().sfls_server_submit(self._h, ptr, int(n), int(tag))
        if st == SFLS_EAGAIN:
            return False
        self.ctx.check(st)
        return True

    def submit_many(self, ptrs, ns, tags) -> int:
        """Admit requests in order (device or host addresses `ptrs`, lengths
        `ns`, tags `tags`) until one is not admitted; returns how many were."""
        ptrs = np.ascontiguousarray(ptrs, dtype=np.uint64)
        ns = np.ascontiguousarray(ns, dtype=np.int64)
        tags = np.ascontiguousarray(tags, dtype=np.uint64)
        if not (len(ptrs) == len(ns) == len(tags)):
            raise ValueError("ptrs, ns and tags differ in length")
        acc = ctypes.c_int32(0)
        self.ctx.check(lib().sfls_server_submit_many(
            self._h, len(ptrs), ptrs.ctypes.data_as(ctypes.c_void_p),
            ns.ctypes.data_as(ctypes.c_void_p), tags.ctypes.data_as(ctypes.c_void_p),
            ctypes.byref(acc)))
        return int(acc.value)

    def launch(self):
        self.ctx.check(lib().sfls_server_launch(self._h))
        self.in_flight = self.stats()["in_flight"] > 0

    def wait(self, block: bool = True):
        ready, fin = ctypes.c_int32(0), ctypes.c_int32(0)
        self.ctx.check(lib().sfls_server_wait(self._h, 1 if block else 0, ctypes.byref(ready),
                                              ctypes.byref(fin)))
        if ready.value:
            self.in_flight = False
        return bool(ready.value), int(fin.value)

    def step(self) -> int:
        fin = ctypes.c_int32(0)
        self.ctx.check(lib().sfls_server_step(self._h, ctypes.byref(fin)))
        return int(fin.value)

    def poll(self, max_results: int = 4096):
        out = []
        while True:
            nres = ctypes.c_int32(0)
            th = self._th.ctypes.data_as(ctypes.c_void_p)
            ga = self._ga.ctypes.data_as(ctypes.c_void_p)
            al = self._al.ctypes.data_as(ctypes.c_void_p)
            st = lib().sfls_server_poll(self._h, self._res, min(max_results - len(out), 4096),
                                        th, ga, al, self._cap, ctypes.byref(nres))
            self.ctx.check(st)
            alc = self._al.view(np.complex128)
            for i in range(nres.value):
                r = self._res[i]
                o, k = int(r.comp_off), int(r.K)
                out.append(ServedResult(tag=int(r.tag), n=int(r.n), K=k,
                                        theta=self._th[o:o + k].copy(),
                                        alpha=alc[o:o + k].copy(),
                                        gamma=self._ga[o:o + k].copy(), beta=r.beta, zeta=r.zeta,
                                        objective=r.objective, iterations=int(r.iters),
                                        evaluations=int(r.evals), status=int(r.status),
                                        t_submit=r.t_submit, t_done=r.t_done))
            if nres.value == 0 or len(out) >= max_results:
                return out

    def stats(self) -> dict:
        s = sfls_server_stats()
        self.ctx.check(lib().sfls_server_get_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in sfls_server_stats._fields_}

    def close(self):
        if self._h:
            lib().sfls_server_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
