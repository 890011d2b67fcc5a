"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/sfls.h, and its defaults agree with the oracle's readings."""
import ctypes
import os
import re

import pytest

import paper_1705_06073_amd as sf
from oracle.estimator import Params

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "sfls.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sfls_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sfls_factor", "sfls_grid_eval", "sfls_estimate", "sfls_create",
                     "sfls_destroy"):
        assert required in names
    assert set(names) == set(sf.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = sf.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_defaults_match_the_oracle_readings():
    p = sf.default_params()
    o = Params()
    assert p.L_mult == o.L_mult and p.tau == o.tau and p.lbfgs_J == o.lbfgs_J
    assert p.max_inner == o.max_inner and p.max_outer == o.max_outer
    assert p.tol_obj == o.tol_obj and p.tol_newton == o.tol_newton
    assert p.eps_beta_rel == o.eps_beta_rel and p.eps_L == o.eps_L
    assert p.approx_max_iters == o.approx_max_iters and bool(p.approx_use_tau) == o.approx_use_tau
    assert p.approx_ratio == o.approx_ratio and p.approx_min_dist == o.approx_min_dist
    assert p.ls_c1 == o.ls_c1 and p.ls_max == o.ls_max and p.curv_eps == o.curv_eps
    assert p.polish_max_iters == o.polish_max_iters and p.polish_tol == o.polish_tol
    assert p.polish_ftol == o.polish_ftol
    assert ctypes.sizeof(sf.sfls_params) == 136  # static_assert in abi.hip


def test_strerror_and_version():
    L = sf.lib()
    assert L.sfls_strerror(0) == b"ok"
    assert b"positive definite" in L.sfls_strerror(sf.SFLS_ENOTPD)
    assert b"gfx950" in L.sfls_version()


def test_null_context_is_rejected_without_touching_the_device():
    L = sf.lib()
    n = (ctypes.c_int64 * 1)(8)
    o = (ctypes.c_int64 * 1)(0)
    assert L.sfls_factor(None, 1, n, o, None, None, None, None, None, None, None) == sf.SFLS_EINVAL
    assert L.sfls_estimate(None, 1, n, o, None, 1, None, n, o, *([None] * 11)) == sf.SFLS_EINVAL
    assert L.sfls_destroy(None) == sf.SFLS_OK
    assert L.sfls_set_speculation(None, 1) == sf.SFLS_EINVAL


def test_server_structs_match_the_header_layout():
    # the library static_asserts the same sizes on its side
    assert ctypes.sizeof(sf.sfls_server_config) == 40
    assert ctypes.sizeof(sf.sfls_result) == 88
    assert ctypes.sizeof(sf.sfls_server_stats) == 72
    assert ctypes.sizeof(sf.sfls_params) == 136
