"""The C-ABI library loads, exports every symbol include/plprof.h declares,
and rejects invalid arguments before touching the GPU (CPU-only tests)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2305_04318_amd as pl
from paper_2305_04318_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "plprof.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pl_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = pl.load()
    names = _declared()
    assert set(names) == set(_lib.EXPORTS), names
    for name in names:
        assert hasattr(lib, name), name
    assert lib.pl_version().startswith(b"plprof")


def test_result_struct_is_80_bytes():
    assert ctypes.sizeof(_lib.PlResult) == 80
    assert _lib.PlResult.info.offset == 72


def _ws(n, p, K, M, opts=None):
    out = ctypes.c_size_t(0)
    rc = pl.load().pl_workspace_size(n, p, K, M, ctypes.byref(opts) if opts else None,
                                     ctypes.byref(out))
    return rc, out.value


def test_workspace_size_validation():
    assert _ws(1, 1, 1, 1)[0] == -1
    assert _ws(10, 0, 1, 1)[0] == -2
    assert _ws(10, 10, 1, 1)[0] == -2
    assert _ws(100, 33, 1, 1)[0] == -2
    assert _ws(100, 2, 0, 1)[0] == -3
    assert _ws(100, 2, 1, 0)[0] == -4
    assert _ws(100, 2, 1, 65)[0] == -4
    rc1, b1 = _ws(2000, 4, 1, 8)
    rc2, b2 = _ws(2000, 4, 1024, 8)
    assert rc1 == 0 and rc2 == 0 and b2 > 500 * b1 / 2
    o = _lib.PlOpts()
    o.chunk = 16
    rc3, b3 = _ws(2000, 4, 1024, 8, o)
    assert rc3 == 0 and b3 < b2 / 10


def _call(locs=1, y=1, X=1, n=100, p=2, omega=None, K=1, lam=None, M=1, out=1, opts=None,
          work=1, wb=1 << 40):
    lib = pl.load()
    om = np.array([[1.0, 1.0, 0.1, 1.0, 0.0]] * max(K, 1)) if omega is None else omega
    lm = np.zeros(max(M, 1)) if lam is None else lam
    vp = lambda v: ctypes.c_void_p(v) if v else None
    return lib.pl_profile_loglik(vp(locs), vp(y), vp(X), n, p,
                                 om.ctypes.data_as(ctypes.c_void_p), K,
                                 lm.ctypes.data_as(ctypes.c_void_p), M, vp(out), None,
                                 ctypes.byref(opts) if opts else None, vp(work), wb, None)


def test_profile_argument_errors():
    assert _call(locs=0) == -1
    assert _call(y=0) == -2
    assert _call(X=0) == -3
    assert _call(n=1) == -4
    assert _call(p=0) == -5 and _call(p=100) == -5
    assert _call(omega=np.array([[-1.0, 1.0, 0.1, 1.0, 0.0]])) == -6
    assert _call(omega=np.array([[1.0, 0.01, 0.1, 1.0, 0.0]])) == -6
    assert _call(omega=np.array([[1.0, 1.0, -0.1, 1.0, 0.0]])) == -6
    assert _call(omega=np.array([[1.0, 1.0, 0.1, 0.0, 0.0]])) == -6
    assert _call(omega=np.array([[1.0, 1.0, np.nan, 1.0, 0.0]])) == -6
    assert _call(K=0) == -7
    assert _call(lam=np.array([np.inf])) == -8
    assert _call(M=0) == -9
    assert _call(out=0) == -10
    o = _lib.PlOpts()
    o.precision = 7
    assert _call(opts=o) == -12
    assert _call(work=0) == -13
    assert _call(wb=16) == -14


def test_matern_and_chol_argument_errors():
    lib = pl.load()
    om = np.array([[1.0, 1.0, 0.1, 1.0, 0.0]])
    P = ctypes.c_void_p
    assert lib.pl_matern_cov(None, 10, om.ctypes.data_as(P), 1, P(1), 10, P(1), 1 << 30, None) == -1
    assert lib.pl_matern_cov(P(1), 0, om.ctypes.data_as(P), 1, P(1), 10, P(1), 1 << 30, None) == -2
    assert lib.pl_matern_cov(P(1), 10, om.ctypes.data_as(P), 1, P(1), 5, P(1), 1 << 30, None) == -6
    assert lib.pl_matern_cov(P(1), 10, om.ctypes.data_as(P), 1, P(1), 10, P(1), 8, None) == -8
    assert lib.pl_chol_batched(None, 10, 1, 10, P(1), P(1), P(1), 1 << 30, None) == -1
    assert lib.pl_chol_batched(P(1), 10, 1, 9, P(1), P(1), P(1), 1 << 30, None) == -4
    assert lib.pl_chol_batched(P(1), 10, 1, 10, P(1), None, P(1), 1 << 30, None) == -6
    assert lib.pl_chol_batched(P(1), 10, 1, 10, P(1), P(1), P(1), 8, None) == -8


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(_lib.PlError):
        _lib.load(str(tmp_path / "nope.so"))
