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
                                 lm.ctypes.data_as(ctypes.c_void_p), M, vp(out), None, None,
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
    assert _call(opts=o) == -13
    o = _lib.PlOpts()
    o.precision = 1
    o.flush = 3
    assert _call(opts=o) == -13
    assert _call(work=0) == -14
    assert _call(wb=16) == -15


def test_matern_and_chol_argument_errors():
    lib = pl.load()
    om = np.array([[1.0, 1.0, 0.1, 1.0, 0.0]])
    P = ctypes.c_void_p
    O = om.ctypes.data_as(P)
    F64, F32 = _lib.PL_F64, _lib.PL_F32
    assert lib.pl_matern_cov(None, 10, O, 1, F64, P(1), 10, P(1), 1 << 30, None) == -1
    assert lib.pl_matern_cov(P(1), 0, O, 1, F64, P(1), 10, P(1), 1 << 30, None) == -2
    assert lib.pl_matern_cov(P(1), 10, O, 1, 2, P(1), 10, P(1), 1 << 30, None) == -5
    assert lib.pl_matern_cov(P(1), 10, O, 1, F32, None, 10, P(1), 1 << 30, None) == -6
    assert lib.pl_matern_cov(P(1), 10, O, 1, F32, P(1), 5, P(1), 1 << 30, None) == -7
    assert lib.pl_matern_cov(P(1), 10, O, 1, F64, P(1), 10, P(1), 8, None) == -9
    FP64, MIX = _lib.PL_FP64, _lib.PL_MIXED
    assert lib.pl_chol_batched(None, 10, 1, 10, FP64, P(1), P(1), P(1), 1 << 30, None) == -1
    assert lib.pl_chol_batched(P(8), 10, 1, 12, MIX, P(1), P(1), P(1), 1 << 30, None) == -1
    assert lib.pl_chol_batched(P(1), 10, 1, 9, FP64, P(1), P(1), P(1), 1 << 30, None) == -4
    assert lib.pl_chol_batched(P(16), 10, 1, 10, MIX, P(1), P(1), P(1), 1 << 30, None) == -4
    assert lib.pl_chol_batched(P(16), 10, 1, 12, 5, P(1), P(1), P(1), 1 << 30, None) == -5
    assert lib.pl_chol_batched(P(1), 10, 1, 10, FP64, P(1), None, P(1), 1 << 30, None) == -7
    assert lib.pl_chol_batched(P(1), 10, 1, 10, FP64, P(1), P(1), P(1), 8, None) == -9
    w64, wmx = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.pl_chol_workspace_size(3, FP64, ctypes.byref(w64)) == 0
    assert lib.pl_chol_workspace_size(3, MIX, ctypes.byref(wmx)) == 0
    assert w64.value >= 3 * 128 * 128 * 8 and wmx.value >= 3 * 128 * 128 * 12
    assert lib.pl_chol_workspace_size(3, 9, ctypes.byref(wmx)) == -2


def test_opts_struct_layout():
    # precision, refine, chunk, flags, flush, wait_us, reserved: 32 bytes
    assert ctypes.sizeof(_lib.PlOpts) == 32
    assert _lib.PlOpts.chunk.offset == 8 and _lib.PlOpts.flush.offset == 20
    assert _lib.PlOpts.wait_us.offset == 24


def test_autotune_argument_errors_and_workspace():
    lib = pl.load()
    P = ctypes.c_void_p
    om = np.array([[1.0, 1.0, 0.1, 1.0, 0.0]] * 100)
    lm = np.zeros(4)
    o = _lib.PlOpts()

    def call(locs=1, tol=1e-3, opts=True, work=1, wb=1 << 40, n=500, sample=0):
        return lib.pl_autotune(P(locs) if locs else None, P(1), P(1), n, 3,
                               om.ctypes.data_as(P), 100, lm.ctypes.data_as(P), 4, sample, tol,
                               ctypes.byref(o) if opts else None, None,
                               P(work) if work else None, wb, None)
    assert call(locs=0) == -1
    assert call(n=1) == -4
    assert call(sample=-1) == -10
    assert call(tol=-1.0) == -11 and call(tol=float("nan")) == -11
    assert call(opts=False) == -12
    assert call(work=0) == -14
    assert call(wb=1024) == -15
    b = ctypes.c_size_t(0)
    assert lib.pl_autotune_workspace_size(500, 3, 100, 4, 0, ctypes.byref(b)) == 0
    # holds the 64-point sample in the larger (mixed) layout plus two record sets
    o2 = _lib.PlOpts()
    o2.precision = 1
    rc, mixed64 = _ws(500, 3, 64, 4, o2)
    assert rc == 0 and b.value >= mixed64 + 2 * 64 * 4 * 80
    assert lib.pl_autotune_workspace_size(500, 3, 0, 4, 0, ctypes.byref(b)) == -3
    assert lib.pl_autotune_workspace_size(500, 3, 100, 4, -2, ctypes.byref(b)) == -5
    b100 = ctypes.c_size_t(0)
    assert lib.pl_autotune_workspace_size(500, 3, 100, 4, 100, ctypes.byref(b100)) == 0
    assert b100.value > b.value


def test_curves_argument_errors():
    lib = pl.load()
    P = ctypes.c_void_p
    lm = np.zeros(3)
    sg = np.array([0.5, 1.0])
    bg = np.zeros((2, 4))

    def call(rec=1, beta=1, xvi=1, n=100, p=2, K=5, M=3, sgrid=sg, Gs=2, bgrid=bg, Gb=4,
             ps=1, pb=1, work=1, wb=1 << 30):
        vp = lambda v: P(v) if v else None
        arr = lambda a: a.ctypes.data_as(P) if a is not None else None
        return lib.pl_profile_curves(vp(rec), vp(beta), vp(xvi), n, p, K, lm.ctypes.data_as(P), M,
                                     arr(sgrid), Gs, arr(bgrid), Gb, vp(ps), None, vp(pb), None,
                                     vp(work), wb, None)
    assert call(rec=0) == -1
    assert call(beta=0) == -2 and call(xvi=0) == -3
    assert call(beta=0, xvi=0, Gb=0) != -2
    assert call(n=1) == -4
    assert call(p=0) == -5
    assert call(K=0) == -6
    assert call(M=0) == -8
    assert call(sgrid=np.array([0.5, -1.0])) == -9
    assert call(sgrid=None) == -10
    assert call(bgrid=np.array([[0.0, np.nan, 0, 0], [0, 0, 0, 0]])) == -11
    assert call(bgrid=None) == -12
    assert call(ps=0) == -13 and call(pb=0) == -15
    assert call(work=0) == -17 and call(wb=8) == -18
    b = ctypes.c_size_t(0)
    assert lib.pl_curves_workspace_size(2, 3, 2, 4, ctypes.byref(b)) == 0 and b.value >= 8 * 13


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(_lib.PlError):
        _lib.load(str(tmp_path / "nope.so"))


def test_noalloc_rejects_problems_beyond_its_scratch():
    """pl_profile_loglik_noalloc refuses, before any device work, a problem
    one omega of which needs more than its fixed array; sizes are checked as
    in pl_profile_loglik."""
    lib = pl.load()
    om = np.array([[1.0, 1.0, 0.1, 1.0, 0.0]])
    lm = np.zeros(4)
    one = ctypes.c_void_p(1)

    def call(n, p=2, K=1, M=4, precision=_lib.PL_FP64):
        o = _lib.PlOpts()
        o.precision = precision
        return lib.pl_profile_loglik_noalloc(one, one, one, n, p,
                                             om.ctypes.data_as(ctypes.c_void_p), K,
                                             lm.ctypes.data_as(ctypes.c_void_p), M, one, None,
                                             None, ctypes.byref(o), None)

    assert call(9000) == 4 and lib.pl_error_string(4).startswith(b"one omega")
    assert call(7000, precision=_lib.PL_MIXED) == 4
    assert call(1) == -4 and call(100, p=0) == -5 and call(100, K=0) == -7
    assert call(100, M=0) == -9 and call(100, precision=7) == -13
    assert call(100, p=30, M=35, precision=_lib.PL_MIXED) == 3
    o = _lib.PlOpts()
    o.precision = _lib.PL_MIXED
    assert _ws(100, 30, 1, 34, o)[0] == 0 and _ws(100, 30, 1, 35, o)[0] == 3  # M + p <= 64
