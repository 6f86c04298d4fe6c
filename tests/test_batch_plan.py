"""Host-side batch planner (no GPU).  Persistent schedule: every task list it
builds passes its own deadlock-freedom check (each wait is met by tasks
listed earlier) and slab counts follow the option.  Size-bucketed schedule:
pass and stream counts follow the options.  Invalid datasets and options
are rejected."""
import ctypes

import numpy as np
import pytest

import paper_2305_04318_amd as pl
from paper_2305_04318_amd import _lib


def _plan(ns, Ks, p=2, M=2, slabs=0, persistent=True, lanes=0, precision=0):
    lib = pl.load()
    D = len(ns)
    oms = [np.tile([[1.0, 1.5, 0.1, 1.0, 0.0]], (K, 1)) for K in Ks]
    arr = (_lib.PlDataset * D)()
    for i, (n, om) in enumerate(zip(ns, oms)):
        arr[i] = _lib.PlDataset(0x1000, 0x2000, 0x3000, n, om.ctypes.data, om.shape[0])
    lam = np.linspace(0.0, 1.0, max(M, 1))
    o = _lib.PlOpts()
    o.chunk = slabs
    o.lanes = lanes
    o.precision = precision
    if persistent:
        o.flags = _lib.PL_OPT_BATCH_PERSISTENT
    h = ctypes.c_void_p()
    rc = lib.pl_batch_create(arr, D, p, lam.ctypes.data_as(ctypes.c_void_p), M, ctypes.byref(o),
                             ctypes.byref(h))
    return rc, h, oms


def _stats(h):
    u, t, s = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    assert pl.load().pl_batch_stats(h, ctypes.byref(u), ctypes.byref(t), ctypes.byref(s)) == 0
    return u.value, t.value, s.value


def _tasks_per_unit(n):
    Nv = (n + 127) // 128
    ph0 = 1 + Nv * (Nv + 1) // 2
    gemm = sum(Nv - J + 1 for J in range(1, Nv + 1))
    return ph0 + gemm + Nv + sum(Nv - J for J in range(Nv)) + 1


@pytest.mark.parametrize("slabs", [0, 1, 3, 1000])
def test_plan_counts_and_validation(slabs):
    rng = np.random.default_rng(0)
    ns = list(rng.integers(10, 1500, 40))
    Ks = list(rng.integers(1, 6, 40))
    rc, h, _ = _plan(ns, Ks, slabs=slabs)
    assert rc == 0
    try:
        units, tasks, nslab = _stats(h)
        assert units == sum(Ks)
        assert tasks == sum(K * _tasks_per_unit(n) for n, K in zip(ns, Ks))
        assert nslab == (min(units, slabs) if slabs > 0 else min(units, 2048))
        sz = ctypes.c_size_t()
        assert pl.load().pl_batch_workspace_size(h, ctypes.byref(sz)) == 0 and sz.value > 0
    finally:
        pl.load().pl_batch_destroy(h)


def test_plan_rejects_bad_datasets():
    rc, h, _ = _plan([100, 2], [2, 2])          # n = 2 with p = 2: n <= p
    assert rc == -1
    rc, h, _ = _plan([100], [1], p=0)
    assert rc == -3
    rc, h, _ = _plan([100], [1], M=0)
    assert rc == -5


def test_plan_tile_index_bound():
    # the task list holds tile indices as int16: a dataset with more than 32767
    # tile rows is rejected before any task is built
    rc, h, _ = _plan([32767 * 128 + 1], [1])
    assert rc == -1
    rc, h, _ = _plan([100], [1], slabs=0)
    assert rc == 0
    pl.load().pl_batch_destroy(h)


def test_plan_rejects_negative_wait_limit():
    lib = pl.load()
    om = np.array([[1.0, 1.5, 0.1, 1.0, 0.0]])
    arr = (_lib.PlDataset * 1)()
    arr[0] = _lib.PlDataset(0x1000, 0x2000, 0x3000, 100, om.ctypes.data, 1)
    lam = np.array([0.0])
    o = _lib.PlOpts()
    o.wait_us = -1
    h = ctypes.c_void_p()
    assert lib.pl_batch_create(arr, 1, 2, lam.ctypes.data_as(ctypes.c_void_p), 1, ctypes.byref(o),
                               ctypes.byref(h)) == -6


@pytest.mark.parametrize("chunk,lanes,precision", [(0, 0, 0), (3, 2, 0), (7, 5, 1), (1, 1, 1)])
def test_bucketed_plan_passes_and_streams(chunk, lanes, precision):
    """Units are grouped by tile-row count and cut into passes of at most
    `chunk` units (as evenly as possible); the workspace holds one region per
    stream."""
    rng = np.random.default_rng(1)
    ns = list(rng.integers(10, 1500, 40))
    Ks = list(rng.integers(1, 6, 40))
    rc, h, _ = _plan(ns, Ks, slabs=chunk, persistent=False, lanes=lanes, precision=precision)
    assert rc == 0
    try:
        units, passes, streams = _stats(h)
        assert units == sum(Ks)
        assert streams == (lanes or 4)
        groups = {}
        for n, K in zip(ns, Ks):
            groups[(n + 127) // 128] = groups.get((n + 127) // 128, 0) + K
        if chunk:
            assert passes == sum(-(-c // chunk) for c in groups.values())
        else:  # the default 4 GiB pass holds every group of these sizes
            assert passes == len(groups)
        sz = ctypes.c_size_t()
        assert pl.load().pl_batch_workspace_size(h, ctypes.byref(sz)) == 0 and sz.value > 0
    finally:
        pl.load().pl_batch_destroy(h)


def test_bucketed_plan_option_checks():
    # the persistent kernel carries FP64 tasks only; the mixed form takes M + p <= 64
    rc, h, _ = _plan([300], [2], persistent=True, precision=1)
    assert rc == -6
    rc, h, _ = _plan([300], [2], p=4, M=61, persistent=False, precision=1)
    assert rc == 3
    rc, h, _ = _plan([300], [2], persistent=False, lanes=17)
    assert rc == -6
