"""Uneven batches of datasets evaluated by one graph launch (pl_batch_* of the
C ABI): the size-bucketed schedule (FP64 or mixed) or the persistent kernel
(FP64)."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import PlDataset, check, load
from .api import Inputs, TuneReport, _host_f64, _opts, _stream_ptr, unpack_records


class Batch:
    """A plan over many datasets; run() evaluates every (dataset, omega, lambda)
    record with one graph launch.  schedule "bucketed" (default): units grouped
    by tile count run the step kernels in passes of at most `chunk` units
    (0: as many as fit 4 GiB) spread over `lanes` streams; "persistent": one
    persistent kernel over a pool of `max_slabs` matrix slabs (FP64 only)."""

    def __init__(self, problems, lam, device="cuda", max_slabs=0, inputs=None, wait_us=0,
                 precision="fp64", schedule="bucketed", lanes=0, chunk=0, flush=0, refine=1,
                 fallback=True):
        lib = load()
        self.device = device
        self.inputs = inputs if inputs is not None else [
            Inputs(pr.locs, pr.y, pr.X, device) for pr in problems]
        self.omegas = [_host_f64(pr.omega, 5) for pr in problems]
        self.lam = _host_f64(lam).reshape(-1)
        ps = {inp.p for inp in self.inputs}
        if len(ps) != 1:
            raise ValueError("all datasets must have the same number of covariates")
        self.p = ps.pop()
        D = len(self.inputs)
        arr = (PlDataset * D)()
        for i, (inp, om) in enumerate(zip(self.inputs, self.omegas)):
            arr[i] = PlDataset(inp.locs.data_ptr(), inp.y.data_ptr(), inp.Xc.data_ptr(), inp.n,
                               om.ctypes.data, om.shape[0])
        self._arr = arr
        if schedule not in ("bucketed", "persistent"):
            raise ValueError(f"unknown schedule {schedule!r}")
        self.schedule, self.precision = schedule, precision
        persistent = schedule == "persistent"
        o = _opts(precision, max_slabs if persistent else chunk, refine, fallback, flush)
        o.wait_us = int(wait_us)  # limit of one task wait (0: the library's default)
        o.lanes = int(lanes)
        if persistent:
            o.flags |= _lib.PL_OPT_BATCH_PERSISTENT
        h = ctypes.c_void_p()
        check(lib.pl_batch_create(arr, D, self.p, self.lam.ctypes.data_as(ctypes.c_void_p),
                                  self.lam.shape[0], ctypes.byref(o), ctypes.byref(h)),
              "pl_batch_create")
        self._h = h
        sz = ctypes.c_size_t(0)
        check(lib.pl_batch_workspace_size(h, ctypes.byref(sz)), "pl_batch_workspace_size")
        self.work = torch.empty(sz.value, dtype=torch.uint8, device=device)
        u, t, s = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(lib.pl_batch_stats(h, ctypes.byref(u), ctypes.byref(t), ctypes.byref(s)),
              "pl_batch_stats")
        self.units, self.tasks, self.slabs = u.value, t.value, s.value
        # size-bucketed: device passes and streams
        self.passes, self.lanes = (0, 0) if persistent else (t.value, s.value)
        M = self.lam.shape[0]
        self.offsets = np.concatenate([[0], np.cumsum([om.shape[0] for om in self.omegas])])
        self.out = torch.empty((self.units, M, 10), dtype=torch.float64, device=device)
        self.beta = torch.empty((self.units, M, self.p), dtype=torch.float64, device=device)

    def run(self, stream=None):
        rc = load().pl_batch_run(self._h, ctypes.c_void_p(self.out.data_ptr()),
                                 ctypes.c_void_p(self.beta.data_ptr()),
                                 ctypes.c_void_p(self.work.data_ptr()), self.work.numel(),
                                 _stream_ptr(stream))
        check(rc, "pl_batch_run")
        return self

    def error(self) -> int:
        e = ctypes.c_int32(0)
        check(load().pl_batch_error(self._h, ctypes.c_void_p(self.work.data_ptr()), ctypes.byref(e)),
              "pl_batch_error")
        return e.value

    def records(self, i=None):
        """Records of dataset i (dict of (K_i, M) tensors) or of all units."""
        rec = self.out if i is None else self.out[self.offsets[i]:self.offsets[i + 1]]
        out = unpack_records(rec)
        out["beta"] = self.beta if i is None else self.beta[self.offsets[i]:self.offsets[i + 1]]
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().pl_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# candidates of pl_batch_autotune, in the order of its report
BATCH_CANDIDATES = ("fp64/bucketed/lanes2", "fp64/bucketed/lanes4", "fp64/bucketed/lanes8",
                    "fp64/bucketed/lanes4/chunk256", "fp64/persistent", "mixed/flush4/lanes4",
                    "mixed/flush2/lanes4")


def autotune(problems, lam, tol=1e-3, device="cuda", inputs=None, stream=None):
    """pl_batch_autotune on these datasets: returns (choice, report); choice is
    a dict of Batch keyword arguments (precision, flush, lanes, chunk,
    schedule), report per candidate {"ms", "max_abs_dl"} (report.cached: the
    choice came from the tuning cache)."""
    lib = load()
    inputs = inputs if inputs is not None else [Inputs(pr.locs, pr.y, pr.X, device)
                                                for pr in problems]
    omegas = [_host_f64(pr.omega, 5) for pr in problems]
    lam = _host_f64(lam).reshape(-1)
    p = inputs[0].p
    D = len(inputs)
    arr = (PlDataset * D)()
    for i, (inp, om) in enumerate(zip(inputs, omegas)):
        arr[i] = PlDataset(inp.locs.data_ptr(), inp.y.data_ptr(), inp.Xc.data_ptr(), inp.n,
                           om.ctypes.data, om.shape[0])
    sz = ctypes.c_size_t(0)
    check(lib.pl_batch_autotune_workspace_size(arr, D, p, lam.ctypes.data_as(ctypes.c_void_p),
                                               lam.shape[0], ctypes.byref(sz)),
          "pl_batch_autotune_workspace_size")
    work = torch.empty(sz.value, dtype=torch.uint8, device=device)
    o = _opts()
    rep = (ctypes.c_double * (2 * len(BATCH_CANDIDATES)))()
    check(lib.pl_batch_autotune(arr, D, p, lam.ctypes.data_as(ctypes.c_void_p), lam.shape[0],
                                float(tol), ctypes.byref(o), rep,
                                ctypes.c_void_p(work.data_ptr()), work.numel(), _stream_ptr(stream)),
          "pl_batch_autotune")
    del work
    choice = {"precision": "mixed" if o.precision == _lib.PL_MIXED else "fp64",
              "flush": int(o.flush), "lanes": int(o.lanes), "chunk": int(o.chunk),
              "schedule": "persistent" if o.flags & _lib.PL_OPT_BATCH_PERSISTENT else "bucketed"}
    nc = len(BATCH_CANDIDATES)
    report = TuneReport({c: {"ms": rep[i], "max_abs_dl": rep[nc + i]}
                         for i, c in enumerate(BATCH_CANDIDATES)})
    report.cached = bool(rep[0] == -2.0)
    return choice, report
