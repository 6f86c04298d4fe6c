"""Serving loop for profile-likelihood requests of different sizes.

Requests (one dataset plus its omega and lambda points) arrive over time.  A
request is admitted as soon as a slot is free and its whole HBM footprint
(inputs, workspace, records, beta) can be carved from the device arena, so
requests arriving while others run start at once and their kernels overlap
on the device: each slot owns a HIP stream and a host worker thread (the
library call for the mixed form waits on its own stream to look for
points that need the FP64 redo, so one thread per slot keeps that wait from
blocking the other slots).  Admission is in arrival order, so a large
request is never starved by smaller ones behind it.  Inputs and factors stay
device-resident for the life of the request; a request whose full workspace
would exceed the per-request cap runs its omega points in chunks.

Failure handling.  A request may carry a deadline (seconds after its
arrival): one still waiting for admission when its deadline passes is
dropped unstarted ("expired").  Server.cancel(rid), callable from any
thread, drops a waiting request at once and, for a request already on the
device, discards its result when its kernels finish (work on the GPU is not
interrupted; its memory and slot are released as usual).  Dropped requests
are kept in Server.dropped with their status; run() returns the completed
ones.

The scheduler (Server) does not touch the device: it drives an executor
through reserve/start/poll/finish/release, so its admission logic is tested
on the CPU with a fake executor.  GpuExecutor is the device one.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

ALIGN = 256


def _up(b: int) -> int:
    return (int(b) + ALIGN - 1) // ALIGN * ALIGN


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    locs: np.ndarray
    y: np.ndarray
    X: np.ndarray
    omega: np.ndarray
    lam: np.ndarray
    precision: str = "fp64"          # "fp64", "mixed" or "auto" (tuning cache)
    deadline: float = float("inf")   # admission deadline, seconds after arrival
    # filled in by the server
    admitted: float = float("nan")
    finished: float = float("nan")
    result: dict = field(default_factory=dict)
    status: str = "pending"          # "done", "expired" or "cancelled" at the end

    @property
    def n(self) -> int:
        return self.locs.shape[0]

    @property
    def p(self) -> int:
        return self.X.shape[1] if self.X.ndim == 2 else 1

    @property
    def K(self) -> int:
        return self.omega.shape[0]

    @property
    def M(self) -> int:
        return self.lam.shape[0]

    @property
    def points(self) -> int:
        return self.K * self.M

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Arena:
    """First-fit allocator of aligned byte ranges in one buffer of `size`
    bytes; freed ranges coalesce with their neighbours."""

    def __init__(self, size: int):
        self.size = int(size) // ALIGN * ALIGN
        self.free_list = [(0, self.size)]      # sorted (offset, length)
        self.live = {}                         # offset -> length

    def alloc(self, nbytes: int):
        need = _up(max(1, nbytes))
        for i, (off, ln) in enumerate(self.free_list):
            if ln >= need:
                if ln == need:
                    self.free_list.pop(i)
                else:
                    self.free_list[i] = (off + need, ln - need)
                self.live[off] = need
                return off
        return None

    def free(self, off: int):
        ln = self.live.pop(off)
        fl = self.free_list
        i = 0
        while i < len(fl) and fl[i][0] < off:
            i += 1
        fl.insert(i, (off, ln))
        # merge with the right then the left neighbour
        if i + 1 < len(fl) and fl[i][0] + fl[i][1] == fl[i + 1][0]:
            fl[i] = (fl[i][0], fl[i][1] + fl[i + 1][1])
            fl.pop(i + 1)
        if i > 0 and fl[i - 1][0] + fl[i - 1][1] == fl[i][0]:
            fl[i - 1] = (fl[i - 1][0], fl[i - 1][1] + fl[i][1])
            fl.pop(i)

    @property
    def used(self) -> int:
        return sum(self.live.values())

    @property
    def largest_free(self) -> int:
        return max((ln for _, ln in self.free_list), default=0)


class Server:
    """Continuous batching over `executor.slots` concurrent requests with
    admission by HBM footprint (see the module docstring)."""

    def __init__(self, executor, poll_sleep: float = 2e-4):
        import threading
        self.ex = executor
        self.poll_sleep = poll_sleep
        self.trace = []          # (time, event, rid)
        self.max_inflight = 0
        self.peak_bytes = 0
        self.dropped = []        # expired or cancelled requests
        self._cancel = set()
        self._lock = threading.Lock()

    def cancel(self, rid) -> None:
        """Drop request `rid`: unstarted, it never runs; on the device, its
        result is discarded when it finishes.  Thread-safe."""
        with self._lock:
            self._cancel.add(rid)

    def _take_cancels(self):
        with self._lock:
            c, self._cancel = self._cancel, set()
        return c

    def run(self, requests, clock=time.perf_counter):
        """Serve `requests` (any order; arrival times relative to the start)
        and return them in completion order with timing and results set."""
        pending = sorted(requests, key=lambda r: r.arrival)
        for r in pending:
            if not self.ex.fits(r):
                raise ValueError(f"request {r.rid} (n={r.n}, K={r.K}) can never fit the HBM budget")
        queue, inflight, done = [], [], []
        free_slots = list(range(self.ex.slots))
        cancelled = set()        # requests to drop, by id
        t0 = clock()
        i = 0

        def drop(req, status, when):
            req.status = status
            req.finished = when
            self.dropped.append(req)
            self.trace.append((when, status, req.rid))

        while len(done) + len(self.dropped) < len(pending):
            now = clock() - t0
            while i < len(pending) and pending[i].arrival <= now:
                queue.append(pending[i])
                self.trace.append((now, "arrive", pending[i].rid))
                i += 1
            cancelled |= self._take_cancels()
            progressed = False
            # unstarted requests that were cancelled or outlived their deadline
            for req in list(queue):
                if req.rid in cancelled:
                    queue.remove(req)
                    drop(req, "cancelled", now)
                    progressed = True
                elif now > req.arrival + req.deadline:
                    queue.remove(req)
                    drop(req, "expired", now)
                    progressed = True
            for h in list(inflight):
                req, slot, tok, handle = h
                if self.ex.poll(handle):
                    result = self.ex.finish(handle)
                    self.ex.release(tok)
                    free_slots.append(slot)
                    inflight.remove(h)
                    if req.rid in cancelled:
                        drop(req, "cancelled", clock() - t0)
                    else:
                        req.result = result
                        req.status = "done"
                        req.finished = clock() - t0
                        done.append(req)
                        self.trace.append((req.finished, "finish", req.rid))
                    progressed = True
            while queue and free_slots:
                tok = self.ex.reserve(queue[0])
                if tok is None:
                    break                       # head of line waits for memory
                req = queue.pop(0)
                slot = free_slots.pop(0)
                req.admitted = clock() - t0
                self.trace.append((req.admitted, "admit", req.rid))
                inflight.append((req, slot, tok, self.ex.start(req, slot, tok)))
                self.max_inflight = max(self.max_inflight, len(inflight))
                self.peak_bytes = max(self.peak_bytes, self.ex.bytes_in_use())
                progressed = True
            if not progressed:
                if not queue and not inflight and i < len(pending):
                    time.sleep(max(0.0, min(0.005, pending[i].arrival - (clock() - t0))))
                else:
                    time.sleep(self.poll_sleep)
        return done


def latency_summary(done) -> dict:
    lat = np.array([r.latency for r in done])
    wait = np.array([r.admitted - r.arrival for r in done])
    pts = sum(r.points for r in done)
    span = max(r.finished for r in done) - min(r.arrival for r in done)
    return {"requests": len(done), "points": int(pts), "span_s": float(span),
            "points_per_s": float(pts / span),
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "max_s": float(lat.max()), "mean_wait_s": float(wait.mean())}


class _ArenaInputs:
    """Device views of one request's dataset inside the arena, with the
    attributes the profile_loglik binding reads."""

    def __init__(self, locs, y, Xc, n, p, device):
        self.locs, self.y, self.Xc, self.n, self.p, self.device = locs, y, Xc, n, p, device


class GpuExecutor:
    """Runs admitted requests with pl_profile_loglik, one stream and one
    worker thread per slot, all memory carved from one arena of
    `hbm_budget` bytes allocated up front."""

    def __init__(self, hbm_budget: int, slots: int = 4, device: str = "cuda",
                 max_request_work: int = 16 << 30, tune_tol: float = 1e-3):
        import concurrent.futures as cf

        import torch

        from . import api
        self.torch, self.api = torch, api
        self.device = device
        self.slots = int(slots)
        self.max_request_work = int(max_request_work)
        self.tune_tol = float(tune_tol)
        self._forms = {}
        self.arena = Arena(hbm_budget)
        self.buf = torch.empty(self.arena.size, dtype=torch.uint8, device=device)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(self.slots)]
        self.pool = cf.ThreadPoolExecutor(max_workers=self.slots)

    # -- form of one request ----------------------------------------------
    def form(self, req):
        """(precision, flush) of a request: as given, or for precision "auto"
        the tuning cache's choice for its size (pl_tune_lookup with the
        executor's budget `tune_tol`), FP64 when nothing is stored."""
        if req.precision != "auto":
            return req.precision, 0
        key = (req.n, req.p + req.M)
        if key not in self._forms:
            c = self.api.tune_lookup(req.n, req.p + req.M, self.tune_tol)
            self._forms[key] = (c["precision"], c["flush"]) if c else ("fp64", 0)
        return self._forms[key]

    # -- memory plan of one request ----------------------------------------
    def plan(self, req):
        """(chunk, [(name, bytes)]) for the request's carve-out."""
        n, p, K, M = req.n, req.p, req.K, req.M
        prec = self.form(req)[0]
        chunk = 0
        work = self.api.workspace_size(n, p, K, M, prec, 0)
        if work > self.max_request_work:
            one = self.api.workspace_size(n, p, K, M, prec, 1)
            two = self.api.workspace_size(n, p, K, M, prec, 2)
            per = max(1, two - one)
            chunk = int(max(1, min(K, 1 + (self.max_request_work - one) // per)))
            work = self.api.workspace_size(n, p, K, M, prec, chunk)
        parts = [("locs", 16 * n), ("y", 8 * n), ("Xc", 8 * n * p), ("out", 80 * K * M),
                 ("beta", 8 * K * M * p), ("work", work)]
        return chunk, parts

    def footprint(self, req) -> int:
        return sum(_up(b) for _, b in self.plan(req)[1])

    def fits(self, req) -> bool:
        return self.footprint(req) <= self.arena.size

    def reserve(self, req):
        fp = self.footprint(req)
        off = self.arena.alloc(fp)
        return None if off is None else off

    def release(self, tok):
        self.arena.free(tok)

    def bytes_in_use(self) -> int:
        return self.arena.used

    # -- execution ------------------------------------------------------------
    def start(self, req, slot, tok):
        return self.pool.submit(self._run, req, slot, tok)

    def _run(self, req, slot, off):
        torch = self.torch
        chunk, parts = self.plan(req)
        views, o = {}, off
        for name, b in parts:
            views[name] = self.buf[o:o + b]
            o += _up(b)
        n, p, K, M = req.n, req.p, req.K, req.M
        s = self.streams[slot]
        with torch.cuda.stream(s):
            locs = views["locs"].view(torch.float64).view(n, 2)
            y = views["y"].view(torch.float64)
            Xc = views["Xc"].view(torch.float64).view(p, n)
            locs.copy_(torch.from_numpy(np.ascontiguousarray(req.locs, dtype=np.float64)))
            y.copy_(torch.from_numpy(np.ascontiguousarray(req.y, dtype=np.float64)))
            Xc.copy_(torch.from_numpy(np.ascontiguousarray(np.asarray(req.X, dtype=np.float64)
                                                           .reshape(n, p).T)))
            inp = _ArenaInputs(locs, y, Xc, n, p, self.device)
            out = views["out"].view(torch.float64).view(K, M, 10)
            beta = views["beta"].view(torch.float64).view(K, M, p)
            prec, flush = self.form(req)
            res = self.api.profile_loglik(None, None, None, req.omega, req.lam,
                                          precision=prec, flush=flush, chunk=chunk,
                                          return_beta=True, out=out, beta=beta,
                                          work=views["work"], stream=s, inputs=inp)
            host = {k: v.to("cpu", non_blocking=False).numpy() for k, v in res.items()}
        s.synchronize()
        return host

    def poll(self, handle) -> bool:
        return handle.done()

    def finish(self, handle):
        return handle.result()

    def close(self):
        self.pool.shutdown(wait=True)
        self.buf = None

