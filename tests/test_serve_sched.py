"""Host logic of the serving loop: the arena allocator and the admission
scheduler, driven by a fake executor (no device)."""
import time

import numpy as np
import pytest

from paper_2305_04318_amd.serve import ALIGN, Arena, Request, Server, latency_summary


def test_arena_against_bitmap():
    """Random alloc/free sequences: live ranges never overlap, stay inside the
    arena, and the free list always equals the complement (fully merged)."""
    rng = np.random.default_rng(7)
    size = 64 * ALIGN
    a = Arena(size)
    live = []
    for _ in range(3000):
        if live and rng.random() < 0.45:
            off = live.pop(int(rng.integers(len(live))))
            a.free(off)
        else:
            off = a.alloc(int(rng.integers(1, 9 * ALIGN)))
            if off is not None:
                live.append(off)
        used = np.zeros(size // ALIGN, bool)
        for off, ln in a.live.items():
            assert off % ALIGN == 0 and ln % ALIGN == 0 and off + ln <= size
            assert not used[off // ALIGN:(off + ln) // ALIGN].any()
            used[off // ALIGN:(off + ln) // ALIGN] = True
        free = np.zeros_like(used)
        prev_end = -1
        for off, ln in a.free_list:
            assert off > prev_end, "free ranges must be sorted and merged"
            free[off // ALIGN:(off + ln) // ALIGN] = True
            prev_end = off + ln
        assert np.array_equal(free, ~used)
    for off in list(live):
        a.free(off)
    assert a.free_list == [(0, a.size)] and a.used == 0


def test_arena_first_fit_reuses_hole():
    a = Arena(10 * ALIGN)
    x = a.alloc(3 * ALIGN)
    y = a.alloc(3 * ALIGN)
    a.alloc(3 * ALIGN)
    assert a.alloc(2 * ALIGN) is None
    a.free(y)
    assert a.alloc(2 * ALIGN) == y
    assert x == 0


class FakeExecutor:
    """Each request needs `mem[rid]` bytes for `dur[rid]` seconds."""

    def __init__(self, budget, slots, mem, dur):
        self.arena = Arena(budget)
        self.slots = slots
        self.mem, self.dur = mem, dur
        self.running = {}
        self.max_running = 0
        self.max_bytes = 0

    def fits(self, req):
        return self.mem[req.rid] <= self.arena.size

    def reserve(self, req):
        return self.arena.alloc(self.mem[req.rid])

    def release(self, tok):
        self.arena.free(tok)

    def bytes_in_use(self):
        return self.arena.used

    def start(self, req, slot, tok):
        assert slot not in self.running
        self.running[slot] = req.rid
        self.max_running = max(self.max_running, len(self.running))
        self.max_bytes = max(self.max_bytes, self.arena.used)
        return (slot, req.rid, time.perf_counter())

    def poll(self, h):
        return time.perf_counter() - h[2] >= self.dur[h[1]]

    def finish(self, h):
        del self.running[h[0]]
        return {"rid": h[1]}


def _req(rid, t, K=4):
    z = np.zeros((8, 2))
    return Request(rid, t, z, np.ones(8), np.ones((8, 1)), np.zeros((K, 5)), np.zeros(2))


def test_server_admission_respects_budget_and_slots():
    rng = np.random.default_rng(3)
    R = 40
    mem = {i: int(rng.integers(1, 40)) * ALIGN for i in range(R)}
    dur = {i: float(rng.uniform(0.001, 0.01)) for i in range(R)}
    reqs = [_req(i, float(t)) for i, t in enumerate(np.sort(rng.uniform(0, 0.08, R)))]
    ex = FakeExecutor(64 * ALIGN, 3, mem, dur)
    srv = Server(ex, poll_sleep=1e-4)
    done = srv.run(reqs)
    assert sorted(r.rid for r in done) == list(range(R))
    assert ex.max_running <= 3 and ex.max_bytes <= 64 * ALIGN
    assert all(r.result["rid"] == r.rid for r in done)
    # admission in arrival order (no overtaking)
    admits = [rid for _, ev, rid in srv.trace if ev == "admit"]
    assert admits == sorted(admits, key=lambda i: reqs[i].arrival)
    for r in done:
        assert r.arrival <= r.admitted <= r.finished
    s = latency_summary(done)
    assert s["requests"] == R and s["p50_s"] <= s["p99_s"] <= s["max_s"]


def test_server_overlaps_requests_that_fit():
    """Requests arriving while another runs are admitted at once when memory
    and a slot are free (continuous batching, not a queue)."""
    mem = {0: ALIGN, 1: ALIGN, 2: ALIGN}
    dur = {0: 0.05, 1: 0.05, 2: 0.05}
    ex = FakeExecutor(8 * ALIGN, 4, mem, dur)
    srv = Server(ex)
    done = srv.run([_req(0, 0.0), _req(1, 0.01), _req(2, 0.02)])
    by = {r.rid: r for r in done}
    assert ex.max_running == 3
    assert by[1].admitted < by[0].finished and by[2].admitted < by[0].finished


def test_server_head_of_line_waits_for_memory():
    mem = {0: 6 * ALIGN, 1: 6 * ALIGN, 2: ALIGN}
    dur = {0: 0.03, 1: 0.01, 2: 0.01}
    ex = FakeExecutor(8 * ALIGN, 4, mem, dur)
    srv = Server(ex)
    done = srv.run([_req(0, 0.0), _req(1, 0.001), _req(2, 0.002)])
    by = {r.rid: r for r in done}
    # request 1 cannot fit beside 0; request 2 could but must not overtake it
    assert by[1].admitted >= by[0].finished
    assert by[2].admitted >= by[1].admitted
    assert ex.max_bytes <= 8 * ALIGN


def test_server_rejects_request_over_budget():
    ex = FakeExecutor(4 * ALIGN, 2, {0: 5 * ALIGN}, {0: 0.0})
    with pytest.raises(ValueError):
        Server(ex).run([_req(0, 0.0)])


def test_server_expires_requests_past_their_deadline():
    """A request still waiting for memory when its admission deadline passes
    is dropped unstarted; the others run."""
    mem = {0: 6 * ALIGN, 1: 6 * ALIGN, 2: ALIGN}
    dur = {0: 0.05, 1: 0.01, 2: 0.01}
    ex = FakeExecutor(8 * ALIGN, 4, mem, dur)
    srv = Server(ex)
    r1 = _req(1, 0.001)
    r1.deadline = 0.01            # request 0 holds the memory for 0.05 s
    done = srv.run([_req(0, 0.0), r1, _req(2, 0.002)])
    assert sorted(r.rid for r in done) == [0, 2]
    assert [(r.rid, r.status) for r in srv.dropped] == [(1, "expired")]
    assert r1.result == {} and np.isnan(r1.admitted)
    assert all(r.status == "done" for r in done)
    assert ex.arena.used == 0 and not ex.running


def test_server_cancel_waiting_and_running_requests():
    """Cancelling a queued request drops it unstarted; cancelling one on the
    device discards its result once it finishes and frees its slot and
    memory."""
    import threading
    mem = {0: 6 * ALIGN, 1: 6 * ALIGN, 2: ALIGN, 3: ALIGN}
    dur = {0: 0.06, 1: 0.01, 2: 0.01, 3: 0.01}
    ex = FakeExecutor(8 * ALIGN, 2, mem, dur)
    srv = Server(ex, poll_sleep=1e-4)
    reqs = [_req(0, 0.0), _req(1, 0.001), _req(2, 0.002), _req(3, 0.003)]
    timer = threading.Timer(0.02, lambda: (srv.cancel(1), srv.cancel(0)))
    timer.start()
    done = srv.run(reqs)
    timer.join()
    st = {r.rid: r.status for r in srv.dropped}
    assert st == {0: "cancelled", 1: "cancelled"}
    assert sorted(r.rid for r in done) == [2, 3]
    assert reqs[0].result == {} and not np.isnan(reqs[0].admitted)   # ran, result discarded
    assert np.isnan(reqs[1].admitted)                                 # never started
    assert ex.arena.used == 0 and not ex.running
    s = latency_summary(done)
    assert s["requests"] == 2
