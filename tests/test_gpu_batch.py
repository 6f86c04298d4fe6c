"""The uneven batch, in both schedules, against the single-dataset path and
the oracle: same records (up to the Jacobian's summation order), independent
of the slab pool size (persistent) or of the pass size and stream count
(size-bucketed), stable across graph replays, failures isolated per unit.
The mixed form of the size-bucketed schedule equals the single-dataset mixed
path and meets the 1e-2 bar against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def _problems(D=10, seed=0, n_lo=40, n_hi=700):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(D):
        n = int(rng.integers(n_lo, n_hi))
        K = int(rng.integers(1, 5))
        out.append(synth.small_problem(n, p=2, K=K, M=2, seed=100 + i, aniso=bool(i % 2)))
    return out


def _check_close(a, b, n, tol=1e-11):
    d = np.abs(a - b)
    assert np.max(d / np.maximum(np.abs(b), 1.0)) <= tol
    assert np.max(d) <= tol * n


@pytest.mark.parametrize("schedule", ["bucketed", "persistent"])
def test_batch_matches_single_path_and_oracle(plprof_lib, schedule):
    pl = plprof_lib
    probs = _problems()
    lam = probs[0].lam
    print(f"batch {schedule}: {len(probs)} datasets", flush=True)
    b = pl.batch.Batch(probs, lam, schedule=schedule).run()
    torch.cuda.synchronize()
    assert b.error() == 0
    for i, pr in enumerate(probs):
        got = {k: v.cpu().numpy() for k, v in b.records(i).items()}
        one = pl.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, lam, return_beta=True)
        one = {k: v.cpu().numpy() for k, v in one.items()}
        assert np.array_equal(got["info"], one["info"])
        _check_close(got["loglik"], one["loglik"], pr.n)
        _check_close(got["loglik_reml"], one["loglik_reml"], pr.n)
        np.testing.assert_allclose(got["beta"], one["beta"], rtol=1e-9, atol=1e-10)
    for i in (0, len(probs) - 1):
        pr = probs[i]
        ref = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, lam)
        got = b.records(i)["loglik"].cpu().numpy()
        _check_close(got, ref["loglik"], pr.n, tol=1e-8)


@pytest.mark.parametrize("schedule", ["bucketed", "persistent"])
def test_batch_pool_size_and_replay_invariance(plprof_lib, schedule):
    pl = plprof_lib
    probs = _problems(D=8, seed=1)
    lam = probs[0].lam
    print(f"batch {schedule}: pool / pass sizes", flush=True)
    big = pl.batch.Batch(probs, lam, schedule=schedule).run()
    if schedule == "persistent":
        small = pl.batch.Batch(probs, lam, schedule=schedule, max_slabs=3).run()
    else:  # passes of at most 3 units on 2 streams
        small = pl.batch.Batch(probs, lam, chunk=3, lanes=2).run()
    torch.cuda.synchronize()
    assert big.error() == 0 and small.error() == 0
    if schedule == "persistent":
        assert small.slabs == 3
    else:
        assert small.lanes == 2 and small.passes > big.passes
    a = big.records()["loglik"].cpu().numpy().copy()
    assert np.array_equal(a, small.records()["loglik"].cpu().numpy())
    for _ in range(3):  # graph replays, with eager work in between
        small.run()
        torch.cuda.synchronize()
        _ = torch.ones(10, device="cuda").sum().item()
        assert np.array_equal(a, small.records()["loglik"].cpu().numpy())


@pytest.mark.parametrize("schedule", ["bucketed", "persistent"])
def test_batch_isolates_failed_unit(plprof_lib, schedule):
    pl = plprof_lib
    probs = _problems(D=4, seed=2)
    pr = probs[1]
    pr.locs = pr.locs.copy()
    pr.locs[3] = pr.locs[1]
    pr.omega = pr.omega.copy()
    pr.omega[0, 2] = 0.0  # nugget 0 with a duplicated location
    lam = probs[0].lam
    b = pl.batch.Batch(probs, lam, schedule=schedule).run()
    torch.cuda.synchronize()
    rec = b.records(1)
    assert np.all(rec["info"].cpu().numpy()[0] > 0)
    for i in (0, 2, 3):
        q = probs[i]
        ref = oracle.profile_loglik(q.locs, q.y, q.X, q.omega, lam)
        _check_close(b.records(i)["loglik"].cpu().numpy(), ref["loglik"], q.n, tol=1e-8)


@pytest.mark.parametrize("schedule", ["bucketed", "persistent"])
def test_batch_large_units_match_oracle(plprof_lib, schedule):
    # units up to n = 1500 (12 block columns, the largest of the uneven
    # workload) beside small ones, so that deep task chains and slabs reused
    # across waves of different sizes are covered; every record against the
    # oracle, FP64 bar
    pl = plprof_lib
    ns = [1500, 1217, 1388, 130, 1452, 101, 777]
    probs = [synth.small_problem(n, p=2, K=2 if n > 1000 else 3, M=2, seed=300 + i,
                                 aniso=bool(i % 2)) for i, n in enumerate(ns)]
    lam = probs[0].lam
    print(f"batch {schedule}: n = {ns}", flush=True)
    b = pl.batch.Batch(probs, lam, schedule=schedule, max_slabs=4, chunk=2).run()
    torch.cuda.synchronize()
    assert b.error() == 0
    for i, pr in enumerate(probs):
        rec = {k: v.cpu().numpy() for k, v in b.records(i).items()}
        ref, refb = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, lam, return_beta=True)
        assert np.array_equal(rec["info"], ref["info"])
        _check_close(rec["loglik"], ref["loglik"], pr.n, tol=1e-8)
        _check_close(rec["loglik_reml"], ref["loglik_reml"], pr.n, tol=1e-8)
        np.testing.assert_allclose(rec["beta"], refb, rtol=1e-7, atol=1e-7)


def test_batch_wait_limit_drains_and_reports(plprof_lib):
    # a 1-microsecond limit on every task wait: waits that are not met at once
    # give up, set the error flag and make every later task skip its work.
    # The launch must still end (this test returning is the proof) and report
    # the error; a plan with the default limit on the same data is then exact.
    pl = plprof_lib
    probs = _problems(D=6, seed=4, n_lo=600, n_hi=1500)
    lam = probs[0].lam
    print("batch: 1 us wait limit", flush=True)
    tight = pl.batch.Batch(probs, lam, wait_us=1, schedule="persistent").run()
    torch.cuda.synchronize()
    assert tight.error() == 1
    tight.run()  # the error flag is cleared by every launch and set again
    torch.cuda.synchronize()
    assert tight.error() == 1
    tight.close()
    print("batch: default wait limit", flush=True)
    ok = pl.batch.Batch(probs, lam, schedule="persistent").run()
    torch.cuda.synchronize()
    assert ok.error() == 0
    pr = probs[0]
    ref = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, lam)
    _check_close(ok.records(0)["loglik"].cpu().numpy(), ref["loglik"], pr.n, tol=1e-8)


def test_batch_mixed_matches_single_mixed_path_and_oracle(plprof_lib):
    """The mixed form in the size-bucketed batch: every record equal to the
    single-dataset mixed call (the same kernels on the same unit), the
    oracle within 1e-2 on n up to 1500, and the FP64 redo of a unit whose
    FP32 factorisation breaks down."""
    pl = plprof_lib
    ns = [1500, 260, 1100, 131, 900, 640]
    probs = [synth.small_problem(n, p=2, K=3, M=2, seed=500 + i, aniso=bool(i % 2))
             for i, n in enumerate(ns)]
    lam = probs[0].lam
    print(f"batch mixed: n = {ns}", flush=True)
    b = pl.batch.Batch(probs, lam, precision="mixed", chunk=2, lanes=3).run()
    torch.cuda.synchronize()
    for i, pr in enumerate(probs):
        got = {k: v.cpu().numpy() for k, v in b.records(i).items()}
        one = pl.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, lam, precision="mixed",
                                return_beta=True)
        one = {k: v.cpu().numpy() for k, v in one.items()}
        assert np.array_equal(got["info"], one["info"])
        _check_close(got["loglik"], one["loglik"], pr.n)
        ref = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, lam)
        assert np.max(np.abs(got["loglik"] - ref["loglik"])) <= 1e-2
    b.close()


def test_batch_mixed_redoes_fp32_breakdown_in_fp64(plprof_lib):
    """A unit whose V is SPD in FP64 but whose FP32 Schur complements lose
    positivity (duplicated locations in different tiles, tiny nugget) is
    redone with the FP64 form: flagged, and at the FP64 bar against the
    oracle; the other units stay within the mixed bar."""
    pl = plprof_lib
    probs = _problems(D=3, seed=6)
    pr = synth.small_problem(260, p=2, K=3, M=2, seed=31)
    locs = pr.locs.copy()
    for i in range(0, 40):
        locs[130 + i] = locs[i] + 1e-9
    pr.locs = locs
    pr.omega = pr.omega.copy()
    pr.omega[1] = [2.0, 2.5, 1e-7, 1.0, 0.0]
    probs.insert(1, pr)
    lam = pr.lam
    print("batch mixed: FP32 breakdown", flush=True)
    b = pl.batch.Batch(probs, lam, precision="mixed").run()
    torch.cuda.synchronize()
    info = b.records(1)["info"].cpu().numpy()
    ll = b.records(1)["loglik"].cpu().numpy()
    ref = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, lam)
    assert ref["info"][1, 0] == 0
    assert np.all((info[1] & pl.PL_INFO_FALLBACK) != 0)
    assert np.all((info[1] & ~pl.PL_INFO_FALLBACK) == 0)
    _check_close(ll[1], ref["loglik"][1], pr.n, tol=1e-8)
    for i in (0, 2, 3):
        q = probs[i]
        ref = oracle.profile_loglik(q.locs, q.y, q.X, q.omega, lam)
        assert np.max(np.abs(b.records(i)["loglik"].cpu().numpy() - ref["loglik"])) <= 1e-2


def test_batch_mixed_tall_border(plprof_lib):
    """The mixed batch with 44 right-hand sides (a 48-row bordered tile row
    of its own): equal to the single-dataset mixed path."""
    pl = plprof_lib
    probs = [synth.small_problem(n, p=4, K=2, M=40, seed=900 + i)
             for i, n in enumerate((500, 140, 333))]
    lam = probs[0].lam
    print("batch mixed: M + p = 44", flush=True)
    b = pl.batch.Batch(probs, lam, precision="mixed").run()
    torch.cuda.synchronize()
    for i, pr in enumerate(probs):
        got = b.records(i)["loglik"].cpu().numpy()
        one = pl.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, lam, precision="mixed")
        _check_close(got, one["loglik"].cpu().numpy(), pr.n)
    b.close()
