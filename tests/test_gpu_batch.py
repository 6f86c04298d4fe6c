"""The persistent uneven batch against the single-dataset path and the oracle:
same records (up to the Jacobian's summation order), independent of the slab
pool size, stable across graph replays, failures isolated per unit."""
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


def test_batch_matches_single_path_and_oracle(plprof_lib):
    pl = plprof_lib
    probs = _problems()
    lam = probs[0].lam
    b = pl.batch.Batch(probs, lam).run()
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


def test_batch_slab_pool_size_and_replay_invariance(plprof_lib):
    pl = plprof_lib
    probs = _problems(D=8, seed=1)
    lam = probs[0].lam
    big = pl.batch.Batch(probs, lam).run()
    small = pl.batch.Batch(probs, lam, max_slabs=3).run()
    torch.cuda.synchronize()
    assert big.error() == 0 and small.error() == 0 and small.slabs == 3
    a = big.records()["loglik"].cpu().numpy().copy()
    assert np.array_equal(a, small.records()["loglik"].cpu().numpy())
    for _ in range(3):  # graph replays, with eager work in between
        small.run()
        torch.cuda.synchronize()
        _ = torch.ones(10, device="cuda").sum().item()
        assert np.array_equal(a, small.records()["loglik"].cpu().numpy())


def test_batch_isolates_failed_unit(plprof_lib):
    pl = plprof_lib
    probs = _problems(D=4, seed=2)
    pr = probs[1]
    pr.locs = pr.locs.copy()
    pr.locs[3] = pr.locs[1]
    pr.omega = pr.omega.copy()
    pr.omega[0, 2] = 0.0  # nugget 0 with a duplicated location
    lam = probs[0].lam
    b = pl.batch.Batch(probs, lam).run()
    torch.cuda.synchronize()
    rec = b.records(1)
    assert np.all(rec["info"].cpu().numpy()[0] > 0)
    for i in (0, 2, 3):
        q = probs[i]
        ref = oracle.profile_loglik(q.locs, q.y, q.X, q.omega, lam)
        _check_close(b.records(i)["loglik"].cpu().numpy(), ref["loglik"], q.n, tol=1e-8)


def test_batch_large_units_match_oracle(plprof_lib):
    # units up to n = 1500 (12 block columns, the largest of the uneven
    # workload) beside small ones, so that deep task chains and slabs reused
    # across waves of different sizes are covered; every record against the
    # oracle, FP64 bar
    pl = plprof_lib
    ns = [1500, 1217, 1388, 130, 1452, 101, 777]
    probs = [synth.small_problem(n, p=2, K=2 if n > 1000 else 3, M=2, seed=300 + i,
                                 aniso=bool(i % 2)) for i, n in enumerate(ns)]
    lam = probs[0].lam
    print(f"batch: n = {ns}, slab pool 4", flush=True)
    b = pl.batch.Batch(probs, lam, max_slabs=4).run()
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
    tight = pl.batch.Batch(probs, lam, wait_us=1).run()
    torch.cuda.synchronize()
    assert tight.error() == 1
    tight.run()  # the error flag is cleared by every launch and set again
    torch.cuda.synchronize()
    assert tight.error() == 1
    tight.close()
    print("batch: default wait limit", flush=True)
    ok = pl.batch.Batch(probs, lam).run()
    torch.cuda.synchronize()
    assert ok.error() == 0
    pr = probs[0]
    ref = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, lam)
    _check_close(ok.records(0)["loglik"].cpu().numpy(), ref["loglik"], pr.n, tol=1e-8)
