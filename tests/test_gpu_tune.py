"""The autotuners and the persisted tuning cache on the GPU: a choice is
measured once, stored in the cache file, and reused (no timing, the same
choice) by the next call and by a process that reloads the file; the chosen
form meets the error budget against the oracle; serving requests of
precision "auto" run the stored form."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2305_04318_amd import api, batch, serve

pytestmark = pytest.mark.gpu
TOL = 1e-3


@pytest.fixture
def cache(tmp_path):
    path = tmp_path / "tune.txt"
    api.tune_cache_set(str(path))
    yield path
    api.tune_cache_set(None)


def test_single_autotune_is_cached_and_meets_budget(plprof_lib, cache):
    pl = plprof_lib
    pr = synth.small_problem(900, p=3, K=16, M=4, seed=61)
    print("autotune n=900: measured", flush=True)
    c1, r1 = pl.autotune(pr.locs, pr.y, pr.X, pr.omega, pr.lam, tol=TOL, sample=16)
    assert not r1.cached
    assert cache.read_text().count("\n") == 1
    c2, r2 = pl.autotune(pr.locs, pr.y, pr.X, pr.omega, pr.lam, tol=TOL, sample=16)
    assert r2.cached and c2 == c1
    st = api.tune_stats()
    assert st["hits"] >= 1 and st["entries"] == 1
    # a fresh table loaded from the file gives the same choice
    api.tune_cache_set(str(cache))
    found = api.tune_lookup(pr.n, pr.p + pr.M, TOL)
    assert found["precision"] == c1["precision"] and found["flush"] == c1["flush"]
    # the chosen form meets the budget against the oracle
    got = pl.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam, **c1)
    torch.cuda.synchronize()
    ref = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam)
    d = np.abs(got["loglik"].cpu().numpy() - ref["loglik"])
    assert d.max() <= TOL + 1e-8 * np.abs(ref["loglik"]).max()


def test_batch_autotune_is_cached_and_meets_budget(plprof_lib, cache):
    pl = plprof_lib
    rng = np.random.default_rng(8)
    probs = [synth.small_problem(int(n), p=2, K=3, M=2, seed=700 + i, aniso=bool(i % 2))
             for i, n in enumerate(rng.integers(100, 900, 12))]
    lam = probs[0].lam
    print("batch autotune: 12 datasets", flush=True)
    c1, r1 = batch.autotune(probs, lam, tol=TOL)
    assert not r1.cached
    assert all(r1[c]["ms"] > 0 for c in batch.BATCH_CANDIDATES)
    c2, r2 = batch.autotune(probs, lam, tol=TOL)
    assert r2.cached and c2 == c1
    b = pl.batch.Batch(probs, lam, **c1).run()
    torch.cuda.synchronize()
    for i in (0, 5, 11):
        q = probs[i]
        ref = oracle.profile_loglik(q.locs, q.y, q.X, q.omega, lam)
        d = np.abs(b.records(i)["loglik"].cpu().numpy() - ref["loglik"])
        assert d.max() <= TOL + 1e-8 * np.abs(ref["loglik"]).max()
    b.close()


def test_serving_auto_precision_uses_the_cache(plprof_lib, cache):
    """Requests of precision "auto" take the stored choice for their size
    (here the mixed form, stored for one size bucket) and FP64 elsewhere."""
    pl = plprof_lib
    small = synth.small_problem(700, p=2, K=5, M=3, seed=81)    # bucket 512..1023: stored
    other = synth.small_problem(300, p=2, K=4, M=3, seed=82)    # bucket 256..511: not stored
    api.tune_store({"precision": "mixed", "flush": 4}, n=small.n, q=5, tol=TOL)
    ex = serve.GpuExecutor(8 << 30, slots=2, tune_tol=TOL)
    reqs = [serve.Request(i, 0.0, pr.locs, pr.y, pr.X, pr.omega, pr.lam, "auto")
            for i, pr in enumerate((small, other))]
    assert ex.form(reqs[0]) == ("mixed", 4) and ex.form(reqs[1]) == ("fp64", 0)
    done = {r.rid: r for r in serve.Server(ex).run(reqs)}
    ex.close()
    for i, pr in enumerate((small, other)):
        ref = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega, pr.lam)
        d = np.abs(done[i].result["loglik"] - ref["loglik"])
        assert d.max() <= (1e-2 if i == 0 else 1e-8 * max(1.0, np.abs(ref["loglik"]).max()))
    # the mixed records differ from FP64 ones: the stored form really ran
    one = pl.profile_loglik(small.locs, small.y, small.X, small.omega, small.lam)
    torch.cuda.synchronize()
    assert not np.array_equal(done[0].result["loglik"], one["loglik"].cpu().numpy())
