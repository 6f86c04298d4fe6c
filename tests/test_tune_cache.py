"""The tuning cache's host logic (no GPU): choices stored under an explicit
architecture name are found again for the same key (size bucket floor(log2
n), right-hand sides, budget; units bucket for batches), missed otherwise,
persisted to the file and reloaded from it (the last line of a key wins)."""
import ctypes

import pytest

import paper_2305_04318_amd as pl
from paper_2305_04318_amd import _lib, api


@pytest.fixture
def cache(tmp_path):
    path = tmp_path / "tune.txt"
    api.tune_cache_set(str(path))
    yield path
    api.tune_cache_set(None)


def test_store_lookup_and_buckets(cache):
    mixed = {"precision": "mixed", "flush": 2, "chunk": 0, "lanes": 0, "schedule": "bucketed"}
    api.tune_store(mixed, n=2000, q=12, tol=1e-3, arch="gfx950", ms=1.5)
    # same bucket of n (1024..2047), same q and budget: a hit
    for n in (1024, 1500, 2047):
        assert api.tune_lookup(n, 12, 1e-3, arch="gfx950") == mixed
    # another bucket, q, budget, architecture or kind: a miss
    assert api.tune_lookup(2048, 12, 1e-3, arch="gfx950") is None
    assert api.tune_lookup(2000, 13, 1e-3, arch="gfx950") is None
    assert api.tune_lookup(2000, 12, 1e-2, arch="gfx950") is None
    assert api.tune_lookup(2000, 12, 1e-3, arch="gfx942") is None
    assert api.tune_lookup(2000, 12, 1e-3, kind=1, units=100, arch="gfx950") is None
    st = api.tune_stats()
    assert st["entries"] == 1 and st["hits"] == 3 and st["misses"] == 5


def test_file_persistence_last_line_wins(cache):
    a = {"precision": "fp64", "flush": 0, "chunk": 0, "lanes": 4, "schedule": "bucketed"}
    b = {"precision": "mixed", "flush": 4, "chunk": 256, "lanes": 8, "schedule": "bucketed"}
    c = {"precision": "fp64", "flush": 0, "chunk": 0, "lanes": 0, "schedule": "persistent"}
    api.tune_store(a, n=1500, q=4, tol=1e-3, kind=1, units=32768, arch="gfx950")
    api.tune_store(b, n=1400, q=4, tol=1e-3, kind=1, units=40000, arch="gfx950")  # same key
    api.tune_store(c, n=300, q=4, tol=1e-3, kind=1, units=32768, arch="gfx950")
    lines = cache.read_text().splitlines()
    assert len(lines) == 3 and all(line.startswith("v1 gfx950 1 ") for line in lines)
    api.tune_cache_set(str(cache))          # reload from the file
    assert api.tune_stats()["entries"] == 2
    assert api.tune_lookup(1500, 4, 1e-3, kind=1, units=60000, arch="gfx950") == b
    assert api.tune_lookup(400, 4, 1e-3, kind=1, units=33000, arch="gfx950") == c
    assert api.tune_lookup(1500, 4, 1e-3, kind=1, units=30000, arch="gfx950") is None


def test_argument_checks(cache):
    lib = pl.load()
    o = _lib.PlOpts()
    g = b"gfx950"
    assert lib.pl_tune_lookup(g, 2, 100, 0, 4, 1e-3, ctypes.byref(o)) == -2
    assert lib.pl_tune_lookup(g, 0, 1, 0, 4, 1e-3, ctypes.byref(o)) == -3
    assert lib.pl_tune_lookup(g, 1, 100, 0, 4, 1e-3, ctypes.byref(o)) == -4
    assert lib.pl_tune_lookup(g, 0, 100, 0, 1, 1e-3, ctypes.byref(o)) == -5
    assert lib.pl_tune_lookup(g, 0, 100, 0, 4, -1.0, ctypes.byref(o)) == -6
    assert lib.pl_tune_lookup(g, 0, 100, 0, 4, 1e-3, None) == -7
    assert lib.pl_tune_lookup(g, 0, 100, 0, 4, 1e-3, ctypes.byref(o)) == _lib.PL_TUNE_MISS
    assert lib.pl_tune_cache_set(b"/nonexistent-dir/x/tune.txt") == -1
