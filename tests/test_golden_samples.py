"""The stored oracle samples of the full-size workloads
(tests/golden/large_samples.json): their inputs regenerate from the seeds on
this machine, and a stored record equals a fresh oracle evaluation.  No GPU."""
import json
import os

import numpy as np

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_fingerprints_and_one_record_recomputed():
    with open(os.path.join(HERE, "golden", "large_samples.json")) as f:
        data = json.load(f)
    assert set(data) == {"aniso_n2000", "aniso_n4000", "aniso_n8000"}
    for name, g in data.items():
        pr = getattr(synth, g["generator"]["function"].split(".", 1)[1])(**g["generator"]["kwargs"])
        fp = g["fingerprint"]
        for key, arr in (("sum_y", pr.y), ("sum_locs", pr.locs), ("sum_X", pr.X)):
            assert abs(float(np.sum(arr)) - fp[key]) <= 1e-12 * max(1.0, abs(fp[key])), (name, key)
        idx = g["omega_index"]
        assert len(idx) == len(set(idx)) and all(0 <= k < pr.K for k in idx)
        assert len(g["records"]["loglik"]) == len(idx)
    # one n=2000 point recomputed by the oracle now
    g = data["aniso_n2000"]
    pr = synth.config_aniso(**g["generator"]["kwargs"])
    k = g["omega_index"][0]
    rec = oracle.profile_loglik(pr.locs, pr.y, pr.X, pr.omega[k:k + 1], pr.lam)
    np.testing.assert_allclose(rec["loglik"][0], g["records"]["loglik"][0], rtol=1e-12, atol=0)
