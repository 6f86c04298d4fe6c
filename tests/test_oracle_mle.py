"""Internal parameters of Step 2 (oracle.mle and the library's host-side
pl_to_internal / pl_from_internal) pinned by the paper's parameter table, the
covariance matrix they describe, and the closed forms of the definitions."""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import mle as om

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    rows = {}
    with open(os.path.join(HERE, "golden", "swiss_soil_params.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, *vals = line.split()
                rows[name] = [float(v) for v in vals]
    return rows


def _random_omega(rng, K):
    return np.column_stack([rng.uniform(0.2, 3.0, K), rng.uniform(0.3, 6.0, K),
                            rng.uniform(0.01, 1.0, K), np.exp(rng.uniform(-1.5, 1.5, K)),
                            rng.uniform(-3.0, 3.0, K)])


def test_combined_range_matches_paper_table():
    # Section 3.2: exp(gamma1 / 2) is the combined range sqrt(phi_X phi_Y);
    # the paper's tables print range, ratio and combined range side by side
    for name, (rng_x, combined, ratio, _sigma, nugget, _tau, *_angle_gammas) in _golden().items():
        w = om.to_internal([[rng_x, 1.0, nugget, ratio, 0.3]])[0]
        assert abs(math.exp(w[0] / 2.0) - combined) <= 0.006 * combined, name
        # gamma2^2 + gamma3^2 = phi_X/phi_Y - 1 and nu = sqrt(nu^2)
        assert abs(w[3] ** 2 + w[4] ** 2 - (ratio - 1.0)) < 1e-12 * ratio
        assert abs(w[2] - math.sqrt(nugget)) < 1e-15


def _printed_interval(v, digits=2):
    h = 0.5 * 10.0 ** -digits
    return v - h, v + h


def _gamma_range(ratio, angle, which):
    """Range of gamma2 (which 3) or gamma3 (which 4) of to_internal over the
    rounding box of the printed ratio and angle (a fine grid of the box; the
    functions are smooth there)."""
    vals = []
    for r in np.linspace(*_printed_interval(ratio), 21):
        for a in np.linspace(*_printed_interval(angle), 21):
            vals.append(om.to_internal([[1.0, 1.0, 0.1, r, a]])[0][which])
    return min(vals), max(vals)


def test_gammas_match_paper_tables():
    # Section 3.2 "Reparameterization": the Swiss and soil tables print the
    # anisotropy ratio, the angle and the internal parameters aniso1 (gamma2)
    # and aniso2 (gamma3) of the same fit.  The printed gammas must lie in the
    # range that the printed (ratio, angle), within their rounding, give.
    # Swiss (angle 0.65) has |gamma2| << |gamma3|, soil (angle -0.82) a
    # negative gamma3: a gamma2/gamma3 swap, a sign slip in the angle or a
    # missing factor 2 fails one of them.
    for name, row in _golden().items():
        ratio, angle, g2, g3 = row[2], row[6], row[7], row[8]
        for which, printed in ((3, g2), (4, g3)):
            lo, hi = _gamma_range(ratio, angle, which)
            plo, phi = _printed_interval(printed)
            assert lo <= phi and plo <= hi, (name, which, lo, hi, printed)


def test_gamma_pin_rejects_plausible_mistakes():
    # the check above is sharp enough to see the mistakes it is meant to catch:
    # each variant of the definition misses at least one printed value
    variants = {
        "swapped": lambda r, a: (math.sqrt(r - 1) * math.sin(2 * a), math.sqrt(r - 1) * math.cos(2 * a)),
        "angle sign": lambda r, a: (math.sqrt(r - 1) * math.cos(-2 * a), math.sqrt(r - 1) * math.sin(-2 * a)),
        "no factor 2": lambda r, a: (math.sqrt(r - 1) * math.cos(a), math.sqrt(r - 1) * math.sin(a)),
        "ratio not - 1": lambda r, a: (math.sqrt(r) * math.cos(2 * a), math.sqrt(r) * math.sin(2 * a)),
    }
    for label, f in variants.items():
        missed = False
        for name, row in _golden().items():
            ratio, angle, g2, g3 = row[2], row[6], row[7], row[8]
            for idx, printed in ((0, g2), (1, g3)):
                vals = [f(r, a)[idx] for r in np.linspace(*_printed_interval(ratio), 21)
                        for a in np.linspace(*_printed_interval(angle), 21)]
                plo, phi = _printed_interval(printed)
                if not (min(vals) <= phi and plo <= max(vals)):
                    missed = True
        assert missed, label


def test_isotropic_model_is_the_origin():
    for angle in (-2.0, 0.0, 0.7, 3.0):
        w = om.to_internal([[1.7, 2.0, 0.3, 1.0, angle]])[0]
        assert w[3] == 0.0 and w[4] == 0.0
        assert abs(w[0] - 2.0 * math.log(1.7)) < 1e-15


def test_shape_transforms():
    w0 = om.to_internal([[1.0, 4.0, 0.25, 2.0, 0.0]], 0)[0]
    w1 = om.to_internal([[1.0, 4.0, 0.25, 2.0, 0.0]], 1)[0]
    assert abs(w0[1] - math.log(4.0)) < 1e-15 and abs(w1[1] - 0.5) < 1e-15
    assert abs(om.from_internal([[0, 0.25, 0.5, 0, 0]], 1)[0, 1] - 16.0) < 1e-12
    # the angle: (gamma2, gamma3) = sqrt(ratio - 1) (cos 2a, sin 2a)
    w = om.to_internal([[2.0, 1.0, 0.1, 5.0, math.pi / 8]])[0]
    assert abs(w[3] - 2.0 * math.cos(math.pi / 4)) < 1e-14
    assert abs(w[4] - 2.0 * math.sin(math.pi / 4)) < 1e-14


@pytest.mark.parametrize("shape_transform", [0, 1])
def test_round_trip_describes_the_same_covariance(shape_transform):
    # any natural omega, including ratio < 1 and angles outside (-pi/2, pi/2],
    # comes back as a (canonical) omega with the same V -- V from the
    # oracle's independently pinned Matern covariance
    rng = np.random.default_rng(7)
    locs = rng.uniform(0, 4, (25, 2))
    omg = _random_omega(rng, 12)
    back = om.from_internal(om.to_internal(omg, shape_transform), shape_transform)
    assert np.all(back[:, 3] >= 1.0)
    assert np.all((back[:, 4] > -math.pi / 2 - 1e-15) & (back[:, 4] <= math.pi / 2 + 1e-15))
    for a, b in zip(omg, back):
        np.testing.assert_allclose(oracle.build_V(locs, b), oracle.build_V(locs, a),
                                   rtol=1e-10, atol=1e-12)


def test_negative_nu_gives_negative_nugget():
    back = om.from_internal([[0.0, 0.0, -0.3, 0.0, 0.0]])[0]
    assert back[2] == pytest.approx(-0.09, abs=1e-15)


def test_search_coordinates_round_trip():
    rng = np.random.default_rng(8)
    for w in _random_omega(rng, 6):
        w = np.asarray(w)
        b = om.from_search(om.to_search(w))
        a = om.from_internal(om.to_internal(w))[0]
        np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-14)


def test_ascent_check_detects_a_non_maximum():
    # the check used on a Step 1 answer must see an ascent direction at a
    # point far from the maximum (range six times the data's)
    from synth import small_problem
    pr = small_problem(60, p=2, K=1, M=3, seed=3)
    w = pr.omega[0].copy()
    w[0] *= 6.0  # a range far from the data's
    assert om.ascent_around(pr.locs, pr.y, pr.X, w, float(pr.lam[1]), 0.2) > 0.0


def test_library_internal_parameters_match_oracle():
    # host code of the library, no GPU call
    import paper_2305_04318_amd as pl
    rng = np.random.default_rng(9)
    omg = _random_omega(rng, 16)
    for st in (0, 1):
        got = pl.to_internal(omg, st)
        np.testing.assert_allclose(got, om.to_internal(omg, st), rtol=1e-13, atol=1e-14)
        w = om.to_internal(omg, st)
        w[::3, 2] *= -1.0
        np.testing.assert_allclose(pl.from_internal(w, st), om.from_internal(w, st),
                                   rtol=1e-13, atol=1e-14)


def test_library_internal_parameters_reject_bad_input():
    import ctypes
    import paper_2305_04318_amd as pl
    lib = pl.load()
    P = ctypes.c_void_p
    a = np.array([[1.0, 1.0, 0.1, 1.0, 0.0]])
    o = np.empty_like(a)
    assert lib.pl_to_internal(None, 1, 0, o.ctypes.data_as(P)) == -1
    assert lib.pl_to_internal(a.ctypes.data_as(P), 0, 0, o.ctypes.data_as(P)) == -2
    assert lib.pl_to_internal(a.ctypes.data_as(P), 1, 2, o.ctypes.data_as(P)) == -3
    assert lib.pl_to_internal(a.ctypes.data_as(P), 1, 0, None) == -4
    bad = np.array([[1.0, 1.0, -0.1, 1.0, 0.0]])
    assert lib.pl_to_internal(bad.ctypes.data_as(P), 1, 0, o.ctypes.data_as(P)) == -1
    z = np.array([[0.0, 0.0, 0.1, 0.0, 0.0]])
    assert lib.pl_from_internal(z.ctypes.data_as(P), 1, 1, o.ctypes.data_as(P)) == -1
    assert lib.pl_from_internal(z.ctypes.data_as(P), 1, 0, o.ctypes.data_as(P)) == 0
