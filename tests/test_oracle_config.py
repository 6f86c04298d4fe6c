"""Step 2 representative points: the oracle (oracle.config) pinned by closed
forms, textbook chi-square and normal quantiles and the paper's evaluation
counts; the library's host-side parts (pl_config_points, pl_lambda_grid,
pl_chisq_quantile, pl_sphere_points) against it.  No GPU."""
import math

import numpy as np
import pytest

from oracle import config as oc
from oracle import mle as om


# ---------------------------------------------------------------- oracle pins

def test_stencil_sizes_are_the_papers_counts():
    # Section 3.2: 51 x 3 likelihoods for the 5-D Hessian, 33 x 3 for 4-D
    assert oc.stencil(5).shape[0] == 51
    assert oc.stencil(4).shape[0] == 33
    assert len(oc.free_coords(False)) == 5 and len(oc.free_coords(True)) == 4


def test_central_hessian_exact_on_polynomials():
    rng = np.random.default_rng(1)
    d, delta = 5, 0.07
    A = rng.standard_normal((d, d))
    A = A + A.T
    b = rng.standard_normal(d)
    x0 = rng.standard_normal(d)
    f = lambda x: 0.5 * x @ A @ x + b @ x + 3.0
    H = oc.central_hessian([f(x0 + delta * e) for e in oc.stencil(d)], d, delta)
    np.testing.assert_allclose(H, A, rtol=0, atol=1e-9)
    # quartic: the diagonal second difference of x^4 is 12 x^2 + 2 delta^2
    # exactly, and the mixed one of x_i^2 x_j^2 is 4 x_i x_j exactly
    g = lambda x: np.sum(x ** 4) + x[0] ** 2 * x[3] ** 2
    H = oc.central_hessian([g(x0 + delta * e) for e in oc.stencil(d)], d, delta)
    want_diag = 12 * x0 ** 2 + 2 * delta ** 2
    want_diag[0] += 2 * x0[3] ** 2
    want_diag[3] += 2 * x0[0] ** 2
    np.testing.assert_allclose(np.diag(H), want_diag, rtol=1e-8)
    assert abs(H[0, 3] - 4 * x0[0] * x0[3]) < 1e-8
    assert abs(H[1, 2]) < 1e-8


def _internal_by_hand(om_row, shape_transform):
    """The internal parameters written out from the definitions of Section 3.2
    (independent of oracle.mle): gamma1 = log phi_X + log phi_Y, kappa~, nu =
    sqrt(nu^2), gamma2/3 = sqrt(phi_X/phi_Y - 1) (cos, sin)(2 phi_A)."""
    phi_x, kappa, nug, ratio, ang = om_row
    phi_y = phi_x / ratio
    r = math.sqrt(max(ratio - 1.0, 0.0))
    ks = math.log(kappa) if shape_transform == 0 else 1.0 / math.sqrt(kappa)
    return np.array([math.log(phi_x) + math.log(phi_y), ks, math.sqrt(nug),
                     r * math.cos(2 * ang), r * math.sin(2 * ang)])


@pytest.mark.parametrize("fix_shape,shape_transform,nu_hat",
                         [(False, 0, 0.6), (True, 1, 0.6), (False, 1, 0.03)])
def test_hessian_wiring_on_a_known_quadratic(monkeypatch, fix_shape, shape_transform, nu_hat):
    # hessian_at's wiring -- which internal coordinates it perturbs and in
    # which order, the |nu| rule of a stencil point, the held shape and the
    # lambda-hat +- delta columns -- against a likelihood that is an exact
    # quadratic in the internal parameters and lambda (central differences
    # are exact on it).  The quadratic depends on nu only through nu^2, so a
    # stencil point nu - delta < 0 (third case) must give the same value as
    # |nu - delta|: the rule that the point's nugget is (nu - delta)^2.
    rng = np.random.default_rng(11)
    d_all = 5
    A = rng.standard_normal((d_all, d_all))
    A = A @ A.T + d_all * np.eye(d_all)
    A[2, :] = A[:, 2] = 0.0
    A[2, 2] = 3.0                      # nu enters as a nu^2 term only
    omega_hat = np.array([1.3, 2.2, nu_hat ** 2, 2.5, 0.4])
    c = _internal_by_hand(omega_hat, shape_transform) + 0.05 * rng.standard_normal(d_all)
    c[2] = 0.0
    b_lam, lam0, cross = 4.0, 0.3, 0.7
    lam_hat, delta = 0.45, 0.05

    def fake_loglik(locs, y, X, omega, lam):
        omega = np.atleast_2d(omega)
        lam = np.asarray(lam, dtype=np.float64)
        ll = np.empty((omega.shape[0], lam.shape[0]))
        for k, row in enumerate(omega):
            assert row[2] >= 0.0                  # a stencil point never has a negative nugget
            if fix_shape:
                assert row[1] == omega_hat[1]     # the held shape exactly
            w = _internal_by_hand(row, shape_transform) - c
            q = -0.5 * w @ A @ w
            for m, l in enumerate(lam):
                ll[k, m] = q - b_lam * (l - lam0) ** 2 + cross * (l - lam0) * w[0]
        return {"loglik": ll}

    monkeypatch.setattr(oc, "profile_loglik", fake_loglik)
    H, curv, l0, rows = oc.hessian_at(None, None, None, omega_hat, lam_hat, shape_transform,
                                      fix_shape, delta)
    idx = oc.free_coords(fix_shape)
    np.testing.assert_allclose(H, -A[np.ix_(idx, idx)], rtol=0, atol=1e-7 * np.abs(A).max())
    assert abs(curv - (-2.0 * b_lam)) < 1e-7
    w0 = _internal_by_hand(omega_hat, shape_transform) - c
    assert abs(l0 - (-0.5 * w0 @ A @ w0 - b_lam * (lam_hat - lam0) ** 2
                     + cross * (lam_hat - lam0) * w0[0])) < 1e-12
    assert rows.shape[0] == oc.stencil(len(idx)).shape[0]


def test_chisq_quantiles_textbook():
    # printed tables: chi^2_5 upper 5% 11.070, 1% 15.086; chi^2_4 upper 5%
    # 9.488; chi^2_1 upper 5% 3.841 (= 1.95996^2); chi^2_2 upper a = -2 log a
    assert abs(oc.chisq_upper(0.05, 5) - 11.0705) < 1e-4
    assert abs(oc.chisq_upper(0.01, 5) - 15.0863) < 1e-4
    assert abs(oc.chisq_upper(0.05, 4) - 9.4877) < 1e-4
    assert abs(oc.chisq_upper(0.05, 1) - 1.959963984540054 ** 2) < 1e-9
    for a in (1e-5, 0.3, 0.999):
        assert abs(oc.chisq_upper(a, 2) + 2 * math.log(a)) < 1e-10 * max(1, -2 * math.log(a))


def _orth(rng, d):
    q, r = np.linalg.qr(rng.standard_normal((d, d)))
    return q * np.sign(np.diag(r))


def test_repair_rules():
    rng = np.random.default_rng(2)
    Q = _orth(rng, 5)
    # -H with eigenvalues (-3, 0.02, 0.5, 2, 7): abs, no raise (max 7 <= 100)
    ev = np.array([-3.0, 0.02, 0.5, 2.0, 7.0])
    D, E = oc.repair(-(Q @ np.diag(ev) @ Q.T))
    np.testing.assert_allclose(np.sort(D), np.sort(np.abs(ev)), rtol=1e-12)
    # largest above 100: everything below 0.1 raised to 0.1
    ev = np.array([-0.05, 0.001, 0.5, 20.0, 400.0])
    D, E = oc.repair(-(Q @ np.diag(ev) @ Q.T))
    np.testing.assert_allclose(np.sort(D), [0.1, 0.1, 0.5, 20.0, 400.0], rtol=1e-10)
    # E orthonormal, sign convention
    np.testing.assert_allclose(E.T @ E, np.eye(5), atol=1e-12)
    for j in range(5):
        assert E[np.argmax(np.abs(E[:, j])), j] > 0


def test_points_lie_on_the_contour_ellipsoids():
    rng = np.random.default_rng(3)
    Q = _orth(rng, 5)
    ev = np.array([20.0, 35.0, 50.0, 90.0, 140.0])
    H = -(Q @ np.diag(ev) @ Q.T)
    omega_hat = np.array([1.3, 1.1, 0.9, 1.8, 0.4])   # large nugget: nu stays positive
    sph = rng.standard_normal((40, 5))
    sph /= np.linalg.norm(sph, axis=1)[:, None]
    alpha = [0.999, 0.5, 0.01]
    pts, D, nrep = oc.config_points(omega_hat, 0, False, H, alpha, sph, np.zeros(120))
    assert nrep == 0
    w0 = om.to_internal([omega_hat])[0]
    w = om.to_internal(pts)
    for l, a in enumerate(alpha):
        q = oc.chisq_upper(a, 5)
        dw = w[40 * l:40 * (l + 1)] - w0
        np.testing.assert_allclose(np.einsum("ki,ij,kj->k", dw, -H, dw), q, rtol=1e-9)


def test_points_diagonal_closed_form_and_fixed_shape():
    # -H = diag(d): omega'_i - omega_hat'_i = sqrt(q / d_i) x_i
    d = np.array([2.0, 5.0, 0.5, 8.0])
    H = -np.diag(d)
    omega_hat = np.array([2.0, 0.5, 0.6, 1.0, 0.0])
    x = np.array([[0.5, 0.5, 0.5, 0.5], [0, 0, 0, 1.0]])
    pts, D, _ = oc.config_points(omega_hat, 0, True, H, [0.05], x, np.zeros(2))
    q = oc.chisq_upper(0.05, 4)
    w = om.to_internal(pts)
    w0 = om.to_internal([omega_hat])[0]
    free = [0, 2, 3, 4]
    for k in range(2):
        np.testing.assert_allclose(w[k, free] - w0[free], np.sqrt(q / d) * x[k], atol=1e-12)
    assert np.all(pts[:, 1] == 0.5)


def test_nugget_repair_alternates():
    H = -np.eye(5) * 4.0
    omega_hat = np.array([1.0, 1.0, 0.01, 1.0, 0.0])   # nu = 0.1: easily negative
    x = np.zeros((4, 5))
    x[:, 2] = -1.0                                       # every point: nu < 0
    u = np.array([0.1, 0.2, 0.3, 0.4])
    pts, _, nrep = oc.config_points(omega_hat, 0, False, H, [0.5], x, u)
    assert nrep == 4
    np.testing.assert_allclose(pts[:, 2], [0.0, 0.4, 0.0, 0.8])


def test_lambda_grid_normal_quantiles():
    # z_0.99 = 2.326348 (normal tables)
    g = oc.lambda_grid(0.3, -25.0, 30, 0.01)
    assert g.shape == (30,)
    assert abs(g[0] - (0.3 - 2.326348 / 5.0)) < 1e-6
    assert abs(g[-1] - (0.3 + 2.326348 / 5.0)) < 1e-6


# ------------------------------------------- library host code vs the oracle

def test_library_chisq_quantile():
    import paper_2305_04318_amd as pl
    for d in (1, 2, 4, 5, 7, 30):
        for a in (1e-5, 0.001, 0.01, 0.1, 0.25, 0.5, 0.8, 0.95, 0.999, 0.99999):
            want = oc.chisq_upper(a, d)
            assert abs(pl.chisq_quantile(d, a) - want) <= 1e-10 * max(1.0, want), (d, a)


@pytest.mark.parametrize("st,fix", [(0, False), (1, False), (0, True), (1, True)])
def test_library_config_points_match_oracle(st, fix):
    import paper_2305_04318_amd as pl
    rng = np.random.default_rng(10 + 2 * st + fix)
    d = 4 if fix else 5
    Q = _orth(rng, d)
    ev = np.array([-2.0, 0.003, 0.8, 6.0, 300.0])[:d]   # negative, tiny, > 100
    H = -(Q @ np.diag(ev) @ Q.T)
    omega_hat = np.array([1.7, 6.0 if st else 1.2, 0.04, 0.7, 2.5])   # ratio < 1
    sph = rng.standard_normal((50, d))
    sph /= np.linalg.norm(sph, axis=1)[:, None]
    alpha = list(pl.PAPER_ALPHA)
    u = rng.uniform(size=len(alpha) * 50)
    got, geig, gn = pl.config_points(omega_hat, H, alpha, sph, u, st, fix)
    want, weig, wn = oc.config_points(omega_hat, st, fix, H, alpha, sph, u)
    assert gn == wn and gn > 0
    np.testing.assert_allclose(geig, weig, rtol=1e-11)
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-12)


def test_library_lambda_grid_matches_oracle():
    import paper_2305_04318_amd as pl
    for lam, c, m in ((0.5, -40.0, 30), (-0.2, -3.0, 7), (1.0, 12.0, 2)):
        np.testing.assert_allclose(pl.lambda_grid(lam, c, m), oc.lambda_grid(lam, c, m),
                                   rtol=1e-12, atol=1e-12)


def test_library_sphere_points_spread():
    # parity unpinned (the paper's optimiser is unspecified): unit vectors,
    # a closest distance far above random directions', near the best known
    # for 120 points on S^3 (the 600-cell: 2 sin(pi/10) = 0.618)
    import paper_2305_04318_amd as pl
    rng = np.random.default_rng(4)
    init = rng.standard_normal((120, 4))
    pts, md = pl.sphere_points(4, 120, init=init, iters=300)
    np.testing.assert_allclose(np.linalg.norm(pts, axis=1), 1.0, atol=1e-14)
    g = pts @ pts.T
    np.fill_diagonal(g, -2.0)
    assert abs(math.sqrt(2 - 2 * g.max()) - md) < 1e-12
    x0 = init / np.linalg.norm(init, axis=1)[:, None]
    g0 = x0 @ x0.T
    np.fill_diagonal(g0, -2.0)
    assert md > 4.0 * math.sqrt(2 - 2 * g0.max())
    assert md > 0.55
    # zero iterations: the normalised input
    p0, _ = pl.sphere_points(4, 120, init=init, iters=0)
    np.testing.assert_allclose(p0, x0, atol=1e-15)


def test_library_step2_errors():
    import ctypes
    import paper_2305_04318_amd as pl
    lib = pl.load()
    P = ctypes.c_void_p
    q = ctypes.c_double()
    assert lib.pl_chisq_quantile(0, 0.5, ctypes.byref(q)) == -1
    assert lib.pl_chisq_quantile(3, 1.0, ctypes.byref(q)) == -2
    assert lib.pl_chisq_quantile(3, 0.5, None) == -3
    out = np.empty(4)
    assert lib.pl_lambda_grid(0.0, 0.0, 0.01, 4, out.ctypes.data_as(P)) == -2
    assert lib.pl_lambda_grid(0.0, -1.0, 0.5, 4, out.ctypes.data_as(P)) == -3
    assert lib.pl_lambda_grid(0.0, -1.0, 0.01, 1, out.ctypes.data_as(P)) == -4
    z = np.zeros((3, 2))
    o = np.empty((3, 2))
    assert lib.pl_sphere_points(2, 3, z.ctypes.data_as(P), 1, o.ctypes.data_as(P), None) == -3
    # a flat Hessian direction cannot be mapped
    H = -np.diag([1.0, 1.0, 0.0, 1.0, 1.0])
    with pytest.raises(pl.PlError):
        pl.config_points([1, 1, 0.1, 1, 0], H, [0.5], np.eye(5), np.zeros(5))
