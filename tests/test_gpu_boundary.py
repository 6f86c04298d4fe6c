"""The stand-alone covariance build and Cholesky in both storage types,
through the C ABI (Section 3.3, Step 3 sub-steps 1-2; the paper makes the
precision a per-call choice).

* pl_matern_cov with PL_F32: every element is the FP64 value rounded once, so
  |V32 - V| <= 2^-24 |V| + the FP64 build's own error (1e-12) against the
  oracle's V; the strict upper triangle is left untouched.
* pl_chol_batched with PL_MIXED on that FP32 V: FP32 factor with FP64
  diagonal tiles and log-determinant.  Bars derived from the arithmetic:
  - backward error: ||L L^T - V||_F <= 2 (n + 1) u ||L||_F^2 with u = 2^-24
    (the componentwise Cholesky bound gamma_{n+1} |L| |L^T|, doubled for the
    rounding of the stored FP32 factor; ||L||_F^2 = trace(V));
  - log-determinant, to first order in that perturbation:
    |logdet - log|V|| <= ||V^-1||_F ||L L^T - V||_F + 2 n u
    (|tr(V^-1 dV)| bounded by Cauchy-Schwarz; 2 n u for the FP32 rounding of
    the diagonal entries that the FP64 sum does not see).
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _lower(Vt, n):
    """(K, n, ld) column-major tensor -> (K, n, n) numpy matrices."""
    return np.transpose(Vt.cpu().double().numpy()[:, :n, :n], (0, 2, 1))


@pytest.mark.parametrize("n,ld", [(7, 8), (261, 264), (300, 300)])
def test_matern_cov_f32_elementwise(plprof_lib, n, ld):
    pl = plprof_lib
    pr = synth.small_problem(n, p=2, K=6, M=1, seed=200 + n,
                             kappas=[0.05, 0.5, 1.0, 2.37, 4.5, 9.8])
    V = pl.matern_cov(pr.locs, pr.omega, dtype="f32", ld=ld)
    torch.cuda.synchronize()
    assert V.dtype == torch.float32
    Vg = _lower(V, n)
    lo = np.tril_indices(n)
    up = np.triu_indices(n, 1)
    for k in range(pr.K):
        ref = oracle.build_V(pr.locs, pr.omega[k])
        err = np.abs(Vg[k][lo] - ref[lo])
        assert np.all(err <= U32 * np.abs(ref[lo]) + 1e-12), (k, err.max())
        assert np.all(Vg[k][up] == 0.0)          # never written
    # the FP32 values are exactly the FP64 build rounded once
    V64 = pl.matern_cov(pr.locs, pr.omega, dtype="f64", ld=ld)
    torch.cuda.synchronize()
    V64r = _lower(V64.float(), n)
    for k in range(pr.K):
        np.testing.assert_array_equal(Vg[k][lo], V64r[k][lo])


@pytest.mark.parametrize("n,ld", [(128, 128), (300, 300), (461, 464)])
def test_chol_mixed_against_lapack(plprof_lib, n, ld):
    pl = plprof_lib
    pr = synth.small_problem(n, p=2, K=4, M=1, seed=300 + n, kappas=[0.5, 1.0, 2.5, 6.0])
    V = pl.matern_cov(pr.locs, pr.omega, dtype="f32", ld=ld)
    torch.cuda.synchronize()
    V0 = _lower(V, n)
    logdet, info = pl.chol_batched(V)
    torch.cuda.synchronize()
    L = np.tril(_lower(V, n))
    assert np.all(info.cpu().numpy() == 0)
    ld_gpu = logdet.cpu().numpy()
    for k in range(pr.K):
        Vk = np.tril(V0[k]) + np.tril(V0[k], -1).T     # the FP32 matrix, exactly, in FP64
        Lr = np.linalg.cholesky(Vk)
        logdet_ref = 2.0 * np.sum(np.log(np.diag(Lr)))
        R = L[k] @ L[k].T - Vk
        bw = np.linalg.norm(R)
        bound_bw = 2 * (n + 1) * U32 * np.linalg.norm(L[k]) ** 2
        assert bw <= bound_bw, (k, bw, bound_bw)
        bound_ld = np.linalg.norm(np.linalg.inv(Vk)) * bw + 2 * n * U32
        assert abs(ld_gpu[k] - logdet_ref) <= bound_ld, (k, ld_gpu[k] - logdet_ref, bound_ld)


def test_chol_fp64_and_mixed_agree_on_the_same_matrix(plprof_lib):
    """FP64 and mixed factorisations of the same FP32-representable V: the
    FP64 factor and log-determinant match LAPACK to 1e-11 and 1e-10 n, the
    mixed log-determinant agrees to 1e-3 n."""
    pl = plprof_lib
    n = 390
    pr = synth.small_problem(n, p=2, K=3, M=1, seed=77, kappas=[0.8, 1.5, 3.0])
    V32 = pl.matern_cov(pr.locs, pr.omega, dtype="f32", ld=392)   # PL_MIXED: ld % 4 == 0
    V64 = V32.double()
    torch.cuda.synchronize()
    ld64, i64 = pl.chol_batched(V64)
    ld32, i32 = pl.chol_batched(V32)
    torch.cuda.synchronize()
    assert np.all(i64.cpu().numpy() == 0) and np.all(i32.cpu().numpy() == 0)
    L64 = _lower(V64, n)  # V64 now holds the FP64 factor
    V0 = _lower(pl.matern_cov(pr.locs, pr.omega, dtype="f32", ld=392), n)
    for k in range(pr.K):
        Vk = np.tril(V0[k]) + np.tril(V0[k], -1).T
        ref = 2.0 * np.sum(np.log(np.diag(np.linalg.cholesky(Vk))))
        assert abs(ld64[k].item() - ref) <= 1e-10 * n
        assert np.allclose(np.tril(L64[k]), np.linalg.cholesky(Vk), rtol=0, atol=1e-11)
        assert abs(ld32[k].item() - ref) <= 1e-3 * n
