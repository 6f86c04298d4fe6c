// The p x p stage of Step 3 (Steps 5-8 of Section 3.3): cross products to
// beta-hat, sigma-hat^2 and the profile log-likelihood (equations "betahat",
// (4), "profile"; Appendix "remlpro").
#pragma once

#include <math.h>

#include "common.h"

namespace plk {

constexpr int FIN_SMEM_DOUBLES = PL_MAX_P * PL_MAX_P + PL_MAX_M * PL_MAX_P + 2;

// S holds minus the cross products (column-major, leading dimension TB): the
// Schur tile of the bordered factorisation, or its mixed-form equivalent.
//   A = X^T V^-1 X = Q Q^T           (Step 5; log|X^T V^-1 X| = 2 sum log Q_ii)
//   c_m = Q^-1 X^T V^-1 y'_m          (Step 6)
//   ssqBetahat_m = c_m^T c_m          (Step 7)
//   ssqResidual_m = ssqY_m - ssqBetahat_m (Step 8); beta-hat = Q^-T c_m.
//   (X^T V^-1 X)^-1 = Q^-T Q^-1     (the sampling covariance of beta-hat up to
//                                    sigma^2; the profile of a single
//                                    coefficient follows from its diagonal)
// All threads of the workgroup take part; records go to out[0..M), beta-hat
// (if not NULL) to beta[0..M*p), (X^T V^-1 X)^-1 (if not NULL, row-major p x p,
// NaN when it does not exist) to xvi[0..p*p).
__device__ __forceinline__ void dev_finalize(const double* S, int TB, double ldv, int inf,
                                             double J, bool bady, const double* __restrict__ lam,
                                             int n, int p, int M, pl_result* __restrict__ out,
                                             double* __restrict__ beta, double* __restrict__ xvi,
                                             double* smem) {
  double* Q = smem;
  double* cm = smem + PL_MAX_P * PL_MAX_P;
  double* shared_ldx = cm + PL_MAX_M * PL_MAX_P;
  int* rank_bad = reinterpret_cast<int*>(shared_ldx + 1);
  const int tid = threadIdx.x, nt = blockDim.x;
  const double LOG2PI = 1.8378770664093454836;
  if (!bady && inf == 0) {
    for (int idx = tid; idx < p * p; idx += nt) {
      const int i = idx / p, j = idx % p;
      const int a = M + (i > j ? i : j), b = M + (i > j ? j : i);
      Q[i * PL_MAX_P + j] = -S[(int64_t)b * TB + a];
    }
    __syncthreads();
    if (tid == 0) {
      // Cholesky of the p x p matrix (row-major, lower used)
      int bad = 0;
      double sl = 0.0;
      for (int j = 0; j < p && !bad; ++j) {
        double d = Q[j * PL_MAX_P + j];
        for (int m = 0; m < j; ++m) d -= Q[j * PL_MAX_P + m] * Q[j * PL_MAX_P + m];
        if (!(d > 0.0)) { bad = 1; break; }
        const double l = sqrt(d);
        Q[j * PL_MAX_P + j] = l;
        sl += log(l);
        for (int i = j + 1; i < p; ++i) {
          double v = Q[i * PL_MAX_P + j];
          for (int m = 0; m < j; ++m) v -= Q[i * PL_MAX_P + m] * Q[j * PL_MAX_P + m];
          Q[i * PL_MAX_P + j] = v / l;
        }
      }
      *rank_bad = bad;
      *shared_ldx = 2.0 * sl;
    }
    __syncthreads();
  } else {
    if (tid == 0) { *rank_bad = 0; *shared_ldx = NAN; }
    __syncthreads();
  }
  const double ldx = *shared_ldx;
  const int rbad = *rank_bad;
  if (xvi) {
    // Q^-1 by forward substitution, one column per thread, in the c buffer
    // (free until the record loop below)
    double* Qi = cm;
    const bool ok = !bady && inf == 0 && !rbad;
    if (ok) {
      for (int j = tid; j < p; j += nt) {
        for (int i = 0; i < p; ++i) {
          double v = 0.0;
          if (i >= j) {
            v = (i == j) ? 1.0 : 0.0;
            for (int k = j; k < i; ++k) v -= Q[i * PL_MAX_P + k] * Qi[k * PL_MAX_P + j];
            v /= Q[i * PL_MAX_P + i];
          }
          Qi[i * PL_MAX_P + j] = v;
        }
      }
      __syncthreads();
    }
    for (int idx = tid; idx < p * p; idx += nt) {
      const int i = idx / p, j = idx % p;
      double v = NAN;
      if (ok) {
        v = 0.0;
        for (int k = (i > j ? i : j); k < p; ++k) v += Qi[k * PL_MAX_P + i] * Qi[k * PL_MAX_P + j];
      }
      xvi[idx] = v;
    }
    __syncthreads();
  }
  for (int m = tid; m < M; m += nt) {
    pl_result rec;
    rec.jacobian = J;
    rec.pad = 0;
    rec.logdet_v = ldv;
    rec.logdet_xvx = ldx;
    const double lm = lam[m];
    if (bady) {
      rec.loglik = NAN; rec.loglik_reml = NAN; rec.info = PL_INFO_BAD_Y;
      rec.logdet_v = NAN; rec.logdet_xvx = NAN;
      rec.ssq_y = rec.ssq_betahat = rec.ssq_resid = rec.sigma2_hat = NAN;
    } else if (inf != 0) {
      rec.loglik = -INFINITY; rec.loglik_reml = -INFINITY; rec.info = inf;
      rec.logdet_v = NAN;
      rec.ssq_y = rec.ssq_betahat = rec.ssq_resid = rec.sigma2_hat = NAN;
    } else if (rbad) {
      rec.loglik = NAN; rec.loglik_reml = NAN; rec.info = PL_INFO_RANK;
      rec.ssq_y = -S[(int64_t)m * TB + m];
      rec.ssq_betahat = rec.ssq_resid = rec.sigma2_hat = NAN;
    } else {
      double* c = cm + m * PL_MAX_P;
      // c = Q^-1 B_m, B_m[i] = ssq(M+i, m) = -S[m*TB + M+i]
      double ssb = 0.0;
      for (int i = 0; i < p; ++i) {
        double v = -S[(int64_t)m * TB + M + i];
        for (int j = 0; j < i; ++j) v -= Q[i * PL_MAX_P + j] * c[j];
        v /= Q[i * PL_MAX_P + i];
        c[i] = v;
        ssb += v * v;
      }
      const double ssy = -S[(int64_t)m * TB + m];
      const double ssr = ssy - ssb;
      const double s2 = ssr / n;
      rec.ssq_y = ssy;
      rec.ssq_betahat = ssb;
      rec.ssq_resid = ssr;
      rec.sigma2_hat = s2;
      rec.info = 0;
      rec.loglik = -0.5 * (n * log(s2) + ldv + n * LOG2PI + n) + (lm - 1.0) * J;
      rec.loglik_reml = -0.5 * ((n - p) * log(ssr / (n - p)) + ldv + ldx + n * LOG2PI + n - p) +
                        (lm - 1.0) * J;
      if (beta) {
        // beta-hat = Q^-T c (back substitution), written in place of c
        double* bo = beta + (int64_t)m * p;
        for (int i = p - 1; i >= 0; --i) {
          double v = c[i];
          for (int j = i + 1; j < p; ++j) v -= Q[j * PL_MAX_P + i] * c[j];
          v /= Q[i * PL_MAX_P + i];
          c[i] = v;
        }
        for (int i = 0; i < p; ++i) bo[i] = c[i];
      }
    }
    if (beta && rec.info != 0) {
      double* bo = beta + (int64_t)m * p;
      for (int i = 0; i < p; ++i) bo[i] = NAN;
    }
    out[m] = rec;
  }
}

}  // namespace plk
