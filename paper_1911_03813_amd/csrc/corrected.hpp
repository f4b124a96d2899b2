// Moments corrected for spherical Gaussian noise of known level sigma (the
// lower-order terms of Section 4.2; the paper leaves them to future work).
//
// With m = sum_l nu_l v_l, M2 = sum_l nu_l v_l v_l' and S = M2 - sigma^2 I,
// the noise adds to the d-th moment the tensor (Isserlis' theorem)
//   d = 3:  Delta = sigma^2 sym3(m (x) I)
//   d = 4:  Delta = sigma^2 sym6(S (x) I) + sigma^4 sym3(I (x) I)
// (symK: the K placements of the factors over the index positions).  The
// corrected objective ||X - Delta - M||^2 = f + 2 sum_j lambda_j Delta a_j^d +
// constant needs, per column a (t = a'a):
//   d = 3:  Delta a^3 = 3 sigma^2 (m'a) t,   Delta a^2 = sigma^2 (t m + 2 (m'a) a)
//   d = 4:  Delta a^4 = 6 sigma^2 (a'Sa) t + 3 sigma^4 t^2,
//           Delta a^3 = 3 sigma^2 (t S a + (a'Sa) a) + 3 sigma^4 t a
// and the constant term of alpha_c = ||X - Delta||^2 = ||X||^2 -
// 2 sum_l nu_l Delta v_l^d + ||Delta||^2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace symtd {

constexpr int CORR_NMAX = 4096;   // covariates supported by the correction kernels (LDS vector)

struct Correction {
  const double* m;     // n
  const double* M2;    // n x n (d = 4), column-major
  double sigma;
  int d;
};

// after an evaluation of `models` models of r columns (A, lambda, g_lambda,
// G as in symtd_fg_multi, f one value per model): add the correction terms;
// lc holds models * r fp64 values of scratch
template <typename T>
void launch_correction(hipStream_t st, const Correction& c, const T* A, int64_t lda, int n, int r, int models,
                       const double* lambda, double* f, double* g_lambda, T* G, int64_t ldg, double* lc);

// part[b] = sum over the observations of block b of nu_l Delta v_l^d
// (256 observations per block); blocks = ceil(p / 256)
template <typename T>
void launch_corr_xdot(hipStream_t st, const Correction& c, const T* V, int64_t ldv, const double* nu, int n,
                      int64_t p, double* part);

// ||Delta||^2 in closed form from the host copies of m and M2
double corr_delta_norm2(const double* m, const double* M2, int64_t n, double sigma, int d);

}  // namespace symtd
