// Kernels of the noise correction (corrected.hpp).
#include "corrected.hpp"
#include "kcommon.hpp"

namespace symtd {

namespace {
__device__ double csum(double v, double* sm) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sm[w] = v;
  __syncthreads();
  return (sm[0] + sm[1]) + (sm[2] + sm[3]);
}
}  // namespace

// one block (256 threads) per column J of all models
template <typename T>
__global__ __launch_bounds__(256) void k_corr_cols(Correction c, const T* A, int64_t lda, int n, int r,
                                                   const double* lambda, double* g_lambda, T* G, int64_t ldg,
                                                   double* lc) {
  __shared__ double sm[4];
  __shared__ double sa[CORR_NMAX];
  const int64_t J = blockIdx.x;
  const T* a = A + J * lda;
  const double s2 = c.sigma * c.sigma;
  double t = 0.0, u = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double ai = (double)a[i];
    t = fma(ai, ai, t);
    if (c.d == 3) u = fma(c.m[i], ai, u);
  }
  t = csum(t, sm);
  double full, q = 0.0;
  if (c.d == 3) {
    u = csum(u, sm);
    full = 3.0 * s2 * u * t;
  } else {
    // S a with S = M2 - sigma^2 I, kept in LDS
    for (int i = threadIdx.x; i < n; i += 256) {
      double v = 0.0;
      for (int k = 0; k < n; ++k) v = fma(c.M2[(int64_t)k * n + i], (double)a[k], v);
      const double ai = (double)a[i];
      sa[i] = v - s2 * ai;
      q = fma(ai, sa[i], q);
    }
    q = csum(q, sm);
    full = 6.0 * s2 * q * t + 3.0 * s2 * s2 * t * t;
  }
  const double lj = lambda[J];
  const double scale = 2.0 * c.d * lj;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double ai = (double)a[i];
    const double part = c.d == 3 ? s2 * (t * c.m[i] + 2.0 * u * ai)
                                 : 3.0 * s2 * (t * sa[i] + q * ai) + 3.0 * s2 * s2 * t * ai;
    T* gp = G + J * ldg + i;
    *gp = (T)((double)*gp + scale * part);
  }
  if (threadIdx.x == 0) {
    g_lambda[J] += 2.0 * full;
    lc[J] = lj * full;
  }
}

// one block per model: f += 2 sum_j lambda_j Delta a_j^d, in column order
__global__ __launch_bounds__(256) void k_corr_f(int r, const double* lc, double* f) {
  __shared__ double sm[4];
  double s = 0.0;
  for (int j = threadIdx.x; j < r; j += 256) s += lc[(int64_t)blockIdx.x * r + j];
  s = csum(s, sm);
  if (threadIdx.x == 0) f[blockIdx.x] += 2.0 * s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_corr_xdot(Correction c, const T* V, int64_t ldv, const double* nu, int n,
                                                   int64_t p, double* part) {
  __shared__ double sm[4];
  const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double s2 = c.sigma * c.sigma;
  double val = 0.0;
  if (l < p) {
    const T* v = V + l * ldv;
    double t = 0.0, u = 0.0;
    for (int i = 0; i < n; ++i) {
      const double vi = (double)v[i];
      t = fma(vi, vi, t);
      if (c.d == 3) u = fma(c.m[i], vi, u);
    }
    if (c.d == 3) {
      val = 3.0 * s2 * u * t;
    } else {
      double q = 0.0;
      for (int i = 0; i < n; ++i) {
        double w = 0.0;
        for (int k = 0; k < n; ++k) w = fma(c.M2[(int64_t)k * n + i], (double)v[k], w);
        q = fma((double)v[i], w, q);
      }
      q -= s2 * t;
      val = 6.0 * s2 * q * t + 3.0 * s2 * s2 * t * t;
    }
    val *= nu[l];
  }
  val = csum(val, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = val;
}

template <typename T>
void launch_correction(hipStream_t st, const Correction& c, const T* A, int64_t lda, int n, int r, int models,
                       const double* lambda, double* f, double* g_lambda, T* G, int64_t ldg, double* lc) {
  hipLaunchKernelGGL(k_corr_cols<T>, dim3((unsigned)((int64_t)r * models)), dim3(256), 0, st, c, A, lda, n, r,
                     lambda, g_lambda, G, ldg, lc);
  hipLaunchKernelGGL(k_corr_f, dim3((unsigned)models), dim3(256), 0, st, r, lc, f);
}

template <typename T>
void launch_corr_xdot(hipStream_t st, const Correction& c, const T* V, int64_t ldv, const double* nu, int n,
                      int64_t p, double* part) {
  hipLaunchKernelGGL(k_corr_xdot<T>, dim3((unsigned)((p + 255) / 256)), dim3(256), 0, st, c, V, ldv, nu, n, p, part);
}

double corr_delta_norm2(const double* m, const double* M2, int64_t n, double sigma, int d) {
  const double s2 = sigma * sigma;
  if (d == 3) {
    double mm = 0.0;
    for (int64_t i = 0; i < n; ++i) mm += m[i] * m[i];
    return s2 * s2 * mm * (3.0 * n + 6.0);
  }
  double fro = 0.0, tr = 0.0;
  for (int64_t k = 0; k < n; ++k)
    for (int64_t i = 0; i < n; ++i) {
      const double sv = M2[k * n + i] - (i == k ? s2 : 0.0);
      fro += sv * sv;
      if (i == k) tr += sv;
    }
  const double nn = (double)n;
  return s2 * s2 * (6.0 * (nn + 4.0) * fro + 6.0 * tr * tr) + 12.0 * s2 * s2 * s2 * (nn + 2.0) * tr +
         s2 * s2 * s2 * s2 * (3.0 * nn * nn + 6.0 * nn);
}

template void launch_correction<float>(hipStream_t, const Correction&, const float*, int64_t, int, int, int,
                                       const double*, double*, double*, float*, int64_t, double*);
template void launch_correction<double>(hipStream_t, const Correction&, const double*, int64_t, int, int, int,
                                        const double*, double*, double*, double*, int64_t, double*);
template void launch_corr_xdot<float>(hipStream_t, const Correction&, const float*, int64_t, const double*, int,
                                      int64_t, double*);
template void launch_corr_xdot<double>(hipStream_t, const Correction&, const double*, int64_t, const double*, int,
                                       int64_t, double*);

}  // namespace symtd
