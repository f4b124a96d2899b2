// Kernels of the explicit route (explicit.hpp).
#include "explicit.hpp"
#include "kcommon.hpp"

namespace symtd {

namespace {
constexpr int MT_TILE = 64, MT_LC = 16;
}

template <typename T>
__global__ __launch_bounds__(256) void k_moment(MomentArgs<T> a) {
  __shared__ double sv[MT_LC][MT_TILE + 1];
  __shared__ double sk[MT_LC][MT_TILE + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * MT_TILE;
  const int64_t c0 = (int64_t)blockIdx.y * MT_TILE;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int64_t l0 = 0; l0 < a.p; l0 += MT_LC) {
#pragma unroll
    for (int q = 0; q < MT_LC * MT_TILE / 256; ++q) {
      const int e = tid + 256 * q;
      const int l = e / MT_TILE, k = e % MT_TILE;
      const int64_t ll = l0 + l;
      const int64_t i = i0 + k, c = c0 + k;
      double x = 0.0, w = 0.0;
      if (ll < a.p) {
        if (i < a.n) x = (double)a.V[ll * a.ldv + i];
        if (c < a.cols) {
          // nu_l times the entries of v_l at the digits of c (base n)
          w = a.nu[ll];
          int64_t cc = c;
          for (int t = 1; t < a.d; ++t) {
            w *= (double)a.V[ll * a.ldv + cc % a.n];
            cc /= a.n;
          }
        }
      }
      sv[l][k] = x;
      sk[l][k] = w;
    }
    __syncthreads();
#pragma unroll
    for (int l = 0; l < MT_LC; ++l) {
      double xv[4], wv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = sv[l][4 * ty + u];
#pragma unroll
      for (int v = 0; v < 4; ++v) wv[v] = sk[l][4 * tx + v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(xv[u], wv[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + 4 * ty + u, c = c0 + 4 * tx + v;
      if (i < a.n && c < a.cols) {
        if (a.X64) a.X64[c * a.n + i] = acc[u][v];
        else a.X[c * a.n + i] = (T)acc[u][v];
      }
    }
}

// element (l, j) of the first product's packed W (kernels.hpp): l = 16 b +
// row(g, s), j = 16 t + c at ((b nt + t) 64 + 16 g + c) 4 + s
template <typename T>
__device__ __forceinline__ int64_t packed_at(int64_t l, int j, int nt) {
  const int64_t b = l >> 4;
  const int rr = (int)(l & 15);
  const int g = sizeof(T) == 8 ? (rr & 3) : (rr >> 2);
  const int s = sizeof(T) == 8 ? (rr >> 2) : (rr & 3);
  return ((b * nt + (j >> 4)) * 64 + 16 * g + (j & 15)) * 4 + s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_ttsv_tail(TtsvTailArgs<T> a) {
  __shared__ double sm[4];
  const int i = blockIdx.x % a.n, j = blockIdx.x / a.n;
  const T* aj = a.A + (int64_t)j * a.lda;
  double y = 0.0;
  for (int64_t m = threadIdx.x; m < a.m2; m += 256) {
    double w = 1.0;
    int64_t mm = m;
    for (int t = 2; t < a.d; ++t) {
      w *= (double)aj[mm % a.n];
      mm /= a.n;
    }
    y = fma((double)a.Wp[packed_at<T>(m + a.m2 * i, j, a.nt_tot)], w, y);
  }
  // fixed-order block reduction
  for (int o = 32; o > 0; o >>= 1) y += __shfl_down(y, o);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = y;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double yy = (sm[0] + sm[1]) + (sm[2] + sm[3]);
    a.Y[(int64_t)j * a.npad + i] = (T)yy;
    a.wterm[(int64_t)i * a.rp + j] = (double)aj[i] * yy;
  }
}

__global__ void k_fill(double* x, int64_t count, double v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) x[e] = v;
}

template <typename T>
void launch_moment(hipStream_t st, const MomentArgs<T>& a) {
  const dim3 grid((unsigned)((a.n + MT_TILE - 1) / MT_TILE), (unsigned)((a.cols + MT_TILE - 1) / MT_TILE));
  hipLaunchKernelGGL(k_moment<T>, grid, dim3(256), 0, st, a);
}
template <typename T>
void launch_ttsv_tail(hipStream_t st, const TtsvTailArgs<T>& a) {
  hipLaunchKernelGGL(k_ttsv_tail<T>, dim3((unsigned)((int64_t)a.n * a.r)), dim3(256), 0, st, a);
}
void launch_fill(hipStream_t st, double* x, int64_t count, double v) {
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, x, count, v);
}

template void launch_moment<float>(hipStream_t, const MomentArgs<float>&);
template void launch_moment<double>(hipStream_t, const MomentArgs<double>&);
template void launch_ttsv_tail<float>(hipStream_t, const TtsvTailArgs<float>&);
template void launch_ttsv_tail<double>(hipStream_t, const TtsvTailArgs<double>&);

}  // namespace symtd
