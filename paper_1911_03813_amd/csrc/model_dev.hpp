// Device parts of the model terms shared by the evaluation paths (fp32 / fp64
// products and the 16-bit products): the Gram matrix B = A'A of the factors
// and C = B^(d-1) (elementwise power), which enter f, g_lambda and G_A through
// the model's own inner products (Algorithm 2 and the gradient of Section 4).
#pragma once

#include "kcommon.hpp"
#include "kernels.hpp"

namespace symtd {

// Rows of A staged in LDS at a time by a Gram-tile block, and the padded
// column stride of the staged panels (in doubles; the pad spreads the 16
// columns of a fragment read over the LDS banks).
constexpr int GRAM_ROWS = 512;
constexpr int GRAM_LD = GRAM_ROWS + 4;
// LDS of a Gram-tile block: the two staged 16-column panels (the wave tiles'
// reduction reuses it).
constexpr int GRAM_LDS_DOUBLES = 2 * 16 * GRAM_LD;

// Gram tile t = (grp rt + kt) rt + jt of model grp: for kt >= jt, the 16 x 16
// tile B[j0 + j][k0 + k] = sum_i A[i][j0 + j] A[i][k0 + k] (j0 = 16 jt,
// k0 = 16 kt) over all n rows, in fp64; blocks with kt < jt return at once
// (their tile is the mirror of (kt, jt), written by that block).
//
// The two 16-column panels of A move to LDS GRAM_ROWS rows at a time with
// coalesced loads (consecutive threads, consecutive rows of one column).
// Wave w then takes the 4-row groups q = w, w + 16, ... of the staged rows and
// accumulates them on the fp64 matrix core (16x16x4): lane 16 g + c supplies
// A[4q + g][j0 + c] as the first operand and A[4q + g][k0 + c] as the second,
// so the product's row is j and its column k.  The 16 wave tiles are summed
// in wave order through LDS.  Writes B and C (and their mirrored tile).
template <typename T>
__device__ __forceinline__ void gram_tile(const GramArgs<T>& a, int64_t t, double* lds) {
  const int rt = a.rt;
  const int jt = (int)(t % rt), kt = (int)((t / rt) % rt);
  const int grp = (int)(t / ((int64_t)rt * rt));
  if (kt < jt) return;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int g = lane >> 4, c = lane & 15;
  const int j0 = jt * 16, k0 = kt * 16;
  const T* Ag = a.A + (int64_t)grp * a.r * a.lda;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i0 = 0; i0 < a.n; i0 += GRAM_ROWS) {
    // panel p (0: columns j0.., 1: columns k0..), column cc, row ii; all of
    // a thread's loads are issued before any is used
    constexpr int IT = 2 * 16 * GRAM_ROWS / GRAM_THREADS;
    T x[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = threadIdx.x + it * GRAM_THREADS;
      const int ii = e % GRAM_ROWS, cc = (e / GRAM_ROWS) % 16, pnl = e / (16 * GRAM_ROWS);
      const int col = (pnl ? k0 : j0) + cc;
      const int64_t i = i0 + ii;
      x[it] = Ag[(int64_t)(col < a.r ? col : 0) * a.lda + (i < a.n ? i : 0)];
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = threadIdx.x + it * GRAM_THREADS;
      const int ii = e % GRAM_ROWS, cc = (e / GRAM_ROWS) % 16, pnl = e / (16 * GRAM_ROWS);
      const int col = (pnl ? k0 : j0) + cc;
      const bool ok = i0 + ii < a.n && col < a.r;
      lds[(pnl * 16 + cc) * GRAM_LD + ii] = ok ? (double)x[it] : 0.0;
    }
    __syncthreads();
    const int nq = (int)((min((int64_t)GRAM_ROWS, a.n - i0) + 3) / 4);
    for (int q = w; q < nq; q += GRAM_THREADS / 64) {
      const double xa = lds[c * GRAM_LD + 4 * q + g];
      const double xb = lds[(16 + c) * GRAM_LD + 4 * q + g];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa, xb, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // acc[v] = this wave's D[g + 4 v][c]; the staging buffer now holds the
  // 16 wave tiles
#pragma unroll
  for (int v = 0; v < 4; ++v) lds[w * 256 + (g + 4 * v) * 16 + c] = acc[v];
  __syncthreads();
  if (threadIdx.x < 256) {
    const int e = threadIdx.x, j = e >> 4, k = e & 15;
    double s = 0.0;
    for (int ww = 0; ww < GRAM_THREADS / 64; ++ww) s += lds[ww * 256 + e];
    if (j0 + j < a.r && k0 + k < a.r) {
      const int64_t rr = (int64_t)a.r * a.r;
      double* Bg = a.B + grp * rr;
      double* Cg = a.C + grp * rr;
      const double cv = ipow(s, a.d - 1);
      Bg[(int64_t)(k0 + k) * a.r + j0 + j] = s;
      Cg[(int64_t)(k0 + k) * a.r + j0 + j] = cv;
      if (kt > jt) {
        Bg[(int64_t)(j0 + j) * a.r + k0 + k] = s;
        Cg[(int64_t)(j0 + j) * a.r + k0 + k] = cv;
      }
    }
  }
}

}  // namespace symtd
