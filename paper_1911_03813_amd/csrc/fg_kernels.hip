// Kernels of the objective/gradient evaluation (Algorithm 2, fg_implicit).
//
//   gemm1   Z = V'A on matrix cores, one 16-row slab of observations per
//           M subtile.  Epilogue: W = D_nu Z^{d-1} (eq. (Y) before the outer
//           product), written in a packed layout that the second product
//           reads with one coalesced vector load per lane, and fp64 partial
//           column sums of nu_l z_lj^d (= w_j by Lemmas 3.2 and 3.5).
//   gemm2   Y = V W on matrix cores, split over the observations (split-K);
//           each split writes its own partial Y, so no atomics are used.
//   gram    B = A'A and C = B^{d-1} in fp64.
//   final_G   Y = fixed-order fp64 sum of the partials; G_A = -2d (Y - A D_lambda C) D_lambda.
//   final_s   w = fixed-order fp64 sum of the column partials; u = (B*C) lambda;
//             f = alpha + lambda'u - 2 w'lambda; g_lambda = -2 (w - u).
//
// Packed W layout: element (l, j) with l = 16*b + row(g, s) and j = 16*t + c
// lives at ((b * nt_tot + t) * 64 + 16*g + c) * 4 + s, where row(g, s) is the
// MFMA output row of lane group g, element s (Mfma<T>::row).  That is exactly
// the order in which gemm1's accumulator registers come out, and exactly the
// B-operand order gemm2 needs when its k index at step s is
// l = 16*b + row(g, s).
#include "kcommon.hpp"
#include "kernels.hpp"

namespace symtd {

// ---------------------------------------------------------------------------
// gemm1 + epilogue
// ---------------------------------------------------------------------------
template <typename T, int MT, int NT, bool VEC>
__global__ __launch_bounds__(256) void k_gemm1(G1Args<T> a) {
  using acc_t = typename Mfma<T>::acc_t;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * MT);

  const T* vp[MT];
  bool vok[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int64_t l = row0 + 16 * m + c;
    vok[m] = l < a.p;
    vp[m] = a.V + (vok[m] ? l : 0) * a.ldv;
  }
  const T* ap[NT];
  bool aok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = a.col0 + 16 * t + c;
    aok[t] = j < a.r;
    ap[t] = a.A + (int64_t)(aok[t] ? j : 0) * a.lda;
  }

  acc_t acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = acc_t{0, 0, 0, 0};

  Quad<T> va0[MT], aa0[NT], va1[MT], aa1[NT];
  const int64_t n = a.n;
  const int64_t nfull = n & ~(int64_t)15;

  auto load = [&](Quad<T>(&va)[MT], Quad<T>(&aa)[NT], int64_t i0) {
    const int64_t i = i0 + 4 * g;
#pragma unroll
    for (int m = 0; m < MT; ++m) load4<T, VEC>(va[m], vp[m], i, n, vok[m]);
#pragma unroll
    for (int t = 0; t < NT; ++t) load4<T, VEC>(aa[t], ap[t], i, n, aok[t]);
  };
  auto mma = [&](const Quad<T>(&va)[MT], const Quad<T>(&aa)[NT]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = Mfma<T>::mac(va[m].e[s], aa[t].e[s], acc[m][t]);
  };

  if (nfull > 0) {
    load(va0, aa0, 0);
    for (int64_t i0 = 0;; i0 += 32) {
      if (i0 + 16 < nfull) load(va1, aa1, i0 + 16);
      mma(va0, aa0);
      if (i0 + 16 >= nfull) break;
      if (i0 + 32 < nfull) load(va0, aa0, i0 + 32);
      mma(va1, aa1);
      if (i0 + 32 >= nfull) break;
    }
  }
  if (nfull < n) {  // ragged tail of the k range
    load(va0, aa0, nfull);
    mma(va0, aa0);
  }

  // Epilogue.  acc[m][t][v] = z at row l = row0 + 16m + row(g, v), column
  // j = col0 + 16t + c.
  const int dm1 = a.d - 1;
  double wsum[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) wsum[t] = 0.0;
  const int64_t nblk = ((int64_t)a.p + 15) >> 4;
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    Quad<T> wq[NT];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t l = row0 + 16 * m + Mfma<T>::row(g, v);
      const double nl = (l < a.p) ? a.nu[l] : 0.0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const double z = (double)acc[m][t][v];
        const double zp = ipow(z, dm1);
        const double wv = nl * zp;
        wsum[t] += wv * z;
        wq[t].e[v] = (T)wv;
      }
    }
    const int64_t b = (row0 >> 4) + m;
    if (b < nblk) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
        vstore4(a.Wp + (((b * a.nt_tot + (a.col0 >> 4) + t) * 64) + lane) * 4, wq[t]);
    }
  }
  // Column sums: across the four row groups g of the wave, then the waves.
  __shared__ double red[4][NT * 16];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double s = wsum[t];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (g == 0) red[wave][t * 16 + c] = s;
  }
  __syncthreads();
  const int rp = a.nt_tot * 16;
  for (int e = threadIdx.x; e < NT * 16; e += blockDim.x) {
    const double s = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
    a.wpart[(int64_t)blockIdx.x * rp + a.col0 + e] = s;
  }
}

// ---------------------------------------------------------------------------
// gemm2: partial Y = V W over one split of the observations
// ---------------------------------------------------------------------------
template <typename T, int NT, bool VEC>
__global__ __launch_bounds__(256) void k_gemm2(G2Args<T> a) {
  using acc_t = typename Mfma<T>::acc_t;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int64_t ibase = (int64_t)blockIdx.x * 256 + wave * 64;
  const int64_t il = ibase + 4 * c;  // this lane's 4 rows (one per M subtile)
  const int64_t n = a.n;
  const bool rows_ok = il < n;

  const int split = blockIdx.y;
  const int64_t b0 = (int64_t)split * a.blk_per_split;
  const int64_t b1 = min((int64_t)a.nblk, b0 + a.blk_per_split);

  acc_t acc[4][NT];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = acc_t{0, 0, 0, 0};

  Quad<T> vq0[4], wq0[NT], vq1[4], wq1[NT];
  const int t0 = a.col0 >> 4;
  auto load = [&](Quad<T>(&vq)[4], Quad<T>(&wq)[NT], int64_t b) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
      vload4(wq[t], a.Wp + (((b * a.nt_tot + t0 + t) * 64) + lane) * 4);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t l = 16 * b + Mfma<T>::row(g, s);
      const bool ok = rows_ok && l < a.p;
      load4<T, VEC>(vq[s], a.V + (ok ? l : 0) * a.ldv, il, n, ok);
    }
  };
  auto mma = [&](const Quad<T>(&vq)[4], const Quad<T>(&wq)[NT]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = Mfma<T>::mac(vq[s].e[m], wq[t].e[s], acc[m][t]);
  };

  if (b0 < b1) {
    load(vq0, wq0, b0);
    for (int64_t b = b0;; b += 2) {
      if (b + 1 < b1) load(vq1, wq1, b + 1);
      mma(vq0, wq0);
      if (b + 1 >= b1) break;
      if (b + 2 < b1) load(vq0, wq0, b + 2);
      mma(vq1, wq1);
      if (b + 2 >= b1) break;
    }
  }

  // acc[m][t][v] = Y[ibase + 4 row(g, v) + m][col0 + 16t + c]
  const int rp = a.nt_tot * 16;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    T* col = a.Ypart + ((int64_t)split * rp + a.col0 + 16 * t + c) * a.npad;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Quad<T> q;
#pragma unroll
      for (int m = 0; m < 4; ++m) q.e[m] = acc[m][t][v];
      vstore4(col + ibase + 4 * Mfma<T>::row(g, v), q);
    }
  }
}

// ---------------------------------------------------------------------------
// gram: B = A'A, C = B^{d-1} (fp64), 16 x 16 output tile per block
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_gram(GramArgs<T> a) {
  __shared__ double sj[64][17];
  __shared__ double sk[64][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int j0 = blockIdx.x * 16, k0 = blockIdx.y * 16;
  double acc = 0.0;
  for (int64_t i0 = 0; i0 < a.n; i0 += 64) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int ii = e & 63, cc = e >> 6;
      const int64_t i = i0 + ii;
      const int j = j0 + cc, k = k0 + cc;
      sj[ii][cc] = (i < a.n && j < a.r) ? (double)a.A[(int64_t)j * a.lda + i] : 0.0;
      sk[ii][cc] = (i < a.n && k < a.r) ? (double)a.A[(int64_t)k * a.lda + i] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int ii = 0; ii < 64; ++ii) acc = fma(sj[ii][tx], sk[ii][ty], acc);
    __syncthreads();
  }
  const int j = j0 + tx, k = k0 + ty;
  if (j < a.r && k < a.r) {
    a.B[(int64_t)k * a.r + j] = acc;
    a.C[(int64_t)k * a.r + j] = ipow(acc, a.d - 1);
  }
}

// ---------------------------------------------------------------------------
// final_G: G_A = -2d (Y - A D_lambda C) D_lambda, Y = fixed-order sum of partials
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_final_G(FinalGArgs<T> a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= a.n) return;
  const int64_t rp = a.rp;
  double y = 0.0;
  const T* yp = a.Ypart + (int64_t)j * a.npad + i;
  for (int s = 0; s < a.nsplit; ++s) y += (double)yp[(int64_t)s * rp * a.npad];
  double adc = 0.0;
  for (int k = 0; k < a.r; ++k)
    adc = fma((double)a.A[(int64_t)k * a.lda + i] * a.lambda[k], a.C[(int64_t)j * a.r + k], adc);
  const double gval = -2.0 * a.d * (y - adc) * a.lambda[j];
  a.G[(int64_t)j * a.ldg + i] = (T)gval;
}

// ---------------------------------------------------------------------------
// final_s: w, u, f, g_lambda (one block)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_final_s(FinalSArgs a) {
  __shared__ double rf[256];
  double fl = 0.0;
  for (int j = threadIdx.x; j < a.r; j += 256) {
    double w = 0.0;
    for (int64_t b = 0; b < a.nwpart; ++b) w += a.wpart[b * a.rp + j];
    double u = 0.0;
    for (int k = 0; k < a.r; ++k) {
      const double bjk = a.B[(int64_t)k * a.r + j];
      u = fma(bjk * a.C[(int64_t)k * a.r + j], a.lambda[k], u);
    }
    a.g_lambda[j] = -2.0 * (w - u);
    fl += a.lambda[j] * u - 2.0 * w * a.lambda[j];
  }
  rf[threadIdx.x] = fl;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) rf[threadIdx.x] += rf[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.f[0] = a.alpha + rf[0];
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <typename T, int MT>
static void dispatch_gemm1(int nt, bool vec, dim3 grid, hipStream_t st, const G1Args<T>& a) {
#define G1_CASE(NTV)                                                            \
  case NTV:                                                                     \
    if (vec) hipLaunchKernelGGL((k_gemm1<T, MT, NTV, true>), grid, dim3(256), 0, st, a);  \
    else hipLaunchKernelGGL((k_gemm1<T, MT, NTV, false>), grid, dim3(256), 0, st, a);    \
    break;
  if constexpr (sizeof(T) == 8) {
    switch (nt) { G1_CASE(1) G1_CASE(2) G1_CASE(3) G1_CASE(4) default: break; }
  } else {
    switch (nt) { G1_CASE(1) G1_CASE(2) G1_CASE(3) G1_CASE(4) G1_CASE(5) G1_CASE(6) G1_CASE(7) default: break; }
  }
#undef G1_CASE
}

template <typename T>
static void dispatch_gemm2(int nt, bool vec, dim3 grid, hipStream_t st, const G2Args<T>& a) {
#define G2_CASE(NTV)                                                            \
  case NTV:                                                                     \
    if (vec) hipLaunchKernelGGL((k_gemm2<T, NTV, true>), grid, dim3(256), 0, st, a);  \
    else hipLaunchKernelGGL((k_gemm2<T, NTV, false>), grid, dim3(256), 0, st, a);    \
    break;
  if constexpr (sizeof(T) == 8) {
    switch (nt) { G2_CASE(1) G2_CASE(2) G2_CASE(3) G2_CASE(4) default: break; }
  } else {
    switch (nt) { G2_CASE(1) G2_CASE(2) G2_CASE(3) G2_CASE(4) G2_CASE(5) G2_CASE(6) G2_CASE(7) default: break; }
  }
#undef G2_CASE
}

void launch_gemm1(int nt, bool vec, dim3 grid, hipStream_t st, const G1Args<float>& a) {
  dispatch_gemm1<float, G1_MT_F32>(nt, vec, grid, st, a);
}
void launch_gemm1(int nt, bool vec, dim3 grid, hipStream_t st, const G1Args<double>& a) {
  dispatch_gemm1<double, G1_MT_F64>(nt, vec, grid, st, a);
}
void launch_gemm2(int nt, bool vec, dim3 grid, hipStream_t st, const G2Args<float>& a) {
  dispatch_gemm2<float>(nt, vec, grid, st, a);
}
void launch_gemm2(int nt, bool vec, dim3 grid, hipStream_t st, const G2Args<double>& a) {
  dispatch_gemm2<double>(nt, vec, grid, st, a);
}
void launch_gram(dim3 grid, hipStream_t st, const GramArgs<float>& a) {
  hipLaunchKernelGGL(k_gram<float>, grid, dim3(256), 0, st, a);
}
void launch_gram(dim3 grid, hipStream_t st, const GramArgs<double>& a) {
  hipLaunchKernelGGL(k_gram<double>, grid, dim3(256), 0, st, a);
}
void launch_final_G(dim3 grid, hipStream_t st, const FinalGArgs<float>& a) {
  hipLaunchKernelGGL(k_final_G<float>, grid, dim3(256), 0, st, a);
}
void launch_final_G(dim3 grid, hipStream_t st, const FinalGArgs<double>& a) {
  hipLaunchKernelGGL(k_final_G<double>, grid, dim3(256), 0, st, a);
}
void launch_final_s(hipStream_t st, const FinalSArgs& a) {
  hipLaunchKernelGGL(k_final_s, dim3(1), dim3(256), 0, st, a);
}

}  // namespace symtd
