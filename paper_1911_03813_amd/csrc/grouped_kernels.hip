// Grouped evaluation kernels (Algorithm 2 over many instances): see grouped.hpp.
//
// The products use the same MFMA operand conventions as the single-instance
// kernels (kcommon.hpp): in ggemm1 a lane supplies observation l = 16 b + c
// of its wave's 16-observation block as the A operand and factor column
// 16 t + c as the B operand, each as 4 consecutive covariates read with one
// vector load; the accumulators come out as Z[16 b + row(g, v)][16 t + c],
// which is the packed order of W.  In ggemm2 a lane supplies 4 consecutive
// rows of V (one per M subtile) and the packed W quad of its observations.
// Instances are small (their data sits in L2), so both products read their
// operands straight from memory; many items per step fill the chip.
#include <type_traits>

#include "grouped.hpp"
#include "kcommon.hpp"
#include "philox.hpp"

namespace symtd {

namespace {

// elements i .. i+3 of a column of n (zero past n).  VEC (leading dimension a
// multiple of 4, 16-byte aligned columns): one 16-byte load of the quad,
// clamped into the column's first 4 ceil(n/4) elements, then the elements
// past n replaced by zero; no branch, so the load never waits on a test.
template <typename T, bool VEC>
__device__ __forceinline__ void quad_at(Quad<T>& q, const T* col, int64_t i, int64_t n) {
  if constexpr (VEC) {
    const int64_t n4 = (n + 3) & ~(int64_t)3;
    vload4(q, col + (i < n4 ? i : n4 - 4));
#pragma unroll
    for (int e = 0; e < 4; ++e) q.e[e] = i + e < n ? q.e[e] : T(0);
  } else {
    load_tail(q, col, i, n);
  }
}

// ---------------------------------------------------------------------------
// ggemm1 body for NT column subtiles
// ---------------------------------------------------------------------------
template <typename T, int NT, bool VEC>
__device__ void ggemm1_body(const GInst<T>& I, int tile, int cg, double (*red)[GG_NT_MAX * 16]) {
  using acc_t = typename Mfma<T>::acc_t;
  constexpr int NTM = std::is_same<T, float>::value ? GG_NT_F32 : GG_NT_F64;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, c = lane & 15;
  const int64_t n = I.n, p = I.p;
  const int col0 = cg * NTM * 16;
  const int dm1 = I.d - 1;
  // factor columns of this lane (one per subtile); columns past cols read as zero
  const T* acol[NT];
  bool aok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = col0 + 16 * t + c;
    aok[t] = col < I.cols;
    acol[t] = I.A + (int64_t)(aok[t] ? col : 0) * I.lda;
  }
  double wsum[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) wsum[t] = 0.0;
  const int64_t nblk = (p + 15) / 16;
  // the wave's four 16-observation blocks b_q = 16 tile + 4 q + wave are
  // multiplied together, so that each factor quad serves all four; blocks
  // past the last are computed from a valid column and not written
  constexpr int QB = GG1_TILE / 64;
  const T* vcol[QB];
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    const int64_t l = 16 * ((int64_t)tile * (GG1_TILE / 16) + 4 * q + wave) + c;
    vcol[q] = I.V + (l < p ? l : p - 1) * I.ldv;
  }
  acc_t acc[QB][NT];
#pragma unroll
  for (int q = 0; q < QB; ++q)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[q][t] = acc_t{0, 0, 0, 0};
  // the accumulators stay in AGPRs (left to the compiler, the fp64 ones are
  // copied to VGPRs and back at every step)
  auto pin = [&]() {
#pragma unroll
    for (int q = 0; q < QB; ++q)
#pragma unroll
      for (int t = 0; t < NT; ++t) asm("" : "+a"(acc[q][t]));
  };
  pin();
  for (int64_t k0 = 0; k0 < n; k0 += 16) {
    const int64_t k = k0 + 4 * g;
    Quad<T> v[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) quad_at<T, VEC>(v[q], vcol[q], k, n);
    Quad<T> a[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      quad_at<T, VEC>(a[t], acol[t], k, n);
      if (!aok[t]) zero4(a[t]);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int q = 0; q < QB; ++q)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[q][t] = Mfma<T>::mac(v[q].e[s], a[t].e[s], acc[q][t]);
    pin();
  }
  // epilogue per block: acc[q][t][v] = z at l = 16 b + row(g, v), column
  // col0 + 16 t + c.  w = nu z^(d-1) in the storage precision (the exponent
  // loop outside, so that the products are independent), the sums of w z in
  // fp64, block by block
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    const int64_t b = (int64_t)tile * (GG1_TILE / 16) + 4 * q + wave;
    if (b >= nblk) break;
    T nl[4];   // clamped loads without branches, issued together
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t lv = 16 * b + Mfma<T>::row(g, v);
      const double x = gload(I.nu + (lv < p ? lv : p - 1));
      nl[v] = lv < p ? (T)x : T(0);
    }
    acc_t zp[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) zp[t] = acc_t{1, 1, 1, 1};
    for (int e = 0; e < dm1; ++e)
#pragma unroll
      for (int t = 0; t < NT; ++t) zp[t] *= acc[q][t];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      Quad<T> wq;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T wv = nl[v] * zp[t][v];
        wq.e[v] = wv;
        wsum[t] += (double)wv * (double)acc[q][t][v];
      }
      vstore4(I.Wp + ((b * I.nt + cg * NTM + t) * 64 + lane) * 4, wq);
    }
  }
  // column sums of nu z^d over this tile: lane groups, then waves (fixed order)
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double s = wsum[t];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (g == 0) red[wave][16 * t + c] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NT * 16; e += 256) {
    const int col = col0 + e;
    if (col < I.cols)
      gstore(I.wpart + (int64_t)tile * I.cols + col, (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]));
  }
}

// ---------------------------------------------------------------------------
// ggemm2 body for NT column subtiles: one wave, 64 rows
// ---------------------------------------------------------------------------
template <typename T, int NT, bool VEC>
__device__ void ggemm2_body(const GInst<T>& I, int rb, int split, int cg) {
  using acc_t = typename Mfma<T>::acc_t;
  constexpr int NTM = std::is_same<T, float>::value ? GG_NT_F32 : GG_NT_F64;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int64_t n = I.n, p = I.p;
  const int64_t ibase = (int64_t)rb * 64;
  const int64_t il = ibase + 4 * c;
  const int64_t n4 = (n + 3) & ~(int64_t)3;
  const int64_t nblk = (p + 15) / 16;
  const int64_t b0 = (int64_t)split * I.split_blk;
  const int64_t b1 = min(nblk, b0 + (int64_t)I.split_blk);
  acc_t acc[4][NT];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = acc_t{0, 0, 0, 0};
  // the accumulators stay in AGPRs, as in ggemm1_body
  auto pin = [&]() {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t) asm("" : "+a"(acc[m][t]));
  };
  pin();
  for (int64_t b = b0; b < b1; ++b) {
    Quad<T> w[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) vload4(w[t], I.Wp + ((b * I.nt + cg * NTM + t) * 64 + lane) * 4);
    Quad<T> v[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int64_t l = 16 * b + Mfma<T>::row(g, s);
      l = l < p ? l : p - 1;            // rows of W past p are zero
      const T* col = I.V + l * I.ldv;
      // rows past n only reach rows of Y that are never read: VEC loads the
      // quad clamped into the column without masking it
      if constexpr (VEC) vload4(v[s], col + (il < n4 ? il : n4 - 4));
      else load_tail(v[s], col, il, n);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = Mfma<T>::mac(v[s].e[m], w[t].e[s], acc[m][t]);
    pin();
  }
  // acc[m][t][v] = Y[ibase + 4 row(g, v) + m][col0 + 16 t + c]
  const int64_t rp = (int64_t)I.nt * 16;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    T* col = I.Ypart + ((int64_t)split * rp + cg * NTM * 16 + 16 * t + c) * I.ldy;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Quad<T> q;
#pragma unroll
      for (int m = 0; m < 4; ++m) q.e[m] = acc[m][t][v];
      vstore4(col + ibase + 4 * Mfma<T>::row(g, v), q);
    }
  }
}

}  // namespace

template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_ggemm1(const GInst<T>* insts, const GItem* items) {
  __shared__ double red[4][GG_NT_MAX * 16];
  const GItem it = items[blockIdx.x];
  const GInst<T> I = insts[it.inst];
  constexpr int NTM = std::is_same<T, float>::value ? GG_NT_F32 : GG_NT_F64;
  const int ntg = min(NTM, I.nt - it.b * NTM);
  switch (ntg) {
    case 1: ggemm1_body<T, 1, VEC>(I, it.a, it.b, red); break;
    case 2: ggemm1_body<T, 2, VEC>(I, it.a, it.b, red); break;
    case 3: ggemm1_body<T, 3, VEC>(I, it.a, it.b, red); break;
    case 4: ggemm1_body<T, 4, VEC>(I, it.a, it.b, red); break;
    default:
      if constexpr (NTM > 4) {
        switch (ntg) {
          case 5: ggemm1_body<T, 5, VEC>(I, it.a, it.b, red); break;
          case 6: ggemm1_body<T, 6, VEC>(I, it.a, it.b, red); break;
          case 7: ggemm1_body<T, 7, VEC>(I, it.a, it.b, red); break;
          case 8: ggemm1_body<T, 8, VEC>(I, it.a, it.b, red); break;
          default: break;
        }
      }
  }
}

template <typename T, bool VEC>
__global__ __launch_bounds__(64) void k_ggemm2(const GInst<T>* insts, const GItem* items) {
  const GItem it = items[blockIdx.x];
  const GInst<T> I = insts[it.inst];
  constexpr int NTM = std::is_same<T, float>::value ? GG_NT_F32 : GG_NT_F64;
  const int ntg = min(NTM, I.nt - it.c * NTM);
  switch (ntg) {
    case 1: ggemm2_body<T, 1, VEC>(I, it.a, it.b, it.c); break;
    case 2: ggemm2_body<T, 2, VEC>(I, it.a, it.b, it.c); break;
    case 3: ggemm2_body<T, 3, VEC>(I, it.a, it.b, it.c); break;
    case 4: ggemm2_body<T, 4, VEC>(I, it.a, it.b, it.c); break;
    default:
      if constexpr (NTM > 4) {
        switch (ntg) {
          case 5: ggemm2_body<T, 5, VEC>(I, it.a, it.b, it.c); break;
          case 6: ggemm2_body<T, 6, VEC>(I, it.a, it.b, it.c); break;
          case 7: ggemm2_body<T, 7, VEC>(I, it.a, it.b, it.c); break;
          case 8: ggemm2_body<T, 8, VEC>(I, it.a, it.b, it.c); break;
          default: break;
        }
      }
  }
}

// ---------------------------------------------------------------------------
// gmodel: one block per (instance, model): B, C, u, w, f, g_lambda, Y_M (fp64)
//
// For r <= GM_RMAX the block moves the model's A to LDS in chunks of GM_ROWS
// rows (every load of a chunk issued before any is used) and keeps B and C in
// LDS; larger r reads A from global memory directly.  Both ways take every
// sum in the same order (B over i ascending, Y_M over l ascending), so the
// results are the same bits.
// ---------------------------------------------------------------------------
constexpr int GM_RMAX = 32;
constexpr int GM_ROWS = 64;
// partials (of w per tile, of Y per split) one thread loads at once: p = 8192
// observations make 32 tiles and 32 splits of 256
constexpr int GF_SPLITS = 32;

// the chunk of rows [i0, i0 + GM_ROWS) of A (r <= GM_RMAX columns) into
// sA[ii][l] as fp64 (times lambda_l when lam is given), zero past n
template <typename T>
__device__ __forceinline__ void gm_stage(const T* A, int64_t lda, int n, int r, int64_t i0, const double* lam,
                                         double (*sA)[GM_RMAX + 1]) {
  constexpr int IT = GM_ROWS * GM_RMAX / 256;
  T x[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + 256 * it;
    const int ii = e % GM_ROWS, l = min(e / GM_ROWS, r - 1);
    const int64_t i = i0 + ii;
    x[it] = gload(A + (int64_t)l * lda + (i < n ? i : 0));
  }
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + 256 * it;
    const int ii = e % GM_ROWS, l = e / GM_ROWS;
    if (l < r) sA[ii][l] = i0 + ii < n ? (lam ? (double)x[it] * lam[l] : (double)x[it]) : 0.0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gmodel(const GInst<T>* insts, const GItem* items) {
  __shared__ double sA[GM_ROWS][GM_RMAX + 1];
  __shared__ double sB[GM_RMAX * GM_RMAX], sC[GM_RMAX * GM_RMAX];
  __shared__ double fs[256];
  const GItem it = items[blockIdx.x];
  const GInst<T> I = insts[it.inst];
  const int k = it.a;                       // model
  const int r = I.r, n = I.n;
  const int64_t rr = (int64_t)r * r;
  const T* A = I.A + (int64_t)k * r * I.lda;
  const double* lam = I.lam + (int64_t)k * r;
  double* B = I.B + k * rr;
  double* C = I.C + k * rr;
  const bool fast = r <= GM_RMAX;
  // B = A'A (upper pairs, mirrored), C = B^{d-1}
  if (fast) {
    // thread t takes the pairs e = t, t + 256, ... (j <= l), at most
    // GM_RMAX^2 / 256 of them
    // pair q of thread t is e = t + 256 q: j = t mod GM_RMAX for every q (256
    // is a multiple of GM_RMAX), l = t / GM_RMAX + (256 / GM_RMAX) q; pairs
    // outside the model are formed from in-range LDS columns and not written
    constexpr int PP = GM_RMAX * GM_RMAX / 256;
    static_assert(256 % GM_RMAX == 0, "pairs of a thread share their first column");
    const int jt = threadIdx.x % GM_RMAX, lt = threadIdx.x / GM_RMAX;
    double s[PP];
#pragma unroll
    for (int q = 0; q < PP; ++q) s[q] = 0.0;
    for (int64_t i0 = 0; i0 < n; i0 += GM_ROWS) {
      gm_stage(A, I.lda, n, r, i0, nullptr, sA);
      __syncthreads();
      const int rows = (int)min((int64_t)GM_ROWS, n - i0);
      // every pair advances in the same row loop (independent chains, no
      // per-thread branch), each summing over the rows in order; A[i][j]
      // is read once for the thread's pairs
#pragma unroll 4
      for (int ii = 0; ii < rows; ++ii) {
        const double aj = sA[ii][jt];
#pragma unroll
        for (int q = 0; q < PP; ++q) s[q] = fma(aj, sA[ii][lt + (256 / GM_RMAX) * q], s[q]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int j = e % GM_RMAX, l = e / GM_RMAX;
      if (j < r && l < r && j <= l) {
        const double cv = ipow(s[q], I.d - 1);
        B[(int64_t)l * r + j] = s[q]; B[(int64_t)j * r + l] = s[q];
        C[(int64_t)l * r + j] = cv; C[(int64_t)j * r + l] = cv;
        sB[l * r + j] = s[q]; sB[j * r + l] = s[q];
        sC[l * r + j] = cv; sC[j * r + l] = cv;
      }
    }
  } else {
    for (int e = threadIdx.x; e < r * r; e += 256) {
      const int j = e % r, l = e / r;
      if (j > l) continue;
      const T* aj = A + (int64_t)j * I.lda;
      const T* al = A + (int64_t)l * I.lda;
      double s = 0.0;
      for (int i = 0; i < n; ++i) s = fma((double)aj[i], (double)al[i], s);
      const double cv = ipow(s, I.d - 1);
      B[(int64_t)l * r + j] = s; B[(int64_t)j * r + l] = s;
      C[(int64_t)l * r + j] = cv; C[(int64_t)j * r + l] = cv;
    }
  }
  __syncthreads();
  const double* Bs = fast ? sB : B;
  const double* Cs = fast ? sC : C;
  // u, w, g_lambda and f: thread t handles columns t, t + 256, ... and its
  // share of f; the shares are then summed in thread order
  double fsh = 0.0;
  for (int j = threadIdx.x; j < r; j += 256) {
    double u = 0.0;
    for (int l = 0; l < r; ++l) u += Bs[(int64_t)l * r + j] * Cs[(int64_t)l * r + j] * lam[l];
    const int col = k * r + j;
    // the tile partials of w, up to GF_SPLITS at a time from valid rows, in order
    double w = 0.0;
    for (int t0 = 0; t0 < I.ntile; t0 += GF_SPLITS) {
      double v[GF_SPLITS];
#pragma unroll
      for (int h = 0; h < GF_SPLITS; ++h) v[h] = gload(I.wpart + (int64_t)min(t0 + h, I.ntile - 1) * I.cols + col);
#pragma unroll
      for (int h = 0; h < GF_SPLITS; ++h)
        if (t0 + h < I.ntile) w += v[h];
    }
    I.glam[col] = -2.0 * (w - u);
    fsh += lam[j] * u - 2.0 * w * lam[j];
  }
  fs[threadIdx.x] = fsh;
  __syncthreads();
  if (threadIdx.x == 0) {
    // shares past thread r - 1 are zero
    double f = 0.0;
    for (int t = 0; t < min(r, 256); ++t) f += fs[t];
    I.f[k] = I.alpha + f;
  }
  // Y_M = A D_lambda C for this model's columns
  if (fast) {
    for (int64_t i0 = 0; i0 < n; i0 += GM_ROWS) {
      __syncthreads();                       // the previous chunk (or B's) is read
      gm_stage(A, I.lda, n, r, i0, lam, sA);
      __syncthreads();
      const int rows = (int)min((int64_t)GM_ROWS, n - i0);
      // lane ii of wave w forms row ii for the columns j = w, w + 4, ...: one
      // read of A[ii][l] serves GM_RMAX / 4 columns, and a wave's reads of C
      // are broadcasts; every element sums over l in order
      static_assert(GM_ROWS == 64 && GM_RMAX % 4 == 0, "one row per lane, four waves");
      constexpr int JB = GM_RMAX / 4;
      const int ii = threadIdx.x % GM_ROWS, jw = threadIdx.x / GM_ROWS;
      if (ii < rows) {
        double s[JB];
#pragma unroll
        for (int b = 0; b < JB; ++b) s[b] = 0.0;
        for (int l = 0; l < r; ++l) {
          const double a = sA[ii][l];
#pragma unroll
          for (int b = 0; b < JB; ++b) s[b] = fma(a, sC[(jw + 4 * b) * r + l], s[b]);
        }
#pragma unroll
        for (int b = 0; b < JB; ++b) {
          const int j = jw + 4 * b;
          if (j < r) gstore(I.YM + ((int64_t)k * r + j) * n + i0 + ii, s[b]);
        }
      }
    }
  } else {
    for (int e = threadIdx.x; e < n * r; e += 256) {
      const int i = e % n, j = e / n;
      double s = 0.0;
      for (int l = 0; l < r; ++l) s = fma((double)A[(int64_t)l * I.lda + i] * lam[l], C[(int64_t)j * r + l], s);
      I.YM[((int64_t)k * r + j) * n + i] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// gfinal: one block per (instance, column): G_A = -2d (Y - Y_M) lambda
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_gfinal(const GInst<T>* insts, const GItem* items) {
  const GItem it = items[blockIdx.x];
  const GInst<T> I = insts[it.inst];
  const int col = it.a;
  const int64_t rp = (int64_t)I.nt * 16;
  const double lj = gload(I.lam + col);
  for (int i = threadIdx.x; i < I.n; i += 256) {
    const double ym = gload(I.YM + (int64_t)col * I.n + i);
    // the split partials (at most GF_SPLITS per pass, from valid splits, all
    // in flight together), summed in split order
    double y = 0.0;
    for (int s0 = 0; s0 < I.nsplit; s0 += GF_SPLITS) {
      T v[GF_SPLITS];
#pragma unroll
      for (int h = 0; h < GF_SPLITS; ++h)
        v[h] = gload(I.Ypart + ((int64_t)min(s0 + h, I.nsplit - 1) * rp + col) * I.ldy + i);
#pragma unroll
      for (int h = 0; h < GF_SPLITS; ++h)
        if (s0 + h < I.nsplit) y += (double)v[h];
    }
    const double gval = -2.0 * I.d * (y - ym) * lj;
    gstore(I.G + (int64_t)col * I.ldg + i, (T)gval);
  }
}

// ---------------------------------------------------------------------------
// gomega: Omega of every restart into the packed W of every instance
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_gomega(const GInst<T>* insts, const uint64_t* seeds) {
  const GInst<T> I = insts[blockIdx.y];
  const uint64_t seed = seeds[blockIdx.y];
  const int64_t nblk = ((int64_t)I.p + 15) / 16;
  const int64_t total = nblk * I.nt * 256;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int s = (int)(idx & 3);
    const int lane = (int)((idx >> 2) & 63);
    const int g = lane >> 4, c = lane & 15;
    const int64_t bt = idx >> 8;
    const int t = (int)(bt % I.nt);
    const int64_t b = bt / I.nt;
    const int64_t l = 16 * b + Mfma<T>::row(g, s);
    const int col = 16 * t + c;
    double v = 0.0;
    if (l < I.p && col < I.cols) {
      const int k = col / I.r, j = col - k * I.r;
      v = normal_at(seed, (uint32_t)k, STREAM_RRF_OMEGA, l + (int64_t)I.p * j);
    }
    I.Wp[idx] = (T)v;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
void launch_ggemm1(bool vec, int nitems, hipStream_t st, const GInst<T>* insts, const GItem* items) {
  if (nitems <= 0) return;
  if (vec) hipLaunchKernelGGL((k_ggemm1<T, true>), dim3(nitems), dim3(256), 0, st, insts, items);
  else hipLaunchKernelGGL((k_ggemm1<T, false>), dim3(nitems), dim3(256), 0, st, insts, items);
}
template <typename T>
void launch_gmodel(int nitems, hipStream_t st, const GInst<T>* insts, const GItem* items) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_gmodel<T>, dim3(nitems), dim3(256), 0, st, insts, items);
}
template <typename T>
void launch_ggemm2(bool vec, int nitems, hipStream_t st, const GInst<T>* insts, const GItem* items) {
  if (nitems <= 0) return;
  if (vec) hipLaunchKernelGGL((k_ggemm2<T, true>), dim3(nitems), dim3(64), 0, st, insts, items);
  else hipLaunchKernelGGL((k_ggemm2<T, false>), dim3(nitems), dim3(64), 0, st, insts, items);
}
template <typename T>
void launch_gfinal(int nitems, hipStream_t st, const GInst<T>* insts, const GItem* items) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(k_gfinal<T>, dim3(nitems), dim3(256), 0, st, insts, items);
}
template <typename T>
void launch_gomega(int maxchunks, int ninst, hipStream_t st, const GInst<T>* insts, const uint64_t* seeds) {
  if (ninst <= 0) return;
  hipLaunchKernelGGL(k_gomega<T>, dim3(maxchunks, ninst), dim3(256), 0, st, insts, seeds);
}

#define SYMTD_GG_INST(T)                                                                              \
  template void launch_ggemm1<T>(bool, int, hipStream_t, const GInst<T>*, const GItem*);              \
  template void launch_gmodel<T>(int, hipStream_t, const GInst<T>*, const GItem*);                    \
  template void launch_ggemm2<T>(bool, int, hipStream_t, const GInst<T>*, const GItem*);              \
  template void launch_gfinal<T>(int, hipStream_t, const GInst<T>*, const GItem*);                    \
  template void launch_gomega<T>(int, int, hipStream_t, const GInst<T>*, const uint64_t*);
SYMTD_GG_INST(float)
SYMTD_GG_INST(double)

}  // namespace symtd
