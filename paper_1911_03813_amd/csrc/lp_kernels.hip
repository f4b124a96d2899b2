// fp16 / bf16x3 products of the evaluation (see lp.hpp).
//
// The MFMA is v_mfma_f32_16x16x32_{f16,bf16}: lane 16 g + c supplies row c
// and k values 8 g .. 8 g + 7 of a 32-deep step, and holds output rows
// 4 g .. 4 g + 3 of column c.  Chunks of the operands move from HBM to LDS as
// 16-byte pieces by direct global-to-LDS loads (every thread moves the same
// number of pieces; the piece for LDS slot s is chosen so that it lands on
// s), and two LDS stages alternate.
//
// The first product is "k-contiguous": every operand column of Vc (an
// observation) and of Ac holds its k values (covariates) contiguously, so a
// lane's operand is one 16-byte LDS vector; slots are XOR-swizzled so that
// the 16 columns of a fragment read hit distinct banks.  The second product
// reads the same Vc with observations as k: a chunk holds, for each of its
// observations, the 8-covariate units of the block's row slab, and a lane's
// operand (8 observations of one covariate) comes from two transposed
// 8-byte LDS reads (ds_read_b64_tr_b16: in each group of 16 lanes, lane c
// receives element c mod 4 of the words of lanes c / 4, 4 + c / 4, 8 + c / 4
// and 12 + c / 4, checked on the hardware), so V is stored once.
#include <type_traits>

#include "kcommon.hpp"
#include "lp.hpp"
#include "model_dev.hpp"

namespace symtd {

namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

template <int KIND> struct LpT;
template <> struct LpT<LP_F16> {
  using E = _Float16;
  static constexpr int PLANES = 1;
  static __device__ __forceinline__ f4 mac(const u4* v, const u4* a, f4 acc) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, v[0]), __builtin_bit_cast(h8, a[0]), acc,
                                                  0, 0, 0);
  }
  static __device__ __forceinline__ void split(double x, E* out) { out[0] = (E)(float)x; }
  static __device__ __forceinline__ void split(float x, E* out) { out[0] = (E)x; }
};
template <> struct LpT<LP_BF16X3> {
  using E = __bf16;
  static constexpr int PLANES = 2;
  // (hi, lo) x (hi, lo) without the lo lo term
  static __device__ __forceinline__ f4 mac(const u4* v, const u4* a, f4 acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, v[1]), __builtin_bit_cast(b8, a[0]), acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, v[0]), __builtin_bit_cast(b8, a[1]), acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, v[0]), __builtin_bit_cast(b8, a[0]), acc, 0, 0, 0);
  }
  static __device__ __forceinline__ void split(double x, E* out) {
    const float xf = (float)x;
    const __bf16 hi = (__bf16)xf;
    out[0] = hi;
    out[1] = (__bf16)(float)(x - (double)(float)hi);
  }
  // from fp32 the difference x - hi is exact
  static __device__ __forceinline__ void split(float x, E* out) {
    const __bf16 hi = (__bf16)x;
    out[0] = hi;
    out[1] = (__bf16)(x - (float)hi);
  }
};

template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// One chunk's LDS stage: V/X part then A/W part, 16-byte units.
template <int KIND, int NT>
struct LpStage {
  static constexpr int PL = LpT<KIND>::PLANES;
  static constexpr int U = lp_chunk(KIND) / 8;                 // units per column per plane
  static constexpr int XU = PL * LP_SLAB * U;                   // units of the slab operand
  static constexpr int YU = PL * 16 * NT * U;                   // units of the column operand
  static constexpr int XP = (XU + 255) / 256;                   // pieces per thread
  static constexpr int YP = (YU + 255) / 256;
  static constexpr int DPC = XP + YP;
  // 16-byte unit q of column col at col U + (q ^ ((col / R) mod U)), R = 16 / U
  // columns per 256-byte bank row: the 16 columns of a fragment read land in
  // 16 distinct 16-byte slots of the bank rows
  static constexpr int RSH = U >= 16 ? 0 : U == 8 ? 1 : 2;
  static_assert(U == 4 || U == 8 || U >= 16, "units per column");
  static __device__ __forceinline__ int swz(int col, int q) { return col * U + (q ^ ((col >> RSH) & (U - 1))); }
  static __device__ __forceinline__ void unswz(int s, int& col, int& q) {
    col = s / U;
    q = (s % U) ^ ((col >> RSH) & (U - 1));
  }
};

// The second product's slab operand in LDS: for each observation k of the
// chunk (row k), the LP_SLAB / 8 = 16 units of 8 covariates of the block's
// slab; unit qc of row k is stored at unit qc ^ 2 sigma(k) of the row, with
// sigma(k) = (k mod 4) + 4 ((k / 4 + k / 8) mod 2).  A transposed read of
// one fragment touches rows k0 + j (j < 4) in each 16-lane group g (k0 = 8 g
// or 8 g + 4), two units per row: the four rows of a group land on four
// distinct unit pairs, and groups g and g + 1 on the two halves of the row,
// so a 16-lane group covers every bank of a 128-byte row once and a
// 32-lane half-wave every bank of a 256-byte row once.
struct TrSwz {
  static constexpr int UPR = LP_SLAB / 8;
  static_assert(UPR == 16, "the transposed-read swizzle is written for 16 units per row");
  static __device__ __forceinline__ int sig2(int k) { return 2 * ((k & 3) | ((((k >> 2) ^ (k >> 3)) & 1) << 2)); }
  static __device__ __forceinline__ int slot(int k, int qc) { return k * UPR + (qc ^ sig2(k)); }
  static __device__ __forceinline__ void unslot(int s, int& k, int& qc) {
    k = s / UPR;
    qc = (s % UPR) ^ sig2(k);
  }
};

// DMA of one chunk: the slab operand's pieces xsrc(plane, col, unit) (for
// TR, col is the chunk's observation and unit its 8-covariate unit) and the
// column operand's pieces ysrc(plane, col, unit)
template <int KIND, int NT, bool TR, typename XF, typename YF>
__device__ __forceinline__ void lp_dma(u4* lx, u4* ly, int tid, int wave, XF xsrc, YF ysrc) {
  using S = LpStage<KIND, NT>;
  constexpr int PU = S::XU / S::PL;                              // units per plane
#pragma unroll
  for (int i = 0; i < S::XP; ++i) {
    const int P = tid + 256 * i;
    const void* src = xsrc(0, 0, 0);                             // padding pieces: any valid address
    if (P < S::XU) {
      const int pl = P / PU;
      int col, q;
      if constexpr (TR) TrSwz::unslot(P % PU, col, q);
      else S::unswz(P % PU, col, q);
      src = xsrc(pl, col, q);
    }
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)((char*)lx + 16 * (256 * i + 64 * wave)),
                                     16, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < S::YP; ++i) {
    const int P = tid + 256 * i;
    const void* src = ysrc(0, 0, 0);
    if (P < S::YU) {
      const int pl = P / (16 * NT * S::U);
      int col, q;
      S::unswz(P % (16 * NT * S::U), col, q);
      src = ysrc(pl, col, q);
    }
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)((char*)ly + 16 * (256 * i + 64 * wave)),
                                     16, 0, 0);
  }
}

// multiply one chunk held in LDS into acc (fragments double-buffered)
template <int KIND, int NT>
__device__ __forceinline__ void lp_compute(const u4* lx, const u4* ly, int wave, int g, int c, f4 (&acc)[LP_MT][NT]) {
  using S = LpStage<KIND, NT>;
  constexpr int PL = S::PL;
  constexpr int J = S::U / 4;
  u4 fv[2][LP_MT][PL], fa[2][NT][PL];
  auto frag = [&](int b, int jg) {
    const int q = 4 * jg + g;
#pragma unroll
    for (int m = 0; m < LP_MT; ++m)
#pragma unroll
      for (int pl = 0; pl < PL; ++pl) fv[b][m][pl] = lx[pl * LP_SLAB * S::U + S::swz(16 * (LP_MT * wave + m) + c, q)];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int pl = 0; pl < PL; ++pl) fa[b][t][pl] = ly[pl * 16 * NT * S::U + S::swz(16 * t + c, q)];
  };
  frag(0, 0);
#pragma unroll
  for (int jg = 0; jg < J; ++jg) {
    if (jg + 1 < J) frag((jg + 1) & 1, jg + 1);
#pragma unroll
    for (int m = 0; m < LP_MT; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[m][t] = LpT<KIND>::mac(fv[jg & 1][m], fa[jg & 1][t], acc[m][t]);
  }
}

// multiply one chunk of the second product held in LDS into acc: the slab
// operand by transposed reads, the column operand (W) as in lp_compute
template <int KIND, int NT>
__device__ __forceinline__ void lp_compute_tr(const u4* lx, const u4* ly, int wave, int g, int c,
                                              f4 (&acc)[LP_MT][NT]) {
  using S = LpStage<KIND, NT>;
  constexpr int PL = S::PL;
  constexpr int J = S::U / 4;
  constexpr int PU = S::XU / PL;
  typedef short s4 __attribute__((ext_vector_type(4)));
  u4 fv[2][LP_MT][PL], fa[2][NT][PL];
  // lane c of group g points at observation k0 + c / 4, covariates
  // 4 (c mod 4) .. + 3 of the subtile, i.e. unit c mod 4 / 2, half c mod 2
  const int krow = 8 * g + (c >> 2);
  const int qoff = (c & 3) >> 1;
  const int boff = 8 * (c & 1);
  auto frag = [&](int b, int jg) {
    const int q = 4 * jg + g;
#pragma unroll
    for (int m = 0; m < LP_MT; ++m)
#pragma unroll
      for (int pl = 0; pl < PL; ++pl) {
        s4 h[2];
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int k = 32 * jg + krow + 4 * hh;
          const int qc = 2 * (LP_MT * wave + m) + qoff;
          const char* addr = (const char*)(lx + pl * PU + TrSwz::slot(k, qc)) + boff;
          h[hh] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s4*)addr);
        }
        const u2 lo = __builtin_bit_cast(u2, h[0]), hi = __builtin_bit_cast(u2, h[1]);
        fv[b][m][pl] = u4{lo[0], lo[1], hi[0], hi[1]};
      }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int pl = 0; pl < PL; ++pl) fa[b][t][pl] = ly[pl * 16 * NT * S::U + S::swz(16 * t + c, q)];
  };
  frag(0, 0);
#pragma unroll
  for (int jg = 0; jg < J; ++jg) {
    if (jg + 1 < J) frag((jg + 1) & 1, jg + 1);
#pragma unroll
    for (int m = 0; m < LP_MT; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[m][t] = LpT<KIND>::mac(fv[jg & 1][m], fa[jg & 1][t], acc[m][t]);
  }
}

}  // namespace

// The chunk loop of a block over nk chunks, with LP_STAGES LDS stages: chunk
// q lives in stage q mod LP_STAGES; `issue(stage, q)` starts its DMA and
// `use(stage)` multiplies it.  A wave waits (vmcnt) until its pieces of the
// chunk it needs have landed, counting the later chunks still in flight, and
// the barrier then guarantees every wave's pieces are in and that the stage
// about to be refilled has been read by all.
#define LP_CHUNK_LOOP                                                                                     \
  auto chunk_loop = [&](int64_t nk, auto issue, auto use) {                                               \
    constexpr int DPC = S::DPC;                                                                           \
    auto arrive = [&](int64_t later) {                                                                    \
      if (LP_STAGES > 2 && later >= 1) wait_vm<DPC>(); else wait_vm<0>();                                  \
      __syncthreads();                                                                                    \
    };                                                                                                    \
    if constexpr (LP_STAGES == 3) {                                                                       \
      if (nk <= 0) return;                                                                                \
      issue(lx0, ly0, 0);                                                                                 \
      if (nk > 1) issue(lx1, ly1, 1);                                                                     \
      int64_t q = 0;                                                                                      \
      for (; q + 3 <= nk; q += 3) {                                                                       \
        arrive(min((int64_t)1, nk - 1 - q));                                                              \
        if (q + 2 < nk) issue(lx2, ly2, q + 2);                                                           \
        use(lx0, ly0);                                                                                    \
        arrive(min((int64_t)1, nk - 2 - q));                                                              \
        if (q + 3 < nk) issue(lx0, ly0, q + 3);                                                           \
        use(lx1, ly1);                                                                                    \
        arrive(min((int64_t)1, nk - 3 - q));                                                              \
        if (q + 4 < nk) issue(lx1, ly1, q + 4);                                                           \
        use(lx2, ly2);                                                                                    \
      }                                                                                                   \
      if (q < nk) { arrive(min((int64_t)1, nk - 1 - q)); use(lx0, ly0); }                                  \
      if (q + 1 < nk) { arrive(0); use(lx1, ly1); }                                                       \
    } else {                                                                                              \
      if (nk > 0) issue(lx0, ly0, 0);                                                                     \
      int64_t q = 0;                                                                                      \
      for (; q + 2 <= nk; q += 2) {                                                                       \
        arrive(0);                                                                                        \
        issue(lx1, ly1, q + 1);                                                                           \
        use(lx0, ly0);                                                                                    \
        arrive(0);                                                                                        \
        if (q + 2 < nk) issue(lx0, ly0, q + 2);                                                           \
        use(lx1, ly1);                                                                                    \
      }                                                                                                   \
      if (q < nk) { arrive(0); use(lx0, ly0); }                                                           \
    }                                                                                                     \
  };

// ---------------------------------------------------------------------------
// gemm1: Z = Vc' Ac for one column group, stream-K over (slab, chunk) as in
// the fp32 kernel; epilogue W = 2^s nu z^{d-1} (column-major, ld ldr) and
// fp64 column sums of nu z^d, one row per wave.
// ---------------------------------------------------------------------------
template <int KIND, int NT>
__global__ __launch_bounds__(256) void k_lp_gemm1(LpG1Args a) {
  using S = LpStage<KIND, NT>;
  using E = typename LpT<KIND>::E;
  constexpr int PL = S::PL;
  constexpr int KCH = lp_chunk(KIND);
  constexpr int PART = LP_WAVES * LP_MT * NT * 256;
  __shared__ u4 lx0[S::XP * 256], lx1[S::XP * 256];
  __shared__ u4 ly0[S::YP * 256], ly1[S::YP * 256];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, c = lane & 15;
  const int64_t B = a.nblocks, blk = blockIdx.x;
  const int64_t KC = a.kc_len / KCH;
  const int64_t U = (int64_t)a.nslab * KC;
  const int64_t u0 = blk * U / B, u1 = (blk + 1) * U / B;
  const E* V = (const E*)a.Vc;
  const E* Ac = (const E*)a.Ac;
  const int dm1 = a.d - 1;
  const int epoch = handoff_epoch(a.ho.epoch);

  f4 acc[LP_MT][NT];
#pragma unroll
  for (int m = 0; m < LP_MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = f4{0, 0, 0, 0};
  double wsum[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) wsum[t] = 0.0;

  auto dma = [&](u4* lx, u4* ly, int64_t sl, int64_t kc) {
    const int64_t k0 = kc * KCH;
    auto xs = [&](int pl, int col, int q) -> const void* {
      int64_t l = (int64_t)LP_SLAB * sl + col;
      l = l < a.p ? l : (int64_t)a.p - 1;                        // columns past p: weight 0
      return V + pl * a.vplane + l * a.ldc + k0 + 8 * q;
    };
    auto ys = [&](int pl, int col, int q) -> const void* {
      return Ac + pl * a.aplane + (int64_t)(a.col0 + col) * a.ldc + k0 + 8 * q;
    };
    lp_dma<KIND, NT, false>(lx, ly, tid, wave, xs, ys);
  };

  // weights of the slab being multiplied, for its owner's epilogue: loaded
  // (clamped, without branches) when the slab begins, so that the loads are
  // long complete when the epilogue needs them
  // (kept as loaded: converting at once would wait for them there)
  double nl[LP_MT][4];
  auto load_nu = [&](int64_t sl) {
#pragma unroll
    for (int m = 0; m < LP_MT; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t l = (int64_t)LP_SLAB * sl + 16 * (LP_MT * wave + m) + 4 * g + v;
        nl[m][v] = a.nu[l < a.p ? l : (int64_t)a.p - 1];
      }
  };

  // end of this block's part of slab sl (chunks kb .. ke-1): publish the
  // partial (not the owner) or merge and run the epilogue (owner)
  auto finish_slab = [&](int64_t sl, int64_t kb, int64_t ke) {
      if (kb > 0) {
        // not the owner: publish this block's partial for the previous block
        float* pp = a.part + blk * PART + (int64_t)wave * (LP_MT * NT * 256);
  #pragma unroll
        for (int m = 0; m < LP_MT; ++m)
  #pragma unroll
          for (int t = 0; t < NT; ++t)
            xput4(pp + ((m * NT + t) * 64 + lane) * 4, acc[m][t]);
        xput_complete();   // each wave's stores are done (visible device-wide)
        __syncthreads();   // ... before the flag is raised
        if (tid == 0) __hip_atomic_store(a.ho.flag + blk, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        // owner (nl holds the slab's weights, loaded when the slab began)
        if (ke < KC) {
          xwait_flag(a.ho.flag + blk + 1, (a.ho.spin >> 31) ? (epoch | 0x40000000) : epoch, a.ho.err,
                     (int)(a.ho.spin & 0x7fffffffu));
          const float* pp = a.part + (blk + 1) * PART + (int64_t)wave * (LP_MT * NT * 256);
  #pragma unroll
          for (int m = 0; m < LP_MT; ++m)
  #pragma unroll
            for (int t = 0; t < NT; ++t) acc[m][t] += xget4v(pp + ((m * NT + t) * 64 + lane) * 4);
          __syncthreads();   // read by every wave; the flag is lowered as in the fp32 / fp64 kernel
          if (tid == 0) __hip_atomic_store(a.ho.flag + blk + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // epilogue: acc[m][t][v] = z at l = lb + v, column col0 + 16 t + c.
        // w = nu z^(d-1) in fp32 (its 16-bit storage rounds far more); the
        // power runs over all of the lane's values at once, and the sum of
        // w z is kept in fp64.
        f4 zp[LP_MT][NT];
#pragma unroll
        for (int m = 0; m < LP_MT; ++m)
#pragma unroll
          for (int t = 0; t < NT; ++t) zp[m][t] = f4{1.0f, 1.0f, 1.0f, 1.0f};
        for (int e = 0; e < dm1; ++e)
#pragma unroll
          for (int m = 0; m < LP_MT; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t) zp[m][t] *= acc[m][t];
        const float ws = (float)a.wscale;
#pragma unroll
        for (int m = 0; m < LP_MT; ++m) {
          const int64_t lb = (int64_t)LP_SLAB * sl + 16 * (LP_MT * wave + m) + 4 * g;
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            E out[PL][4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const float wv = (lb + v < a.p ? (float)nl[m][v] : 0.0f) * zp[m][t][v];
              wsum[t] += (double)wv * (double)acc[m][t][v];
              E parts[PL];
              LpT<KIND>::split(ws * wv, parts);
#pragma unroll
              for (int pl = 0; pl < PL; ++pl) out[pl][v] = parts[pl];
            }
            // W is unit-major: the 8 observations of unit u of column j at
            // (u rp + j) 8; this lane's 4 observations are half of unit lb / 8
            const int64_t col = a.col0 + 16 * t + c;
#pragma unroll
            for (int pl = 0; pl < PL; ++pl) {
              E* dst = (E*)a.W + pl * a.wplane + ((lb >> 3) * a.rp + col) * 8 + (lb & 7);
              uint2 packed;
              __builtin_memcpy(&packed, out[pl], sizeof(packed));
              *reinterpret_cast<uint2*>(dst) = packed;
            }
          }
        }
      }
#pragma unroll
    for (int m = 0; m < LP_MT; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[m][t] = f4{0, 0, 0, 0};
  };

  if (u0 < u1) {
    // the block's (slab, chunk) units in order through one continuous
    // two-stage pipeline (whatever LP_STAGES says for the second product): a
    // slab's epilogue runs while the next chunk (the next slab's first) is
    // already in flight
    // (slab, chunk) of the unit being multiplied and of the next one issued
    int64_t sl = u0 / KC, kc = u0 - sl * KC;
    int64_t isl = sl, ikc = kc;
    auto issue_next = [&](int stage) {
      dma(stage ? lx1 : lx0, stage ? ly1 : ly0, isl, ikc);
      if (++ikc == KC) { ikc = 0; ++isl; }
    };
    issue_next(0);
    int64_t kb = kc;           // first chunk of the current slab segment
    for (int64_t u = u0; u < u1; ++u) {
      const int st = (int)((u - u0) & 1);
      wait_vm<0>();
      __syncthreads();         // chunk u has landed everywhere; the other stage is free
      if (kc == 0) load_nu(sl);
      if (u + 1 < u1) issue_next(st ^ 1);
      lp_compute<KIND, NT>(st ? lx1 : lx0, st ? ly1 : ly0, wave, g, c, acc);
      if (kc == KC - 1 || u + 1 == u1) {
        finish_slab(sl, kb, kc + 1);
        kb = 0;
      }
      if (++kc == KC) { kc = 0; ++sl; }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double s = wsum[t];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (g == 0) a.wpart[(blk * LP_WAVES + wave) * (int64_t)a.rp + a.col0 + 16 * t + c] = s;
  }
  handoff_done(a.ho.epoch, B, epoch);
}

// ---------------------------------------------------------------------------
// gemm1 with the observations streamed straight into registers
// (k_lp_gemm1v): the same product, stream-K split, hand-off and epilogue as
// k_lp_gemm1, but a wave's own observation rows never pass through LDS.  A
// lane loads its 16-byte fragments (8 covariates of one observation, unit
// 4 jg + g of the chunk, for both of its M subtiles) into a ring of
// LP_VRING chunks, LP_VRING - 1 units ahead of the one being multiplied, so
// that several chunks of V are in flight per wave; only the factor copy,
// which all four waves share, is staged in LDS (two stages, loaded through
// registers after the chunk's multiplies).  The compiler places every wait.
// ---------------------------------------------------------------------------
constexpr int LP_VRING = 4;

template <int KIND, int NT>
__global__ __launch_bounds__(256) void k_lp_gemm1v(LpG1Args a) {
  using S = LpStage<KIND, NT>;
  using E = typename LpT<KIND>::E;
  constexpr int PL = S::PL;
  constexpr int KCH = lp_chunk(KIND);
  constexpr int J = S::U / 4;                    // 32-deep k steps per chunk
  constexpr int PART = LP_WAVES * LP_MT * NT * 256;
  constexpr int YPU = 16 * NT * S::U;            // factor units per plane and chunk
  __shared__ u4 ly0[S::YP * 256], ly1[S::YP * 256];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, c = lane & 15;
  const int64_t B = a.nblocks, blk = blockIdx.x;
  const int64_t KC = a.kc_len / KCH;
  const int64_t U = (int64_t)a.nslab * KC;
  const int64_t u0 = blk * U / B, u1 = (blk + 1) * U / B;
  const E* V = (const E*)a.Vc;
  const E* Ac = (const E*)a.Ac;
  const int dm1 = a.d - 1;
  const int epoch = handoff_epoch(a.ho.epoch);

  f4 acc[LP_MT][NT];
#pragma unroll
  for (int m = 0; m < LP_MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = f4{0, 0, 0, 0};
  double wsum[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) wsum[t] = 0.0;

  // V fragments of one unit: [m][jg][plane]
  u4 vr0[LP_MT][J][PL], vr1[LP_MT][J][PL], vr2[LP_MT][J][PL], vr3[LP_MT][J][PL];
  static_assert(LP_VRING == 4, "four ring slots below");
  auto vissue = [&](u4 (&vr)[LP_MT][J][PL], int64_t u) {
    u = u < u1 ? u : u1 - 1;                     // past the block's range: repeat its last unit (unused)
    const int64_t sl = u / KC, kc = u - sl * KC;
#pragma unroll
    for (int m = 0; m < LP_MT; ++m) {
      int64_t l = (int64_t)LP_SLAB * sl + 16 * (LP_MT * wave + m) + c;
      l = l < a.p ? l : (int64_t)a.p - 1;        // observations past p: weight 0
      const E* col = V + l * a.ldc + kc * KCH + 8 * g;
#pragma unroll
      for (int jg = 0; jg < J; ++jg)
#pragma unroll
        for (int pl = 0; pl < PL; ++pl) vr[m][jg][pl] = gload(reinterpret_cast<const u4*>(col + pl * a.vplane + 32 * jg));
    }
  };
  // factor units of one chunk: slot P of a stage holds unit unswz(P)
  u4 ra[S::YP];
  auto aload = [&](int64_t kc) {
    const int64_t k0 = kc * KCH;
#pragma unroll
    for (int i = 0; i < S::YP; ++i) {
      const int P = tid + 256 * i;
      const int PP = P < S::YU ? P : 0;
      const int pl = PP / YPU;
      int col, q;
      S::unswz(PP % YPU, col, q);
      ra[i] = gload(reinterpret_cast<const u4*>(Ac + pl * a.aplane + (int64_t)(a.col0 + col) * a.ldc + k0 + 8 * q));
    }
  };
  auto astore = [&](u4* ly) {
#pragma unroll
    for (int i = 0; i < S::YP; ++i) {
      const int P = tid + 256 * i;
      if (P < S::YU) ly[P] = ra[i];
    }
  };
  auto compute = [&](const u4 (&vr)[LP_MT][J][PL], const u4* ly) {
    u4 fa[2][NT][PL];
    auto frag = [&](int b, int jg) {
      const int q = 4 * jg + g;
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int pl = 0; pl < PL; ++pl) fa[b][t][pl] = ly[pl * YPU + S::swz(16 * t + c, q)];
    };
    frag(0, 0);
#pragma unroll
    for (int jg = 0; jg < J; ++jg) {
      if (jg + 1 < J) frag((jg + 1) & 1, jg + 1);
#pragma unroll
      for (int m = 0; m < LP_MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = LpT<KIND>::mac(vr[m][jg], fa[jg & 1][t], acc[m][t]);
    }
  };

  double nl[LP_MT][4];
  auto load_nu = [&](int64_t sl) {
#pragma unroll
    for (int m = 0; m < LP_MT; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t l = (int64_t)LP_SLAB * sl + 16 * (LP_MT * wave + m) + 4 * g + v;
        nl[m][v] = a.nu[l < a.p ? l : (int64_t)a.p - 1];
      }
  };

  auto finish_slab = [&](int64_t sl, int64_t kb, int64_t ke) {
      if (kb > 0) {
        float* pp = a.part + blk * PART + (int64_t)wave * (LP_MT * NT * 256);
#pragma unroll
        for (int m = 0; m < LP_MT; ++m)
#pragma unroll
          for (int t = 0; t < NT; ++t)
            xput4(pp + ((m * NT + t) * 64 + lane) * 4, acc[m][t]);
        xput_complete();
        __syncthreads();
        if (tid == 0) __hip_atomic_store(a.ho.flag + blk, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        if (ke < KC) {
          xwait_flag(a.ho.flag + blk + 1, (a.ho.spin >> 31) ? (epoch | 0x40000000) : epoch, a.ho.err,
                     (int)(a.ho.spin & 0x7fffffffu));
          const float* pp = a.part + (blk + 1) * PART + (int64_t)wave * (LP_MT * NT * 256);
#pragma unroll
          for (int m = 0; m < LP_MT; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[m][t] += xget4v(pp + ((m * NT + t) * 64 + lane) * 4);
          __syncthreads();
          if (tid == 0) __hip_atomic_store(a.ho.flag + blk + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        f4 zp[LP_MT][NT];
#pragma unroll
        for (int m = 0; m < LP_MT; ++m)
#pragma unroll
          for (int t = 0; t < NT; ++t) zp[m][t] = f4{1.0f, 1.0f, 1.0f, 1.0f};
        for (int e = 0; e < dm1; ++e)
#pragma unroll
          for (int m = 0; m < LP_MT; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t) zp[m][t] *= acc[m][t];
        const float ws = (float)a.wscale;
#pragma unroll
        for (int m = 0; m < LP_MT; ++m) {
          const int64_t lb = (int64_t)LP_SLAB * sl + 16 * (LP_MT * wave + m) + 4 * g;
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            E out[PL][4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const float wv = (lb + v < a.p ? (float)nl[m][v] : 0.0f) * zp[m][t][v];
              wsum[t] += (double)wv * (double)acc[m][t][v];
              E parts[PL];
              LpT<KIND>::split(ws * wv, parts);
#pragma unroll
              for (int pl = 0; pl < PL; ++pl) out[pl][v] = parts[pl];
            }
            const int64_t col = a.col0 + 16 * t + c;
#pragma unroll
            for (int pl = 0; pl < PL; ++pl) {
              E* dst = (E*)a.W + pl * a.wplane + ((lb >> 3) * a.rp + col) * 8 + (lb & 7);
              uint2 packed;
              __builtin_memcpy(&packed, out[pl], sizeof(packed));
              *reinterpret_cast<uint2*>(dst) = packed;
            }
          }
        }
      }
#pragma unroll
    for (int m = 0; m < LP_MT; ++m)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[m][t] = f4{0, 0, 0, 0};
  };

  if (u0 < u1) {
    int64_t sl = u0 / KC, kc = u0 - sl * KC;
    int64_t kb = kc;
    // prologue: the factor chunk of the first unit in stage 0, V of the first three units
    aload(kc);
    vissue(vr0, u0);
    vissue(vr1, u0 + 1);
    vissue(vr2, u0 + 2);
    astore(ly0);
    __syncthreads();
    // one unit: its V in ring slot SLOT, its factor chunk in stage SLOT mod 2
    auto step = [&](int64_t u, u4 (&vcur)[LP_MT][J][PL], u4 (&vnext)[LP_MT][J][PL], u4* lcur, u4* lnext) {
      if (kc == 0) load_nu(sl);
      const bool more = u + 1 < u1;
      const int64_t nsl = kc + 1 == KC ? sl + 1 : sl, nkc = kc + 1 == KC ? 0 : kc + 1;
      if (more) aload(nkc);
      vissue(vnext, u + LP_VRING - 1);
      compute(vcur, lcur);
      if (more) astore(lnext);
      if (kc == KC - 1 || !more) {
        finish_slab(sl, kb, kc + 1);
        kb = 0;
      }
      __syncthreads();   // the next stage is written everywhere; this one is read
      sl = nsl;
      kc = nkc;
    };
    for (int64_t u = u0; u < u1; u += LP_VRING) {
      step(u, vr0, vr3, ly0, ly1);
      if (u + 1 < u1) step(u + 1, vr1, vr0, ly1, ly0);
      if (u + 2 < u1) step(u + 2, vr2, vr1, ly0, ly1);
      if (u + 3 < u1) step(u + 3, vr3, vr2, ly1, ly0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double sm = wsum[t];
    sm += __shfl_xor(sm, 16);
    sm += __shfl_xor(sm, 32);
    if (g == 0) a.wpart[(blk * LP_WAVES + wave) * (int64_t)a.rp + a.col0 + 16 * t + c] = sm;
  }
  handoff_done(a.ho.epoch, B, epoch);
}

// ---------------------------------------------------------------------------
// gemm2: partial Y = V W over one split of the observations, one block per
// (row slab, split), reading Vc; rows past n are zero in Vc and not read
// ---------------------------------------------------------------------------
template <int KIND, int NT>
__global__ __launch_bounds__(256) void k_lp_gemm2(LpG2Args a) {
  using S = LpStage<KIND, NT>;
  using E = typename LpT<KIND>::E;
  constexpr int KCH = lp_chunk(KIND);
  __shared__ u4 lx0[S::XP * 256], lx1[S::XP * 256], lx2[LP_STAGES > 2 ? S::XP * 256 : 1];
  __shared__ u4 ly0[S::YP * 256], ly1[S::YP * 256], ly2[LP_STAGES > 2 ? S::YP * 256 : 1];
  LP_CHUNK_LOOP
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, c = lane & 15;
  // block -> (slab, split): the slabs of one split get ids with the same
  // residue mod 8, so they run on one XCD and share its L2 for W
  const int64_t bid = blockIdx.x;
  const int split = (int)(bid % 8 + 8 * (bid / (8 * (int64_t)a.nslab)));
  const int slab = (int)((bid / 8) % a.nslab);
  if (split >= a.nsplit) return;
  const int64_t KC = a.kr_len / KCH;
  const int64_t kb = (int64_t)split * a.chunks_per_split;
  const int64_t ke = min(KC, kb + a.chunks_per_split);
  const E* Vc = (const E*)a.Vc;
  const E* W = (const E*)a.W;
  f4 acc[LP_MT][NT];
#pragma unroll
  for (int m = 0; m < LP_MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = f4{0, 0, 0, 0};
  auto dma = [&](u4* lx, u4* ly, int64_t kc) {
    const int64_t k0 = kc * KCH;
    // piece (observation k0 + k, covariate unit q of the slab)
    auto xs = [&](int pl, int k, int q) -> const void* {
      return Vc + pl * a.vplane + (k0 + k) * a.ldc + (int64_t)LP_SLAB * slab + 8 * q;
    };
    auto ys = [&](int pl, int col, int q) -> const void* {
      return W + pl * a.wplane + ((k0 >> 3) + q) * (int64_t)a.rp * 8 + (int64_t)(a.col0 + col) * 8;
    };
    lp_dma<KIND, NT, true>(lx, ly, tid, wave, xs, ys);
  };
  const int64_t nk = ke - kb;
  chunk_loop(nk, [&](u4* lx, u4* ly, int64_t q) { dma(lx, ly, kb + q); },
             [&](const u4* lx, const u4* ly) { lp_compute_tr<KIND, NT>(lx, ly, wave, g, c, acc); });
  // acc[m][t][v] = Y[slab rows + 16 (MT wave + m) + 4 g + v][col0 + 16 t + c]
#pragma unroll
  for (int m = 0; m < LP_MT; ++m) {
    const int64_t row = (int64_t)LP_SLAB * slab + 16 * (LP_MT * wave + m) + 4 * g;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      float* col = a.Ypart + ((int64_t)split * a.rp + a.col0 + 16 * t + c) * a.npad;
      *reinterpret_cast<f4*>(col + row) = acc[m][t];
    }
  }
}

// ---------------------------------------------------------------------------
// conversions
// ---------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ void lp_pack_a_blocks(const LpPackArgs& a, int64_t b, int64_t nb) {
  using E = typename LpT<KIND>::E;
  constexpr int PL = LpT<KIND>::PLANES;
  const int64_t total = (int64_t)a.rp * a.kc_len;
  const int64_t bs = blockDim.x;
  for (int64_t e = b * bs + threadIdx.x; e < total; e += nb * bs) {
    const int64_t j = e / a.kc_len, k = e - j * a.kc_len;
    const double x = (k < a.n && j < a.r) ? (double)a.A[j * a.lda + k] : 0.0;
    E parts[PL];
    LpT<KIND>::split(x, parts);
#pragma unroll
    for (int pl = 0; pl < PL; ++pl) ((E*)a.Ac)[pl * a.aplane + j * a.ldc + k] = parts[pl];
  }
}

// the 16-bit copy of A and the Gram tiles of the fp32 A in one launch:
// blocks [0, npack) convert, the rest are Gram tiles
template <int KIND>
__global__ __launch_bounds__(GRAM_THREADS) void k_lp_prep(LpPackArgs pk, int64_t npack, GramArgs<float> gram) {
  __shared__ double lds[GRAM_LDS_DOUBLES];
  const int64_t b = blockIdx.x;
  if (b < npack) {
    lp_pack_a_blocks<KIND>(pk, b, npack);
    return;
  }
  gram_tile(gram, b - npack, lds);
}

// Vc (column-major, ld ldc, kr_len columns) elementwise, zero past n and p
template <int KIND>
__global__ __launch_bounds__(256) void k_lp_conv_c(LpConvArgs a) {
  using E = typename LpT<KIND>::E;
  constexpr int PL = LpT<KIND>::PLANES;
  const int64_t total = a.kr_len * a.kc_len;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t l = e / a.kc_len, k = e - l * a.kc_len;
    const double x = (k < a.n && l < a.p) ? (double)a.V[l * a.ldv + k] : 0.0;
    E parts[PL];
    LpT<KIND>::split(x, parts);
#pragma unroll
    for (int pl = 0; pl < PL; ++pl) ((E*)a.Vc)[pl * a.plane_c + l * a.ldc + k] = parts[pl];
  }
}

__global__ __launch_bounds__(256) void k_max_abs(const double* x, int64_t count, double* out) {
  __shared__ double sm[256];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) m = fmax(m, fabs(x[i]));
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sm[0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {
#ifndef SYMTD_LP_G1V
#define SYMTD_LP_G1V 1
#endif
template <int KIND, int NT>
void g1n(dim3 grid, hipStream_t st, const LpG1Args& a) {
  if (SYMTD_LP_G1V) hipLaunchKernelGGL((k_lp_gemm1v<KIND, NT>), grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL((k_lp_gemm1<KIND, NT>), grid, dim3(256), 0, st, a);
}
template <int KIND>
void g1(int nt, dim3 grid, hipStream_t st, const LpG1Args& a) {
  switch (nt) {
    case 1: g1n<KIND, 1>(grid, st, a); break;
    case 2: g1n<KIND, 2>(grid, st, a); break;
    case 3: g1n<KIND, 3>(grid, st, a); break;
    case 4: g1n<KIND, 4>(grid, st, a); break;
    case 5: g1n<KIND, 5>(grid, st, a); break;
    case 6: g1n<KIND, 6>(grid, st, a); break;
    case 7: g1n<KIND, 7>(grid, st, a); break;
    default: break;
  }
}
template <int KIND>
void g2(int nt, dim3 grid, hipStream_t st, const LpG2Args& a) {
  switch (nt) {
    case 1: hipLaunchKernelGGL((k_lp_gemm2<KIND, 1>), grid, dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_lp_gemm2<KIND, 2>), grid, dim3(256), 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_lp_gemm2<KIND, 3>), grid, dim3(256), 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_lp_gemm2<KIND, 4>), grid, dim3(256), 0, st, a); break;
    case 5: hipLaunchKernelGGL((k_lp_gemm2<KIND, 5>), grid, dim3(256), 0, st, a); break;
    case 6: hipLaunchKernelGGL((k_lp_gemm2<KIND, 6>), grid, dim3(256), 0, st, a); break;
    case 7: hipLaunchKernelGGL((k_lp_gemm2<KIND, 7>), grid, dim3(256), 0, st, a); break;
    default: break;
  }
}
}  // namespace

void launch_lp_gemm1(int kind, int nt, dim3 grid, hipStream_t st, const LpG1Args& a) {
  if (kind == LP_F16) g1<LP_F16>(nt, grid, st, a);
  else g1<LP_BF16X3>(nt, grid, st, a);
}
void launch_lp_gemm2(int kind, int nt, dim3 grid, hipStream_t st, const LpG2Args& a) {
  if (kind == LP_F16) g2<LP_F16>(nt, grid, st, a);
  else g2<LP_BF16X3>(nt, grid, st, a);
}
void launch_lp_prep(int kind, int64_t gram_blocks, hipStream_t st, const LpPackArgs& a, const GramArgs<float>& g) {
  const int64_t total = (int64_t)a.rp * a.kc_len;
  const int64_t npack = std::min<int64_t>((total + GRAM_THREADS - 1) / GRAM_THREADS, 1024);
  const dim3 grid((unsigned)(npack + gram_blocks));
  if (kind == LP_F16) hipLaunchKernelGGL(k_lp_prep<LP_F16>, grid, dim3(GRAM_THREADS), 0, st, a, npack, g);
  else hipLaunchKernelGGL(k_lp_prep<LP_BF16X3>, grid, dim3(GRAM_THREADS), 0, st, a, npack, g);
}
void launch_lp_convert(int kind, hipStream_t st, const LpConvArgs& a) {
  const int64_t total = a.kr_len * a.kc_len;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  if (kind == LP_F16) hipLaunchKernelGGL(k_lp_conv_c<LP_F16>, dim3(blocks), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(k_lp_conv_c<LP_BF16X3>, dim3(blocks), dim3(256), 0, st, a);
}
void launch_max_abs(hipStream_t st, const double* x, int64_t count, double* out) {
  hipLaunchKernelGGL(k_max_abs, dim3(1), dim3(256), 0, st, x, count, out);
}

}  // namespace symtd
