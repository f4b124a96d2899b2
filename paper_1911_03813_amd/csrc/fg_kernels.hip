// Kernels of the objective/gradient evaluation (Algorithm 2, fg_implicit).
//
//   gemm1     Z = V'A on matrix cores, 16 observations (one slab) at a time.
//             Epilogue: W = D_nu Z^{d-1} (eq. (Y) before the outer product),
//             written in a packed layout that gemm2 reads with one coalesced
//             vector load per lane, and fp64 column sums of nu_l z_lj^d
//             (= w_j by Lemmas 3.2 and 3.5), one partial row per wave.
//   gemm2     Y = V W on matrix cores, split over the observations; each split
//             writes its own partial Y (no atomics, fixed reduction order).
//   gram_part / gram_fin   B = A'A in fp64 (split over rows, then summed),
//             C = B^{d-1}.
//   ymodel    Y_M = A D_lambda C in fp64 (the model's own TTSVs, M a_j^{d-1}).
//   final_s / final_f   w = fixed-order sum of the column partials,
//             u = (B*C) lambda, g_lambda = -2 (w - u),
//             f = alpha + lambda'u - 2 w'lambda.
//   final_G   G_A = -2d (Y - Y_M) D_lambda with Y the fixed-order fp64 sum of
//             the gemm2 partials.
//
// Packed W layout: element (l, j) with l = 16*b + row(g, s) and j = 16*t + c
// lives at ((b * nt_tot + t) * 64 + 16*g + c) * 4 + s, where row(g, s) is the
// MFMA output row of lane group g, element s (Mfma<T>::row).  That is exactly
// the order in which gemm1's accumulator registers come out, and exactly the
// B-operand order gemm2 needs when its k index at step s is
// l = 16*b + row(g, s).  Rows l >= p hold zeros (their weight nu is zero).
#include <type_traits>

#include "kcommon.hpp"
#include "kernels.hpp"
#include "model_dev.hpp"

namespace symtd {

// ---------------------------------------------------------------------------
// gemm1 + epilogue
//
// A block of NW = g1_waves<T>() waves works in lockstep on one slab of
// 16*MT*NW observations (16*MT per wave, MT = g1_mt<T>()).  The k range (the n covariates) is cut into
// chunks of KCH = 4*QPC; for every chunk the block moves the slab's
// observation columns and the factor columns into LDS, each column as one
// contiguous run of g1_run<T>() bytes (QPC quads of 4 elements), and the waves read
// their MFMA fragments from LDS.  LDS holds a column's quads at a swizzled
// slot (quad q of column col at col*QPC + (q ^ (col mod QPC))), so the 16
// columns of one fragment read fall in distinct banks.
//
// When the observations are 16-byte aligned with n a multiple of 4, the
// chunk's 16-byte pieces go from global memory straight into LDS
// (global_load_lds), issued by the first g1_dma_waves<T>() waves (all when
// 0): every lane of those fetches the piece whose LDS slot is its own, and
// each of their threads issues the same number of pieces per chunk, so a
// wave can wait for exactly one chunk with vmcnt (the other waves have
// nothing in flight; the stage barrier publishes the pieces to them).  Chunks rotate through g1_stages<T>()
// LDS stages: with two, the next chunk is in flight while one is multiplied
// (with three, the next two).  Other
// layouts pass through registers with two stages.  The factors are read from
// a zero-padded copy (Apad) so that they never need masking.
//
// The (slab, chunk) pairs are numbered slab-major and every block takes one
// contiguous range of them (stream-K), so all blocks get the same work to
// within one chunk.  There are never more blocks than slabs, so a slab is
// shared by at most two blocks: the block holding its first chunks owns it;
// the block holding its last chunks (at the start of its range) publishes
// that partial accumulator through `part` and raises its flag to the
// launch's epoch; the owner, which reaches the slab at the end of its own
// range, waits for that value, adds the partial and runs the epilogue.  A
// block waits only after its own work, and only for its successor, which
// publishes before it waits for anything, so the wait ends once the
// successor has run.  There are never more blocks than compute units and a
// block fits one, so on a device the launch has to itself all blocks are
// resident together; work on another stream holding compute units could
// delay a successor, so a spin limit bounds the wait and a give-up is
// reported through the context's error word (Handoff).
// ---------------------------------------------------------------------------
template <typename T>
struct G1Shape {
  static constexpr int QPC = g1_run<T>() / (4 * (int)sizeof(T));   // quads per column per chunk
  static constexpr int KCH = 4 * QPC;                         // k values per chunk
};

// s_waitcnt immediate that waits until at most `n` vector-memory operations
// of this wave are outstanding (other counters untouched).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

template <typename T, int NT, bool DMA, bool NARROW>
__global__ __launch_bounds__(64 * g1_waves<T>()) void k_gemm1(G1Args<T> a) {
  using acc_t = typename Mfma<T>::acc_t;
  constexpr int NW = g1_waves<T>();
  constexpr int MT = g1_mt<T>();
  constexpr int NTH = 64 * NW;
  constexpr int NS = g1_stages<T>();
  constexpr int QPC = G1Shape<T>::QPC;
  constexpr int KCH = G1Shape<T>::KCH;
  constexpr int H = (int)sizeof(T) / 4;          // 16-byte pieces per quad
  constexpr int VCOLS = 16 * MT * NW;            // observation columns of a block slab
  constexpr int VQ = VCOLS * QPC;                // quads of a chunk
  constexpr int AQ = 16 * NT * QPC;
  // the first DW waves move the chunks (one per SIMD when DW = NW / 2, so
  // that the other wave on each SIMD keeps multiplying while they issue)
  constexpr int DW = (g1_dma_waves<T>() > 0 && g1_dma_waves<T>() < NW) ? g1_dma_waves<T>() : NW;
  constexpr int DT = 64 * DW;                    // threads that move chunks
  constexpr int VP = (VQ * H + DT - 1) / DT;     // 16-byte pieces per moving thread and chunk
  constexpr int AP = (AQ * H + DT - 1) / DT;
  constexpr int DPC = VP + AP;                   // DMA instructions per thread and chunk
  constexpr int PART = NW * MT * NT * 4 * 64;    // elements of one block's published partial
  static_assert(NS == 2 || NS == 3, "the chunk loop below is written for two or three stages");
  static_assert(QPC >= 4 && (QPC & (QPC - 1)) == 0, "chunk run length");
  // NARROW: the launch's last column subtile holds at most 4 factor columns
  // (the rest is zero padding) and is multiplied on the narrow form
  // (Narrow<T>), a quarter of the matrix work of a 16x16x4 subtile; its
  // accumulator is acc[m][NT - 1]: element 0 in fp64 (the other three stay
  // zero), all four in fp32 (one lane group's share, see Narrow<float>)
  constexpr int NF = NARROW ? NT - 1 : NT;       // column subtiles on the 16x16x4 form
  // LDS stages as distinct objects, so that the compiler can tell the loads
  // filling one stage from the reads of another; each is padded to whole
  // rounds of pieces so that every thread moves the same number of them
  constexpr int LVQ = DMA ? VP * DT / H : VQ, LAQ = DMA ? AP * DT / H : AQ;
  __shared__ Quad<T> lv0[LVQ], lv1[LVQ], lv2[NS > 2 ? LVQ : 1];
  __shared__ Quad<T> la0[LAQ], la1[LAQ], la2[NS > 2 ? LAQ : 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  const int g = lane >> 4, c = lane & 15;
  const int64_t B = a.nblocks;
  const int64_t blk = blockIdx.x;
  const int64_t n = a.n;
  const int64_t KC = (n + KCH - 1) / KCH;        // chunks per slab (the last may be ragged)
  const int64_t U = (int64_t)a.nslab * KC;
  const int64_t u0 = blk * U / B, u1 = (blk + 1) * U / B;
  const int tg = a.col0 >> 4;
  const int dm1 = a.d - 1;
  const int epoch = handoff_epoch(a.ho.epoch);

  acc_t acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = acc_t{0, 0, 0, 0};
  double wsum[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) wsum[t] = 0.0;

  auto swz = [](int col, int q) { return col * QPC + (q ^ (col & (QPC - 1))); };
  auto unswz = [](int P, int& col, int& q) { col = P / QPC; q = (P % QPC) ^ (col & (QPC - 1)); };
  auto vcolumn = [&](int64_t sl, int col) {
    int64_t l = (int64_t)VCOLS * sl + col;
    return a.V + (l < a.p ? l : (int64_t)a.p - 1) * a.ldv;    // columns past p: weight 0
  };

  // DMA of chunk kc of slab sl into one stage (same instruction count on every thread)
  auto dma = [&](Quad<T>* lv, Quad<T>* la, int64_t sl, int64_t kc) {
    if (DW < NW && wave >= DW) return;            // wave-uniform
    const int64_t k0 = kc * KCH;
#pragma unroll
    for (int i = 0; i < VP; ++i) {
      const int P16 = tid + DT * i;
      const T* src = a.V;                         // padding pieces: any valid address
      if (P16 < VQ * H) {
        int col, q;
        unswz(P16 / H, col, q);
        int64_t k = k0 + 4 * q;
        k = k + 3 < n ? k : n - 4;                // whole quads past n: any valid quad
        src = vcolumn(sl, col) + k + (P16 % H) * (4 / H);
      }
      __builtin_amdgcn_global_load_lds((const void*)src,
          (__attribute__((address_space(3))) void*)((char*)lv + 16 * (DT * i + 64 * wave)), 16, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < AP; ++i) {
      const int P16 = tid + DT * i;
      const T* src = a.Apad;
      if (P16 < AQ * H) {
        int col, q;
        unswz(P16 / H, col, q);
        src = a.Apad + (int64_t)(a.col0 + col) * a.ldap + k0 + 4 * q + (P16 % H) * (4 / H);
      }
      __builtin_amdgcn_global_load_lds((const void*)src,
          (__attribute__((address_space(3))) void*)((char*)la + 16 * (DT * i + 64 * wave)), 16, 0, 0);
    }
  };

  // register path (any alignment): global -> registers -> LDS, two stages
  constexpr int VQT = (VQ + NTH - 1) / NTH, AQT = (AQ + NTH - 1) / NTH;
  Quad<T> rv[DMA ? 1 : VQT], ra[DMA ? 1 : AQT];
  auto gload = [&](int64_t sl, int64_t kc) {
    const int64_t k0 = kc * KCH;
    const bool rag = k0 + KCH > n;
#pragma unroll
    for (int i = 0; i < (DMA ? 0 : VQT); ++i) {
      const int P = tid + NTH * i;
      if (P < VQ) {
        const int col = P / QPC, q = P % QPC;
        const T* src = vcolumn(sl, col);
        const int64_t k = k0 + 4 * q;
        if (!rag) { rv[i].e[0] = src[k]; rv[i].e[1] = src[k + 1]; rv[i].e[2] = src[k + 2]; rv[i].e[3] = src[k + 3]; }
        else load_tail(rv[i], src, k, n);
      }
    }
#pragma unroll
    for (int i = 0; i < (DMA ? 0 : AQT); ++i) {
      const int P = tid + NTH * i;
      if (P < AQ) {
        const int col = P / QPC, q = P % QPC;
        vload4(ra[i], a.Apad + (int64_t)(a.col0 + col) * a.ldap + k0 + 4 * q);
      }
    }
  };
  auto lstore = [&](Quad<T>* lv, Quad<T>* la) {
#pragma unroll
    for (int i = 0; i < (DMA ? 0 : VQT); ++i) {
      const int P = tid + NTH * i;
      if (P < VQ) lv[swz(P / QPC, P % QPC)] = rv[i];
    }
#pragma unroll
    for (int i = 0; i < (DMA ? 0 : AQT); ++i) {
      const int P = tid + NTH * i;
      if (P < AQ) la[swz(P / QPC, P % QPC)] = ra[i];
    }
  };

  // multiply one chunk held in an LDS stage; the fragments of 16-k group jg+1
  // are read from LDS while group jg is multiplied
  auto compute = [&](const Quad<T>* lv, const Quad<T>* la) {
    constexpr int J = QPC / 4;
    Quad<T> fv[2][MT], fa[2][NT];
    auto frag = [&](int b, int jg) {
      const int q = 4 * jg + g;            // this lane's quad: k = k0 + 16 jg + 4 g + s
#pragma unroll
      for (int m = 0; m < MT; ++m) fv[b][m] = lv[swz(16 * (MT * wave + m) + c, q)];
#pragma unroll
      for (int t = 0; t < NF; ++t) fa[b][t] = la[swz(16 * t + c, q)];
      if constexpr (NARROW) fa[b][NT - 1] = la[swz(16 * (NT - 1) + (c & 3), q)];
    };
    auto mfma = [&](int b) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int m = 0; m < MT; ++m) {
#pragma unroll
          for (int t = 0; t < NF; ++t) acc[m][t] = Mfma<T>::mac(fv[b][m].e[s], fa[b][t].e[s], acc[m][t]);
          if constexpr (NARROW) {
            if constexpr (sizeof(T) == 8)
              acc[m][NT - 1][0] = Narrow<T>::mac(fv[b][m].e[s], fa[b][NT - 1].e[s], acc[m][NT - 1][0]);
            else
              acc[m][NT - 1] = Narrow<T>::mac(fv[b][m].e[s], fa[b][NT - 1].e[s], acc[m][NT - 1]);
          }
        }
    };
    frag(0, 0);
#pragma unroll
    for (int jg = 0; jg < J; ++jg) {
      if (jg + 1 < J) frag((jg + 1) & 1, jg + 1);
      mfma(jg & 1);
    }
  };
  // a slab's last chunk when n is not a whole number of chunks: only its
  // first jlast 16-k groups reach covariates below n (the rest would
  // multiply the factor copy's zero rows), so only those are multiplied
  // (fp64; in fp32 the extra body costs the chunk loop registers)
  constexpr int JG = QPC / 4;
  const int jlast = (int)((n - (KC - 1) * KCH + 15) / 16);
  auto compute_last = [&](const Quad<T>* lv, const Quad<T>* la) {
    for (int jg = 0; jg < jlast; ++jg) {
      const int q = 4 * jg + g;
      Quad<T> fv[MT], fa[NT];
#pragma unroll
      for (int m = 0; m < MT; ++m) fv[m] = lv[swz(16 * (MT * wave + m) + c, q)];
#pragma unroll
      for (int t = 0; t < NF; ++t) fa[t] = la[swz(16 * t + c, q)];
      if constexpr (NARROW) fa[NT - 1] = la[swz(16 * (NT - 1) + (c & 3), q)];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int m = 0; m < MT; ++m) {
#pragma unroll
          for (int t = 0; t < NF; ++t) acc[m][t] = Mfma<T>::mac(fv[m].e[s], fa[t].e[s], acc[m][t]);
          if constexpr (NARROW) {
            if constexpr (sizeof(T) == 8)
              acc[m][NT - 1][0] = Narrow<T>::mac(fv[m].e[s], fa[NT - 1].e[s], acc[m][NT - 1][0]);
            else
              acc[m][NT - 1] = Narrow<T>::mac(fv[m].e[s], fa[NT - 1].e[s], acc[m][NT - 1]);
          }
        }
    }
  };
  // chunk kc of a slab, through the shortened product when it is the ragged last one
  auto compute_chunk = [&](const Quad<T>* lv, const Quad<T>* la, int64_t kc) {
    if (sizeof(T) == 8 && kc == KC - 1 && jlast < JG) compute_last(lv, la);
    else compute(lv, la);
  };
  // wait until chunk kc (with `later` chunks issued after it) has landed, then
  // the block-wide barrier: everyone's pieces are in, and the stage read in the
  // previous step is free again
  auto arrive = [&](int later) {
    if (later >= 1) wait_vm<DPC>();
    else wait_vm<0>();
    __syncthreads();
  };

  // weights of the slab being multiplied, for its owner's epilogue: loaded
  // (clamped, without branches) when the slab begins and kept as loaded, so
  // that they arrive with the slab's first chunk
  double nlr[MT][4];
  auto load_nu = [&](int64_t sl) {
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t l = 16 * ((int64_t)NW * MT * sl + MT * wave + m) + Mfma<T>::row(g, v);
        nlr[m][v] = a.nu[l < a.p ? l : (int64_t)a.p - 1];
      }
  };

  if (u0 < u1) {
    int64_t sl = u0 / KC, kb = u0 - sl * KC;
    const int64_t sl_last = (u1 - 1) / KC;
    while (true) {
      const int64_t ke = (sl == sl_last) ? u1 - sl * KC : KC;
      const int64_t nk = ke - kb;
      if (kb == 0) load_nu(sl);
      if constexpr (DMA) {
        if constexpr (NS == 3) {
          // chunk kb+q lives in stage q mod 3
          dma(lv0, la0, sl, kb);
          if (nk > 1) dma(lv1, la1, sl, kb + 1);
          int64_t q = 0;
          for (; q + 3 <= nk; q += 3) {
            arrive((int)min((int64_t)1, nk - 1 - q));
            if (q + 2 < nk) dma(lv2, la2, sl, kb + q + 2);
            compute(lv0, la0);
            arrive((int)min((int64_t)1, nk - 2 - q));
            if (q + 3 < nk) dma(lv0, la0, sl, kb + q + 3);
            compute(lv1, la1);
            arrive((int)min((int64_t)1, nk - 3 - q));
            if (q + 4 < nk) dma(lv1, la1, sl, kb + q + 4);
            compute(lv2, la2);
          }
          // fewer than three chunks remain, in stages 0, 1
          if (q < nk) { arrive((int)min((int64_t)1, nk - 1 - q)); compute(lv0, la0); }
          if (q + 1 < nk) { arrive(0); compute(lv1, la1); }
        } else {
          // chunk kb+q lives in stage q mod 2
          dma(lv0, la0, sl, kb);
          int64_t q = 0;
          for (; q + 2 <= nk; q += 2) {
            arrive(0);
            dma(lv1, la1, sl, kb + q + 1);
            compute(lv0, la0);
            arrive(0);
            if (q + 2 < nk) dma(lv0, la0, sl, kb + q + 2);
            compute_chunk(lv1, la1, kb + q + 1);
          }
          if (q < nk) { arrive(0); compute_chunk(lv0, la0, kb + q); }
        }
      } else {
        gload(sl, kb);
        lstore(lv0, la0);
        __syncthreads();
        int64_t kc = kb;
        for (; kc + 1 < ke; kc += 2) {
          gload(sl, kc + 1);
          compute(lv0, la0);
          lstore(lv1, la1);
          __syncthreads();
          if (kc + 2 < ke) gload(sl, kc + 2);
          compute(lv1, la1);
          if (kc + 2 < ke) lstore(lv0, la0);
          __syncthreads();
        }
        if (kc < ke) compute(lv0, la0);
      }
      __syncthreads();   // every stage is read before the next slab overwrites it

      if (kb > 0) {
        // not the owner: publish this block's partial for the previous block
        T* pp = a.part + opaque_uniform(blk) * PART + (int64_t)wave * (MT * NT * 4 * 64);
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            Quad<T> q4;
#pragma unroll
            for (int v = 0; v < 4; ++v) q4.e[v] = acc[m][t][v];
            xput4(pp + ((m * NT + t) * 64 + lane) * 4, q4);
          }
        xput_complete();   // each wave's stores are done (visible device-wide)
        __syncthreads();   // ... before the flag is raised
        if (tid == 0) __hip_atomic_store(a.ho.flag + blk, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        if (ke < KC) {
          // the next block holds chunks [ke, KC) of this slab
          xwait_flag(a.ho.flag + blk + 1, (a.ho.spin >> 31) ? (epoch | 0x40000000) : epoch, a.ho.err,
                     (int)(a.ho.spin & 0x7fffffffu));
          const T* pp = a.part + opaque_uniform(blk + 1) * PART + (int64_t)wave * (MT * NT * 4 * 64);
#pragma unroll
          for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
              Quad<T> q4;
              xget4(q4, pp + ((m * NT + t) * 64 + lane) * 4);
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[m][t][v] += q4.e[v];
            }
          // every wave has read the partial; the flag is lowered (the epoch
          // tags do not need it, but with the store in place the compiler
          // does not overlap the partial's loads with the epilogue, which
          // made the fp64 kernel spill 59 registers)
          __syncthreads();
          if (tid == 0) __hip_atomic_store(a.ho.flag + blk + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // epilogue: acc[m][t][v] = z at l = 16 b + row(g, v), j = col0 + 16t + c.
        // w = nu z^(d-1) in the storage precision, the power taken over all
        // of the lane's values at once (the exponent loop outside, so that
        // the products are independent); the sums of w z in fp64.  nlr holds
        // the slab's weights, loaded when the slab began.
        acc_t zp[MT][NT];
#pragma unroll
        for (int m = 0; m < MT; ++m)
#pragma unroll
          for (int t = 0; t < NT; ++t) zp[m][t] = acc_t{1, 1, 1, 1};
        for (int e = 0; e < dm1; ++e)
#pragma unroll
          for (int m = 0; m < MT; ++m)
#pragma unroll
            for (int t = 0; t < NT; ++t) zp[m][t] *= acc[m][t];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          const int64_t b = (int64_t)NW * MT * sl + MT * wave + m;   // 16-observation block
          T nl[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) nl[v] = 16 * b + Mfma<T>::row(g, v) < a.p ? (T)nlr[m][v] : T(0);
#pragma unroll
          for (int t = 0; t < NF; ++t) {
            Quad<T> wq;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const T wv = nl[v] * zp[m][t][v];
              wq.e[v] = wv;
              wsum[t] += (double)wv * (double)acc[m][t][v];
            }
            if (b < a.nblk) vstore4(a.Wp + (((b * a.nt_tot + tg + t) * 64) + lane) * 4, wq);
          }
          if constexpr (NARROW && sizeof(T) == 8) {
            // lane (g, c) holds z at observation 16 b + 4 (c / 4) + g, which is
            // row(g, v) with v = c / 4, and column c mod 4 of the subtile: its
            // w goes to element v of packed quad (g, c mod 4); the quads of
            // the padding columns (c >= 4) are written as zeros
            const int v = c >> 2;
            const T nv = v == 0 ? nl[0] : v == 1 ? nl[1] : v == 2 ? nl[2] : nl[3];
            const T wv = nv * zp[m][NT - 1][0];
            wsum[NT - 1] += (double)wv * (double)acc[m][NT - 1][0];
            if (b < a.nblk) {
              T* wb = a.Wp + ((b * a.nt_tot + tg + NT - 1) * 64 + 16 * g) * 4;
              gstore(wb + (c & 3) * 4 + v, wv);
              if (c >= 4) {
                Quad<T> zq;
                zero4(zq);
                vstore4(wb + c * 4, zq);
              }
            }
          } else if constexpr (NARROW) {
            // the four lane groups' shares add up to z at observations
            // 16 b + 4 (c / 4) + x (element x), column c mod 4; with the fp32
            // row(g, v) = 4 g + v these rows are packed quad (c / 4, c mod 4),
            // which the lanes of group 0 write (their weights loaded here);
            // the quads of the padding columns (c >= 4) are written as zeros
            acc_t z = acc[m][NT - 1];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
              z[x] += __shfl_xor(z[x], 16);
              z[x] += __shfl_xor(z[x], 32);
            }
            T* wb = a.Wp + (b * a.nt_tot + tg + NT - 1) * 64 * 4;
            if (g == 0) {
              Quad<T> wq;
#pragma unroll
              for (int x = 0; x < 4; ++x) {
                const int64_t l = 16 * b + 4 * (c >> 2) + x;
                const T nv = l < a.p ? (T)a.nu[l] : T(0);
                T zp1 = T(1);
                for (int e = 0; e < dm1; ++e) zp1 *= z[x];
                wq.e[x] = nv * zp1;
                wsum[NT - 1] += (double)wq.e[x] * (double)z[x];
              }
              if (b < a.nblk) vstore4(wb + (16 * (c >> 2) + (c & 3)) * 4, wq);
            }
            if (c >= 4 && b < a.nblk) {
              Quad<T> zq;
              zero4(zq);
              vstore4(wb + (16 * g + c) * 4, zq);
            }
          }
        }
      }
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = acc_t{0, 0, 0, 0};
      if (sl == sl_last) break;
      ++sl;
      kb = 0;
    }
  }

  // this wave's column sums: across the four lane groups, then one row of wpart
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double s = wsum[t];
    const bool nar = NARROW && t == NT - 1;
    if (nar) {
      // the narrow subtile's column is c mod 4: first across the lanes c, c ^ 4, c ^ 8, c ^ 12
      s += __shfl_xor(s, 4);
      s += __shfl_xor(s, 8);
    }
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (g == 0) a.wpart[(blk * NW + wave) * (int64_t)a.rp + a.col0 + 16 * t + c] = nar && c >= 4 ? 0.0 : s;
  }
  handoff_done(a.ho.epoch, B, epoch);
}

// ---------------------------------------------------------------------------
// gemm2: partial Y = V W over one split of the observations
// ---------------------------------------------------------------------------
template <typename T, int NT, int NS, bool VEC, bool NARROW>
__global__ __launch_bounds__(256) void k_gemm2(G2Args<T> a) {
  using acc_t = typename Mfma<T>::acc_t;
  // NARROW: the last column subtile holds at most 4 columns of W and runs on
  // the narrow form (Narrow<T>) into accn[m]; lane (g, c) loads the W quad
  // of column c mod 4
  constexpr int NF = NARROW ? NT - 1 : NT;
  // Block -> (row block x, split y).  Consecutive block ids go to different
  // XCDs (id mod 8), so the row blocks of one split get ids with the same
  // residue mod 8: they run on one XCD and share the W slabs in its L2.
  const int64_t bid = blockIdx.x;
  const int RB = a.rowblocks;
  const int y = (int)(bid % 8 + 8 * (bid / (8 * RB)));
  const int x = (int)((bid / 8) % RB);
  if (y >= a.nsplit) return;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int g = lane >> 4, c = lane & 15;
  const int64_t ibase = (int64_t)x * 256 + wave * 64;
  const int64_t n = a.n;
  // this lane's 4 rows (one per M subtile); rows past n are clamped to valid
  // ones and their results are never read back (VEC needs n % 4 == 0, so a
  // quad is wholly inside or wholly past n; otherwise each element is clamped)
  const int64_t il = ibase + 4 * c;
  const int64_t ilc = (il < n) ? il : n - 4;

  const int64_t b0 = (int64_t)y * a.blk_per_split;
  const int64_t b1 = min((int64_t)a.nblk, b0 + a.blk_per_split);
  const int tg = a.col0 >> 4;

  acc_t acc[4][NF > 0 ? NF : 1];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int t = 0; t < NF; ++t) acc[m][t] = acc_t{0, 0, 0, 0};
  using nacc_t = typename Narrow<T>::acc_t;
  nacc_t accn[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) accn[m] = nacc_t{0};
  // the narrow accumulators stay in AGPRs beside the others (left to the
  // compiler, they move to VGPRs and back every iteration)
  auto pin_narrow = [&]() {
    if constexpr (NARROW) {
#pragma unroll
      for (int m = 0; m < 4; ++m) asm("" : "+a"(accn[m]));
    }
  };
  pin_narrow();

  Quad<T> vb[NS][4];
  Quad<T> wb[NS][NT];
  auto issue = [&](int buf, int64_t b) {
#pragma unroll
    for (int t = 0; t < NF; ++t) vload4(wb[buf][t], a.Wp + (((b * a.nt_tot + tg + t) * 64) + lane) * 4);
    if constexpr (NARROW)
      vload4(wb[buf][NT - 1], a.Wp + (((b * a.nt_tot + tg + NT - 1) * 64) + 16 * g + (c & 3)) * 4);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int64_t l = 16 * b + Mfma<T>::row(g, s);
      l = l < a.p ? l : (int64_t)a.p - 1;     // zero rows of W: contribute nothing
      const T* col = a.V + l * a.ldv;
      if constexpr (VEC) {
        vload4(vb[buf][s], col + ilc);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) vb[buf][s].e[e] = col[min(il + e, n - 1)];
      }
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int t = 0; t < NF; ++t) acc[m][t] = Mfma<T>::mac(vb[buf][s].e[m], wb[buf][t].e[s], acc[m][t]);
        if constexpr (NARROW) accn[m] = Narrow<T>::mac(vb[buf][s].e[m], wb[buf][NT - 1].e[s], accn[m]);
      }
    pin_narrow();
  };

  const int64_t Q = b1 - b0;
  if (Q > 0) {
#pragma unroll
    for (int s = 0; s < NS - 1; ++s) issue(s, b0 + min((int64_t)s, Q - 1));
    int64_t qb = 0;
    for (; qb + NS <= Q; qb += NS) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        issue((s + NS - 1) % NS, b0 + min(qb + s + NS - 1, Q - 1));
        compute(s);
        if constexpr (sizeof(T) == 4 && VEC) {
          // keep each step's loads ahead of its multiplies: left alone, the
          // scheduler sinks the last step's loads to the end of the loop,
          // which halves the distance they have to arrive
          __builtin_amdgcn_sched_group_barrier(0x020, NT + 4, 0);   // vector-memory reads
          __builtin_amdgcn_sched_group_barrier(0x008, 16 * NT, 0);  // MFMAs
        }
      }
    }
#pragma unroll
    for (int s = 0; s < NS - 1; ++s)
      if (s < Q - qb) compute(s);
  }

  // acc[m][t][v] = Y[ibase + 4 row(g, v) + m][col0 + 16t + c]
#pragma unroll
  for (int t = 0; t < NF; ++t) {
    T* col = a.Ypart + ((int64_t)y * a.rp + a.col0 + 16 * t + c) * a.npad;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Quad<T> q;
#pragma unroll
      for (int m = 0; m < 4; ++m) q.e[m] = acc[m][t][v];
      vstore4(col + ibase + 4 * Mfma<T>::row(g, v), q);
    }
  }
  // the narrow subtile: the padding columns of Y are not written (the
  // closing step reads columns below r only)
  if constexpr (NARROW && sizeof(T) == 8) {
    // accn[m] = Y[ibase + 4 (4 (c / 4) + g) + m][col0 + 16 (NT - 1) + c mod 4]
    T* col = a.Ypart + ((int64_t)y * a.rp + a.col0 + 16 * (NT - 1) + (c & 3)) * a.npad;
    Quad<T> q;
#pragma unroll
    for (int m = 0; m < 4; ++m) q.e[m] = (T)accn[m];
    vstore4(col + ibase + 4 * (4 * (c >> 2) + g), q);
  } else if constexpr (NARROW) {
    // summed over the four lane groups, accn[m][x] = Y[ibase + 4 (4 (c / 4) + x) + m]
    // [col0 + 16 (NT - 1) + c mod 4]; the lanes of group 0 write them
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        accn[m][x] += __shfl_xor(accn[m][x], 16);
        accn[m][x] += __shfl_xor(accn[m][x], 32);
      }
    if (g == 0) {
      T* col = a.Ypart + ((int64_t)y * a.rp + a.col0 + 16 * (NT - 1) + (c & 3)) * a.npad;
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        Quad<T> q;
#pragma unroll
        for (int m = 0; m < 4; ++m) q.e[m] = accn[m][x];
        vstore4(col + ibase + 4 * (4 * (c >> 2) + x), q);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// prep: Apad[j][k] = A[k][j] for k < n, j < r, and 0 elsewhere (column-major,
// leading dimension ldap = whole gemm1 chunks, rp columns), and the Gram
// tiles of B = A'A, C = B^{d-1} (gram_tile, model_dev.hpp), in one launch of
// 1024-thread blocks.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void pack_a_block(const PackAArgs<T>& a, int64_t bx, int j) {
  const int64_t k = bx * GRAM_THREADS + threadIdx.x;
  if (k >= a.ldap) return;
  a.Apad[(int64_t)j * a.ldap + k] = (k < a.n && j < a.r) ? a.A[(int64_t)j * a.lda + k] : T(0);
}

template <typename T>
__global__ __launch_bounds__(GRAM_THREADS) void k_prep(PrepArgs<T> a) {
  __shared__ double lds[GRAM_LDS_DOUBLES];
  const int64_t b = blockIdx.x;
  if (b < a.npack) {
    pack_a_block(a.pack, b % a.npack_x, (int)(b / a.npack_x));
    return;
  }
  gram_tile(a.gram, b - a.npack, lds);
}

// ---------------------------------------------------------------------------
// final: the closing step of an evaluation in one launch of 1024-thread
// blocks, each kind of block needing about one round trip to memory.
//   blocks [0, ntile): a 64 x 8 tile of G_A = -2d (Y - Y_M) D_lambda, one
//     element per thread, with Y the fixed-order sum of the second product's
//     partials (their loads issued first) and Y_M = A D_lambda C computed in
//     place from LDS copies of up to FINAL_K columns of A and rows of
//     D_lambda C at a time;
//   blocks [ntile, ntile + ng r): column J: g_lambda[J] = -2 (w_J - u_J)
//     with w_J the sum of the first product's column partials and
//     u_J = sum_k B_kJ C_kJ lambda_k, and J's share lambda_J (u_J - 2 w_J)
//     of f; the last column block of a model to arrive (an arrival counter
//     per model, back at zero after every launch) adds alpha and the shares
//     in column order into that model's f.  The shares move between blocks
//     through device-coherent accesses.
// ---------------------------------------------------------------------------
// partials of Y whose loads are issued before Y_M is computed (128 bytes of
// registers per thread)
template <typename T> constexpr int final_pf() { return 128 / (int)sizeof(T); }
constexpr int FINAL_K = 128;    // k values of A D_lambda and C staged in LDS at once

__device__ __forceinline__ double block_sum(double v, double* sm) {
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int s = FINAL_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sm[0];
  __syncthreads();
  return r;
}

// Y_M[i0 + tr][j0 + tc] of model grp (tr = thread % 64, tc = thread / 64 <
// FINAL_COLS), fp64: sum over k of A[i][k] (lambda_k C[k][j]), in four
// interleaved partial sums (k mod 4) added at the end.  A slice of up to
// FINAL_K values of k moves to LDS in two steps: ym_load issues every load of
// the slice and uses none, ym_use stores the slice and multiplies it in; the
// caller can issue its own loads in between so that they overlap.  (All
// array indices are static, so that nothing leaves registers.)
constexpr int YM_ITA = FINAL_K * 64 / FINAL_THREADS;
constexpr int YM_ITC = (FINAL_K * FINAL_COLS + FINAL_THREADS - 1) / FINAL_THREADS;

template <typename T>
__device__ __forceinline__ void ym_load(const T* Ag, int64_t lda, int n, int r, const double* lg, const double* Cg,
                                        int64_t i0, int j0, int k0, T (&xa)[YM_ITA], double (&xc)[YM_ITC],
                                        double (&xl)[YM_ITC]) {
  const int kn = min(FINAL_K, r - k0);
#pragma unroll
  for (int it = 0; it < YM_ITA; ++it) {
    const int e = threadIdx.x + it * FINAL_THREADS;
    const int ii = e & 63, kk = min(e >> 6, kn - 1);
    const int64_t i = i0 + ii;
    xa[it] = Ag[(int64_t)(k0 + kk) * lda + (i < n ? i : 0)];
  }
#pragma unroll
  for (int it = 0; it < YM_ITC; ++it) {
    const int e = threadIdx.x + it * FINAL_THREADS;
    const int cc = e % FINAL_COLS, kk = min(e / FINAL_COLS, kn - 1), j = j0 + cc;
    xc[it] = Cg[(int64_t)(j < r ? j : 0) * r + k0 + kk];
    xl[it] = lg[k0 + kk];
  }
}

template <typename T>
__device__ __forceinline__ void ym_use(int n, int r, int64_t i0, int j0, int k0, const T (&xa)[YM_ITA],
                                       const double (&xc)[YM_ITC], const double (&xl)[YM_ITC], double (*sa)[65],
                                       double (*sc)[FINAL_COLS + 1], double (&acc)[4]) {
  const int kn = min(FINAL_K, r - k0);
#pragma unroll
  for (int it = 0; it < YM_ITA; ++it) {
    const int e = threadIdx.x + it * FINAL_THREADS;
    const int ii = e & 63, kk = e >> 6;
    if (kk < kn) sa[kk][ii] = i0 + ii < n ? (double)xa[it] : 0.0;
  }
#pragma unroll
  for (int it = 0; it < YM_ITC; ++it) {
    const int e = threadIdx.x + it * FINAL_THREADS;
    const int cc = e % FINAL_COLS, kk = e / FINAL_COLS;
    if (kk < kn) sc[kk][cc] = j0 + cc < r ? xl[it] * xc[it] : 0.0;
  }
  __syncthreads();
  const int tr = threadIdx.x & 63, tc = threadIdx.x >> 6;
  int kk = 0;
  for (; kk + 4 <= kn; kk += 4) {
#pragma unroll
    for (int h = 0; h < 4; ++h) acc[h] = fma(sa[kk + h][tr], sc[kk + h][tc], acc[h]);
  }
  if (kk < kn) acc[0] = fma(sa[kk][tr], sc[kk][tc], acc[0]);
  if (kk + 1 < kn) acc[1] = fma(sa[kk + 1][tr], sc[kk + 1][tc], acc[1]);
  if (kk + 2 < kn) acc[2] = fma(sa[kk + 2][tr], sc[kk + 2][tc], acc[2]);
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ double sum8(const T* v) {
  return (((double)v[0] + (double)v[1]) + ((double)v[2] + (double)v[3])) +
         (((double)v[4] + (double)v[5]) + ((double)v[6] + (double)v[7]));
}

template <typename T>
__global__ __launch_bounds__(FINAL_THREADS) void k_final(FinalArgs<T> a) {
  __shared__ double sa[FINAL_K][65];
  __shared__ double sc[FINAL_K][FINAL_COLS + 1];
  __shared__ double sm[FINAL_THREADS];
  const int64_t b = blockIdx.x;
  if (b < a.ntile) {
    const int64_t nrb = (a.n + 63) / 64;
    const int64_t i0 = (b % nrb) * 64;
    const int64_t z = b / nrb;
    const int j0 = (int)(z % a.ct) * FINAL_COLS, grp = (int)(z / a.ct);
    const int tr = threadIdx.x & 63, tc = threadIdx.x >> 6;
    const int64_t i = i0 + tr;
    const int j = j0 + tc;
    const bool live = i < a.n && j < a.r;
    const int64_t J = (int64_t)grp * a.r + j;
    const int64_t stride = a.rp * a.npad;
    const T* yp = a.Ypart + (live ? J * a.npad + i : 0);
    // Y = the partials summed in groups of eight (pairwise within a group),
    // then the remaining ones in order; the first groups' loads go out now
    constexpr int PF = final_pf<T>();
    const int npf = min(a.nsplit, PF) & ~7;
    const T* Ag = a.A + (int64_t)grp * a.r * a.lda;
    const double* lg = a.lambda + (int64_t)grp * a.r;
    const double* Cg = a.C + (int64_t)grp * a.r * a.r;
    T xa[YM_ITA];
    double xc[YM_ITC], xl[YM_ITC];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    ym_load(Ag, a.lda, a.n, a.r, lg, Cg, i0, j0, 0, xa, xc, xl);
    // the first partials of Y: unconditional loads from valid partials (a
    // condition would make each load a branch that waits for it), issued
    // behind the first slice of Y_M's loads; only the first npf are used
    T yv[PF];
#pragma unroll
    for (int s = 0; s < PF; ++s) yv[s] = yp[(int64_t)min(s, a.nsplit - 1) * stride];
    ym_use(a.n, a.r, i0, j0, 0, xa, xc, xl, sa, sc, acc);
    for (int k0 = FINAL_K; k0 < a.r; k0 += FINAL_K) {
      ym_load(Ag, a.lda, a.n, a.r, lg, Cg, i0, j0, k0, xa, xc, xl);
      ym_use(a.n, a.r, i0, j0, k0, xa, xc, xl, sa, sc, acc);
    }
    const double ym = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if (!live) return;
    double y = 0.0;
#pragma unroll
    for (int s = 0; s < PF; s += 8)
      if (s < npf) y += sum8(yv + s);
    int s = npf;
    for (; s + 8 <= a.nsplit; s += 8) {
      T v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = yp[(s + q) * stride];
      y += sum8(v);
    }
    for (; s < a.nsplit; ++s) y += (double)yp[s * stride];
    a.G[J * a.ldg + i] = (T)(-2.0 * a.d * (a.yscale * y - ym) * a.lambda[J]);
    return;
  }
  // column J; the last column block of a model to arrive adds its f
  const int J = (int)(b - a.ntile);
  const int grp = J / a.r, jl = J - grp * a.r;
  const int64_t rr = (int64_t)a.r * a.r;
  const double* Bg = a.B + grp * rr;
  const double* Cg = a.C + grp * rr;
  const double* lg = a.lambda + (int64_t)grp * a.r;
  double w = 0.0, u = 0.0;
  // loads in batches of four, issued (from valid rows, without branches)
  // before they are summed
  for (int64_t q0 = threadIdx.x; q0 < a.nwpart; q0 += 4 * FINAL_THREADS) {
    double v[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int64_t q = q0 + h * FINAL_THREADS;
      v[h] = a.wpart[(q < a.nwpart ? q : q0) * a.rp + J];
    }
#pragma unroll
    for (int h = 0; h < 4; ++h)
      if (q0 + h * FINAL_THREADS >= a.nwpart) v[h] = 0.0;
    w += (v[0] + v[1]) + (v[2] + v[3]);
  }
  for (int k = threadIdx.x; k < a.r; k += FINAL_THREADS)
    u += Bg[(int64_t)k * a.r + jl] * Cg[(int64_t)k * a.r + jl] * lg[k];
  w = block_sum(w, sm);
  u = block_sum(u, sm);
  __shared__ int sflag;
  if (threadIdx.x == 0) {
    a.g_lambda[J] = -2.0 * (w - u);
    xput64(a.fpart + J, __builtin_bit_cast(uint64_t, a.lambda[J] * u - 2.0 * w * a.lambda[J]));
    xput_complete();
    sflag = __hip_atomic_fetch_add(a.count + grp, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (sflag != a.r - 1) return;                            // not the model's last column (block-uniform)
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  double s = 0.0;
  for (int j = threadIdx.x; j < a.r; j += FINAL_THREADS)
    s += __builtin_bit_cast(double, xget64(a.fpart + (int64_t)grp * a.r + j));
  s = block_sum(s, sm);
  if (threadIdx.x == 0) {
    a.f[grp] = a.alpha + s;
    __hip_atomic_store(a.count + grp, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
template <typename T, int NS2>
struct Dispatch {
  template <int NTV>
  static void g1(bool dma, bool narrow, dim3 grid, hipStream_t st, const G1Args<T>& a) {
    if (narrow) {
      if (dma) hipLaunchKernelGGL((k_gemm1<T, NTV, true, true>), grid, dim3(64 * g1_waves<T>()), 0, st, a);
      else hipLaunchKernelGGL((k_gemm1<T, NTV, false, true>), grid, dim3(64 * g1_waves<T>()), 0, st, a);
      return;
    }
    if (dma) hipLaunchKernelGGL((k_gemm1<T, NTV, true, false>), grid, dim3(64 * g1_waves<T>()), 0, st, a);
    else hipLaunchKernelGGL((k_gemm1<T, NTV, false, false>), grid, dim3(64 * g1_waves<T>()), 0, st, a);
  }
  template <int NTV>
  static void g2(bool vec, bool narrow, dim3 grid, hipStream_t st, const G2Args<T>& a) {
    if (narrow) {
      if (vec) hipLaunchKernelGGL((k_gemm2<T, NTV, NS2, true, true>), grid, dim3(256), 0, st, a);
      else hipLaunchKernelGGL((k_gemm2<T, NTV, NS2, false, true>), grid, dim3(256), 0, st, a);
      return;
    }
    if (vec) hipLaunchKernelGGL((k_gemm2<T, NTV, NS2, true, false>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_gemm2<T, NTV, NS2, false, false>), grid, dim3(256), 0, st, a);
  }
};

using DF32 = Dispatch<float, G2_STAGES_F32>;
using DF64 = Dispatch<double, G2_STAGES_F64>;

void launch_gemm1(int nt, bool vec, dim3 grid, hipStream_t st, const G1Args<float>& a, bool narrow) {
  switch (nt) {
    case 1: DF32::g1<1>(vec, narrow, grid, st, a); break;
    case 2: DF32::g1<2>(vec, narrow, grid, st, a); break;
    case 3: DF32::g1<3>(vec, narrow, grid, st, a); break;
    case 4: DF32::g1<4>(vec, narrow, grid, st, a); break;
    case 5: DF32::g1<5>(vec, narrow, grid, st, a); break;
    case 6: DF32::g1<6>(vec, narrow, grid, st, a); break;
    case 7: DF32::g1<7>(vec, narrow, grid, st, a); break;
    default: break;
  }
}
void launch_gemm1(int nt, bool vec, dim3 grid, hipStream_t st, const G1Args<double>& a, bool narrow) {
  switch (nt) {
    case 1: DF64::g1<1>(vec, narrow, grid, st, a); break;
    case 2: DF64::g1<2>(vec, narrow, grid, st, a); break;
    case 3: DF64::g1<3>(vec, narrow, grid, st, a); break;
    case 4: DF64::g1<4>(vec, narrow, grid, st, a); break;
    case 5: DF64::g1<5>(vec, narrow, grid, st, a); break;
    case 6: DF64::g1<6>(vec, narrow, grid, st, a); break;
    case 7: DF64::g1<7>(vec, narrow, grid, st, a); break;
    default: break;
  }
}
void launch_gemm2(int nt, bool vec, dim3 grid, hipStream_t st, const G2Args<float>& a, bool narrow) {
  switch (nt) {
    case 1: DF32::g2<1>(vec, narrow, grid, st, a); break;
    case 2: DF32::g2<2>(vec, narrow, grid, st, a); break;
    case 3: DF32::g2<3>(vec, narrow, grid, st, a); break;
    case 4: DF32::g2<4>(vec, narrow, grid, st, a); break;
    case 5: DF32::g2<5>(vec, narrow, grid, st, a); break;
    case 6: DF32::g2<6>(vec, narrow, grid, st, a); break;
    case 7: DF32::g2<7>(vec, narrow, grid, st, a); break;
    default: break;
  }
}
void launch_gemm2(int nt, bool vec, dim3 grid, hipStream_t st, const G2Args<double>& a, bool narrow) {
  switch (nt) {
    case 1: DF64::g2<1>(vec, narrow, grid, st, a); break;
    case 2: DF64::g2<2>(vec, narrow, grid, st, a); break;
    case 3: DF64::g2<3>(vec, narrow, grid, st, a); break;
    case 4: DF64::g2<4>(vec, narrow, grid, st, a); break;
    case 5: DF64::g2<5>(vec, narrow, grid, st, a); break;
    case 6: DF64::g2<6>(vec, narrow, grid, st, a); break;
    case 7: DF64::g2<7>(vec, narrow, grid, st, a); break;
    default: break;
  }
}
void launch_prep(int64_t blocks, hipStream_t st, const PrepArgs<float>& a) {
  hipLaunchKernelGGL(k_prep<float>, dim3((unsigned)blocks), dim3(GRAM_THREADS), 0, st, a);
}
void launch_prep(int64_t blocks, hipStream_t st, const PrepArgs<double>& a) {
  hipLaunchKernelGGL(k_prep<double>, dim3((unsigned)blocks), dim3(GRAM_THREADS), 0, st, a);
}
void launch_final(hipStream_t st, const FinalArgs<float>& a) {
  const int64_t blocks = a.ntile + (int64_t)a.ng * a.r;
  hipLaunchKernelGGL(k_final<float>, dim3((unsigned)blocks), dim3(FINAL_THREADS), 0, st, a);
}
void launch_final(hipStream_t st, const FinalArgs<double>& a) {
  const int64_t blocks = a.ntile + (int64_t)a.ng * a.r;
  hipLaunchKernelGGL(k_final<double>, dim3((unsigned)blocks), dim3(FINAL_THREADS), 0, st, a);
}
}  // namespace symtd
