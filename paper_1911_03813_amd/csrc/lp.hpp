// 16-bit product paths: fp16 and bf16x3 (split bf16) storage of V, A and W
// with fp32 matrix-core accumulation; reductions and assembly stay fp64.
//
// bf16x3: x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to nearest
// even both times); a product x y is taken as hi_x hi_y + hi_x lo_y + lo_x hi_y
// (the lo lo term, of relative size 2^-16, is dropped), accumulated in fp32.
// fp16: plain fp16 storage; W = nu z^{d-1} is stored times 2^s (s from the
// largest nu) so that it stays in fp16's normal range, and Y is divided by
// 2^s in fp64.
//
// Layout (prepared once per data set, see symtd_data_create):
//   Vc  column-major n x kr_len: kc_len = n rounded up to LP_PAD covariates
//       per column (rows past n zero), kr_len = p rounded up to LP_PAD
//       columns (columns past p zero), column stride ldc = kc_len + LP_SKEW.
//       Both products read this one copy: the first with covariates as its
//       k dimension, the second with observations as k, taking its operand
//       fragments out of LDS with transposed reads.
// per evaluation:
//   Ac  A as kc_len rows x rp columns (zero padded), stride ldc, like Vc
//   W   unit-major kr_len x rp: observation l of column j at
//       ((l / 8) rp + j) 8 + l % 8, so that a unit (8 observations) of
//       consecutive columns is contiguous for both gemm1's stores and
//       gemm2's loads
// bf16x3 keeps a hi and a lo plane of each, `plane` elements apart.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace symtd {

enum LpKind { LP_F16 = 0, LP_BF16X3 = 1 };

// Shape of both products: waves per block, 16-row subtiles per wave, bytes of
// one column run per chunk and plane, and LDS stages.
#ifndef SYMTD_LP_MT
#define SYMTD_LP_MT 2
#endif
#ifndef SYMTD_LP_RUN
#define SYMTD_LP_RUN 256
#endif
#ifndef SYMTD_LP_RUN_BF
#define SYMTD_LP_RUN_BF 128
#endif
#ifndef SYMTD_LP_STAGES
#define SYMTD_LP_STAGES 2
#endif
constexpr int LP_WAVES = 4;
constexpr int LP_MT = SYMTD_LP_MT;
constexpr int LP_SLAB = 16 * LP_MT * LP_WAVES;   // rows of a block (gemm1: observations, gemm2: covariates)
constexpr int LP_NT_MAX = 7;             // 16-column subtiles per launch
constexpr int LP_STAGES = SYMTD_LP_STAGES;
// k values per chunk: a run of SYMTD_LP_RUN (fp16) or SYMTD_LP_RUN_BF (bf16x3,
// per plane) bytes per column
constexpr int lp_chunk(int kind) { return (kind == LP_F16 ? SYMTD_LP_RUN : SYMTD_LP_RUN_BF) / 2; }
constexpr int LP_PAD = 256;              // kc_len / kr_len multiple (whole chunks, whole slabs)

// ldc is the column stride; kc_len / kr_len (multiples of LP_PAD) are the
// extents the products run over (zero beyond the data).  The stride exceeds
// kc_len by LP_SKEW elements so that a chunk's column reads do not fall on a
// power-of-two stride.
constexpr int LP_SKEW = 64;

struct LpG1Args {
  const void* Vc; int64_t ldc; int64_t kc_len; int64_t vplane;   // vplane: elements between the hi and lo planes
  const double* nu; int n; int p;
  const void* Ac; int64_t aplane;
  int col0, rp, nslab, nblocks, d;
  double wscale;                                 // 2^s (fp16) or 1
  void* W; int64_t kr_len; int64_t wplane;       // W rows: kr_len observations
  double* wpart;                                 // [4 nblocks][rp]
  float* part; Handoff ho;                       // stream-K hand-off
};

struct LpG2Args {
  const void* Vc; int64_t ldc; int64_t kr_len; int64_t vplane;
  const void* W; int64_t wplane;
  int n; int col0; int rp;
  int nslab;                                     // ceil(n / LP_SLAB)
  int nsplit; int chunks_per_split;
  float* Ypart; int64_t npad;                    // [nsplit][rp][npad]
};

struct LpPackArgs {
  const float* A; int64_t lda; int n; int r;
  void* Ac; int64_t ldc; int64_t kc_len; int rp; int64_t aplane;
};

struct LpConvArgs {
  const float* V; int64_t ldv; int n; int p;
  void* Vc; int64_t ldc; int64_t kc_len; int64_t kr_len; int64_t plane_c;
};

void launch_lp_gemm1(int kind, int nt, dim3 grid, hipStream_t st, const LpG1Args& a);
void launch_lp_gemm2(int kind, int nt, dim3 grid, hipStream_t st, const LpG2Args& a);
// the 16-bit copy of A and gram_blocks Gram tiles (model_dev.hpp) in one launch
void launch_lp_prep(int kind, int64_t gram_blocks, hipStream_t st, const LpPackArgs& a, const GramArgs<float>& g);
void launch_lp_convert(int kind, hipStream_t st, const LpConvArgs& a);
void launch_max_abs(hipStream_t st, const double* x, int64_t count, double* out);

}  // namespace symtd
