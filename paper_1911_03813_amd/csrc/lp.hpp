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
//   Vc  column-major n x p, leading dimension ldc = n rounded up to the chunk
//       (rows past n zero): the first product's operand (covariates contiguous)
//   Vr  row-major n x p, leading dimension ldr = p rounded up to 128 (columns
//       past p zero): the second product's operand (observations contiguous)
// per evaluation:
//   Ac  A in ldc rows x rp columns (zero padded), like Vc
//   W   column-major ldr x rp (observations contiguous), written by gemm1
// bf16x3 keeps a hi and a lo plane of each, `plane` elements apart.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace symtd {

enum LpKind { LP_F16 = 0, LP_BF16X3 = 1 };

constexpr int LP_WAVES = 4;
constexpr int LP_MT = 2;                 // 16-row subtiles per wave
constexpr int LP_SLAB = 16 * LP_MT * LP_WAVES;   // 128 rows (gemm1: observations, gemm2: covariates)
constexpr int LP_NT_MAX = 7;             // 16-column subtiles per launch
// k values per chunk: one 256-byte run per column (fp16), 128 bytes per plane (bf16x3)
constexpr int lp_chunk(int kind) { return kind == LP_F16 ? 128 : 64; }
constexpr int LP_PAD = 128;              // ldr / ldc multiple (covers both chunks)

struct LpG1Args {
  const void* Vc; int64_t ldc; int64_t vplane;   // elements between the hi and lo planes
  const double* nu; int n; int p;
  const void* Ac; int64_t aplane;
  int col0, rp, nslab, nblocks, d;
  double wscale;                                 // 2^s (fp16) or 1
  void* W; int64_t ldr; int64_t wplane;
  double* wpart;                                 // [4 nblocks][rp]
  float* part; int* flag; int* err;              // stream-K hand-off
};

struct LpG2Args {
  const void* Vr; int64_t ldr; int64_t vplane;
  const void* W; int64_t wplane;
  int n; int col0; int rp;
  int nslab;                                     // ceil(n / LP_SLAB)
  int nsplit; int chunks_per_split;
  float* Ypart; int64_t npad;                    // [nsplit][rp][npad]
};

struct LpPackArgs {
  const float* A; int64_t lda; int n; int r;
  void* Ac; int64_t ldc; int rp; int64_t aplane;
};

struct LpConvArgs {
  const float* V; int64_t ldv; int n; int p;
  void* Vc; int64_t ldc; void* Vr; int64_t ldr; int64_t plane_c, plane_r;
};

void launch_lp_gemm1(int kind, int nt, dim3 grid, hipStream_t st, const LpG1Args& a);
void launch_lp_gemm2(int kind, int nt, dim3 grid, hipStream_t st, const LpG2Args& a);
void launch_lp_pack_a(int kind, hipStream_t st, const LpPackArgs& a);
void launch_lp_convert(int kind, hipStream_t st, const LpConvArgs& a);
void launch_max_abs(hipStream_t st, const double* x, int64_t count, double* out);

}  // namespace symtd
