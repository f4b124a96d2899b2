// Argument blocks and host-side launchers of the symtd kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace symtd {

// Column subtiles handled by one launch of gemm1/gemm2 (16 columns each);
// wider ranks are processed in several column groups.
// Both products handle up to 7 in one launch (fp32 and fp64).
constexpr int NT_MAX_G1_F32 = 7;
constexpr int NT_MAX_G1_F64 = 7;
constexpr int NT_MAX_G2_F32 = 7;
constexpr int NT_MAX_G2_F64 = 7;
// gemm1 shape of the fp32 kernel: waves per block, M subtiles (16
// observations) per wave, bytes of one column run per chunk, and LDS stages
// of the chunk ring; and the chunk run and stages of the fp64 kernel.
// fp32: eight one-subtile waves (two per SIMD) on 256-byte chunks in two
// stages (120 KiB of LDS); fp64: 256-byte chunks in two stages (128 KiB).
#ifndef SYMTD_G1_WAVES
#define SYMTD_G1_WAVES 8
#endif
#ifndef SYMTD_G1_MT
#define SYMTD_G1_MT 1
#endif
#ifndef SYMTD_G1_RUN
#define SYMTD_G1_RUN 256
#endif
#ifndef SYMTD_G1_STAGES
#define SYMTD_G1_STAGES 2
#endif
// waves of a gemm1 block that move the chunks into LDS (0: all of them):
// fp32 the first four (one per SIMD, so that the other wave on each SIMD
// keeps the matrix core busy while they issue), fp64 all eight
#ifndef SYMTD_G1_DMA_WAVES
#define SYMTD_G1_DMA_WAVES 4
#endif
#ifndef SYMTD_G1_DMA_WAVES_F64
#define SYMTD_G1_DMA_WAVES_F64 0
#endif
#ifndef SYMTD_G1_RUN_F64
#define SYMTD_G1_RUN_F64 256
#endif
#ifndef SYMTD_G1_STAGES_F64
#define SYMTD_G1_STAGES_F64 2
#endif
constexpr int G1_WAVES = SYMTD_G1_WAVES;
constexpr int G1_MT = SYMTD_G1_MT;
template <typename T> constexpr int g1_run() { return sizeof(T) == 8 ? SYMTD_G1_RUN_F64 : SYMTD_G1_RUN; }
template <typename T> constexpr int g1_stages() { return sizeof(T) == 8 ? SYMTD_G1_STAGES_F64 : SYMTD_G1_STAGES; }
template <typename T> constexpr int g1_dma_waves() { return sizeof(T) == 8 ? SYMTD_G1_DMA_WAVES_F64 : SYMTD_G1_DMA_WAVES; }
// M subtiles per wave of the first product: fp64 takes one, so that seven
// column subtiles of fp64 accumulators fit the register file and r <= 112
// needs one launch (V read once)
template <typename T> constexpr int g1_mt() { return sizeof(T) == 8 ? 1 : G1_MT; }
// Waves per block of the first product: fp64 takes eight one-subtile waves
// (two per SIMD, so that one multiplies while the other waits at a stage
// boundary; its registers allow it), fp32 G1_WAVES waves of G1_MT subtiles.
template <typename T> constexpr int g1_waves() { return sizeof(T) == 8 ? 8 : G1_WAVES; }
// Depth of the register prefetch ring of gemm2.
constexpr int G2_STAGES_F32 = 3;
constexpr int G2_STAGES_F64 = 2;

// Stream-K hand-off of a split product: flag[b] is raised to the launch's
// epoch (handoff_epoch) by block b once its partial is published; block b-1
// waits for that value for at most `spin` polls (bits 0-30), after which it
// sets *err (pinned host memory).  With bit 31 of `spin` set (testing) it
// waits for a value that no block writes.
struct Handoff {
  int* flag;       // [blocks] hand-off flags
  int* err;        // device address of the context's error word
  int* epoch;      // the context's epoch word, then its arrival counter (zero at creation)
  unsigned spin;
};

template <typename T>
struct G1Args {
  const T* V; int64_t ldv; const double* nu; int n; int p;
  const T* A; int64_t lda; int r;
  int col0;      // first column of this launch's column group (multiple of 16)
  int nt_tot;    // column subtiles over all groups: ceil(r / 16)
  int rp;        // 16 * nt_tot
  int nblk;      // ceil(p / 16) blocks of 16 observations (packed W)
  int nslab;     // ceil(p / (16 * g1_mt<T>() * g1_waves<T>())) block slabs
  int nblocks;   // blocks taking part (<= nslab, all resident)
  int d;
  const T* Apad; int64_t ldap;   // zero-padded factor copy (see k_pack_a)
  T* Wp;         // packed W
  double* wpart; // [g1_waves<T>() * nblocks][rp] fp64 column partials, one row per wave
  T* part;       // [nblocks][g1_waves<T>() * g1_mt<T>() * NT * 256] published partial accumulators
  Handoff ho;    // stream-K hand-off between neighbouring blocks
};

template <typename T>
struct G2Args {
  const T* V; int64_t ldv; int n; int p;
  const T* Wp; int nt_tot; int rp; int col0;
  int nblk;           // ceil(p / 16)
  int blk_per_split;  // 16-observation slabs per split
  int nsplit;
  int rowblocks;      // npad / 256
  T* Ypart;           // [nsplit][rp][npad]
  int64_t npad;       // rows of a partial column, multiple of 256
};

template <typename T>
struct PackAArgs {
  const T* A; int64_t lda; int n; int r;
  T* Apad; int64_t ldap;   // rp columns of ldap rows
};

// k values per gemm1 chunk (one g1_run<T>()-byte run per column)
template <typename T> constexpr int g1_chunk() { return g1_run<T>() / (int)sizeof(T); }

// The model terms work on ng independent models of r columns each, stored
// side by side (model m = columns m*r .. m*r + r - 1 of A, lambda, G_A).
template <typename T>
struct GramArgs {
  const T* A; int64_t lda; int n; int r; int ng;
  int rt;             // ceil(r / 16) tiles per side
  int d;
  double* B; double* C;   // ng blocks of r x r, column-major: B = A'A, C = B^(d-1)
};

// The closing step of an evaluation (k_final, FINAL_THREADS-thread blocks):
// G tiles of 64 rows x FINAL_COLS columns (the model term A D_lambda C
// computed in place), then one block per column for w, u, g_lambda and the
// column's share of f; the last column block of each model to finish adds f.
constexpr int FINAL_THREADS = 512;
constexpr int FINAL_COLS = FINAL_THREADS / 64;
template <typename T>
struct FinalArgs {
  const T* Ypart; int64_t npad; int64_t rp; int nsplit; double yscale;
  const T* A; int64_t lda; int n; int r; int ng;
  int ct;                                // ceil(r / FINAL_COLS) column tiles per model
  const double* lambda; const double* B; const double* C; int d;
  const double* wpart; int64_t nwpart;   // rows of rp column partials of w
  double alpha;
  T* G; int64_t ldg;
  double* fpart; double* f; double* g_lambda;   // fpart: ng r shares of f
  int* count;                            // ng arrival counters, zero between launches
  int64_t ntile;                         // G tile blocks: ceil(n / 64) ct ng
};

// Threads of a prep block (16 waves; a Gram tile per block).
constexpr int GRAM_THREADS = 1024;

// pack_a and the Gram tiles in one launch: blocks [0, npack) pack (npack_x
// blocks of GRAM_THREADS elements per column), then rt rt ng Gram tiles
template <typename T>
struct PrepArgs {
  PackAArgs<T> pack; int npack_x; int64_t npack;
  GramArgs<T> gram;
};

template <typename S>
struct NormXArgs {
  const S* V; int64_t ldv; const double* nu; int n; int p; int d;
  int64_t ntile;      // ceil(p / 128)
  double* part;       // one fp64 partial per block
};

struct ReduceArgs {
  const double* part; int64_t count; double* out;
};

// narrow: the launch's last column subtile holds at most 4 factor columns
// (it is then multiplied on the narrow MFMA form, Narrow<T>)
void launch_gemm1(int nt, bool vec, dim3 grid, hipStream_t st, const G1Args<float>& a, bool narrow = false);
void launch_gemm1(int nt, bool vec, dim3 grid, hipStream_t st, const G1Args<double>& a, bool narrow = false);
void launch_gemm2(int nt, bool vec, dim3 grid, hipStream_t st, const G2Args<float>& a, bool narrow = false);
void launch_gemm2(int nt, bool vec, dim3 grid, hipStream_t st, const G2Args<double>& a, bool narrow = false);
void launch_prep(int64_t blocks, hipStream_t st, const PrepArgs<float>& a);
void launch_prep(int64_t blocks, hipStream_t st, const PrepArgs<double>& a);
void launch_final(hipStream_t st, const FinalArgs<float>& a);
void launch_final(hipStream_t st, const FinalArgs<double>& a);

void launch_widen(hipStream_t st, const float* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                  int64_t cols);

void launch_normx(bool vec, dim3 grid, hipStream_t st, const NormXArgs<float>& a);
void launch_normx(bool vec, dim3 grid, hipStream_t st, const NormXArgs<double>& a);
void launch_reduce(hipStream_t st, const ReduceArgs& a);

// ||X||^2 of several data sets in one launch (vector loads: 16-byte aligned
// V, leading dimension a multiple of 16 bytes): block b forms tile pair
// items[b].pair of set items[b].set into that set's partials; then one block
// per set sums its partials in the same order as launch_reduce.
struct NormXItem { int set; int pair; };
template <typename S>
struct GNormX {
  NormXArgs<S> a;     // a.part: this set's partials
  int64_t pairs;      // ntile (ntile + 1) / 2
  double* alpha;
};
void launch_normx_grouped(int nitems, int nsets, hipStream_t st, const GNormX<float>* sets, const NormXItem* items);
void launch_normx_grouped(int nitems, int nsets, hipStream_t st, const GNormX<double>* sets, const NormXItem* items);

}  // namespace symtd
