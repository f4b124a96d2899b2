// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller normals
// (Box & Muller, 1958) on the device.
//
// Normal number e of (seed, restart, stream) is normal e mod 4 of the Philox
// block with counter (e/4 low word, e/4 high word, restart, stream) and key
// (seed low word, seed high word): block words (x0, x1) give normals 0, 1 and
// (x2, x3) normals 2, 3 through u = (x + 1/2) 2^-32,
// sqrt(-2 ln u_a) (cos, sin)(2 pi u_b).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace symtd {

constexpr uint32_t STREAM_GAUSS_A0 = 1, STREAM_RRF_OMEGA = 2;

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd > 0) { k0 += W0; k1 += W1; }
    const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

__device__ __forceinline__ double normal_at(uint64_t seed, uint32_t restart, uint32_t stream, int64_t e) {
  const uint64_t blk = (uint64_t)e >> 2;
  uint32_t c[4] = {(uint32_t)blk, (uint32_t)(blk >> 32), restart, stream};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const int q = (int)(e & 3);
  const int pr = q >> 1;
  const double u1 = ((double)c[2 * pr] + 0.5) * (1.0 / 4294967296.0);
  const double u2 = ((double)c[2 * pr + 1] + 0.5) * (1.0 / 4294967296.0);
  const double rad = sqrt(-2.0 * log(u1));
  const double th = 2.0 * M_PI * u2;
  return (q & 1) ? rad * sin(th) : rad * cos(th);
}

}  // namespace symtd
