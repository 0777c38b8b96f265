// Device-side counter-based random numbers for the never-stored embedding.
//
// Philox4x32-10 (Salmon et al., SC'11): 4x32-bit counter, 2x32-bit key,
// ten rounds, Weyl key schedule.  Stream layout (key = seed split in two
// 32-bit halves; counter = (i low, i high, c2, tag)):
//   tag 0  Gaussian embedding, c2 = row-pair index, one Box-Muller pair
//   tag 1  sparse-sign embedding, c2 in {0, 1}: words r0..r7 of column i
//   tag 2  start vector, entry i = first Box-Muller output of c2 = 0
// A uniform in (0,1) is ((hi << 20) | (lo >> 12)) + 1/2, times 2^-52 (exact).
// Sparse-sign column i: draw t = 0..zeta-1 takes j = d - zeta + t,
// v = mulhi(r_t, j + 1) in [0, j], keeps v unless already taken, else j
// (Floyd's sampling without replacement); the sign is negative iff r_t is odd.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rks {

struct Philox4 {
  uint32_t v[4];
};

__device__ __forceinline__ Philox4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
  Philox4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

__device__ __forceinline__ double uniform01(uint32_t hi, uint32_t lo) {
  const uint64_t x = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
  return ((double)x + 0.5) * 0x1.0p-52;
}

// Box-Muller pair from counter (i, c2, tag).
__device__ __forceinline__ void gauss_pair(uint64_t i, uint32_t c2, uint32_t tag, uint32_t k0,
                                           uint32_t k1, double& g0, double& g1) {
  const Philox4 w = philox10((uint32_t)i, (uint32_t)(i >> 32), c2, tag, k0, k1);
  const double u1 = uniform01(w.v[0], w.v[1]);
  const double u2 = uniform01(w.v[2], w.v[3]);
  const double r = sqrt(-2.0 * log(u1));
  const double th = 2.0 * 3.14159265358979323846 * u2;
  double s, c;
  sincos(th, &s, &c);
  g0 = r * c;
  g1 = r * s;
}

// Rows and signs (+-1) of sparse-sign column i.
__device__ __forceinline__ void sparse_column(uint64_t i, int d, int zeta, uint32_t k0, uint32_t k1,
                                              int rows[8], float sgn[8]) {
  uint32_t r[8];
  const Philox4 a = philox10((uint32_t)i, (uint32_t)(i >> 32), 0u, 1u, k0, k1);
  r[0] = a.v[0]; r[1] = a.v[1]; r[2] = a.v[2]; r[3] = a.v[3];
  if (zeta > 4) {
    const Philox4 b = philox10((uint32_t)i, (uint32_t)(i >> 32), 1u, 1u, k0, k1);
    r[4] = b.v[0]; r[5] = b.v[1]; r[6] = b.v[2]; r[7] = b.v[3];
  } else {
    r[4] = r[5] = r[6] = r[7] = 0u;
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    if (t < zeta) {
      const int j = d - zeta + t;
      const int v = (int)__umulhi(r[t], (uint32_t)(j + 1));
      bool taken = false;
#pragma unroll
      for (int s = 0; s < t; ++s) taken |= (rows[s] == v);
      rows[t] = taken ? j : v;
      sgn[t] = (r[t] & 1u) ? -1.0f : 1.0f;
    }
  }
}

}  // namespace rks
