// HIP kernels of the rKS hot path (CDNA4, wave64).
//
// One Arnoldi step of Algorithm 2 runs as three launches on one stream:
//   k_spmv_sketch  w' = A u_t  and per-block partial sums of Omega w'   (Algorithm 2: product with A, its sketch)
//   k_reduce       deterministic bin-parallel sum of the partials
//   k_ls_update    every workgroup: finalise the previous column (beta, s,
//                  B(t,t-1)) and solve the FP64 least squares h = S^+ z  (Algorithm 2: low-dimensional projection);
//                  then u~ = w - U_t h, stored, and partial sums of Omega u~ (Algorithm 2: update in R^n, its sketch)
// (k_ls alone finalises the last column of an extension; k_update alone
// serves the deterministic Krylov-Schur step.)
// The new column is kept unnormalised; its scale 1/beta is folded into the
// next step's coefficients (lazy normalisation saves one pass over n).
// k_rotate applies the restart rotation U <- U Y (Algorithm 1, truncation).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "layout.hpp"
#include "philox.hpp"

namespace rks {

constexpr int kMaxD = 1024;      // largest sketch size (LDS bins)
constexpr int kMaxM = 255;       // largest Krylov dimension
constexpr int kMaxG = 512;       // largest number of partial-sum rows (producer blocks)
constexpr int kMaxPart0 = kSpmvMaxG > kMaxG ? kSpmvMaxG : kMaxG;
constexpr int kMaxPart = kSellMaxG > kMaxPart0 ? kSellMaxG : kMaxPart0;  // partial rows of the row-tile or sliced SpMV's sketch
constexpr int kRotMax = 128;     // output columns per rotation pass (8 MFMA column tiles)
constexpr size_t kRotLdsMax = 160 * 1024;  // Y in LDS up to this size, else read from global memory
constexpr size_t kLsLdsMax = 150 * 1024;  // LDS budget of the least-squares kernel

struct bf16_t {
  uint16_t b;
};

template <typename T>
struct Conv;
template <>
struct Conv<double> {
  __device__ static double ld(double v) { return v; }
  __device__ static double st(double v) { return v; }
};
template <>
struct Conv<float> {
  __device__ static double ld(float v) { return (double)v; }
  __device__ static float st(double v) { return (float)v; }
};
template <>
struct Conv<bf16_t> {
  __device__ static double ld(bf16_t v) { return (double)__uint_as_float((uint32_t)v.b << 16); }
  __device__ static bf16_t st(double v) {
    // round to nearest even via FP32
    uint32_t u = __float_as_uint((float)v);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
    bf16_t r;
    r.b = (uint16_t)(u >> 16);
    return r;
  }
};

struct SketchP {
  int d;
  int zeta;
  uint32_t k0, k1;
  double scale;
};

}  // namespace rks
