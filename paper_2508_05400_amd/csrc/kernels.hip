// HIP kernels of the rKS hot path.  See kernels.hpp for the step layout.
#include "kernels.hpp"
#include "launch.hpp"

#include <hip/hip_ext.h>
#include <mutex>
#include <type_traits>
#include <unordered_map>

namespace rks {

__device__ uint32_t g_read_sink[8192];  // written by k_read16 in the rare case described there

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Sum over the block; every thread gets the total.  red holds >= 16 doubles.
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int q = 0; q < nw; ++q) t += red[q];
  return t;
}

// Scatter v * Omega[:, i] into the block's LDS bins (unscaled).
// KIND 1: sparse-sign Omega, accumulated by the producing kernel; 2: no
// sketch (deterministic Krylov-Schur, whose kernels accumulate a squared norm
// instead); 3: no sketch in the producing kernel: a Gaussian Omega (d dense
// entries per column) is applied by k_gauss_sketch afterwards, which spreads
// its Box-Muller work over the whole grid instead of one lane per element.
template <int KIND>
__device__ __forceinline__ void sketch_add(double* bins, uint64_t i, double v, const SketchP& sp) {
  if (KIND != 1) return;
  int rows[8];
  float sg[8];
  sparse_column(i, sp.d, sp.zeta, sp.k0, sp.k1, rows, sg);
#pragma unroll
  for (int t = 0; t < 8; ++t)
    if (t < sp.zeta) atomicAdd(&bins[rows[t]], (double)sg[t] * v);
}

__device__ __forceinline__ double readlane_f64(double v, int j) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, j);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), j);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sketch bins in dynamic LDS, one set of d per wave: wave w adds into
// bins + w d only, so no two waves add to the same word and a wave's adds
// follow its program order; bins_store then adds the waves' bins in wave
// order.  The partial rows are the same on every run.
__device__ __forceinline__ void bins_zero(double* bins, int d) {
  const int nb = d * (int)(blockDim.x >> 6);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) bins[b] = 0.0;
}

__device__ __forceinline__ void bins_store(const double* bins, double* part, int d, double scale) {
  const int nw = blockDim.x >> 6;
  for (int b = threadIdx.x; b < d; b += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += bins[w * d + b];
    part[(size_t)blockIdx.x * d + b] = s * scale;
  }
}

__device__ __forceinline__ double* wave_bins(double* bins, int d) {
  return bins + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * d;
}

// ---------------------------------------------------------------------------
// Row sums of one wave tile {first row r0, rows nr, first nonzero e0,
// nonzeros ne} of a CSR matrix times x.  A lane loads up to 4 pairs of
// nonzeros (8-byte column and 8- or 16-byte value loads, coalesced, all issued
// before any use; pairs start at the even index at or below e0, and the
// arrays carry kCsrPad readable entries at the end), gathers x for them, and
// stages the products in the wave's own LDS slice pw; then 64/nr lanes per
// row reduce the row from LDS.  LDS operations of one wave complete in program
// order, so the wave needs no block-level barrier.  A tile that is a single
// row longer than kTileFill nonzeros is reduced by the whole wave.  The row sum ends
// in the lane with sub == 0 of row rr (< nr).  after_loads(rr, sub) runs while
// the loads are in flight (independent work can hide under them), then
// prepare_values(), which a long tile runs before its loop.
// TS: the stored values (TA itself), or one-byte indices into the table vt
// of the matrix's distinct values (the FP64 product's value-indexed
// storage; vt in LDS, 256 entries).
template <typename TA, typename TS>
__device__ __forceinline__ TA a_value(TS v, const double* vt) {
  if constexpr (sizeof(TS) == 1) return (TA)vt[v];
  else return (TA)v;
}

// A pair of stored values as loaded, and value h (0 or 1) of it.  A pair of
// one-byte indices is one 16-bit load kept whole in a 32-bit register and
// unpacked only where the values are used: packed into shared registers,
// the loads of a lane's pairs would each wait for the one before.
template <typename TS>
struct APair {
  typedef TS TS2 __attribute__((ext_vector_type(2)));
  typedef typename std::conditional<sizeof(TS) == 1, uint32_t, TS2>::type type;
  __device__ static type load(const TS* p) {
    if constexpr (sizeof(TS) == 1) return (uint32_t)*(const uint16_t*)p;
    else return *(const TS2*)p;
  }
};
template <typename TA, typename TS>
__device__ __forceinline__ TA a_value2(typename APair<TS>::type p, int h, const double* vt) {
  if constexpr (sizeof(TS) == 1) return (TA)vt[(p >> (8 * h)) & 0xFF];
  else return (TA)(h ? p.y : p.x);
}

template <typename TV, typename TA, typename TS, typename F, typename G>
__device__ __forceinline__ TA tile_rows(const int* __restrict__ rp, const int* __restrict__ col,
                                        const TS* __restrict__ val, const double* vt, const TV* __restrict__ x,
                                        int4 dsc, TA* pw, int lane, int& rr, int& sub, F&& after_loads,
                                        G&& prepare_values) {
  typedef typename APair<TS>::type VP;
  constexpr int NP = kTileNnz / 128;  // pairs per lane
  const int r0 = dsc.x, nr = dsc.y, e0 = dsc.z, ne = dsc.w;
  TA s = 0;
  if (ne <= kTileFill) {
    int lpr = 64;
    while (lpr > 1 && lpr * nr > 64) lpr >>= 1;
    rr = lane / lpr;
    sub = lane - rr * lpr;
    int ra = 0, rb = 0;
    if (rr < nr) {
      ra = rp[r0 + rr] - e0;
      rb = rp[r0 + rr + 1] - e0;
    }
    // pair p covers tile entries 2p - sh and 2p + 1 - sh (ne + sh <= 2 NP 64)
    const int e0a = e0 & ~1, sh = e0 - e0a, nea = ne + sh;
    int2 ci[NP];
    VP vv[NP];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int p2 = 2 * (lane + 64 * u);
      // index pairs: loaded by every lane (pairs past the tile reload its
      // first, in bounds), since a load under the branch is merged there
      if constexpr (sizeof(TS) == 1) vv[u] = APair<TS>::load(val + e0a + (p2 < nea ? p2 : 0));
      if (p2 < nea) {
        ci[u] = *(const int2*)(col + e0a + p2);
        if constexpr (sizeof(TS) != 1) vv[u] = APair<TS>::load(val + e0a + p2);
      }
    }
    after_loads(rr, sub);
    prepare_values();
    TA xa[NP], xb[NP];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int p2 = 2 * (lane + 64 * u);
      if (p2 < nea) {
        if (p2 >= sh) xa[u] = (TA)Conv<TV>::ld(x[ci[u].x]);
        if (p2 + 1 < nea) xb[u] = (TA)Conv<TV>::ld(x[ci[u].y]);
      }
    }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int p2 = 2 * (lane + 64 * u);
      if (p2 < nea) {
        if (p2 >= sh) pw[p2 - sh] = a_value2<TA, TS>(vv[u], 0, vt) * xa[u];
        if (p2 + 1 < nea) pw[p2 + 1 - sh] = a_value2<TA, TS>(vv[u], 1, vt) * xb[u];
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (rr < nr)
      for (int e = ra + sub; e < rb; e += lpr) s += pw[e];
    for (int off = lpr >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off);
    __builtin_amdgcn_wave_barrier();
  } else {
    rr = 0;
    sub = lane;
    prepare_values();
    for (int e = lane; e < ne; e += 64) s += a_value<TA>(val[e0 + e], vt) * (TA)Conv<TV>::ld(x[col[e0 + e]]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  }
  return s;
}

// w = A x (CSR, wave tiles staged through LDS; see tile_rows) and partials of
// Omega w.  Workgroups are dealt to the 8 XCDs round-robin (block b runs on
// XCD b % 8); giving each XCD one contiguous eighth of the tiles keeps the x
// entries that neighbouring rows share (stencil offsets) inside one XCD's L2.
// The kernel is bound by the latency of its two dependent loads per tile
// (nonzeros, then the gathered x), so it wants many resident waves: small
// workgroups (kSpmvWaves waves, each with its LDS slice and d sketch bins)
// let five of them share a CU, where two 8-wave workgroups fit before.
// TS = uint8_t: A's values as one-byte indices into vtab (256 FP64 entries,
// copied to LDS; otherwise vtab is unused).  Every wave copies the whole
// table in its first tile, once that tile's nonzero loads are in flight, so
// the copy's latency hides under theirs and no barrier waits for it: the
// waves write the same values, and a wave's own LDS writes complete before
// its later LDS reads.
template <typename TV, typename TW, typename TA, int KIND, typename TS = TA>
__global__ __launch_bounds__(64 * kSpmvWaves) void k_spmv_sketch(const int* __restrict__ rp, const int* __restrict__ col,
                                                     const TS* __restrict__ val, const double* __restrict__ vtab,
                                                     const int4* __restrict__ tdesc, int ntiles,
                                                     const TV* __restrict__ x, TW* __restrict__ w,
                                                     double* __restrict__ zpart, SketchP sp, int do_sketch_arg) {
  extern __shared__ double bins[];  // kSpmvWaves waves x d
  __shared__ TA prod[kSpmvWaves][kTileNnz];
  __shared__ double vt[sizeof(TS) == 1 ? 256 : 1];
  const int do_sketch = KIND == 1 ? do_sketch_arg : 0;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  bool tab = sizeof(TS) != 1;
  if (do_sketch) bins_zero(bins, sp.d);
  __syncthreads();
  TA* pw = prod[wv];
  double* wb = wave_bins(bins, sp.d);
  const int Gx = gridDim.x >> 3;
  int t0, tend, tstep;
  if (Gx > 0 && (gridDim.x & 7) == 0) {
    const int xcd = blockIdx.x & 7, lb = blockIdx.x >> 3;
    const int chunk = (ntiles + 7) >> 3;
    t0 = xcd * chunk + lb * kSpmvWaves + wv;
    tend = min(ntiles, (xcd + 1) * chunk);
    tstep = Gx * kSpmvWaves;
  } else {
    t0 = blockIdx.x * kSpmvWaves + wv;
    tend = ntiles;
    tstep = gridDim.x * kSpmvWaves;
  }
  for (int t = t0; t < tend; t += tstep) {
    const int4 dsc = tdesc[t];  // wave-uniform
    int rr, sub;
    int hrows[8];
    float hsg[8];
    int have = 0;
    // the row's sketch column does not depend on the data: hash it while the
    // tile's loads are in flight
    const TA s = tile_rows<TV, TA, TS>(
        rp, col, val, vt, x, dsc, pw, lane, rr, sub,
        [&](int r_, int s_) {
          if (KIND == 1 && do_sketch && r_ < dsc.y && s_ == 0) {
            sparse_column((uint64_t)(dsc.x + r_), sp.d, sp.zeta, sp.k0, sp.k1, hrows, hsg);
            have = 1;
          }
        },
        [&] {
          if constexpr (sizeof(TS) == 1) {
            if (!tab) {
              double tv[4];
#pragma unroll
              for (int q = 0; q < 4; ++q) tv[q] = vtab[64 * q + lane];
#pragma unroll
              for (int q = 0; q < 4; ++q) vt[64 * q + lane] = tv[q];
              tab = true;
            }
          }
        });
    if (rr < dsc.y && sub == 0) {
      const int r = dsc.x + rr;
      const TW ws = (TW)s;
      w[r] = ws;
      if (do_sketch) {
        if (KIND == 1 && have) {
#pragma unroll
          for (int q = 0; q < 8; ++q)
            if (q < sp.zeta) atomicAdd(&wb[hrows[q]], (double)hsg[q] * (double)ws);
        } else {
          sketch_add<KIND>(wb, (uint64_t)r, (double)ws, sp);
        }
      }
    }
  }
  __syncthreads();
  if (do_sketch) bins_store(bins, zpart, sp.d, sp.scale);
}

// w = A x and partials of Omega w in the sliced layout (see LaunchEnv): one
// wave per slice of kSliceRows rows, lane l owning row kSliceRows s + l and
// adding its products in order (k = 0, 1, ...) in a register, so no LDS
// staging and no cross-lane reduction.  A wave's loads of the k-th nonzeros
// are contiguous (256 bytes of columns, 64 of value indices), and on a banded
// matrix so are its gathers of x.  Loads go in groups of 8 k, every one issued
// before the first use and none under a branch (k past the slice's longest
// row is clamped to its last: in bounds, not added).  Padding (k >= the row's
// length) holds +0.0 when pad0, and is then added like the nonzeros (exactly
// 0 for finite x, and no row lengths are read); otherwise it is loaded but not
// added.  The row's sketch column is hashed while the first group is in
// flight.  Slices are dealt to the XCDs in contiguous eighths, as the row
// tiles are.  TS as in k_spmv_sketch.
template <typename TV, typename TW, typename TA, int KIND, typename TS>
__global__ __launch_bounds__(64 * kSpmvWaves) void k_spmv_sell(const int* __restrict__ rp,
                                                   const int64_t* __restrict__ sl_off, int nsl,
                                                   const int* __restrict__ col, const TS* __restrict__ val,
                                                   const double* __restrict__ vtab, int64_t n,
                                                   const TV* __restrict__ x, TW* __restrict__ w,
                                                   double* __restrict__ zpart, SketchP sp, int do_sketch_arg,
                                                   int pad0) {
  extern __shared__ double bins[];  // kSpmvWaves waves x d
  __shared__ double vt[sizeof(TS) == 1 ? 256 : 1];
  typedef typename std::conditional<sizeof(TS) == 1, uint32_t, TS>::type VL;
  const int do_sketch = KIND == 1 ? do_sketch_arg : 0;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  bool tab = sizeof(TS) != 1;
  if (do_sketch) bins_zero(bins, sp.d);
  __syncthreads();
  double* wb = wave_bins(bins, sp.d);
  const int Gx = gridDim.x >> 3;
  int s0, send, sstep;
  if (Gx > 0 && (gridDim.x & 7) == 0) {
    const int xcd = blockIdx.x & 7, lb = blockIdx.x >> 3;
    const int chunk = (nsl + 7) >> 3;
    s0 = xcd * chunk + lb * kSpmvWaves + wv;
    send = min(nsl, (xcd + 1) * chunk);
    sstep = Gx * kSpmvWaves;
  } else {
    s0 = blockIdx.x * kSpmvWaves + wv;
    send = nsl;
    sstep = gridDim.x * kSpmvWaves;
  }
  for (int s = s0; s < send; s += sstep) {
    const int64_t b0 = sl_off[s];  // wave-uniform
    const int slen = (int)((sl_off[s + 1] - b0) / kSliceRows);
    const int64_t r = (int64_t)s * kSliceRows + lane;
    const int len = pad0 ? slen : (r < n ? rp[r + 1] - rp[r] : 0);
    TA acc = 0;
    int hrows[8];
    float hsg[8];
    for (int k0 = 0; k0 < slen; k0 += 8) {
      int cc[8];
      VL vv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t e = b0 + (int64_t)kSliceRows * (k0 + q < slen ? k0 + q : slen - 1) + lane;
        cc[q] = col[e];
        vv[q] = (VL)val[e];
      }
      if (k0 == 0) {
        if (KIND == 1 && do_sketch && r < n) sparse_column((uint64_t)r, sp.d, sp.zeta, sp.k0, sp.k1, hrows, hsg);
        if constexpr (sizeof(TS) == 1) {
          if (!tab) {
            double tv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) tv[q] = vtab[64 * q + lane];
#pragma unroll
            for (int q = 0; q < 4; ++q) vt[64 * q + lane] = tv[q];
            tab = true;
          }
        }
      }
      TA xv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) xv[q] = (TA)Conv<TV>::ld(x[cc[q]]);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        TA a;
        if constexpr (sizeof(TS) == 1) a = (TA)vt[vv[q]];
        else a = (TA)vv[q];
        if (k0 + q < len) acc += a * xv[q];
      }
    }
    if (r < n) {
      const TW ws = (TW)acc;
      w[r] = ws;
      // (a slice of empty rows hashes nothing and adds nothing: its sums are 0)
      if (KIND == 1 && do_sketch && slen > 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q < sp.zeta) atomicAdd(&wb[hrows[q]], (double)hsg[q] * (double)ws);
      }
    }
  }
  __syncthreads();
  if (do_sketch) bins_store(bins, zpart, sp.d, sp.scale);
}

// Row sums of one panel tile {first row r0 (within the panel), rows nr, first
// nonzero e0, nonzeros ne} of the column-blocked layout, added to the panel's
// row sums acc (LDS).  As in tile_rows, a lane loads up to 4 pairs of
// nonzeros and gathers x for them, all issued before any use, and the products
// go to the wave's LDS slice pw; here a lane also loads the 16-bit row
// offsets of its rows (lane + 64 j, j < kPanelTileRows / 64) with them, and
// then sums each of its rows from LDS in order.  A long tile (ob < 0: one row
// with more than kTileFill nonzeros) is summed by the whole wave.  Only the
// lane that sums a row touches acc for it, and rows of different tiles of one
// column block are disjoint, so no two waves write the same sum between the
// workgroup's barriers.
template <typename TV, typename TA>
__device__ __forceinline__ void panel_tile(const int* __restrict__ col, const TA* __restrict__ val,
                                           const uint16_t* __restrict__ off, int ob, const TV* __restrict__ x,
                                           int4 dsc, TA* pw, double* acc, int lane) {
  typedef TA TA2 __attribute__((ext_vector_type(2)));
  constexpr int NP = kTileNnz / 128;       // pairs per lane
  constexpr int RL = kPanelTileRows / 64;  // rows per lane
  const int r0 = dsc.x, nr = dsc.y, e0 = dsc.z, ne = dsc.w;
  if (ob < 0) {
    TA s = 0;
    for (int e = lane; e < ne; e += 64) s += val[e0 + e] * (TA)Conv<TV>::ld(x[col[e0 + e]]);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) acc[r0] += (double)s;
    return;
  }
  int ra[RL], rb[RL];
#pragma unroll
  for (int j = 0; j < RL; ++j) {
    const int r = lane + 64 * j;
    ra[j] = 0;
    rb[j] = 0;
    if (r < nr) {
      ra[j] = off[ob + r];
      rb[j] = off[ob + r + 1];
    }
  }
  // pair p covers tile entries 2p - sh and 2p + 1 - sh (ne + sh <= 2 NP 64)
  const int e0a = e0 & ~1, sh = e0 - e0a, nea = ne + sh;
  int2 ci[NP];
  TA2 vv[NP];
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    const int p2 = 2 * (lane + 64 * u);
    if (p2 < nea) {
      ci[u] = *(const int2*)(col + e0a + p2);
      vv[u] = *(const TA2*)(val + e0a + p2);
    }
  }
  TA xa[NP], xb[NP];
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    const int p2 = 2 * (lane + 64 * u);
    if (p2 < nea) {
      if (p2 >= sh) xa[u] = (TA)Conv<TV>::ld(x[ci[u].x]);
      if (p2 + 1 < nea) xb[u] = (TA)Conv<TV>::ld(x[ci[u].y]);
    }
  }
#pragma unroll
  for (int u = 0; u < NP; ++u) {
    const int p2 = 2 * (lane + 64 * u);
    if (p2 < nea) {
      if (p2 >= sh) pw[p2 - sh] = vv[u].x * xa[u];
      if (p2 + 1 < nea) pw[p2 + 1 - sh] = vv[u].y * xb[u];
    }
  }
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int j = 0; j < RL; ++j) {
    const int r = lane + 64 * j;
    if (r < nr) {
      TA s = 0;
      for (int e = ra[j]; e < rb[j]; ++e) s += pw[e];
      acc[r0 + r] += (double)s;
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// Column-blocked SpMV for operators whose rows gather x from everywhere (x
// larger than an XCD's L2, no locality to exploit), on the layout of
// panels.hpp: kCb column blocks of n / kCb columns (that much of x fits in an
// XCD's L2) and one workgroup per row panel.  The workgroup multiplies block
// 0 of its rows, then block 1, and so on, streaming its panel's nonzeros in
// one contiguous pass and keeping the panel's row sums in LDS, with a barrier
// between blocks (so each row adds its block sums in block order).  All
// workgroups start on block 0 and move on at about the same pace, so the x
// entries the chip gathers at any moment lie in one or two blocks, held in
// every XCD's L2.  The sums leave the workgroup once, as w, with the sketch of
// w added on the way.  LDS: the row sums (rows_pp FP64, rounded up to even),
// then either the waves' product slices (during the blocks) or their sketch
// bins (afterwards) in the same space.
template <typename TV, typename TW, typename TA, int KIND>
__global__ __launch_bounds__(64 * kSpmvWaves) void k_spmv_panel(
    int64_t n, int rows_pp, const int* __restrict__ col, const TA* __restrict__ val, const int4* __restrict__ tdesc,
    const int* __restrict__ toff, const uint16_t* __restrict__ off, const int* __restrict__ ptile,
    const TV* __restrict__ x, TW* __restrict__ w, double* __restrict__ zpart, SketchP sp, int do_sketch_arg) {
  extern __shared__ double smem[];
  const int accn = (rows_pp + 1) & ~1;
  double* acc = smem;
  TA* stage = (TA*)(smem + accn);
  double* bins = smem + accn;
  const int do_sketch = KIND == 1 ? do_sketch_arg : 0;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t R0 = (int64_t)blockIdx.x * rows_pp;
  const int nrows = (int)min((int64_t)rows_pp, n - R0);
  for (int i = tid; i < nrows; i += blockDim.x) acc[i] = 0.0;
  __syncthreads();
  TA* pw = stage + wv * kTileNnz;
  const int* pt = ptile + (size_t)blockIdx.x * (kCb + 1);
  for (int c = 0; c < kCb; ++c) {
    const int t1 = pt[c + 1];
    for (int t = pt[c] + wv; t < t1; t += kSpmvWaves) panel_tile<TV, TA>(col, val, off, toff[t], x, tdesc[t], pw, acc, lane);
    __syncthreads();
  }
  if (do_sketch) bins_zero(bins, sp.d);
  __syncthreads();
  double* wb = wave_bins(bins, sp.d);
  for (int i = tid; i < nrows; i += blockDim.x) {
    const TW ws = (TW)acc[i];
    w[R0 + i] = ws;
    if (do_sketch) sketch_add<KIND>(wb, (uint64_t)(R0 + i), (double)ws, sp);
  }
  __syncthreads();
  if (do_sketch) bins_store(bins, zpart, sp.d, sp.scale);
}

// Deterministic sum of G partial rows: block (x, y) sums kRedBins bins of
// array y.  Each of the kRedSl row slices adds every kRedSl-th row with two
// chains; a fixed tree over the slices finishes the sum (same order every
// call).  A wave reads 8 rows x 64 contiguous bytes per load.  128 slices
// (10 rows each for the SpMV's 1,280 partial rows) took the launch from 4.8
// to 4.0 us against 64 slices; 4 bins per block or 4 chains per slice did
// not help further.
constexpr int kRedBins = 8;
constexpr int kRedSl = 128;

__global__ __launch_bounds__(kRedBins * kRedSl) void k_reduce(const double* __restrict__ pa,
                                                             const double* __restrict__ pb, int Ga, int Gb, int d,
                                                             double* __restrict__ oa, double* __restrict__ ob) {
  const double* p = blockIdx.y ? pb : pa;
  double* o = blockIdx.y ? ob : oa;
  const int G = blockIdx.y ? Gb : Ga;
  if (p == nullptr) return;
  __shared__ double red[kRedSl][kRedBins + 1];
  const int lb = threadIdx.x % kRedBins, sl = threadIdx.x / kRedBins;
  const int b = blockIdx.x * kRedBins + lb;
  double a0 = 0.0, a1 = 0.0;
  if (b < d) {
    int g = sl;
    for (; g + kRedSl < G; g += 2 * kRedSl) {
      a0 += p[(size_t)g * d + b];
      a1 += p[(size_t)(g + kRedSl) * d + b];
    }
    for (; g < G; g += kRedSl) a0 += p[(size_t)g * d + b];
  }
  red[sl][lb] = a0 + a1;
  __syncthreads();
  for (int s = kRedSl / 2; s > 0; s >>= 1) {
    if (sl < s) red[sl][lb] += red[sl + s][lb];
    __syncthreads();
  }
  if (sl == 0 && b < d) o[b] = red[0][lb];
}

// Finalise column t when pending (beta = ||s~||, S(:,t) = s~/beta, scale
// 1/beta, B(t, t-1) = beta, breakdown test), then the low-dimensional
// projection h = S_t^+ z.  With E = S^T S - I (kept up to date column by
// column; the host resets it after each contraction) the least-squares
// solution is (I + E)^{-1} S^T z = y - E y + O(|E|^2 |y|), y = S^T z: the same
// value as one re-projection h = y + S^T (z - S y), but it needs a single
// pass over S (for y and, for the new column, its inner products with the
// old ones) and an O(t^2) correction instead of two more passes.
// Both block products use a 16 x 64 thread grid: thread (r, c) sums rows
// r, r + 16, r + 32, ... of column c (16 consecutive rows per column in a
// wave: coalesced from L2, at most 2-way LDS bank conflicts), and 64 threads
// add the 16 partial sums.
// Writes B(0:t, t) = h and the coefficients the update needs:
// coef[l] = h_l * scale_l (l <= t), coef[t+1] = scale_t.
// When S(:, 0:t) fits in LDS, every global load of the kernel (S, the two raw
// sketches, E) is issued in one round at entry.
constexpr int kLsPre = 20;  // S values per thread staged through registers (LDS path)
constexpr int kLsPreE = 4;  // E values per thread prefetched at entry (t <= 64)
constexpr int kRC = 16;     // row chunks of the block products (1024 threads = 16 x 64)

__global__ __launch_bounds__(1024) void k_ls(int t, int d, int pending, int finalize_only, int use_lds,
                                             const double* __restrict__ zraw, const double* __restrict__ sraw,
                                             double* __restrict__ S, double* __restrict__ B, int ldb,
                                             double* __restrict__ E, double* __restrict__ cs,
                                             double* __restrict__ coef, double* __restrict__ scal,
                                             int* __restrict__ flags, double bd_rel) {
  extern __shared__ double sm[];
  double* snew = sm;
  double* zs = snew + d;
  double* ys = zs + d;             // kMaxM + 2
  double* gs = ys + kMaxM + 2;     // kMaxM + 2
  double* red = gs + kMaxM + 2;    // 32
  double* pa = red + 32;           // 64 x 17 partial sums
  double* pg = pa + 64 * 17;       // 64 x 17 partial sums
  double* Ssh = pg + 64 * 17;      // d * (t + 1) when use_lds
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  const int rc = tid & (kRC - 1), cl = tid >> 4;  // chunk of rows, column slot
  // ---- every global load up front ----
  const int tot = use_lds ? d * t : 0;
  double sv[kLsPre];
#pragma unroll
  for (int u = 0; u < kLsPre; ++u) {
    const int idx = tid + 1024 * u;
    sv[u] = (idx < tot) ? S[idx] : 0.0;
  }
  double srv = 0.0, zrv = 0.0, stv = 0.0, ctg = 0.0;
  if (tid < d) {
    if (pending) srv = sraw[tid];
    else if (use_lds) stv = S[(size_t)t * d + tid];
    if (!finalize_only) zrv = zraw[tid];
  }
  if (!pending) ctg = cs[t];
  const bool pre_e = !finalize_only && t <= kRC * kLsPreE;
  double ev[kLsPreE];
#pragma unroll
  for (int i = 0; i < kLsPreE; ++i) {
    const int c = rc + kRC * i;
    ev[i] = (pre_e && c < t && cl < t) ? E[c + (size_t)cl * ldb] : 0.0;
  }
  // ---- both squared norms in one block reduction ----
  {
    double a = wave_sum(srv * srv), b = wave_sum(zrv * zrv);
    if (lane == 0) {
      red[wv] = a;
      red[16 + wv] = b;
    }
  }
  if (use_lds) {
#pragma unroll
    for (int u = 0; u < kLsPre; ++u) {
      const int idx = tid + 1024 * u;
      if (idx < tot) Ssh[idx] = sv[u];
    }
  }
  __syncthreads();
  double ss = 0.0, zz = 0.0;
  for (int q = 0; q < nw; ++q) {
    ss += red[q];
    zz += red[16 + q];
  }
  // ---- finalise the pending column ----
  double ct;
  if (pending) {
    const double beta = sqrt(ss);
    const double inv = 1.0 / beta;
    if (tid < d) {
      stv = srv * inv;
      snew[tid] = stv;
      S[tid + (size_t)t * d] = stv;
    }
    if (tid == 0) {
      cs[t] = inv;
      if (t > 0) {
        // column t replaces a vanished remainder: its subdiagonal entry is 0
        const bool repl = flags[1] == t;
        B[t + (size_t)(t - 1) * ldb] = repl ? 0.0 : beta;
        if (repl) flags[1] = 0;
        const double sc = scal[0];
        if (!(beta > bd_rel * sc) && flags[0] == 0) {
          flags[0] = t;
          flags[2] = sc == 0.0 ? 1 : 0;
        }
      }
    }
    ct = inv;
  } else {
    ct = ctg;
  }
  if (finalize_only) return;
  const int ncol = t + 1;
  if (use_lds && tid < d) Ssh[(size_t)t * d + tid] = stv;
  if (tid < d) zs[tid] = zrv * ct;
  if (tid == 0) scal[0] = sqrt(zz) * ct;
  __syncthreads();
  // ---- one pass over S: y_l = s_l . z, and g_l = s_l . s_t for a new column ----
  const double* Sc = use_lds ? Ssh : S;
  for (int c0 = 0; c0 < ncol; c0 += 64) {
    const int l = c0 + cl;
    double a = 0.0, g = 0.0;
    if (l < ncol) {
      const double* Sl = (!use_lds && pending && l == t) ? snew : Sc + (size_t)l * d;
      if (pending && l < t) {
#pragma unroll 4
        for (int b = rc; b < d; b += kRC) {
          const double v = Sl[b];
          a += v * zs[b];
          g += v * snew[b];
        }
      } else {
#pragma unroll 4
        for (int b = rc; b < d; b += kRC) a += Sl[b] * zs[b];
      }
    }
    pa[cl * 17 + rc] = a;
    pg[cl * 17 + rc] = g;
    __syncthreads();
    if (tid < 64 && c0 + tid < ncol) {
      double sa = 0.0, sg = 0.0;
#pragma unroll
      for (int r = 0; r < kRC; ++r) {
        sa += pa[tid * 17 + r];
        sg += pg[tid * 17 + r];
      }
      ys[c0 + tid] = sa;
      gs[c0 + tid] = sg;
    }
    __syncthreads();
  }
  // ---- the new column of E, then h = y - E y ----
  if (pending) {
    for (int l = tid; l <= t; l += blockDim.x) {
      const double g = (l < t) ? gs[l] : 0.0;
      E[l + (size_t)t * ldb] = g;
      E[t + (size_t)l * ldb] = g;
    }
  }
  for (int c0 = 0; c0 < ncol; c0 += 64) {
    const int l = c0 + cl;
    double a = 0.0;
    if (l < t) {  // columns c < t of row l (= column l, E is symmetric)
      if (pre_e && c0 == 0) {
#pragma unroll
        for (int i = 0; i < kLsPreE; ++i)
          if (rc + kRC * i < t) a += ev[i] * ys[rc + kRC * i];
      } else {
        for (int c = rc; c < t; c += kRC) a += E[c + (size_t)l * ldb] * ys[c];
      }
    } else if (l == t) {
      for (int c = rc; c < t; c += kRC) a += (pending ? gs[c] : E[c + (size_t)t * ldb]) * ys[c];
    }
    pa[cl * 17 + rc] = a;
    __syncthreads();
    if (tid < 64 && c0 + tid < ncol) {
      const int l2 = c0 + tid;
      double sa = 0.0;
#pragma unroll
      for (int r = 0; r < kRC; ++r) sa += pa[tid * 17 + r];
      // column t of row l2 (just finalised, or from the host)
      if (l2 < t) sa += (pending ? gs[l2] : E[l2 + (size_t)t * ldb]) * ys[t];
      else if (!pending) sa += E[t + (size_t)t * ldb] * ys[t];
      const double h = ys[l2] - sa;
      B[l2 + (size_t)t * ldb] = h;
      coef[l2] = h * ((l2 == t) ? ct : cs[l2]);
    }
    __syncthreads();
  }
  if (tid == 0) coef[t + 1] = ct;
}

// The least squares of k_ls (finalise the pending column, then h = y - E y)
// as run by every workgroup of k_ls_update on its own, arranged so that the
// workgroup waits for global memory once and crosses five barriers:
//   A  every global load at entry: the raw sketches z~ (of A u~_t) and s~ (of
//      the pending column), this thread's rows of its column of S (d <= 256,
//      t < 64), its E values, the scales; the raw sketches go to LDS;
//   B  one pass of inner products with the raw vectors, Y_l = s_l . z~ and
//      G_l = s_l . s~ (slot t takes s~ itself, so G_t = ||s~||^2), and z~ . z~;
//   C  wave 0: beta = sqrt(G_t); then y = ct Y (ct the scale of u~_t), with
//      y_t = Y_t ct / beta, and E's new column g_l = G_l / beta: the same
//      quantities as from the normalised vectors, up to rounding;
//   D  the 16-way partial sums of E y;   E  wave 0: h = y - E y, coefficients.
// Everything it reads is left unchanged by the launch (column t and E's new
// column come from LDS; the other columns and scales were written by earlier
// launches), and the sums run in a fixed order, so every workgroup obtains the
// same h to the last bit; only the writer (workgroup 0) stores S(:, t),
// cs[t], B, E's new column, scal, the breakdown flag and the coefficients to
// global memory.  The coefficients also land in hc[0..t+1] (LDS).  sm holds
// ls_work_doubles(d) doubles; the function ends with a barrier, after which
// sm may be reused.
constexpr int kLsPreS = 16;  // S values per thread prefetched at entry (d <= 256)
constexpr int kLsPreU = 8;   // basis columns of the first packet loaded during the least squares
__host__ __device__ constexpr size_t ls_work_doubles(int d) {
  return 2 * (size_t)d + 4 * (size_t)(kMaxM + 2) + 2 * 64 * 17 + 17;
}

template <typename Pre>
__device__ __forceinline__ void ls_solve(int t, int d, int pending, const double* __restrict__ zraw,
                                         const double* __restrict__ sraw, double* __restrict__ S,
                                         double* __restrict__ B, int ldb, double* __restrict__ E,
                                         double* __restrict__ cs, double* __restrict__ coef,
                                         double* __restrict__ scal, int* __restrict__ flags, double bd_rel,
                                         bool writer, double* sm, double* hc, Pre&& prefetch) {
  double* zr = sm;               // d: z~
  double* sr = zr + d;           // d: s~
  double* yr = sr + d;           // kMaxM + 2: Y (raw inner products with z~)
  double* gr = yr + kMaxM + 2;   // kMaxM + 2: G (raw inner products with s~)
  double* ys = gr + kMaxM + 2;   // kMaxM + 2: y
  double* gs = ys + kMaxM + 2;   // kMaxM + 2: E's new column g
  double* pa = gs + kMaxM + 2;   // 64 x 17 partial sums
  double* pg = pa + 64 * 17;     // 64 x 17 partial sums
  double* pz = pg + 64 * 17;     // 16 partial sums of z~ . z~
  const int tid = threadIdx.x, lane = tid & 63;
  const int rc = tid & (kRC - 1), cl = tid >> 4;
  const int ncol = t + 1;
  // ---- A: every global load, in one round ----
  double zv = 0.0, sv0 = 0.0;
  if (tid < d) {
    zv = zraw[tid];
    if (pending) sv0 = sraw[tid];
  }
  const double ctg = pending ? 0.0 : cs[t];
  const bool pre_s = d <= kRC * kLsPreS && ncol <= 64;
  const bool s_glob = cl < ncol && !(pending && cl == t);  // slot cl reads column cl of S
  double sv[kLsPreS];
#pragma unroll
  for (int i = 0; i < kLsPreS; ++i) {
    const int b = rc + kRC * i;
    sv[i] = (pre_s && s_glob && b < d) ? S[b + (size_t)cl * d] : 0.0;
  }
  const bool pre_e = t <= kRC * kLsPreE;
  double ev[kLsPreE];
#pragma unroll
  for (int i = 0; i < kLsPreE; ++i) {
    const int c = rc + kRC * i;
    ev[i] = (pre_e && c < t && cl < t) ? E[c + (size_t)cl * ldb] : 0.0;
  }
  const double csv = (tid < 64 && tid < t) ? cs[tid] : 0.0;
  const double etv = (!pending && tid < 64 && tid <= t) ? E[tid + (size_t)t * ldb] : 0.0;  // E(tid, t)
  double sc0 = 0.0;
  int fl0 = 1, fl1 = -1;
  if (writer && tid == 0 && pending && t > 0) {
    sc0 = scal[0];
    fl0 = flags[0];
    fl1 = flags[1];
  }
  // the caller's loads go after these (loads complete in order, so waiting
  // for the ones above does not wait for them)
  __builtin_amdgcn_sched_barrier(0);
  prefetch();
  __builtin_amdgcn_sched_barrier(0);
  if (tid < d) {
    zr[tid] = zv;
    sr[tid] = sv0;
  }
  __syncthreads();
  // ---- B: Y, G and z~ . z~ in one pass ----
  for (int c0 = 0; c0 < ncol; c0 += 64) {
    const int l = c0 + cl;
    double a = 0.0, g = 0.0;
    if (l < ncol) {
      const bool newcol = pending && l == t;
      if (pre_s && !newcol) {
#pragma unroll
        for (int i = 0; i < kLsPreS; ++i) {
          const int b = rc + kRC * i;
          if (b < d) {
            a += sv[i] * zr[b];
            if (pending) g += sv[i] * sr[b];
          }
        }
      } else {
        const double* Sl = newcol ? sr : S + (size_t)l * d;
        if (pending) {
#pragma unroll 4
          for (int b = rc; b < d; b += kRC) {
            const double v = Sl[b];
            a += v * zr[b];
            g += v * sr[b];
          }
        } else {
#pragma unroll 4
          for (int b = rc; b < d; b += kRC) a += Sl[b] * zr[b];
        }
      }
    }
    pa[cl * 17 + rc] = a;
    pg[cl * 17 + rc] = g;
    if (c0 == 0 && cl == 0) {
      double zz = 0.0;
      for (int b = rc; b < d; b += kRC) zz += zr[b] * zr[b];
      pz[rc] = zz;
    }
    __syncthreads();
    if (tid < 64 && c0 + tid < ncol) {
      double sa = 0.0, sg = 0.0;
#pragma unroll
      for (int r = 0; r < kRC; ++r) {
        sa += pa[tid * 17 + r];
        sg += pg[tid * 17 + r];
      }
      yr[c0 + tid] = sa;
      gr[c0 + tid] = sg;
    }
    if (c0 + 64 < ncol) __syncthreads();  // the partial sums are reused by the next 64 columns
  }
  // ---- C: wave 0 finalises column t and scales y and g ----
  double ct = ctg;
  if (tid < 64) {
    double inv = 0.0, beta = 0.0;
    if (pending) {
      beta = sqrt(gr[t]);
      inv = 1.0 / beta;
      ct = inv;
    }
    for (int l = lane; l <= t; l += 64) {
      double y = yr[l] * ct;
      if (pending && l == t) y *= inv;
      ys[l] = y;
      gs[l] = (pending && l < t) ? gr[l] * inv : 0.0;
    }
    if (lane == 0) hc[t + 1] = ct;
    if (writer) {
      if (pending) {
        for (int b = lane; b < d; b += 64) S[b + (size_t)t * d] = sr[b] * inv;
        for (int l = lane; l <= t; l += 64) {
          const double g = (l < t) ? gr[l] * inv : 0.0;
          E[l + (size_t)t * ldb] = g;
          E[t + (size_t)l * ldb] = g;
        }
      }
      if (lane == 0) {
        double zz = 0.0;
#pragma unroll
        for (int r = 0; r < kRC; ++r) zz += pz[r];
        scal[0] = sqrt(zz) * ct;
        coef[t + 1] = ct;
        if (pending) {
          cs[t] = inv;
          if (t > 0) {
            // column t replaces a vanished remainder: its subdiagonal entry is 0
            const bool repl = fl1 == t;
            B[t + (size_t)(t - 1) * ldb] = repl ? 0.0 : beta;
            if (repl) flags[1] = 0;
            if (!(beta > bd_rel * sc0) && fl0 == 0) {
              flags[0] = t;
              flags[2] = sc0 == 0.0 ? 1 : 0;
            }
          }
        }
      }
    }
  }
  __syncthreads();
  // ---- D, E: h = y - E y ----
  for (int c0 = 0; c0 < ncol; c0 += 64) {
    const int l = c0 + cl;
    double a = 0.0;
    if (l < t) {  // columns c < t of row l (= column l, E is symmetric)
      if (pre_e && c0 == 0) {
#pragma unroll
        for (int i = 0; i < kLsPreE; ++i)
          if (rc + kRC * i < t) a += ev[i] * ys[rc + kRC * i];
      } else {
        for (int c = rc; c < t; c += kRC) a += E[c + (size_t)l * ldb] * ys[c];
      }
    } else if (l == t) {
      for (int c = rc; c < t; c += kRC) a += (pending ? gs[c] : E[c + (size_t)t * ldb]) * ys[c];
    }
    pa[cl * 17 + rc] = a;
    __syncthreads();
    if (tid < 64 && c0 + tid < ncol) {
      const int l2 = c0 + tid;
      double sa = 0.0;
#pragma unroll
      for (int r = 0; r < kRC; ++r) sa += pa[tid * 17 + r];
      // column t of row l2 (just finalised, or from the host)
      const double e_lt = pending ? gs[l2] : (c0 == 0 ? etv : E[l2 + (size_t)t * ldb]);
      if (l2 < t || !pending) sa += e_lt * ys[t];
      const double h = ys[l2] - sa;
      const double cf = h * ((l2 == t) ? ct : (c0 == 0 ? csv : cs[l2]));
      hc[l2] = cf;
      if (writer) {
        B[l2 + (size_t)t * ldb] = h;
        coef[l2] = cf;
      }
    }
    __syncthreads();
  }
}

// Packets of the basis: PB bytes (16, or 8 for columns too short to give
// every CU a workgroup of 16-byte packets), V = PB / sizeof(TV) consecutive rows.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <int PB>
struct RawOf;
template <>
struct RawOf<16> {
  typedef u32x4 type;
};
template <>
struct RawOf<8> {
  typedef u32x2 type;
};
template <>
struct RawOf<4> {
  typedef unsigned int type;
};
template <typename T, int PB = 16>
union Pack16 {
  typename RawOf<PB>::type raw;
  T v[PB / sizeof(T)];
};

// The pair basis stores x as hi, its binary32 rounding, and lo, a 16-bit
// signed integer: the remainder x - hi (exact in FP64) in units of
// delta = 2^-15 ulp(hi), rounded to nearest even, where ulp(hi) =
// 2^(max(e, 1) - 150) for the biased binary32 exponent e of hi.  |x - hi| <=
// ulp(hi) / 2, so |lo| <= 2^14; the stored value hi + lo delta (exact in
// FP64) is within delta / 2 <= 2^-39 |hi| of x.
// pair_unit(hi, s) = 2^(s (max(e, 1) - 165)) as a double: delta for s = 1,
// 1 / delta for s = -1 (built from its exponent bits; always a normal double).
__device__ __forceinline__ double pair_unit(float hi, int s) {
  const int e = (int)((__float_as_uint(hi) >> 23) & 0xFFu);
  const int k = s * ((e > 1 ? e : 1) - 165);
  return __longlong_as_double((long long)((unsigned long long)(k + 1023) << 52));
}
__device__ __forceinline__ double pair_val(float hi, int16_t lo) { return (double)hi + (double)lo * pair_unit(hi, 1); }
__device__ __forceinline__ void split_pair(double x, float& hi, int16_t& lo) {
  hi = (float)x;
  lo = (int16_t)__builtin_rint((x - (double)hi) * pair_unit(hi, -1));
}

// One packet of a basis column: PB bytes of TV values and, for the pair basis
// (SPLIT, TV = float), the 16-bit remainders of the same rows from the second
// array (PB / 2 bytes); the value of a row is pair_val(hi, lo).
template <typename TV, int PB, bool SPLIT>
struct ColPk {
  typedef typename RawOf<PB>::type Raw;
  typedef typename RawOf<SPLIT ? PB / 2 : 4>::type RawL;
  Pack16<TV, PB> h;
  union {
    RawL raw;
    int16_t v[SPLIT ? PB / 4 : 2];
  } l;
  __device__ __forceinline__ void load(const TV* hi, const int16_t* lo, int64_t off) {
    h.raw = __builtin_nontemporal_load((const Raw*)(hi + off));
    if constexpr (SPLIT) l.raw = __builtin_nontemporal_load((const RawL*)(lo + off));
  }
  __device__ __forceinline__ double val(int r) const {
    if constexpr (SPLIT) return pair_val(h.v[r], l.v[r]);
    else return Conv<TV>::ld(h.v[r]);
  }
  // stores a (rounded to the basis format) as row r of the packet
  __device__ __forceinline__ void set(int r, double a) {
    if constexpr (SPLIT) split_pair(a, h.v[r], l.v[r]);
    else h.v[r] = Conv<TV>::st(a);
  }
};

// u~ = coef[ncol] * w - sum_{l < ncol} coef[l] U(:, l), stored (rounded to the
// basis precision) as the new column; partials of Omega of the stored value.
// SPLIT: the basis is the pair basis (U, Ulo; the new column to unew,
// unew_lo), and the stored value of the new column also goes to xout in FP64
// (the next product with A reads it there).
// Each thread owns V consecutive rows and streams every basis column once
// with one 16-byte non-temporal load per column, in groups of 8 (8 loads,
// then their FMAs).  ROLL: a rolling window of 8 instead, where the slot of
// column l is refilled with column l + 8 as soon as it is consumed.  Measured:
// the window pays in k_ls_update without its prefetch when each thread walks
// 4 or more packets (one 16-wave workgroup per CU; 393 -> 364 us per launch
// on the 160^3 operator in FP64, 212 -> 198 us in FP32) and costs 1-8% with 1
// or 2 packets per thread and in k_update (more waves per CU), which keep the
// groups.  Either way the columns are added in order, one FMA chain per row,
// so both give the same bits.  The coefficients are wave-uniform.  Padding rows (>= n, < ldu)
// are zero in U and w, so packets may run past n; they stay zero and are
// left out of the sketch.
template <typename TV, typename TW, int KIND, int NPRE = 0, bool PREW = false, int PB = 16, bool ROLL = false,
          bool SPLIT = false>
__device__ __forceinline__ void update_body(int64_t n, int64_t npk, int ncol, const TV* __restrict__ U, int64_t ldu,
                                            const TW* __restrict__ w, const double* __restrict__ coef,
                                            TV* __restrict__ unew, double* __restrict__ spart, SketchP sp,
                                            double* bins, const typename RawOf<PB>::type* pre = nullptr,
                                            bool use_pre = false, const int16_t* __restrict__ Ulo = nullptr,
                                            int16_t* __restrict__ unew_lo = nullptr, double* __restrict__ xout = nullptr) {
  // pre: NPRE leading basis columns, then (PREW) the w chunks, of the first packet
  typedef typename RawOf<PB>::type Raw;
  constexpr int V = PB / sizeof(TV);
  constexpr int WCH = (V * (int)sizeof(TW)) / PB;  // PB-byte chunks of w per packet
  constexpr int WV = PB / (int)sizeof(TW);          // w values per chunk
  if (KIND != 3) bins_zero(bins, sp.d);
  __syncthreads();
  double* wb = wave_bins(bins, sp.d);
  const double ws = coef[ncol];
  double nrm = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < npk; g += stride) {
    const int64_t i0 = g * V;
    double a[V];
    {
      Pack16<TW, PB> wp[WCH];
#pragma unroll
      for (int c = 0; c < WCH; ++c)
        wp[c].raw = (PREW && use_pre) ? pre[NPRE + c] : *(const Raw*)(w + i0 + c * WV);
#pragma unroll
      for (int c = 0; c < WCH; ++c)
#pragma unroll
        for (int r = 0; r < WV; ++r) a[c * WV + r] = ws * (double)wp[c].v[r];
    }
    const TV* col0 = U + i0;
    const int16_t* col0l = SPLIT ? Ulo + i0 : nullptr;
    int l = 0;
    if (NPRE > 0 && use_pre) {  // the first packet's leading columns, loaded before the least squares
#pragma unroll
      for (int q = 0; q < NPRE; ++q) {
        Pack16<TV, PB> pq;
        pq.raw = pre[q];
        const double cq = coef[q];
#pragma unroll
        for (int r = 0; r < V; ++r) a[r] -= cq * Conv<TV>::ld(pq.v[r]);
      }
      l = NPRE;
      use_pre = false;
    }
    if (ROLL) {
      ColPk<TV, PB, SPLIT> p[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (l + q < ncol) p[q].load(col0, col0l, (int64_t)(l + q) * ldu);
      for (; l < ncol; l += 8) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (l + q < ncol) {
            const ColPk<TV, PB, SPLIT> cur = p[q];
            if (l + q + 8 < ncol) p[q].load(col0, col0l, (int64_t)(l + q + 8) * ldu);
            const double cq = coef[l + q];
#pragma unroll
            for (int r = 0; r < V; ++r) a[r] -= cq * cur.val(r);
          }
        }
      }
    } else {
      for (; l + 8 <= ncol; l += 8) {
        ColPk<TV, PB, SPLIT> p[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) p[q].load(col0, col0l, (int64_t)(l + q) * ldu);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const double cq = coef[l + q];
#pragma unroll
          for (int r = 0; r < V; ++r) a[r] -= cq * p[q].val(r);
        }
      }
      for (; l < ncol; ++l) {
        ColPk<TV, PB, SPLIT> p;
        p.load(col0, col0l, (int64_t)l * ldu);
        const double cq = coef[l];
#pragma unroll
        for (int r = 0; r < V; ++r) a[r] -= cq * p.val(r);
      }
    }
    ColPk<TV, PB, SPLIT> o;
#pragma unroll
    for (int r = 0; r < V; ++r) o.set(r, a[r]);
    __builtin_nontemporal_store(o.h.raw, (Raw*)(unew + i0));
    if constexpr (SPLIT)
      __builtin_nontemporal_store(o.l.raw, (typename ColPk<TV, PB, SPLIT>::RawL*)(unew_lo + i0));
    if constexpr (SPLIT) {
      typedef double d2v __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int c = 0; c < V / 2; ++c) *(d2v*)(xout + i0 + 2 * c) = (d2v){o.val(2 * c), o.val(2 * c + 1)};
    }
#pragma unroll
    for (int r = 0; r < V; ++r) {
      const double v = o.val(r);
      if (i0 + r >= n) continue;
      if (KIND == 2) nrm += v * v;
      else sketch_add<KIND>(wb, (uint64_t)(i0 + r), v, sp);
    }
  }
  if (KIND == 2) {  // Euclidean inner product (deterministic Krylov-Schur): ||u~||^2 partial
    nrm = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) wb[0] = nrm;
  }
  if (KIND == 3) return;
  __syncthreads();
  bins_store(bins, spart, sp.d, sp.scale);
}

template <typename TV, typename TW, int KIND>
__global__ __launch_bounds__(1024) void k_update(int64_t n, int64_t npk, int ncol, const TV* __restrict__ U,
                                                int64_t ldu, const TW* __restrict__ w,
                                                const double* __restrict__ coef, TV* __restrict__ unew,
                                                double* __restrict__ spart, SketchP sp) {
  extern __shared__ double bins[];  // 16 waves x d (none for KIND 3)
  update_body<TV, TW, KIND>(n, npk, ncol, U, ldu, w, coef, unew, spart, sp, bins);
}

// One randomized Arnoldi step's least squares and update in one launch: every
// workgroup solves the small least squares itself (ls_solve; identical
// results, workgroup 0 stores them), then streams its rows of the update with
// the coefficients from LDS.  This takes the least-squares kernel, a
// latency-bound single workgroup, off the step's critical path.  LDS: the
// coefficients (kMaxM + 2), then the least-squares scratch, reused afterwards
// for the per-wave sketch bins.
template <typename TV, typename TW, int KIND, bool PRE, int PB, bool ROLL, bool SPLIT>
__global__ __launch_bounds__(1024) void k_ls_update(int t, int d, int pending, const double* __restrict__ zraw,
                                                   const double* __restrict__ sraw, double* __restrict__ S,
                                                   double* __restrict__ B, int ldb, double* __restrict__ E,
                                                   double* __restrict__ cs, double* __restrict__ coef,
                                                   double* __restrict__ scal, int* __restrict__ flags, double bd_rel,
                                                   int64_t n, int64_t npk, const TV* __restrict__ U, int64_t ldu,
                                                   const TW* __restrict__ w, TV* __restrict__ unew,
                                                   double* __restrict__ spart, SketchP sp,
                                                   const int16_t* __restrict__ Ulo, int16_t* __restrict__ unew_lo,
                                                   double* __restrict__ xout) {
  extern __shared__ double smem[];
  double* hc = smem;
  double* work = smem + kMaxM + 2;
  // the first kLsPreU basis columns and the w values of this thread's first
  // packet are loaded right after the least squares' own loads, so that their
  // latency passes (and HBM is busy) while the workgroup solves
  // (PRE: only where the least squares has no global loads of its own after
  // its first round, d <= 256 and t < 64, which would wait for these; and not
  // for BF16, whose eight rows per packet leave no registers for it)
  typedef typename RawOf<PB>::type Raw;
  constexpr int V = PB / sizeof(TV);
  constexpr int NP = PRE && sizeof(TV) >= 4 && !SPLIT ? kLsPreU : 0;
  const int64_t g0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool use_pre = NP > 0 && g0 < npk && t + 1 >= NP;
  constexpr int WCH = (V * (int)sizeof(TW)) / PB;  // PB-byte chunks of w per packet
  constexpr bool PREW = NP > 0 && sizeof(TV) == 8;  // w too (FP64: registers allow it)
  Raw pre[NP > 0 ? NP + WCH : 1];
  // The loads are issued by every thread, from clamped (in-bounds) addresses
  // when unused: a load under a branch would make the least squares wait for
  // all of them (wait counts are merged over both paths).
  const int64_t gl = g0 < npk ? g0 : npk - 1;
  ls_solve(t, d, pending, zraw, sraw, S, B, ldb, E, cs, coef, scal, flags, bd_rel, blockIdx.x == 0, work, hc, [&] {
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      const int qc = q <= t ? q : t;
      pre[q] = __builtin_nontemporal_load((const Raw*)(U + gl * V + (int64_t)qc * ldu));
    }
#pragma unroll
    for (int c = 0; c < (PREW ? WCH : 0); ++c) pre[NP + c] = *(const Raw*)(w + gl * V + c * (PB / sizeof(TW)));
  });
  update_body<TV, TW, KIND, NP, PREW, PB, ROLL && NP == 0, SPLIT>(n, npk, t + 1, U, ldu, w, hc, unew, spart, sp,
                                                              work, pre, use_pre, Ulo, unew_lo, xout);
}

// Sums over the wave of eight values per lane: lane L returns the total of
// v[(L >> 3) & 7] (a butterfly that halves the values carried at each of the
// first three steps: 10 shuffles instead of 48).
__device__ __forceinline__ double wave_sum8(const double v[8], int lane) {
  double a[4], b[2];
  const bool h32 = lane & 32, h16 = lane & 16, h8 = lane & 8;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double keep = h32 ? v[i + 4] : v[i], send = h32 ? v[i] : v[i + 4];
    a[i] = keep + __shfl_xor(send, 32);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double keep = h16 ? a[i + 2] : a[i], send = h16 ? a[i] : a[i + 2];
    b[i] = keep + __shfl_xor(send, 16);
  }
  double c = (h8 ? b[1] : b[0]) + __shfl_xor(h8 ? b[0] : b[1], 8);
  c += __shfl_xor(c, 4);
  c += __shfl_xor(c, 2);
  c += __shfl_xor(c, 1);
  return c;
}

// Partial sums (one row of ncol values per block) of U(:, l)^T x, l < ncol,
// for the Euclidean Gram-Schmidt of deterministic Krylov-Schur.  Each thread
// owns one 16-byte packet of rows (as in k_update); columns go in groups of
// eight with one wave_sum8 per group.
template <typename TV, typename TX>
__global__ __launch_bounds__(1024) void k_dots(int64_t n, int64_t npk, int ncol, const TV* __restrict__ U,
                                               int64_t ldu, const TX* __restrict__ x, double* __restrict__ part) {
  constexpr int V = 16 / sizeof(TV);
  __shared__ double bins[16][kMaxM + 8];  // one row per wave, added in wave order at the end
  for (int b = threadIdx.x; b < 16 * (kMaxM + 8); b += blockDim.x) bins[b / (kMaxM + 8)][b % (kMaxM + 8)] = 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t gs = (int64_t)blockIdx.x * blockDim.x; gs < npk; gs += stride) {  // block-uniform trip count
    const int64_t g = gs + threadIdx.x;
    const bool act = g < npk;
    const int64_t i0 = g * V;
    double xv[V];
#pragma unroll
    for (int r = 0; r < V; ++r) xv[r] = (act && i0 + r < n) ? Conv<TX>::ld(x[i0 + r]) : 0.0;
    const TV* col0 = U + i0;
    for (int l0 = 0; l0 < ncol; l0 += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        v[q] = 0.0;
        if (act && l0 + q < ncol) {
          Pack16<TV> p;
          p.raw = __builtin_nontemporal_load((const u32x4*)(col0 + (int64_t)(l0 + q) * ldu));
#pragma unroll
          for (int r = 0; r < V; ++r) v[q] += Conv<TV>::ld(p.v[r]) * xv[r];
        }
      }
      const double sv = wave_sum8(v, lane);
      const int c = l0 + ((lane >> 3) & 7);
      if ((lane & 7) == 0 && c < ncol) bins[wv][c] += sv;
    }
  }
  __syncthreads();
  const int nw = blockDim.x >> 6;
  for (int b = threadIdx.x; b < ncol; b += blockDim.x) {
    double t = 0.0;
    for (int q = 0; q < nw; ++q) t += bins[q][b];
    part[(size_t)blockIdx.x * ncol + b] = t;
  }
}

// Coefficients of one classical Gram-Schmidt pass from y_raw = sum of the
// stored columns' products with the input (scaled by `scale`):
// y_l = cs_l y_raw_l scale, coef_l = cs_l y_l, coef_ncol = scale; h += y.
__global__ void k_ks_coef(int ncol, const double* __restrict__ cs, const double* __restrict__ yraw, double scale_in,
                          const double* __restrict__ scale_ptr, double* __restrict__ coef, double* __restrict__ h,
                          int accumulate) {
  const double sc = scale_ptr ? *scale_ptr * scale_in : scale_in;
  for (int l = threadIdx.x; l < ncol; l += blockDim.x) {
    const double y = cs[l] * yraw[l] * sc;
    coef[l] = cs[l] * y;
    h[l] = accumulate ? h[l] + y : y;
  }
  if (threadIdx.x == 0) coef[ncol] = sc;
}

// Close step t of deterministic Krylov-Schur: B(0:t, t) = h, B(t+1, t) = beta
// = ||u~|| (from the squared norm), cs[t+1] = 1 / beta; breakdown test.
__global__ void k_ks_finalize(int t, const double* __restrict__ h, const double* __restrict__ nrm2, double* __restrict__ B,
                              int ldb, double* __restrict__ cs, int* __restrict__ flags, double bd_rel) {
  double hn = 0.0;
  for (int l = threadIdx.x; l <= t; l += blockDim.x) {
    B[l + (size_t)t * ldb] = h[l];
  }
  if (threadIdx.x == 0) {
    for (int l = 0; l <= t; ++l) hn += h[l] * h[l];
    const double beta = sqrt(*nrm2);
    B[t + 1 + (size_t)t * ldb] = beta;
    cs[t + 1] = 1.0 / beta;
    if (!(beta > bd_rel * sqrt(hn + beta * beta)) && flags[0] == 0) flags[0] = t + 1;
  }
}

// First column: u0 (device FP64) or a seeded N(0,1) vector (Philox counter
// (i, c2, tag): tag 2 the start vector, tag 3 the replacement after a
// breakdown), stored in TV when `store`; partials of Omega of the stored value.
// SPLIT (TV = float): stored as the pair (u, ulo; see split_pair), the stored
// value also to xout in FP64.
template <typename TV, int KIND, bool SPLIT = false>
__global__ __launch_bounds__(512) void k_init(int64_t n, TV* __restrict__ u, const double* __restrict__ u0,
                                              uint32_t s0, uint32_t s1, uint32_t c2, uint32_t tag,
                                              double* __restrict__ spart, SketchP sp, int store,
                                              int16_t* __restrict__ ulo = nullptr, double* __restrict__ xout = nullptr) {
  extern __shared__ double bins[];  // 8 waves x d (none for KIND 3)
  if (KIND != 3) bins_zero(bins, sp.d);
  __syncthreads();
  double* wb = wave_bins(bins, sp.d);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double nrm = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double v;
    if (u0) {
      v = u0[i];
    } else {
      double g1;
      gauss_pair((uint64_t)i, c2, tag, s0, s1, v, g1);
    }
    double vs;
    if constexpr (SPLIT) {
      float hi;
      int16_t lo;
      split_pair(v, hi, lo);
      vs = pair_val(hi, lo);
      if (store) {
        u[i] = hi;
        ulo[i] = lo;
        xout[i] = vs;
      }
    } else {
      const TV st = Conv<TV>::st(v);
      if (store) u[i] = st;
      vs = Conv<TV>::ld(st);
    }
    if (KIND == 2) nrm += vs * vs;
    else sketch_add<KIND>(wb, (uint64_t)i, vs, sp);
  }
  if (KIND == 2) {
    nrm = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) wb[0] = nrm;
  }
  if (KIND == 3) return;
  __syncthreads();
  bins_store(bins, spart, sp.d, sp.scale);
}

// O(:, out0 + o) = sum_l U(:, in0 + l) Y(l, o) for o < kout on the FP64
// matrix cores (v_mfma_f64_16x16x4f64), computed transposed: D = Y^T U^T.
// A wave owns 16 R consecutive rows; lane (c, k) = (lane % 16, lane / 16)
// owns rows R c .. R c + R - 1 of them and loads those R values of input
// column k0 + k with one load (R sizeof(TI) bytes, up to 16).  Each of the R
// rows feeds its own MFMA: A(c', k) = Y(k0 + k, 16 nt + c') (from LDS, shared
// by the R products) and B(k, c) = the row's value, so accumulator r holds
// D(lane / 16 + 4 i, lane % 16) = output column 16 nt + lane / 16 + 4 i of row
// R (lane % 16) + r, and the lane stores its R rows of a column with one
// store.  For 2- and 4-byte inputs this trades many narrow loads for fewer
// wide ones (the vector-memory data path is the busiest unit here, the
// matrix cores less than half busy).  Loads may read rows
// past n (every leading dimension passed is a multiple of 128 >= n for the
// inputs); stores skip rows >= n.  The wave reads every input column of its
// rows before it writes any output, so outputs may overlap inputs (in-place
// restart); optionally U(:, xdst) = xscale * U(:, xsrc) as well.
// SPLIT: the input is the pair basis (U, Ulo; TI = float; see split_pair),
// and an FP32 output (TO = float) is stored as pairs too (O, Olo); the column
// U(:, xdst) is then also written to xcur in FP64.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T, int R>
struct __attribute__((aligned(sizeof(T) * R))) RowPack {
  T v[R];
};

// Rows per lane of the rotation.  FP64 inputs: two (one 16-byte load) up to
// 3 column tiles, else one (measured 5% faster on the 160^3 restart and 10%
// on the 1000^2 one).  FP32 and BF16 inputs: the largest power of two with at
// most 16 bytes per load and at most 6 accumulator tiles (R NT) per lane;
// more tiles cost occupancy and measured slower (the pair basis, whose FP32
// part sets R, included: 4 rows at 3 tiles measured 5% slower).
template <typename TI>
__host__ __device__ constexpr int rot_rows(int nt) {
  int r = 1;
  if (sizeof(TI) == 8 && nt <= 3) return 2;
  if (sizeof(TI) < 8)
    while (2 * r * (int)sizeof(TI) <= 16 && 2 * r * nt <= 6) r *= 2;
  return r;
}

// YG: Y (minp x 16 NT FP64) does not fit in LDS (more than 160 KB: min and
// kout both large); each lane then reads its Y entries from global memory
// (Y is small and stays in L2).  Occupancy: asked for at least 3 waves per
// SIMD, the compiler keeps the accumulators in VGPRs instead of AGPRs and
// reaches 4 or 5 waves for up to 5 column tiles (2 without the request;
// measured 5% faster for the FP64 basis and 30% for the pair basis on the
// 160^3 restart); with Y from global memory (more address registers), and
// for the pair basis with 7 or 8 tiles, it would spill, so those get no
// request.
template <typename TI, typename TO, int NT, bool YG, int R, bool SPLIT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(YG || (SPLIT && NT >= 7) ? 1 : 3))) void k_rotate(int64_t n, const TI* U, int64_t ldu, int in0, int min, TO* O,
                                                int64_t ldo, int out0, int kout, const double* __restrict__ Y,
                                                int xsrc, int xdst, double xscale, const int16_t* Ulo, int16_t* Olo,
                                                double* __restrict__ xcur) {
  extern __shared__ double Ys[];  // minp x (16 NT), zero padded (unused when YG)
  constexpr int KC = 16 * NT;
  constexpr bool SO = SPLIT && sizeof(TO) == 4;  // pair output
  constexpr int RL = SPLIT ? R : 1;              // 16-bit parts per lane
  const int minp = (min + 15) & ~15;
  if (!YG) {
    for (int idx = threadIdx.x; idx < minp * KC; idx += blockDim.x) {
      const int l = idx / KC, o = idx - l * KC;
      Ys[idx] = (l < min && o < kout) ? Y[l + (size_t)o * min] : 0.0;
    }
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t ntile = (n + 16 * R - 1) / (16 * R);
  const bool vec_out = ldo % R == 0;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < ntile; tile += (int64_t)gridDim.x * 4) {
    const int64_t row = tile * 16 * R + (int64_t)R * lr;  // this lane's first row
    const bool full = row + R <= n;
    RowPack<TI, R> xe;
    RowPack<int16_t, RL> xel;
    if (xsrc >= 0 && lk == 0) {
      xe = *(const RowPack<TI, R>*)(U + row + (int64_t)xsrc * ldu);
      if constexpr (SPLIT) xel = *(const RowPack<int16_t, R>*)(Ulo + row + (int64_t)xsrc * ldu);
    }
    f64x4 acc[R][NT];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[r][t] = (f64x4){0.0, 0.0, 0.0, 0.0};
    const TI* urow = U + row + (int64_t)in0 * ldu;
    const int16_t* urowl = SPLIT ? Ulo + row + (int64_t)in0 * ldu : nullptr;
    for (int k0 = 0; k0 < minp; k0 += 16) {
      RowPack<TI, R> a[4];
      RowPack<int16_t, RL> al[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = k0 + 4 * s + lk;
        if (kk < min) {
          a[s] = *(const RowPack<TI, R>*)(urow + (int64_t)kk * ldu);
          if constexpr (SPLIT) al[s] = *(const RowPack<int16_t, R>*)(urowl + (int64_t)kk * ldu);
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) a[s].v[r] = Conv<TI>::st(0.0);
#pragma unroll
          for (int r = 0; r < RL; ++r) al[s].v[r] = 0;
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          double yv;
          if (YG) {
            const int kk = k0 + 4 * s + lk, oc = 16 * t + lr;
            yv = (kk < min && oc < kout) ? Y[kk + (size_t)oc * min] : 0.0;
          } else {
            yv = Ys[(size_t)(k0 + 4 * s + lk) * KC + 16 * t + lr];
          }
#pragma unroll
          for (int r = 0; r < R; ++r) {
            double uv;
            if constexpr (SPLIT) uv = pair_val(a[s].v[r], al[s].v[r]);
            else uv = Conv<TI>::ld(a[s].v[r]);
            acc[r][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(yv, uv, acc[r][t], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int oc = 16 * t + lk + 4 * i;
        if (oc >= kout) continue;
        TO* dst = O + row + (int64_t)(out0 + oc) * ldo;
        if constexpr (SO) {
          int16_t* dstl = Olo + row + (int64_t)(out0 + oc) * ldo;
          RowPack<float, R> o;
          RowPack<int16_t, R> ol;
#pragma unroll
          for (int r = 0; r < R; ++r) split_pair(acc[r][t][i], o.v[r], ol.v[r]);
          if (full && vec_out) {
            *(RowPack<float, R>*)dst = o;
            *(RowPack<int16_t, R>*)dstl = ol;
          } else {
#pragma unroll
            for (int r = 0; r < R; ++r)
              if (row + r < n) {
                dst[r] = o.v[r];
                dstl[r] = ol.v[r];
              }
          }
        } else if (full && vec_out) {
          RowPack<TO, R> o;
#pragma unroll
          for (int r = 0; r < R; ++r) o.v[r] = Conv<TO>::st(acc[r][t][i]);
          *(RowPack<TO, R>*)dst = o;
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r)
            if (row + r < n) dst[r] = Conv<TO>::st(acc[r][t][i]);
        }
      }
    }
    if (xsrc >= 0 && lk == 0) {
      TI* xd = (TI*)U + row + (int64_t)xdst * ldu;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (row + r >= n) continue;
        if constexpr (SPLIT) {
          float hi;
          int16_t lo;
          split_pair(pair_val(xe.v[r], xel.v[r]) * xscale, hi, lo);
          xd[r] = hi;
          ((int16_t*)Ulo)[row + r + (int64_t)xdst * ldu] = lo;
          xcur[row + r] = pair_val(hi, lo);
        } else {
          xd[r] = Conv<TI>::st(Conv<TI>::ld(xe.v[r]) * xscale);
        }
      }
    }
  }
}

// Residual pieces for one Ritz pair: with r = AX_a - re X_a + im X_b and, for
// a complex pair, r2 = AX_b - re X_b - im X_a; per-block partial sums of
// ||r||^2 + ||r2||^2 and ||X_a||^2 + ||X_b||^2.
__global__ __launch_bounds__(256) void k_resid(int64_t n, const double* __restrict__ xa, const double* __restrict__ xb,
                                               const double* __restrict__ axa, const double* __restrict__ axb,
                                               double re, double im, double* __restrict__ part) {
  __shared__ double red[16];
  double rr = 0.0, xx = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double a = xa[i];
    if (xb) {
      const double b = xb[i];
      const double r1 = axa[i] - re * a + im * b;
      const double r2 = axb[i] - re * b - im * a;
      rr += r1 * r1 + r2 * r2;
      xx += a * a + b * b;
    } else {
      const double r1 = axa[i] - re * a;
      rr += r1 * r1;
      xx += a * a;
    }
  }
  rr = block_sum(rr, red);
  xx = block_sum(xx, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = rr;
    part[2 * blockIdx.x + 1] = xx;
  }
}

__global__ __launch_bounds__(256) void k_scale(int64_t n, double* __restrict__ x, double s) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] *= s;
}

__global__ __launch_bounds__(256) void k_fill(int64_t n, double* __restrict__ x, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = v;
}

// Plain streaming copy of n 16-byte packets (bandwidth reference).
__global__ __launch_bounds__(256) void k_copy16(const u32x4* __restrict__ src, u32x4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Plain streaming read of n 16-byte packets (bandwidth reference).  Each
// lane folds its words into one value that is stored (to g_read_sink, an
// externally visible array) only when it equals a fixed constant (almost
// never), so that the loads cannot be removed.
__global__ __launch_bounds__(256) void k_read16(const u32x4* __restrict__ src, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const u32x4 v = __builtin_nontemporal_load(src + i);
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (acc == 0x9E3779B9u) g_read_sink[(blockIdx.x * 256 + threadIdx.x) & 8191] = acc;
}

inline int grid_for(int64_t work, int per_block, int cap) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// Partial sums of Omega x for a Gaussian Omega generated on the fly (entry
// pair (2p, 2p+1) of column i comes from one Philox block, counter (i, p,
// tag 0), and Box-Muller).  Block (bx, by) owns rows [bx R, bx R + R) and
// the pairs p = 64 by + lane.  Its four waves take consecutive quarters of
// those rows; a wave loads 64 entries of x at a time and walks them in
// order, every lane reading the current entry from the lane that loaded it
// and adding its own pair's two products.  So each of the n (d/2) pairs is
// evaluated once, by a different lane than its neighbours in the sum, and
// nothing is accumulated atomically.  The waves' sums are added in a fixed
// order; row bx of part gets this block's bins.
constexpr int kGsMinRows = 32;

template <typename TX>
__global__ __launch_bounds__(256) void k_gauss_sketch(int64_t n, const TX* __restrict__ x, int64_t R,
                                                      double* __restrict__ part, SketchP sp) {
  __shared__ double acc[4][2][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int np = (sp.d + 1) >> 1;
  const int p = (int)blockIdx.y * 64 + lane;
  const int64_t r0 = (int64_t)blockIdx.x * R;
  const int64_t rend = min(n, r0 + R);
  const int64_t Rw = (R + 3) >> 2;
  const int64_t a0 = min(rend, r0 + wv * Rw), a1 = min(rend, a0 + Rw);
  double s0 = 0.0, s1 = 0.0;
  for (int64_t c = a0; c < a1; c += 64) {  // wave-uniform trip count
    const int64_t i = c + lane;
    const double xv = i < a1 ? Conv<TX>::ld(x[i]) : 0.0;
    const int cnt = (int)min((int64_t)64, a1 - c);
    for (int j = 0; j < cnt; ++j) {
      const double v = readlane_f64(xv, j);
      if (p < np) {
        double g0, g1;
        gauss_pair((uint64_t)(c + j), (uint32_t)p, 0u, sp.k0, sp.k1, g0, g1);
        s0 += g0 * v;
        s1 += g1 * v;
      }
    }
  }
  acc[wv][0][lane] = s0;
  acc[wv][1][lane] = s1;
  __syncthreads();
  if (wv == 0 && p < np) {
    const double t0 = ((acc[0][0][lane] + acc[1][0][lane]) + acc[2][0][lane]) + acc[3][0][lane];
    const double t1 = ((acc[0][1][lane] + acc[1][1][lane]) + acc[2][1][lane]) + acc[3][1][lane];
    double* row = part + (size_t)blockIdx.x * sp.d;
    row[2 * p] = t0 * sp.scale;
    if (2 * p + 1 < sp.d) row[2 * p + 1] = t1 * sp.scale;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers.

#define RKS_SKETCH_SWITCH(kind, ...) \
  do {                               \
    if ((kind) == 1) {               \
      constexpr int KIND = 1;        \
      __VA_ARGS__;                   \
    } else if ((kind) == 2) {        \
      constexpr int KIND = 2;        \
      __VA_ARGS__;                   \
    } else {                         \
      constexpr int KIND = 3;        \
      __VA_ARGS__;                   \
    }                                \
  } while (0)

// Dynamic LDS of the per-wave sketch bins (waves x d FP64, none when the
// kernel sketches nothing); the kernel's dynamic-LDS limit is raised to the
// largest size it is launched with (once per size increase).
static size_t bins_lds(const LaunchEnv& e, int waves, bool sketched) {
  return sketched ? (size_t)waves * e.sp.d * 8 : 0;
}

static void lds_allow(const void* f, size_t bytes) {
  if (bytes == 0) return;
  static std::mutex mu;
  static std::unordered_map<const void*, size_t> raised;
  std::lock_guard<std::mutex> lock(mu);
  size_t& cur = raised[f];
  if (bytes > cur) {
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    cur = bytes;
  }
}

// A kernel launch that carries the environment's timing events: with `first`
// the kernel's start is recorded in ev0, with `last` its end in ev1.
template <typename... KArgs, typename... Args>
static void launch_k(const LaunchEnv& e, bool first, bool last, void (*k)(KArgs...), dim3 grid, dim3 block,
                     size_t lds, Args... args) {
  hipEvent_t a = first ? e.ev0 : nullptr, b = last ? e.ev1 : nullptr;
  if (a || b)
    hipExtLaunchKernelGGL(k, grid, block, (uint32_t)lds, e.stream, a, b, 0u, static_cast<KArgs>(args)...);
  else
    k<<<grid, block, lds, e.stream>>>(static_cast<KArgs>(args)...);
}

// The Gaussian sketch of x (n entries of type TX) as partial rows of part;
// returns the number of rows (<= kMaxG).
template <typename TX>
static int gauss_t(const LaunchEnv& e, const TX* x, double* part) {
  const int np = (e.sp.d + 1) >> 1;
  int64_t R = (e.n + kMaxG - 1) / kMaxG;
  if (R < kGsMinRows) R = kGsMinRows;
  const int Gx = (int)((e.n + R - 1) / R);
  dim3 grid(Gx, (np + 63) / 64), block(256);
  launch_k(e, false, true, k_gauss_sketch<TX>, grid, block, 0, e.n, x, R, part, e.sp);
  return Gx;
}

template <typename TV, typename TW, typename TA>
static int spmv_panel_t(const LaunchEnv& e, const TA* val, const TV* x, TW* w, double* zpart, int do_sketch) {
  const size_t accn = (size_t)((e.rows_pp + 1) & ~1);
  const size_t stage = (size_t)kSpmvWaves * kTileNnz * sizeof(TA);
  const size_t bins = bins_lds(e, kSpmvWaves, do_sketch && e.sp_kind == 1);
  const size_t lds = accn * 8 + (stage > bins ? stage : bins);
  RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_spmv_panel<TV, TW, TA, KIND>, lds);
                    launch_k(e, true, !(do_sketch && e.sp_kind == 0), k_spmv_panel<TV, TW, TA, KIND>,
                             dim3(e.npanels), dim3(64 * kSpmvWaves), lds, e.n, e.rows_pp, e.col_pn, val,
                             (const int4*)e.tiles_pn, e.toff_pn, e.off_pn, e.ptile, x, w, zpart, e.sp, do_sketch));
  if (do_sketch && e.sp_kind == 0) return gauss_t<TW>(e, w, zpart);
  return e.npanels;
}

template <typename TV, typename TW, typename TA, typename TS>
static int spmv_sell_t(const LaunchEnv& e, const TS* val, const TV* x, TW* w, double* zpart, int do_sketch) {
  int G = grid_for(e.nsl, kSpmvWaves, kSellMaxG);
  if (G >= 8) G &= ~7;  // a multiple of the XCD count (see the slice mapping)
  const size_t lds = bins_lds(e, kSpmvWaves, do_sketch && e.sp_kind == 1);
  RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_spmv_sell<TV, TW, TA, KIND, TS>, lds);
                    launch_k(e, true, !(do_sketch && e.sp_kind == 0), k_spmv_sell<TV, TW, TA, KIND, TS>, dim3(G),
                             dim3(64 * kSpmvWaves), lds, e.rp, e.sl_off, e.nsl, e.col_sl, val, e.vtab, e.n, x, w,
                             zpart, e.sp, do_sketch, e.sl_pad0));
  if (do_sketch && e.sp_kind == 0) return gauss_t<TW>(e, w, zpart);
  return G;
}

int launch_spmv_sketch(const LaunchEnv& e, const void* x, void* w, double* zpart, int do_sketch, int prec_override) {
  int prec = prec_override >= 0 ? prec_override : e.prec;
  if (prec == 3) prec = 0;  // the pair basis multiplies FP64 copies of its columns
  if (e.sl) {
    if (prec == 0 && e.vidx_sl)
      return spmv_sell_t<double, double, double, uint8_t>(e, e.vidx_sl, (const double*)x, (double*)w, zpart, do_sketch);
    if (prec == 0) return spmv_sell_t<double, double, double, double>(e, e.val_sl, (const double*)x, (double*)w, zpart, do_sketch);
    if (prec == 1) return spmv_sell_t<float, float, float, float>(e, e.val32_sl, (const float*)x, (float*)w, zpart, do_sketch);
    return spmv_sell_t<bf16_t, float, float, float>(e, e.val32_sl, (const bf16_t*)x, (float*)w, zpart, do_sketch);
  }
  if (e.cb) {
    if (prec == 0) return spmv_panel_t<double, double, double>(e, e.val_pn, (const double*)x, (double*)w, zpart, do_sketch);
    if (prec == 1) return spmv_panel_t<float, float, float>(e, e.val32_pn, (const float*)x, (float*)w, zpart, do_sketch);
    return spmv_panel_t<bf16_t, float, float>(e, e.val32_pn, (const bf16_t*)x, (float*)w, zpart, do_sketch);
  }
  int G = grid_for(e.ntiles, kSpmvWaves, kSpmvMaxG);
  if (G >= 8) G &= ~7;  // a multiple of the XCD count (see the tile mapping)
  dim3 grid(G), block(64 * kSpmvWaves);
  const size_t lds = bins_lds(e, kSpmvWaves, do_sketch && e.sp_kind == 1);
  if (prec == 0 && e.vidx) {  // value-indexed FP64 product
    RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_spmv_sketch<double, double, double, KIND, uint8_t>, lds);
                      launch_k(e, true, !(do_sketch && e.sp_kind == 0), k_spmv_sketch<double, double, double, KIND, uint8_t>,
                               grid, block, lds, e.rp, e.col, e.vidx, e.vtab, (const int4*)e.tiles, e.ntiles,
                               (const double*)x, (double*)w, zpart, e.sp, do_sketch));
  } else if (prec == 0) {
    RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_spmv_sketch<double, double, double, KIND>, lds);
                      launch_k(e, true, !(do_sketch && e.sp_kind == 0), k_spmv_sketch<double, double, double, KIND>, grid, block, lds,
                               e.rp, e.col, e.val, nullptr, (const int4*)e.tiles, e.ntiles, (const double*)x, (double*)w,
                               zpart, e.sp, do_sketch));
  } else if (prec == 1) {
    RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_spmv_sketch<float, float, float, KIND>, lds);
                      launch_k(e, true, !(do_sketch && e.sp_kind == 0), k_spmv_sketch<float, float, float, KIND>, grid, block, lds,
                               e.rp, e.col, e.val32, nullptr, (const int4*)e.tiles, e.ntiles, (const float*)x, (float*)w,
                               zpart, e.sp, do_sketch));
  } else {
    RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_spmv_sketch<bf16_t, float, float, KIND>, lds);
                      launch_k(e, true, !(do_sketch && e.sp_kind == 0), k_spmv_sketch<bf16_t, float, float, KIND>, grid, block, lds,
                               e.rp, e.col, e.val32, nullptr, (const int4*)e.tiles, e.ntiles, (const bf16_t*)x, (float*)w,
                               zpart, e.sp, do_sketch));
  }
  if (do_sketch && e.sp_kind == 0)
    return prec == 0 ? gauss_t<double>(e, (const double*)w, zpart) : gauss_t<float>(e, (const float*)w, zpart);
  return G;
}

void launch_reduce(const LaunchEnv& e, const double* pa, int Ga, const double* pb, int Gb, double* oa, double* ob) {
  dim3 grid((e.sp.d + kRedBins - 1) / kRedBins, 2), block(kRedBins * kRedSl);
  launch_k(e, true, true, k_reduce, grid, block, 0, pa, pb, Ga, Gb, e.sp.d, oa, ob);
}

void launch_ls(const LaunchEnv& e, int t, int pending, int finalize_only, const double* zraw, const double* sraw,
               double* S, double* B, int ldb, double* E, double* cs, double* coef, double* scal, int* flags,
               double bd_rel) {
  const int d = e.sp.d;
  const size_t base = (size_t)(2 * d + 2 * (kMaxM + 2) + 32 + 2 * 64 * 17) * 8;
  const size_t full = base + (size_t)d * (t + 1) * 8;
  const int use_lds = (!finalize_only && full <= kLsLdsMax && (size_t)d * t <= (size_t)kLsPre * 1024) ? 1 : 0;
  const size_t lds = use_lds ? full : base;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_ls, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLsLdsMax);
    attr = true;
  }
  k_ls<<<1, 1024, lds, e.stream>>>(t, d, pending, finalize_only, use_lds, zraw, sraw, S, B, ldb, E, cs, coef,
                                   scal, flags, bd_rel);
}

int launch_update(const LaunchEnv& e, int ncol, const void* U, int64_t ldu, const void* w, const double* coef,
                  void* unew, double* spart) {
  const int V = 16 / e.vbytes();
  const int64_t npk = (e.n + V - 1) / V;
  const int G = grid_for(npk, 1024, kMaxG);
  dim3 grid(G), block(1024);
  const size_t lds = bins_lds(e, 16, e.sp_kind != 0);
  if (e.prec == 0) {
    RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_update<double, double, KIND>, lds);
                      k_update<double, double, KIND><<<grid, block, lds, e.stream>>>(
                          e.n, npk, ncol, (const double*)U, ldu, (const double*)w, coef, (double*)unew, spart, e.sp));
  } else if (e.prec == 1) {
    RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_update<float, float, KIND>, lds);
                      k_update<float, float, KIND><<<grid, block, lds, e.stream>>>(
                          e.n, npk, ncol, (const float*)U, ldu, (const float*)w, coef, (float*)unew, spart, e.sp));
  } else {
    RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_update<bf16_t, float, KIND>, lds);
                      k_update<bf16_t, float, KIND><<<grid, block, lds, e.stream>>>(
                          e.n, npk, ncol, (const bf16_t*)U, ldu, (const float*)w, coef, (bf16_t*)unew, spart, e.sp));
  }
  if (e.sp_kind == 0) {  // sketch of the stored value
    if (e.prec == 0) return gauss_t<double>(e, (const double*)unew, spart);
    if (e.prec == 1) return gauss_t<float>(e, (const float*)unew, spart);
    return gauss_t<bf16_t>(e, (const bf16_t*)unew, spart);
  }
  return G;
}

template <typename TV, typename TW, bool PRE, int PB, bool ROLL, bool SPLIT>
static void ls_update_t(const LaunchEnv& e, dim3 grid, size_t lds, int t, int pending, const double* zraw,
                        const double* sraw, double* S, double* B, int ldb, double* E, double* cs, double* coef,
                        double* scal, int* flags, double bd_rel, int64_t npk, const void* U, int64_t ldu,
                        const void* w, void* unew, double* spart) {
  const int16_t* Ulo = SPLIT ? e.lo_of(U) : nullptr;
  int16_t* unew_lo = SPLIT ? e.lo_of(unew) : nullptr;
  double* xout = SPLIT ? e.xcur : nullptr;
  RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_ls_update<TV, TW, KIND, PRE, PB, ROLL, SPLIT>, lds);
                    launch_k(e, true, e.sp_kind != 0, k_ls_update<TV, TW, KIND, PRE, PB, ROLL, SPLIT>, grid, dim3(1024),
                             lds, t, e.sp.d, pending, zraw, sraw, S, B, ldb, E, cs, coef, scal, flags, bd_rel, e.n,
                             npk, (const TV*)U, ldu, (const TW*)w, (TV*)unew, spart, e.sp, Ulo, unew_lo, xout));
}

int launch_ls_update(const LaunchEnv& e, int t, int pending, const double* zraw, const double* sraw, double* S,
                     double* B, int ldb, double* E, double* cs, double* coef, double* scal, int* flags,
                     double bd_rel, const void* U, int64_t ldu, const void* w, void* unew, double* spart) {
  // 16-byte packets, or 8-byte packets when a column is too short to give
  // 200 CUs a workgroup of 16-byte packets (then twice as many workgroups)
  const int64_t npk16 = (e.n + 16 / e.vbytes() - 1) / (16 / e.vbytes());
  const int PBy = npk16 < 200 * 1024 ? 8 : 16;
  const int V = PBy / e.vbytes();
  const int64_t npk = (e.n + V - 1) / V;
  // at most one workgroup per CU (256): the kernel's registers allow one
  // 1024-thread workgroup per CU anyway, and fewer workgroups repeat the least
  // squares fewer times; the count is trimmed so that every workgroup makes
  // the same number of grid-stride passes
  const int64_t passes = (npk + 256 * 1024 - 1) / (256 * 1024);
  const int G = grid_for(npk, (int)(1024 * passes), 256);
  const size_t ls_work = ls_work_doubles(e.sp.d);
  const size_t bins = e.sp_kind != 0 ? (size_t)16 * e.sp.d : 0;
  const size_t lds = ((size_t)kMaxM + 2 + (ls_work > bins ? ls_work : bins)) * 8;
  // basis loads during the least squares where its own loads all come first
  const bool pre = e.sp.d <= kRC * kLsPreS && t + 1 <= 64 && t + 1 >= kLsPreU;
  // rolling window of column loads (update_body) when each thread walks at
  // least 4 packets: measured faster there (FP64 and FP32 on the 160^3
  // operator), slower with 1 or 2 packets per thread
  // (the pair basis takes no prefetch: its loads of two arrays leave no
  // registers for it)
  const bool roll = !pre && passes >= 4;
#define RKS_LSU_PB(TV, TW, PB, SP)                                                                                    \
  (pre && !SP ? ls_update_t<TV, TW, true, PB, false, SP>(e, dim3(G), lds, t, pending, zraw, sraw, S, B, ldb, E, cs,   \
                                                         coef, scal, flags, bd_rel, npk, U, ldu, w, unew, spart)     \
   : roll ? ls_update_t<TV, TW, false, PB, true, SP>(e, dim3(G), lds, t, pending, zraw, sraw, S, B, ldb, E, cs, coef, \
                                                     scal, flags, bd_rel, npk, U, ldu, w, unew, spart)               \
          : ls_update_t<TV, TW, false, PB, false, SP>(e, dim3(G), lds, t, pending, zraw, sraw, S, B, ldb, E, cs,      \
                                                      coef, scal, flags, bd_rel, npk, U, ldu, w, unew, spart))
#define RKS_LSU(TV, TW, SP) (PBy == 8 ? RKS_LSU_PB(TV, TW, 8, SP) : RKS_LSU_PB(TV, TW, 16, SP))
  if (e.prec == 0) RKS_LSU(double, double, false);
  else if (e.prec == 1) RKS_LSU(float, float, false);
  else if (e.prec == 2) RKS_LSU(bf16_t, float, false);
  else RKS_LSU(float, double, true);
#undef RKS_LSU
#undef RKS_LSU_PB
  if (e.sp_kind == 0) {  // sketch of the stored value (the pair basis: of its FP64 copy)
    if (e.prec == 0) return gauss_t<double>(e, (const double*)unew, spart);
    if (e.prec == 1) return gauss_t<float>(e, (const float*)unew, spart);
    if (e.prec == 2) return gauss_t<bf16_t>(e, (const bf16_t*)unew, spart);
    return gauss_t<double>(e, e.xcur, spart);
  }
  return G;
}

int launch_init(const LaunchEnv& e, void* u, const double* u0, uint32_t s0, uint32_t s1, double* spart, int store,
                int prec_override, uint32_t c2, uint32_t tag) {
  const int prec = prec_override >= 0 ? prec_override : e.prec;
  const int G = grid_for(e.n, 512, kMaxG);
  dim3 grid(G), block(512);
  const size_t lds = bins_lds(e, 8, e.sp_kind != 0);
  if (prec == 0) {
    RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_init<double, KIND>, lds);
                      k_init<double, KIND><<<grid, block, lds, e.stream>>>(e.n, (double*)u, u0, s0, s1, c2, tag, spart, e.sp,
                                                                        store));
  } else if (prec == 1) {
    RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_init<float, KIND>, lds);
                      k_init<float, KIND><<<grid, block, lds, e.stream>>>(e.n, (float*)u, u0, s0, s1, c2, tag, spart, e.sp,
                                                                        store));
  } else if (prec == 2) {
    RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_init<bf16_t, KIND>, lds);
                      k_init<bf16_t, KIND><<<grid, block, lds, e.stream>>>(e.n, (bf16_t*)u, u0, s0, s1, c2, tag, spart, e.sp,
                                                                        store));
  } else {
    RKS_SKETCH_SWITCH(e.sp_kind, lds_allow((const void*)k_init<float, KIND, true>, lds);
                      k_init<float, KIND, true><<<grid, block, lds, e.stream>>>(
                          e.n, (float*)u, u0, s0, s1, c2, tag, spart, e.sp, store, store ? e.lo_of(u) : nullptr,
                          e.xcur));
  }
  if (e.sp_kind == 0) {
    // sketch of the stored value; without a store, of u0 itself (FP64 only)
    if (!store) return u0 ? gauss_t<double>(e, u0, spart) : 0;
    if (prec == 0) return gauss_t<double>(e, (const double*)u, spart);
    if (prec == 1) return gauss_t<float>(e, (const float*)u, spart);
    if (prec == 2) return gauss_t<bf16_t>(e, (const bf16_t*)u, spart);
    return gauss_t<double>(e, e.xcur, spart);
  }
  return G;
}

template <typename TI, typename TO, int NT, bool SPLIT>
static void rotate_nt(const LaunchEnv& e, const TI* U, int64_t ldu, int in0, int min, TO* O, int64_t ldo, int out0,
                      int kout, const double* Y, int xsrc, int xdst, double xscale) {
  constexpr int R = rot_rows<TI>(NT);
  const int64_t ntile = (e.n + 16 * R - 1) / (16 * R);
  const int G = grid_for(ntile, 4, 2048);
  const size_t lds = (size_t)((min + 15) & ~15) * 16 * NT * 8;
  // the pair basis: the bfloat16 parts of the input, of an FP32 output, and
  // the FP64 copy of the column xdst
  const int16_t* Ulo = SPLIT ? e.lo_of(U) : nullptr;
  int16_t* Olo = SPLIT && sizeof(TO) == 4 ? e.lo_of(O) : nullptr;
  double* xcur = SPLIT && xsrc >= 0 ? e.xcur : nullptr;
  if (lds > kRotLdsMax) {
    launch_k(e, true, true, k_rotate<TI, TO, NT, true, R, SPLIT>, dim3(G), dim3(256), 0, e.n, U, ldu, in0, min, O,
             ldo, out0, kout, Y, xsrc, xdst, xscale, Ulo, Olo, xcur);
    return;
  }
  lds_allow((const void*)k_rotate<TI, TO, NT, false, R, SPLIT>, lds);
  launch_k(e, true, true, k_rotate<TI, TO, NT, false, R, SPLIT>, dim3(G), dim3(256), lds, e.n, U, ldu, in0, min, O,
           ldo, out0, kout, Y, xsrc, xdst, xscale, Ulo, Olo, xcur);
}

template <typename TI, typename TO, bool SPLIT = false>
static void rotate_t(const LaunchEnv& e, const TI* U, int64_t ldu, int in0, int min, TO* O, int64_t ldo, int out0,
                     int kout, const double* Y, int xsrc, int xdst, double xscale) {
#define RKS_ROT(NT) rotate_nt<TI, TO, NT, SPLIT>(e, U, ldu, in0, min, O, ldo, out0, kout, Y, xsrc, xdst, xscale)
  switch ((kout + 15) / 16) {
    case 0:
    case 1: RKS_ROT(1); break;
    case 2: RKS_ROT(2); break;
    case 3: RKS_ROT(3); break;
    case 4: RKS_ROT(4); break;
    case 5: RKS_ROT(5); break;
    case 6: RKS_ROT(6); break;
    case 7: RKS_ROT(7); break;
    default: RKS_ROT(8); break;
  }
#undef RKS_ROT
}

void launch_rotate(const LaunchEnv& e, const void* U, int64_t ldu, int in0, int min, void* O, int64_t ldo, int out0,
                   int kout, const double* Y, int xsrc, int xdst, double xscale, int out_fp64) {
  if (e.prec == 0) {
    rotate_t<double, double>(e, (const double*)U, ldu, in0, min, (double*)O, ldo, out0, kout, Y, xsrc, xdst, xscale);
  } else if (e.prec == 1) {
    if (out_fp64)
      rotate_t<float, double>(e, (const float*)U, ldu, in0, min, (double*)O, ldo, out0, kout, Y, xsrc, xdst, xscale);
    else
      rotate_t<float, float>(e, (const float*)U, ldu, in0, min, (float*)O, ldo, out0, kout, Y, xsrc, xdst, xscale);
  } else if (e.prec == 2) {
    if (out_fp64)
      rotate_t<bf16_t, double>(e, (const bf16_t*)U, ldu, in0, min, (double*)O, ldo, out0, kout, Y, xsrc, xdst,
                               xscale);
    else
      rotate_t<bf16_t, bf16_t>(e, (const bf16_t*)U, ldu, in0, min, (bf16_t*)O, ldo, out0, kout, Y, xsrc, xdst,
                               xscale);
  } else {
    if (out_fp64)
      rotate_t<float, double, true>(e, (const float*)U, ldu, in0, min, (double*)O, ldo, out0, kout, Y, xsrc, xdst,
                                    xscale);
    else
      rotate_t<float, float, true>(e, (const float*)U, ldu, in0, min, (float*)O, ldo, out0, kout, Y, xsrc, xdst,
                                   xscale);
  }
}

int launch_resid(const LaunchEnv& e, const double* xa, const double* xb, const double* axa, const double* axb,
                 double re, double im, double* part) {
  const int G = grid_for(e.n, 256, kMaxG);
  k_resid<<<G, 256, 0, e.stream>>>(e.n, xa, xb, axa, axb, re, im, part);
  return G;
}

void launch_scale(const LaunchEnv& e, double* x, double s) {
  k_scale<<<grid_for(e.n, 256, kMaxG), 256, 0, e.stream>>>(e.n, x, s);
}

int launch_dots(const LaunchEnv& e, int ncol, const void* U, int64_t ldu, const void* x, int x_is_basis, double* part) {
  const int V = 16 / e.vbytes();
  const int64_t npk = (e.n + V - 1) / V;
  const int G = grid_for(npk, 1024, kMaxG);
  if (e.prec == 0) {
    k_dots<double, double><<<G, 1024, 0, e.stream>>>(e.n, npk, ncol, (const double*)U, ldu, (const double*)x, part);
  } else if (e.prec == 1) {
    k_dots<float, float><<<G, 1024, 0, e.stream>>>(e.n, npk, ncol, (const float*)U, ldu, (const float*)x, part);
  } else if (x_is_basis) {
    k_dots<bf16_t, bf16_t><<<G, 1024, 0, e.stream>>>(e.n, npk, ncol, (const bf16_t*)U, ldu, (const bf16_t*)x, part);
  } else {
    k_dots<bf16_t, float><<<G, 1024, 0, e.stream>>>(e.n, npk, ncol, (const bf16_t*)U, ldu, (const float*)x, part);
  }
  return G;
}

void launch_reduce_len(const LaunchEnv& e, const double* pa, int Ga, double* oa, int len) {
  dim3 grid((len + kRedBins - 1) / kRedBins, 1), block(kRedBins * kRedSl);
  k_reduce<<<grid, block, 0, e.stream>>>(pa, nullptr, Ga, 0, len, oa, nullptr);
}

void launch_ks_coef(const LaunchEnv& e, int ncol, const double* cs, const double* yraw, double scale,
                    const double* scale_ptr, double* coef, double* h, int accumulate) {
  k_ks_coef<<<1, 256, 0, e.stream>>>(ncol, cs, yraw, scale, scale_ptr, coef, h, accumulate);
}

__global__ void k_ks_start(const double* __restrict__ nrm2, double* __restrict__ cs) {
  if (threadIdx.x == 0) cs[0] = 1.0 / sqrt(*nrm2);
}

void launch_ks_start(const LaunchEnv& e, const double* nrm2, double* cs) { k_ks_start<<<1, 64, 0, e.stream>>>(nrm2, cs); }

void launch_ks_finalize(const LaunchEnv& e, int t, const double* h, const double* nrm2, double* B, int ldb, double* cs,
                        int* flags, double bd_rel) {
  k_ks_finalize<<<1, 256, 0, e.stream>>>(t, h, nrm2, B, ldb, cs, flags, bd_rel);
}

// ---------------------------------------------------------------------------
// No-allocation sketch: the partial rows live in a fixed device array of the
// library instead of a context's buffer.  In host code `scratch` names a
// host-side stand-in, not a device address: its address on the current
// device is obtained once per device with hipGetSymbolAddress and only that
// address is passed to kernels.
constexpr int kScratchDevices = 64;
static __device__ __align__(256) double scratch[(size_t)kMaxG * kMaxD];

int scratch_address(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return -1;
  static std::mutex mu;
  static double* addr[kScratchDevices] = {};
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return -2;
    addr[dev] = (double*)p;
  }
  *out = addr[dev];
  return 0;
}

int launch_sketch_scratch(const LaunchEnv& e, const double* x, double* part, double* z) {
  // the kernels and grid of launch_init (store = 0) and launch_reduce, with
  // no host-side bookkeeping: the bins of 8 waves x d <= 1024 FP64 fit the
  // default 64 KB of dynamic LDS
  int G;
  if (e.sp_kind == 0) {
    G = gauss_t<double>(e, x, part);
  } else {
    G = grid_for(e.n, 512, kMaxG);
    const size_t lds = bins_lds(e, 8, true);
    k_init<double, 1><<<G, 512, lds, e.stream>>>(e.n, nullptr, x, 0u, 0u, 0u, 2u, part, e.sp, 0);
  }
  launch_reduce(e, part, G, nullptr, 0, z, nullptr);
  return G;
}

void launch_read16(hipStream_t stream, const void* src, int64_t packets) {
  k_read16<<<grid_for(packets, 256, 8192), 256, 0, stream>>>((const u32x4*)src, packets);
}

void launch_copy16(hipStream_t stream, const void* src, void* dst, int64_t packets) {
  k_copy16<<<grid_for(packets, 256, 8192), 256, 0, stream>>>((const u32x4*)src, (u32x4*)dst, packets);
}

void launch_fill(const LaunchEnv& e, int64_t len, double* x, double v) {
  k_fill<<<grid_for(len, 256, kMaxG), 256, 0, e.stream>>>(len, x, v);
}

}  // namespace rks
