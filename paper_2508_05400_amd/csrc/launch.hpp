// Host-side launchers of the hot-path kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace rks {

// What every launch needs to know about the operator and the sketch.
struct LaunchEnv {
  hipStream_t stream;
  int64_t n;
  int prec;            // 0 FP64 basis, 1 FP32 basis, 2 BF16 basis, 3 pair basis (FP32 + 16-bit remainder)
  const int* rp;       // CSR row pointers (device)
  const int* col;      // CSR columns (device)
  const double* val;   // FP64 values (device)
  const float* val32;  // FP32 values (device, mixed precision only)
  // value-indexed storage of A for the FP64 product (row tiles; null when
  // unused): one byte per nonzero indexing vtab, the matrix's distinct FP64
  // values (256 entries, unused ones zero)
  const uint8_t* vidx = nullptr;
  const double* vtab = nullptr;
  const int* tiles;    // SpMV wave tiles: {first row, rows, first nonzero, nonzeros} per tile
  int ntiles;
  int64_t ldu;         // basis leading dimension (n rounded up to 128; padding rows are zero)
  int sp_kind;         // 0 Gaussian (applied by k_gauss_sketch), 1 sparse-sign, 2 none (deterministic KS)
  SketchP sp;
  // column-blocked SpMV (used when cb = 1): the layout of panels.hpp, one
  // workgroup per row panel of rows_pp rows
  int cb = 0;
  int npanels = 0;
  int rows_pp = 0;
  const int* col_pn = nullptr;
  const double* val_pn = nullptr;
  const float* val32_pn = nullptr;  // mixed precision only
  const int* tiles_pn = nullptr;    // 4 per tile: first row within the panel, rows, first nonzero, nonzeros
  const int* toff_pn = nullptr;     // per tile: first row offset, -1 for a long tile
  const uint16_t* off_pn = nullptr; // row offsets of the tiles
  const int* ptile = nullptr;       // (kCb + 1) per panel: first tile of each column block, then the end
  // sliced layout (used when sl = 1): nsl slices of kSliceRows rows; slice s
  // holds entries sl_off[s] .. sl_off[s+1] - 1, entry (k, lane) at
  // sl_off[s] + kSliceRows k + lane (the k-th nonzero of row kSliceRows s +
  // lane; rows shorter than the slice's longest are padded, see sl_pad0)
  int sl = 0;
  int nsl = 0;
  const int64_t* sl_off = nullptr;
  const int* col_sl = nullptr;
  const double* val_sl = nullptr;    // FP64 values (unless value-indexed)
  const uint8_t* vidx_sl = nullptr;  // value indices (value-indexed storage)
  const float* val32_sl = nullptr;   // mixed precision only
  int sl_pad0 = 0;                   // padding holds +0.0 (added like the nonzeros; no row lengths read)
  // Timing (null when off): a launcher that runs with these set records ev0 at
  // the start of its first kernel and ev1 at the end of its last one, from the
  // dispatches' own timestamps (no marker packets between the kernels).
  hipEvent_t ev0 = nullptr;
  hipEvent_t ev1 = nullptr;
  // the pair basis (prec 3): the FP32 parts at pair_hi (the basis pointer the
  // launchers get), the 16-bit remainders of the same elements at pair_lo, and
  // xcur (ldu FP64 values, padding rows zero), the FP64 copy of the column
  // written last, which the SpMV of the next step reads
  const float* pair_hi = nullptr;
  int16_t* pair_lo = nullptr;
  double* xcur = nullptr;
  int16_t* lo_of(const void* hi) const { return pair_lo + ((const float*)hi - pair_hi); }
  // bytes between consecutive rows of a basis column (the pair basis: of its FP32 part)
  int vbytes() const { return prec == 0 ? 8 : (prec == 2 ? 2 : 4); }
};

// w = A x, partials of Omega w (returns the number of partial rows: at most
// kMaxPart for the row tiles, npanels for the column-blocked layout).  For the
// pair basis (prec 3) x and w are FP64.
int launch_spmv_sketch(const LaunchEnv& e, const void* x, void* w, double* zpart, int do_sketch, int prec_override);
void launch_reduce(const LaunchEnv& e, const double* pa, int Ga, const double* pb, int Gb, double* oa, double* ob);
// E = S^T S - I ((m+1) x (m+1), leading dimension ldb), kept current column by column.
void launch_ls(const LaunchEnv& e, int t, int pending, int finalize_only, const double* zraw, const double* sraw,
               double* S, double* B, int ldb, double* E, double* cs, double* coef, double* scal, int* flags,
               double bd_rel);
// (FP64, FP32 and BF16 bases: the deterministic Krylov-Schur step, which
// takes no pair basis)
int launch_update(const LaunchEnv& e, int ncol, const void* U, int64_t ldu, const void* w, const double* coef,
                  void* unew, double* spart);
// Least squares (as launch_ls, not finalize-only) and update (as launch_update
// with ncol = t + 1) in one launch; returns the number of partial rows.
int launch_ls_update(const LaunchEnv& e, int t, int pending, const double* zraw, const double* sraw, double* S,
                     double* B, int ldb, double* E, double* cs, double* coef, double* scal, int* flags,
                     double bd_rel, const void* U, int64_t ldu, const void* w, void* unew, double* spart);
// u = u0, or the seeded N(0,1) vector of Philox counter (i, c2, tag) (tag 2:
// start vector, tag 3: breakdown replacement), stored in the basis type (or
// prec_override's); partials of Omega of the stored value.  The pair basis
// (prec 3) also writes the stored value to xcur.
int launch_init(const LaunchEnv& e, void* u, const double* u0, uint32_t s0, uint32_t s1, double* spart, int store,
                int prec_override, uint32_t c2 = 0, uint32_t tag = 2);
// O(:, out0 .. out0 + kout) = U(:, in0 .. in0 + min) Y.  ldu must be a multiple of
// 128 (the kernel reads whole row tiles up to ldu); O's rows >= n are not written.
void launch_rotate(const LaunchEnv& e, const void* U, int64_t ldu, int in0, int min, void* O, int64_t ldo, int out0,
                   int kout, const double* Y, int xsrc, int xdst, double xscale, int out_fp64);
int launch_resid(const LaunchEnv& e, const double* xa, const double* xb, const double* axa, const double* axb,
                 double re, double im, double* part);
void launch_scale(const LaunchEnv& e, double* x, double s);
void launch_fill(const LaunchEnv& e, int64_t len, double* x, double v);
void launch_copy16(hipStream_t stream, const void* src, void* dst, int64_t packets);
void launch_read16(hipStream_t stream, const void* src, int64_t packets);
// Deterministic Krylov-Schur (Euclidean classical Gram-Schmidt, twice):
// partials of U(:, 0:ncol)^T x (returns the number of partial rows), their sum,
// the coefficients of one pass, and the closing of a step.
int launch_dots(const LaunchEnv& e, int ncol, const void* U, int64_t ldu, const void* x, int x_is_basis, double* part);
void launch_reduce_len(const LaunchEnv& e, const double* pa, int Ga, double* oa, int len);
void launch_ks_coef(const LaunchEnv& e, int ncol, const double* cs, const double* yraw, double scale,
                    const double* scale_ptr, double* coef, double* h, int accumulate);
void launch_ks_finalize(const LaunchEnv& e, int t, const double* h, const double* nrm2, double* B, int ldb, double* cs,
                        int* flags, double bd_rel);
void launch_ks_start(const LaunchEnv& e, const double* nrm2, double* cs);
// Device address of the library's fixed sketch scratch (kMaxG x kMaxD FP64)
// on the current device, resolved once per device; 0 on success.
int scratch_address(double** out);
// z = Omega x with partial rows in `part` (at least kMaxG x d FP64): the
// kernels of launch_init (store = 0) and launch_reduce, no host allocation.
int launch_sketch_scratch(const LaunchEnv& e, const double* x, double* part, double* z);

}  // namespace rks
