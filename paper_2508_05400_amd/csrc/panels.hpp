// Host-side SpMV layouts: column-blocked (row panels x column blocks) and sliced.
//
// The columns are split into kCb contiguous blocks of ceil(n / kCb) columns
// and the rows into panels of rows_pp consecutive rows (the last panel may be
// shorter).  Inside a panel the nonzeros are stored block after block, and
// inside a block row after row with the columns in increasing order, so the
// workgroup that owns a panel streams one contiguous range of the arrays.
// Each (panel, block) is cut into tiles of consecutive rows: at most
// kPanelTileRows rows and kTileFill nonzeros, or one row with more than
// kTileFill nonzeros in that block (a long tile).  A tile's rows start at
// 16-bit offsets from its first nonzero: tile t of nr rows owns
// off[toff[t] .. toff[t] + nr] (nr + 1 values, the last = its nonzeros);
// a long tile has toff[t] = -1 and no offsets.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "layout.hpp"

namespace rks {

struct PanelLayout {
  int64_t rows_pp = 0;          // rows per panel
  int npanels = 0;
  std::vector<int32_t> col;     // nnz column indices in panel / block / row order
  std::vector<double> val;      // the matching values
  std::vector<int32_t> tiles;   // 4 per tile: first row within the panel, rows, first nonzero, nonzeros
  std::vector<int32_t> toff;    // per tile: first offset in `off`, or -1 for a long tile
  std::vector<uint16_t> off;    // row offsets of the tiles
  std::vector<int32_t> ptile;   // (kCb + 1) per panel: first tile of each block, then the end
};

// Rows per panel for n rows: enough panels for one workgroup per SpMV slot
// (kSpmvMaxG), with kPanelRowsMin <= rows_pp <= kPanelRowsMax.
int64_t panel_rows(int64_t n);

// Builds the layout of the n x n CSR matrix (rp, col, val: columns strictly
// increasing in each row, as validated by the caller).  Returns false with a
// reason if an index of the layout would overflow 32 bits.
bool build_panels(int64_t n, const int32_t* rp, const int32_t* col, const double* val, PanelLayout& L,
                  std::string& why);

// Sliced layout (host side): slices of kSliceRows consecutive rows, each
// padded to its longest row; slice s holds entries off[s] .. off[s+1] - 1,
// entry (k, lane) at off[s] + kSliceRows k + lane being the k-th nonzero of
// row kSliceRows s + lane, or padding.  slice_offsets fills off (nslices + 1
// values; off[nslices] = padded entries).  build_slices fills, per entry, its
// column and src, the index of its nonzero in the CSR arrays, or -1 for
// padding, whose column is the row's first (the row itself if the row is
// empty, 0 past n), so that every entry's column is a valid index of x.
void slice_offsets(int64_t n, const int32_t* rp, std::vector<int64_t>& off);
void build_slices(int64_t n, const int32_t* rp, const int32_t* col, const std::vector<int64_t>& off,
                  std::vector<int32_t>& scol, std::vector<int32_t>& src);

}  // namespace rks
