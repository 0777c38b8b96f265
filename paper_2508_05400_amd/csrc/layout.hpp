// Sizes of the SpMV data layouts, shared by the kernels (kernels.hip) and the
// host code that builds the layouts (rks_api.cpp, panels.cpp).  Plain C++: no
// HIP types, so host-only code can include it.
#pragma once
#include <stddef.h>

namespace rks {

constexpr int kTileRows = 64;    // rows per SpMV wave tile
constexpr int kTileNnz = 512;    // nonzeros staged per SpMV wave tile (LDS slice)
constexpr int kTileFill = kTileNnz - 2;  // nonzeros a tile may hold: paired loads start at the even
                                         // index at or below its first nonzero
constexpr int kCsrPad = 2;       // readable padding entries after col[] and val[] (paired loads)
constexpr int kSpmvWaves = 4;    // waves per SpMV workgroup
constexpr int kSpmvMaxG = 1280;  // SpMV workgroups at most (5 per CU: LDS-bound for FP64 with d <= 360)

// Sliced layout: slices of kSliceRows consecutive rows (one per lane of a
// wave), each stored k-th nonzero of every row together; at most
// kSellMaxG workgroups of kSpmvWaves waves (6 per CU; no product staging in
// LDS, only the sketch bins).
constexpr int kSliceRows = 64;
constexpr int kSellMaxG = 1536;

// Column-blocked layout (operators whose rows gather x from everywhere):
// kCb column blocks (n / kCb values of x, which fit in an XCD's L2); row
// panels of consecutive rows, one workgroup each; panel tiles of up to
// kPanelTileRows rows.  Measured on a 2M-row power-law operator: 4, 16 or 32
// blocks and 128-row tiles are slower, as are twice as many, smaller panels.
constexpr int kCb = 8;
constexpr int kPanelTileRows = 256;
constexpr int kPanelRowsMin = 64;    // rows per panel at least (small matrices)
constexpr int kPanelRowsMax = 4096;  // rows per panel at most (the row sums live in LDS)

}  // namespace rks
