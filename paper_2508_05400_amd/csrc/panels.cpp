// Host-side SpMV layouts: column blocks and slices (see panels.hpp).
#include "panels.hpp"

#include <algorithm>
#include <limits>

namespace rks {

int64_t panel_rows(int64_t n) {
  int64_t r = (n + kSpmvMaxG - 1) / kSpmvMaxG;
  return std::min<int64_t>(std::max<int64_t>(r, kPanelRowsMin), kPanelRowsMax);
}

bool build_panels(int64_t n, const int32_t* rp, const int32_t* col, const double* val, PanelLayout& L,
                  std::string& why) {
  const int64_t nnz = n > 0 ? rp[n] : 0;
  const int64_t bw = std::max<int64_t>((n + kCb - 1) / kCb, 1);  // columns per block
  L = PanelLayout();
  L.rows_pp = panel_rows(n);
  const int64_t np = n > 0 ? (n + L.rows_pp - 1) / L.rows_pp : 0;
  if (np > std::numeric_limits<int32_t>::max() / (kCb + 1)) {
    why = "too many row panels for the column-blocked layout";
    return false;
  }
  L.npanels = (int)np;
  L.col.resize(nnz);
  L.val.resize(nnz);
  L.ptile.reserve((size_t)np * (kCb + 1));
  std::vector<int32_t> cnt, pos;  // per (block, row of the panel)
  int64_t base = 0;               // first nonzero of the panel
  for (int64_t p = 0; p < np; ++p) {
    const int64_t r0 = p * L.rows_pp, nr = std::min(L.rows_pp, n - r0);
    cnt.assign((size_t)kCb * nr, 0);
    for (int64_t r = 0; r < nr; ++r)
      for (int64_t e = rp[r0 + r]; e < rp[r0 + r + 1]; ++e) ++cnt[(size_t)(col[e] / bw) * nr + r];
    // positions: block after block, row after row
    pos.resize(cnt.size());
    int64_t at = base;
    for (size_t i = 0; i < cnt.size(); ++i) {
      pos[i] = (int32_t)at;
      at += cnt[i];
    }
    for (int64_t r = 0; r < nr; ++r)
      for (int64_t e = rp[r0 + r]; e < rp[r0 + r + 1]; ++e) {
        int32_t& q = pos[(size_t)(col[e] / bw) * nr + r];
        L.col[q] = col[e];
        L.val[q] = val[e];
        ++q;
      }
    // tiles of each block
    int64_t e0 = base;  // first nonzero of the current row
    for (int c = 0; c < kCb; ++c) {
      L.ptile.push_back((int32_t)(L.tiles.size() / 4));
      const int32_t* cc = &cnt[(size_t)c * nr];
      for (int64_t r = 0; r < nr;) {
        if (cc[r] > kTileFill) {  // a long tile
          L.tiles.insert(L.tiles.end(), {(int32_t)r, 1, (int32_t)e0, cc[r]});
          L.toff.push_back(-1);
          e0 += cc[r];
          ++r;
          continue;
        }
        const int64_t s0 = r;
        int32_t acc = 0;
        while (r < nr && r - s0 < kPanelTileRows && acc + cc[r] <= kTileFill) acc += cc[r++];
        if (L.off.size() > (size_t)std::numeric_limits<int32_t>::max() - kPanelTileRows - 1) {
          why = "too many row offsets for the column-blocked layout";
          return false;
        }
        L.tiles.insert(L.tiles.end(), {(int32_t)s0, (int32_t)(r - s0), (int32_t)e0, acc});
        L.toff.push_back((int32_t)L.off.size());
        int32_t o = 0;
        for (int64_t q = s0; q < r; ++q) {
          L.off.push_back((uint16_t)o);
          o += cc[q];
        }
        L.off.push_back((uint16_t)o);
        e0 += acc;
      }
    }
    L.ptile.push_back((int32_t)(L.tiles.size() / 4));
    base = at;
    if (L.tiles.size() / 4 > (size_t)std::numeric_limits<int32_t>::max() - kCb) {
      why = "too many tiles for the column-blocked layout";
      return false;
    }
  }
  return true;
}

void slice_offsets(int64_t n, const int32_t* rp, std::vector<int64_t>& off) {
  const int64_t ns = (n + kSliceRows - 1) / kSliceRows;
  off.assign(ns + 1, 0);
  for (int64_t s = 0; s < ns; ++s) {
    int32_t ml = 0;
    for (int64_t r = s * kSliceRows; r < std::min<int64_t>(n, (s + 1) * kSliceRows); ++r)
      ml = std::max(ml, rp[r + 1] - rp[r]);
    off[s + 1] = off[s] + (int64_t)kSliceRows * ml;
  }
}

void build_slices(int64_t n, const int32_t* rp, const int32_t* col, const std::vector<int64_t>& off,
                  std::vector<int32_t>& scol, std::vector<int32_t>& src) {
  const int64_t ns = (int64_t)off.size() - 1, P = off[ns];
  scol.assign((size_t)P, 0);
  src.assign((size_t)P, -1);
  for (int64_t s = 0; s < ns; ++s) {
    const int64_t b0 = off[s], slen = (off[s + 1] - b0) / kSliceRows;
    for (int lane = 0; lane < kSliceRows; ++lane) {
      const int64_t r = s * kSliceRows + lane;
      const int64_t len = r < n ? rp[r + 1] - rp[r] : 0;
      const int32_t pad = len > 0 ? col[rp[r]] : (int32_t)(r < n ? r : 0);
      for (int64_t k = 0; k < slen; ++k) {
        const size_t e = (size_t)(b0 + k * kSliceRows + lane);
        if (k < len) {
          scol[e] = col[rp[r] + k];
          src[e] = (int32_t)(rp[r] + k);
        } else {
          scol[e] = pad;
        }
      }
    }
  }
}

}  // namespace rks
