// Column-blocked SpMV layout (see panels.hpp).
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

}  // namespace rks
