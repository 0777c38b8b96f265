// Host check of the sliced SpMV layout (slice_offsets and build_slices in
// csrc/panels.cpp), built with AddressSanitizer and
// UndefinedBehaviorSanitizer.  For matrices with empty rows, whole slices of
// empty rows, rows of up to 700 nonzeros and a ragged last slice it checks
// the offsets (each slice padded to its longest row), that every nonzero
// lands once at (slice, k, lane) with its column, that every entry's column
// is a valid index of x, and that a walk in the kernel's order (each row's
// entries k = 0, 1, ... with padding weighted 0) gives the CSR product to
// the bit.  Prints "ok: 0 failures" at the end when all pass.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "panels.hpp"

using namespace rks;

static int failures = 0;
#define CHECK(cond, ...)               \
  do {                                 \
    if (!(cond)) {                     \
      ++failures;                      \
      std::printf("FAIL %s: ", #cond); \
      std::printf(__VA_ARGS__);        \
      std::printf("\n");               \
      if (failures > 20) return;       \
    }                                  \
  } while (0)

static uint64_t lcg(uint64_t& s) {
  s = s * 6364136223846793005ull + 1442695040888963407ull;
  return s >> 17;
}

// rows of 0..maxlen nonzeros (sorted, distinct columns), rows [g0, g1) empty
static void make(int64_t n, int maxlen, int64_t g0, int64_t g1, uint64_t seed, std::vector<int32_t>& rp,
                 std::vector<int32_t>& col, std::vector<double>& val) {
  rp.assign(n + 1, 0);
  col.clear();
  val.clear();
  uint64_t s = seed;
  for (int64_t r = 0; r < n; ++r) {
    int len = (int)(lcg(s) % (uint64_t)(maxlen + 1));
    if (r >= g0 && r < g1) len = 0;
    if (len > n) len = (int)n;
    std::vector<char> used(n, 0);
    std::vector<int32_t> cs;
    while ((int)cs.size() < len) {
      const int32_t c = (int32_t)(lcg(s) % (uint64_t)n);
      if (!used[c]) {
        used[c] = 1;
        cs.push_back(c);
      }
    }
    std::sort(cs.begin(), cs.end());
    for (int32_t c : cs) {
      col.push_back(c);
      val.push_back((double)(int64_t)(lcg(s) % 2001) / 1000.0 - 1.0);
    }
    rp[r + 1] = (int32_t)col.size();
  }
}

static void check(int64_t n, int maxlen, int64_t g0, int64_t g1, uint64_t seed) {
  std::vector<int32_t> rp, col;
  std::vector<double> val;
  make(n, maxlen, g0, g1, seed, rp, col, val);
  const int64_t nnz = rp[n];
  std::vector<int64_t> off;
  slice_offsets(n, rp.data(), off);
  const int64_t ns = (n + kSliceRows - 1) / kSliceRows;
  CHECK((int64_t)off.size() == ns + 1, "n %lld: %zu offsets", (long long)n, off.size());
  CHECK(off[0] == 0, "first offset %lld", (long long)off[0]);
  for (int64_t s = 0; s < ns; ++s) {
    int32_t ml = 0;
    for (int64_t r = s * kSliceRows; r < std::min<int64_t>(n, (s + 1) * kSliceRows); ++r)
      ml = std::max(ml, rp[r + 1] - rp[r]);
    CHECK(off[s + 1] - off[s] == (int64_t)kSliceRows * ml, "slice %lld: %lld entries, longest row %d", (long long)s,
          (long long)(off[s + 1] - off[s]), ml);
  }
  std::vector<int32_t> scol, src;
  build_slices(n, rp.data(), col.data(), off, scol, src);
  const int64_t P = off[ns];
  CHECK((int64_t)scol.size() == P && (int64_t)src.size() == P, "sizes %zu %zu, %lld entries", scol.size(),
        src.size(), (long long)P);
  std::vector<int> seen(nnz, 0);
  for (int64_t e = 0; e < P; ++e) {
    CHECK(scol[e] >= 0 && scol[e] < n, "entry %lld column %d (n %lld)", (long long)e, scol[e], (long long)n);
    if (src[e] >= 0) {
      CHECK(src[e] < nnz, "entry %lld source %d", (long long)e, src[e]);
      seen[src[e]] += 1;
      CHECK(scol[e] == col[src[e]], "entry %lld column %d, nonzero's %d", (long long)e, scol[e], col[src[e]]);
    }
  }
  for (int64_t j = 0; j < nnz; ++j) CHECK(seen[j] == 1, "nonzero %lld seen %d times", (long long)j, seen[j]);
  // positions, and the product in the kernel's order
  std::vector<double> x(n);
  uint64_t sx = seed ^ 0x9E3779B97F4A7C15ull;
  for (auto& v : x) v = (double)(int64_t)(lcg(sx) % 4001) / 1000.0 - 2.0;
  for (int64_t s = 0; s < ns; ++s) {
    const int64_t slen = (off[s + 1] - off[s]) / kSliceRows;
    for (int lane = 0; lane < kSliceRows; ++lane) {
      const int64_t r = s * kSliceRows + lane;
      if (r >= n) continue;
      double ys = 0.0, yc = 0.0;
      for (int64_t k = 0; k < slen; ++k) {
        const int64_t e = off[s] + k * kSliceRows + lane;
        if (k < rp[r + 1] - rp[r]) CHECK(src[e] == rp[r] + k, "row %lld k %lld source %d", (long long)r, (long long)k, src[e]);
        else CHECK(src[e] == -1, "row %lld k %lld padding source %d", (long long)r, (long long)k, src[e]);
        ys += (src[e] >= 0 ? val[src[e]] : 0.0) * x[scol[e]];
      }
      for (int32_t j = rp[r]; j < rp[r + 1]; ++j) yc += val[j] * x[col[j]];
      CHECK(ys == yc, "row %lld: %.17g against %.17g", (long long)r, ys, yc);
    }
  }
}

int main() {
  check(1, 1, 0, 0, 1);
  check(5, 3, 2, 3, 2);
  check(63, 9, 0, 0, 3);
  check(64, 9, 0, 64, 4);         // one slice, all rows empty
  check(65, 9, 64, 65, 5);        // the ragged last slice is one empty row
  check(1000, 12, 64, 192, 6);    // two whole slices of empty rows
  check(4099, 20, 700, 701, 7);
  check(3000, 700, 0, 0, 8);      // long rows: heavy padding
  std::printf("ok: %d failures\n", failures);
  return failures ? 1 : 0;
}
