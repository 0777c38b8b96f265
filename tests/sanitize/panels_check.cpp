// Host check of the column-blocked SpMV layout (csrc/panels.cpp), built with
// AddressSanitizer and UndefinedBehaviorSanitizer.  For several matrices it
// checks the layout's invariants, including every read the GPU kernel
// (k_spmv_panel) makes: the paired nonzero loads stay inside the padded
// arrays, the row offsets inside `off`, the rows inside their panel.  It then
// walks the layout the way the kernel does (block after block, tile after
// tile, each row summed from its offsets) and compares the product with a
// plain CSR product.  Prints "ok: 0 failures" at the end when all pass.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "panels.hpp"

using namespace rks;

static int failures = 0;
#define CHECK(cond, ...)                      \
  do {                                        \
    if (!(cond)) {                            \
      ++failures;                             \
      std::printf("FAIL %s: ", #cond);        \
      std::printf(__VA_ARGS__);               \
      std::printf("\n");                      \
      if (failures > 20) return;              \
    }                                         \
  } while (0)

struct Csr {
  int64_t n = 0;
  std::vector<int32_t> rp, col;
  std::vector<double> val;
};

static uint64_t lcg(uint64_t& s) {
  s = s * 6364136223846793005ull + 1442695040888963407ull;
  return s >> 17;
}

// a row of `len` distinct sorted columns drawn from [lo, hi), random values
static void add_row(Csr& A, uint64_t& s, int64_t len, int64_t lo, int64_t hi) {
  std::vector<int32_t> cs;
  len = std::min<int64_t>(len, hi - lo);
  while ((int64_t)cs.size() < len) {
    for (int64_t i = (int64_t)cs.size(); i < len; ++i) cs.push_back((int32_t)(lo + (int64_t)(lcg(s) % (uint64_t)(hi - lo))));
    std::sort(cs.begin(), cs.end());
    cs.erase(std::unique(cs.begin(), cs.end()), cs.end());
  }
  for (int32_t c : cs) {
    A.col.push_back(c);
    A.val.push_back(((double)(lcg(s) % 2000001) - 1000000.0) / 1000000.0);
  }
  A.rp.push_back((int32_t)A.col.size());
}

static void check(const char* name, const Csr& A) {
  const int64_t n = A.n, nnz = A.rp[n];
  PanelLayout L;
  std::string why;
  CHECK(build_panels(n, A.rp.data(), A.col.data(), A.val.data(), L, why), "%s: %s", name, why.c_str());
  CHECK(L.rows_pp >= 1 && L.rows_pp <= kPanelRowsMax, "%s rows_pp %lld", name, (long long)L.rows_pp);
  CHECK((int64_t)L.npanels * L.rows_pp >= n && (int64_t)(L.npanels - 1) * L.rows_pp < std::max<int64_t>(n, 1),
        "%s panels", name);
  CHECK(L.ptile.size() == (size_t)L.npanels * (kCb + 1), "%s ptile size", name);
  CHECK(L.tiles.size() == 4 * L.toff.size(), "%s tiles", name);
  const int64_t bw = std::max<int64_t>((n + kCb - 1) / kCb, 1);
  // x and the two products
  std::vector<double> x(n), yk(n, 0.0), yr(n, 0.0), ab(n, 0.0);
  uint64_t s = 99;
  for (auto& v : x) v = ((double)(lcg(s) % 2000001) - 1000000.0) / 1000000.0;
  for (int64_t r = 0; r < n; ++r)
    for (int64_t e = A.rp[r]; e < A.rp[r + 1]; ++e) {
      yr[r] += A.val[e] * x[A.col[e]];
      ab[r] += std::fabs(A.val[e] * x[A.col[e]]);
    }
  std::vector<int> seen(nnz, 0);  // layout entries matched to CSR entries
  int64_t next = 0;               // nonzeros are consumed in order, panel after panel
  for (int p = 0; p < L.npanels; ++p) {
    const int64_t r0 = (int64_t)p * L.rows_pp, nrows = std::min(L.rows_pp, n - r0);
    std::vector<double> acc(nrows, 0.0);
    const int32_t* pt = &L.ptile[(size_t)p * (kCb + 1)];
    for (int c = 0; c < kCb; ++c) {
      CHECK(pt[c] <= pt[c + 1], "%s ptile order", name);
      std::vector<int> covered(nrows, 0);
      for (int t = pt[c]; t < pt[c + 1]; ++t) {
        const int32_t tr = L.tiles[4 * t], nr = L.tiles[4 * t + 1], e0 = L.tiles[4 * t + 2], ne = L.tiles[4 * t + 3];
        const int32_t ob = L.toff[t];
        CHECK(e0 == next, "%s tile %d starts at %d, expected %lld", name, t, e0, (long long)next);
        CHECK(tr >= 0 && nr >= 1 && tr + nr <= nrows, "%s tile rows", name);
        for (int r = tr; r < tr + nr; ++r) ++covered[r];
        std::vector<double> prod(std::max(ne, 1));
        if (ob < 0) {
          CHECK(nr == 1 && ne > kTileFill, "%s long tile", name);
        } else {
          CHECK(nr <= kPanelTileRows && ne <= kTileFill, "%s tile size %d %d", name, nr, ne);
          // the kernel's paired loads: pairs from the even index at or below e0
          const int e0a = e0 & ~1, sh = e0 - e0a, nea = ne + sh;
          CHECK(nea <= kTileNnz, "%s pairs", name);
          if (nea > 0) CHECK((int64_t)e0a + 2 * ((nea + 1) / 2) <= nnz + kCsrPad, "%s pair loads past the pad", name);
          CHECK((size_t)ob + nr < L.off.size(), "%s offsets", name);
          CHECK(L.off[ob] == 0 && L.off[ob + nr] == ne, "%s offset ends", name);
        }
        for (int q = 0; q < ne; ++q) prod[q] = L.val[e0 + q] * x[L.col[e0 + q]];
        for (int j = 0; j < nr; ++j) {
          const int r = tr + j;
          const int a = ob < 0 ? 0 : L.off[ob + j], b = ob < 0 ? ne : L.off[ob + j + 1];
          CHECK(a <= b, "%s offsets order", name);
          double sr = 0.0;
          for (int q = a; q < b; ++q) {
            const int64_t e = e0 + q;
            const int32_t cc = L.col[e];
            CHECK(cc / bw == c, "%s column %d outside block %d", name, cc, c);
            // the CSR entry of row r0 + r with this column
            int64_t lo = A.rp[r0 + r], hi = A.rp[r0 + r + 1], f = -1;
            while (lo < hi) {
              const int64_t mid = (lo + hi) / 2;
              if (A.col[mid] < cc) lo = mid + 1;
              else hi = mid;
            }
            if (lo < A.rp[r0 + r + 1] && A.col[lo] == cc) f = lo;
            CHECK(f >= 0 && A.val[f] == L.val[e], "%s entry (%lld, %d) missing", name, (long long)(r0 + r), cc);
            if (f >= 0) ++seen[f];
            sr += prod[q];
          }
          acc[r] += sr;
        }
        next += ne;
      }
      for (int64_t r = 0; r < nrows; ++r) CHECK(covered[r] <= 1, "%s row %lld in two tiles", name, (long long)r);
    }
    for (int64_t r = 0; r < nrows; ++r) yk[r0 + r] = acc[r];
  }
  CHECK(next == nnz, "%s consumed %lld of %lld", name, (long long)next, (long long)nnz);
  for (int64_t e = 0; e < nnz; ++e) CHECK(seen[e] == 1, "%s entry %lld seen %d times", name, (long long)e, seen[e]);
  double worst = 0.0;
  for (int64_t r = 0; r < n; ++r) {
    const double err = std::fabs(yk[r] - yr[r]), bound = 64 * std::ldexp(1.0, -53) * ab[r];
    CHECK(err <= bound, "%s row %lld: %g > %g", name, (long long)r, err, bound);
    if (ab[r] > 0) worst = std::max(worst, err / ab[r]);
  }
  std::printf("%s: n=%lld nnz=%lld panels=%d rows_pp=%lld tiles=%zu long=%d worst=%.2e\n", name, (long long)n,
              (long long)nnz, L.npanels, (long long)L.rows_pp, L.toff.size(),
              (int)std::count(L.toff.begin(), L.toff.end(), -1), worst);
}

int main() {
  setvbuf(stdout, nullptr, _IOLBF, 0);
  uint64_t s = 12345;
  {  // power-law-like rows, some empty, a few long rows packed into one column block
    Csr A;
    A.n = 9001;
    A.rp.push_back(0);
    for (int64_t r = 0; r < A.n; ++r) {
      if (r % 97 == 5) add_row(A, s, 0, 0, A.n);
      else if (r % 1000 == 7) add_row(A, s, 700, 0, A.n / 8);           // > kTileFill in block 0
      else if (r % 1000 == 8) add_row(A, s, 511, A.n / 2, A.n / 2 + 1100);  // 511 in one block
      else if (r % 1000 == 9) add_row(A, s, 510, 3 * A.n / 8 + 1, A.n / 2 - 10);  // exactly kTileFill
      else add_row(A, s, 1 + (int64_t)(lcg(s) % 40) * (lcg(s) % 7 == 0 ? 8 : 1), 0, A.n);
    }
    check("mixed-9001", A);
  }
  {  // fewer columns than blocks
    Csr A;
    A.n = 5;
    A.rp.push_back(0);
    for (int64_t r = 0; r < A.n; ++r) add_row(A, s, 1 + r % 5, 0, A.n);
    check("tiny-5", A);
  }
  {  // one entry
    Csr A;
    A.n = 1;
    A.rp.push_back(0);
    add_row(A, s, 1, 0, 1);
    check("one", A);
  }
  {  // tridiagonal, several panels, a ragged last one
    Csr A;
    A.n = 100003;
    A.rp.push_back(0);
    for (int64_t r = 0; r < A.n; ++r) add_row(A, s, 3, std::max<int64_t>(r - 1, 0), std::min<int64_t>(r + 2, A.n));
    check("tridiag-100003", A);
  }
  {  // a row with more than 65535 nonzeros in one column block (beyond 16-bit offsets)
    Csr A;
    A.n = 600000;
    A.rp.push_back(0);
    for (int64_t r = 0; r < A.n; ++r) add_row(A, s, r == 300000 ? 70000 : 2, 0, r == 300000 ? A.n / 8 : A.n);
    check("longrow-600000", A);
  }
  {  // panels at the largest size: rows_pp = kPanelRowsMax
    Csr A;
    A.n = (int64_t)kSpmvMaxG * kPanelRowsMax + 77;
    A.rp.push_back(0);
    for (int64_t r = 0; r < A.n; ++r) add_row(A, s, 2, 0, A.n);
    check("large-rows_pp", A);
  }
  std::printf("ok: %d failures\n", failures);
  return failures ? 1 : 0;
}
