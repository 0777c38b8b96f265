// Host check of the small dense FP64 routines, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitize.py (no GPU involved).
// Runs the contraction's dense steps on random and structured matrices of the
// sizes the solver meets (up to 121 x 120 Rayleigh quotients, 480 x 120
// sketches) and checks their defining identities; any out-of-bounds access or
// undefined operation aborts the run through the sanitizers.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "dense.h"

namespace {

int failures = 0;

void expect(bool ok, const char* what, int n, double v) {
  if (!ok) {
    std::printf("FAIL %s n=%d value=%.3e\n", what, n, v);
    ++failures;
  }
}

double frob(const std::vector<double>& a) {
  double s = 0.0;
  for (double v : a) s += v * v;
  return std::sqrt(s);
}

// || Z T Z^T - A ||_F / ||A||_F and || Z^T Z - I ||_F
void schur_errors(int n, const std::vector<double>& A, const std::vector<double>& T, const std::vector<double>& Z,
                  double* rel, double* orth) {
  std::vector<double> ZT((size_t)n * n, 0.0), R((size_t)n * n, 0.0), G((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int l = 0; l < n; ++l) {
      const double t = T[l + (size_t)j * n];
      if (t == 0.0) continue;
      for (int i = 0; i < n; ++i) ZT[i + (size_t)j * n] += Z[i + (size_t)l * n] * t;
    }
  for (int j = 0; j < n; ++j)
    for (int l = 0; l < n; ++l) {
      const double z = Z[j + (size_t)l * n];
      for (int i = 0; i < n; ++i) R[i + (size_t)j * n] += ZT[i + (size_t)l * n] * z;
    }
  for (size_t i = 0; i < R.size(); ++i) R[i] -= A[i];
  *rel = frob(R) / frob(A);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int l = 0; l < n; ++l) s += Z[l + (size_t)i * n] * Z[l + (size_t)j * n];
      G[i + (size_t)j * n] = s - (i == j ? 1.0 : 0.0);
    }
  *orth = frob(G);
}

bool quasi_triangular(int n, const std::vector<double>& T) {
  for (int j = 0; j < n; ++j)
    for (int i = j + 2; i < n; ++i)
      if (T[i + (size_t)j * n] != 0.0) return false;
  for (int j = 0; j + 2 < n; ++j)  // no two consecutive subdiagonal entries
    if (T[(j + 1) + (size_t)j * n] != 0.0 && T[(j + 2) + (size_t)(j + 1) * n] != 0.0) return false;
  return true;
}

void check_matrix(int n, const std::vector<double>& A, int which, int kw) {
  std::vector<double> T = A, Z((size_t)n * n);
  const int rc = rks::real_schur(n, T.data(), n, Z.data(), n);
  expect(rc == 0, "real_schur converged", n, rc);
  double rel, orth;
  schur_errors(n, A, T, Z, &rel, &orth);
  expect(rel < 1e-12, "Schur backward error", n, rel);
  expect(orth < 1e-12, "Schur vectors orthonormal", n, orth);
  expect(quasi_triangular(n, T), "quasi-triangular", n, 0.0);
  int p = 0;
  const int ro = rks::order_wanted(n, T.data(), n, Z.data(), n, which, kw, &p);
  expect(ro == 0 && (p == kw || p == kw + 1), "order_wanted", n, p);
  schur_errors(n, A, T, Z, &rel, &orth);
  expect(rel < 1e-11, "reordered backward error", n, rel);
  expect(orth < 1e-11, "reordered vectors orthonormal", n, orth);
  expect(quasi_triangular(n, T), "reordered quasi-triangular", n, 0.0);
  // the leading p eigenvalues are the most wanted ones
  std::vector<rks::cplx> lam(n);
  std::vector<rks::cplx> Y((size_t)n * n);
  rks::quasi_tri_eig(n, T.data(), n, lam.data(), Y.data());
  for (int i = 0; i < p; ++i)
    for (int j = p; j < n; ++j)
      expect(!rks::more_wanted(lam[j], lam[i], which) || std::abs(lam[j] - lam[i]) < 1e-9 * std::abs(lam[i]),
             "wanted set leads", n, std::abs(lam[j]));
  // eigenvectors of the quasi-triangular factor: || T y - lam y || small
  for (int i = 0; i < n; ++i) {
    double r2 = 0.0;
    for (int a = 0; a < n; ++a) {
      rks::cplx s = 0.0;
      for (int b = 0; b < n; ++b) s += T[a + (size_t)b * n] * Y[b + (size_t)i * n];
      s -= lam[i] * Y[a + (size_t)i * n];
      r2 += std::norm(s);
    }
    expect(std::sqrt(r2) < 1e-9 * (1.0 + std::abs(lam[i])) * n, "quasi-triangular eigenvector", n, std::sqrt(r2));
  }
}

}  // namespace

int main() {
  std::mt19937_64 gen(12345);
  std::normal_distribution<double> nd(0.0, 1.0);
  const int sizes[] = {1, 2, 3, 7, 24, 60, 90, 120};
  for (int n : sizes) {
    for (int which = 0; which < 4; ++which) {
      std::vector<double> A((size_t)n * n);
      for (double& v : A) v = nd(gen);
      check_matrix(n, A, which, n > 4 ? n / 3 : 1);
      // Hessenberg-plus-row shape of a contraction (upper Hessenberg)
      for (int j = 0; j < n; ++j)
        for (int i = j + 2; i < n; ++i) A[i + (size_t)j * n] = 0.0;
      check_matrix(n, A, which, n > 4 ? n / 4 : 1);
    }
  }
  // a matrix with many equal eigenvalues (diagonal, repeated values)
  {
    const int n = 30;
    std::vector<double> A((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) A[i + (size_t)i * n] = (double)(i % 4);
    check_matrix(n, A, 0, 10);
  }
  // Householder QR and the triangular inverse of a tall sketch (whitening)
  for (int k : {1, 5, 45, 120}) {
    const int m = 4 * k;
    std::vector<double> S((size_t)m * k), Q((size_t)m * k), R((size_t)k * k), Ri((size_t)k * k);
    for (double& v : S) v = nd(gen);
    rks::householder_qr(m, k, S.data(), m, Q.data(), m, R.data(), k);
    rks::upper_tri_inverse(k, R.data(), k, Ri.data(), k);
    double e = 0.0, o = 0.0, iv = 0.0;
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < m; ++i) {
        double s = 0.0;
        for (int l = 0; l <= j; ++l) s += Q[i + (size_t)l * m] * R[l + (size_t)j * k];
        e += (s - S[i + (size_t)j * m]) * (s - S[i + (size_t)j * m]);
      }
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < k; ++i) {
        double s = 0.0, t = 0.0;
        for (int l = 0; l < m; ++l) s += Q[l + (size_t)i * m] * Q[l + (size_t)j * m];
        for (int l = 0; l < k; ++l) t += R[i + (size_t)l * k] * Ri[l + (size_t)j * k];
        o += (s - (i == j)) * (s - (i == j));
        iv += (t - (i == j)) * (t - (i == j));
      }
    expect(std::sqrt(e) < 1e-12 * std::sqrt((double)m * k), "QR reproduces S", k, std::sqrt(e));
    expect(std::sqrt(o) < 1e-12 * k, "Q orthonormal", k, std::sqrt(o));
    expect(std::sqrt(iv) < 1e-9 * k, "R R^-1 = I", k, std::sqrt(iv));
  }
  std::printf("%s: %d failures\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
