// Host FP64 small dense linear algebra for the rKS contraction step.
// Algorithms: Householder Hessenberg reduction and Francis double-shift QR
// (Golub & Van Loan, "Matrix Computations", Sec. 7.4-7.5) with the
// Ahues-Tisseur deflation test; 2x2 standardisation; Bai & Demmel direct
// swapping of adjacent diagonal blocks (LAPACK Working Note 54) for the
// reordering step of Algorithm 1; back-substitution eigenvectors of a
// quasi-triangular matrix; Householder QR for whitening (Section 3.3).
//
// The 2x2 standardisation (std2x2) follows the case analysis of LAPACK's
// DLANV2, and the negligible-subdiagonal test in real_schur follows the
// Ahues-Tisseur test as LAPACK's DLAHQR implements it, so that the Schur form
// has LAPACK's standardised blocks.  Those two parts are derived from LAPACK,
// which carries this notice:
//
//   Copyright (c) 1992-2013 The University of Tennessee and The University
//                           of Tennessee Research Foundation.  All rights
//                           reserved.
//   Copyright (c) 2000-2013 The University of California Berkeley.  All
//                           rights reserved.
//   Copyright (c) 2006-2013 The University of Colorado Denver.  All rights
//                           reserved.
//
//   Redistribution and use in source and binary forms, with or without
//   modification, are permitted provided that the following conditions are
//   met:
//   - Redistributions of source code must retain the above copyright notice,
//     this list of conditions and the following disclaimer.
//   - Redistributions in binary form must reproduce the above copyright
//     notice, this list of conditions and the following disclaimer listed in
//     this license in the documentation and/or other materials provided with
//     the distribution.
//   - Neither the name of the copyright holders nor the names of its
//     contributors may be used to endorse or promote products derived from
//     this software without specific prior written permission.
//
//   The copyright holders provide no reassurances that the source code
//   provided does not infringe any patent, copyright, or any other
//   intellectual property rights of third parties.  The copyright holders
//   disclaim any liability to any recipient for claims brought against
//   recipient by any third party for infringement of that parties
//   intellectual property rights.
//
//   THIS SOFTWARE IS PROVIDED BY THE COPYRIGHT HOLDERS AND CONTRIBUTORS
//   "AS IS" AND ANY EXPRESS OR IMPLIED WARRANTIES, INCLUDING, BUT NOT
//   LIMITED TO, THE IMPLIED WARRANTIES OF MERCHANTABILITY AND FITNESS FOR A
//   PARTICULAR PURPOSE ARE DISCLAIMED.  IN NO EVENT SHALL THE COPYRIGHT
//   OWNER OR CONTRIBUTORS BE LIABLE FOR ANY DIRECT, INDIRECT, INCIDENTAL,
//   SPECIAL, EXEMPLARY, OR CONSEQUENTIAL DAMAGES (INCLUDING, BUT NOT LIMITED
//   TO, PROCUREMENT OF SUBSTITUTE GOODS OR SERVICES; LOSS OF USE, DATA, OR
//   PROFITS; OR BUSINESS INTERRUPTION) HOWEVER CAUSED AND ON ANY THEORY OF
//   LIABILITY, WHETHER IN CONTRACT, STRICT LIABILITY, OR TORT (INCLUDING
//   NEGLIGENCE OR OTHERWISE) ARISING IN ANY WAY OUT OF THE USE OF THIS
//   SOFTWARE, EVEN IF ADVISED OF THE POSSIBILITY OF SUCH DAMAGE.
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <limits>

namespace rks {

namespace {

constexpr double kUlp = std::numeric_limits<double>::epsilon();  // 2^-52
constexpr double kSafmin = std::numeric_limits<double>::min();

inline double& at(double* A, int ld, int i, int j) { return A[(size_t)i + (size_t)j * ld]; }
inline double at(const double* A, int ld, int i, int j) { return A[(size_t)i + (size_t)j * ld]; }
inline double sgn(double a, double b) { return b >= 0.0 ? std::fabs(a) : -std::fabs(a); }

// Apply the plane rotation R = [cs -sn; sn cs] as a similarity at rows/cols
// (p, p+1): T <- G^T T G restricted to the affected parts, Z <- Z G.
// Rows p, p+1 are updated over columns [c0, n); columns p, p+1 over rows [0, r1).
void rot_sim(int n, double* T, int ldt, double* Z, int ldz, int p, double cs, double sn,
             int c0, int r1) {
  for (int j = c0; j < n; ++j) {
    double x = at(T, ldt, p, j), y = at(T, ldt, p + 1, j);
    at(T, ldt, p, j) = cs * x + sn * y;
    at(T, ldt, p + 1, j) = -sn * x + cs * y;
  }
  for (int i = 0; i < r1; ++i) {
    double x = at(T, ldt, i, p), y = at(T, ldt, i, p + 1);
    at(T, ldt, i, p) = cs * x + sn * y;
    at(T, ldt, i, p + 1) = -sn * x + cs * y;
  }
  if (Z) {
    for (int i = 0; i < n; ++i) {
      double x = at(Z, ldz, i, p), y = at(Z, ldz, i, p + 1);
      at(Z, ldz, i, p) = cs * x + sn * y;
      at(Z, ldz, i, p + 1) = -sn * x + cs * y;
    }
  }
}

// Householder vector for x (len k): returns beta and v (v[0] = 1) with
// (I - beta v v^T) x = alpha e1.
double house(int k, const double* x, double* v) {
  double sigma = 0.0;
  for (int i = 1; i < k; ++i) sigma += x[i] * x[i];
  v[0] = 1.0;
  for (int i = 1; i < k; ++i) v[i] = x[i];
  if (sigma == 0.0) return 0.0;
  double mu = std::sqrt(x[0] * x[0] + sigma);
  double v0 = (x[0] <= 0.0) ? x[0] - mu : -sigma / (x[0] + mu);
  double beta = 2.0 * v0 * v0 / (sigma + v0 * v0);
  for (int i = 1; i < k; ++i) v[i] /= v0;
  return beta;
}

// Householder reduction to upper Hessenberg form.  Each reflector only spans
// rows k+1 .. (last nonzero row of column k): a matrix that is already
// Hessenberg except for a few rows (the Krylov-Schur contraction's T_k with
// the residual row b^T below it) costs O(k^2 n) instead of O(n^3).
void hessenberg(int n, double* A, int lda, double* Z, int ldz) {
  std::vector<double> v(n), x(n);
  for (int k = 0; k + 2 < n; ++k) {
    int last = n - 1;
    while (last > k + 1 && at(A, lda, last, k) == 0.0) --last;
    if (last <= k + 1) continue;
    int len = last - k;
    for (int i = 0; i < len; ++i) x[i] = at(A, lda, k + 1 + i, k);
    double beta = house(len, x.data(), v.data());
    if (beta == 0.0) continue;
    for (int j = k; j < n; ++j) {  // rows k+1.. : A <- H A
      double s = 0.0;
      for (int i = 0; i < len; ++i) s += v[i] * at(A, lda, k + 1 + i, j);
      s *= beta;
      for (int i = 0; i < len; ++i) at(A, lda, k + 1 + i, j) -= s * v[i];
    }
    // cols k+1.. : A <- A H and Z <- Z H, column-wise so the inner loops are contiguous
    auto right = [&](double* M, int ld) {
      std::fill(x.begin(), x.end(), 0.0);
      for (int j = 0; j < len; ++j) {
        const double* c = &M[(size_t)(k + 1 + j) * ld];
        const double vj = v[j];
        for (int i = 0; i < n; ++i) x[i] += c[i] * vj;
      }
      for (int j = 0; j < len; ++j) {
        double* c = &M[(size_t)(k + 1 + j) * ld];
        const double f = beta * v[j];
        for (int i = 0; i < n; ++i) c[i] -= x[i] * f;
      }
    };
    right(A, lda);
    right(Z, ldz);
    for (int i = k + 2; i < n; ++i) at(A, lda, i, k) = 0.0;
  }
}

// Apply reflector (I - beta v v^T) of length K (2 or 3, the Francis sweep's
// bulge size) from the left to rows r0..r0+K-1, columns [c0, c1), and from
// the right to columns r0.., rows [0, rr) of H and rows [0, n) of Z.  The
// fixed length lets the compiler keep v in registers and vectorise the
// column updates (contiguous rows of a column-major matrix).
template <int K>
void refl_sim(int n, double* H, int ldh, double* Z, int ldz, const double* v, double beta, int r0, int c0, int c1,
              int rr) {
  double vv[K];
  for (int i = 0; i < K; ++i) vv[i] = v[i];
  for (int j = c0; j < c1; ++j) {
    double* col = &H[(size_t)r0 + (size_t)j * ldh];
    double s = 0.0;
    for (int i = 0; i < K; ++i) s += vv[i] * col[i];
    s *= beta;
    for (int i = 0; i < K; ++i) col[i] -= s * vv[i];
  }
  auto right = [&](double* M, int ld, int rows) {
    double* __restrict__ c0 = &M[(size_t)r0 * ld];
    double* __restrict__ c1 = &M[(size_t)(r0 + 1) * ld];
    double* __restrict__ c2 = &M[(size_t)(r0 + (K > 2 ? 2 : 1)) * ld];
    const double b0 = beta * vv[0], b1 = beta * vv[1], b2 = K > 2 ? beta * vv[K - 1] : 0.0;
    if (K == 3) {
      for (int i = 0; i < rows; ++i) {
        const double s = c0[i] * vv[0] + c1[i] * vv[1] + c2[i] * vv[K - 1];
        c0[i] -= s * b0;
        c1[i] -= s * b1;
        c2[i] -= s * b2;
      }
    } else {
      for (int i = 0; i < rows; ++i) {
        const double s = c0[i] * vv[0] + c1[i] * vv[1];
        c0[i] -= s * b0;
        c1[i] -= s * b1;
      }
    }
  };
  right(H, ldh, rr);
  if (Z) right(Z, ldz, n);
}

// Solve T11 X - X T22 = T12 (n1 x n2, each <= 2) by Gaussian elimination
// with complete pivoting on the Kronecker form; tiny pivots are raised to smin.
void sylvester_small(int n1, int n2, const double* T11, int l1, const double* T22, int l2,
                     const double* T12, int l12, double* X, int lx) {
  const int nk = n1 * n2;
  double K[16], rhs[4];
  int colperm[4];
  double kmax = 0.0;
  for (int c = 0; c < nk; ++c) {
    colperm[c] = c;
    int i2 = c % n1, j2 = c / n1;
    for (int r = 0; r < nk; ++r) {
      int i = r % n1, j = r / n1;
      double v = 0.0;
      if (j == j2) v += at(T11, l1, i, i2);
      if (i == i2) v -= at(T22, l2, j2, j);
      K[r + 4 * c] = v;
      kmax = std::max(kmax, std::fabs(v));
    }
  }
  for (int r = 0; r < nk; ++r) rhs[r] = at(T12, l12, r % n1, r / n1);
  const double smin = std::max(kUlp * kmax, kSafmin);
  for (int p = 0; p < nk; ++p) {
    int pr = p, pc = p;
    double best = -1.0;
    for (int c = p; c < nk; ++c)
      for (int r = p; r < nk; ++r)
        if (std::fabs(K[r + 4 * c]) > best) { best = std::fabs(K[r + 4 * c]); pr = r; pc = c; }
    if (pr != p) {
      for (int c = 0; c < nk; ++c) std::swap(K[p + 4 * c], K[pr + 4 * c]);
      std::swap(rhs[p], rhs[pr]);
    }
    if (pc != p) {
      for (int r = 0; r < nk; ++r) std::swap(K[r + 4 * p], K[r + 4 * pc]);
      std::swap(colperm[p], colperm[pc]);
    }
    if (std::fabs(K[p + 4 * p]) < smin) K[p + 4 * p] = K[p + 4 * p] >= 0 ? smin : -smin;
    for (int r = p + 1; r < nk; ++r) {
      double f = K[r + 4 * p] / K[p + 4 * p];
      for (int c = p; c < nk; ++c) K[r + 4 * c] -= f * K[p + 4 * c];
      rhs[r] -= f * rhs[p];
    }
  }
  double sol[4];
  for (int p = nk - 1; p >= 0; --p) {
    double s = rhs[p];
    for (int c = p + 1; c < nk; ++c) s -= K[p + 4 * c] * sol[c];
    sol[p] = s / K[p + 4 * p];
  }
  double out[4];
  for (int p = 0; p < nk; ++p) out[colperm[p]] = sol[p];
  for (int c = 0; c < nk; ++c) at(X, lx, c % n1, c / n1) = out[c];
}

}  // namespace

bool more_wanted(cplx a, cplx b, int which) {
  double ka, kb;
  switch (which) {
    case kLM: ka = std::abs(a); kb = std::abs(b); break;
    case kSM: ka = -std::abs(a); kb = -std::abs(b); break;
    case kLR: ka = a.real(); kb = b.real(); break;
    default: ka = -a.real(); kb = -b.real(); break;
  }
  if (ka != kb) return ka > kb;
  return a.imag() > b.imag();
}

void std2x2(double& a, double& b, double& c, double& d, double& cs, double& sn) {
  const double eps = kUlp;
  if (c == 0.0) {
    cs = 1.0; sn = 0.0;
  } else if (b == 0.0) {
    cs = 0.0; sn = 1.0;
    double t = d; d = a; a = t; b = -c; c = 0.0;
  } else if ((a - d) == 0.0 && (b > 0.0) != (c > 0.0)) {
    cs = 1.0; sn = 0.0;
  } else {
    double temp = a - d;
    double p = 0.5 * temp;
    double bcmax = std::max(std::fabs(b), std::fabs(c));
    double bcmis = std::min(std::fabs(b), std::fabs(c)) * sgn(1.0, b) * sgn(1.0, c);
    double scale = std::max(std::fabs(p), bcmax);
    double z = (p / scale) * p + (bcmax / scale) * bcmis;
    if (z >= 4.0 * eps) {
      // real eigenvalues: triangularise
      z = p + sgn(std::sqrt(scale) * std::sqrt(z), p);
      a = d + z;
      d = d - (bcmax / z) * bcmis;
      double tau = std::hypot(c, z);
      cs = z / tau;
      sn = c / tau;
      b = b - c;
      c = 0.0;
    } else {
      // complex or almost equal real eigenvalues: equalise the diagonal
      double sigma = b + c;
      double tau = std::hypot(sigma, temp);
      cs = std::sqrt(0.5 * (1.0 + std::fabs(sigma) / tau));
      sn = -(p / (tau * cs)) * sgn(1.0, sigma);
      double aa = a * cs + b * sn, bb = -a * sn + b * cs;
      double cc = c * cs + d * sn, dd = -c * sn + d * cs;
      a = aa * cs + cc * sn;
      b = bb * cs + dd * sn;
      c = -aa * sn + cc * cs;
      d = -bb * sn + dd * cs;
      temp = 0.5 * (a + d);
      a = temp;
      d = temp;
      if (c != 0.0) {
        if (b != 0.0) {
          if ((b > 0.0) == (c > 0.0)) {
            // real eigenvalues after all
            double sab = std::sqrt(std::fabs(b)), sac = std::sqrt(std::fabs(c));
            p = sgn(sab * sac, c);
            tau = 1.0 / std::sqrt(std::fabs(b + c));
            a = temp + p;
            d = temp - p;
            b = b - c;
            c = 0.0;
            double cs1 = sab * tau, sn1 = sac * tau;
            temp = cs * cs1 - sn * sn1;
            sn = cs * sn1 + sn * cs1;
            cs = temp;
          }
        } else {
          b = -c;
          c = 0.0;
          temp = cs;
          cs = -sn;
          sn = temp;
        }
      }
    }
  }
}

// Standardise the 2x2 diagonal block at p and propagate the rotation.
static void standardize_block(int n, double* T, int ldt, double* Z, int ldz, int p) {
  double a = at(T, ldt, p, p), b = at(T, ldt, p, p + 1);
  double c = at(T, ldt, p + 1, p), d = at(T, ldt, p + 1, p + 1);
  double cs, sn;
  std2x2(a, b, c, d, cs, sn);
  // rest of rows p, p+1 (columns right of the block) and columns (rows above)
  rot_sim(n, T, ldt, Z, ldz, p, cs, sn, p + 2, p);
  at(T, ldt, p, p) = a; at(T, ldt, p, p + 1) = b;
  at(T, ldt, p + 1, p) = c; at(T, ldt, p + 1, p + 1) = d;
}

int real_schur(int n, double* A, int lda, double* Z, int ldz) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) at(Z, ldz, i, j) = (i == j) ? 1.0 : 0.0;
  if (n == 0) return 0;
  hessenberg(n, A, lda, Z, ldz);
  const double ulp = kUlp;
  const double smlnum = kSafmin * ((double)n / ulp);
  int i = n - 1;
  int its = 0;
  const int itmax = 60;
  while (i >= 0) {
    // look for a negligible subdiagonal entry (Ahues-Tisseur criterion)
    int l = i;
    for (; l > 0; --l) {
      double hll1 = std::fabs(at(A, lda, l, l - 1));
      if (hll1 <= smlnum) break;
      double tst = std::fabs(at(A, lda, l - 1, l - 1)) + std::fabs(at(A, lda, l, l));
      if (tst == 0.0) {
        if (l - 2 >= 0) tst += std::fabs(at(A, lda, l - 1, l - 2));
        if (l + 1 <= i) tst += std::fabs(at(A, lda, l + 1, l));
      }
      if (hll1 <= ulp * tst) {
        double ab = std::max(hll1, std::fabs(at(A, lda, l - 1, l)));
        double ba = std::min(hll1, std::fabs(at(A, lda, l - 1, l)));
        double aa = std::max(std::fabs(at(A, lda, l, l)),
                             std::fabs(at(A, lda, l - 1, l - 1) - at(A, lda, l, l)));
        double bb = std::min(std::fabs(at(A, lda, l, l)),
                             std::fabs(at(A, lda, l - 1, l - 1) - at(A, lda, l, l)));
        double s = aa + ab;
        if (ba * (ab / s) <= std::max(smlnum, ulp * (bb * (aa / s)))) break;
      }
    }
    if (l > 0) at(A, lda, l, l - 1) = 0.0;
    if (l == i) {  // 1x1 block converged
      --i;
      its = 0;
      continue;
    }
    if (l == i - 1) {  // 2x2 block converged: standardise
      standardize_block(n, A, lda, Z, ldz, i - 1);
      i -= 2;
      its = 0;
      continue;
    }
    if (++its > itmax) return i + 1;
    // double shift from the trailing 2x2 (exceptional shifts now and then)
    double s, t;
    if (its % 10 == 0) {
      double sig = std::fabs(at(A, lda, i, i - 1)) + std::fabs(at(A, lda, i - 1, i - 2));
      double re = at(A, lda, i, i) + 0.75 * sig;
      s = 2.0 * re;
      t = re * re + 0.4375 * sig * sig;
    } else {
      double h11 = at(A, lda, i - 1, i - 1), h12 = at(A, lda, i - 1, i);
      double h21 = at(A, lda, i, i - 1), h22 = at(A, lda, i, i);
      s = h11 + h22;
      t = h11 * h22 - h12 * h21;
    }
    double x = at(A, lda, l, l) * at(A, lda, l, l) + at(A, lda, l, l + 1) * at(A, lda, l + 1, l) -
               s * at(A, lda, l, l) + t;
    double y = at(A, lda, l + 1, l) * (at(A, lda, l, l) + at(A, lda, l + 1, l + 1) - s);
    double z = at(A, lda, l + 1, l) * at(A, lda, l + 2, l + 1);
    double v[3], xv[3];
    for (int k = l; k <= i - 2; ++k) {
      xv[0] = x; xv[1] = y; xv[2] = z;
      double beta = house(3, xv, v);
      if (beta != 0.0) {
        int q = std::max(l, k - 1);
        int r = std::min(k + 4, i + 1);
        refl_sim<3>(n, A, lda, Z, ldz, v, beta, k, q, n, r);
        if (k > l) {
          at(A, lda, k + 1, k - 1) = 0.0;
          at(A, lda, k + 2, k - 1) = 0.0;
        }
      }
      x = at(A, lda, k + 1, k);
      y = at(A, lda, k + 2, k);
      if (k < i - 2) z = at(A, lda, k + 3, k);
    }
    xv[0] = x; xv[1] = y;
    double beta = house(2, xv, v);
    if (beta != 0.0) {
      refl_sim<2>(n, A, lda, Z, ldz, v, beta, i - 1, i - 2, n, i + 1);
      at(A, lda, i, i - 2) = 0.0;
    }
  }
  // make sure everything below the first subdiagonal is exactly zero
  for (int j = 0; j < n; ++j)
    for (int r = j + 2; r < n; ++r) at(A, lda, r, j) = 0.0;
  return 0;
}

void blocks(int n, const double* T, int ldt, std::vector<int>& start, std::vector<int>& size) {
  start.clear();
  size.clear();
  int i = 0;
  while (i < n) {
    int s = (i + 1 < n && at(T, ldt, i + 1, i) != 0.0) ? 2 : 1;
    start.push_back(i);
    size.push_back(s);
    i += s;
  }
}

cplx block_eig(const double* T, int ldt, int p, int s) {
  if (s == 1) return cplx(at(T, ldt, p, p), 0.0);
  double a = at(T, ldt, p, p), b = at(T, ldt, p, p + 1);
  double c = at(T, ldt, p + 1, p), d = at(T, ldt, p + 1, p + 1);
  double half = 0.5 * (a + d);
  double dd = 0.5 * (a - d);
  double disc = dd * dd + b * c;
  if (disc >= 0.0) {
    double r = std::sqrt(disc);
    return cplx(half + (half >= 0 ? r : -r), 0.0);
  }
  return cplx(half, std::sqrt(-disc));
}

// T(p:p+ND, p+ND:n) <- Q^T T(p:p+ND, p+ND:n); T(0:p, p:p+ND) <- T(0:p, p:p+ND) Q;
// Z(:, p:p+ND) <- Z(:, p:p+ND) Q  (Q is ND x ND with leading dimension 4).  The
// column updates run over contiguous memory with the ND columns as streams.
template <int ND>
void apply_swap(int n, double* T, int ldt, double* Z, int ldz, int p, const double* Q) {
  for (int j = p + ND; j < n; ++j) {
    double* c = &T[(size_t)p + (size_t)j * ldt];
    double x[ND];
    for (int r = 0; r < ND; ++r) x[r] = c[r];
    for (int r = 0; r < ND; ++r) {
      double s = 0.0;
      for (int q = 0; q < ND; ++q) s += Q[q + 4 * r] * x[q];
      c[r] = s;
    }
  }
  auto cols = [&](double* M, int ld, int rows) {
    double* __restrict__ c[ND];
    for (int j = 0; j < ND; ++j) c[j] = &M[(size_t)(p + j) * ld];
    double q[ND][ND];
    for (int a = 0; a < ND; ++a)
      for (int b = 0; b < ND; ++b) q[a][b] = Q[a + 4 * b];
    for (int i = 0; i < rows; ++i) {
      double x[ND];
      for (int a = 0; a < ND; ++a) x[a] = c[a][i];
      for (int b = 0; b < ND; ++b) {
        double s = 0.0;
        for (int a = 0; a < ND; ++a) s += x[a] * q[a][b];
        c[b][i] = s;
      }
    }
  };
  cols(T, ldt, p);
  cols(Z, ldz, n);
}

int swap_blocks(int n, double* T, int ldt, double* Z, int ldz, int p, int n1, int n2) {
  if (n1 == 1 && n2 == 1) {
    double t11 = at(T, ldt, p, p), t22 = at(T, ldt, p + 1, p + 1), t12 = at(T, ldt, p, p + 1);
    double f = t12, g = t22 - t11;
    double r = std::hypot(f, g);
    if (r == 0.0) return 0;  // equal eigenvalues, nothing to do
    double cs = f / r, sn = g / r;
    rot_sim(n, T, ldt, Z, ldz, p, cs, sn, p, p + 2);
    at(T, ldt, p, p) = t22;
    at(T, ldt, p + 1, p + 1) = t11;
    at(T, ldt, p + 1, p) = 0.0;
    return 0;
  }
  const int nd = n1 + n2;
  double D[16];
  double dnorm = 0.0;
  for (int j = 0; j < nd; ++j)
    for (int r = 0; r < nd; ++r) {
      D[r + 4 * j] = at(T, ldt, p + r, p + j);
      dnorm = std::max(dnorm, std::fabs(D[r + 4 * j]));
    }
  double X[4];
  sylvester_small(n1, n2, D, 4, D + n1 + 4 * n1, 4, D + 4 * n1, 4, X, 2);
  // QR of [-X; I] (nd x n2) -> Q (nd x nd) with Householder reflectors
  double M[16];
  for (int j = 0; j < n2; ++j) {
    for (int r = 0; r < n1; ++r) M[r + 4 * j] = -X[r + 2 * j];
    for (int r = 0; r < n2; ++r) M[n1 + r + 4 * j] = (r == j) ? 1.0 : 0.0;
  }
  double Q[16];
  for (int j = 0; j < nd; ++j)
    for (int r = 0; r < nd; ++r) Q[r + 4 * j] = (r == j) ? 1.0 : 0.0;
  double vs[2][4], betas[2];
  for (int j = 0; j < n2; ++j) {
    int len = nd - j;
    double x[4];
    for (int r = 0; r < len; ++r) x[r] = M[j + r + 4 * j];
    betas[j] = house(len, x, vs[j]);
    for (int c = j; c < n2; ++c) {  // update remaining columns of M
      double s = 0.0;
      for (int r = 0; r < len; ++r) s += vs[j][r] * M[j + r + 4 * c];
      s *= betas[j];
      for (int r = 0; r < len; ++r) M[j + r + 4 * c] -= s * vs[j][r];
    }
  }
  for (int j = n2 - 1; j >= 0; --j) {  // Q = H_0 H_1 ... applied to I
    int len = nd - j;
    for (int c = 0; c < nd; ++c) {
      double s = 0.0;
      for (int r = 0; r < len; ++r) s += vs[j][r] * Q[j + r + 4 * c];
      s *= betas[j];
      for (int r = 0; r < len; ++r) Q[j + r + 4 * c] -= s * vs[j][r];
    }
  }
  // trial: D' = Q^T D Q, test the block that must vanish
  double W[16], Dp[16];
  for (int j = 0; j < nd; ++j)
    for (int r = 0; r < nd; ++r) {
      double s = 0.0;
      for (int c = 0; c < nd; ++c) s += D[r + 4 * c] * Q[c + 4 * j];
      W[r + 4 * j] = s;
    }
  for (int j = 0; j < nd; ++j)
    for (int r = 0; r < nd; ++r) {
      double s = 0.0;
      for (int c = 0; c < nd; ++c) s += Q[c + 4 * r] * W[c + 4 * j];
      Dp[r + 4 * j] = s;
    }
  double low = 0.0;
  for (int j = 0; j < n2; ++j)
    for (int r = n2; r < nd; ++r) low = std::max(low, std::fabs(Dp[r + 4 * j]));
  const double thresh = std::max(20.0 * kUlp * dnorm, kSafmin);
  if (low > thresh) return 1;
  // accept: apply Q to the full T (rows p..p+nd-1 right part, columns above) and Z
  if (nd == 3) apply_swap<3>(n, T, ldt, Z, ldz, p, Q);
  else apply_swap<4>(n, T, ldt, Z, ldz, p, Q);
  for (int j = 0; j < nd; ++j)
    for (int r = 0; r < nd; ++r) at(T, ldt, p + r, p + j) = Dp[r + 4 * j];
  for (int j = 0; j < n2; ++j)
    for (int r = n2; r < nd; ++r) at(T, ldt, p + r, p + j) = 0.0;
  if (n2 == 2) standardize_block(n, T, ldt, Z, ldz, p);
  if (n1 == 2) standardize_block(n, T, ldt, Z, ldz, p + n2);
  if (n2 == 1 && nd == 3) {
    // the 1x1 now on top is exactly separated; nothing else to clean
  }
  return 0;
}

int move_block(int n, double* T, int ldt, double* Z, int ldz, int f, int l) {
  int here = f;
  int nb = (here + 1 < n && at(T, ldt, here + 1, here) != 0.0) ? 2 : 1;
  while (here > l) {
    int na = (here - 2 >= l && at(T, ldt, here - 1, here - 2) != 0.0) ? 2 : 1;
    if (swap_blocks(n, T, ldt, Z, ldz, here - na, na, nb) != 0) return 1;
    here -= na;
    nb = (here + 1 < n && at(T, ldt, here + 1, here) != 0.0) ? 2 : 1;
  }
  return 0;
}

int order_wanted(int n, double* T, int ldt, double* Z, int ldz, int which, int kw, int* p) {
  int pos = 0;
  std::vector<int> st, sz;
  while (pos < kw && pos < n) {
    blocks(n, T, ldt, st, sz);
    int best = -1;
    cplx bl;
    for (size_t b = 0; b < st.size(); ++b) {
      if (st[b] < pos) continue;
      cplx e = block_eig(T, ldt, st[b], sz[b]);
      if (best < 0 || more_wanted(e, bl, which)) { best = st[b]; bl = e; }
    }
    if (best != pos) {
      if (move_block(n, T, ldt, Z, ldz, best, pos) != 0) { *p = pos; return 1; }
    }
    pos += (pos + 1 < n && at(T, ldt, pos + 1, pos) != 0.0) ? 2 : 1;
  }
  *p = pos;
  return 0;
}

void quasi_tri_eig(int n, const double* T, int ldt, cplx* lam, cplx* Y) {
  std::vector<int> st, sz;
  blocks(n, T, ldt, st, sz);
  double tnorm = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= std::min(j + 1, n - 1); ++i) tnorm = std::max(tnorm, std::fabs(at(T, ldt, i, j)));
  const double smin = std::max(kUlp * tnorm, kSafmin);
  std::vector<cplx> y(n);
  int col = 0;
  for (size_t b = 0; b < st.size(); ++b) {
    int p = st[b], s = sz[b];
    int nev = (s == 2 && block_eig(T, ldt, p, 2).imag() != 0.0) ? 2 : s;
    for (int e = 0; e < nev; ++e) {
      std::fill(y.begin(), y.end(), cplx(0.0, 0.0));
      cplx l;
      int top;  // last index of the triangular part solved by back-substitution
      if (s == 1) {
        l = cplx(at(T, ldt, p, p), 0.0);
        y[p] = 1.0;
        top = p;
      } else {
        double a = at(T, ldt, p, p), bb = at(T, ldt, p, p + 1);
        double c = at(T, ldt, p + 1, p), d = at(T, ldt, p + 1, p + 1);
        cplx e0 = block_eig(T, ldt, p, 2);
        if (e0.imag() == 0.0) {
          // a 2x2 block with real eigenvalues (not standardised): both real
          double half = 0.5 * (a + d), dd = 0.5 * (a - d);
          double r = std::sqrt(std::max(dd * dd + bb * c, 0.0));
          l = cplx(e == 0 ? half + r : half - r, 0.0);
        } else {
          l = (e == 0) ? e0 : std::conj(e0);
        }
        cplx v0 = bb, v1 = l - a;
        cplx w0 = l - d, w1 = c;
        if (std::abs(v0) + std::abs(v1) >= std::abs(w0) + std::abs(w1)) {
          y[p] = v0; y[p + 1] = v1;
        } else {
          y[p] = w0; y[p + 1] = w1;
        }
        top = p;
      }
      // back-substitute through the blocks above
      for (int bb2 = (int)b - 1; bb2 >= 0; --bb2) {
        int q = st[bb2], qs = sz[bb2];
        int last = p + s - 1;
        if (qs == 1) {
          cplx r = 0.0;
          for (int j = q + 1; j <= last; ++j) r -= at(T, ldt, q, j) * y[j];
          cplx den = at(T, ldt, q, q) - l;
          if (std::abs(den) < smin) den = smin;
          y[q] = r / den;
        } else {
          cplx r0 = 0.0, r1 = 0.0;
          for (int j = q + 2; j <= last; ++j) {
            r0 -= at(T, ldt, q, j) * y[j];
            r1 -= at(T, ldt, q + 1, j) * y[j];
          }
          cplx m00 = at(T, ldt, q, q) - l, m01 = at(T, ldt, q, q + 1);
          cplx m10 = at(T, ldt, q + 1, q), m11 = at(T, ldt, q + 1, q + 1) - l;
          cplx det = m00 * m11 - m01 * m10;
          if (std::abs(det) < smin * smin) det = smin * smin;
          y[q] = (r0 * m11 - m01 * r1) / det;
          y[q + 1] = (m00 * r1 - m10 * r0) / det;
        }
      }
      (void)top;
      double nrm = 0.0;
      for (int i = 0; i < n; ++i) nrm += std::norm(y[i]);
      nrm = std::sqrt(nrm);
      for (int i = 0; i < n; ++i) Y[(size_t)i + (size_t)col * n] = y[i] / nrm;
      lam[col] = l;
      ++col;
    }
  }
}

void householder_qr(int m, int k, const double* S, int lds, double* Q, int ldq, double* R, int ldr) {
  std::vector<double> A((size_t)m * k), v(m), x(m), betas(k);
  std::vector<std::vector<double>> vs(k);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < m; ++i) A[i + (size_t)j * m] = at(S, lds, i, j);
  for (int j = 0; j < k; ++j) {
    int len = m - j;
    for (int i = 0; i < len; ++i) x[i] = A[j + i + (size_t)j * m];
    vs[j].resize(len);
    betas[j] = house(len, x.data(), vs[j].data());
    for (int c = j; c < k; ++c) {
      double s = 0.0;
      for (int i = 0; i < len; ++i) s += vs[j][i] * A[j + i + (size_t)c * m];
      s *= betas[j];
      for (int i = 0; i < len; ++i) A[j + i + (size_t)c * m] -= s * vs[j][i];
    }
  }
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < k; ++i) at(R, ldr, i, j) = (i <= j) ? A[i + (size_t)j * m] : 0.0;
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < m; ++i) at(Q, ldq, i, j) = (i == j) ? 1.0 : 0.0;
  for (int j = k - 1; j >= 0; --j) {
    int len = m - j;
    for (int c = 0; c < k; ++c) {
      double s = 0.0;
      for (int i = 0; i < len; ++i) s += vs[j][i] * at(Q, ldq, j + i, c);
      s *= betas[j];
      for (int i = 0; i < len; ++i) at(Q, ldq, j + i, c) -= s * vs[j][i];
    }
  }
}

void upper_tri_inverse(int k, const double* R, int ldr, double* Ri, int ldi) {
  for (int j = 0; j < k; ++j) {
    for (int i = k - 1; i >= 0; --i) {
      double s = (i == j) ? 1.0 : 0.0;
      for (int c = i + 1; c < k; ++c) s -= at(R, ldr, i, c) * at(Ri, ldi, c, j);
      at(Ri, ldi, i, j) = (i <= j) ? s / at(R, ldr, i, i) : 0.0;
    }
  }
}

}  // namespace rks
