// Small dense FP64 linear algebra run on the host once per restart.
//
// The contraction step of randomized Krylov-Schur (Algorithm 1)
// needs, for the m x m Rayleigh quotient (m <= a few hundred):
//   * a real Schur form  B = Q T Q^T  (Proposition "realSchur"): Householder
//     Hessenberg reduction followed by the Francis double-shift QR iteration;
//   * reordering of the diagonal blocks by orthogonal similarity so that the
//     wanted eigenvalues lead (Bai-Demmel direct swapping of adjacent 1x1/2x2
//     blocks, the stable reordering the paper relies on);
//   * eigenpairs of the truncated quasi-triangular factor for the
//     residual estimates of Section 4.1;
//   * a Householder QR of the sketched basis for whitening (Section 3.3).
// All matrices are column-major with an explicit leading dimension.
#pragma once
#include <complex>
#include <vector>

namespace rks {

using cplx = std::complex<double>;

enum Which { kLM = 0, kSM = 1, kLR = 2, kSR = 3 };

// Sort key: a is more wanted than b.
bool more_wanted(cplx a, cplx b, int which);

// Reduce A (n x n, lda) to real Schur form in place; Z (n x n, ldz) is
// overwritten with the orthogonal Schur vectors (A_in = Z T Z^T).
// Returns 0 on success, >0 if the QR iteration failed to converge.
int real_schur(int n, double* A, int lda, double* Z, int ldz);

// Standardise the 2x2 block [[a,b],[c,d]] (LAPACK-style: real eigenvalues ->
// upper triangular; complex -> equal diagonal with b*c < 0).  Returns the
// rotation (cs, sn) with [a b; c d]_new = R^T [a b; c d] R, R = [cs -sn; sn cs].
void std2x2(double& a, double& b, double& c, double& d, double& cs, double& sn);

// Diagonal block structure of a quasi-triangular T: block starts and sizes.
void blocks(int n, const double* T, int ldt, std::vector<int>& start, std::vector<int>& size);

// Eigenvalue of the block at position p (size s); for a 2x2 block the member
// with non-negative imaginary part.
cplx block_eig(const double* T, int ldt, int p, int s);

// Swap the adjacent diagonal blocks at p (size n1) and p+n1 (size n2) of the
// quasi-triangular T (n x n), updating Z.  Returns 0, or 1 if the swap was
// rejected as numerically unsafe (T and Z then unchanged).
int swap_blocks(int n, double* T, int ldt, double* Z, int ldz, int p, int n1, int n2);

// Move the block starting at f up to position l < f by adjacent swaps.
// Returns 0 on success.
int move_block(int n, double* T, int ldt, double* Z, int ldz, int f, int l);

// Bring the kw most wanted eigenvalues to the leading positions, one block at
// a time in priority order.  *p receives kw, or kw+1 when a conjugate pair
// straddles the boundary.  Returns 0 on success.
int order_wanted(int n, double* T, int ldt, double* Z, int ldz, int which, int kw, int* p);

// Eigenpairs of the quasi-triangular T (n x n): lam[n], Y (n x n complex,
// column i = unit 2-norm eigenvector of lam[i]).
void quasi_tri_eig(int n, const double* T, int ldt, cplx* lam, cplx* Y);

// Eigenvalues of a general small matrix in Hessenberg/quasi-triangular form
// after whitening (blocks need not be standardised).
// Householder QR of S (m x k, lds): Q (m x k, ldq) explicit, R (k x k, ldr).
void householder_qr(int m, int k, const double* S, int lds, double* Q, int ldq, double* R, int ldr);

// Inverse of an upper-triangular k x k matrix.
void upper_tri_inverse(int k, const double* R, int ldr, double* Rinv, int ldi);

}  // namespace rks
