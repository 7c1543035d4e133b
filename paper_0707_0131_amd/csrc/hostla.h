// Host FP64 dense linear algebra for the small matrices of eigCG.
//
// The eigCG restart (Figure 3.1, eq. (2.3)) needs the lowest nev
// eigenpairs of the m x m window matrix T_m and of its leading (m-1) x (m-1)
// block, a thin QR of the m x 2nev block [Y Ybar] and a full eigensolve of the
// 2nev x 2nev projection H.  init-CG (eq. (2.1)) needs a Cholesky solve with
// the l x l bank matrix H = U^H A U.  All of it runs here in FP64 on the host;
// matrices are column-major std::complex<double> with an explicit leading
// dimension.
#pragma once

#include <complex>

namespace eigcg {
namespace hostla {

using cplx = std::complex<double>;

// Eigenvalues (ascending, all n) and the eigenvectors of the k smallest
// eigenvalues of the Hermitian matrix A (only the upper triangle is read).
// Householder reduction to real tridiagonal form (columns whose part above the
// superdiagonal is already zero cost nothing, so a tridiagonal or
// arrowhead-plus-tridiagonal matrix reduces in O(n + b^3) for a dense block
// of size b), implicit QL for the eigenvalues, inverse iteration for the
// wanted eigenvectors (reorthogonalised inside clusters), then the
// back-transformation.  Returns 0, or -1 if QL fails to converge.
int herm_eig_lowest(int n, const cplx* A, int lda, int k, double* w, cplx* Z, int ldz);

// Thin Householder QR of the m x n (m >= n) matrix A: Q (m x n) with
// orthonormal columns and upper triangular R (n x n, may be null).
void qr_thin(int m, int n, const cplx* A, int lda, cplx* Q, int ldq, cplx* R, int ldr);

// In-place lower Cholesky factor of the Hermitian positive definite A (n x n,
// lower triangle read and written).  Returns 0, or the 1-based index of the
// first non-positive pivot.
int cholesky(int n, cplx* A, int lda);

// Solve (L L^H) X = B in place for the factor from cholesky().
void cholesky_solve(int n, const cplx* L, int ldl, int nrhs, cplx* B, int ldb);

// C (m x n) = A (m x k) * B (k x n), skipping zero entries of A.
void matmul_sparse_a(int m, int n, int k, const cplx* A, int lda, const cplx* B, int ldb,
                     cplx* C, int ldc);

// C (m x n) = A^H (m x k)^H ... i.e. C = A^H B with A (k x m), B (k x n).
void matmul_ah_b(int m, int n, int k, const cplx* A, int lda, const cplx* B, int ldb, cplx* C,
                 int ldc);

}  // namespace hostla
}  // namespace eigcg
