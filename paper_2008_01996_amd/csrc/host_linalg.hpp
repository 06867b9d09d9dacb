// Dense FP64 host linear algebra for the once-per-problem setup of the FD
// solver (steps 1a and 1b of Algorithm FD): Cholesky, a nonsymmetric
// eigensolver (Householder-Hessenberg reduction + shifted complex QR with
// eigenvectors from the Schur form) and a one-sided Jacobi SVD.
#pragma once

#include <complex>
#include <string>
#include <vector>

namespace stfd {

using cd = std::complex<double>;

// Row-major n x n dense matrices throughout.

// In-place Cholesky A = L L^T (lower triangle of a holds L on return).
// Returns false if a pivot is not positive and finite.
bool cholesky(int n, std::vector<double>& a);

// Solves L y = b (lower) and L^T x = y in place for a column-major set of
// nrhs right-hand sides stored row-major as b[i*nrhs + r].
void chol_forward(int n, const std::vector<double>& L, double* b, int nrhs);
void chol_backward(int n, const std::vector<double>& L, double* b, int nrhs);
void chol_forward(int n, const std::vector<double>& L, cd* b, int nrhs);
void chol_backward(int n, const std::vector<double>& L, cd* b, int nrhs);

// Eigenvalues and right eigenvectors of a real nonsymmetric matrix a (n x n,
// row-major, destroyed).  Returns false if the QR iteration does not
// converge.  vecs[i*n + k] = component i of eigenvector k (unnormalised).
bool eig_real(int n, std::vector<double>& a, std::vector<cd>& vals, std::vector<cd>& vecs,
              std::string* err);

// Complex Schur form of a real nonsymmetric matrix a (n x n, row-major,
// destroyed): a = Z T Z^H with Z unitary and T upper triangular (row-major,
// the eigenvalues on its diagonal).  Returns false if the QR iteration does
// not converge.
bool schur_real(int n, std::vector<double>& a, std::vector<cd>& t, std::vector<cd>& z, std::string* err);

// Relative eigen residual of the pencil (M, A) (real row-major n x n) for the
// eigenvalues lam and the columns of X (row-major n x n):
// max_k ||(M - lam_k A) x_k||_inf / ((||M||_inf + |lam_k| ||A||_inf) ||x_k||_inf).
double eig_residual(int n, const double* A, const double* M, const std::vector<cd>& lam,
                    const std::vector<cd>& X);

// One-sided Jacobi SVD of a complex n x n matrix: a = U diag(s) V^H.
// a is row-major; U, V row-major; s descending.  v0 (optional, row-major,
// unitary): the sweeps start from the columns of a v0 with v0 as the
// accumulated rotations.
bool svd_jacobi(int n, std::vector<cd>& a, std::vector<cd>& U, std::vector<double>& s,
                std::vector<cd>& V, std::string* err, const std::vector<cd>* v0 = nullptr);

// The same SVD, the Jacobi sweeps started from the right singular vectors of
// a QR-with-column-pivoting preconditioned run (a few sweeps instead of tens
// for a matrix with nearly parallel columns); U keeps the direct method's
// column orthogonality.
bool svd_jacobi_preconditioned(int n, std::vector<cd>& a, std::vector<cd>& U, std::vector<double>& s,
                               std::vector<cd>& V, std::string* err);

// C = A B for row-major real A (m x k), B (k x n), C (m x n); parallel over
// the rows of C, each row summed over k in order.
void matmul_rowmajor(int m, int k, int n, const double* A, const double* B, double* C);

}  // namespace stfd
