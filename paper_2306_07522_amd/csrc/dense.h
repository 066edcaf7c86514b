// Small dense complex linear algebra on the host, for the projected
// (restart-length sized) matrices of the Krylov solvers.  All matrices are
// column-major: A[i + j * lda] is row i, column j.
#pragma once

#include <complex>
#include <vector>

namespace heom {

using cd = std::complex<double>;

// Eigenvalues w[n] and unit right eigenvectors (columns of vecs, n x n) of a
// general complex n x n matrix A (copied).  Householder reduction to upper
// Hessenberg form, then the implicitly shifted complex QR iteration with
// Wilkinson shifts (Schur form T and Schur vectors Z), then the eigenvectors
// of T by back substitution, mapped back through Z.  Returns false if the QR
// iteration did not converge.
bool eig_general(int n, const std::vector<cd> &A, std::vector<cd> &w, std::vector<cd> &vecs);

// Unitary reduction to upper Hessenberg form by Householder reflections:
// H (n x n, in place) <- Q^H H Q and Z <- Z Q.
void hessenberg_reduce(int n, std::vector<cd> &H, std::vector<cd> &Z);

// Complex Schur form A = Z T Z^H (T upper triangular with the eigenvalues on
// its diagonal, Z unitary): Hessenberg reduction, then the shifted QR
// iteration.  Returns false if the QR iteration did not converge.
bool schur_complex(int n, const std::vector<cd> &A, std::vector<cd> &T, std::vector<cd> &Z);

// Reorder a Schur form (T, Z) in place so that the diagonal entries flagged
// in sel[0..n) come first, in their present order, by unitary swaps of
// neighbouring diagonal entries; Z T Z^H is unchanged and the leading k
// columns of Z then span the invariant subspace of the k flagged eigenvalues.
void schur_reorder(int n, std::vector<cd> &T, std::vector<cd> &Z, const std::vector<char> &sel);

// Solves (H + sigma I) y = rhs for an upper-Hessenberg k x k matrix H
// (column-major, leading dimension ld; entries below the subdiagonal are not
// read) by Gaussian elimination with partial pivoting between neighbouring
// rows, in plain real arithmetic (the projected entries of the Krylov
// solvers are finite and moderate, so the special-case handling of library
// complex products and quotients is not needed); the buffers are kept
// between calls.  Returns false when singular or not finite.
struct HessSolver {
  std::vector<double> ar, ai, br, bi;
  bool solve(const std::vector<cd> &H, int ld, int k, cd sigma, const std::vector<cd> &rhs, std::vector<cd> &y);
};

// Eigen-decomposition of a Hermitian n x n matrix A = U diag(E) U^H by
// cyclic complex Jacobi rotations (orthonormal U also for degenerate
// eigenvalues); E ascending.  Returns false if the sweeps did not converge.
bool eigh_jacobi(int n, const std::vector<cd> &A, std::vector<double> &E, std::vector<cd> &U);

// Solve A x = b (n x n, A copied) by Gaussian elimination with partial
// pivoting; returns false for an exactly singular pivot.
bool lu_solve(int n, const std::vector<cd> &A, std::vector<cd> &x);

// Orthonormalise the columns of P (rows x cols, in place) with two passes of
// classical Gram-Schmidt per column; a column whose remaining norm falls
// below drop_tol times its original norm is removed.  Returns the number of
// columns kept (they are packed to the front).
int orthonormalise_columns(int rows, int cols, std::vector<cd> &P, double drop_tol);

}  // namespace heom
