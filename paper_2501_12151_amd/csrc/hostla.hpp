// Small dense linear algebra on the host (FP64, row-major), used to build the
// load TT during assembly.  The sweep itself never calls these.
#pragma once

#include <vector>

namespace tnfem {
namespace hostla {

// Thin Householder QR of the m x n matrix A: Q (m x c), R (c x n), c = min(m, n).
void qr(int m, int n, const double* A, std::vector<double>& Q, std::vector<double>& R);

// Thin SVD of the m x n matrix A: U (m x c), S (c, descending), Vt (c x n).
// Householder QR, then one-sided Jacobi on the square factor.
void svd(int m, int n, const double* A, std::vector<double>& U, std::vector<double>& S,
         std::vector<double>& Vt);

// C (m x n) = A (m x k) * B (k x n), all row-major.
void gemm(int m, int n, int k, const double* A, const double* B, double* C);

// Rank kept by truncation: smallest r with sum_{j>=r} s_j^2 <= tol^2 sum s^2, in [1, cap].
int trunc_rank(const double* s, int len, double tol, int cap);

// Frobenius norm of a TT (cores row-major [r_k][n_k][r_{k+1}]): QR of each unfolding, R carried
// into the next core.
double tt_norm(std::vector<int> modes, std::vector<int> ranks, std::vector<std::vector<double>> cores);

}  // namespace hostla
}  // namespace tnfem
