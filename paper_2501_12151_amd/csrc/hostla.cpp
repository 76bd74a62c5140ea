// Host dense linear algebra for assembly-time TT rounding.
#include "hostla.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace tnfem {
namespace hostla {

void gemm(int m, int n, int k, const double* A, const double* B, double* C) {
  for (int i = 0; i < m; ++i) {
    double* c = C + (size_t)i * n;
    std::fill(c, c + n, 0.0);
    for (int p = 0; p < k; ++p) {
      const double a = A[(size_t)i * k + p];
      if (a == 0.0) continue;
      const double* b = B + (size_t)p * n;
      for (int j = 0; j < n; ++j) c[j] += a * b[j];
    }
  }
}

void qr(int m, int n, const double* A, std::vector<double>& Q, std::vector<double>& R) {
  const int c = std::min(m, n);
  // Work column-major for contiguous Householder vectors.
  std::vector<double> W((size_t)m * n);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) W[(size_t)j * m + i] = A[(size_t)i * n + j];
  std::vector<double> tau(c, 0.0), diag(c, 0.0);
  for (int j = 0; j < c; ++j) {
    double* v = &W[(size_t)j * m];
    double s = 0.0;
    for (int i = j; i < m; ++i) s += v[i] * v[i];
    const double nrm = std::sqrt(s);
    if (nrm == 0.0) {
      tau[j] = 0.0;
      diag[j] = 0.0;
      continue;
    }
    const double x0 = v[j];
    const double alpha = x0 >= 0.0 ? -nrm : nrm;
    const double v0 = x0 - alpha;
    v[j] = v0;
    const double vtv = s - x0 * x0 + v0 * v0;
    tau[j] = 2.0 / vtv;
    diag[j] = alpha;
    for (int col = j + 1; col < n; ++col) {
      double* w = &W[(size_t)col * m];
      double d = 0.0;
      for (int i = j; i < m; ++i) d += v[i] * w[i];
      d *= tau[j];
      for (int i = j; i < m; ++i) w[i] -= d * v[i];
    }
  }
  R.assign((size_t)c * n, 0.0);
  for (int i = 0; i < c; ++i) {
    R[(size_t)i * n + i] = diag[i];
    for (int j = i + 1; j < n; ++j) R[(size_t)i * n + j] = W[(size_t)j * m + i];
  }
  // Q = H_0 ... H_{c-1} [I_c; 0], accumulated backwards, column-major work array.
  std::vector<double> Qc((size_t)m * c, 0.0);
  for (int j = 0; j < c; ++j) Qc[(size_t)j * m + j] = 1.0;
  for (int j = c - 1; j >= 0; --j) {
    if (tau[j] == 0.0) continue;
    const double* v = &W[(size_t)j * m];
    for (int col = j; col < c; ++col) {
      double* q = &Qc[(size_t)col * m];
      double d = 0.0;
      for (int i = j; i < m; ++i) d += v[i] * q[i];
      d *= tau[j];
      for (int i = j; i < m; ++i) q[i] -= d * v[i];
    }
  }
  Q.resize((size_t)m * c);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < c; ++j) Q[(size_t)i * c + j] = Qc[(size_t)j * m + i];
}

// One-sided Jacobi SVD of a square n x n matrix G (row-major): G = U diag(S) V^T.  The
// columns are rotated in a column-major copy (each column contiguous in memory).
static void jacobi_square(int n, const std::vector<double>& Grow, std::vector<double>& U, std::vector<double>& S,
                          std::vector<double>& V) {
  std::vector<double> G((size_t)n * n), Vc((size_t)n * n, 0.0);  // column-major
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) G[(size_t)j * n + i] = Grow[(size_t)i * n + j];
  for (int i = 0; i < n; ++i) Vc[(size_t)i * n + i] = 1.0;
  const double eps = 1e-15;
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p) {
      double* gp = &G[(size_t)p * n];
      double* vp = &Vc[(size_t)p * n];
      for (int q = p + 1; q < n; ++q) {
        double* gq = &G[(size_t)q * n];
        double a = 0, b = 0, c = 0;
        for (int i = 0; i < n; ++i) {
          a += gp[i] * gp[i];
          b += gq[i] * gq[i];
          c += gp[i] * gq[i];
        }
        if (c == 0.0 || std::fabs(c) <= eps * std::sqrt(a * b)) continue;
        rotated = true;
        const double zeta = (b - a) / (2.0 * c);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        double* vq = &Vc[(size_t)q * n];
        for (int i = 0; i < n; ++i) {
          const double x = gp[i], y = gq[i];
          gp[i] = cs * x - sn * y;
          gq[i] = sn * x + cs * y;
          const double xv = vp[i], yv = vq[i];
          vp[i] = cs * xv - sn * yv;
          vq[i] = sn * xv + cs * yv;
        }
      }
    }
    if (!rotated) break;
  }
  S.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += G[(size_t)j * n + i] * G[(size_t)j * n + i];
    S[j] = std::sqrt(s);
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return S[x] > S[y]; });
  std::vector<double> S2(n);
  U.assign((size_t)n * n, 0.0);
  V.assign((size_t)n * n, 0.0);
  for (int jj = 0; jj < n; ++jj) {
    const int j = order[jj];
    S2[jj] = S[j];
    for (int i = 0; i < n; ++i) {
      U[(size_t)i * n + jj] = S[j] > 0 ? G[(size_t)j * n + i] / S[j] : (i == jj ? 1.0 : 0.0);
      V[(size_t)i * n + jj] = Vc[(size_t)j * n + i];
    }
  }
  S = S2;
}

void svd(int m, int n, const double* A, std::vector<double>& U, std::vector<double>& S,
         std::vector<double>& Vt) {
  if (m >= n) {
    std::vector<double> Q, R, UR, V;
    qr(m, n, A, Q, R);  // Q m x n, R n x n
    jacobi_square(n, R, UR, S, V);
    U.assign((size_t)m * n, 0.0);
    gemm(m, n, n, Q.data(), UR.data(), U.data());
    Vt.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) Vt[(size_t)i * n + j] = V[(size_t)j * n + i];
  } else {
    // A^T = U' S V'^T  =>  A = V' S U'^T
    std::vector<double> At((size_t)n * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) At[(size_t)j * m + i] = A[(size_t)i * n + j];
    std::vector<double> U2, Vt2;
    svd(n, m, At.data(), U2, S, Vt2);  // U2 n x m, Vt2 m x m
    U.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) U[(size_t)i * m + j] = Vt2[(size_t)j * m + i];
    Vt.assign((size_t)m * n, 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) Vt[(size_t)i * n + j] = U2[(size_t)j * m + i];
  }
}

int trunc_rank(const double* s, int len, double tol, int cap) {
  double tot = 0;
  for (int j = 0; j < len; ++j) tot += s[j] * s[j];
  double tail = 0;
  int r = len;
  for (int j = len - 1; j >= 0; --j) {
    if (tail + s[j] * s[j] <= tol * tol * tot) {
      tail += s[j] * s[j];
      r = j;
    } else {
      break;
    }
  }
  return std::max(1, std::min(r, cap));
}

double tt_norm(std::vector<int> modes, std::vector<int> ranks, std::vector<std::vector<double>> cores) {
  const int K = (int)modes.size();
  for (int k = 0; k + 1 < K; ++k) {
    const int m = ranks[k] * modes[k], nc = ranks[k + 1];
    std::vector<double> Q, R;
    qr(m, nc, cores[k].data(), Q, R);
    const int c = std::min(m, nc);
    const int cols = modes[k + 1] * ranks[k + 2];
    std::vector<double> next((size_t)c * cols);
    gemm(c, cols, nc, R.data(), cores[k + 1].data(), next.data());
    cores[k + 1].swap(next);
    ranks[k + 1] = c;
  }
  double s = 0.0;
  for (double v : cores[K - 1]) s += v * v;
  return std::sqrt(s);
}

}  // namespace hostla
}  // namespace tnfem
