// Small dense FP64 linear algebra on the host for the per-right-hand-side and
// per-wavelength set-up of Algorithm 1 (Sec. 3.1): the harmonic-Ritz
// generalised eigenproblem (step 2), the thin QR of step 4, the multi-shift
// least-squares problems of step 1 and the k x k Cholesky factorisations of
// the per-wavelength Gram matrices (Sec. 3.2).  Sizes are at most ~130, so
// plain O(n^3) loops are used.  Column-major storage throughout.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

namespace hydot {
namespace dense {

using zc = std::complex<double>;

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix A (column-major,
// overwritten).  Returns eigenvalues in w and eigenvectors as columns of Q.
inline void sym_eig(int n, std::vector<double>& A, std::vector<double>& w, std::vector<double>& Q) {
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[i + (size_t)n * i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[i + (size_t)n * j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        tot += a(i, j) * a(i, j);
        if (i != j) off += a(i, j) * a(i, j);
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {   // A <- A J (columns p, q)
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - s * akq;
          a(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // A <- J^T A (rows p, q)
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - s * aqk;
          a(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double qkp = Q[k + (size_t)n * p], qkq = Q[k + (size_t)n * q];
          Q[k + (size_t)n * p] = c * qkp - s * qkq;
          Q[k + (size_t)n * q] = s * qkp + c * qkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = a(i, i);
}

// Real Cholesky A = L L^T (lower, column-major). Returns false if not SPD.
inline bool chol_real(int n, const std::vector<double>& A, std::vector<double>& L) {
  L.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[j + (size_t)n * j];
    for (int k = 0; k < j; ++k) d -= L[j + (size_t)n * k] * L[j + (size_t)n * k];
    if (!(d > 0.0)) return false;
    const double ljj = std::sqrt(d);
    L[j + (size_t)n * j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double s = A[i + (size_t)n * j];
      for (int k = 0; k < j; ++k) s -= L[i + (size_t)n * k] * L[j + (size_t)n * k];
      L[i + (size_t)n * j] = s / ljj;
    }
  }
  return true;
}

// Complex Hermitian Cholesky G = L L^H (lower). Returns false if not positive definite.
inline bool chol_herm(int n, const std::vector<zc>& G, std::vector<zc>& L) {
  L.assign((size_t)n * n, zc(0.0, 0.0));
  for (int j = 0; j < n; ++j) {
    double d = G[j + (size_t)n * j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(L[j + (size_t)n * k]);
    if (!(d > 0.0)) return false;
    const double ljj = std::sqrt(d);
    L[j + (size_t)n * j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      zc s = G[i + (size_t)n * j];
      for (int k = 0; k < j; ++k) s -= L[i + (size_t)n * k] * std::conj(L[j + (size_t)n * k]);
      L[i + (size_t)n * j] = s / ljj;
    }
  }
  return true;
}

// Thin QR of an m x k matrix P (column-major) by Householder reflections:
// P = Q R with Q m x k orthonormal columns and R k x k upper triangular.
inline void thin_qr(int m, int k, const std::vector<double>& P, std::vector<double>& Q,
                    std::vector<double>& R) {
  std::vector<double> A(P);
  std::vector<std::vector<double>> vs;
  std::vector<double> taus;
  for (int j = 0; j < k; ++j) {
    double nrm = 0.0;
    for (int i = j; i < m; ++i) nrm += A[i + (size_t)m * j] * A[i + (size_t)m * j];
    nrm = std::sqrt(nrm);
    std::vector<double> v(m, 0.0);
    const double a0 = A[j + (size_t)m * j];
    const double alpha = (a0 >= 0 ? -nrm : nrm);
    for (int i = j; i < m; ++i) v[i] = A[i + (size_t)m * j];
    v[j] -= alpha;
    double vn = 0.0;
    for (int i = j; i < m; ++i) vn += v[i] * v[i];
    double tau = vn > 0 ? 2.0 / vn : 0.0;
    for (int c = j; c < k; ++c) {
      double s = 0.0;
      for (int i = j; i < m; ++i) s += v[i] * A[i + (size_t)m * c];
      s *= tau;
      for (int i = j; i < m; ++i) A[i + (size_t)m * c] -= s * v[i];
    }
    vs.push_back(v);
    taus.push_back(tau);
  }
  R.assign((size_t)k * k, 0.0);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i <= j; ++i) R[i + (size_t)k * j] = A[i + (size_t)m * j];
  // Q = H_0 H_1 ... H_{k-1} [I; 0]
  Q.assign((size_t)m * k, 0.0);
  for (int j = 0; j < k; ++j) Q[j + (size_t)m * j] = 1.0;
  for (int h = k - 1; h >= 0; --h) {
    const std::vector<double>& v = vs[h];
    for (int c = 0; c < k; ++c) {
      double s = 0.0;
      for (int i = h; i < m; ++i) s += v[i] * Q[i + (size_t)m * c];
      s *= taus[h];
      for (int i = h; i < m; ++i) Q[i + (size_t)m * c] -= s * v[i];
    }
  }
  // make diag(R) positive
  for (int j = 0; j < k; ++j)
    if (R[j + (size_t)k * j] < 0) {
      for (int c = j; c < k; ++c) R[j + (size_t)k * c] = -R[j + (size_t)k * c];
      for (int i = 0; i < m; ++i) Q[i + (size_t)m * j] = -Q[i + (size_t)m * j];
    }
}

// Harmonic Ritz pairs of an Arnoldi/Lanczos factorisation K V_n = V_{n+1} Hbar
// (Alg. 1 step 2): Hbar^T Hbar z = theta H_n^T z, with H_n symmetric positive
// definite (Lanczos on an SPD matrix).  Keeps the k pairs of smallest |theta|
// (ties broken by index) and returns Z_k (n x k, column-major).
// Hbar is (n+1) x n column-major.  Returns false if H_n is not SPD.
inline bool harmonic_ritz(int n, int k, const std::vector<double>& Hbar, std::vector<double>& Zk,
                          std::vector<double>& theta_k) {
  const int ld = n + 1;
  std::vector<double> B((size_t)n * n), A((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i)
      B[i + (size_t)n * j] = 0.5 * (Hbar[i + (size_t)ld * j] + Hbar[j + (size_t)ld * i]);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int r = 0; r < n + 1; ++r) s += Hbar[r + (size_t)ld * i] * Hbar[r + (size_t)ld * j];
      A[i + (size_t)n * j] = s;
    }
  std::vector<double> L;
  if (!chol_real(n, B, L)) return false;
  // M = L^-1 A L^-T
  std::vector<double> T(A);
  for (int c = 0; c < n; ++c)  // T = L^-1 A (columns)
    for (int i = 0; i < n; ++i) {
      double s = T[i + (size_t)n * c];
      for (int q = 0; q < i; ++q) s -= L[i + (size_t)n * q] * T[q + (size_t)n * c];
      T[i + (size_t)n * c] = s / L[i + (size_t)n * i];
    }
  std::vector<double> M((size_t)n * n);
  for (int r = 0; r < n; ++r)  // M^T = L^-1 T^T  -> solve on rows of T
    for (int i = 0; i < n; ++i) {
      double s = T[r + (size_t)n * i];
      for (int q = 0; q < i; ++q) s -= L[i + (size_t)n * q] * M[r + (size_t)n * q];
      M[r + (size_t)n * i] = s / L[i + (size_t)n * i];
    }
  for (int j = 0; j < n; ++j)  // symmetrise rounding
    for (int i = j + 1; i < n; ++i) {
      const double a = 0.5 * (M[i + (size_t)n * j] + M[j + (size_t)n * i]);
      M[i + (size_t)n * j] = a;
      M[j + (size_t)n * i] = a;
    }
  std::vector<double> w, Q;
  sym_eig(n, M, w, Q);
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return std::fabs(w[a]) < std::fabs(w[b]); });
  Zk.assign((size_t)n * k, 0.0);
  theta_k.assign(k, 0.0);
  for (int c = 0; c < k; ++c) {
    const int e = idx[c];
    theta_k[c] = w[e];
    // z = L^-T q
    for (int i = n - 1; i >= 0; --i) {
      double s = Q[i + (size_t)n * e];
      for (int q = i + 1; q < n; ++q) s -= L[q + (size_t)n * i] * Zk[q + (size_t)n * c];
      Zk[i + (size_t)n * c] = s / L[i + (size_t)n * i];
    }
  }
  return true;
}

// min_y || beta e1 - (Hbar + sigma [I; 0]) y ||_2 for an (n+1) x n real Hessenberg
// Hbar and complex shift sigma, by complex Givens rotations (Alg. 1 step 1).
inline void shifted_ls(int n, const std::vector<double>& Hbar, zc sigma, double beta, std::vector<zc>& y) {
  const int ld = n + 1;
  std::vector<zc> H((size_t)ld * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < ld; ++i) H[i + (size_t)ld * j] = Hbar[i + (size_t)ld * j];
  for (int j = 0; j < n; ++j) H[j + (size_t)ld * j] += sigma;
  std::vector<zc> g(ld, zc(0, 0));
  g[0] = beta;
  for (int j = 0; j < n; ++j) {
    // eliminate below-diagonal entries of column j (Hessenberg: only row j+1)
    const zc a = H[j + (size_t)ld * j], b = H[j + 1 + (size_t)ld * j];
    const double r = std::sqrt(std::norm(a) + std::norm(b));
    zc c, s;  // [c s; -conj(s) conj(c)] unitary with c real
    if (std::abs(a) == 0.0) {
      c = 0.0;
      s = std::conj(b) / std::abs(b);
    } else {
      c = std::abs(a) / r;
      s = (a / std::abs(a)) * std::conj(b) / r;
    }
    for (int col = j; col < n; ++col) {
      const zc h1 = H[j + (size_t)ld * col], h2 = H[j + 1 + (size_t)ld * col];
      H[j + (size_t)ld * col] = c * h1 + s * h2;
      H[j + 1 + (size_t)ld * col] = -std::conj(s) * h1 + c * h2;
    }
    const zc g1 = g[j], g2 = g[j + 1];
    g[j] = c * g1 + s * g2;
    g[j + 1] = -std::conj(s) * g1 + c * g2;
  }
  y.assign(n, zc(0, 0));
  for (int i = n - 1; i >= 0; --i) {
    zc s = g[i];
    for (int q = i + 1; q < n; ++q) s -= H[i + (size_t)ld * q] * y[q];
    y[i] = s / H[i + (size_t)ld * i];
  }
}

}  // namespace dense
}  // namespace hydot
