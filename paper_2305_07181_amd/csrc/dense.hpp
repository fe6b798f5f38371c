// Small dense linear algebra for host-side setup (row-major, double).
#pragma once
#include <cmath>
#include <stdexcept>
#include <vector>

namespace sbp {

template <typename R>
struct MatT {
  int r = 0, c = 0;
  std::vector<R> a;
  MatT() = default;
  MatT(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, R(0)) {}
  R &operator()(int i, int j) { return a[(size_t)i * c + j]; }
  R operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};
using Mat = MatT<double>;

inline Mat matmul(const Mat &A, const Mat &B) {
  if (A.c != B.r) throw std::runtime_error("matmul shape");
  Mat C(A.r, B.c);
  for (int i = 0; i < A.r; ++i)
    for (int k = 0; k < A.c; ++k) {
      double v = A(i, k);
      if (v == 0.0) continue;
      for (int j = 0; j < B.c; ++j) C(i, j) += v * B(k, j);
    }
  return C;
}

inline Mat transpose(const Mat &A) {
  Mat T(A.c, A.r);
  for (int i = 0; i < A.r; ++i)
    for (int j = 0; j < A.c; ++j) T(j, i) = A(i, j);
  return T;
}

// Householder QR of A (m x n, m >= n).  Returns thin Q (m x n) and R (n x n).
template <typename T>
inline void qr_thin(const MatT<T> &A, MatT<T> &Q, MatT<T> &R) {
  const int m = A.r, n = A.c;
  if (m < n) throw std::runtime_error("qr_thin: m < n");
  MatT<T> W = A;                      // reflected in place
  std::vector<std::vector<T>> vs(n);  // Householder vectors
  for (int k = 0; k < n; ++k) {
    T nrm = 0.0;
    for (int i = k; i < m; ++i) nrm += W(i, k) * W(i, k);
    nrm = std::sqrt(nrm);
    std::vector<T> v(m - k, T(0));
    if (nrm == T(0)) { vs[k] = v; continue; }
    T alpha = W(k, k) > 0 ? -nrm : nrm;
    for (int i = k; i < m; ++i) v[i - k] = W(i, k);
    v[0] -= alpha;
    T vn = 0.0;
    for (T x : v) vn += x * x;
    vn = std::sqrt(vn);
    if (vn > 0)
      for (T &x : v) x /= vn;
    for (int j = k; j < n; ++j) {
      T s = 0.0;
      for (int i = k; i < m; ++i) s += v[i - k] * W(i, j);
      for (int i = k; i < m; ++i) W(i, j) -= 2.0 * v[i - k] * s;
    }
    vs[k] = v;
  }
  R = MatT<T>(n, n);
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) R(i, j) = W(i, j);
  // Q = H_0 H_1 ... H_{n-1} applied to the first n columns of I
  Q = MatT<T>(m, n);
  for (int j = 0; j < n; ++j) Q(j, j) = 1.0;
  for (int k = n - 1; k >= 0; --k) {
    const auto &v = vs[k];
    for (int j = 0; j < n; ++j) {
      T s = 0.0;
      for (int i = k; i < m; ++i) s += v[i - k] * Q(i, j);
      for (int i = k; i < m; ++i) Q(i, j) -= 2.0 * v[i - k] * s;
    }
  }
}

// Solve R x = y for upper-triangular R.
template <typename T>
inline std::vector<T> back_subst(const MatT<T> &R, const std::vector<T> &y) {
  const int n = R.r;
  std::vector<T> x(n);
  for (int i = n - 1; i >= 0; --i) {
    T s = y[i];
    for (int j = i + 1; j < n; ++j) s -= R(i, j) * x[j];
    if (R(i, i) == 0.0) throw std::runtime_error("singular R");
    x[i] = s / R(i, i);
  }
  return x;
}

// Least-squares solution of A x = b (A full column rank).
template <typename T>
inline std::vector<T> lstsq(const MatT<T> &A, const std::vector<T> &b) {
  MatT<T> Q, R;
  qr_thin(A, Q, R);
  std::vector<T> y(A.c, T(0));
  for (int j = 0; j < A.c; ++j)
    for (int i = 0; i < A.r; ++i) y[j] += Q(i, j) * b[i];
  return back_subst(R, y);
}

}  // namespace sbp
