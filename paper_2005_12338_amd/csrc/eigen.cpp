// Host FP64 numerics for the set-up steps of the hot path.
//
// sym_eigen: symmetric eigendecomposition by Householder reduction to
// tridiagonal form followed by the implicit-shift QL iteration on the
// tridiagonal matrix (the textbook two-phase method, e.g. Golub & Van Loan,
// "Matrix Computations", sections 8.3).  The transforms are accumulated in a
// column-major copy so that every update runs over contiguous memory; the
// O(n^2)-per-step updates are spread over OpenMP threads.
//
// gauss_legendre: nodes are the roots of P_n found by Newton's method from
// the Chebyshev-like guess cos(pi (i + 3/4) / (n + 1/2)); weights
// 2 / ((1 - x^2) P_n'(x)^2).
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "kernels.hpp"

void sym_eigen(int64_t n, double* a, double* e_out, double* v_out) {
  std::vector<double> qt((size_t)(n * n), 0.0);   // Q^T, row r = column r of Q
  for (int64_t i = 0; i < n; ++i) qt[i * n + i] = 1.0;
  std::vector<double> vv(n), p(n), w(n), q(n);

  // ---- Householder: A <- H A H, zeroing column k below the sub-diagonal
  for (int64_t k = 0; k + 2 < n; ++k) {
    const int64_t m = n - k - 1;        // length of x = a[k+1.., k]
    double nrm = 0.0;
    for (int64_t i = 0; i < m; ++i) nrm += a[(k + 1 + i) * n + k] * a[(k + 1 + i) * n + k];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const double x0 = a[(k + 1) * n + k];
    const double alpha = x0 > 0 ? -nrm : nrm;
    for (int64_t i = 0; i < m; ++i) vv[i] = a[(k + 1 + i) * n + k];
    vv[0] -= alpha;
    double vn2 = 0.0;
    for (int64_t i = 0; i < m; ++i) vn2 += vv[i] * vv[i];
    if (vn2 == 0.0) continue;
    const double beta = 2.0 / vn2;
    // p = beta * A22 v
#pragma omp parallel for schedule(static) if (m > 256)
    for (int64_t i = 0; i < m; ++i) {
      const double* row = a + (k + 1 + i) * n + (k + 1);
      double s = 0.0;
      for (int64_t j = 0; j < m; ++j) s += row[j] * vv[j];
      p[i] = beta * s;
    }
    double kk = 0.0;
    for (int64_t i = 0; i < m; ++i) kk += vv[i] * p[i];
    kk *= 0.5 * beta;
    for (int64_t i = 0; i < m; ++i) w[i] = p[i] - kk * vv[i];
    // A22 -= v w^T + w v^T
#pragma omp parallel for schedule(static) if (m > 256)
    for (int64_t i = 0; i < m; ++i) {
      double* row = a + (k + 1 + i) * n + (k + 1);
      const double vi = vv[i], wi = w[i];
      for (int64_t j = 0; j < m; ++j) row[j] -= vi * w[j] + wi * vv[j];
    }
    a[(k + 1) * n + k] = alpha;
    a[k * n + k + 1] = alpha;
    for (int64_t i = 1; i < m; ++i) {
      a[(k + 1 + i) * n + k] = 0.0;
      a[k * n + k + 1 + i] = 0.0;
    }
    // Q <- Q H:  rows k+1.. of Q^T change by -beta v (v^T Q^T[k+1..])
    std::fill(q.begin(), q.end(), 0.0);
#pragma omp parallel for schedule(static) if (m > 256)
    for (int64_t r = 0; r < n; ++r) {
      double s = 0.0;
      for (int64_t i = 0; i < m; ++i) s += vv[i] * qt[(k + 1 + i) * n + r];
      q[r] = beta * s;
    }
#pragma omp parallel for schedule(static) if (m > 256)
    for (int64_t i = 0; i < m; ++i) {
      double* row = qt.data() + (k + 1 + i) * n;
      const double vi = vv[i];
      for (int64_t r = 0; r < n; ++r) row[r] -= vi * q[r];
    }
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int64_t i = 0; i < n; ++i) d[i] = a[i * n + i];
  for (int64_t i = 0; i + 1 < n; ++i) e[i] = a[(i + 1) * n + i];

  // ---- implicit QL on (d, e); rotations act on rows i, i+1 of Q^T
  const double tiny = 2.220446049250313e-16;
  for (int64_t l = 0; l < n; ++l) {
    for (int iter = 0; iter < 200; ++iter) {
      int64_t m = l;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= tiny * dd) break;
      }
      if (m == l) break;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      bool early = false;
      for (int64_t i = m - 1; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= pp;
          e[m] = 0.0;
          early = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        double* zi = qt.data() + i * n;
        double* zj = qt.data() + (i + 1) * n;
        for (int64_t k = 0; k < n; ++k) {
          const double fz = zj[k];
          zj[k] = s * zi[k] + c * fz;
          zi[k] = c * zi[k] - s * fz;
        }
      }
      if (early) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }

  // ---- sort ascending
  std::vector<int64_t> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return d[x] < d[y]; });
  for (int64_t c = 0; c < n; ++c) {
    e_out[c] = d[ord[c]];
    const double* src = qt.data() + ord[c] * n;
    for (int64_t r = 0; r < n; ++r) v_out[r * n + c] = src[r];
  }
}

void gauss_legendre(int64_t n, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  for (int64_t i = 0; i < n; ++i) {
    double z = std::cos(pi * ((double)i + 0.75) / ((double)n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      // P_n(z) and P_n'(z) by the three-term recurrence
      double p0 = 1.0, p1 = z;
      for (int64_t k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / (double)k;
        p0 = p1;
        p1 = pk;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = (double)n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        p0 = 1.0; p1 = z;
        for (int64_t k = 2; k <= n; ++k) {
          double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / (double)k;
          p0 = p1;
          p1 = pk;
        }
        if (n == 1) { p1 = z; p0 = 1.0; }
        dp = (double)n * (z * p1 - p0) / (z * z - 1.0);
        break;
      }
    }
    x[n - 1 - i] = z;              // ascending order
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}
