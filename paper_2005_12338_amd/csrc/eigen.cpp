// Host FP64 numerics for the set-up steps of the hot path.
//
// sym_eigen: symmetric eigendecomposition by Householder reduction to
// tridiagonal form followed by the implicit-shift QL iteration on the
// tridiagonal matrix (the textbook two-phase method, e.g. Golub & Van Loan,
// "Matrix Computations", sections 8.3).  The transforms are accumulated in a
// transposed copy Q^T so that every update runs over contiguous memory; the
// O(n^2)-per-step updates are spread over OpenMP threads.  The QL iteration
// on the tridiagonal matrix does not depend on the vectors, so its plane
// rotations are recorded and applied to Q^T afterwards, one block of
// columns per thread through all sweeps: the same arithmetic in the same
// order per element as applying each sweep as it is found.
//
// gauss_legendre: nodes are the roots of P_n found by Newton's method from
// the Chebyshev-like guess cos(pi (i + 3/4) / (n + 1/2)); weights
// 2 / ((1 - x^2) P_n'(x)^2).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include <omp.h>

#include "host_numerics.hpp"

namespace {
constexpr int64_t kColBlock = 32;

// Threads of the O(n^2)-per-step Householder updates.
int nthreads() { return std::max(1, std::min(16, omp_get_max_threads())); }

// x . y with four interleaved partial sums (vectorises without reassociation
// flags; a fixed summation order either way).
inline double dot4(const double* x, const double* y, int64_t m) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t j = 0;
  for (; j + 4 <= m; j += 4) {
    s0 += x[j] * y[j];
    s1 += x[j + 1] * y[j + 1];
    s2 += x[j + 2] * y[j + 2];
    s3 += x[j + 3] * y[j + 3];
  }
  for (; j < m; ++j) s0 += x[j] * y[j];
  return (s0 + s1) + (s2 + s3);
}

// sqrt(x^2 + y^2); the library hypot (which rescales, and is several times
// slower) only where the plain sum of squares could over- or underflow.
inline double hyp(double x, double y) {
  const double s = x * x + y * y;
  if (s > 1e-290 && s < 1e290) return std::sqrt(s);
  return std::hypot(x, y);
}

// The plane rotations of the QL iteration, recorded sweep by sweep: sweep w
// acts on rows lo[w] .. hi[w] with (c, s) of rotation i = hi-1 .. lo at
// cs[2 (off[w] + hi-1-i)], cs[2 (off[w] + hi-1-i) + 1].
struct Sweeps {
  std::vector<int64_t> lo, hi, off;
  std::vector<double> cs;
};

// All sweeps on the columns k0 .. k0+kn-1 of Q^T.  The block is first
// copied to a contiguous buffer (row stride kn), so consecutive rotations
// walk consecutive memory; KN > 0 fixes kn at compile time.
template <int KN>
void apply_block(double* qt, int64_t n, int64_t k0, int64_t kn_rt, const Sweeps& sw, double* buf) {
  const int64_t kn = KN > 0 ? KN : kn_rt;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = 0; k < kn; ++k) buf[i * kn + k] = qt[i * n + k0 + k];
  double carry[KN > 0 ? KN : kColBlock];
  const int64_t nsw = (int64_t)sw.lo.size();
  for (int64_t w = 0; w < nsw; ++w) {
    const int64_t lo = sw.lo[w], hi = sw.hi[w];
    const double* r = sw.cs.data() + 2 * sw.off[w];
    const double* top = buf + hi * kn;
    for (int64_t k = 0; k < kn; ++k) carry[k] = top[k];
    for (int64_t i = hi - 1; i >= lo; --i, r += 2) {
      const double c = r[0], s = r[1];
      double* zi = buf + i * kn;
      double* zj = zi + kn;
      for (int64_t k = 0; k < kn; ++k) {
        const double fz = carry[k], xi = zi[k];
        zj[k] = s * xi + c * fz;
        carry[k] = c * xi - s * fz;
      }
    }
    double* bot = buf + lo * kn;
    for (int64_t k = 0; k < kn; ++k) bot[k] = carry[k];
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = 0; k < kn; ++k) qt[i * n + k0 + k] = buf[i * kn + k];
}

// Apply every recorded sweep, in order, to the rows of Q^T.  Rotations mix
// rows only, so each block of columns is independent: one thread per block
// runs all sweeps on its block (which stays in cache), with a single
// fork/join for the whole iteration.  Within a sweep, rotation i leaves row
// i+1 final and row i as the input of rotation i-1, so the running row stays
// in registers and every element is read and written once per sweep.
void apply_sweeps(double* qt, int64_t n, const Sweeps& sw) {
  const int64_t nb = (n + kColBlock - 1) / kColBlock;
  const int64_t nsw = (int64_t)sw.lo.size();
  std::vector<double> buf((size_t)(nb * kColBlock * n));
#pragma omp parallel for num_threads(nthreads()) schedule(dynamic, 1) if (nsw * n > 65536)
  for (int64_t bk = 0; bk < nb; ++bk) {
    const int64_t k0 = bk * kColBlock, k1 = std::min(n, k0 + kColBlock), kn = k1 - k0;
    double* b = buf.data() + bk * kColBlock * n;
    if (kn == kColBlock)
      apply_block<kColBlock>(qt, n, k0, kColBlock, sw, b);
    else
      apply_block<0>(qt, n, k0, kn, sw, b);
  }
}
}  // namespace

void sym_eigen(int64_t n, double* a, double* e_out, double* v_out) {
  // reflector k: v_k (length n-k-1, stored in row k of refl) and beta_k;
  // H_k = I - beta_k v_k v_k^T acts on indices k+1..n-1.
  std::vector<double> refl((size_t)(n * n), 0.0), betas(n, 0.0);
  std::vector<double> p(n), w(n);

  // ---- Householder: A <- H A H, zeroing column k below the sub-diagonal
  for (int64_t k = 0; k + 2 < n; ++k) {
    const int64_t m = n - k - 1;        // length of x = a[k+1.., k]
    double* vv = refl.data() + k * n;
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
    betas[k] = beta;
    // p = beta * A22 v
#pragma omp parallel for num_threads(nthreads()) schedule(static) if (m > 256)
    for (int64_t i = 0; i < m; ++i) {
      p[i] = beta * dot4(a + (k + 1 + i) * n + (k + 1), vv, m);
    }
    double kk = 0.0;
    for (int64_t i = 0; i < m; ++i) kk += vv[i] * p[i];
    kk *= 0.5 * beta;
    for (int64_t i = 0; i < m; ++i) w[i] = p[i] - kk * vv[i];
    // A22 -= v w^T + w v^T
#pragma omp parallel for num_threads(nthreads()) schedule(static) if (m > 256)
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
  }

  // ---- Q^T = H_{n-3} ... H_0, accumulated backwards: X <- X H_k for
  // k = n-3 .. 0 starting from X = I.  Before step k, X differs from I only
  // in rows/columns k+2.., so the step touches the block X[k+1.., k+1..].
  std::vector<double> qt((size_t)(n * n), 0.0);   // Q^T, row r = column r of Q
  for (int64_t i = 0; i < n; ++i) qt[i * n + i] = 1.0;
  for (int64_t k = n - 3; k >= 0; --k) {
    const double beta = betas[k];
    if (beta == 0.0) continue;
    const int64_t m = n - k - 1;
    const double* vv = refl.data() + k * n;
    // y = X[k+1.., k+1..] v (rows contiguous), then X -= beta y v^T
#pragma omp parallel for num_threads(nthreads()) schedule(static) if (m > 128)
    for (int64_t i = 0; i < m; ++i) {
      double* row = qt.data() + (k + 1 + i) * n + (k + 1);
      const double bs = beta * dot4(row, vv, m);
      for (int64_t j = 0; j < m; ++j) row[j] -= bs * vv[j];
    }
  }
  std::vector<double> d(n), e(n, 0.0);
  for (int64_t i = 0; i < n; ++i) d[i] = a[i * n + i];
  for (int64_t i = 0; i + 1 < n; ++i) e[i] = a[(i + 1) * n + i];

  // ---- implicit QL on (d, e); the rotations (acting on rows i, i+1 of
  // Q^T) are recorded and applied afterwards, all sweeps at once
  const double tiny = 2.220446049250313e-16;
  std::vector<double> rc(n), rs(n);
  Sweeps sw;
  for (int64_t l = 0; l < n; ++l) {
    for (int iter = 0; iter < 200; ++iter) {
      int64_t m = l;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= tiny * dd) break;
      }
      if (m == l) break;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = hyp(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      bool early = false;
      int64_t ilo = m;                  // rotations recorded for rows ilo .. m-1
      for (int64_t i = m - 1; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = hyp(f, g);
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
        rc[i] = c;
        rs[i] = s;
        ilo = i;
      }
      if (m > ilo) {
        sw.lo.push_back(ilo);
        sw.hi.push_back(m);
        sw.off.push_back((int64_t)sw.cs.size() / 2);
        for (int64_t i = m - 1; i >= ilo; --i) {
          sw.cs.push_back(rc[i]);
          sw.cs.push_back(rs[i]);
        }
      }
      if (early) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }

  apply_sweeps(qt.data(), n, sw);

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
