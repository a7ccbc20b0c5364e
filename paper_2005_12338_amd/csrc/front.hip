// Screening of the three-index integrals (eq:V_ijA): (ij|A)^L keeps the
// elements with |(ij|A)| >= (eps' / N) M_j, M_j the largest |(ij|A)| over
// i and A for orbital j.  Layout [N_aux][N][N] (A, i, j), FP64 or FP32.
#include "kernels.hpp"

namespace {

__device__ __forceinline__ double load_x(const void* p, int64_t at, int f64) {
  return f64 ? ((const double*)p)[at] : (double)((const float*)p)[at];
}

constexpr int kRows = 64;   // (A, i) rows per block of the column maximum

// mbits[j] = bits of max |x| over the rows of column j.  Non-negative
// doubles order like their bit patterns, so the maximum is an integer one.
__global__ __launch_bounds__(256) void k_colmax(const void* x, int f64, int64_t n, int64_t rows,
                                                unsigned long long* mbits) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const int64_t r0 = (int64_t)blockIdx.y * kRows, r1 = r0 + kRows < rows ? r0 + kRows : rows;
  double m = 0.0;
  for (int64_t r = r0; r < r1; ++r) m = fmax(m, fabs(load_x(x, r * n + j, f64)));
  atomicMax(mbits + j, (unsigned long long)__double_as_longlong(m));
}

__global__ __launch_bounds__(256) void k_screen(const void* x, int f64, int64_t n, int64_t total, double c,
                                                const unsigned long long* mbits, void* out,
                                                unsigned long long* kept) {
  __shared__ unsigned int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < total) {
    const double v = load_x(x, e, f64);
    const double thr = c * __longlong_as_double((long long)mbits[e % n]);
    const bool keep = fabs(v) >= thr;
    if (f64)
      ((double*)out)[e] = keep ? v : 0.0;
    else
      ((float*)out)[e] = keep ? ((const float*)x)[e] : 0.0f;
    if (keep) atomicAdd(&cnt, 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0 && cnt) atomicAdd(kept, (unsigned long long)cnt);
}

}  // namespace

void launch_screen_ija(const void* x, bool f64, int64_t n, int64_t naux, double eps_over_n,
                       unsigned long long* mbits, void* out, unsigned long long* kept, hipStream_t st) {
  const int64_t rows = naux * n;
  dim3 g1((unsigned)((n + 255) / 256), (unsigned)((rows + kRows - 1) / kRows));
  hipLaunchKernelGGL(k_colmax, g1, dim3(256), 0, st, x, (int)f64, n, rows, mbits);
  const int64_t total = rows * n;
  hipLaunchKernelGGL(k_screen, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, x, (int)f64, n, total,
                     eps_over_n, (const unsigned long long*)mbits, out, kept);
}
