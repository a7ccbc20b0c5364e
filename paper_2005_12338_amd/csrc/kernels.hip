// Bandwidth-bound and small-block kernels of the RS-SRI-GF2 hot path:
// synthetic factors, the range-separation scans, stochastic-vector builds,
// the block-sparse Coulomb/exchange map JK, reductions and the energy.
#include "kernels.hpp"

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27; z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

__device__ __forceinline__ bf16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (bf16_t)0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Write v to a padded matrix in storage format `p` (planes at +plane).
__device__ __forceinline__ void put_st(void* base, int64_t i, int64_t plane, Prec p, double v) {
  switch (p) {
    case Prec::F64: ((double*)base)[i] = v; break;
    case Prec::F32: ((float*)base)[i] = (float)v; break;
    case Prec::BF16: ((bf16_t*)base)[i] = f2bf((float)v); break;
    case Prec::BF16X3: {
      float f = (float)v;
      bf16_t hi = f2bf(f);
      ((bf16_t*)base)[i] = hi;
      ((bf16_t*)base)[i + plane] = f2bf(f - bf2f(hi));
    } break;
  }
}
// Read element i of a padded matrix in storage format `p` (hi + lo planes for BF16X3).
__device__ __forceinline__ double get_st(const void* base, int64_t i, int64_t plane, Prec p) {
  switch (p) {
    case Prec::F64: return ((const double*)base)[i];
    case Prec::F32: return (double)((const float*)base)[i];
    case Prec::BF16: return (double)bf2f(((const bf16_t*)base)[i]);
    default: return (double)bf2f(((const bf16_t*)base)[i]) + (double)bf2f(((const bf16_t*)base)[i + plane]);
  }
}
__device__ __forceinline__ double get_acc(const void* base, int64_t i, bool f64) {
  return f64 ? ((const double*)base)[i] : (double)((const float*)base)[i];
}

// ------------------------------------------------------------- RNG words --
__global__ void k_rng_words(uint64_t seed, uint32_t stream, uint32_t s, uint32_t q0,
                            int64_t count, uint64_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint64_t ctr = ((uint64_t)stream << 62) | ((uint64_t)s << 32) | (uint64_t)(q0 + (uint32_t)i);
  out[i] = mix64(seed * 0x9E3779B97F4A7C15ull + ctr + 1ull);
}

// theta[v][Q] = +-1 for vector v = (stream, s0 + s) with stream = v / ns.
__global__ void k_theta(uint64_t seed, int64_t ns, int64_t s0, int64_t naux, int8_t* theta) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = 2 * ns * naux;
  if (i >= total) return;
  int64_t v = i / naux, q = i % naux;
  uint64_t stream = (uint64_t)(v / ns), s = (uint64_t)(s0 + v % ns);
  uint64_t ctr = (stream << 62) | (s << 32) | (uint64_t)q;
  uint64_t w = mix64(seed * 0x9E3779B97F4A7C15ull + ctr + 1ull);
  theta[i] = (w >> 63) ? (int8_t)-1 : (int8_t)1;
}

// Importance draws: for vector v (stream v / ns, sample s0 + v % ns) and
// draw j: u from q = 2j, sign from q = 2j + 1; Q = min{i : u < cdf[i]}.
__global__ void k_draws(uint64_t seed, int64_t ns, int64_t s0, int32_t k, const double* cdf,
                        int64_t naux, const double* p, int32_t* qout, double* wout) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * ns * k) return;
  int64_t v = i / k;
  uint64_t j = (uint64_t)(i % k);
  uint64_t stream = (uint64_t)(v / ns), s = (uint64_t)(s0 + v % ns);
  uint64_t base = seed * 0x9E3779B97F4A7C15ull + ((stream << 62) | (s << 32)) + 1ull;
  uint64_t wu = mix64(base + 2 * j);
  uint64_t ws = mix64(base + 2 * j + 1);
  double u = (double)(wu >> 11) * 0x1.0p-53;
  int64_t lo = 0, hi = naux - 1;            // smallest index with u < cdf[index]
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (u < cdf[mid]) hi = mid; else lo = mid + 1;
  }
  qout[i] = (int32_t)lo;
  double sg = (ws >> 63) ? -1.0 : 1.0;
  wout[i] = sg / sqrt((double)k * p[lo]);
}

// Stratified vectors: vector v (stream v / ns, sample s0 + v % ns) draws its
// class c (u of q = 0xFFFFFFFF, smallest c with u < cdf[c]); theta[v][Q] is
// the +-1 sign of (stream, s, Q) on the class members (Q = c mod nclass), 0
// elsewhere, and vscale[v] = 1 / sqrt(pi_c).
__global__ void k_theta_strat(uint64_t seed, int64_t ns, int64_t s0, int64_t naux, int32_t nclass,
                              const double* cdf, const double* pi, int8_t* theta, double* vscale) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * ns * naux) return;
  int64_t v = i / naux, q = i % naux;
  uint64_t stream = (uint64_t)(v / ns), s = (uint64_t)(s0 + v % ns);
  uint64_t base = seed * 0x9E3779B97F4A7C15ull + ((stream << 62) | (s << 32)) + 1ull;
  const double u = (double)(mix64(base + 0xFFFFFFFFull) >> 11) * 0x1.0p-53;
  int lo = 0, hi = nclass - 1;               // smallest class with u < cdf[class]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (u < cdf[mid]) hi = mid; else lo = mid + 1;
  }
  const uint64_t w = mix64(base + (uint64_t)q);
  theta[i] = (q % nclass == lo) ? ((w >> 63) ? (int8_t)-1 : (int8_t)1) : (int8_t)0;
  if (q == 0) vscale[v] = 1.0 / sqrt(pi[lo]);
}

// ------------------------------------------------------------- B build ----
// One workgroup per (row i, kSynthQ consecutive Q), its threads along the
// row: the (i, j) factor amp exp(-a d^2) is evaluated once for those Q, and
// every element is the same product as B's definition evaluated directly.
constexpr int kSynthQ = 8;
__global__ __launch_bounds__(256) void k_synth_b(int64_t n, int64_t naux, const double* x, const double* xq,
                                                 double amp, double a, double c, void* out, int f64) {
  const int64_t i = blockIdx.x, q0 = (int64_t)blockIdx.y * kSynthQ;
  const double xi = x[i];
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    const double xj = x[j];
    const double d = xi - xj;
    const double f = amp * exp(-a * d * d);
    const double mid = 0.5 * (xi + xj);
    for (int64_t q = q0; q < q0 + kSynthQ && q < naux; ++q) {
      const double m = xq[q] - mid;
      const double v = f * exp(-c * m * m);
      const int64_t e = (q * n + i) * n + j;
      if (f64) ((double*)out)[e] = v; else ((float*)out)[e] = (float)v;
    }
  }
}

// ------------------------------------------------------------- split ------
__global__ void k_maxabs(const void* b, int f64, int64_t total, double* part) {
  __shared__ double sm[256];
  double m = 0.0;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
  if (!f64 && total % 4 == 0 && ((uintptr_t)b & 15) == 0) {
    // FP32: four elements per 16-byte load (the maximum does not depend on
    // the order it is taken in)
    const float4* b4 = (const float4*)b;
    float m4 = 0.0f;
    for (int64_t e = t0; e < total / 4; e += stride) {
      const float4 v = b4[e];
      m4 = fmaxf(m4, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
    m = (double)m4;
  } else {
    for (int64_t e = t0; e < total; e += stride) m = fmax(m, fabs(get_acc(b, e, f64)));
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + d]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// One wave per (Q, i): flag rows with a kept element, count kept elements.
__global__ void k_rowflags(const void* b, int f64, int64_t n, int64_t naux, double thr,
                           uint8_t* flags, unsigned long long* nnz) {
  int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int lane = threadIdx.x & 63;
  if (wid >= naux * n) return;
  const int64_t base = wid * n;
  int cnt = 0;
  if (!f64 && n % 4 == 0 && ((uintptr_t)b & 15) == 0) {
    // FP32 rows: four elements per 16-byte load
    const float4* r4 = (const float4*)((const float*)b + base);
    for (int64_t j = lane; j < n / 4; j += 64) {
      const float4 v = r4[j];
      cnt += (fabs((double)v.x) >= thr) + (fabs((double)v.y) >= thr) + (fabs((double)v.z) >= thr) +
             (fabs((double)v.w) >= thr);
    }
  } else {
    for (int64_t j = lane; j < n; j += 64) cnt += fabs(get_acc(b, base + j, f64)) >= thr ? 1 : 0;
  }
  for (int d = 32; d > 0; d >>= 1) cnt += __shfl_down(cnt, d, 64);
  if (lane == 0) {
    flags[wid] = cnt > 0;
    if (cnt) atomicAdd(nnz, (unsigned long long)cnt);
  }
}

__global__ void k_extract_blocks(const void* b, int f64, int64_t n, int64_t naux, double thr,
                                 const int32_t* w, const int32_t* idx, double* blk, float* blk32) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= naux * kWMax * kWMax) return;
  int64_t q = e / (kWMax * kWMax);
  int r = (int)((e / kWMax) % kWMax), c = (int)(e % kWMax);
  double v = 0.0;
  if (r < w[q] && c < w[q]) {
    int64_t i = idx[q * kWMax + r], j = idx[q * kWMax + c];
    double x = get_acc(b, (q * n + i) * n + j, f64);
    v = fabs(x) >= thr ? x : 0.0;
  }
  blk[e] = v;
  blk32[e] = (float)v;
}

// ------------------------------------------------------------- R build ----
// Dense pass over B for a batch of vectors: X_L = sum_Q theta_Q K^L_Q and
// X_S = sum_Q theta_Q (B_Q - K^L_Q) (elements below the threshold), written
// to padded storage.  One thread per (i, j) and RV vectors; theta staged in
// LDS per chunk of Q.
template <int RV, typename T>
__global__ __launch_bounds__(256) void k_rbuild(const void* b, const void* lsrc, int f64, int64_t n, int64_t naux,
                                                 double thr, const int8_t* theta, int64_t nvec,
                                                 int64_t v0, Prec prec, void* xl, void* xs,
                                                 int64_t np, int64_t plane, int64_t mstride,
                                                 const double* vscale) {
  constexpr int QC = 64;
  __shared__ __attribute__((aligned(16))) T th[QC][RV];   // the RV signs of one Q side by side
  const int64_t ij = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t vb = v0 + (int64_t)blockIdx.y * RV;
  const bool ok = ij < n * n;
  T al[RV], as[RV];
#pragma unroll
  for (int r = 0; r < RV; ++r) { al[r] = 0; as[r] = 0; }
  for (int64_t q0 = 0; q0 < naux; q0 += QC) {
    __syncthreads();
    for (int e = threadIdx.x; e < RV * QC; e += blockDim.x) {
      int r = e / QC, qq = e % QC;
      int64_t v = vb + r, q = q0 + qq;
      th[qq][r] = (v < nvec && q < naux) ? (T)theta[v * naux + q] : (T)0;
    }
    __syncthreads();
    if (ok) {
      const int qe = (int)((naux - q0) < QC ? (naux - q0) : QC);
      for (int qq = 0; qq < qe; ++qq) {
        const int64_t at = (q0 + qq) * n * n + ij;
        T x = f64 ? (T)((const double*)b)[at] : (T)((const float*)b)[at];
        // large part: the source element where it passes the threshold
        // (the source is B itself unless the split has its own)
        T y = !lsrc ? x : f64 ? (T)((const double*)lsrc)[at] : (T)((const float*)lsrc)[at];
        T lx = fabs((double)y) >= thr ? y : (T)0;
        T sx = x - lx;
#pragma unroll
        for (int r = 0; r < RV; ++r) {
          al[r] += th[qq][r] * lx;
          as[r] += th[qq][r] * sx;
        }
      }
    }
  }
  if (!ok) return;
  const int64_t i = ij / n, j = ij % n;
#pragma unroll
  for (int r = 0; r < RV; ++r) {
    int64_t v = vb + r;
    if (v >= nvec) break;
    int64_t o = v * mstride + i * np + j;
    const double sc = vscale ? vscale[v] : 1.0;     // stratified vectors: 1/sqrt(pi_c)
    put_st(xl, o, plane, prec, (double)al[r] * sc);
    put_st(xs, o, plane, prec, (double)as[r] * sc);
  }
}

// Importance vectors: X = sum_j wgt_j B_{Q_j} split into L and S parts.
__global__ void k_rimportance(const void* b, const void* lsrc, int f64, int64_t n, double thr, const int32_t* q,
                              const double* wgt, int32_t k, int64_t nvec, Prec prec, void* xl,
                              void* xs, int64_t np, int64_t plane, int64_t mstride) {
  const int64_t ij = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t v = blockIdx.y;
  if (ij >= n * n || v >= nvec) return;
  double al = 0.0, as = 0.0;
  for (int j = 0; j < k; ++j) {
    int64_t qq = q[v * k + j];
    const double x = get_acc(b, qq * n * n + ij, f64);
    const double y = lsrc ? get_acc(lsrc, qq * n * n + ij, f64) : x;
    const double lx = fabs(y) >= thr ? y : 0.0;
    al += wgt[v * k + j] * lx;
    as += wgt[v * k + j] * (x - lx);
  }
  const int64_t i = ij / n, jj = ij % n;
  int64_t o = v * mstride + i * np + jj;
  put_st(xl, o, plane, prec, al);
  put_st(xs, o, plane, prec, as);
}

// ------------------------------------------------------------- G ----------
// A[t][i][k] = C[i][k] * exp(lw[t][k]) (padded), the left factor of
// G = -C diag(weights) C^T.
__global__ void k_scale_cols(const double* c, const double* lw, int64_t n, int64_t np,
                             int64_t ntau, double* out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ntau * np * np) return;
  int64_t t = e / (np * np), ik = e % (np * np), i = ik / np, k = ik % np;
  double v = 0.0;
  if (i < n && k < n) v = c[i * n + k] * exp(lw[t * n + k]);
  out[e] = v;
}

// out[t] (n x n) = (P[t] + P[t]^T) / 2 * sign from padded P.
// out[t][i][j] = sign (p[t][i][j] + p[t][j][i]) / 2 on 32 x 32 tiles: one
// workgroup per (output tile, tau t0 + blockIdx.y); the mirror tile is read
// row by row and transposed through LDS, so every global access is
// contiguous.
__global__ __launch_bounds__(256) void k_unpad_sym(const double* p, int64_t n, int64_t np, int64_t t0,
                                                   int64_t ntile, double sign, double* out) {
  __shared__ double tb[32][33];
  const int64_t t = t0 + blockIdx.y;
  const int64_t bi = blockIdx.x / ntile, bj = blockIdx.x % ntile;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const double* pt = p + t * np * np;
  for (int r = ty; r < 32; r += 8) {           // tb[r][c] = p[32 bj + r][32 bi + c]
    const int64_t gi = bj * 32 + r, gj = bi * 32 + tx;
    tb[r][tx] = (gi < n && gj < n) ? pt[gi * np + gj] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi * 32 + r, j = bj * 32 + tx;
    if (i < n && j < n) out[(t * n + i) * n + j] = sign * 0.5 * (pt[i * np + j] + tb[tx][r]);
  }
}

// Padded copies of G(tau) in storage format and FP64.
// One workgroup per (padded row i, tau t0 + blockIdx.y), its threads along
// the row: contiguous reads and writes, no index divisions per element.
__global__ __launch_bounds__(256) void k_pad_convert(const double* g, int64_t n, int64_t np, int64_t t0,
                                                     Prec prec, void* st, int64_t plane, int64_t mstride,
                                                     double* f64pad) {
  const int64_t i = blockIdx.x, t = t0 + blockIdx.y;
  const double* grow = g + (t * n + i) * n;
  for (int64_t j = threadIdx.x; j < np; j += blockDim.x) {
    const int64_t ij = i * np + j;
    const double v = (i < n && j < n) ? grow[j] : 0.0;
    put_st(st, t * mstride + ij, plane, prec, v);
    if (f64pad) f64pad[t * np * np + ij] = v;
  }
}

// ------------------------------------------------------------- JK ---------
// Block pitch of the J blocks: the split's widest block rounded up to 8, 16
// or kWMax.
__host__ __device__ __forceinline__ int jk_pitch(int32_t wmax) { return wmax <= 8 ? 8 : wmax <= 16 ? 16 : kWMax; }

// For every (slot, Q) and m in 0..3: J = 2 Tr(k W) k - k W k with k the
// w x w block of K^L_Q on its support and W the m-th matrix of the slot
// (accumulator format, row-major padded) restricted to that support.  One
// wave per (slot, Q) computes all four m, so k and the support are read
// once; lane e holds block element (e / w, e % w) of every m (w <= WB).
// Output jout[((slot naux + Q) JP^2 + a JP + c) 4 + m], JP = WB: the four m
// of an element side by side for the scatter.  Waves share nothing: each
// keeps its blocks in its own LDS slice, ordered by a wave-level fence (LDS
// operations of one wave complete in order).
template <typename T, int WB, int NW>
__global__ __launch_bounds__(64 * NW) void k_jk_blocks(const void* wbase, int64_t w_st_slot,
                                                       int64_t w_st_m, int64_t np, int64_t naux,
                                                       int32_t nslot, const int32_t* wq,
                                                       const int32_t* idx, const T* blk, T* jout) {
  constexpr int E = WB * WB;
  __shared__ T sk[NW][E];
  __shared__ T sw[NW][4][E];
  __shared__ T st[NW][4][E];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t task = (int64_t)blockIdx.x * NW + wv;
  if (task >= (int64_t)nslot * naux) return;       // whole wave leaves together
  const int64_t q = task % naux;
  const int64_t slot = task / naux;
  const int w = wq[q];
  const T* W = (const T*)wbase + slot * w_st_slot;
  const int32_t* s = idx + q * kWMax;
  const int ww = w * w;
  for (int e = lane; e < ww; e += 64) {
    const int a = e / w, c = e % w;
    sk[wv][e] = blk[q * kWMax * kWMax + a * kWMax + c];
    const int64_t o = (int64_t)s[a] * np + s[c];
#pragma unroll
    for (int m = 0; m < 4; ++m) sw[wv][m][e] = W[m * w_st_m + o];
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // t_m = Tr(k W_m) = sum_ac k_ac (W_m)_ca
  T tr[4] = {0, 0, 0, 0};
  for (int e = lane; e < ww; e += 64) {
    const int a = e / w, c = e % w;
    const T kv = sk[wv][e];
#pragma unroll
    for (int m = 0; m < 4; ++m) tr[m] += kv * sw[wv][m][c * w + a];
  }
#pragma unroll
  for (int m = 0; m < 4; ++m)
    for (int d = 32; d > 0; d >>= 1) tr[m] += __shfl_xor(tr[m], d, 64);
  for (int e = lane; e < ww; e += 64) {
    const int a = e / w, c = e % w;
    T acc[4] = {0, 0, 0, 0};
    for (int x = 0; x < w; ++x) {
      const T kv = sk[wv][a * w + x];
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m] += kv * sw[wv][m][x * w + c];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) st[wv][m][e] = acc[m];
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  T* out = jout + task * E * 4;
  for (int e = lane; e < ww; e += 64) {
    const int a = e / w, c = e % w;
    T acc[4] = {0, 0, 0, 0};
    for (int x = 0; x < w; ++x) {
      const T kv = sk[wv][x * w + c];
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m] += st[wv][m][a * w + x] * kv;
    }
    const T kv = sk[wv][e];
    T* o = out + (a * WB + c) * 4;
#pragma unroll
    for (int m = 0; m < 4; ++m) o[m] = 2 * tr[m] * kv - acc[m];
  }
}

// Scatter the J blocks onto the union pattern: for every pattern entry (i,j)
// sum the contributions in their fixed order (the four m of a contribution
// are adjacent).  m = 0, 1 (W_L, W_S) go to row-major outputs; m = 2, 3
// (Z_L, Z_S) to transposed outputs, with the second transposed output
// holding J(Z_L) + J(Z_S).
template <typename T>
__global__ void k_jk_scatter(const T* jblk, int64_t naux, int32_t nslot, int64_t npat, int jp,
                             const int32_t* pat_ij, const int32_t* pat_off, const int32_t* pat_q,
                             int64_t np, Prec prec, int64_t plane, void* jw_l, void* jw_s,
                             void* jz_st, void* jz_sum_t, int64_t out_st_slot) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nslot * npat) return;
  int64_t slot = e / npat, p = e % npat;
  int64_t ij = pat_ij[p], i = ij / np, j = ij % np;
  const T* jb = jblk + slot * naux * jp * jp * 4;
  double v[4] = {0, 0, 0, 0};
  for (int c = pat_off[p]; c < pat_off[p + 1]; ++c) {
    const int32_t code = pat_q[c];
    const int64_t q = code >> 10;
    const int a = (code >> 5) & 31, b = code & 31;
    const T* x = jb + ((q * jp + a) * jp + b) * 4;
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] += (double)x[m];
  }
  int64_t o = slot * out_st_slot;
  put_st(jw_l, o + i * np + j, plane, prec, v[0]);
  put_st(jw_s, o + i * np + j, plane, prec, v[1]);
  put_st(jz_st, o + j * np + i, plane, prec, v[3]);
  put_st(jz_sum_t, o + j * np + i, plane, prec, v[2] + v[3]);
}

// ------------------------------------------------------------- reductions -
// Direct-term coefficients from the Hadamard partials c_xy = Tr(M_xy Gb):
// coef = 2 (c_SS, c_SL + c_SS, c_LS + c_SS, c_LL + c_LS + c_SL + c_SS).
// Fixed-order sum of p[0..cnt) by one wave: lane l takes l, l+64, ... in
// order, then a butterfly over the lanes (the same pattern on every call).
__device__ __forceinline__ double wave_sum_fixed(const double* p, int64_t cnt) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int64_t t = lane; t < cnt; t += 64) s += p[t];
  for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
  return s;
}

// Direct-term coefficients of a slot from its Hadamard-trace partials: one
// workgroup per slot, one wave per trace.
__global__ __launch_bounds__(256) void k_trace_coef(const double* part, int64_t ntiles, int32_t nslot,
                                                    double* coef, int mode) {
  __shared__ double c[4];
  const int slot = blockIdx.x, h = threadIdx.x >> 6;
  const double s = wave_sum_fixed(part + ((int64_t)slot * 4 + h) * ntiles, ntiles);
  if ((threadIdx.x & 63) == 0) c[h] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double* o = coef + (int64_t)slot * kCoefStride;
    if (mode == 0) {
      o[0] = 2.0 * c[3];
      o[1] = 2.0 * (c[2] + c[3]);
      o[2] = 2.0 * (c[1] + c[3]);
      o[3] = 2.0 * (c[0] + c[1] + c[2] + c[3]);
      for (int h = 0; h < 4; ++h) o[4 + h] = c[h];       // Tr(T_h) = Tr(M_h Gbar)
    } else {
      // control-variate form: direct terms 2 Tr(T_t) M_t - 2 Tr(T_L) M_L
      o[0] = 2.0 * c[0];
      o[1] = -2.0 * c[1];
      o[2] = o[3] = 0.0;
      o[4] = c[0];
      o[5] = c[1];
      o[6] = o[7] = 0.0;
    }
  }
}

// Sigma_sum[tau] += sum of the chunk's Sigma_s in unit order, each the
// product stage's output plus its direct terms sum_x coef_x M_x (M_x the
// slot's four M matrices in storage format, coef from k_trace_coef).  One
// thread per (tau-group, i, four consecutive j): the padded rows (np a
// multiple of 32) give aligned 4-element vectors.
__global__ void k_accumulate(const Unit* units, int32_t nunit, const void* sig, int f64,
                             int64_t sig_st_slot, int64_t n, int64_t np, double* sum,
                             int32_t tau_lo, int32_t tau_hi, const void* mst, Prec prec,
                             int64_t m_st_slot, int64_t m_st_m, int64_t plane, const double* coef) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ntau = tau_hi - tau_lo, nq = np / 4;
  if (e >= ntau * n * nq) return;
  const int32_t t = tau_lo + (int32_t)(e / (n * nq));
  const int64_t r = e % (n * nq), i = r / nq, j0 = 4 * (r % nq);
  if (j0 >= n) return;
  const int nj = (int)(n - j0 < 4 ? n - j0 : 4);
  double* srow = sum + (int64_t)t * n * n + i * n + j0;
  double acc[4];
  for (int k = 0; k < nj; ++k) acc[k] = srow[k];
  for (int k = nj; k < 4; ++k) acc[k] = 0.0;
  for (int u = 0; u < nunit; ++u) {
    if (units[u].tau != t) continue;
    const int64_t slot = units[u].slot;
    const int64_t o = i * np + j0;
    double v[4];
    if (f64) {
      const double* p = (const double*)sig + slot * sig_st_slot + o;
      for (int k = 0; k < 4; ++k) v[k] = p[k];
    } else {
      const float4 x = *(const float4*)((const float*)sig + slot * sig_st_slot + o);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    }
    const double* cf = coef + slot * kCoefStride;
    for (int x = 0; x < 4; ++x) {
      if (cf[x] == 0.0) continue;                     // matrices a form does not use are never read
      const int64_t mo = slot * m_st_slot + x * m_st_m + o;
      if (prec == Prec::BF16) {
        const uint2 h = *(const uint2*)((const bf16_t*)mst + mo);
        v[0] += cf[x] * (double)bf2f((bf16_t)(h.x & 0xffffu));
        v[1] += cf[x] * (double)bf2f((bf16_t)(h.x >> 16));
        v[2] += cf[x] * (double)bf2f((bf16_t)(h.y & 0xffffu));
        v[3] += cf[x] * (double)bf2f((bf16_t)(h.y >> 16));
      } else {
        for (int k = 0; k < 4; ++k) v[k] += cf[x] * get_st(mst, mo + k, plane, prec);
      }
    }
    for (int k = 0; k < 4; ++k) acc[k] += v[k];
  }
  for (int k = 0; k < nj; ++k) srow[k] = acc[k];
}

// e_s(tau) of every unit: its per-tile partials of Tr(product part Gbar)
// plus the direct terms' sum_x coef_x Tr(M_x Gbar).  One wave per unit.
__global__ __launch_bounds__(256) void k_esamples(const Unit* units, int32_t nunit, const double* part,
                                                  int64_t ntiles, int64_t s0, int64_t ntau, double* es,
                                                  const double* coef) {
  const int u = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (u >= nunit) return;                        // whole wave leaves together
  const double s = wave_sum_fixed(part + (int64_t)units[u].slot * ntiles, ntiles);
  if ((threadIdx.x & 63) == 0) {
    const double* cf = coef + (int64_t)units[u].slot * kCoefStride;
    double d = 0.0;
    for (int x = 0; x < 4; ++x) d += cf[x] * cf[4 + x];
    es[((int64_t)units[u].row - s0) * ntau + units[u].tau] = s + d;
  }
}

__global__ void k_finalize(const double* det, const double* sum, int64_t n, int64_t ntau,
                           double inv2ns, double* out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ntau * n * n) return;
  int64_t t = e / (n * n), ij = e % (n * n), i = ij / n, j = ij % n;
  const double* s = sum + t * n * n;
  out[e] = det[e] + inv2ns * (s[i * n + j] + s[j * n + i]);
}

// Two-level correction of the BF16 estimator.  sum += lo + c (hi - lo):
// the BF16 sum of the probe pairs (lo) joins the rest of the pairs, and c =
// ns / k times the probe pairs' BF16X3 - BF16 difference moves the total to
// the BF16X3 level in expectation.
__global__ void k_level_correct(double* sum, const double* hi, const double* lo, int64_t count, double c) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  sum[e] += lo[e] + c * (hi[e] - lo[e]);
}
// shift[t] = (1/k) sum_{q<k} (hi[q][t] - es[q][t]) (fixed order), then every
// sample row q < ns gets es[q][t] += shift[t].  One block, ntau <= 4096.
__global__ void k_level_shift(double* es, const double* hi, int64_t k, int64_t ns, int64_t ntau) {
  __shared__ double shift[4096];
  for (int64_t t = threadIdx.x; t < ntau; t += blockDim.x) {
    double d = 0.0;
    for (int64_t q = 0; q < k; ++q) d += hi[q * ntau + t] - es[q * ntau + t];
    shift[t] = d / (double)k;
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < ns * ntau; e += blockDim.x) es[e] += shift[e % ntau];
}

// Energy of the double average: out[0] = -gm sum_t w_t tr[t] (tr from the
// final Sigma), out[2] = its first-order U-statistic standard error
// sqrt(Var_i(r_i)/ns + Var_j(c_j)/ns) with r_i, c_j the row and column means
// of the per-combination energies E_ij = -gm sum_t w_t es[i ns + j][t].
// One block; ns <= 256; fixed summation orders.
__global__ void k_double_stats(const double* tr, const double* w, int64_t ntau, const double* es, int64_t ns,
                               double gm, double* out) {
  __shared__ double rm[256], cm[256];
  for (int64_t k = threadIdx.x; k < 2 * ns; k += blockDim.x) {
    const int64_t a = k % ns;
    const bool row = k < ns;
    double acc = 0.0;
    for (int64_t b = 0; b < ns; ++b) {
      const double* e = es + (row ? a * ns + b : b * ns + a) * ntau;
      double v = 0.0;
      for (int64_t t = 0; t < ntau; ++t) v += w[t] * e[t];
      acc += -gm * v;
    }
    (row ? rm : cm)[a] = acc / (double)ns;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double e = 0.0;
    for (int64_t t = 0; t < ntau; ++t) e += w[t] * tr[t];
    double mr = 0.0, mc = 0.0;
    for (int64_t a = 0; a < ns; ++a) { mr += rm[a]; mc += cm[a]; }
    mr /= (double)ns;
    mc /= (double)ns;
    double vr = 0.0, vc = 0.0;
    for (int64_t a = 0; a < ns; ++a) { vr += (rm[a] - mr) * (rm[a] - mr); vc += (cm[a] - mc) * (cm[a] - mc); }
    vr /= (double)(ns - 1);
    vc /= (double)(ns - 1);
    out[0] = -gm * e;
    out[1] = 0.0;
    out[2] = sqrt(vr / (double)ns + vc / (double)ns);
  }
}

// xt = xl + xs element by element (storage format; count elements of the
// hi plane, each matrix of mstride elements also carrying its lo plane).
__global__ void k_vec_sum(const void* xl, const void* xs, void* xt, int64_t count, Prec prec, int64_t plane,
                          int64_t mstride) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  if (prec == Prec::BF16X3 && (e % mstride) >= plane) return;   // lo planes: written with their hi element
  put_st(xt, e, plane, prec, get_st(xl, e, plane, prec) + get_st(xs, e, plane, prec));
}

// ------------------------------------------------------------- energy -----
// tr[t] = sum_ij Sigma[t]_ij Gbar[t]_ji: one block per tau, fixed-order tree.
__global__ void k_trace_prod(const double* sig, const double* gb, int64_t n, double* tr) {
  __shared__ double sm[256];
  const int64_t t = blockIdx.x;
  const double* s = sig + t * n * n;
  const double* g = gb + t * n * n;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < n * n; e += blockDim.x) {
    int64_t i = e / n, j = e % n;
    acc += s[e] * g[j * n + i];
  }
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) sm[threadIdx.x] += sm[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) tr[t] = sm[0];
}

// out[0] = E_tot, out[1] = mean_s E_s - E_tot (~0), out[2] = stderr.
// E_tot = -gm sum_t w_t (tr[t] + [add_mean] mean_s e_s(t)) and the
// standard error of the per-sample totals (one block, fixed order).
__global__ void k_energy_stats(const double* tr, const double* w, int64_t ntau, const double* es,
                               int64_t ns, double gm, int add_mean, double* out) {
  __shared__ double sm[256];
  __shared__ double ebar[512];
  __shared__ double etot_s;
  // mean over samples of e_s(tau), per tau (tau <= 512 handled in shared)
  for (int64_t t = threadIdx.x; t < ntau && t < 512; t += blockDim.x) {
    double m = 0.0;
    for (int64_t s = 0; s < ns; ++s) m += es ? es[s * ntau + t] : 0.0;
    ebar[t] = ns ? m / (double)ns : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double e = 0.0;
    for (int64_t t = 0; t < ntau; ++t) e += w[t] * (tr[t] + (add_mean ? ebar[t] : 0.0));
    etot_s = -gm * e;
  }
  __syncthreads();
  const double etot = etot_s;
  double acc = 0.0, acc2 = 0.0;
  for (int64_t s = threadIdx.x; s < ns && es; s += blockDim.x) {
    double d = 0.0;
    for (int64_t t = 0; t < ntau; ++t) d += w[t] * (es[s * ntau + t] - ebar[t]);
    double e_s = etot - gm * d;
    acc += e_s - etot;
    acc2 += (e_s - etot) * (e_s - etot);
  }
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) sm[threadIdx.x] += sm[threadIdx.x + d];
    __syncthreads();
  }
  double sum1 = sm[0];
  __syncthreads();
  sm[threadIdx.x] = acc2;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) sm[threadIdx.x] += sm[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = etot;
    out[1] = ns ? sum1 / (double)ns : 0.0;
    double var = ns > 1 ? (sm[0] - sum1 * sum1 / (double)ns) / (double)(ns - 1) : 0.0;
    out[2] = ns > 1 ? sqrt(fmax(var, 0.0) / (double)ns) : 0.0;
  }
}

__global__ void k_count_nonfinite(const double* x, int64_t count, unsigned long long* bad) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count && !isfinite(x[e])) atomicAdd(bad, 1ull);
}

// dst[c * ld + r] = src[r][c] (src rows x cols, FP64 or FP32) into FP64.
__global__ void k_transpose(const void* src, int f64, int64_t rows, int64_t cols, double* dst, int64_t ld) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  int64_t r = e / cols, c = e % cols;
  dst[c * ld + r] = get_acc(src, e, f64);
}
// dst[c][r] = src[r * ld + c] for r < rows, c < cols (dst cols x rows).
__global__ void k_untranspose(const double* src, int64_t rows, int64_t cols, int64_t ld, void* dst, int f64) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  int64_t c = e / rows, r = e % rows;
  double v = src[r * ld + c];
  if (f64) ((double*)dst)[e] = v; else ((float*)dst)[e] = (float)v;
}

inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ------------------------------------------------------------- launchers --

void launch_rng_words(uint64_t seed, uint32_t stream, uint32_t s, uint32_t q0, int64_t count,
                      uint64_t* out, hipStream_t st) {
  hipLaunchKernelGGL(k_rng_words, dim3(blocks(count)), dim3(256), 0, st, seed, stream, s, q0, count, out);
}
void launch_theta(uint64_t seed, int64_t ns, int64_t s0, int64_t naux, int8_t* theta, hipStream_t st) {
  hipLaunchKernelGGL(k_theta, dim3(blocks(2 * ns * naux)), dim3(256), 0, st, seed, ns, s0, naux, theta);
}
void launch_draws(uint64_t seed, int64_t ns, int64_t s0, int32_t k, const double* cdf, int64_t naux,
                  const double* p, int32_t* q, double* w, hipStream_t st) {
  hipLaunchKernelGGL(k_draws, dim3(blocks(2 * ns * k)), dim3(256), 0, st, seed, ns, s0, k, cdf, naux, p, q, w);
}
void launch_synth_b(int64_t n, int64_t naux, const double* x, const double* xq, double amp, double a,
                    double c, void* out, bool f64, hipStream_t st) {
  const int64_t nqb = (naux + kSynthQ - 1) / kSynthQ;
  for (int64_t b0 = 0; b0 < nqb; b0 += 65535) {
    const unsigned nb = (unsigned)std::min<int64_t>(65535, nqb - b0);
    const int64_t off = b0 * kSynthQ * n * n;           // elements before this group of Q
    char* o = (char*)out + off * (f64 ? 8 : 4);
    hipLaunchKernelGGL(k_synth_b, dim3((unsigned)n, nb), dim3(256), 0, st, n, naux - b0 * kSynthQ, x,
                       xq + b0 * kSynthQ, amp, a, c, (void*)o, (int)f64);
  }
}
void launch_maxabs(const void* b, bool f64, int64_t total, double* part, int nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_maxabs, dim3(nblk), dim3(256), 0, st, b, (int)f64, total, part);
}
void launch_rowflags(const void* b, bool f64, int64_t n, int64_t naux, double thr, uint8_t* flags,
                     unsigned long long* nnz, hipStream_t st) {
  int64_t waves = naux * n;
  hipLaunchKernelGGL(k_rowflags, dim3(blocks(waves * 64)), dim3(256), 0, st, b, (int)f64, n, naux, thr, flags, nnz);
}
void launch_extract_blocks(const void* b, bool f64, int64_t n, int64_t naux, double thr,
                           const int32_t* w, const int32_t* idx, double* blk, float* blk32,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_extract_blocks, dim3(blocks(naux * kWMax * kWMax)), dim3(256), 0, st, b,
                     (int)f64, n, naux, thr, w, idx, blk, blk32);
}
void launch_rbuild(const void* b, bool f64, int64_t n, int64_t naux, double thr, const int8_t* theta,
                   int64_t nvec, Prec prec, void* xl, void* xs, int64_t np, int64_t plane,
                   int64_t mstride, hipStream_t st, const double* vscale, const void* lsrc) {
  // vectors per thread: B is streamed once per RV vectors, so RV is as large
  // as the batch allows (up to 32) without idle vector slots
  auto go = [&](auto rv) {
    constexpr int RV = decltype(rv)::value;
    dim3 grid(blocks(n * n), (unsigned)((nvec + RV - 1) / RV));
    if (prec == Prec::F64)
      hipLaunchKernelGGL((k_rbuild<RV, double>), grid, dim3(256), 0, st, b, lsrc, (int)f64, n, naux, thr,
                         theta, nvec, (int64_t)0, prec, xl, xs, np, plane, mstride, vscale);
    else
      hipLaunchKernelGGL((k_rbuild<RV, float>), grid, dim3(256), 0, st, b, lsrc, (int)f64, n, naux, thr,
                         theta, nvec, (int64_t)0, prec, xl, xs, np, plane, mstride, vscale);
  };
  if (nvec <= 8) go(std::integral_constant<int, 8>{});
  else if (nvec <= 16) go(std::integral_constant<int, 16>{});
  else go(std::integral_constant<int, 32>{});
}
void launch_theta_strat(uint64_t seed, int64_t ns, int64_t s0, int64_t naux, int32_t nclass, const double* cdf,
                        const double* pi, int8_t* theta, double* vscale, hipStream_t st) {
  hipLaunchKernelGGL(k_theta_strat, dim3(blocks(2 * ns * naux)), dim3(256), 0, st, seed, ns, s0, naux, nclass, cdf,
                     pi, theta, vscale);
}
void launch_rimportance(const void* b, bool f64, int64_t n, double thr, const int32_t* q,
                        const double* w, int32_t k, int64_t nvec, Prec prec, void* xl, void* xs,
                        int64_t np, int64_t plane, int64_t mstride, hipStream_t st, const void* lsrc) {
  dim3 grid(blocks(n * n), (unsigned)nvec);
  hipLaunchKernelGGL(k_rimportance, grid, dim3(256), 0, st, b, lsrc, (int)f64, n, thr, q, w, k, nvec, prec,
                     xl, xs, np, plane, mstride);
}
void launch_scale_cols(const double* c, const double* lw, int64_t n, int64_t np, int64_t ntau,
                       double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_cols, dim3(blocks(ntau * np * np)), dim3(256), 0, st, c, lw, n, np, ntau, out);
}
void launch_unpad_sym(const double* p, int64_t n, int64_t np, int64_t ntau, double sign, double* out,
                      hipStream_t st) {
  const int64_t ntile = (n + 31) / 32;
  for (int64_t t0 = 0; t0 < ntau; t0 += 65535) {
    const unsigned nt = (unsigned)std::min<int64_t>(65535, ntau - t0);
    hipLaunchKernelGGL(k_unpad_sym, dim3((unsigned)(ntile * ntile), nt), dim3(256), 0, st, p, n, np, t0, ntile,
                       sign, out);
  }
}
void launch_pad_convert(const double* g, int64_t n, int64_t np, int64_t ntau, Prec prec, void* stbuf,
                        int64_t plane, int64_t mstride, double* f64pad, hipStream_t st) {
  for (int64_t t0 = 0; t0 < ntau; t0 += 65535) {
    const unsigned nt = (unsigned)std::min<int64_t>(65535, ntau - t0);
    hipLaunchKernelGGL(k_pad_convert, dim3((unsigned)np, nt), dim3(256), 0, st, g, n, np, t0, prec, stbuf, plane,
                       mstride, f64pad);
  }
}
template <typename T>
void jk_blocks_launch(int32_t wmax, int64_t tasks, hipStream_t st, const void* wbase, int64_t w_st_slot,
                      int64_t w_st_m, int64_t np, int64_t naux, int32_t nslot, const int32_t* wq, const int32_t* idx,
                      const T* blk, T* jout) {
  // four waves per workgroup up to 16-wide blocks; one for the widest, whose
  // LDS slices (9 x 1024 elements) would not fit four times
  auto grid = [&](int nw) { return dim3((unsigned)((tasks + nw - 1) / nw)); };
  if (wmax <= 8)
    hipLaunchKernelGGL((k_jk_blocks<T, 8, 4>), grid(4), dim3(256), 0, st, wbase, w_st_slot, w_st_m, np, naux, nslot,
                       wq, idx, blk, jout);
  else if (wmax <= 16)
    hipLaunchKernelGGL((k_jk_blocks<T, 16, 4>), grid(4), dim3(256), 0, st, wbase, w_st_slot, w_st_m, np, naux, nslot,
                       wq, idx, blk, jout);
  else
    hipLaunchKernelGGL((k_jk_blocks<T, kWMax, 1>), grid(1), dim3(64), 0, st, wbase, w_st_slot, w_st_m, np, naux,
                       nslot, wq, idx, blk, jout);
}
void launch_jk_blocks(bool f64, const void* wbase, int64_t w_st_slot, int64_t w_st_m, int64_t np,
                      int64_t naux, int32_t nslot, int32_t wmax, const int32_t* wq, const int32_t* idx,
                      const void* blk, void* jout, hipStream_t st) {
  const int64_t tasks = (int64_t)nslot * naux;
  if (f64)
    jk_blocks_launch<double>(wmax, tasks, st, wbase, w_st_slot, w_st_m, np, naux, nslot, wq, idx, (const double*)blk,
                             (double*)jout);
  else
    jk_blocks_launch<float>(wmax, tasks, st, wbase, w_st_slot, w_st_m, np, naux, nslot, wq, idx, (const float*)blk,
                            (float*)jout);
}
size_t jk_block_bytes(bool f64, int64_t nslot, int64_t naux, int32_t wmax) {
  const int64_t jp = jk_pitch(wmax);
  return (size_t)(nslot * naux * jp * jp * 4) * (f64 ? 8 : 4);
}
void launch_jk_scatter(bool f64, const void* jblk, int64_t naux, int32_t nslot, int32_t wmax, int64_t npat,
                       const int32_t* pat_ij, const int32_t* pat_off, const int32_t* pat_q, int64_t np,
                       Prec prec, int64_t plane, void* jw_l, void* jw_s, void* jz_st, void* jz_sum_t,
                       int64_t out_st_slot, hipStream_t st) {
  if ((int64_t)nslot * npat == 0) return;     // no large part: J and K vanish
  dim3 grid(blocks((int64_t)nslot * npat));
  const int jp = jk_pitch(wmax);
  if (f64)
    hipLaunchKernelGGL((k_jk_scatter<double>), grid, dim3(256), 0, st, (const double*)jblk, naux, nslot,
                       npat, jp, pat_ij, pat_off, pat_q, np, prec, plane, jw_l, jw_s, jz_st, jz_sum_t,
                       out_st_slot);
  else
    hipLaunchKernelGGL((k_jk_scatter<float>), grid, dim3(256), 0, st, (const float*)jblk, naux, nslot,
                       npat, jp, pat_ij, pat_off, pat_q, np, prec, plane, jw_l, jw_s, jz_st, jz_sum_t,
                       out_st_slot);
}
void launch_trace_coef(const double* part, int64_t ntiles, int32_t nslot, double* coef, int mode,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_trace_coef, dim3((unsigned)nslot), dim3(256), 0, st, part, ntiles, nslot, coef, mode);
}
void launch_double_stats(const double* tr, const double* w, int64_t ntau, const double* es, int64_t ns, double gm,
                         double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_double_stats, dim3(1), dim3(256), 0, st, tr, w, ntau, es, ns, gm, out);
}
void launch_vec_sum(const void* xl, const void* xs, void* xt, int64_t count, Prec prec, int64_t plane,
                    int64_t mstride, hipStream_t st) {
  hipLaunchKernelGGL(k_vec_sum, dim3(blocks(count)), dim3(256), 0, st, xl, xs, xt, count, prec, plane, mstride);
}
void launch_accumulate(const Unit* units, int32_t nunit, const void* sig, bool f64, int64_t sig_st_slot,
                       int64_t n, int64_t np, double* sum, int32_t tau_lo, int32_t tau_hi, const void* mst,
                       Prec prec, int64_t m_st_slot, int64_t m_st_m, int64_t plane, const double* coef,
                       hipStream_t st) {
  int64_t total = (int64_t)(tau_hi - tau_lo) * n * (np / 4);
  hipLaunchKernelGGL(k_accumulate, dim3(blocks(total)), dim3(256), 0, st, units, nunit, sig, (int)f64,
                     sig_st_slot, n, np, sum, tau_lo, tau_hi, mst, prec, m_st_slot, m_st_m, plane, coef);
}
void launch_esamples(const Unit* units, int32_t nunit, const double* part, int64_t ntiles, int64_t s0,
                     int64_t ntau, double* es, const double* coef, hipStream_t st) {
  hipLaunchKernelGGL(k_esamples, dim3((unsigned)((nunit + 3) / 4)), dim3(256), 0, st, units, nunit, part, ntiles, s0,
                     ntau, es, coef);
}
void launch_finalize(const double* det, const double* sum, int64_t n, int64_t ntau, double inv2ns,
                     double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(blocks(ntau * n * n)), dim3(256), 0, st, det, sum, n, ntau, inv2ns, out);
}
void launch_level_correct(double* sum, const double* hi, const double* lo, int64_t count, double c,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_level_correct, dim3(blocks(count)), dim3(256), 0, st, sum, hi, lo, count, c);
}
void launch_level_shift(double* es, const double* hi, int64_t k, int64_t ns, int64_t ntau, hipStream_t st) {
  hipLaunchKernelGGL(k_level_shift, dim3(1), dim3(256), 0, st, es, hi, k, ns, ntau);
}
void launch_trace_prod(const double* sig, const double* gb, int64_t n, int64_t ntau, double* tr,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_trace_prod, dim3((unsigned)ntau), dim3(256), 0, st, sig, gb, n, tr);
}
void launch_energy_stats(const double* tr, const double* w, int64_t ntau, const double* es, int64_t ns,
                         double gm, double* out, hipStream_t st, bool add_mean) {
  hipLaunchKernelGGL(k_energy_stats, dim3(1), dim3(256), 0, st, tr, w, ntau, es, ns, gm, add_mean ? 1 : 0, out);
}
void launch_transpose(const void* src, bool f64, int64_t rows, int64_t cols, double* dst, int64_t ld,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_transpose, dim3(blocks(rows * cols)), dim3(256), 0, st, src, (int)f64, rows, cols, dst, ld);
}
void launch_untranspose(const double* src, int64_t rows, int64_t cols, int64_t ld, void* dst, bool f64,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_untranspose, dim3(blocks(rows * cols)), dim3(256), 0, st, src, rows, cols, ld, dst, (int)f64);
}
void launch_count_nonfinite(const double* x, int64_t count, unsigned long long* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_count_nonfinite, dim3(blocks(count)), dim3(256), 0, st, x, count, bad);
}
