// Deterministic block Sigma[D, D] of eq:sigma_2 in FP64:
//
//   Sigma[D,D] = sum_{Q,Q'} 2 Tr(T) M - T M   on S_Q x S_Q',
//   M = k_Q G[S_Q, S_Q'] k_Q',  T = M Gbar[S_Q', S_Q],
//
// (the bilinear form of eq:sigma with K^L_Q (x) K^L_Q on both vertices,
// restricted to the supports).  Output-stationary: one workgroup per
// (tau, TD x TD output tile) visits every pair (Q, Q') whose supports touch
// the tile's rows and columns.  Each wave evaluates one pair at a time with
// its lanes on block elements and accumulates into its own LDS tile; the
// wave tiles are summed in a fixed order, so the result is deterministic.
#include "kernels.hpp"

namespace {

constexpr int TD = 32;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int WMX, int NW>
__global__ __launch_bounds__(64 * NW) void k_dblock(const double* G, const double* Gb, int64_t n,
                                                   int64_t np_unused, const int32_t* wq,
                                                   const int32_t* idx, const double* blk,
                                                   const int32_t* tq_off, const int32_t* tq,
                                                   int64_t ntile, double* out) {
  (void)np_unused;
  constexpr int W2 = WMX * WMX;
  __shared__ double acc[NW][TD * TD];
  __shared__ double sm[NW][7][W2];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t t = blockIdx.y;
  const int64_t bi = blockIdx.x / ntile, bj = blockIdx.x % ntile;
  const int64_t i0 = bi * TD, j0 = bj * TD;
  const double* g = G + t * n * n;
  const double* gb = Gb + t * n * n;

  for (int e = threadIdx.x; e < NW * TD * TD; e += 64 * NW) (&acc[0][0])[e] = 0.0;
  __syncthreads();

  double* kq = sm[wv][0];
  double* kr = sm[wv][1];
  double* gx = sm[wv][2];
  double* gbx = sm[wv][3];
  double* t1 = sm[wv][4];
  double* mm = sm[wv][5];
  double* tt = sm[wv][6];
  double* ac = acc[wv];

  const int32_t qa0 = tq_off[bi], qa1 = tq_off[bi + 1];
  const int32_t qb0 = tq_off[bj], qb1 = tq_off[bj + 1];
  const int64_t nb = qb1 - qb0;
  const int64_t npair = (int64_t)(qa1 - qa0) * nb;
  for (int64_t pr = wv; pr < npair; pr += NW) {
    const int q = tq[qa0 + pr / nb];
    const int r = tq[qb0 + pr % nb];
    const int w1 = wq[q], w2 = wq[r];
    const int32_t* s1 = idx + (int64_t)q * kWMax;
    const int32_t* s2 = idx + (int64_t)r * kWMax;
    for (int e = lane; e < w1 * w1; e += 64) kq[e] = blk[(int64_t)q * kWMax * kWMax + (e / w1) * kWMax + e % w1];
    for (int e = lane; e < w2 * w2; e += 64) kr[e] = blk[(int64_t)r * kWMax * kWMax + (e / w2) * kWMax + e % w2];
    for (int e = lane; e < w1 * w2; e += 64) {
      int a = e / w2, c = e % w2;
      gx[e] = g[(int64_t)s1[a] * n + s2[c]];             // G[S_Q, S_Q']   (w1 x w2)
      gbx[c * w1 + a] = gb[(int64_t)s2[c] * n + s1[a]];  // Gb[S_Q', S_Q]  (w2 x w1)
    }
    wave_sync();
    for (int e = lane; e < w1 * w2; e += 64) {            // t1 = G[S_Q,S_Q'] k_Q'
      int a = e / w2, d = e % w2;
      double s = 0.0;
      for (int c = 0; c < w2; ++c) s += gx[a * w2 + c] * kr[c * w2 + d];
      t1[e] = s;
    }
    wave_sync();
    for (int e = lane; e < w1 * w2; e += 64) {            // M = k_Q t1
      int a = e / w2, d = e % w2;
      double s = 0.0;
      for (int b = 0; b < w1; ++b) s += kq[a * w1 + b] * t1[b * w2 + d];
      mm[e] = s;
    }
    wave_sync();
    double trp = 0.0;
    for (int e = lane; e < w1 * w1; e += 64) {            // T = M Gb[S_Q', S_Q]
      int a = e / w1, f = e % w1;
      double s = 0.0;
      for (int d = 0; d < w2; ++d) s += mm[a * w2 + d] * gbx[d * w1 + f];
      tt[e] = s;
      if (a == f) trp += s;
    }
    for (int d = 32; d > 0; d >>= 1) trp += __shfl_xor(trp, d, 64);
    wave_sync();
    for (int e = lane; e < w1 * w2; e += 64) {            // C = 2 Tr(T) M - T M
      int a = e / w2, d = e % w2;
      int64_t gi = s1[a] - i0, gj = s2[d] - j0;
      if (gi < 0 || gi >= TD || gj < 0 || gj >= TD) continue;
      double s = 0.0;
      for (int f = 0; f < w1; ++f) s += tt[a * w1 + f] * mm[f * w2 + d];
      ac[gi * TD + gj] += 2.0 * trp * mm[e] - s;
    }
    wave_sync();
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TD * TD; e += 64 * NW) {
    int64_t gi = i0 + e / TD, gj = j0 + e % TD;
    if (gi >= n || gj >= n) continue;
    double s = acc[0][e];
    for (int w = 1; w < NW; ++w) s += acc[w][e];
    out[(t * n + gi) * n + gj] = s;
  }
}

}  // namespace

int dblock_tile() { return TD; }

void launch_dblock(const double* G, const double* Gb, int64_t n, int64_t ntau, int32_t wmax,
                   const int32_t* wq, const int32_t* idx, const double* blk, const int32_t* tq_off,
                   const int32_t* tq, double* out, hipStream_t st) {
  const int64_t ntile = (n + TD - 1) / TD;
  dim3 grid((unsigned)(ntile * ntile), (unsigned)ntau);
  if (wmax <= 8)
    hipLaunchKernelGGL((k_dblock<8, 4>), grid, dim3(256), 0, st, G, Gb, n, (int64_t)0, wq, idx, blk,
                       tq_off, tq, ntile, out);
  else if (wmax <= 16)
    hipLaunchKernelGGL((k_dblock<16, 2>), grid, dim3(128), 0, st, G, Gb, n, (int64_t)0, wq, idx, blk,
                       tq_off, tq, ntile, out);
  else
    hipLaunchKernelGGL((k_dblock<32, 1>), grid, dim3(64), 0, st, G, Gb, n, (int64_t)0, wq, idx, blk,
                       tq_off, tq, ntile, out);
  GF2_HIP(hipGetLastError());
}
