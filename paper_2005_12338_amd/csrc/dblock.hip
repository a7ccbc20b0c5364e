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

// Add one chunk's blocks C_QQ' (cbuf, one W x W block per Q' of the chunk) to
// column j of the strip: every row a of S_Q at once, contributions in
// increasing Q' (the entries of column j with Q' in [c0, c0 + CH)).  One
// lane per column, so the strip is read and written along contiguous j.
template <int W, int CH>
__device__ __forceinline__ void add_column(const double* cbuf, const int32_t* col_q, const int32_t* col_cs,
                                           int32_t ncs, int64_t c0, int j, int w1, int64_t n, double* st) {
  const int32_t* cs = col_cs + (int64_t)j * ncs;
  const int c64 = (int)(c0 >> 6);
  const int lo = cs[c64], hi = cs[min(c64 + CH / 64, ncs - 1)];
  double acc[W];
#pragma unroll
  for (int a = 0; a < W; ++a) acc[a] = 0.0;
  for (int k = lo; k < hi; ++k) {
    const int32_t cq = col_q[k];
    const double* cb = cbuf + ((cq >> 5) - c0) * W * W + (cq & 31);
#pragma unroll
    for (int a = 0; a < W; ++a)
      if (a < w1) acc[a] += cb[a * W];
  }
#pragma unroll
  for (int a = 0; a < W; ++a)
    if (a < w1) st[(int64_t)a * n + j] += acc[a];
}

// ---------------------------------------------------------------------------
// Register form for supports of at most W orbitals.  One workgroup per
// (tau, Q) builds the strip P_Q[a][j] = sum_Q' sum_d [S_Q'(d) = j] C_QQ'[a][d]
// (rows S_Q, all columns): each lane evaluates one pair (Q, Q') with its
// W x W blocks in registers,
//   u = k_Q G[S_Q, S_Q'],  M = u k_Q',  T = M Gb[S_Q', S_Q],
//   C = 2 Tr(T) M - T M,
// and writes C to LDS; the chunk's contributions are then added to the
// strip column by column in increasing Q' (fixed order).  A second kernel
// sums the strips of every (Q, a) with S_Q(a) = i into row i of Sigma.
//
// With G and Gb symmetric, C_Q'Q = C_QQ'^T and Sigma[D,D] is symmetric, so
// only its upper triangle is formed: strip Q keeps the columns j >= min S_Q,
// and a pair whose S_Q' lies wholly below min S_Q (it touches no such
// column) is skipped, about half of all pairs.  The gather mirrors the rest.
// ---------------------------------------------------------------------------
template <int W, int CH>
__global__ __launch_bounds__(256) void k_dd_strip(const double* G, const double* Gb, int64_t n,
                                                  int64_t naux, int32_t tau0, const int32_t* wq,
                                                  const int32_t* idx, const double* blk,
                                                  const int32_t* col_q, const int32_t* col_cs,
                                                  int32_t ncs, double* strip) {
  __shared__ double cbuf[CH * W * W];
  __shared__ double kq[W * W];
  __shared__ int32_t span[2];
  const int tid = threadIdx.x;
  const int64_t q = blockIdx.x;
  const int64_t t = tau0 + blockIdx.y;
  const double* g = G + t * n * n;
  const double* gb = Gb + t * n * n;
  double* st = strip + ((int64_t)blockIdx.y * naux + q) * W * n;
  const int w1 = wq[q];
  const int32_t* s1 = idx + q * kWMax;
  for (int e = tid; e < W * W; e += blockDim.x) {
    const int a = e / W, b = e % W;
    kq[e] = (a < w1 && b < w1) ? blk[q * kWMax * kWMax + a * kWMax + b] : 0.0;
  }
  for (int64_t e = tid; e < (int64_t)W * n; e += blockDim.x) st[e] = 0.0;
  int sq[W];
#pragma unroll
  for (int a = 0; a < W; ++a) sq[a] = a < w1 ? s1[a] : 0;
  __syncthreads();
  if (w1 == 0) return;

  const int qlo = sq[0];                    // lowest orbital of S_Q
  for (int64_t c0 = 0; c0 < naux; c0 += CH) {
    const int64_t r = c0 + tid;
    // pairs whose S_Q' lies wholly below S_Q feed only the lower triangle
    const int w2r = (tid < CH && r < naux) ? wq[r] : 0;
    const bool act = w2r > 0 && idx[r * kWMax + w2r - 1] >= qlo;
    if (tid == 0) { span[0] = (int32_t)n; span[1] = -1; }
    __syncthreads();
    if (act) {
      const int w2 = w2r;
      const int32_t* s2 = idx + r * kWMax;
      int sr[W];
#pragma unroll
      for (int c = 0; c < W; ++c) sr[c] = c < w2 ? s2[c] : 0;
      if (w2 > 0) {
        atomicMin(&span[0], sr[0]);
        atomicMax(&span[1], sr[w2 - 1]);
      }
      // u = k_Q G[S_Q, S_Q']  (W x W)
      double u[W][W];
#pragma unroll
      for (int a = 0; a < W; ++a)
#pragma unroll
        for (int c = 0; c < W; ++c) u[a][c] = 0.0;
#pragma unroll
      for (int b = 0; b < W; ++b) {
        if (b >= w1) break;
#pragma unroll
        for (int c = 0; c < W; ++c) {
          const double gv = c < w2 ? g[(int64_t)sq[b] * n + sr[c]] : 0.0;
#pragma unroll
          for (int a = 0; a < W; ++a) u[a][c] += kq[a * W + b] * gv;
        }
      }
      // M = u k_Q'
      double m[W][W];
#pragma unroll
      for (int a = 0; a < W; ++a)
#pragma unroll
        for (int d = 0; d < W; ++d) m[a][d] = 0.0;
      const double* kr = blk + r * kWMax * kWMax;
#pragma unroll
      for (int c = 0; c < W; ++c) {
        double row[W];
#pragma unroll
        for (int d = 0; d < W; ++d) row[d] = kr[c * kWMax + d];   // zero padded beyond w2
#pragma unroll
        for (int a = 0; a < W; ++a)
#pragma unroll
          for (int d = 0; d < W; ++d) m[a][d] += u[a][c] * row[d];
      }
      // T = M Gb[S_Q', S_Q]
      double tt[W][W];
#pragma unroll
      for (int a = 0; a < W; ++a)
#pragma unroll
        for (int f = 0; f < W; ++f) tt[a][f] = 0.0;
#pragma unroll
      for (int d = 0; d < W; ++d) {
        double row[W];
#pragma unroll
        for (int f = 0; f < W; ++f) row[f] = (d < w2 && f < w1) ? gb[(int64_t)sr[d] * n + sq[f]] : 0.0;
#pragma unroll
        for (int a = 0; a < W; ++a)
#pragma unroll
          for (int f = 0; f < W; ++f) tt[a][f] += m[a][d] * row[f];
      }
      double tr = 0.0;
#pragma unroll
      for (int a = 0; a < W; ++a) tr += tt[a][a];
      double* cb = cbuf + tid * W * W;
#pragma unroll
      for (int a = 0; a < W; ++a)
#pragma unroll
        for (int d = 0; d < W; ++d) {
          double s = 0.0;
#pragma unroll
          for (int f = 0; f < W; ++f) s += tt[a][f] * m[f][d];
          cb[a * W + d] = 2.0 * tr * m[a][d] - s;
        }
    }
    __syncthreads();
    // add the chunk to the strip: output (a, j), contributions from the
    // chunk's Q' with S_Q'(d) = j in increasing Q'; only columns j >= qlo
    // (the upper triangle of every row of S_Q) are kept
    const int jlo = max(span[0], qlo), jhi = span[1];
    for (int j = jlo + tid; j <= jhi; j += blockDim.x) add_column<W, CH>(cbuf, col_q, col_cs, ncs, c0, j, w1, n, st);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Row-staged form of the same strip (G and Gb symmetric, as G(tau) is for a
// real symmetric F and S).  Pairs (Q, Q') are taken in chunks of CH
// consecutive Q'; the orbitals those supports touch form a column window
// [jlo, jhi] of at most kDdSpan columns.  The workgroup stages
//   u[a][j] = sum_b k_Q[a][b] G[S_Q(b)][j]   and   gq[f][j] = Gb[S_Q(f)][j]
// over the window in LDS, so that each lane's pair needs only its own k_Q'
// block from memory:
//   M = u[:, S_Q'] k_Q',  T = M Gb[S_Q', S_Q],  C = 2 Tr(T) M - T M.
// Sums run in the same order as the register form, so the two agree bitwise.
// ---------------------------------------------------------------------------
template <int W, int CH>
__global__ __launch_bounds__(CH) void k_dd_rows(const double* G, const double* Gb, int64_t n, int64_t naux,
                                                int32_t tau0, const int32_t* wq, const int32_t* idx,
                                                const double* blk, const int32_t* idx_t, const double* blk_t,
                                                const int32_t* col_q, const int32_t* col_cs, int32_t ncs,
                                                double* strip) {
  // one lane's C block in LDS: W x W, padded to an odd number of doubles so
  // that the lanes' writes spread over the banks
  constexpr int CS = W * W + 1;
  __shared__ double cbuf[CH * CS];
  __shared__ double uq[W * kDdSpan];
  __shared__ double gq[W * kDdSpan];
  __shared__ double kq[W * W];
  __shared__ int32_t span[2];
  const int tid = threadIdx.x;
  const int64_t q = blockIdx.x;
  const int64_t t = tau0 + blockIdx.y;
  const double* g = G + t * n * n;
  const double* gb = Gb + t * n * n;
  double* st = strip + ((int64_t)blockIdx.y * naux + q) * W * n;
  const int w1 = wq[q];
  const int32_t* s1 = idx + q * kWMax;
  for (int e = tid; e < W * W; e += CH) {
    const int a = e / W, b = e % W;
    kq[e] = (a < w1 && b < w1) ? blk[q * kWMax * kWMax + a * kWMax + b] : 0.0;
  }
  for (int64_t e = tid; e < (int64_t)W * n; e += CH) st[e] = 0.0;
  int sq[W];
#pragma unroll
  for (int a = 0; a < W; ++a) sq[a] = a < w1 ? s1[a] : 0;
  __syncthreads();
  if (w1 == 0) return;

  const int qlo = sq[0];                    // lowest orbital of S_Q
  // Every dependent global round trip of a chunk costs a memory latency, so
  // the loads whose addresses are known early are issued early: the next
  // chunk's supports during this chunk, and the column entries of the
  // accumulation before the pair products.
  int w2n;
  int srn[W];
  // the chunk's supports and blocks are read from the by-column tables
  // (element c of S_Q' at idx_t[c naux + Q'], block element (c, d) at
  // blk_t[(c kDdW + d) naux + Q']), so that a wave's loads are contiguous
  auto load_meta = [&](int64_t cc) {
    const int64_t rr = cc + tid;
    w2n = rr < naux ? wq[rr] : 0;
#pragma unroll
    for (int c = 0; c < W; ++c) srn[c] = rr < naux ? idx_t[c * naux + rr] : -1;
  };
  load_meta(0);
  constexpr int NJ = kDdSpan / CH;          // strip columns per lane and chunk
  constexpr int NPRE = NJ == 1 ? 24 : 8;    // column entries fetched ahead
  for (int64_t c0 = 0; c0 < naux; c0 += CH) {
    const int64_t r = c0 + tid;
    const int w2r = w2n;
    int sr[W];
    int hi2 = -1;                             // last orbital of S_Q' (ascending)
#pragma unroll
    for (int c = 0; c < W; ++c) {
      sr[c] = srn[c];
      if (c < w2r) hi2 = sr[c];
    }
    // pairs whose S_Q' lies wholly below S_Q feed only the lower triangle
    const bool act = w2r > 0 && hi2 >= qlo;
    const int w2 = act ? w2r : 0;
    if (tid == 0) { span[0] = (int32_t)n; span[1] = -1; }
    __syncthreads();
    if (w2 > 0) {
      atomicMin(&span[0], sr[0]);
      atomicMax(&span[1], hi2);
    }
    if (c0 + CH < naux) load_meta(c0 + CH);
    __syncthreads();
    const int jlo = span[0], jhi = span[1];
    if (jhi < jlo) {                          // no pair of this chunk is needed
      __syncthreads();                        // span is reset only after every lane read it
      continue;
    }
    // accumulation operands of this lane's strip columns j >= qlo (the upper
    // triangle of every row of S_Q): entry range of column j for this chunk
    const int jl = max(jlo, qlo);
    const int c64 = (int)(c0 >> 6);
    int klo[NJ], khi[NJ];
#pragma unroll
    for (int u = 0; u < NJ; ++u) {
      const int j = jl + tid + u * CH;
      klo[u] = khi[u] = 0;
      if (j <= jhi) {
        const int32_t* cs = col_cs + (int64_t)j * ncs;
        klo[u] = cs[c64];
        khi[u] = cs[min(c64 + CH / 64, ncs - 1)];
      }
    }
    // Loads whose addresses are known now go out with the staging loads, so
    // that the chunk waits on memory once before its products: the lane's
    // k_Q' block (zero padded beyond w2), and (one strip column per lane)
    // the strip values the chunk adds to.
    double kv[W][W];
    {
      const double* kr = blk_t + r;
#pragma unroll
      for (int c = 0; c < W; ++c)
#pragma unroll
        for (int d = 0; d < W; ++d) kv[c][d] = (act && c < w2) ? kr[(c * kDdW + d) * naux] : 0.0;
    }
    constexpr bool kEarlySt = NJ == 1;
    double sv[W];
    if constexpr (kEarlySt) {
      const int j = jl + tid;
#pragma unroll
      for (int a = 0; a < W; ++a) sv[a] = (j <= jhi && a < w1) ? st[(int64_t)a * n + j] : 0.0;
    }
    const int width = jhi - jlo + 1;          // <= kDdSpan (checked on the host)
    // each lane stages whole window columns: the rows S_Q of G and Gb are
    // read once per column, all loads issued before the sums
#pragma unroll
    for (int u = 0; u < NJ; ++u) {
      const int jj = tid + u * CH;
      if (jj >= width) break;
      const int64_t j = jlo + jj;
      double gv[W], gbv[W];
#pragma unroll
      for (int b = 0; b < W; ++b) {
        gv[b] = b < w1 ? g[(int64_t)sq[b] * n + j] : 0.0;
        gbv[b] = b < w1 ? gb[(int64_t)sq[b] * n + j] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < W; ++a) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < W; ++b)
          if (b < w1) s += kq[a * W + b] * gv[b];
        uq[a * kDdSpan + jj] = s;
        gq[a * kDdSpan + jj] = gbv[a];
      }
    }
    __syncthreads();
    if (act) {
      // M = u[:, S_Q'] k_Q'
      double m[W][W];
#pragma unroll
      for (int a = 0; a < W; ++a)
#pragma unroll
        for (int d = 0; d < W; ++d) m[a][d] = 0.0;
#pragma unroll
      for (int c = 0; c < W; ++c) {
        if (c >= w2) break;
        const int col = sr[c] - jlo;            // c < w2: inside the window
#pragma unroll
        for (int a = 0; a < W; ++a) {
          const double uv = uq[a * kDdSpan + col];
#pragma unroll
          for (int d = 0; d < W; ++d) m[a][d] += uv * kv[c][d];
        }
      }
      // T = M Gb[S_Q', S_Q]
      double tt[W][W];
#pragma unroll
      for (int a = 0; a < W; ++a)
#pragma unroll
        for (int f = 0; f < W; ++f) tt[a][f] = 0.0;
#pragma unroll
      for (int d = 0; d < W; ++d) {
        double row[W];
        const int col = d < w2 ? sr[d] - jlo : 0;
#pragma unroll
        for (int f = 0; f < W; ++f) row[f] = d < w2 ? gq[f * kDdSpan + col] : 0.0;
#pragma unroll
        for (int a = 0; a < W; ++a)
#pragma unroll
          for (int f = 0; f < W; ++f) tt[a][f] += m[a][d] * row[f];
      }
      double tr = 0.0;
#pragma unroll
      for (int a = 0; a < W; ++a) tr += tt[a][a];
      double* cb = cbuf + tid * CS;
#pragma unroll
      for (int a = 0; a < W; ++a)
#pragma unroll
        for (int d = 0; d < W; ++d) {
          double s = 0.0;
#pragma unroll
          for (int f = 0; f < W; ++f) s += tt[a][f] * m[f][d];
          cb[a * W + d] = 2.0 * tr * m[a][d] - s;
        }
    }
    // the first column entries, fetched before the barrier
    int cqa[NJ][NPRE];
#pragma unroll
    for (int u = 0; u < NJ; ++u)
#pragma unroll
      for (int x = 0; x < NPRE; ++x) cqa[u][x] = klo[u] + x < khi[u] ? col_q[klo[u] + x] : 0;
    __syncthreads();
    // add the chunk to the strip: output (a, j), contributions from the
    // chunk's Q' with S_Q'(d) = j in increasing Q'
#pragma unroll
    for (int u = 0; u < NJ; ++u) {
      const int j = jl + tid + u * CH;
      if (j > jhi) continue;
      const int* cq = cqa[u];
      double acc[W];
#pragma unroll
      for (int a = 0; a < W; ++a) acc[a] = 0.0;
#pragma unroll
      for (int x = 0; x < NPRE; ++x) {
        if (klo[u] + x >= khi[u]) break;
        const double* cb = cbuf + ((cq[x] >> 5) - c0) * CS + (cq[x] & 31);
#pragma unroll
        for (int a = 0; a < W; ++a)
          if (a < w1) acc[a] += cb[a * W];
      }
      for (int k = klo[u] + NPRE; k < khi[u]; ++k) {
        const int32_t c = col_q[k];
        const double* cb = cbuf + ((c >> 5) - c0) * CS + (c & 31);
#pragma unroll
        for (int a = 0; a < W; ++a)
          if (a < w1) acc[a] += cb[a * W];
      }
#pragma unroll
      for (int a = 0; a < W; ++a) {
        if (a >= w1) continue;
        if constexpr (kEarlySt) st[(int64_t)a * n + j] = sv[a] + acc[a];
        else st[(int64_t)a * n + j] += acc[a];
      }
    }
    __syncthreads();
  }
}

// Sigma[t][i][j] = sum over (Q, a) with S_Q(a) = i of strip[t][Q][a][j] for
// j >= i; the strips hold only the upper triangle, and Sigma[D,D] is
// symmetric, so an element below the diagonal takes its mirror's value.
// One workgroup per (tau, 32 x 32 tile pair (bi, bj), bi <= bj): the upper
// tile is summed along rows of the strips (coalesced in j) and written, and
// its transpose goes to the mirror tile through LDS (coalesced too).
template <int W>
__global__ __launch_bounds__(256) void k_dd_gather(const double* strip, int64_t n, int64_t naux, int32_t tau0,
                                                   int64_t nt, const int32_t* col_off, const int32_t* col_q,
                                                   double* out) {
  __shared__ double tile[32][33];
  const int64_t bi = blockIdx.x / nt, bj = blockIdx.x % nt, tb = blockIdx.y;
  if (bi > bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  double* o = out + (int64_t)(tau0 + tb) * n * n;
  const double* sbase = strip + tb * naux * W * n;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = ty + 8 * u;
    const int64_t i = bi * 32 + r, j = bj * 32 + tx;
    double acc = 0.0;
    if (i < n && j < n && j >= i) {
      for (int k = col_off[i]; k < col_off[i + 1]; ++k) {
        const int64_t q = col_q[k] >> 5;
        const int a = col_q[k] & 31;
        acc += sbase[(q * W + a) * n + j];
      }
    }
    tile[r][tx] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = ty + 8 * u;
    // upper tile (bi, bj): element (i, j); on the diagonal tile the part
    // below the diagonal is the transpose of the part above
    const int64_t i = bi * 32 + r, j = bj * 32 + tx;
    if (i < n && j < n) o[i * n + j] = (bi < bj || tx >= r) ? tile[r][tx] : tile[tx][r];
    // mirror tile (bj, bi): element (bj*32 + r, bi*32 + tx) = tile[tx][r]
    if (bi < bj) {
      const int64_t i2 = bj * 32 + r, j2 = bi * 32 + tx;
      if (i2 < n && j2 < n) o[i2 * n + j2] = tile[tx][r];
    }
  }
}

}  // namespace

int dblock_tile() { return TD; }

// By-column copies of the supports and blocks of width at most kDdW:
// idx_t[c naux + Q] = S_Q(c) (-1 beyond w_Q), blk_t[(c kDdW + d) naux + Q] =
// k_Q[c][d] (0 beyond w_Q).
__global__ void k_dd_tables(const int32_t* idx, const double* blk, int64_t naux, int32_t* idx_t, double* blk_t) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= naux * kDdW * kDdW) return;
  const int64_t q = e % naux;
  const int cd = (int)(e / naux), c = cd / kDdW, d = cd % kDdW;
  blk_t[e] = blk[q * kWMax * kWMax + c * kWMax + d];
  if (cd < kDdW) idx_t[e] = idx[q * kWMax + cd];
}

void launch_dd_tables(const int32_t* idx, const double* blk, int64_t naux, int32_t* idx_t, double* blk_t,
                      hipStream_t st) {
  const int64_t tot = naux * kDdW * kDdW;
  hipLaunchKernelGGL(k_dd_tables, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, idx, blk, naux, idx_t,
                     blk_t);
}

int64_t dd_strip_bytes(int64_t n, int64_t naux, int32_t wmax, int64_t ntau_batch) {
  const int W = wmax <= 4 ? 4 : wmax <= 6 ? 6 : 8;
  return ntau_batch * naux * W * n * (int64_t)sizeof(double);
}

bool launch_dd_strips(const double* G, const double* Gb, int64_t n, int64_t naux, int64_t ntau, int32_t wmax,
                      int32_t span128, const int32_t* wq, const int32_t* idx, const double* blk,
                      const int32_t* idx_t, const double* blk_t, const int32_t* col_off, const int32_t* col_q, const int32_t* col_cs, int32_t ncs,
                      double* strip, int64_t ntau_batch, double* out, hipStream_t st) {
  if (wmax > 8) return false;
  const bool rows = span128 <= kDdSpan;
  for (int64_t t0 = 0; t0 < ntau; t0 += ntau_batch) {
    const int32_t ntb = (int32_t)std::min<int64_t>(ntau_batch, ntau - t0);
    dim3 grid((unsigned)naux, (unsigned)ntb);
    const int64_t gnt = (n + 31) / 32;
    const dim3 ggrid((unsigned)(gnt * gnt), (unsigned)ntb);
    if (rows) {
      if (wmax <= 4)
        hipLaunchKernelGGL((k_dd_rows<4, 128>), grid, dim3(128), 0, st, G, Gb, n, naux, (int32_t)t0, wq, idx, blk,
                           idx_t, blk_t, col_q, col_cs, ncs, strip);
      else if (wmax <= 6)
        hipLaunchKernelGGL((k_dd_rows<6, 128>), grid, dim3(128), 0, st, G, Gb, n, naux, (int32_t)t0, wq, idx, blk,
                           idx_t, blk_t, col_q, col_cs, ncs, strip);
      else
        hipLaunchKernelGGL((k_dd_rows<8, 64>), grid, dim3(64), 0, st, G, Gb, n, naux, (int32_t)t0, wq, idx, blk,
                           idx_t, blk_t, col_q, col_cs, ncs, strip);
      GF2_HIP(hipGetLastError());
      const int W = wmax <= 4 ? 4 : wmax <= 6 ? 6 : 8;
      if (W == 4)
        hipLaunchKernelGGL((k_dd_gather<4>), ggrid, dim3(256), 0, st, strip, n, naux, (int32_t)t0, gnt, col_off,
                           col_q, out);
      else if (W == 6)
        hipLaunchKernelGGL((k_dd_gather<6>), ggrid, dim3(256), 0, st, strip, n, naux, (int32_t)t0, gnt, col_off,
                           col_q, out);
      else
        hipLaunchKernelGGL((k_dd_gather<8>), ggrid, dim3(256), 0, st, strip, n, naux, (int32_t)t0, gnt, col_off,
                           col_q, out);
    } else if (wmax <= 4) {
      hipLaunchKernelGGL((k_dd_strip<4, 256>), grid, dim3(256), 0, st, G, Gb, n, naux, (int32_t)t0, wq, idx, blk,
                         col_q, col_cs, ncs, strip);
      hipLaunchKernelGGL((k_dd_gather<4>), ggrid, dim3(256), 0, st, strip, n, naux, (int32_t)t0, gnt, col_off,
                           col_q, out);
    } else if (wmax <= 6) {
      hipLaunchKernelGGL((k_dd_strip<6, 256>), grid, dim3(256), 0, st, G, Gb, n, naux, (int32_t)t0, wq, idx, blk,
                         col_q, col_cs, ncs, strip);
      hipLaunchKernelGGL((k_dd_gather<6>), ggrid, dim3(256), 0, st, strip, n, naux, (int32_t)t0, gnt, col_off,
                           col_q, out);
    } else {
      hipLaunchKernelGGL((k_dd_strip<8, 128>), grid, dim3(256), 0, st, G, Gb, n, naux, (int32_t)t0, wq, idx, blk,
                         col_q, col_cs, ncs, strip);
      hipLaunchKernelGGL((k_dd_gather<8>), ggrid, dim3(256), 0, st, strip, n, naux, (int32_t)t0, gnt, col_off,
                           col_q, out);
    }
    GF2_HIP(hipGetLastError());
  }
  return true;
}

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
