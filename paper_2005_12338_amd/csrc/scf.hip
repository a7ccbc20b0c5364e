// Kernels of the self-consistent GF2 steps on either side of the self-energy
// (Section III): the tau -> i w quadrature of eq:GFT, the per-frequency Dyson
// inversion of eq:dyson, and the back-transform of eq:Ginverse with the
// non-interacting G0 of eq:G0 subtracted, plus the RI Fock build of eq:F.
//
// Everything runs in the orthonormal eigenbasis of (F, S) (C^T S C = I,
// C^T F C = diag(eps)): there G0(i w) is diagonal, the Dyson matrix is
//   A(i w) = diag(mu + i w - eps) - Sigma~(i w),  Sigma~ = C^T Sigma C,
// and N_e = -2 Tr G~(beta-).  Matrices are padded to np (a multiple of 32)
// with the identity on the padded diagonal, so the padded inverse is the
// inverse plus the identity block.  Complex matrices are planar: the real
// np x np plane, then the imaginary one.
//
// The inversion is blocked Gauss-Jordan without pivoting over 32-wide panels.
// A(i w) is complex symmetric with imaginary part w I - Im Sigma~(i w), which
// is positive definite for a self-energy with a positive spectral function
// (Im Sigma(i w) <= 0 for w > 0), so every leading block is invertible and
// elimination without pivoting is stable; a vanishing or non-finite pivot
// sets an error word that the host turns into GF2_E_NUMERIC.
#include "kernels.hpp"

namespace {

typedef double f64x4_t __attribute__((ext_vector_type(4)));

constexpr int kNB = 64;    // Gauss-Jordan panel width (a narrower last panel is handled too)
constexpr int kTW = 64;    // output tile width of the panel kernels
constexpr int kFG = 16;    // frequencies per thread in the forward transform
constexpr int kOG = 16;    // output times are padded to a multiple of this (the back-transform's MFMA rows)

// Blocks that share an element tile land on one XCD (blockIdx % 8 picks
// the XCD), one after the other: the tile's input stays in that XCD's L2.
__device__ __forceinline__ void xcd_split(unsigned b, int ng, int64_t& tile, int& g) {
  const unsigned xcd = b & 7u, r = b >> 3;
  g = (int)(r % (unsigned)ng);
  tile = (int64_t)(r / (unsigned)ng) * 8 + xcd;
}

// Workgroup b of a 1-D grid of `total` -> logical index, so that each XCD
// (workgroups are dispatched round-robin over the 8) runs one contiguous
// range of logical indices: with index = matrix * tiles + tile, whole
// matrices stay on one XCD and the panels a kernel writes for a matrix are
// read by the next kernel from the same L2.
__device__ __forceinline__ int64_t xcd_range(int64_t b, int64_t total) {
  const int64_t per = total / 8, rem = total % 8, xcd = b % 8, idx = b / 8;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// A(i w_f) for the frequencies of one chunk from Sigma~(tau_t) (padded,
// [ntau][np][np]): Sigma~(i w_f) = sum_t ph[t][f] Sigma~(tau_t) with
// ph[t][f] = w_t (cos, sin)(w_f tau_t).  shift[i] = mu - eps_i.
__global__ __launch_bounds__(256) void k_sig_iw(const double* __restrict__ sig, int64_t ntau, int64_t np,
                                                 int64_t n, const double* __restrict__ ph, int32_t nc, int32_t ncp,
                                                 const double* __restrict__ shift, const double* __restrict__ om,
                                                 double* __restrict__ a) {
  int64_t tile;
  int g;
  xcd_split(blockIdx.x, ncp / kFG, tile, g);
  const int64_t np2 = np * np;
  const int64_t e = tile * 256 + threadIdx.x;
  if (e >= np2) return;
  const int f0 = g * kFG;
  double sr[kFG], si[kFG];
#pragma unroll
  for (int f = 0; f < kFG; ++f) sr[f] = si[f] = 0.0;
  for (int64_t t = 0; t < ntau; ++t) {
    const double x = sig[t * np2 + e];
    const double* p = ph + (t * ncp + f0) * 2;
#pragma unroll
    for (int f = 0; f < kFG; ++f) {
      sr[f] = fma(p[2 * f], x, sr[f]);
      si[f] = fma(p[2 * f + 1], x, si[f]);
    }
  }
  const int64_t i = e / np, j = e - i * np;
#pragma unroll
  for (int f = 0; f < kFG; ++f) {
    const int fi = f0 + f;
    if (fi >= nc) break;
    double re = -sr[f], im = -si[f];
    if (i == j) {
      if (i < n) {
        re += shift[i];
        im += om[fi];
      } else {
        re = 1.0;
        im = 0.0;
      }
    }
    a[(int64_t)(2 * fi) * np2 + e] = re;
    a[(int64_t)(2 * fi + 1) * np2 + e] = im;
  }
}

__device__ __forceinline__ void cmul(double ar, double ai, double br, double bi, double& cr, double& ci) {
  cr = ar * br - ai * bi;
  ci = ar * bi + ai * br;
}

// Gauss-Jordan, panel k0 (columns K = [k0, k0 + 32), or fewer at the end), first step: one block
// per matrix inverts the diagonal block P = A_KK^{-1} in LDS (without
// pivoting: the Dyson matrices are complex symmetric with a positive
// definite imaginary part, so every leading block is invertible) and stores
// it in pbuf.  A vanishing or non-finite pivot sets *err.  Grid (matrices).
constexpr int kPivT = kNB == 64 ? 1024 : 256;   // threads of the pivot-block kernel
__global__ __launch_bounds__(kPivT) void k_gj_pivot(const double* a, int64_t np, int64_t k0, double* pbuf,
                                                    int* err) {
  __shared__ double dr[kNB][kNB + 1], di[kNB][kNB + 1];
  __shared__ double fr[kNB], fi[kNB];
  const int tid = threadIdx.x;
  const int64_t mat = xcd_range(blockIdx.x, gridDim.x), np2 = np * np;
  const double* ar = a + mat * 2 * np2;
  const double* ai = ar + np2;
  const int kb = (int)(np - k0 < kNB ? np - k0 : kNB);     // width of this panel
  // a narrower last panel is completed by the identity, so P = diag(A_KK^{-1}, I)
  for (int x = tid; x < kNB * kNB; x += kPivT) {
    const int r = x / kNB, c = x % kNB;
    const bool in = r < kb && c < kb;
    dr[r][c] = in ? ar[(k0 + r) * np + k0 + c] : (r == c ? 1.0 : 0.0);
    di[r][c] = in ? ai[(k0 + r) * np + k0 + c] : 0.0;
  }
  __syncthreads();
  for (int p = 0; p < kNB; ++p) {
    if (tid < kNB) {
      fr[tid] = dr[tid][p];
      fi[tid] = di[tid][p];
    }
    __syncthreads();
    const double pr = fr[p], pi = fi[p];
    const double den = pr * pr + pi * pi;
    if (tid == 0 && !(den >= 1e-280 && den <= 1e280)) atomicOr(err, 1);
    const double vr = pr / den, vi = -pi / den;   // 1 / pivot
    if (tid < kNB) {
      if (tid == p) {
        dr[p][tid] = vr;
        di[p][tid] = vi;
      } else {
        double xr, xi;
        cmul(dr[p][tid], di[p][tid], vr, vi, xr, xi);
        dr[p][tid] = xr;
        di[p][tid] = xi;
      }
    }
    __syncthreads();
    for (int x = tid; x < kNB * kNB; x += kPivT) {
      const int r = x / kNB, c = x % kNB;
      if (r == p) continue;
      double xr, xi;
      if (c == p) {
        cmul(fr[r], fi[r], vr, vi, xr, xi);
        dr[r][c] = -xr;
        di[r][c] = -xi;
      } else {
        cmul(fr[r], fi[r], dr[p][c], di[p][c], xr, xi);
        dr[r][c] -= xr;
        di[r][c] -= xi;
      }
    }
    __syncthreads();
  }
  double* pr_ = pbuf + mat * 2 * kNB * kNB;
  for (int x = tid; x < kNB * kNB; x += kPivT) {
    const int r = x / kNB, c = x % kNB;
    pr_[x] = dr[r][c];
    pr_[kNB * kNB + x] = di[r][c];
  }
}

// Second step: every block copies rows [64 ct, 64 ct + 64) of the column
// panel A_{:,K} to colbuf and replaces its 64 columns j (outside K) of the
// row panel by P A_Kj, with P from pbuf, on FP64 MFMAs (complex product as
// four real ones; each lane loads its operands from P and A_K directly).
// Every wave reads all of A_K's rows for its columns before any wave
// overwrites them: the new row panel is written after a barrier.
// 1-D grid of (matrix, column tile).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_gj_panel(double* a, int64_t np, int64_t k0, double* colbuf,
                                                  const double* pbuf) {
  constexpr int BI = kNB / 32;                  // 16-row MFMA blocks per wave (rows of P)
  const int tid = threadIdx.x;
  const int64_t tiles = (np + kTW - 1) / kTW, q = xcd_range(blockIdx.x, gridDim.x);
  const int64_t ct = q % tiles, mat = q / tiles, np2 = np * np;
  double* ar = a + mat * 2 * np2;
  double* ai = ar + np2;
  const int64_t j0 = (int64_t)ct * kTW;
  const int kb = (int)(np - k0 < kNB ? np - k0 : kNB);     // width of this panel
  const double* pr_ = pbuf + mat * 2 * kNB * kNB;
  const double* pi_ = pr_ + kNB * kNB;
  double* cbr = colbuf + mat * 2 * np * kNB;
  double* cbi = cbr + np * kNB;
  for (int x = tid; x < kTW * kNB; x += 256) {
    const int r = x / kNB, c = x % kNB;
    const int64_t i = j0 + r;
    if (i < np) {
      cbr[i * kNB + c] = c < kb ? ar[i * np + k0 + c] : 0.0;
      cbi[i * kNB + c] = c < kb ? ai[i * np + k0 + c] : 0.0;
    }
  }
  const int lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  const int lr = lane & 15, lg = lane >> 4;
  int64_t col[2];
  bool cok[2];
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    col[bj] = j0 + 32 * wc + 16 * bj + lr;
    cok[bj] = col[bj] < np && !(col[bj] >= k0 && col[bj] < k0 + kb);
  }
  f64x4_t accr[BI][2], acci[BI][2];
#pragma unroll
  for (int bi = 0; bi < BI; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) accr[bi][bj][r] = acci[bi][bj][r] = 0.0;
#pragma unroll 4
  for (int ks = 0; ks < kNB / 4; ++ks) {
    const int l = 4 * ks + lg;                 // panel index of this lane's operands
    double xr[BI], xi[BI], yr[2], yi[2], yn[2];
#pragma unroll
    for (int bi = 0; bi < BI; ++bi) {
      const int r = (kNB / 2) * wr + 16 * bi + lr;
      xr[bi] = pr_[r * kNB + l];
      xi[bi] = pi_[r * kNB + l];
    }
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const bool ok = cok[bj] && l < kb;
      yr[bj] = ok ? ar[(k0 + l) * np + col[bj]] : 0.0;
      yi[bj] = ok ? ai[(k0 + l) * np + col[bj]] : 0.0;
      yn[bj] = -yi[bj];
    }
#pragma unroll
    for (int bi = 0; bi < BI; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        accr[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[bi], yr[bj], accr[bi][bj], 0, 0, 0);
        accr[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi[bi], yn[bj], accr[bi][bj], 0, 0, 0);
        acci[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[bi], yi[bj], acci[bi][bj], 0, 0, 0);
        acci[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi[bi], yr[bj], acci[bi][bj], 0, 0, 0);
      }
  }
  __syncthreads();                              // every wave has read A_K before it is overwritten
#pragma unroll
  for (int bi = 0; bi < BI; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      if (!cok[bj]) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (kNB / 2) * wr + 16 * bi + lg + 4 * r;   // accumulator r: row lane / 16 + 4 r
        if (row >= kb) continue;
        ar[(k0 + row) * np + col[bj]] = accr[bi][bj][r];
        ai[(k0 + row) * np + col[bj]] = acci[bi][bj][r];
      }
    }
}

// Second half: every 64 x 64 tile outside the panel rows takes
//   A_ij <- (j in K ? 0 : A_ij) - sum_k C_ik R'_kj
// with C the column panel saved by the first half and R' the new row panel
// (P on the K columns), on FP64 MFMAs (complex product as four real ones);
// the (K, K) block takes P.  1-D grid of (matrix, row tile, column tile).
// Each lane loads its MFMA operands straight from the panels (which stay in
// L2: every tile of a matrix reads the same ones), so the kernel needs no
// LDS and enough workgroups stay resident to keep many tiles' loads in
// flight; the update is a stream over the matrices (8 flop per byte).
__global__ __launch_bounds__(256) void k_gj_update(double* a, int64_t np, int64_t k0, const double* colbuf,
                                                   const double* pbuf) {
  const int tid = threadIdx.x;
  const int64_t tiles = (np + kTW - 1) / kTW, q = xcd_range(blockIdx.x, gridDim.x);
  const int64_t mat = q / (tiles * tiles), t2 = q % (tiles * tiles);
  const int64_t j0 = (t2 % tiles) * kTW, i0 = (t2 / tiles) * kTW;
  const int64_t np2 = np * np;
  double* ar = a + mat * 2 * np2;
  double* ai = ar + np2;
  const double* cbr = colbuf + mat * 2 * np * kNB;
  const double* cbi = cbr + np * kNB;
  const double* pr_ = pbuf + mat * 2 * kNB * kNB;
  const double* pi_ = pr_ + kNB * kNB;
  const int lane = tid & 63, w = tid >> 6, wr = w >> 1, wc = w & 1;
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t k1 = np - k0 < kNB ? np : k0 + kNB;       // K = [k0, k1)
  // operand rows (column panel) and columns (row panel) of this lane
  int64_t crow[2], rcol[2];
  bool cok[2], rin[2], rok[2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) {
    crow[bi] = i0 + 32 * wr + 16 * bi + lr;
    cok[bi] = crow[bi] < np;
  }
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
    rcol[bj] = j0 + 32 * wc + 16 * bj + lr;
    rok[bj] = rcol[bj] < np;
    rin[bj] = rcol[bj] >= k0 && rcol[bj] < k1;
  }
  f64x4_t accr[2][2], acci[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) accr[bi][bj][r] = acci[bi][bj][r] = 0.0;
#pragma unroll
  for (int ks = 0; ks < kNB / 4; ++ks) {
    const int k = 4 * ks + lg;                  // panel index of this lane's operands
    double xr[2], xi[2], yr[2], yi[2], yn[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      xr[bi] = cok[bi] ? cbr[crow[bi] * kNB + k] : 0.0;
      xi[bi] = cok[bi] ? cbi[crow[bi] * kNB + k] : 0.0;
    }
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      double vr = 0.0, vi = 0.0;
      if (rok[bj] && k0 + k < k1) {
        if (rin[bj]) {
          vr = pr_[k * kNB + (rcol[bj] - k0)];
          vi = pi_[k * kNB + (rcol[bj] - k0)];
        } else {
          vr = ar[(k0 + k) * np + rcol[bj]];
          vi = ai[(k0 + k) * np + rcol[bj]];
        }
      }
      yr[bj] = vr;
      yi[bj] = vi;
      yn[bj] = -vi;
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        accr[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[bi], yr[bj], accr[bi][bj], 0, 0, 0);
        accr[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi[bi], yn[bj], accr[bi][bj], 0, 0, 0);
        acci[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(xr[bi], yi[bj], acci[bi][bj], 0, 0, 0);
        acci[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(xi[bi], yr[bj], acci[bi][bj], 0, 0, 0);
      }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + 32 * wr + 16 * bi + lg + 4 * r;
        const int64_t gj = j0 + 32 * wc + 16 * bj + lr;
        if (gi >= np || gj >= np) continue;
        const bool ki = gi >= k0 && gi < k1, kj = gj >= k0 && gj < k1;
        const int64_t o = gi * np + gj;
        if (ki) {
          if (kj) {
            ar[o] = pr_[(gi - k0) * kNB + (gj - k0)];
            ai[o] = pi_[(gi - k0) * kNB + (gj - k0)];
          }
          continue;
        }
        // the old value (zero on the K columns) is read only now, so that it
        // holds no registers during the MFMAs (more waves per SIMD hide the
        // load latency); accumulator r of a lane: row lane / 16 + 4 r,
        // column lane % 16
        const double ovr = kj ? 0.0 : ar[o], ovi = kj ? 0.0 : ai[o];
        ar[o] = ovr - accr[bi][bj][r];
        ai[o] = ovi - acci[bi][bj][r];
      }
}

// D(i w_f) = A^{-1} - G0~(i w_f) (G0~ = diag 1 / (mu - eps_i + i w_f), zero
// on the padding, where A^{-1} holds 1) accumulated into the back-transform
// sums
//   pc[o][e] += sum_f cs[f][o].cos Re D_f[e],  ps[o][e] += sum_f cs[f][o].sin Im D_f[e]
// (cs [nc][ntop][2]) as two products (output times x frequencies) x
// (frequencies x matrix elements) on FP64 MFMAs.  A block of 8 waves covers
// kBR output rows and 64 elements: waves 0-3 the cosine sums of 16 elements
// each, waves 4-7 the sine sums.  The phases of kBK frequencies at a time
// are staged in LDS and shared by the waves; every wave streams its
// elements of D once per row block, with the G0 correction applied to the
// diagonal as it is loaded.  Grid (element tiles, row blocks).
constexpr int kBRT = 10;             // 16-row MFMA tiles per row block
constexpr int kBR = 16 * kBRT;       // output rows per block
constexpr int kBK = 16;              // frequencies per LDS stage
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_iw_back(const double* __restrict__ a, int32_t nc, int64_t np, int64_t n,
                                                  const double* __restrict__ shift, const double* __restrict__ om,
                                                  const double* __restrict__ cs, int32_t nto, int32_t ntop,
                                                  double* __restrict__ pc, double* __restrict__ ps) {
  __shared__ double ph[2][kBK][kBR];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int part = w >> 2, cb = w & 3;               // part 0: cosine / Re, 1: sine / Im
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t np2 = np * np;
  const int64_t e = (int64_t)blockIdx.x * 64 + 16 * cb + lr;   // this lane's element (B operand column)
  const int o0 = blockIdx.y * kBR;
  const bool live = e < np2;
  const int64_t i = live ? e / np : 0, j = live ? e - i * np : 1;
  const bool dg = live && i == j && i < n, pad = live && i == j && i >= n;
  const double sh = dg ? shift[i] : 0.0;
  const double* src = a + (int64_t)part * np2 + (live ? e : 0);
  // operand of k step ks of the stage starting at frequency f0: D_f[e], f = f0 + 4 ks + lg
  auto bval = [&](int f) -> double {
    if (!live || f >= nc) return 0.0;
    double v = src[(int64_t)(2 * f) * np2];
    if (dg) {
      const double wf = om[f], den = sh * sh + wf * wf;
      v += part == 0 ? -sh / den : wf / den;
    } else if (pad && part == 0) {
      v -= 1.0;
    }
    return v;
  };
  f64x4_t acc[kBRT];
#pragma unroll
  for (int t = 0; t < kBRT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[t][r] = 0.0;
  double bn[kBK / 4];
#pragma unroll
  for (int ks = 0; ks < kBK / 4; ++ks) bn[ks] = bval(4 * ks + lg);
  for (int f0 = 0; f0 < nc; f0 += kBK) {
    __syncthreads();                                 // the previous stage's phases are consumed
    for (int x = tid; x < 2 * kBK * kBR; x += 512) {
      const int pp = x / (kBK * kBR), kk = (x / kBR) % kBK, o = x % kBR;
      const int f = f0 + kk, oo = o0 + o;
      ph[pp][kk][o] = f < nc && oo < ntop ? cs[((int64_t)f * ntop + oo) * 2 + pp] : 0.0;
    }
    double bc[kBK / 4];
#pragma unroll
    for (int ks = 0; ks < kBK / 4; ++ks) bc[ks] = bn[ks];
    if (f0 + kBK < nc) {
#pragma unroll
      for (int ks = 0; ks < kBK / 4; ++ks) bn[ks] = bval(f0 + kBK + 4 * ks + lg);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kBK / 4; ++ks)
#pragma unroll
      for (int t = 0; t < kBRT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ph[part][4 * ks + lg][16 * t + lr], bc[ks], acc[t], 0, 0, 0);
  }
  if (!live) return;
  double* out = part == 0 ? pc : ps;
#pragma unroll
  for (int t = 0; t < kBRT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = o0 + 16 * t + lg + 4 * r;        // accumulator r: row lane / 16 + 4 r, column lane % 16
      if (o < nto) out[(int64_t)o * np2 + e] += acc[t][r];
    }
}

// Per matrix f of a chunk: tr[2f] = sum_{i<n} Re D_ii(i w_f) and tr[2f + 1] =
// sum_{i<n} Re G0~_ii^2 - sum_{i,j<n} Re G_ij^2, the derivative of tr[2f]
// with respect to mu (dG/dmu = -G^2, G complex symmetric).  One block per
// matrix, a fixed reduction order.
__global__ __launch_bounds__(256) void k_iw_diag(const double* a, int64_t np, int64_t n, const double* shift,
                                                 const double* om, double* tr) {
  __shared__ double red[2][256];
  const int64_t f = blockIdx.x, np2 = np * np;
  const double* ar = a + f * 2 * np2;
  const double* ai = ar + np2;
  const double wf = om[f];
  double s = 0.0, d = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double sh = shift[i], den = sh * sh + wf * wf;
    s += ar[i * np + i] - sh / den;
    d += (sh * sh - wf * wf) / (den * den);
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = threadIdx.x; j < n; j += 256) {
      const double gr = ar[i * np + j], gi = ai[i * np + j];
      d -= gr * gr - gi * gi;
    }
  red[0][threadIdx.x] = s;
  red[1][threadIdx.x] = d;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tr[2 * f] = red[0][0];
    tr[2 * f + 1] = red[1][0];
  }
}

__device__ __forceinline__ double softplus_d(double x) { return fmax(x, 0.0) + log1p(exp(-fabs(x))); }

// G~ in the eigenbasis from the back-transform sums: for output time o
//   G~(tau_o)      = G0~(tau_o)      + (2/beta) (pc + ps)
//   G~(beta-tau_o) = G0~(beta-tau_o) - (2/beta) (pc - ps)
// with G0~ = -diag((1-f) e^{-e tau}) and -diag(f e^{e tau}) (e = eps - mu).
// out: [ntau] G, then [ntau] Gbar, then G(beta-) (o = ntau is tau = beta).
__global__ void k_g_mo(const double* pc, const double* ps, int64_t np, int64_t n, int64_t ntau,
                       const double* tau, const double* emu, double beta, double* out) {
  const int64_t np2 = np * np;
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= (ntau + 1) * np2) return;
  const int64_t o = x / np2, e = x - o * np2, i = e / np, j = e - i * np;
  const double c = 2.0 / beta, vc = pc[x], vs = ps[x];
  if (o == ntau) {
    double v = c * (vc + vs);
    if (i == j && i < n) v -= exp(-softplus_d(beta * emu[i]));
    out[2 * ntau * np2 + e] = v;
    return;
  }
  double g = c * (vc + vs), gb = -c * (vc - vs);
  if (i == j && i < n) {
    const double et = emu[i], t = tau[o];
    g -= exp(-et * t - softplus_d(-beta * et));
    gb -= exp(et * t - softplus_d(beta * et));
  }
  out[o * np2 + e] = g;
  out[(ntau + o) * np2 + e] = gb;
}

// ------------------------------------------------------ quasiparticles --

struct cplx {
  double r, i;
};
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.r - b.r, a.i - b.i}; }
__device__ __forceinline__ cplx cmulc(cplx a, cplx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cplx cdivc(cplx a, cplx b) {
  const double d = b.r * b.r + b.i * b.i;
  return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}

// Thiele continued fraction through (z_p, a_p), p < m, at z (the convergent
// recurrence A_p = A_{p-1} + (z - z_{p-1}) a_p A_{p-2}, B likewise).
__device__ cplx pade_at(const cplx* a, const double* om, int m, cplx z) {
  cplx am2 = {0.0, 0.0}, am1 = a[0], bm2 = {1.0, 0.0}, bm1 = {1.0, 0.0};
  for (int p = 1; p < m; ++p) {
    const cplx t = cmulc(cplx{z.r, z.i - om[p - 1]}, a[p]);
    const cplx an = cadd(am1, cmulc(t, am2)), bn = cadd(bm1, cmulc(t, bm2));
    am2 = am1;
    am1 = an;
    bm2 = bm1;
    bm1 = bn;
  }
  return cdivc(am1, bm1);
}

// One thread per orbital k: s_k(i w_f) = sum_t ph[t][f] Sigma~_kk(tau_t) for
// f < m, the Pade coefficients through (i w_f, s_k), and the fixed point of
// E = eps_k + Re C(E - mu + i eta) from E = eps_k, stopped at |dE| <= 1e-13.
// work: [n][2 m] complex.
__global__ void k_qp(const double* __restrict__ sig, int64_t ntau, int64_t np, int64_t n,
                     const double* __restrict__ ph, int32_t m, int32_t ncp, const double* __restrict__ om,
                     const double* __restrict__ eps, double mu, double eta, int32_t iters, cplx* work,
                     double* e_out, int32_t* conv) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  cplx* g = work + k * 2 * m;
  cplx* a = g + m;
  const int64_t np2 = np * np;
  for (int f = 0; f < m; ++f) g[f] = {0.0, 0.0};
  for (int64_t t = 0; t < ntau; ++t) {
    const double x = sig[t * np2 + k * np + k];
    for (int f = 0; f < m; ++f) {
      g[f].r = fma(ph[(t * ncp + f) * 2], x, g[f].r);
      g[f].i = fma(ph[(t * ncp + f) * 2 + 1], x, g[f].i);
    }
  }
  for (int p = 0; p < m; ++p) a[p] = {0.0, 0.0};
  a[0] = g[0];
  for (int p = 1; p < m; ++p) {
    if (a[p - 1].r == 0.0 && a[p - 1].i == 0.0) break;     // the fraction ends
    const cplx prev = g[p - 1];
    for (int f = p; f < m; ++f) g[f] = cdivc(csub(prev, g[f]), cmulc(cplx{0.0, om[f] - om[p - 1]}, g[f]));
    a[p] = g[p];
  }
  const double e0 = eps[k];
  double e = e0;
  int ok = 0;
  for (int it = 0; it < iters; ++it) {
    const double en = e0 + pade_at(a, om, m, cplx{e - mu, eta}).r;
    const bool done = fabs(en - e) <= 1e-13;
    e = en;
    if (done) {
      ok = 1;
      break;
    }
  }
  e_out[k] = e;
  conv[k] = ok;
}

// ----------------------------------------------------------------- Fock --

// Padded FP64 copies of B^Q for Q in [q0, q0 + qc) (zero for Q >= naux).
__global__ void k_pad_bq(const void* b, int f64, int64_t n, int64_t naux, int64_t np, int64_t q0, int64_t qc,
                         double* out) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= qc * np * np) return;
  const int64_t q = x / (np * np), e = x - q * np * np, i = e / np, j = e - i * np;
  double v = 0.0;
  if (i < n && j < n && q0 + q < naux) {
    const int64_t s = ((q0 + q) * n + i) * n + j;
    v = f64 ? ((const double*)b)[s] : (double)((const float*)b)[s];
  }
  out[x] = v;
}

// c_Q = Tr(B^Q P) = sum_ij B^Q_ij P_ij, one block per Q.
__global__ __launch_bounds__(256) void k_bq_dot(const void* b, int f64, int64_t n, const double* p, double* c) {
  __shared__ double red[256];
  const int64_t q = blockIdx.x, nn = n * n;
  double s = 0.0;
  if (f64) {
    const double* bq = (const double*)b + q * nn;
    for (int64_t e = threadIdx.x; e < nn; e += 256) s = fma(bq[e], p[e], s);
  } else {
    const float* bq = (const float*)b + q * nn;
    for (int64_t e = threadIdx.x; e < nn; e += 256) s = fma((double)bq[e], p[e], s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) c[q] = red[0];
}

// F = h + J - K/2 with J_ij = sum_Q c_Q B^Q_ij and K the sum of the padded
// partial products kp[g] (ng of them).
__global__ void k_fock_final(const void* b, int f64, int64_t n, int64_t naux, const double* c, const double* h,
                             const double* kp, int64_t ng, int64_t np, double* f) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = n * n;
  if (e >= nn) return;
  double jv = 0.0;
  if (f64) {
    const double* bb = (const double*)b;
    for (int64_t q = 0; q < naux; ++q) jv = fma(c[q], bb[q * nn + e], jv);
  } else {
    const float* bb = (const float*)b;
    for (int64_t q = 0; q < naux; ++q) jv = fma(c[q], (double)bb[q * nn + e], jv);
  }
  const int64_t i = e / n, j = e - i * n;
  double kv = 0.0;
  for (int64_t g = 0; g < ng; ++g) kv += kp[g * np * np + i * np + j];
  f[e] = h[e] + jv - 0.5 * kv;
}

// P = -2 G(beta-) (n x n).
__global__ void k_density(const double* gbeta, int64_t nn, double* p) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nn) p[e] = -2.0 * gbeta[e];
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int scf_freq_group() { return kFG; }
int scf_time_group() { return kOG; }
int scf_panel() { return kNB; }

void launch_sig_iw(const double* sig, int64_t ntau, int64_t np, int64_t n, const double* ph, int32_t nc, int32_t ncp,
                   const double* shift, const double* om, double* a, hipStream_t st) {
  const int64_t tiles = (np * np + 255) / 256;
  const unsigned grid = (unsigned)(((tiles + 7) / 8) * 8 * (ncp / kFG));
  hipLaunchKernelGGL(k_sig_iw, dim3(grid), dim3(256), 0, st, sig, ntau, np, n, ph, nc, ncp, shift, om, a);
}

void launch_gj_invert(double* a, int32_t nmat, int64_t np, double* colbuf, double* pbuf, int* err, hipStream_t st) {
  const unsigned tiles = (unsigned)((np + kTW - 1) / kTW);
  for (int64_t k0 = 0; k0 < np; k0 += kNB) {
    hipLaunchKernelGGL(k_gj_pivot, dim3((unsigned)nmat), dim3(kPivT), 0, st, (const double*)a, np, k0, pbuf, err);
    hipLaunchKernelGGL(k_gj_panel, dim3(tiles * (unsigned)nmat), dim3(256), 0, st, a, np, k0, colbuf,
                       (const double*)pbuf);
    hipLaunchKernelGGL(k_gj_update, dim3(tiles * tiles * (unsigned)nmat), dim3(256), 0, st, a, np, k0,
                       (const double*)colbuf, (const double*)pbuf);
  }
}

void launch_iw_back(const double* a, int32_t nc, int64_t np, int64_t n, const double* shift, const double* om,
                    const double* cs, int32_t nto, int32_t ntop, double* pc, double* ps, hipStream_t st) {
  const dim3 grid((unsigned)((np * np + 63) / 64), (unsigned)((ntop + kBR - 1) / kBR));
  hipLaunchKernelGGL(k_iw_back, grid, dim3(512), 0, st, a, nc, np, n, shift, om, cs, nto, ntop, pc, ps);
}

void launch_iw_diag(const double* a, int32_t nc, int64_t np, int64_t n, const double* shift, const double* om,
                    double* tr, hipStream_t st) {
  hipLaunchKernelGGL(k_iw_diag, dim3((unsigned)nc), dim3(256), 0, st, a, np, n, shift, om, tr);
}

void launch_g_mo(const double* pc, const double* ps, int64_t np, int64_t n, int64_t ntau, const double* tau,
                 const double* emu, double beta, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_g_mo, dim3(nblk((ntau + 1) * np * np)), dim3(256), 0, st, pc, ps, np, n, ntau, tau, emu, beta,
                     out);
}

void launch_pad_bq(const void* b, bool f64, int64_t n, int64_t naux, int64_t np, int64_t q0, int64_t qc, double* out,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_pad_bq, dim3(nblk(qc * np * np)), dim3(256), 0, st, b, (int)f64, n, naux, np, q0, qc, out);
}

void launch_bq_dot(const void* b, bool f64, int64_t n, int64_t naux, const double* p, double* c, hipStream_t st) {
  hipLaunchKernelGGL(k_bq_dot, dim3((unsigned)naux), dim3(256), 0, st, b, (int)f64, n, p, c);
}

void launch_fock_final(const void* b, bool f64, int64_t n, int64_t naux, const double* c, const double* h,
                       const double* kp, int64_t ng, int64_t np, double* f, hipStream_t st) {
  hipLaunchKernelGGL(k_fock_final, dim3(nblk(n * n)), dim3(256), 0, st, b, (int)f64, n, naux, c, h, kp, ng, np, f);
}

void launch_qp(const double* sig, int64_t ntau, int64_t np, int64_t n, const double* ph, int32_t m, int32_t ncp,
               const double* om, const double* eps, double mu, double eta, int32_t iters, void* work, double* e_out,
               int32_t* conv, hipStream_t st) {
  hipLaunchKernelGGL(k_qp, dim3(nblk(n, 64)), dim3(64), 0, st, sig, ntau, np, n, ph, m, ncp, om, eps, mu, eta, iters,
                     (cplx*)work, e_out, conv);
}

void launch_density(const double* gbeta, int64_t nn, double* p, hipStream_t st) {
  hipLaunchKernelGGL(k_density, dim3(nblk(nn)), dim3(256), 0, st, gbeta, nn, p);
}
