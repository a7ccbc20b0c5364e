// Kernels of the learned importance proposal (a project form on top of the
// paper's stochastic orbitals): per-Q features, per-Q contribution tables
// from the energy of eq:sigma, and a 4 -> 128 -> 1 network trained and
// evaluated on the device.  Every reduction runs in a fixed order.
#include "kernels.hpp"
#include "gf2_proposal.h"

namespace {

constexpr int HID = GF2_MLP_HIDDEN;
constexpr int DIN = GF2_MLP_IN;
constexpr int NPAR = HID * DIN + 2 * HID;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27; z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}
__device__ __forceinline__ double getb(const void* b, int64_t i, bool f64) {
  return f64 ? ((const double*)b)[i] : (double)((const float*)b)[i];
}
__device__ __forceinline__ float bfround(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// Block-wide fixed-order sum of one double per thread (256 threads).
__device__ double block_sum256(double v, double* sm) {
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) sm[threadIdx.x] += sm[threadIdx.x + d];
    __syncthreads();
  }
  double r = sm[0];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------ features ----
__global__ __launch_bounds__(256) void k_features(const void* b, int f64, int64_t n, int64_t naux, double thr,
                                                  const double* x, const double* xq, const double* gbeta,
                                                  double* phi) {
  __shared__ double sm[256];
  const int64_t q = blockIdx.x;
  const int64_t nn = n * n;
  double bb = 0.0, bs = 0.0, bp = 0.0;
  auto take = [&](double v, double g) {
    bb += v * v;
    if (fabs(v) < thr) bs += v * v;
    bp += v * g;
  };
  if (!f64 && nn % 4 == 0 && ((uintptr_t)b & 15) == 0) {
    // FP32 B: four elements per 16-byte load (B_Q starts 16-byte aligned)
    const float4* b4 = (const float4*)((const float*)b + q * nn);
    const int64_t n4 = nn / 4;
    for (int64_t e = threadIdx.x; e < n4; e += blockDim.x) {
      const float4 v = b4[e];
      const double* g = gbeta + 4 * e;
      take(v.x, g[0]);
      take(v.y, g[1]);
      take(v.z, g[2]);
      take(v.w, g[3]);
    }
  } else {
    for (int64_t e = threadIdx.x; e < nn; e += blockDim.x) take(getb(b, q * nn + e, f64), gbeta[e]);
  }
  bb = block_sum256(bb, sm);
  bs = block_sum256(bs, sm);
  bp = block_sum256(bp, sm);
  if (threadIdx.x == 0) {
    const double d = fmin(xq[q] - x[0], x[n - 1] - xq[q]);
    phi[q * 4 + 0] = tanh(d / 4.0);
    phi[q * 4 + 1] = log(sqrt(bb) + 1e-30);
    phi[q * 4 + 2] = log(sqrt(bs) + 1e-30);
    phi[q * 4 + 3] = -2.0 * bp;
  }
}

// ------------------------------------------------------------ pair tables -
// One wave per (combo, Q, R); lanes walk block elements.  For combo (x, y)
// with x, y in {B (truncated), K}: over tau, M = x_Q G[Sx, Sy] y_R,
// T = M Gb[Sy, Sx], accumulate w_t (2 Tr(T)^2 - Tr(T T)).
template <int W>
__global__ __launch_bounds__(64) void k_pair_tables(const double* G, const double* Gb, int64_t n, int64_t ntau,
                                                    const double* w, int64_t naux,
                                                    const int32_t* wb, const int32_t* ib, const double* bb,
                                                    const int32_t* wk, const int32_t* ik, const double* kb,
                                                    double* tab) {
  __shared__ double xs[W * W], ys[W * W], gx[W * W], gbx[W * W], m1[W * W], mm[W * W], tt[W * W];
  const int lane = threadIdx.x;
  const int64_t task = blockIdx.x;
  const int combo = (int)(task / (naux * naux));
  const int64_t q = (task / naux) % naux, r = task % naux;
  const bool xB = combo < 2, yB = (combo & 1) == 0;   // BB, BK, KB, KK
  const int wx = xB ? wb[q] : wk[q];
  const int wy = yB ? wb[r] : wk[r];
  const int32_t* sx = (xB ? ib : ik) + q * kWMax;
  const int32_t* sy = (yB ? ib : ik) + r * kWMax;
  const double* xblk = (xB ? bb : kb) + q * kWMax * kWMax;
  const double* yblk = (yB ? bb : kb) + r * kWMax * kWMax;
  double acc = 0.0;
  if (wx > 0 && wy > 0) {
    for (int e = lane; e < wx * wx; e += 64) xs[e] = xblk[(e / wx) * kWMax + e % wx];
    for (int e = lane; e < wy * wy; e += 64) ys[e] = yblk[(e / wy) * kWMax + e % wy];
    for (int64_t t = 0; t < ntau; ++t) {
      const double* g = G + t * n * n;
      const double* gb = Gb + t * n * n;
      __syncthreads();
      for (int e = lane; e < wx * wy; e += 64) {
        const int a = e / wy, c = e % wy;
        gx[e] = g[(int64_t)sx[a] * n + sy[c]];
        gbx[c * wx + a] = gb[(int64_t)sy[c] * n + sx[a]];
      }
      __syncthreads();
      for (int e = lane; e < wx * wy; e += 64) {           // m1 = G[Sx,Sy] y
        const int a = e / wy, d = e % wy;
        double s = 0.0;
        for (int c = 0; c < wy; ++c) s += gx[a * wy + c] * ys[c * wy + d];
        m1[e] = s;
      }
      __syncthreads();
      for (int e = lane; e < wx * wy; e += 64) {           // M = x m1
        const int a = e / wy, d = e % wy;
        double s = 0.0;
        for (int b = 0; b < wx; ++b) s += xs[a * wx + b] * m1[b * wy + d];
        mm[e] = s;
      }
      __syncthreads();
      double tr = 0.0;
      for (int e = lane; e < wx * wx; e += 64) {           // T = M Gb[Sy,Sx]
        const int a = e / wx, f = e % wx;
        double s = 0.0;
        for (int d = 0; d < wy; ++d) s += mm[a * wy + d] * gbx[d * wx + f];
        tt[e] = s;
        if (a == f) tr += s;
      }
      __syncthreads();
      double tr2 = 0.0;
      for (int e = lane; e < wx * wx; e += 64) {
        const int a = e / wx, f = e % wx;
        tr2 += tt[e] * tt[f * wx + a];
      }
      for (int d = 32; d > 0; d >>= 1) {
        tr += __shfl_xor(tr, d, 64);
        tr2 += __shfl_xor(tr2, d, 64);
      }
      acc += w[t] * (2.0 * tr * tr - tr2);
    }
  }
  if (lane == 0) tab[((int64_t)combo * naux + q) * naux + r] = acc;
}

__global__ void k_targets(const double* tab, int64_t naux, double* t) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= naux) return;
  const double* BB = tab;
  const double* BK = tab + naux * naux;
  const double* KB = tab + 2 * naux * naux;
  const double* KK = tab + 3 * naux * naux;
  double cl = 0.0, cr = 0.0, dsum = 0.0;
  for (int64_t r = 0; r < naux; ++r) {
    cl += KB[r * naux + q] - KK[r * naux + q];
    cr += BK[q * naux + r] - KK[q * naux + r];
    dsum += fabs(BB[q * naux + r] - BK[q * naux + r] - KB[q * naux + r] + KK[q * naux + r]);
  }
  t[q] = fabs(cl) + fabs(cr) + dsum;
}

// ------------------------------------------------------------ network -----
__global__ void k_mlp_init(const double* phi, int64_t ntotal, uint64_t seed, gf2_mlp m) {
  const int tid = threadIdx.x;
  if (tid < DIN) {
    double mu = 0.0;
    for (int64_t i = 0; i < ntotal; ++i) mu += phi[i * DIN + tid];
    mu /= (double)ntotal;
    double var = 0.0;
    for (int64_t i = 0; i < ntotal; ++i) {
      const double d = phi[i * DIN + tid] - mu;
      var += d * d;
    }
    double sd = sqrt(var / (double)ntotal);
    if (!(sd > 1e-12)) sd = 1.0;
    m.mean[tid] = (float)mu;
    m.std[tid] = (float)sd;
  }
  for (int p = tid; p < NPAR; p += blockDim.x) {
    // word(seed, 2, 0, p)
    const uint64_t ctr = (2ull << 62) | (uint64_t)p;
    const uint64_t wd = mix64(seed * 0x9E3779B97F4A7C15ull + ctr + 1ull);
    const double r = 2.0 * ((double)(wd >> 11) * 0x1.0p-53) - 1.0;
    if (p < HID * DIN) m.w1[p] = (float)(r / sqrt((double)DIN));
    else if (p < HID * DIN + HID) m.b1[p - HID * DIN] = (float)(r / sqrt((double)DIN));
    else m.w2[p - HID * DIN - HID] = (float)(r / sqrt((double)HID));
    m.adam_m[p] = 0.0f;
    m.adam_v[p] = 0.0f;
  }
}

__device__ __forceinline__ float mlp_param(const gf2_mlp& m, int p) {
  if (p < HID * DIN) return m.w1[p];
  if (p < HID * DIN + HID) return m.b1[p - HID * DIN];
  return m.w2[p - HID * DIN - HID];
}
__device__ __forceinline__ void mlp_set(gf2_mlp& m, int p, float v) {
  if (p < HID * DIN) m.w1[p] = v;
  else if (p < HID * DIN + HID) m.b1[p - HID * DIN] = v;
  else m.w2[p - HID * DIN - HID] = v;
}

// Full-batch loss/gradient and (optionally) Adam steps in one workgroup of
// 1024 threads.  z, dz: scratch [ntotal] float.  grad_out: [NPAR] double
// (last gradient), loss_out: [steps] (or [1] when steps == 0).
__global__ __launch_bounds__(1024) void k_mlp_train(gf2_mlp m, int32_t nchains, const int64_t* coff,
                                                    const double* phi, const double* that, int32_t steps,
                                                    float lr, int64_t step0, float* z, float* dz,
                                                    double* grad_out, double* loss_out) {
  __shared__ double lossc[1024];
  __shared__ double gsh[NPAR];
  const int tid = threadIdx.x;
  const int64_t ntotal = coff[nchains];
  const int nit = steps > 0 ? steps : 1;
  for (int it = 0; it < nit; ++it) {
    // forward: z_i
    for (int64_t i = tid; i < ntotal; i += blockDim.x) {
      float xs[DIN];
      for (int d = 0; d < DIN; ++d) xs[d] = ((float)phi[i * DIN + d] - m.mean[d]) / m.std[d];
      float zi = 0.0f;
      for (int k = 0; k < HID; ++k) {
        float a = m.b1[k];
        for (int d = 0; d < DIN; ++d) a += m.w1[k * DIN + d] * xs[d];
        zi += m.w2[k] * tanhf(a);
      }
      z[i] = zi;
    }
    __syncthreads();
    // per-chain softmax, loss and dL/dz
    for (int c = tid; c < nchains; c += blockDim.x) {
      const int64_t i0 = coff[c], i1 = coff[c + 1];
      double zmax = -1e300;
      for (int64_t i = i0; i < i1; ++i) zmax = fmax(zmax, (double)z[i]);
      double s = 0.0;
      for (int64_t i = i0; i < i1; ++i) s += exp((double)z[i] - zmax);
      const double ls = log(s);
      double l = 0.0;
      for (int64_t i = i0; i < i1; ++i) {
        const double lp = (double)z[i] - zmax - ls;
        const double th = that[i];
        if (th > 0) l += th * (log(th) - lp);
        dz[i] = (float)(exp(lp) - th);
      }
      lossc[c] = l;
    }
    __syncthreads();
    if (tid == 0) {
      double l = 0.0;
      for (int c = 0; c < nchains; ++c) l += lossc[c];
      loss_out[steps > 0 ? it : 0] = l;
    }
    // gradients: one thread per parameter, samples in order
    for (int p = tid; p < NPAR; p += blockDim.x) {
      int k, d = -1, kind;
      if (p < HID * DIN) { kind = 0; k = p / DIN; d = p % DIN; }
      else if (p < HID * DIN + HID) { kind = 1; k = p - HID * DIN; }
      else { kind = 2; k = p - HID * DIN - HID; }
      double g = 0.0;
      for (int64_t i = 0; i < ntotal; ++i) {
        float xs[DIN];
        for (int e = 0; e < DIN; ++e) xs[e] = ((float)phi[i * DIN + e] - m.mean[e]) / m.std[e];
        float a = m.b1[k];
        for (int e = 0; e < DIN; ++e) a += m.w1[k * DIN + e] * xs[e];
        const float h = tanhf(a);
        const double dzi = dz[i];
        if (kind == 2) g += dzi * h;
        else {
          const double ga = dzi * m.w2[k] * (1.0 - (double)h * h);
          g += kind == 1 ? ga : ga * xs[d];
        }
      }
      gsh[p] = g;
    }
    __syncthreads();
    if (steps > 0) {
      const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
      const double t = (double)(step0 + it + 1);
      for (int p = tid; p < NPAR; p += blockDim.x) {
        const double g = gsh[p];
        const double mo = b1 * m.adam_m[p] + (1.0 - b1) * g;
        const double vo = b2 * m.adam_v[p] + (1.0 - b2) * g * g;
        m.adam_m[p] = (float)mo;
        m.adam_v[p] = (float)vo;
        const double mh = mo / (1.0 - pow(b1, t));
        const double vh = vo / (1.0 - pow(b2, t));
        mlp_set(m, p, (float)(mlp_param(m, p) - lr * mh / (sqrt(vh) + eps)));
      }
    }
    __syncthreads();
  }
  for (int p = tid; p < NPAR; p += blockDim.x) grad_out[p] = gsh[p];
}

__global__ void k_mlp_logits(gf2_mlp m, const double* phi, int64_t naux, int bf16, float* z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= naux) return;
  float xs[DIN];
  for (int d = 0; d < DIN; ++d) {
    xs[d] = ((float)phi[i * DIN + d] - m.mean[d]) / m.std[d];
    if (bf16) xs[d] = bfround(xs[d]);
  }
  float zi = 0.0f;
  for (int k = 0; k < HID; ++k) {
    float a = bf16 ? bfround(m.b1[k]) : m.b1[k];
    for (int d = 0; d < DIN; ++d) a += (bf16 ? bfround(m.w1[k * DIN + d]) : m.w1[k * DIN + d]) * xs[d];
    float h = tanhf(a);
    if (bf16) h = bfround(h);
    zi += (bf16 ? bfround(m.w2[k]) : m.w2[k]) * h;
  }
  z[i] = zi;
}

__global__ __launch_bounds__(256) void k_softmax_mix(const float* z, int64_t naux, double alpha, double* p) {
  __shared__ double sm[256];
  double mx = -1e300;
  for (int64_t i = threadIdx.x; i < naux; i += blockDim.x) mx = fmax(mx, (double)z[i]);
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + d]);
    __syncthreads();
  }
  mx = sm[0];
  __syncthreads();
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < naux; i += blockDim.x) s += exp((double)z[i] - mx);
  s = block_sum256(s, sm);
  for (int64_t i = threadIdx.x; i < naux; i += blockDim.x)
    p[i] = (1.0 - alpha) * exp((double)z[i] - mx) / s + alpha / (double)naux;
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int mlp_nparam() { return NPAR; }

void launch_features(const void* b, bool f64, int64_t n, int64_t naux, double thr, const double* x,
                     const double* xq, const double* gbeta, double* phi, hipStream_t st) {
  hipLaunchKernelGGL(k_features, dim3((unsigned)naux), dim3(256), 0, st, b, (int)f64, n, naux, thr, x, xq, gbeta, phi);
}
void launch_pair_tables(int wmax, const double* G, const double* Gb, int64_t n, int64_t ntau, const double* w,
                        int64_t naux, const int32_t* wb, const int32_t* ib, const double* bb, const int32_t* wk,
                        const int32_t* ik, const double* kb, double* tab, hipStream_t st) {
  const int64_t tasks = 4 * naux * naux;
  if (wmax <= 16)
    hipLaunchKernelGGL((k_pair_tables<16>), dim3((unsigned)tasks), dim3(64), 0, st, G, Gb, n, ntau, w, naux, wb,
                       ib, bb, wk, ik, kb, tab);
  else
    hipLaunchKernelGGL((k_pair_tables<32>), dim3((unsigned)tasks), dim3(64), 0, st, G, Gb, n, ntau, w, naux, wb,
                       ib, bb, wk, ik, kb, tab);
}
void launch_targets(const double* tab, int64_t naux, double* t, hipStream_t st) {
  hipLaunchKernelGGL(k_targets, dim3(nblk(naux)), dim3(256), 0, st, tab, naux, t);
}
void launch_mlp_init(const double* phi, int64_t ntotal, uint64_t seed, const gf2_mlp& m, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_init, dim3(1), dim3(256), 0, st, phi, ntotal, seed, m);
}
void launch_mlp_train(const gf2_mlp& m, int32_t nchains, const int64_t* coff, const double* phi, const double* that,
                      int32_t steps, float lr, int64_t step0, float* z, float* dz, double* grad, double* loss,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(1024), 0, st, m, nchains, coff, phi, that, steps, lr, step0, z, dz,
                     grad, loss);
}
void launch_mlp_infer(const gf2_mlp& m, const double* phi, int64_t naux, int bf16, double alpha, float* z, double* p,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_logits, dim3(nblk(naux)), dim3(256), 0, st, m, phi, naux, bf16, z);
  hipLaunchKernelGGL(k_softmax_mix, dim3(1), dim3(256), 0, st, z, naux, alpha, p);
}
