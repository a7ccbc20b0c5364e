// Grouped MFMA GEMM for the dense N x N products of the RS-SRI chains.
//
// C = sum_s A_s B_s^T for every unit (tau, pair) of a launch, where every
// operand is an np x np row-major matrix (B is passed as B^T, so both
// operands stream rows with contiguous k).  A tile may also hold the four
// products A_a B_b (a, b in {0, 1}) of two A and two B matrices at the same
// output position, so that the epilogue can form sums of products (e.g.
// M_SL + M_SS) without re-reading them from memory.
//
// gfx950 matrix cores:
//   FP64   v_mfma_f64_16x16x4_f64     64 x 64 tile, 4 waves of 32 x 32
//   FP32   v_mfma_f32_32x32x2_f32     128 x 128 tile, 4 waves of 64 x 64
//   BF16   v_mfma_f32_32x32x16_bf16   128 x 128 tile, 4 waves of 64 x 64
//   BF16X3 three bf16 MFMAs per step (hi*hi + hi*lo + lo*hi)
// Operands are double-buffered through LDS (global -> registers -> LDS);
// the accumulators are staged through LDS for the epilogue so that stores
// are coalesced in both row-major and transposed layouts.
#include <type_traits>

#include "gf2_internal.hpp"

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

template <Prec P> struct Cfg;
template <> struct Cfg<Prec::F64> {
  using E = double; using Acc = double;
  static constexpr int BM = 64, BN = 64, BK = 16, PAD = 2, PLANES = 1;
  static constexpr int MT = 16, TM = 2, TN = 2;    // wave tile 32 x 32
};
template <> struct Cfg<Prec::F32> {
  using E = float; using Acc = float;
  static constexpr int BM = 128, BN = 128, BK = 32, PAD = 4, PLANES = 1;
  static constexpr int MT = 32, TM = 2, TN = 2;    // wave tile 64 x 64
};
template <> struct Cfg<Prec::BF16> {
  using E = bf16_t; using Acc = float;
  static constexpr int BM = 128, BN = 128, BK = 64, PAD = 8, PLANES = 1;
  static constexpr int MT = 32, TM = 2, TN = 2;
};
template <> struct Cfg<Prec::BF16X3> {
  using E = bf16_t; using Acc = float;
  static constexpr int BM = 128, BN = 128, BK = 32, PAD = 8, PLANES = 2;
  static constexpr int MT = 32, TM = 2, TN = 2;
};

constexpr int kThreads = 256;

__device__ __forceinline__ bf16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (bf16_t)0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ int64_t off(const OpRef& r, const Unit& u) {
  return (int64_t)u.tau * r.st_tau + (int64_t)u.s * r.st_s + (int64_t)u.slot * r.st_slot;
}
__device__ __forceinline__ int64_t off(const OutSpec& r, const Unit& u) {
  return (int64_t)u.tau * r.st_tau + (int64_t)u.s * r.st_s + (int64_t)u.slot * r.st_slot;
}

// Storage-format load of one element as the accumulator type.
template <Prec P>
__device__ __forceinline__ typename Cfg<P>::Acc load_st(const void* base, int64_t i, int64_t plane) {
  if constexpr (P == Prec::F64) return ((const double*)base)[i];
  else if constexpr (P == Prec::F32) return ((const float*)base)[i];
  else if constexpr (P == Prec::BF16) return bf2f(((const bf16_t*)base)[i]);
  else return bf2f(((const bf16_t*)base)[i]) + bf2f(((const bf16_t*)base)[i + plane]);
}

template <Prec P>
__device__ __forceinline__ void store_st(void* base, int64_t i, int64_t plane, typename Cfg<P>::Acc v) {
  if constexpr (P == Prec::F64) ((double*)base)[i] = v;
  else if constexpr (P == Prec::F32) ((float*)base)[i] = v;
  else if constexpr (P == Prec::BF16) ((bf16_t*)base)[i] = f2bf(v);
  else {
    bf16_t hi = f2bf(v);
    ((bf16_t*)base)[i] = hi;
    ((bf16_t*)base)[i + plane] = f2bf(v - bf2f(hi));
  }
}

template <Prec P>
__device__ __forceinline__ void store_out(const OutSpec& o, int64_t i, int64_t plane, typename Cfg<P>::Acc v) {
  if (o.type == 0) {
    if constexpr (P == Prec::F64) ((double*)o.base)[i] = v;
    else ((float*)o.base)[i] = v;
  } else {
    store_st<P>(o.base, i, plane, v);
  }
}

// Remap the linear workgroup id so that consecutive tiles of one problem
// land on the same XCD (workgroups are dispatched round-robin over 8 XCDs,
// each with its own L2).
__device__ __forceinline__ int64_t xcd_remap(int64_t wg, int64_t total) {
  const int64_t nx = 8;
  int64_t per = total / nx, rem = total % nx;
  int64_t xcd = wg % nx, idx = wg / nx;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

template <Prec P>
__global__ __launch_bounds__(kThreads) void gemm_kernel(GemmLaunch L) {
  using C = Cfg<P>;
  using E = typename C::E;
  using Acc = typename C::Acc;
  constexpr int BM = C::BM, BN = C::BN, BK = C::BK, PAD = C::PAD, PL = C::PLANES;
  constexpr int PITCH = BK + PAD;                         // elements per LDS row
  constexpr int VE = 16 / sizeof(E);                      // elements per 16 B vector
  constexpr int VPR = BK / VE;                            // vectors per tile row
  constexpr int AVEC = BM * VPR * PL;                     // vectors per A tile
  constexpr int BVEC = BN * VPR * PL;
  constexpr int AV = AVEC / kThreads, BV = BVEC / kThreads;
  static_assert(AVEC % kThreads == 0 && BVEC % kThreads == 0, "tile/threads");
  constexpr int TILE_A = PL * BM * PITCH, TILE_B = PL * BN * PITCH;
  constexpr int CPITCH = BN + 1;
  constexpr int LDS_AB = 2 * (TILE_A + TILE_B) * (int)sizeof(E);
  constexpr int LDS_C = BM * CPITCH * (int)sizeof(Acc);
  constexpr int LDS_BYTES = LDS_AB > LDS_C ? LDS_AB : LDS_C;
  __shared__ __attribute__((aligned(16))) unsigned char smem[LDS_BYTES];
  __shared__ double red[4 * kMaxHad];

  E* As = (E*)smem;                    // [2][PL][BM][PITCH]
  E* Bs = As + 2 * TILE_A;             // [2][PL][BN][PITCH]

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const int64_t total = (int64_t)gridDim.x * gridDim.y;
  const int64_t lin = xcd_remap((int64_t)blockIdx.y * gridDim.x + blockIdx.x, total);
  const int tile = (int)(lin % gridDim.x);
  const int py = (int)(lin / gridDim.x);
  const int ui = py / L.nprob, pi = py % L.nprob;
  const Prob& pb = L.probs[pi];
  const Unit u = L.units[ui];
  const int nA = pb.nA, nB = pb.nB;
  const int SM = BM / nA, SN = BN / nB;                  // sub-tile extent
  const int64_t mrows = L.m, ncols = L.nc, kk = L.k, ld = L.ld;
  const int tiles_n = (int)((ncols + SN - 1) / SN);
  const int tiles_m = (int)((mrows + SM - 1) / SM);
  const int tm = tile / tiles_n, tn = tile % tiles_n;
  if (tm >= tiles_m) return;
  const int64_t row0 = (int64_t)tm * SM, col0 = (int64_t)tn * SN;

  const int kps = (int)((kk + BK - 1) / BK);             // k tiles per segment
  const int ktiles = kps * pb.nseg;

  // -------- global -> register staging
  u32x4_t ra[AV], rb[BV];
  auto gload = [&](int kt) {
    const int seg = kt / kps;
    const int64_t k0 = (int64_t)(kt % kps) * BK;
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const int v = tid + i * kThreads;
      const int pl = v / (BM * VPR);
      const int vv = v % (BM * VPR);
      const int r = vv / VPR, kv = vv % VPR;
      const int sel = r / SM;
      const int64_t grow = row0 + (r % SM);
      const int64_t k = k0 + (int64_t)kv * VE;
      const OpRef& ar = pb.a[nA == 2 ? sel : seg];
      u32x4_t val = {0u, 0u, 0u, 0u};
      if (grow < mrows && k < kk) {
        const E* p = (const E*)ar.base + off(ar, u) + (int64_t)pl * L.plane + grow * ld + k;
        val = *(const u32x4_t*)p;
      }
      ra[i] = val;
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      const int v = tid + i * kThreads;
      const int pl = v / (BN * VPR);
      const int vv = v % (BN * VPR);
      const int r = vv / VPR, kv = vv % VPR;
      const int sel = r / SN;
      const int64_t gcol = col0 + (r % SN);
      const int64_t k = k0 + (int64_t)kv * VE;
      const OpRef& br = pb.b[nB == 2 ? sel : seg];
      u32x4_t val = {0u, 0u, 0u, 0u};
      if (gcol < ncols && k < kk) {
        const E* p = (const E*)br.base + off(br, u) + (int64_t)pl * L.plane + gcol * ld + k;
        val = *(const u32x4_t*)p;
      }
      rb[i] = val;
    }
  };
  auto sstore = [&](int buf) {
    E* a = As + buf * TILE_A;
    E* b = Bs + buf * TILE_B;
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const int v = tid + i * kThreads;
      const int pl = v / (BM * VPR);
      const int vv = v % (BM * VPR);
      const int r = vv / VPR, kv = vv % VPR;
      *(u32x4_t*)(a + pl * BM * PITCH + r * PITCH + kv * VE) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      const int v = tid + i * kThreads;
      const int pl = v / (BN * VPR);
      const int vv = v % (BN * VPR);
      const int r = vv / VPR, kv = vv % VPR;
      *(u32x4_t*)(b + pl * BN * PITCH + r * PITCH + kv * VE) = rb[i];
    }
  };

  // -------- accumulators
  constexpr int MT = C::MT, TM = C::TM, TN = C::TN;
  constexpr int WTM = MT * TM, WTN = MT * TN;             // wave tile
  constexpr int NACC = (P == Prec::F64) ? 4 : 16;
  using AccV = typename std::conditional<P == Prec::F64, f64x4_t, f32x16_t>::type;
  AccV acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < NACC; ++r) acc[i][j][r] = 0;

  auto compute = [&](int buf) {
    const E* a = As + buf * TILE_A;
    const E* b = Bs + buf * TILE_B;
    if constexpr (P == Prec::F64) {
      // lane group g = lane/16 owns k in [4g, 4g+4) of the 16-wide k tile
      const int lr = lane & 15, g = lane >> 4;
      double av[TM][4], bv[TN][4];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const double* p = a + (wm * WTM + i * MT + lr) * PITCH + g * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) av[i][q] = p[q];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const double* p = b + (wn * WTN + j * MT + lr) * PITCH + g * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) bv[j][q] = p[q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][q], bv[j][q], acc[i][j], 0, 0, 0);
    } else if constexpr (P == Prec::F32) {
      // lane group g = lane/32 owns k in [16g, 16g+16) of the 32-wide k tile
      const int lr = lane & 31, g = lane >> 5;
#pragma unroll
      for (int kq = 0; kq < 4; ++kq) {
        float av[TM][4], bv[TN][4];
#pragma unroll
        for (int i = 0; i < TM; ++i) {
          const float* p = a + (wm * WTM + i * MT + lr) * PITCH + g * 16 + kq * 4;
          float4 t = *(const float4*)p;
          av[i][0] = t.x; av[i][1] = t.y; av[i][2] = t.z; av[i][3] = t.w;
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const float* p = b + (wn * WTN + j * MT + lr) * PITCH + g * 16 + kq * 4;
          float4 t = *(const float4*)p;
          bv[j][0] = t.x; bv[j][1] = t.y; bv[j][2] = t.z; bv[j][3] = t.w;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i][q], bv[j][q], acc[i][j], 0, 0, 0);
      }
    } else {
      // lane group g = lane/32 owns k in [8g, 8g+8) of each 16-wide k step
      const int lr = lane & 31, g = lane >> 5;
#pragma unroll
      for (int ks = 0; ks < BK / 16; ++ks) {
        bf16x8_t ah[TM], bh[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          ah[i] = *(const bf16x8_t*)(a + (wm * WTM + i * MT + lr) * PITCH + ks * 16 + g * 8);
#pragma unroll
        for (int j = 0; j < TN; ++j)
          bh[j] = *(const bf16x8_t*)(b + (wn * WTN + j * MT + lr) * PITCH + ks * 16 + g * 8);
        if constexpr (P == Prec::BF16X3) {
          bf16x8_t al[TM], bl[TN];
#pragma unroll
          for (int i = 0; i < TM; ++i)
            al[i] = *(const bf16x8_t*)(a + BM * PITCH + (wm * WTM + i * MT + lr) * PITCH + ks * 16 + g * 8);
#pragma unroll
          for (int j = 0; j < TN; ++j)
            bl[j] = *(const bf16x8_t*)(b + BN * PITCH + (wn * WTN + j * MT + lr) * PITCH + ks * 16 + g * 8);
#pragma unroll
          for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
            }
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
    }
  };

  // -------- main loop (double-buffered)
  if (ktiles > 0) {
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < ktiles; ++kt) {
      const bool more = kt + 1 < ktiles;
      if (more) gload(kt + 1);
      compute(kt & 1);
      if (more) sstore((kt + 1) & 1);
      __syncthreads();
    }
  }

  // -------- stage accumulators through LDS
  Acc* Cs = (Acc*)smem;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < NACC; ++r) {
        int rr, cc;
        if constexpr (P == Prec::F64) {
          // f64 16x16x4: accumulator r of lane l holds row l/16 + 4r
          rr = (lane >> 4) + 4 * r;
          cc = lane & 15;
        } else {
          rr = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          cc = lane & 31;
        }
        Cs[(wm * WTM + i * MT + rr) * CPITCH + wn * WTN + j * MT + cc] = acc[i][j][r];
      }
  __syncthreads();

  // -------- epilogue
  const int np_ = nA * nB;
  Acc addc[kMaxAdd];
  const void* addp[kMaxAdd];
  for (int x = 0; x < pb.nadd; ++x) {
    addc[x] = (Acc)pb.add_coef[(int64_t)u.slot * kMaxAdd + x];
    addp[x] = (const char*)pb.add[x].base + off(pb.add[x], u) * (int64_t)sizeof(E);
  }
  auto vals_at = [&](int r, int c, Acc* v) {
    for (int a = 0; a < nA; ++a)
      for (int b = 0; b < nB; ++b) v[a * nB + b] = Cs[(a * SM + r) * CPITCH + b * SN + c];
    if (pb.nadd) {
      const int64_t gi = (row0 + r) * ld + col0 + c;
      for (int x = 0; x < pb.nadd; ++x) v[0] += addc[x] * load_st<P>(addp[x], gi, L.plane);
    }
  };
  double hsum[kMaxHad] = {0.0, 0.0, 0.0, 0.0};
  const double* hmat = pb.nhad ? (const double*)pb.had_h.base + off(pb.had_h, u) : nullptr;
  // row-major outputs, Hadamard sums
  for (int e = tid; e < SM * SN; e += kThreads) {
    const int r = e / SN, c = e % SN;
    const int64_t gr = row0 + r, gc = col0 + c;
    if (gr >= mrows || gc >= ncols) continue;
    Acc v[4];
    vals_at(r, c, v);
    for (int o = 0; o < pb.nout; ++o) {
      const OutSpec& os = pb.out[o];
      if (os.layout != 0) continue;
      Acc s = 0;
      for (int q = 0; q < np_; ++q) s += (Acc)os.coef[q] * v[q];
      store_out<P>(os, off(os, u) + gr * ld + gc, L.plane, s);
    }
    if (pb.nhad) {
      const double h = hmat[gr * ld + gc];
      for (int q = 0; q < pb.nhad; ++q) {
        double s = 0.0;
        for (int t = 0; t < np_; ++t) s += (double)pb.had_coef[q][t] * (double)v[t];
        hsum[q] += s * h;
      }
    }
  }
  // transposed outputs: consecutive threads walk down a column
  bool anyT = false;
  for (int o = 0; o < pb.nout; ++o) anyT |= pb.out[o].layout != 0;
  if (anyT) {
    for (int e = tid; e < SM * SN; e += kThreads) {
      const int r = e % SM, c = e / SM;
      const int64_t gr = row0 + r, gc = col0 + c;
      if (gr >= mrows || gc >= ncols) continue;
      Acc v[4];
      vals_at(r, c, v);
      for (int o = 0; o < pb.nout; ++o) {
        const OutSpec& os = pb.out[o];
        if (os.layout == 0) continue;
        Acc s = 0;
        for (int q = 0; q < np_; ++q) s += (Acc)os.coef[q] * v[q];
        store_out<P>(os, off(os, u) + gc * ld + gr, L.plane, s);
      }
    }
  }
  if (pb.nhad) {
    // deterministic block reduction: wave tree, then waves in order
    for (int q = 0; q < pb.nhad; ++q) {
      double s = hsum[q];
      for (int d = 32; d > 0; d >>= 1) s += __shfl_down(s, d, 64);
      if (lane == 0) red[wave * kMaxHad + q] = s;
    }
    __syncthreads();
    if (tid < pb.nhad) {
      double s = red[0 * kMaxHad + tid] + red[1 * kMaxHad + tid];
      s += red[2 * kMaxHad + tid];
      s += red[3 * kMaxHad + tid];
      pb.had_part[((int64_t)u.slot * pb.nhad + tid) * pb.had_ntiles + tile] = s;
    }
  }
}

}  // namespace

int gemm_tile_m(Prec p) {
  return p == Prec::F64 ? Cfg<Prec::F64>::BM : Cfg<Prec::F32>::BM;
}
int gemm_tile_n(Prec p) {
  return p == Prec::F64 ? Cfg<Prec::F64>::BN : Cfg<Prec::F32>::BN;
}

void launch_gemm(Prec p, const GemmLaunch& L, int max_tiles, hipStream_t st) {
  if (L.nunit <= 0 || L.nprob <= 0 || max_tiles <= 0) return;
  dim3 grid((unsigned)max_tiles, (unsigned)(L.nunit * L.nprob));
  switch (p) {
    case Prec::F64: hipLaunchKernelGGL(gemm_kernel<Prec::F64>, grid, dim3(kThreads), 0, st, L); break;
    case Prec::F32: hipLaunchKernelGGL(gemm_kernel<Prec::F32>, grid, dim3(kThreads), 0, st, L); break;
    case Prec::BF16: hipLaunchKernelGGL(gemm_kernel<Prec::BF16>, grid, dim3(kThreads), 0, st, L); break;
    case Prec::BF16X3: hipLaunchKernelGGL(gemm_kernel<Prec::BF16X3>, grid, dim3(kThreads), 0, st, L); break;
  }
  GF2_HIP(hipGetLastError());
}
