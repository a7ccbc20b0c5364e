// Grouped MFMA GEMM for the dense N x N products of the RS-SRI chains.
//
// C = sum_s A_s B_s^T for every unit (tau, pair) of a launch, where every
// operand is a row-major matrix with leading dimension ld (B is passed as
// B^T, so both operands stream rows with contiguous k).  A tile may also
// hold the products A_a B_b of two A and/or two B matrices at the same
// output positions; each wave then owns the same positions of every product,
// so sums of products (e.g. M_SL + M_SS) are formed in registers.
//
// gfx950 matrix cores:
//   FP64   v_mfma_f64_16x16x4_f64     64 x 64 tile, 4 waves
//   FP32   v_mfma_f32_32x32x2_f32     128 x 128 tile, 4 waves
//   BF16   v_mfma_f32_32x32x16_bf16   128 x 128 tile, 4 waves
//   BF16X3 three bf16 MFMAs per step (hi*hi + hi*lo + lo*hi)
//   BF16, wide tile (W = 1, single-product problems):
//          v_mfma_f32_16x16x32_bf16   160 x 160 tile, 4 waves of 80 x 80;
//          160 divides N = 800 and 400, where 128 pads by 12%.  Its LDS rows
//          are unpadded and XOR-swizzled (16-byte chunk c of row r stored at
//          c ^ (r mod 8)), so two workgroups fit the 160 KB of a CU.
// Operands are double-buffered through LDS (global -> registers -> LDS).
// The epilogue writes straight from the accumulators: combinations of the
// tile's products, row-major or transposed, in accumulator or storage
// format, optional addends and FP64 Hadamard partial sums (deterministic
// fixed-order block reduction).
#include <type_traits>

#include "gf2_internal.hpp"

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
// 16-byte vector in the global address space (global_load, not flat_load)
typedef __attribute__((address_space(1))) const u32x4_t GVec;

template <Prec P, int W = 0> struct Cfg;
// BM x BN block tile, 2 x 2 waves, each TM x TN MFMA tiles of MT x MT.
// SWZ: unpadded XOR-swizzled LDS rows; PF: k tiles in flight in registers
// (0: none, the operands go straight from global memory to LDS).
template <> struct Cfg<Prec::F64> {
  using E = double; using Acc = double;
  static constexpr int BM = 64, BN = 64, BK = 16, PAD = 2, PLANES = 1;
  static constexpr int MT = 16, NACC = 4, TM = 2, TN = 2;
  static constexpr bool SWZ = false; static constexpr int PF = 2;
};
template <> struct Cfg<Prec::F32> {
  using E = float; using Acc = float;
  static constexpr int BM = 128, BN = 128, BK = 32, PAD = 4, PLANES = 1;
  static constexpr int MT = 32, NACC = 16, TM = 2, TN = 2;
  static constexpr bool SWZ = false; static constexpr int PF = 2;
};
template <> struct Cfg<Prec::BF16> {
  using E = bf16_t; using Acc = float;
  static constexpr int BM = 128, BN = 128, BK = 64, PAD = 8, PLANES = 1;
  static constexpr int MT = 32, NACC = 16, TM = 2, TN = 2;
  static constexpr bool SWZ = false; static constexpr int PF = 2;
};
template <> struct Cfg<Prec::BF16X3> {
  using E = bf16_t; using Acc = float;
  static constexpr int BM = 128, BN = 128, BK = 32, PAD = 8, PLANES = 2;
  static constexpr int MT = 32, NACC = 16, TM = 2, TN = 2;
  static constexpr bool SWZ = false; static constexpr int PF = 2;
};
template <> struct Cfg<Prec::BF16, 1> {
  using E = bf16_t; using Acc = float;
  static constexpr int BM = 160, BN = 160, BK = 64, PAD = 0, PLANES = 1;
  static constexpr int MT = 16, NACC = 4, TM = 5, TN = 5;
  static constexpr bool SWZ = true; static constexpr int PF = 0;   // PF 0: direct global -> LDS loads
  static constexpr int STAGES = 2;
};
// 160-wide tiles with 32-wide k tiles (half the LDS per stage, so three
// stages fit two workgroups per CU): single products (W = 2), and dual-A
// products (W = 3: A_0 rows in [0, 160), A_1 rows in [160, 320), both times
// the same B tile; every wave owns the same 80 x 80 positions of both).
template <> struct Cfg<Prec::BF16, 2> {
  using E = bf16_t; using Acc = float;
  static constexpr int BM = 160, BN = 160, BK = 32, PAD = 0, PLANES = 1;
  static constexpr int MT = 16, NACC = 4, TM = 5, TN = 5;
  static constexpr bool SWZ = true; static constexpr int PF = 0;
  static constexpr int STAGES = 3;
};
template <> struct Cfg<Prec::BF16, 3> {
  using E = bf16_t; using Acc = float;
  static constexpr int BM = 320, BN = 160, BK = 32, PAD = 0, PLANES = 1;
  static constexpr int MT = 16, NACC = 4, TM = 10, TN = 5;
  static constexpr bool SWZ = true; static constexpr int PF = 0;
  static constexpr int STAGES = 3;
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
  return (int64_t)u.tau * r.st_tau + (int64_t)u.s * r.st_s + (int64_t)u.s2 * r.st_s2 + (int64_t)u.slot * r.st_slot;
}
__device__ __forceinline__ int64_t off(const OutSpec& r, const Unit& u) {
  return (int64_t)u.tau * r.st_tau + (int64_t)u.s * r.st_s + (int64_t)u.slot * r.st_slot;
}

template <Prec P>
__device__ __forceinline__ typename Cfg<P>::Acc load_st(const void* base, int64_t i, int64_t plane) {
  if constexpr (P == Prec::F64) return ((const double*)base)[i];
  else if constexpr (P == Prec::F32) return ((const float*)base)[i];
  else if constexpr (P == Prec::BF16) return bf2f(((const bf16_t*)base)[i]);
  else return bf2f(((const bf16_t*)base)[i]) + bf2f(((const bf16_t*)base)[i + plane]);
}

template <Prec P>
__device__ __forceinline__ void store_out(int type, void* base, int64_t i, int64_t plane,
                                          typename Cfg<P>::Acc v) {
  if constexpr (P == Prec::F64) {
    ((double*)base)[i] = v;
  } else if constexpr (P == Prec::F32) {
    ((float*)base)[i] = v;
  } else {
    if (type == 0) {
      ((float*)base)[i] = v;
    } else if constexpr (P == Prec::BF16) {
      ((bf16_t*)base)[i] = f2bf(v);
    } else {
      bf16_t hi = f2bf(v);
      ((bf16_t*)base)[i] = hi;
      ((bf16_t*)base)[i + plane] = f2bf(v - bf2f(hi));
    }
  }
}

// Four consecutive elements (i .. i+3) of one output row.
template <Prec P>
__device__ __forceinline__ void store_out_vec4(int type, void* base, int64_t i, int64_t plane,
                                               const typename Cfg<P>::Acc* v) {
  if constexpr (P == Prec::F64) {
    for (int e = 0; e < 4; ++e) ((double*)base)[i + e] = v[e];
  } else {
    if (type == 0 || P == Prec::F32) {
      if ((i & 3) == 0) {
        *(float4*)((float*)base + i) = make_float4(v[0], v[1], v[2], v[3]);
      } else {
        for (int e = 0; e < 4; ++e) ((float*)base)[i + e] = v[e];
      }
    } else {
      bf16_t h[4], l[4];
      for (int e = 0; e < 4; ++e) {
        h[e] = f2bf(v[e]);
        l[e] = f2bf(v[e] - bf2f(h[e]));
      }
      uint2 hv = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16));
      if ((i & 3) == 0) {
        *(uint2*)((bf16_t*)base + i) = hv;
      } else {
        for (int e = 0; e < 4; ++e) ((bf16_t*)base)[i + e] = h[e];
      }
      if constexpr (P == Prec::BF16X3) {
        uint2 lv = make_uint2((uint32_t)l[0] | ((uint32_t)l[1] << 16), (uint32_t)l[2] | ((uint32_t)l[3] << 16));
        if (((i + plane) & 3) == 0) {
          *(uint2*)((bf16_t*)base + i + plane) = lv;
        } else {
          for (int e = 0; e < 4; ++e) ((bf16_t*)base)[i + plane + e] = l[e];
        }
      }
    }
  }
}

// Wait until at most N vector-memory operations of this wave are outstanding.
template <int N> __device__ __forceinline__ void waitcnt_vm() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Sixteen zero bytes: the source of every out-of-range operand vector.
__device__ __attribute__((aligned(16))) const u32x4_t kZeroVec = {0u, 0u, 0u, 0u};

// Remap the linear workgroup id so that consecutive tiles of one problem
// land on the same XCD (workgroups are dispatched round-robin over 8 XCDs,
// each with its own L2).
__device__ __forceinline__ int64_t xcd_remap(int64_t wg, int64_t total) {
  const int64_t nx = 8;
  int64_t per = total / nx, rem = total % nx;
  int64_t xcd = wg % nx, idx = wg / nx;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Direct global -> LDS loads: one instruction fills 1 KB per wave, i.e.
// 1024 / (2 BK) rows; a workgroup round covers four times that many, and
// tiles are padded (in LDS only) to whole rounds.
template <int BK> constexpr int direct_rows() { return 8 * 64 / BK; }
template <int R, int BK> constexpr int direct_pad(int rows) {
  return (rows + 4 * direct_rows<BK>() - 1) / (4 * direct_rows<BK>()) * (4 * direct_rows<BK>());
}
template <Prec P, int W> struct Stages { static constexpr int N = 2; };
template <> struct Stages<Prec::BF16, 1> { static constexpr int N = Cfg<Prec::BF16, 1>::STAGES; };
template <> struct Stages<Prec::BF16, 2> { static constexpr int N = Cfg<Prec::BF16, 2>::STAGES; };
template <> struct Stages<Prec::BF16, 3> { static constexpr int N = Cfg<Prec::BF16, 3>::STAGES; };

template <Prec P, int W = 0>
struct Smem {
  using C = Cfg<P, W>;
  using E = typename C::E;
  static constexpr int PITCH = C::BK + C::PAD;
  static constexpr int ROWS_A = C::PF == 0 ? direct_pad<0, C::BK>(C::BM) : C::BM;
  static constexpr int ROWS_B = C::PF == 0 ? direct_pad<0, C::BK>(C::BN) : C::BN;
  static constexpr int TILE_A = C::PLANES * ROWS_A * PITCH;
  static constexpr int TILE_B = C::PLANES * ROWS_B * PITCH;
  static constexpr int STAGES = Stages<P, W>::N;
  static constexpr int BYTES = STAGES * (TILE_A + TILE_B) * (int)sizeof(E);
};

// Row (within the 32 x 32 or 16 x 16 MFMA tile) held by accumulator r of a lane.
template <Prec P, int MT>
__device__ __forceinline__ int acc_row(int lane, int r) {
  if constexpr (P == Prec::F64) return (lane >> 4) + 4 * r;       // f64 16x16x4
  else if constexpr (MT == 16) return 4 * (lane >> 4) + r;        // f32 16x16x32 bf16
  else return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);           // 32x32 f32 / bf16
}
template <Prec P, int MT>
__device__ __forceinline__ int acc_col(int lane) {
  if constexpr (P == Prec::F64 || MT == 16) return lane & 15;
  else return lane & 31;
}

// LDS byte address of a pointer into a __shared__ array.
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// Fragments of one 32-wide k step of the 160-wide tiles: TN = 5 B fragments
// at bbase + j * STEP and TM = 5 (or 10: two products) A fragments at abase
// + (i / FR) * PROD + (i % FR) * STEP, read back to back with one wait at
// the end of the same asm block.
template <int TM, int FR, int PROD, int STEP>
__device__ __forceinline__ void lds_frags(bf16x8_t* ah, bf16x8_t* bh, uint32_t abase, uint32_t bbase) {
  static_assert(TM == 5 || TM == 10, "fragment count");
  static_assert((TM / FR - 1) * PROD + (FR - 1) * STEP < 65536 && 4 * STEP < 65536, "ds offsets");
  if constexpr (TM == 5) {
    asm volatile(
        "ds_read_b128 %0, %10 offset:%c12\n\t"
        "ds_read_b128 %1, %10 offset:%c13\n\t"
        "ds_read_b128 %2, %10 offset:%c14\n\t"
        "ds_read_b128 %3, %10 offset:%c15\n\t"
        "ds_read_b128 %4, %10 offset:%c16\n\t"
        "ds_read_b128 %5, %11 offset:%c12\n\t"
        "ds_read_b128 %6, %11 offset:%c13\n\t"
        "ds_read_b128 %7, %11 offset:%c14\n\t"
        "ds_read_b128 %8, %11 offset:%c15\n\t"
        "ds_read_b128 %9, %11 offset:%c16\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(ah[0]), "=&v"(ah[1]), "=&v"(ah[2]), "=&v"(ah[3]), "=&v"(ah[4]),
          "=&v"(bh[0]), "=&v"(bh[1]), "=&v"(bh[2]), "=&v"(bh[3]), "=&v"(bh[4])
        : "v"(abase), "v"(bbase), "n"(0), "n"(STEP), "n"(2 * STEP), "n"(3 * STEP), "n"(4 * STEP)
        : "memory");
  } else {
    asm volatile(
        "ds_read_b128 %0, %15 offset:%c17\n\t"
        "ds_read_b128 %1, %15 offset:%c18\n\t"
        "ds_read_b128 %2, %15 offset:%c19\n\t"
        "ds_read_b128 %3, %15 offset:%c20\n\t"
        "ds_read_b128 %4, %15 offset:%c21\n\t"
        "ds_read_b128 %5, %15 offset:%c22\n\t"
        "ds_read_b128 %6, %15 offset:%c23\n\t"
        "ds_read_b128 %7, %15 offset:%c24\n\t"
        "ds_read_b128 %8, %15 offset:%c25\n\t"
        "ds_read_b128 %9, %15 offset:%c26\n\t"
        "ds_read_b128 %10, %16 offset:%c17\n\t"
        "ds_read_b128 %11, %16 offset:%c18\n\t"
        "ds_read_b128 %12, %16 offset:%c19\n\t"
        "ds_read_b128 %13, %16 offset:%c20\n\t"
        "ds_read_b128 %14, %16 offset:%c21\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(ah[0]), "=&v"(ah[1]), "=&v"(ah[2]), "=&v"(ah[3]), "=&v"(ah[4]),
          "=&v"(ah[5]), "=&v"(ah[6]), "=&v"(ah[7]), "=&v"(ah[8]), "=&v"(ah[9]),
          "=&v"(bh[0]), "=&v"(bh[1]), "=&v"(bh[2]), "=&v"(bh[3]), "=&v"(bh[4])
        : "v"(abase), "v"(bbase), "n"(0), "n"(STEP), "n"(2 * STEP), "n"(3 * STEP), "n"(4 * STEP),
          "n"(PROD), "n"(PROD + STEP), "n"(PROD + 2 * STEP), "n"(PROD + 3 * STEP), "n"(PROD + 4 * STEP)
        : "memory");
  }
}

// Epilogue of the 160-wide BF16 tiles (16x16 MFMA fragments; each wave
// owns 80 x 80 positions of every product of the tile).
//  1. Trace partials (against a matrix, or of the diagonal) from the
//     registers, reduced in a fixed order into had_part.
//  2. Each output in turn is staged through the LDS operand buffers (free
//     after the main loop) in its own orientation -- row-major, or
//     transposed -- and copied out as 16-byte vectors along its rows.  FP32
//     outputs that do not fit are staged in two halves of the tile rows.
// Problems on these tiles carry no addends.
__device__ __forceinline__ uint16_t bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

template <Prec P, int W, int NA, typename AccT>
__device__ __forceinline__ void wide_epilogue(const InstGeo& L, const Prob& pb, const Unit& u, int tile, int64_t row0,
                                              int64_t col0, unsigned char* smem, double* red, AccT& acc) {
  using C = Cfg<P, W>;
  constexpr int SM = C::BM / NA, SN = C::BN;
  constexpr int FR = C::TM / NA, FC = C::TN;
  constexpr int HALF_R = SM / 2, HALF_C = SN / 2;
  static_assert(P == Prec::BF16 && C::MT == 16 && C::NACC == 4 && SM == SN, "wide epilogue: BF16 16x16 square tiles");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t mrows = L.m, ncols = L.nc, ld = L.ld;
  const int g4 = 4 * (lane >> 4), lc0 = lane & 15;
  // tile-local row / column of accumulator (gi, gj, r) of this lane
  auto lrow = [&](int gi, int r) { return wm * HALF_R + gi * 16 + g4 + r; };
  auto lcol = [&](int gj) { return wn * HALF_C + gj * 16 + lc0; };

  // 1. trace partials
  const int nh = pb.nhad;
  if (nh) {
    const bool hdiag = pb.had_diag != 0;
    const double* hmat = hdiag ? nullptr : (const double*)pb.had_h.base + off(pb.had_h, u);
    double hs0 = 0.0, hs1 = 0.0, hs2 = 0.0, hs3 = 0.0;
    float hc[kMaxHad][NA];
#pragma unroll
    for (int q = 0; q < kMaxHad; ++q)
#pragma unroll
      for (int a = 0; a < NA; ++a) hc[q][a] = q < nh ? pb.had_coef[q][a] : 0.0f;
    auto add = [&](int gi, int gj, int r, double hv) {
      double s[kMaxHad];
#pragma unroll
      for (int q = 0; q < kMaxHad; ++q) {
        s[q] = 0.0;
#pragma unroll
        for (int a = 0; a < NA; ++a) s[q] += (double)hc[q][a] * (double)acc[a * FR + gi][gj][r];
      }
      hs0 += s[0] * hv; hs1 += s[1] * hv; hs2 += s[2] * hv; hs3 += s[3] * hv;
    };
    if (hdiag) {
      // the diagonal lies in tiles with row0 == col0, on the waves with wm == wn
      if (row0 == col0 && wm == wn) {
#pragma unroll
        for (int gi = 0; gi < FR; ++gi)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            // fragment row gi holds tile rows lrow(gi, r); its diagonal element is in column fragment gi
            if (lrow(gi, r) != lcol(gi) || row0 + lrow(gi, r) >= mrows) continue;
            add(gi, gi, r, 1.0);
          }
      }
    } else {
#pragma unroll
      for (int gi = 0; gi < FR; ++gi)
#pragma unroll
        for (int gj = 0; gj < FC; ++gj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t gr = row0 + lrow(gi, r), gc = col0 + lcol(gj);
            if (gr >= mrows || gc >= ncols) continue;
            add(gi, gj, r, hmat[gr * ld + gc]);
          }
    }
    const double hsv[kMaxHad] = {hs0, hs1, hs2, hs3};
#pragma unroll
    for (int q = 0; q < kMaxHad; ++q) {
      if (q >= nh) break;
      double sq = hsv[q];
      for (int d = 32; d > 0; d >>= 1) sq += __shfl_down(sq, d, 64);
      if (lane == 0) red[wave * kMaxHad + q] = sq;
    }
    __syncthreads();
    if (tid < nh) {
      double sq = red[0 * kMaxHad + tid] + red[1 * kMaxHad + tid];
      sq += red[2 * kMaxHad + tid];
      sq += red[3 * kMaxHad + tid];
      pb.had_part[((int64_t)u.slot * pb.had_slot_stride + tid) * pb.had_ntiles + tile] = sq;
    }
  }

  // 2. outputs, staged. A first pass writes every output (FP32, BF16, or the
  // hi plane bf16(x) of type 2, the BF16X3 storage of a split product); a
  // second pass writes the lo planes bf16(x - hi) of type 2 outputs, L.plane
  // elements further. The plane is a compile-time flag so that the first
  // pass carries no per-element work for the second.
  constexpr int CAP = Smem<P, W>::BYTES;
  auto pass = [&](auto lo_plane) {
    constexpr bool LO = decltype(lo_plane)::value;
    for (int o = 0; o < pb.nout; ++o) {
      const OutSpec& os = pb.out[o];
      if (LO && os.type != 2) continue;
      const int es = os.type == 0 ? 4 : 2;              // bytes per element
      const int vl = 16 / es;                            // elements per 16-byte vector
      char* dst = (char*)os.base + (off(os, u) + (LO ? L.plane : 0)) * (int64_t)es;
      float cf[NA];
#pragma unroll
      for (int a = 0; a < NA; ++a) cf[a] = os.coef[a];
      const bool tr = os.layout != 0;
      // staged region: tile rows [h RS, (h+1) RS); pitch padded by 16 bytes
      const int pr = SN + vl, pt_full = SM + vl, pt_half = HALF_R + vl;
      const bool halves = (tr ? SN * pt_full : SM * pr) * es > CAP;
      const int rs = halves ? HALF_R : SM;
      const int pt = halves ? pt_half : pt_full;
      // single-product wide tiles write row-major FP32 outputs only (the
      // deep-K stage's; the host checks), which keeps their epilogue within
      // two workgroups' registers
      const int kind = (tr ? 2 : 0) + (es == 4 ? 1 : 0);
      if (NA == 1 && kind != 1) continue;
      if (LO && (es != 2 || NA != 2)) continue;          // lo planes: dual-A BF16 outputs only
      for (int h = 0; h < (halves ? 2 : 1); ++h) {
        __syncthreads();                               // LDS free (main loop, traces, last copy-out)
        if (!halves || wm == h) {
          auto val = [&](int gi, int gj, int r) {
            float x = 0.0f;
#pragma unroll
            for (int a = 0; a < NA; ++a) x += cf[a] * acc[a * FR + gi][gj][r];
            return x;
          };
          // BF16 bits of an output element: x, or on a lo plane x - bf16(x)
          auto b16 = [&](float x) {
            if constexpr (LO) return bf16_bits(x - __uint_as_float((uint32_t)bf16_bits(x) << 16));
            else return bf16_bits(x);
          };
          const int hr = h * rs;
          if (NA == 2 && kind == 0) {  // row-major BF16
#pragma unroll
            for (int gi = 0; gi < FR; ++gi)
#pragma unroll
              for (int gj = 0; gj < FC; ++gj)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                  ((uint16_t*)smem)[(lrow(gi, r) - hr) * pr + lcol(gj)] = b16(val(gi, gj, r));
          } else if (!LO && kind == 1) {      // row-major FP32
#pragma unroll
            for (int gi = 0; gi < FR; ++gi)
#pragma unroll
              for (int gj = 0; gj < FC; ++gj)
#pragma unroll
                for (int r = 0; r < 4; ++r) ((float*)smem)[(lrow(gi, r) - hr) * pr + lcol(gj)] = val(gi, gj, r);
          } else if (NA == 2 && kind == 2) {   // transposed BF16: four consecutive tile rows = four elements of an output row
#pragma unroll
            for (int gi = 0; gi < FR; ++gi)
#pragma unroll
              for (int gj = 0; gj < FC; ++gj) {
                const uint32_t lo = (uint32_t)b16(val(gi, gj, 0)) | ((uint32_t)b16(val(gi, gj, 1)) << 16);
                const uint32_t hi = (uint32_t)b16(val(gi, gj, 2)) | ((uint32_t)b16(val(gi, gj, 3)) << 16);
                *(uint2*)((uint16_t*)smem + lcol(gj) * pt + lrow(gi, 0) - hr) = make_uint2(lo, hi);
              }
          } else if (!LO && NA == 2) {        // transposed FP32
#pragma unroll
            for (int gi = 0; gi < FR; ++gi)
#pragma unroll
              for (int gj = 0; gj < FC; ++gj)
                *(float4*)((float*)smem + lcol(gj) * pt + lrow(gi, 0) - hr) =
                    make_float4(val(gi, gj, 0), val(gi, gj, 1), val(gi, gj, 2), val(gi, gj, 3));
          }
        }
        __syncthreads();
        // copy-out: output rows of the staged region as 16-byte vectors
        const int orows = tr ? SN : rs, ocols = tr ? rs : SN;
        const int64_t grow0 = tr ? col0 : row0 + h * rs, gcol0 = tr ? row0 + h * rs : col0;
        const int64_t grows = tr ? ncols : mrows, gcols = tr ? mrows : ncols;
        const int opitch = tr ? pt : pr;
        const int vpr = ocols / vl;
        for (int idx = tid; idx < orows * vpr; idx += kThreads) {
          const int rr = idx / vpr, cc = (idx % vpr) * vl;
          const int64_t gr = grow0 + rr, gc = gcol0 + cc;
          if (gr >= grows || gc >= gcols) continue;
          const unsigned char* src = smem + ((int64_t)rr * opitch + cc) * es;
          char* d = dst + (gr * ld + gc) * es;
          if (gc + vl <= gcols) {
            *(u32x4_t*)d = *(const u32x4_t*)src;
          } else {
            for (int e = 0; e < vl && gc + e < gcols; ++e)
              for (int bq = 0; bq < es; ++bq) d[e * es + bq] = (char)src[e * es + bq];
          }
        }
      }
    }
  };
  pass(std::false_type{});
  pass(std::true_type{});
}

template <Prec P, int W, int NA, int NB>
__device__ __forceinline__ void gemm_body(const InstGeo& L, const Prob& pb, const Unit& u, int tile,
                                          unsigned char* smem, double* red) {
  using C = Cfg<P, W>;
  using E = typename C::E;
  using Acc = typename C::Acc;
  constexpr int BM = C::BM, BN = C::BN, BK = C::BK, PL = C::PLANES;
  constexpr int PITCH = Smem<P, W>::PITCH;
  constexpr int VE = 16 / sizeof(E);                      // elements per 16 B vector
  constexpr int VPR = BK / VE;                            // vectors per tile row
  constexpr int AV = BM * VPR * PL / kThreads, BV = BN * VPR * PL / kThreads;
  static_assert(C::PF == 0 || (BM * VPR * PL % kThreads == 0 && BN * VPR * PL % kThreads == 0), "tile/threads");
  constexpr int TILE_A = Smem<P, W>::TILE_A, TILE_B = Smem<P, W>::TILE_B;
  constexpr int SM = BM / NA, SN = BN / NB;               // output rows / cols per tile
  constexpr int MT = C::MT, NACC = C::NACC;
  constexpr int TM = C::TM, TN = C::TN;                   // MFMA tiles per wave
  constexpr int FR = TM / NA, FC = TN / NB;               // ... per product
  static_assert(TM % NA == 0 && TN % NB == 0 && FR * MT * 2 == SM && FC * MT * 2 == SN, "wave tiling");

  E* As = (E*)smem;                    // [STAGES][PL][rows][PITCH]
  E* Bs = As + Smem<P, W>::STAGES * TILE_A;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform (scalar)
  const int wm = wave >> 1, wn = wave & 1;

  const int64_t mrows = L.m, ncols = L.nc, kk = L.k, ld = L.ld;
  const int tiles_n = (int)((ncols + SN - 1) / SN);
  const int tiles_m = (int)((mrows + SM - 1) / SM);
  const int tm = tile / tiles_n, tn = tile % tiles_n;
  if (tm >= tiles_m) return;
  const int64_t row0 = (int64_t)tm * SM, col0 = (int64_t)tn * SN;
  const int kps = (int)((kk + BK - 1) / BK);
  const int ktiles = kps * pb.nseg;

  // LDS row of MFMA row-fragment i (column fragment j) of this wave, and the
  // output row (column) offset it covers.  With two A matrices the tile holds
  // A_0 rows in [0, SM) and A_1 rows in [SM, 2 SM); fragments
  // [a FR, (a+1) FR) belong to product a and cover the same output rows.
  auto frag_row_lds = [&](int i) { return (i / FR) * SM + wm * (FR * MT) + (i % FR) * MT; };
  auto frag_col_lds = [&](int j) { return (j / FC) * SN + wn * (FC * MT) + (j % FC) * MT; };
  auto frag_row_out = [&](int i) { return wm * (FR * MT) + i * MT; };   // i < FR
  auto frag_col_out = [&](int j) { return wn * (FC * MT) + j * MT; };   // j < FC
  // element (row, k) of a tile plane in LDS; k a multiple of 8 with SWZ
  // 16-byte chunk c of row r sits at chunk c ^ swz(r).  A 16-byte fragment
  // read is served 8 lanes (8 consecutive rows, one logical chunk) at a time
  // from 32 banks of 4 bytes, so those 8 rows must hit 8 distinct 16-byte
  // bank groups: 128-byte rows (BK 64) rotate by r mod 8; 64-byte rows (BK
  // 32, two rows per 32 banks) by (r / 2) mod 4, which gives each of the
  // two row parities 4 distinct chunks
  auto swz = [&](int row) { return BK == 64 ? (row & 7) : ((row >> 1) & 3); };
  auto lds_at = [&](int row, int k) {
    if constexpr (C::SWZ) return row * PITCH + ((((k >> 3) ^ swz(row))) << 3);
    else return row * PITCH + k;
  };

  // Staging geometry.  Vector i of thread t covers tile row trow + c_i
  // (c_i = (i * RSTEP) % rows) of plane (i * RSTEP) / rows and k offset kv;
  // everything but trow and kv is uniform over the workgroup, so each load
  // is a uniform base plus one per-thread offset.
  constexpr int RSTEP = kThreads / VPR;
  static_assert(C::PF == 0 || (BM % RSTEP == 0 && BN % RSTEP == 0 && SM % RSTEP == 0 && SN % RSTEP == 0),
                "staging rows");
  const int trow = tid / VPR;
  const int kv = (tid % VPR) * VE;
  const int64_t toff = (int64_t)trow * ld + kv;
  const E* abase[AV];
  const E* bbase[BV];
  int adr[AV], bdr[BV];                  // row offset of the vector in its matrix (uniform)
  auto set_seg = [&](int seg) {
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const int pl = (i * RSTEP) / BM, c = (i * RSTEP) % BM;
      const int sel = NA == 2 ? c / SM : seg;
      adr[i] = NA == 2 ? c % SM : c;
      const OpRef& ar = pb.a[sel];
      abase[i] = (const E*)ar.base + off(ar, u) + (int64_t)pl * L.plane + (row0 + adr[i]) * ld;
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      const int pl = (i * RSTEP) / BN, c = (i * RSTEP) % BN;
      const int sel = NB == 2 ? c / SN : seg;
      bdr[i] = NB == 2 ? c % SN : c;
      const OpRef& br = pb.b[sel];
      bbase[i] = (const E*)br.base + off(br, u) + (int64_t)pl * L.plane + (col0 + bdr[i]) * ld;
    }
  };
  // Loads are unconditional: out-of-range vectors read 16 zero bytes from
  // kZeroVec instead, so every k tile issues the same instruction stream
  // without branches and no load result is inspected before it is stored.
  const E* zvec = (const E*)&kZeroVec;
  auto gload = [&](int kt, u32x4_t* ra, u32x4_t* rb) {
    const int64_t k0 = (int64_t)(kt % kps) * BK;
    const bool kok = kt < ktiles && k0 + kv < kk;
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const bool ok = kok && row0 + adr[i] + trow < mrows;
      ra[i] = *(const GVec*)(ok ? abase[i] + toff + k0 : zvec);
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      const bool ok = kok && col0 + bdr[i] + trow < ncols;
      rb[i] = *(const GVec*)(ok ? bbase[i] + toff + k0 : zvec);
    }
  };
  static_assert(!C::SWZ || RSTEP % 8 == 0, "swizzle: staged rows share row mod 8");
  auto sstore = [&](int buf, const u32x4_t* ra, const u32x4_t* rb) {
    E* a = As + buf * TILE_A + lds_at(trow, kv);
    E* b = Bs + buf * TILE_B + lds_at(trow, kv);
#pragma unroll
    for (int i = 0; i < AV; ++i) {
      const int pl = (i * RSTEP) / BM, c = (i * RSTEP) % BM;
      *(u32x4_t*)(a + pl * BM * PITCH + c * PITCH) = ra[i];
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
      const int pl = (i * RSTEP) / BN, c = (i * RSTEP) % BN;
      *(u32x4_t*)(b + pl * BN * PITCH + c * PITCH) = rb[i];
    }
  };

  using AccV = typename std::conditional<P == Prec::F64, f64x4_t,
                                         typename std::conditional<NACC == 4, f32x4_t, f32x16_t>::type>::type;
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
        const double* p = a + (frag_row_lds(i) + lr) * PITCH + g * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) av[i][q] = p[q];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const double* p = b + (frag_col_lds(j) + lr) * PITCH + g * 4;
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
          float4 t = *(const float4*)(a + (frag_row_lds(i) + lr) * PITCH + g * 16 + kq * 4);
          av[i][0] = t.x; av[i][1] = t.y; av[i][2] = t.z; av[i][3] = t.w;
        }
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          float4 t = *(const float4*)(b + (frag_col_lds(j) + lr) * PITCH + g * 16 + kq * 4);
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
    } else if constexpr (MT == 16) {
      // 16x16x32: lane group g = lane/16 owns k in [8g, 8g+8) of each 32-wide k step
      const int lr = lane & 15, g = lane >> 4;
#pragma unroll
      for (int ks = 0; ks < BK / 32; ++ks) {
        bf16x8_t ah[TM], bh[TN];
        if constexpr (C::PF == 0 && (TM == 5 || TM == 10) && TN == 5) {
          // Direct-load tiles: the fragments are read by one asm block (all
          // reads, then one wait in the same block).  Through ordinary loads
          // the compiler cannot tell these reads from the direct loads still
          // filling another stage of the ring, and waits for those first.
          // Fragment rows differ by multiples of 16 rows, which leaves the
          // swizzle unchanged, so one base address and immediate offsets
          // cover each operand.
          constexpr int RB = PITCH * (int)sizeof(E);                  // bytes per LDS row
          const uint32_t abase = lds_addr(a + lds_at(frag_row_lds(0) + lr, ks * 32 + g * 8));
          const uint32_t bbase = lds_addr(b + lds_at(frag_col_lds(0) + lr, ks * 32 + g * 8));
          lds_frags<TM, FR, SM * RB, 16 * RB>(ah, bh, abase, bbase);
        } else {
#pragma unroll
          for (int j = 0; j < TN; ++j) bh[j] = *(const bf16x8_t*)(b + lds_at(frag_col_lds(j) + lr, ks * 32 + g * 8));
#pragma unroll
          for (int i = 0; i < TM; ++i) ah[i] = *(const bf16x8_t*)(a + lds_at(frag_row_lds(i) + lr, ks * 32 + g * 8));
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
    } else {
      // lane group g = lane/32 owns k in [8g, 8g+8) of each 16-wide k step
      const int lr = lane & 31, g = lane >> 5;
#pragma unroll
      for (int ks = 0; ks < BK / 16; ++ks) {
        bf16x8_t ah[TM], bh[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          ah[i] = *(const bf16x8_t*)(a + (frag_row_lds(i) + lr) * PITCH + ks * 16 + g * 8);
#pragma unroll
        for (int j = 0; j < TN; ++j)
          bh[j] = *(const bf16x8_t*)(b + (frag_col_lds(j) + lr) * PITCH + ks * 16 + g * 8);
        if constexpr (P == Prec::BF16X3) {
          bf16x8_t al[TM], bl[TN];
#pragma unroll
          for (int i = 0; i < TM; ++i)
            al[i] = *(const bf16x8_t*)(a + BM * PITCH + (frag_row_lds(i) + lr) * PITCH + ks * 16 + g * 8);
#pragma unroll
          for (int j = 0; j < TN; ++j)
            bl[j] = *(const bf16x8_t*)(b + BN * PITCH + (frag_col_lds(j) + lr) * PITCH + ks * 16 + g * 8);
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

  // -------- main loop: LDS double buffer, two k tiles in flight in
  // registers (tile t is loaded two steps before it is computed), one
  // barrier per k tile.  Unrolled by two so that each register set is static.
  // Every step issues its loads and stores (tiles past the end load zeros),
  // so the outstanding-load count is the same on every path and each store
  // waits only for the loads of its own tile.
  u32x4_t ra0[AV], rb0[BV];
  auto issue = [&](int t, u32x4_t* ra, u32x4_t* rb) {
    if (t < ktiles && t % kps == 0) set_seg(t / kps);
    gload(t, ra, rb);
  };
  if constexpr (C::PF == 0) {
    // Direct global -> LDS loads (global_load_lds_dwordx4): instruction i of
    // wave w fills the RPI tile rows RPI (4 i + w) .. +RPI-1 (1 KB), lane L
    // row RPI (4 i + w) + L / CPR at physical chunk L mod CPR, i.e. logical
    // chunk (L mod CPR) ^ swz(row) of the swizzled layout.  Rows past the
    // tile (LDS padding) load zeros.  STAGES-deep ring: tile t+STAGES-1
    // streams in while tile t is computed; one barrier per k tile.  Every
    // wave issues the same loads per tile, so the wait for tile t is
    // "at most (STAGES-2) tiles of loads outstanding".
    constexpr int STG = Smem<P, W>::STAGES;
    constexpr int RPI = direct_rows<BK>(), CPR = BK / 8;
    constexpr int NLA = Smem<P, W>::ROWS_A / (4 * RPI), NLB = Smem<P, W>::ROWS_B / (4 * RPI);
    static_assert(C::SWZ && PL == 1 && NB == 1 && (NA == 1 || W == 3),
                  "direct loads: swizzled single-plane tiles, single products or dual-A");
    static_assert(SM % RPI == 0 && STG >= 2 && (STG - 2) * (NLA + NLB) < 64, "direct-load geometry");
    const int lrow = lane / CPR, pch = lane % CPR;
    const E* dab[NLA];
    const E* dbb[NLB];
    auto dseg = [&](int seg) {
      const OpRef& br = pb.b[seg];
#pragma unroll
      for (int i = 0; i < NLA; ++i) {
        const int r = RPI * (4 * i + wave) + lrow;
        const int sel = NA == 2 ? 2 * seg + (r < SM ? 0 : 1) : seg;   // dual-A: a[2 seg], a[2 seg + 1]
        const OpRef& ar = pb.a[sel];
        const int rr = NA == 2 ? r % SM : r;
        dab[i] = (const E*)ar.base + off(ar, u) + (row0 + rr) * ld;
      }
#pragma unroll
      for (int i = 0; i < NLB; ++i)
        dbb[i] = (const E*)br.base + off(br, u) + (col0 + RPI * (4 * i + wave) + lrow) * ld;
    };
    int dseg_i = 0, dk = 0;                 // segment and k tile within it of the next load
    auto dload = [&](int t) {
      if (dk == 0) dseg(dseg_i);
      const int64_t k0 = (int64_t)dk * BK;
      E* sa = As + (t % STG) * TILE_A;
      E* sb = Bs + (t % STG) * TILE_B;
#pragma unroll
      for (int i = 0; i < NLA; ++i) {
        const int r = RPI * (4 * i + wave) + lrow;
        const int rr = NA == 2 ? r % SM : r;
        const int64_t kc = k0 + ((pch ^ swz(r)) << 3);
        const bool ok = r < BM && kc < kk && row0 + rr < mrows;
        const E* src = ok ? dab[i] + kc : zvec;
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                         (__attribute__((address_space(3))) void*)(sa + (4 * i + wave) * 512),
                                         16, 0, 0);
      }
#pragma unroll
      for (int i = 0; i < NLB; ++i) {
        const int r = RPI * (4 * i + wave) + lrow;
        const int64_t kc = k0 + ((pch ^ swz(r)) << 3);
        const bool ok = r < BN && kc < kk && col0 + r < ncols;
        const E* src = ok ? dbb[i] + kc : zvec;
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                         (__attribute__((address_space(3))) void*)(sb + (4 * i + wave) * 512),
                                         16, 0, 0);
      }
      if (++dk == kps) {
        dk = 0;
        ++dseg_i;
      }
    };
    if (ktiles > 0) {
#pragma unroll
      for (int t = 0; t < STG - 1; ++t)
        if (t < ktiles) dload(t);
      for (int kt = 0; kt < ktiles; ++kt) {
        // this lane's loads of tile kt have landed (the only ones that may
        // still be outstanding belong to the STG-2 tiles after it), then
        // every lane's have; every wave is also done with tile kt-1, whose
        // buffer the next loads overwrite
        if (kt + STG - 2 < ktiles) waitcnt_vm<(STG - 2) * (NLA + NLB)>();
        else waitcnt_vm<0>();
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        if (kt + STG - 1 < ktiles) dload(kt + STG - 1);
        compute(kt % STG);
      }
      __syncthreads();       // LDS free for the epilogue's reduction slots
    }
  } else if constexpr (C::PF == 1) {
    // one k tile in flight in registers: tile t+1 loads while tile t computes
    if (ktiles > 0) {
      issue(0, ra0, rb0);
      sstore(0, ra0, rb0);
      __syncthreads();
      for (int kt = 0; kt < ktiles; ++kt) {
        issue(kt + 1, ra0, rb0);
        compute(kt & 1);
        sstore((kt + 1) & 1, ra0, rb0);
        __syncthreads();
      }
    }
  } else if (ktiles > 0) {
    u32x4_t ra1[AV], rb1[BV];
    issue(0, ra0, rb0);
    issue(1, ra1, rb1);
    sstore(0, ra0, rb0);
    __syncthreads();
    for (int kt = 0; kt < ktiles; kt += 2) {
      issue(kt + 2, ra0, rb0);
      compute(0);
      sstore(1, ra1, rb1);
      __syncthreads();
      if (kt + 1 >= ktiles) break;
      issue(kt + 3, ra1, rb1);
      compute(1);
      sstore(0, ra0, rb0);
      __syncthreads();
    }
  }

  if constexpr (W != 0) {
    wide_epilogue<P, W, NA>(L, pb, u, tile, row0, col0, smem, red, acc);
    return;
  }
  // -------- epilogue straight from the accumulators
  constexpr int NPROD = NA * NB;
  constexpr int GI = FR;                      // distinct row positions
  constexpr int GJ = FC;                      // distinct column positions
  Acc addc[kMaxAdd];
  const void* addp[kMaxAdd];
  // dual-A wide tiles carry no addends and no Hadamard partials against a
  // matrix (their problems have none; diagonal traces they do carry):
  // compiled out, which keeps the tile in registers
  constexpr bool kExtras = W != 3;
  const int nadd = kExtras ? pb.nadd : 0;
  for (int x = 0; x < nadd; ++x) {
    addc[x] = (Acc)pb.add_coef[(int64_t)u.slot * kMaxAdd + x];
    addp[x] = (const char*)pb.add[x].base + off(pb.add[x], u) * (int64_t)sizeof(E);
  }
  const int nout = pb.nout;
  void* obase[kMaxOut];
  for (int o = 0; o < nout; ++o)
    obase[o] = (char*)pb.out[o].base +
               off(pb.out[o], u) * (int64_t)(pb.out[o].type == 0 ? sizeof(Acc) : sizeof(E));
  const bool hdiag = pb.had_diag != 0;      // traces of the products (H = I): no matrix read
  const double* hmat = pb.nhad && !hdiag ? (const double*)pb.had_h.base + off(pb.had_h, u) : nullptr;
  double hsum[kMaxHad] = {0.0, 0.0, 0.0, 0.0};
  const int nh = (kExtras || hdiag) ? pb.nhad : 0;
  const int ac = acc_col<P, MT>(lane);
  // For 32 x 32 tiles, accumulators 4q .. 4q+3 of a lane are four
  // consecutive rows, so transposed outputs are written as one 4-element
  // vector per lane.  Row-major outputs hold consecutive columns in
  // consecutive lanes: in BF16 (128-wide tiles) they are staged through the
  // LDS operand buffers (free after the main loop) and written out as
  // 16-byte row vectors; otherwise element by element.
  constexpr int RG = (P == Prec::F64) ? 1 : 4;            // rows packed per transposed store
  constexpr bool kStageRows = P == Prec::BF16 && W == 0;
  int soff[kMaxOut];                                       // byte offset of a staged output
  bool staged = false;
  if constexpr (kStageRows) {
    int total = 0;
    for (int o = 0; o < nout; ++o) {
      soff[o] = -1;
      if (pb.out[o].layout == 0) {
        soff[o] = total;
        total += SM * SN * (pb.out[o].type == 0 ? 4 : 2);
      }
    }
    staged = total > 0 && total <= Smem<P, W>::BYTES;
  }
#pragma unroll
  for (int gi = 0; gi < GI; ++gi)
#pragma unroll
    for (int gj = 0; gj < GJ; ++gj) {
      const int64_t rbase = row0 + frag_row_out(gi);
      const int64_t gc = col0 + frag_col_out(gj) + ac;
      const bool colok = gc < ncols;
#pragma unroll
      for (int q = 0; q < NACC / RG; ++q) {
        Acc v[RG][NPROD];
        int64_t grs[RG];
#pragma unroll
        for (int e = 0; e < RG; ++e) {
          const int r = q * RG + e;
          grs[e] = rbase + acc_row<P, MT>(lane, r);
#pragma unroll
          for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) v[e][a * NB + b] = acc[a * FR + gi][b * FC + gj][r];
          if (nadd && colok && grs[e] < mrows) {
            const int64_t gn = grs[e] * ld + gc;
            for (int x = 0; x < nadd; ++x) v[e][0] += addc[x] * load_st<P>(addp[x], gn, L.plane);
          }
        }
        const bool full = colok && grs[RG - 1] < mrows;   // all RG rows in range (they are consecutive)
        for (int o = 0; o < nout; ++o) {
          const OutSpec& os = pb.out[o];
          Acc sv[RG];
#pragma unroll
          for (int e = 0; e < RG; ++e) {
            Acc s = 0;
#pragma unroll
            for (int t = 0; t < NPROD; ++t) s += (Acc)os.coef[t] * v[e][t];
            sv[e] = s;
          }
          if (kStageRows && staged && os.layout == 0) {
            // tile-local (row, column); out-of-range positions are staged
            // too but never copied out
            const int lc = (int)(gc - col0);
#pragma unroll
            for (int e = 0; e < RG; ++e) {
              const int lrw = (int)(grs[e] - row0);
              if (os.type == 0)
                ((float*)(smem + soff[o]))[lrw * SN + lc] = sv[e];
              else
                ((bf16_t*)(smem + soff[o]))[lrw * SN + lc] = f2bf(sv[e]);
            }
          } else if (os.layout != 0 && RG == 4 && full) {
            store_out_vec4<P>(os.type, obase[o], gc * ld + grs[0], L.plane, sv);
          } else {
#pragma unroll
            for (int e = 0; e < RG; ++e) {
              if (!colok || grs[e] >= mrows) continue;
              store_out<P>(os.type, obase[o], os.layout == 0 ? grs[e] * ld + gc : gc * ld + grs[e], L.plane, sv[e]);
            }
          }
        }
        if (nh && colok) {
#pragma unroll
          for (int e = 0; e < RG; ++e) {
            if (grs[e] >= mrows) continue;
            double h;
            if (hdiag) {
              if (grs[e] != gc) continue;
              h = 1.0;
            } else {
              if constexpr (!kExtras) continue;
              h = hmat[grs[e] * ld + gc];
            }
            for (int hq = 0; hq < nh; ++hq) {
              double s = 0.0;
#pragma unroll
              for (int t = 0; t < NPROD; ++t) s += (double)pb.had_coef[hq][t] * (double)v[e][t];
              hsum[hq] += s * h;
            }
          }
        }
      }
    }
  if (kStageRows && staged) {
    __syncthreads();
    for (int o = 0; o < nout; ++o) {
      if (pb.out[o].layout != 0) continue;
      const int es = pb.out[o].type == 0 ? 4 : 2;
      const int vl = 16 / es;                 // elements per 16-byte vector
      const int vpr = SN / vl;                // vectors per tile row
      const unsigned char* src = smem + soff[o];
      char* dst = (char*)obase[o];
      for (int idx = tid; idx < SM * vpr; idx += kThreads) {
        const int r = idx / vpr, c = (idx % vpr) * vl;
        const int64_t gr = row0 + r, gcc = col0 + c;
        if (gr >= mrows || gcc >= ncols) continue;
        const int64_t gi = gr * ld + gcc;
        if (gcc + vl <= ncols) {
          *(u32x4_t*)(dst + gi * es) = *(const u32x4_t*)(src + (r * SN + c) * es);
        } else {
          for (int e = 0; e < vl && gcc + e < ncols; ++e)
            for (int bq = 0; bq < es; ++bq) dst[(gi + e) * es + bq] = (char)src[(r * SN + c + e) * es + bq];
        }
      }
    }
  }
  if (nh) {
    // deterministic block reduction: wave tree, then the four waves in order
    for (int q = 0; q < nh; ++q) {
      double s = hsum[q];
      for (int d = 32; d > 0; d >>= 1) s += __shfl_down(s, d, 64);
      if (lane == 0) red[wave * kMaxHad + q] = s;
    }
    __syncthreads();
    if (tid < nh) {
      double s = red[0 * kMaxHad + tid] + red[1 * kMaxHad + tid];
      s += red[2 * kMaxHad + tid];
      s += red[3 * kMaxHad + tid];
      pb.had_part[((int64_t)u.slot * pb.had_slot_stride + tid) * pb.had_ntiles + tile] = s;
    }
  }
}

template <Prec P, int W, bool MI>
__device__ __forceinline__ void gemm_item(const GemmLaunch& L, int tile, int py, unsigned char* smem,
                                          double* red) {
  const int ui = py / L.nprob, pi = py % L.nprob;
  const Unit u = L.units[ui];
  const Prob& pb = MI ? L.probs[(int64_t)u.inst * L.pstride + pi] : L.probs[pi];
  const InstGeo g = MI ? L.geo[u.inst] : L.g;
  if constexpr (W == 1 || W == 2) {
    gemm_body<P, W, 1, 1>(g, pb, u, tile, smem, red);   // single-product problems only
  } else if constexpr (W == 3) {
    gemm_body<P, W, 2, 1>(g, pb, u, tile, smem, red);   // dual-A problems only
  } else {
    const int mode = (pb.nA == 2 ? 2 : 0) + (pb.nB == 2 ? 1 : 0);
    switch (mode) {
      case 0: gemm_body<P, W, 1, 1>(g, pb, u, tile, smem, red); break;
      case 1: gemm_body<P, W, 1, 2>(g, pb, u, tile, smem, red); break;
      case 2: gemm_body<P, W, 2, 1>(g, pb, u, tile, smem, red); break;
      default: gemm_body<P, W, 2, 2>(g, pb, u, tile, smem, red); break;
    }
  }
}

// Work item -> (tile, unit * nprob + problem).
template <bool MI>
__device__ __forceinline__ void decode_item(const GemmLaunch& L, int64_t item, int& tile, int& py) {
  if (!MI) {
    tile = (int)(item % L.tiles);
    py = (int)(item / L.tiles);
    return;
  }
  int lo = 0, hi = L.nseg - 1;                 // last run with item0 <= item
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (L.segs[mid].item0 <= item) lo = mid; else hi = mid - 1;
  }
  const BatchSeg sg = L.segs[lo];
  const int64_t local = item - sg.item0;
  const int64_t per_unit = (int64_t)L.nprob * sg.tiles;
  const int64_t ui = sg.unit0 + local / per_unit;
  const int64_t rem = local % per_unit;
  tile = (int)(rem % sg.tiles);
  py = (int)(ui * L.nprob + rem / sg.tiles);
}

// MI: a multi-instance launch (per-unit instance geometry and problems, work
// list of runs); otherwise one instance, items tile-major per (unit, problem).
// PERSIST: a grid-stride loop over the items, else one item per workgroup
// (kept loop-free, so nothing is hoisted across items).
// W = 1: the wide tile fills exactly half of a CU's LDS, so the epilogue's
// reduction slots reuse the operand buffers (the main loop ends with a
// barrier); otherwise they have their own.
template <Prec P, int W> struct RedSlots {
  static constexpr int N = W == 1 ? 1 : 4 * kMaxHad;
};

// Workgroups per CU the register budget is sized for: the dual-A wide tile
// keeps 200 accumulator registers live through its staged epilogue and
// takes a whole CU's register file; the others fit two.
template <int W> struct MinBlocks { static constexpr int N = W == 3 ? 1 : 2; };

template <Prec P, int W, bool MI, bool PERSIST>
__global__ __launch_bounds__(kThreads, MinBlocks<W>::N) void gemm_kernel(GemmLaunch L) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[Smem<P, W>::BYTES];
  __shared__ double red_own[RedSlots<P, W>::N];
  double* red = W == 1 ? (double*)smem : red_own;
  int tile, py;
  if constexpr (!PERSIST) {
    decode_item<MI>(L, xcd_remap((int64_t)blockIdx.x, (int64_t)gridDim.x), tile, py);
    gemm_item<P, W, MI>(L, tile, py, smem, red);
  } else {
    // XCD x = b % 8 takes the contiguous x-th eighth of the items
    // (consecutive items share a (unit, problem)); its workgroups stride
    // through it.
    const int64_t items = MI ? L.nitems : (int64_t)L.tiles * L.nunit * L.nprob;
    const int x = blockIdx.x & 7;
    const int64_t per = items / 8, rem = items % 8;
    const int64_t lo = x * per + (x < rem ? x : rem);
    const int64_t hi = lo + per + (x < rem ? 1 : 0);
    for (int64_t j = lo + (blockIdx.x >> 3); j < hi; j += gridDim.x >> 3) {
      decode_item<MI>(L, j, tile, py);
      gemm_item<P, W, MI>(L, tile, py, smem, red);
      __syncthreads();                   // LDS of the next item
    }
  }
}

}  // namespace

int gemm_tile_m(Prec p, int wide) {
  switch (p) {
    case Prec::F64: return Cfg<Prec::F64>::BM;
    case Prec::F32: return Cfg<Prec::F32>::BM;
    case Prec::BF16: return wide == 1 ? Cfg<Prec::BF16, 1>::BM : wide == 2 ? Cfg<Prec::BF16, 2>::BM
                            : wide == 3 ? Cfg<Prec::BF16, 3>::BM : Cfg<Prec::BF16>::BM;
    default: return Cfg<Prec::BF16X3>::BM;
  }
}
int gemm_tile_n(Prec p, int wide) {
  switch (p) {
    case Prec::F64: return Cfg<Prec::F64>::BN;
    case Prec::F32: return Cfg<Prec::F32>::BN;
    case Prec::BF16: return wide == 1 ? Cfg<Prec::BF16, 1>::BN : wide == 2 ? Cfg<Prec::BF16, 2>::BN
                            : wide == 3 ? Cfg<Prec::BF16, 3>::BN : Cfg<Prec::BF16>::BN;
    default: return Cfg<Prec::BF16X3>::BN;
  }
}

bool gemm_wide_supports(int wide, const Prob& pb) {
  if (wide == 3)
    return pb.nA == 2 && pb.nB == 1 && pb.nseg >= 1 && 2 * pb.nseg <= kMaxSeg && pb.nadd == 0 &&
           (pb.nhad == 0 || pb.had_diag);
  if (wide == 1 || wide == 2) {
    if (pb.nA != 1 || pb.nB != 1 || pb.nadd != 0) return false;
    for (int o = 0; o < pb.nout; ++o)
      if (pb.out[o].type != 0 || pb.out[o].layout != 0) return false;
    return true;
  }
  return true;
}

void launch_gemm(Prec p, const GemmLaunch& Lin, int max_tiles, hipStream_t st) {
  if (Lin.nunit <= 0 || Lin.nprob <= 0 || max_tiles <= 0) return;
  GemmLaunch L = Lin;
  L.tiles = max_tiles;
  const int64_t items = L.segs ? L.nitems : (int64_t)max_tiles * L.nunit * L.nprob;
  if (items <= 0) return;
  // a grid of at most 2^31 - 1 workgroups; beyond, run persistent
  if (L.persist == 0 && items > 0x7fffffffLL) L.persist = 8192;
  if (!L.segs) L.persist = 0;    // single-instance launches: one item per workgroup
  dim3 grid(L.persist > 0 ? (unsigned)(((L.persist + 7) / 8) * 8) : (unsigned)items);
  const bool mi = L.segs != nullptr, pers = L.persist > 0;
  auto go = [&](auto kern) { hipLaunchKernelGGL(kern, grid, dim3(kThreads), 0, st, L); };
  if (L.wide) {
    // the 160-wide tiles: BF16, one instance; W 1 and 2 single-product
    // problems, W 3 dual-A problems
    if (p != Prec::BF16 || mi) throw Gf2Error{GF2_E_STATE, "wide GEMM tile: BF16 single-instance launches only"};
    if (L.wide == 1) go(gemm_kernel<Prec::BF16, 1, false, false>);
    else if (L.wide == 2) go(gemm_kernel<Prec::BF16, 2, false, false>);
    else if (L.wide == 3) go(gemm_kernel<Prec::BF16, 3, false, false>);
    else throw Gf2Error{GF2_E_STATE, "unknown GEMM tile"};
    GF2_HIP(hipGetLastError());
    return;
  }
  switch (p) {
    case Prec::F64:
      if (!mi) go(gemm_kernel<Prec::F64, 0, false, false>);
      else if (pers) go(gemm_kernel<Prec::F64, 0, true, true>);
      else go(gemm_kernel<Prec::F64, 0, true, false>);
      break;
    case Prec::F32:
      if (!mi) go(gemm_kernel<Prec::F32, 0, false, false>);
      else if (pers) go(gemm_kernel<Prec::F32, 0, true, true>);
      else go(gemm_kernel<Prec::F32, 0, true, false>);
      break;
    case Prec::BF16:
      if (!mi) go(gemm_kernel<Prec::BF16, 0, false, false>);
      else if (pers) go(gemm_kernel<Prec::BF16, 0, true, true>);
      else go(gemm_kernel<Prec::BF16, 0, true, false>);
      break;
    case Prec::BF16X3:
      if (!mi) go(gemm_kernel<Prec::BF16X3, 0, false, false>);
      else if (pers) go(gemm_kernel<Prec::BF16X3, 0, true, true>);
      else go(gemm_kernel<Prec::BF16X3, 0, true, false>);
      break;
  }
  GF2_HIP(hipGetLastError());
}
