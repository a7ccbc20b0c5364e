// Internal definitions shared by the HIP sources of libgf2 (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "gf2.h"

// ---------------------------------------------------------------- errors --

struct Gf2Error {
  gf2_status code;
  std::string msg;
};

#define GF2_HIP(call)                                                         \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw Gf2Error{GF2_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define GF2_REQUIRE(cond, code, what)                                         \
  do {                                                                        \
    if (!(cond)) throw Gf2Error{code, std::string(what)};                    \
  } while (0)

// ---------------------------------------------------------------- types ---

typedef unsigned short bf16_t;   // raw bfloat16 bits

enum class Prec : int { F64 = 0, F32 = 1, BF16 = 2, BF16X3 = 3 };

// Element counts are padded: every N x N matrix of the chain is stored as
// np x np with np = pad_dim(n), zero outside [0,n) x [0,n).
inline int64_t pad_dim(int64_t n) { return (n + 31) / 32 * 32; }

// Address of an operand for one (tau, sample, slot) unit, in elements:
// base + tau st_tau + s st_s + s2 st_s2 + slot st_slot (s indexes the
// first set of stochastic vectors, s2 the second).
struct OpRef {
  const void* base;
  int64_t st_tau, st_s, st_slot, st_s2;
};

// One output of a GEMM tile: a combination of the nA x nB products written
// to `base` in accumulator (type 0) or storage (type 1) format, row-major
// (layout 0) or transposed (layout 1).
struct OutSpec {
  void* base;
  int64_t st_tau, st_s, st_slot;
  float coef[4];
  int32_t layout;
  int32_t type;
};

constexpr int kMaxSeg = 24;   // 8 segments, or 24 when each runs as three BF16 products (BF16X3)
constexpr int kMaxOut = 8;
constexpr int kMaxHad = 4;
constexpr int kMaxAdd = 4;

// One GEMM sub-problem per unit.  nA = nB = 1 with nseg K-segments
// (C = sum_s A_s B_s^T), or nseg = 1 with nA, nB in {1, 2}: the tile holds
// the products A_a B_b for every pair (a, b).
struct Prob {
  int32_t nseg, nA, nB, nout, nhad, nadd;
  OpRef a[kMaxSeg];
  OpRef b[kMaxSeg];
  OutSpec out[kMaxOut];
  // Hadamard partial sums: part[(slot*had_slot_stride + h)*ntiles + tile] =
  //   sum over the tile of (sum_ab had_coef[h][ab] P_ab)_ij * H_ij.
  // had_diag: H is the identity (traces of the product combinations; had_h
  // unused).  Partials of slot s go to had_part[(s * had_slot_stride + h) *
  // had_ntiles + tile].
  OpRef had_h;              // FP64 np x np
  float had_coef[kMaxHad][4];
  double* had_part;
  int64_t had_ntiles;
  int32_t had_diag;
  int32_t had_slot_stride;
  // Addends (nA = nB = 1 only): P += sum_x add_coef[slot][x] * Add_x (storage
  // format, row-major).
  OpRef add[kMaxAdd];
  const double* add_coef;   // [slot][kMaxAdd]
};

// One (tau, pair) unit: s and s2 index the first- and second-set vectors
// of the pair (equal for the paired estimator), row its per-pair sample row.
struct Unit {
  int32_t tau, s, slot, inst;   // inst: instance of a multi-instance launch (0 otherwise)
  int32_t s2, row;
};

// Geometry of one instance of a launch.
struct InstGeo {
  int64_t m, nc, k;     // rows of C, columns of C, reduction length
  int64_t ld;           // leading dimension of every operand and output
  int64_t plane;        // element stride of the lo plane (BF16X3)
};

// C (m x nc) = sum_s A_s (m x k, leading dim ld) B_s^T (nc x k, leading dim
// ld); outputs use leading dim ld as well.  k must be a multiple of 8 and
// the operands zero beyond their logical extent in k.
// A run of consecutive units of one instance in a multi-instance launch: its
// work items are the (unit, problem, tile) triples, tile fastest, with
// `tiles` tiles per (unit, problem) (the instance's largest problem).
struct BatchSeg {
  int64_t item0;        // first work item of the run
  int32_t unit0;        // first unit (index into GemmLaunch::units)
  int32_t nunits;
  int32_t tiles;
  int32_t pad;
};

struct GemmLaunch {
  const Prob* probs;    // device; problem j of instance i at probs[i * pstride + j]
  int32_t nprob;
  int32_t pstride;
  const Unit* units;    // device
  int32_t nunit;
  InstGeo g;            // geometry when geo is null (single instance)
  const InstGeo* geo;   // device, per instance, or null
  int32_t tiles;        // tiles per (unit, problem) covered by the launch
  int32_t persist;      // 0: one workgroup per work item; else a grid-stride
                        // loop over the items (grid a multiple of 8)
  const BatchSeg* segs; // device work list (multi-instance), or null: items are
  int32_t nseg;         // tile + tiles * (unit * nprob + problem)
  int64_t nitems;       // items of the work list
  int32_t wide;         // BF16 wide tile (single instance, single-product problems)
};

// Resolves the fixed scratch of gf2_energy_noalloc on `device` (current).
gf2_status noalloc_attach(int device);

// Kernel launchers (device code in separate translation units).
void launch_gemm(Prec p, const GemmLaunch& L, int max_tiles, hipStream_t st);
// Chain launch: square n x n products stored with leading dimension np.
inline GemmLaunch chain_launch(const Prob* probs, int nprob, const Unit* units, int nunit, int64_t n,
                               int64_t np, int64_t plane) {
  return GemmLaunch{probs, nprob, 0, units, nunit, InstGeo{n, n, np, np, plane}, nullptr, 0, 0, nullptr, 0, 0, 0};
}
// Whether a problem fits the epilogue of wide tile `wide` (1 and 2: single
// products with row-major FP32 outputs; 3: dual-A products without addends
// or matrix Hadamard partials).
bool gemm_wide_supports(int wide, const Prob& pb);
int gemm_tile_m(Prec p, int wide = 0);     // BM
int gemm_tile_n(Prec p, int wide = 0);     // BN

// ---------------------------------------------------------------- context -

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct gf2_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t aux = nullptr;      // second stream (default priority, non-blocking), made on first use
  std::string err;
  std::map<std::string, DevBuf> bufs;   // named scratch buffers owned by the context
  int64_t max_units = 0;          // chunk size tuning (0 = automatic)
  int32_t gemm_wide = 2;          // BF16 tiles where 160 pads less than 128: 2 all stages, 1 s4 only, 0 none
  // (n, np, precision) of the last chain layout per buffer-tag prefix
  std::map<std::string, std::string> chain_keys;
  // per prefix and buffer: bytes cleared under that prefix's current layout
  std::map<std::string, std::map<std::string, size_t>> chain_cleared;
  // launch shapes chosen by the batch autotuner, per batch signature
  std::map<std::string, std::pair<int32_t, int32_t>> tuned;
  // tile mode (as gemm_wide) chosen by the batch autotuner per (precision, N);
  // it takes precedence over gemm_wide for chains of that size
  std::map<std::pair<int32_t, int64_t>, int32_t> tiles_tuned;
  // optional per-kernel-class timing with HIP events on ctx->stream
  bool prof = false;
  struct Ev { std::string name; hipEvent_t a, b; double flops, bytes; };
  std::vector<Ev> events;
};

// Records HIP events around one launch when profiling is on.
struct ProfScope {
  gf2_ctx* ctx;
  size_t idx = (size_t)-1;
  ProfScope(gf2_ctx* c, const char* name, double flops = 0.0, double bytes = 0.0) : ctx(c) {
    if (!ctx->prof) return;
    gf2_ctx::Ev e{name, nullptr, nullptr, flops, bytes};
    if (hipEventCreate(&e.a) != hipSuccess || hipEventCreate(&e.b) != hipSuccess) return;
    (void)hipEventRecord(e.a, ctx->stream);
    ctx->events.push_back(e);
    idx = ctx->events.size() - 1;
  }
  ~ProfScope() {
    if (idx != (size_t)-1) (void)hipEventRecord(ctx->events[idx].b, ctx->stream);
  }
};

struct gf2_split_h {
  gf2_ctx* owner = nullptr;
  const void* bsrc = nullptr;
  // The tensor whose elements at or above `thresh` form the large part
  // (null: B itself).  R^L takes those elements, R^S = R - R^L.
  const void* lsrc = nullptr;
  gf2_dtype dtype = GF2_F64;
  int64_t n = 0, naux = 0, np = 0;
  double eps = 0.0, kmax = 0.0, thresh = 0.0;
  int64_t nnz = 0;
  int32_t wmax = 0;
  int32_t span128 = 0;         // widest orbital range touched by 128 consecutive Q
  // device arrays
  int32_t* w = nullptr;        // [naux]
  int32_t* idx = nullptr;      // [naux][32], -1 padded
  double* blk = nullptr;       // [naux][32][32]
  float* blk32 = nullptr;      // same in FP32
  // by-column copies for supports of at most kDdW orbitals (else null):
  // idx_t[c * naux + Q] = idx[Q][c], blk_t[(c * kDdW + d) * naux + Q] = blk[Q][c][d]
  int32_t* idx_t = nullptr;    // [kDdW][naux]
  double* blk_t = nullptr;     // [kDdW * kDdW][naux]
  // union pattern of the blocks: for every nonzero (i, j) of
  // U_Q S_Q x S_Q (sorted row-major) the list of contributing (Q, a, b).
  int64_t npat = 0;
  int32_t* pat_ij = nullptr;   // [npat] i * np + j
  int32_t* pat_off = nullptr;  // [npat + 1]
  int32_t* pat_q = nullptr;    // [ncontrib] Q * 1024 + a * 32 + b
  int64_t ncontrib = 0;
  // rows: for each orbital i the (Q, a) with S_Q[a] = i
  int32_t* row_off = nullptr;  // [n + 1]
  int32_t* row_q = nullptr;    // [..] Q * 32 + a
  // per orbital i: the (Q, a) with S_Q[a] = i, sorted by Q (Q << 5 | a)
  int32_t* orb_off = nullptr;  // [n + 1]
  int32_t* orb_q = nullptr;
  // orb_cs[i * orb_ncs + c]: first entry of orbital i's list with Q >= 64 c
  // (c = 0 .. orb_ncs - 1; the last is orb_off[i + 1])
  int32_t* orb_cs = nullptr;
  int32_t orb_ncs = 0;
};

constexpr int kWMax = 32;
// Widest column window the row-staged deterministic block stages in LDS.
constexpr int kDdSpan = 128;
// Widest support the register form of the deterministic block takes.
constexpr int kDdW = 8;
