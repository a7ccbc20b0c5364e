// C ABI of libgf2: argument checking, device buffers, and the launch
// schedule of the RS-SRI-GF2 hot path (see include/gf2.h).
#include <algorithm>
#include <array>
#include <cmath>
#include <limits>
#include <cstring>
#include <map>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "gf2_proposal.h"

void launch_mlp_init(const double* phi, int64_t ntotal, uint64_t seed, const gf2_mlp& m, hipStream_t st);
void launch_mlp_train(const gf2_mlp& m, int32_t nchains, const int64_t* coff, const double* phi, const double* that,
                      int32_t steps, float lr, int64_t step0, float* z, float* dz, double* grad, double* loss,
                      hipStream_t st);
void launch_mlp_infer(const gf2_mlp& m, const double* phi, int64_t naux, int bf16, double alpha, float* z, double* p,
                      hipStream_t st);

namespace {

constexpr double kGM = 0.5;   // E = -1/2 int Tr(Sigma Gbar): the MP2 limit fixes it
constexpr int64_t kLevelProbe = 8;   // pairs run at both levels (BF16 and BF16X3) by BF16C and AUTO
constexpr int64_t kAutoProbe0 = 2;   // AUTO's first probe; it grows to kLevelProbe where needed
// AUTO goes to BF16X3 at once when its first probe already puts the BF16
// correction this many times above what the error bar allows
constexpr double kAutoEarly = 3.0;

// ------------------------------------------------------------ scratch ----
// Named device buffers owned by the context (grown on demand, never shrunk,
// freed by gf2_destroy).  The map lives in the context, so contexts used
// from different host threads share nothing.
void* ctx_buf(gf2_ctx* ctx, const std::string& tag, size_t bytes, bool zero = false) {
  DevBuf& b = ctx->bufs[tag];
  if (bytes == 0) bytes = 16;
  if (b.bytes < bytes) {
    if (b.p) {
      GF2_HIP(hipStreamSynchronize(ctx->stream));
      GF2_HIP(hipFree(b.p));
      b.p = nullptr;
      b.bytes = 0;
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
      b.p = nullptr;
      (void)hipGetLastError();   // clear the runtime's sticky error: later launch checks must not see it
      throw Gf2Error{GF2_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes for " + tag +
                                      " failed: " + hipGetErrorString(e)};
    }
    b.bytes = bytes;
    zero = true;
  }
  if (zero) GF2_HIP(hipMemsetAsync(b.p, 0, bytes, ctx->stream));
  return b.p;
}

void free_scratch(gf2_ctx* ctx) {
  for (auto& kv : ctx->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  ctx->bufs.clear();
}

template <typename T>
void h2d(gf2_ctx* ctx, T* dst, const T* src, size_t count) {
  GF2_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
}
template <typename T>
void d2h(gf2_ctx* ctx, T* dst, const T* src, size_t count) {
  GF2_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToHost, ctx->stream));
  GF2_HIP(hipStreamSynchronize(ctx->stream));
}

template <typename F>
gf2_status guarded(gf2_ctx* ctx, F&& f) {
  if (!ctx) return GF2_E_ARG;
  try {
    GF2_HIP(hipSetDevice(ctx->device));
    f();
    ctx->err.clear();
    return GF2_OK;
  } catch (const Gf2Error& e) {
    ctx->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return GF2_E_NOMEM;
  } catch (...) {
    ctx->err = "unexpected internal error";
    return GF2_E_DEVICE;
  }
}

Prec to_prec(gf2_precision p) {
  switch (p) {
    case GF2_PREC_FP64: return Prec::F64;
    case GF2_PREC_FP32: return Prec::F32;
    case GF2_PREC_BF16: return Prec::BF16;
    case GF2_PREC_BF16X3: return Prec::BF16X3;
    default: break;
  }
  throw Gf2Error{GF2_E_ARG, "precision not available here (AUTO: adaptive calls; BF16C: single-chain calls)"};
}
size_t st_elem(Prec p) { return p == Prec::F64 ? 8 : p == Prec::F32 ? 4 : 2; }
int st_planes(Prec p) { return p == Prec::BF16X3 ? 2 : 1; }
size_t acc_elem(Prec p) { return p == Prec::F64 ? 8 : 4; }

double softplus(double x) { return std::max(x, 0.0) + std::log1p(std::exp(-std::fabs(x))); }

void check_finite(gf2_ctx* ctx, const double* x, int64_t count, const char* what) {
  auto* bad = (unsigned long long*)ctx_buf(ctx, "nonfinite", sizeof(unsigned long long), true);
  launch_count_nonfinite(x, count, bad, ctx->stream);
  unsigned long long h = 0;
  d2h(ctx, &h, bad, 1);
  if (h) throw Gf2Error{GF2_E_NUMERIC, std::to_string(h) + " non-finite values in " + what};
}

OpRef opref(const void* base, int64_t st_tau = 0, int64_t st_s = 0, int64_t st_slot = 0, int64_t st_s2 = 0) {
  OpRef r;
  r.base = base; r.st_tau = st_tau; r.st_s = st_s; r.st_slot = st_slot; r.st_s2 = st_s2;
  return r;
}
Unit mk_unit(int64_t tau, int64_t s, int64_t slot, int64_t s2, int64_t row) {
  return Unit{(int32_t)tau, (int32_t)s, (int32_t)slot, 0, (int32_t)s2, (int32_t)row};
}
OutSpec outspec(void* base, int64_t st_slot, std::initializer_list<float> coef, int layout, int type,
                int64_t st_tau = 0) {
  OutSpec o;
  std::memset(&o, 0, sizeof(o));
  o.base = base; o.st_tau = st_tau; o.st_s = 0; o.st_slot = st_slot;
  int i = 0;
  for (float c : coef) o.coef[i++] = c;
  o.layout = layout; o.type = type;
  return o;
}
Prob prob0() {
  Prob p;
  std::memset(&p, 0, sizeof(p));
  p.nseg = 1; p.nA = 1; p.nB = 1;
  p.had_slot_stride = 1;
  return p;
}
int tiles_of(const Prob& p, Prec prec, int64_t m, int64_t nc, int wide = 0) {
  const int64_t sm = gemm_tile_m(prec, wide) / p.nA, sn = gemm_tile_n(prec, wide) / p.nB;
  return (int)(((m + sm - 1) / sm) * ((nc + sn - 1) / sn));
}
int tiles_of(const Prob& p, Prec prec, int64_t n, int wide = 0) { return tiles_of(p, prec, n, n, wide); }

// Tile mode for chains of size n: the autotuner's choice for (prec, n) if
// it made one, else the context's setting.
int32_t tile_mode(const gf2_ctx* ctx, Prec prec, int64_t n) {
  const auto it = ctx->tiles_tuned.find({(int32_t)prec, n});
  return it != ctx->tiles_tuned.end() ? it->second : ctx->gemm_wide;
}

// Whether a 160-wide BF16 tile pads an n x n product less than the standard
// tile (n = 150, 300, 400, 800, ...): the sizes where the tile mode matters.
bool wide_pads_less(Prec prec, int64_t n) {
  if (prec != Prec::BF16) return false;
  const int64_t w = gemm_tile_m(prec, 1), s = gemm_tile_m(prec, 0);
  return ((n + w - 1) / w) * w < ((n + s - 1) / s) * s;
}

// The wide BF16 tile for the chain's single-product stage when it pads an
// n x n product less than the standard tile and the tile mode allows it.
int wide_for(const gf2_ctx* ctx, Prec prec, int64_t n) {
  return tile_mode(ctx, prec, n) && wide_pads_less(prec, n) ? 1 : 0;
}

// Orthonormal eigenbasis of (F, S) on the host in FP64: F C = S C diag(eps)
// with C^T S C = I (S = null: the identity), eps ascending; c[i * n + k] is
// the i-th component of orbital k.  Through S^{-1/2} from S's eigenvectors.
void orbitals_fs(int64_t n, const double* F, const double* S, std::vector<double>& eps, std::vector<double>& c) {
  eps.assign((size_t)n, 0.0);
  c.assign((size_t)(n * n), 0.0);
  if (!S) {
    std::vector<double> a(F, F + n * n);
    sym_eigen(n, a.data(), eps.data(), c.data());
    return;
  }
  std::vector<double> a(S, S + n * n), se(n), su((size_t)(n * n));
  sym_eigen(n, a.data(), se.data(), su.data());
  GF2_REQUIRE(se[0] > 0, GF2_E_ARG, "S is not positive definite");
  std::vector<double> x((size_t)(n * n)), fx((size_t)(n * n)), xfx((size_t)(n * n)), y((size_t)(n * n));
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (int64_t k = 0; k < n; ++k) s += su[i * n + k] * su[j * n + k] / std::sqrt(se[k]);
      x[i * n + j] = s;
    }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (int64_t k = 0; k < n; ++k) s += F[i * n + k] * x[k * n + j];
      fx[i * n + j] = s;
    }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (int64_t k = 0; k < n; ++k) s += x[i * n + k] * fx[k * n + j];
      xfx[i * n + j] = s;
    }
  sym_eigen(n, xfx.data(), eps.data(), y.data());
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (int64_t k = 0; k < n; ++k) s += x[i * n + k] * y[k * n + j];
      c[i * n + j] = s;
    }
}

void run_dd(gf2_ctx* ctx, const gf2_split_h* sp, const double* G, const double* Gb, int64_t ntau,
            double* out);

}  // namespace

// ======================================================================= API

extern "C" {

const char* gf2_version(void) { return "gf2 0.1 (gfx950)"; }

gf2_status gf2_create(gf2_ctx** out, int device, void* stream) {
  if (!out) return GF2_E_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return GF2_E_DEVICE;
  if (device < 0 || device >= ndev) return GF2_E_ARG;
  {
    // the no-allocation entry point's fixed scratch, resolved once per device
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return GF2_E_DEVICE;
    const gf2_status st = noalloc_attach(device);
    (void)hipSetDevice(prev);
    if (st != GF2_OK) return st;
  }
  gf2_ctx* c = new (std::nothrow) gf2_ctx();
  if (!c) return GF2_E_NOMEM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  *out = c;
  return GF2_OK;
}

void gf2_destroy(gf2_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->aux) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  free_scratch(ctx);
  delete ctx;
}

gf2_status gf2_set_gemm_tiles(gf2_ctx* ctx, int32_t mode) {
  if (!ctx || mode < 0 || mode > 2) return GF2_E_ARG;
  ctx->gemm_wide = mode;
  ctx->tiles_tuned.clear();       // an explicit choice replaces the autotuner's
  return GF2_OK;
}

gf2_status gf2_tuned_tiles(gf2_ctx* ctx, gf2_precision prec, int64_t n, int32_t* mode) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(mode && n > 0, GF2_E_ARG, "bad arguments");
    const auto it = ctx->tiles_tuned.find({(int32_t)to_prec(prec), n});
    *mode = it != ctx->tiles_tuned.end() ? it->second : -1;
  });
}

gf2_status gf2_set_stream(gf2_ctx* ctx, void* stream) {
  if (!ctx) return GF2_E_ARG;
  ctx->stream = (hipStream_t)stream;
  return GF2_OK;
}

const char* gf2_last_error(const gf2_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

gf2_status gf2_rng_words(gf2_ctx* ctx, uint64_t seed, uint32_t stream, uint32_t s, uint32_t q0,
                         int64_t count, uint64_t* out) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(out && count >= 0 && stream < 4 && s < (1u << 30), GF2_E_ARG, "bad rng arguments");
    if (count == 0) return;
    auto* d = (uint64_t*)ctx_buf(ctx, "rng", (size_t)count * 8);
    launch_rng_words(seed, stream, s, q0, count, d, ctx->stream);
    GF2_HIP(hipGetLastError());
    d2h(ctx, out, d, (size_t)count);
  });
}

// ------------------------------------------------------------ tau grid ----
gf2_status gf2_tau_grid(double beta, int64_t ntau, double* tau, double* w) {
  if (!(beta > 0) || ntau < 1 || !tau || !w) return GF2_E_ARG;
  std::vector<double> x(ntau), ww(ntau);
  gauss_legendre(ntau, x.data(), ww.data());
  for (int64_t i = 0; i < ntau; ++i) {
    tau[i] = 0.5 * beta * (1.0 + x[i]);
    w[i] = 0.5 * beta * ww[i];
  }
  return GF2_OK;
}

// ------------------------------------------------------------ B -----------
gf2_status gf2_build_B(gf2_ctx* ctx, int64_t n, int64_t naux, const void* ijA, const double* V,
                       const gf2_chain_geom* geom, gf2_dtype out_dtype, void* B) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(n > 0 && naux > 0 && B, GF2_E_ARG, "n, naux must be positive and B non-null");
    GF2_REQUIRE(out_dtype == GF2_F64 || out_dtype == GF2_F32, GF2_E_ARG, "bad dtype");
    const bool f64 = out_dtype == GF2_F64;
    if (!ijA) {
      GF2_REQUIRE(geom && geom->x && geom->xq, GF2_E_ARG, "synthetic mode needs a geometry");
      GF2_REQUIRE(geom->n == n && geom->naux == naux, GF2_E_ARG, "geometry size mismatch");
      auto* dx = (double*)ctx_buf(ctx, "geom_x", (size_t)n * 8);
      auto* dq = (double*)ctx_buf(ctx, "geom_xq", (size_t)naux * 8);
      h2d(ctx, dx, geom->x, (size_t)n);
      h2d(ctx, dq, geom->xq, (size_t)naux);
      launch_synth_b(n, naux, dx, dq, geom->amp, geom->a, geom->c, B, f64, ctx->stream);
      GF2_HIP(hipGetLastError());
      GF2_HIP(hipStreamSynchronize(ctx->stream));
      return;
    }
    const size_t es = f64 ? 8 : 4;
    if (!V) {
      GF2_HIP(hipMemcpyAsync(B, ijA, (size_t)naux * n * n * es, hipMemcpyDeviceToDevice, ctx->stream));
      GF2_HIP(hipStreamSynchronize(ctx->stream));
      return;
    }
    // V^{-1/2} from V's eigendecomposition (FP64, host, O(naux^3) once)
    std::vector<double> a(V, V + naux * naux), e(naux), u((size_t)(naux * naux));
    sym_eigen(naux, a.data(), e.data(), u.data());
    GF2_REQUIRE(e[0] > 0, GF2_E_ARG, "V is not positive definite");
    const int64_t kp = pad_dim(naux);
    const int64_t nn = n * n;
    std::vector<double> w((size_t)(naux * kp), 0.0);    // W[q][A] = V^{-1/2}_{AQ}
    for (int64_t q = 0; q < naux; ++q)
      for (int64_t A = 0; A < naux; ++A) {
        double s = 0.0;
        for (int64_t k = 0; k < naux; ++k) s += u[A * naux + k] * u[q * naux + k] / std::sqrt(e[k]);
        w[q * kp + A] = s;
      }
    // out^T[ij][q] = sum_A ijA^T[ij][A] W[q][A] on the FP64 MFMA GEMM
    auto* wd = (double*)ctx_buf(ctx, "bw", w.size() * 8);
    auto* tin = (double*)ctx_buf(ctx, "bt_in", (size_t)(nn * kp) * 8, true);
    auto* tout = (double*)ctx_buf(ctx, "bt_out", (size_t)(nn * kp) * 8);
    h2d(ctx, wd, w.data(), w.size());
    launch_transpose(ijA, f64, naux, nn, tin, kp, ctx->stream);
    Prob pb = prob0();
    pb.a[0] = opref(tin);
    pb.b[0] = opref(wd);
    pb.nout = 1;
    pb.out[0] = outspec(tout, 0, {1.0f}, 0, 0);
    auto* probs = (Prob*)ctx_buf(ctx, "bprob", sizeof(Prob));
    h2d(ctx, probs, &pb, 1);
    Unit uh{0, 0, 0, 0};
    auto* units = (Unit*)ctx_buf(ctx, "bunit", sizeof(Unit));
    h2d(ctx, units, &uh, 1);
    GemmLaunch L{probs, 1, 0, units, 1, InstGeo{nn, naux, kp, kp, 0}, nullptr, 0, 0, nullptr, 0, 0, 0};
    launch_gemm(Prec::F64, L, tiles_of(pb, Prec::F64, nn, naux), ctx->stream);
    launch_untranspose(tout, nn, naux, kp, B, f64, ctx->stream);
    GF2_HIP(hipGetLastError());
    GF2_HIP(hipStreamSynchronize(ctx->stream));
  });
}

// ------------------------------------------------------------ split -------
namespace {
// eq:K_L on the large-part source L (B itself, or K^L of screened integrals):
// supports, dense blocks and the deterministic-block lists of the elements
// with |L| >= eps max|L|.
gf2_status split_impl(gf2_ctx* ctx, const void* B, const void* L, gf2_dtype dtype, int64_t n, int64_t naux,
                      double eps, gf2_split_h** out, int64_t* nnzL, int64_t* wmax) {
  gf2_split_h* h = nullptr;
  gf2_status st = guarded(ctx, [&] {
    GF2_REQUIRE(out && B && L && n > 0 && naux > 0 && eps >= 0.0 && std::isfinite(eps), GF2_E_ARG,
                "bad split arguments");
    GF2_REQUIRE(n <= 32768 && naux < (1 << 21), GF2_E_ARG, "n or naux too large");
    const bool f64 = dtype == GF2_F64;
    const int64_t total = naux * n * n;
    const int nblk = 1024;
    auto* part = (double*)ctx_buf(ctx, "split_part", nblk * 8);
    launch_maxabs(L, f64, total, part, nblk, ctx->stream);
    GF2_HIP(hipGetLastError());
    std::vector<double> ph(nblk);
    d2h(ctx, ph.data(), part, nblk);
    double kmax = 0.0;
    for (double v : ph) kmax = std::max(kmax, v);
    GF2_REQUIRE(std::isfinite(kmax), GF2_E_NUMERIC, L == B ? "non-finite value in B" : "non-finite value in K^L");
    const double thr = eps * kmax;
    auto* flags = (uint8_t*)ctx_buf(ctx, "split_flags", (size_t)(naux * n));
    auto* cnt = (unsigned long long*)ctx_buf(ctx, "split_cnt", 8, true);
    launch_rowflags(L, f64, n, naux, thr, flags, cnt, ctx->stream);
    GF2_HIP(hipGetLastError());
    std::vector<uint8_t> fh((size_t)(naux * n));
    unsigned long long nnz = 0;
    d2h(ctx, fh.data(), flags, fh.size());
    d2h(ctx, &nnz, cnt, 1);

    h = new gf2_split_h();
    h->owner = ctx; h->bsrc = B; h->lsrc = L == B ? nullptr : L; h->dtype = dtype; h->n = n; h->naux = naux; h->np = pad_dim(n);
    h->eps = eps; h->kmax = kmax; h->thresh = thr; h->nnz = (int64_t)nnz;
    std::vector<int32_t> w(naux, 0), idx((size_t)naux * kWMax, -1);
    int32_t wm = 0;
    for (int64_t q = 0; q < naux; ++q) {
      int32_t c = 0;
      for (int64_t i = 0; i < n; ++i)
        if (fh[q * n + i]) {
          GF2_REQUIRE(c < kWMax, GF2_E_ARG,
                      "support of Q=" + std::to_string(q) + " is wider than 32 orbitals (raise eps)");
          idx[q * kWMax + c++] = (int32_t)i;
        }
      w[q] = c;
      wm = std::max(wm, c);
    }
    h->wmax = wm;
    for (int64_t c0 = 0; c0 < naux; c0 += 128) {
      int32_t lo = (int32_t)n, hi = -1;
      for (int64_t q = c0; q < std::min<int64_t>(naux, c0 + 128); ++q)
        if (w[q] > 0) {
          lo = std::min(lo, idx[q * kWMax]);
          hi = std::max(hi, idx[q * kWMax + w[q] - 1]);
        }
      h->span128 = std::max(h->span128, hi - lo + 1);
    }
    // union pattern with its contribution lists (ordered by Q, a, b)
    std::vector<std::pair<int64_t, int32_t>> contrib;
    for (int64_t q = 0; q < naux; ++q)
      for (int a = 0; a < w[q]; ++a)
        for (int b = 0; b < w[q]; ++b) {
          int64_t i = idx[q * kWMax + a], j = idx[q * kWMax + b];
          contrib.push_back({i * h->np + j, (int32_t)(q * 1024 + a * 32 + b)});
        }
    std::stable_sort(contrib.begin(), contrib.end(),
                     [](const std::pair<int64_t, int32_t>& x, const std::pair<int64_t, int32_t>& y) {
                       return x.first < y.first;
                     });
    std::vector<int32_t> pij, poff, pq;
    for (size_t c = 0; c < contrib.size(); ++c) {
      if (c == 0 || contrib[c].first != contrib[c - 1].first) {
        pij.push_back((int32_t)contrib[c].first);
        poff.push_back((int32_t)c);
      }
      pq.push_back(contrib[c].second);
    }
    poff.push_back((int32_t)contrib.size());
    h->npat = (int64_t)pij.size();
    h->ncontrib = (int64_t)pq.size();
    // Q lists per row block of the deterministic-block tiles
    const int td = dblock_tile();
    const int64_t nbk = (n + td - 1) / td;
    std::vector<std::vector<int32_t>> lists(nbk);
    for (int64_t q = 0; q < naux; ++q) {
      int64_t last = -1;
      for (int a = 0; a < w[q]; ++a) {
        int64_t bk = idx[q * kWMax + a] / td;
        if (bk != last) lists[bk].push_back((int32_t)q);
        last = bk;
      }
    }
    std::vector<int32_t> toff(nbk + 1, 0), tq;
    for (int64_t b = 0; b < nbk; ++b) {
      toff[b] = (int32_t)tq.size();
      tq.insert(tq.end(), lists[b].begin(), lists[b].end());
    }
    toff[nbk] = (int32_t)tq.size();

    // per-orbital (Q, a) lists, Q ascending
    std::vector<int32_t> ooff(n + 1, 0), oq;
    {
      std::vector<std::vector<int32_t>> ol(n);
      for (int64_t q = 0; q < naux; ++q)
        for (int a = 0; a < w[q]; ++a) ol[idx[q * kWMax + a]].push_back((int32_t)((q << 5) | a));
      for (int64_t i = 0; i < n; ++i) {
        ooff[i] = (int32_t)oq.size();
        oq.insert(oq.end(), ol[i].begin(), ol[i].end());
      }
      ooff[n] = (int32_t)oq.size();
    }
    // chunk starts of every orbital's list, at a granularity of 64 Q
    const int32_t ncs = (int32_t)((naux + 63) / 64 + 1);
    std::vector<int32_t> ocs((size_t)(n * ncs));
    for (int64_t i = 0; i < n; ++i) {
      int32_t k = ooff[i];
      for (int32_t c = 0; c < ncs; ++c) {
        while (k < ooff[i + 1] && (oq[k] >> 5) < 64 * c) ++k;
        ocs[(size_t)(i * ncs + c)] = k;
      }
    }
    auto alloc = [&](void** p, size_t bytes) {
      if (bytes == 0) bytes = 16;
      hipError_t e = hipMalloc(p, bytes);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Gf2Error{GF2_E_NOMEM, "split allocation failed"};
      }
    };
    alloc((void**)&h->w, naux * 4);
    alloc((void**)&h->idx, naux * kWMax * 4);
    alloc((void**)&h->blk, naux * kWMax * kWMax * 8);
    alloc((void**)&h->blk32, naux * kWMax * kWMax * 4);
    alloc((void**)&h->pat_ij, pij.size() * 4);
    alloc((void**)&h->pat_off, poff.size() * 4);
    alloc((void**)&h->pat_q, pq.size() * 4);
    alloc((void**)&h->row_off, toff.size() * 4);
    alloc((void**)&h->row_q, tq.size() * 4);
    alloc((void**)&h->orb_off, ooff.size() * 4);
    alloc((void**)&h->orb_q, oq.size() * 4);
    alloc((void**)&h->orb_cs, ocs.size() * 4);
    h->orb_ncs = ncs;
    h2d(ctx, h->orb_cs, ocs.data(), ocs.size());
    h2d(ctx, h->orb_off, ooff.data(), ooff.size());
    if (!oq.empty()) h2d(ctx, h->orb_q, oq.data(), oq.size());
    h2d(ctx, h->w, w.data(), w.size());
    h2d(ctx, h->idx, idx.data(), idx.size());
    if (!pij.empty()) h2d(ctx, h->pat_ij, pij.data(), pij.size());
    h2d(ctx, h->pat_off, poff.data(), poff.size());
    if (!pq.empty()) h2d(ctx, h->pat_q, pq.data(), pq.size());
    h2d(ctx, h->row_off, toff.data(), toff.size());
    if (!tq.empty()) h2d(ctx, h->row_q, tq.data(), tq.size());
    launch_extract_blocks(L, f64, n, naux, thr, h->w, h->idx, h->blk, h->blk32, ctx->stream);
    GF2_HIP(hipGetLastError());
    if (h->wmax <= kDdW) {
      alloc((void**)&h->idx_t, naux * kDdW * 4);
      alloc((void**)&h->blk_t, naux * kDdW * kDdW * 8);
      launch_dd_tables(h->idx, h->blk, naux, h->idx_t, h->blk_t, ctx->stream);
      GF2_HIP(hipGetLastError());
    }
    GF2_HIP(hipStreamSynchronize(ctx->stream));
    *out = h;
    if (nnzL) *nnzL = h->nnz;
    if (wmax) *wmax = h->wmax;
  });
  if (st != GF2_OK && h) {
    gf2_split_free(h);
    if (out) *out = nullptr;
  }
  return st;
}

}  // namespace

gf2_status gf2_split(gf2_ctx* ctx, const void* B, gf2_dtype dtype, int64_t n, int64_t naux, double eps,
                     gf2_split_h** out, int64_t* nnzL, int64_t* wmax) {
  return split_impl(ctx, B, B, dtype, n, naux, eps, out, nnzL, wmax);
}

gf2_status gf2_split_large(gf2_ctx* ctx, const void* B, const void* KL, gf2_dtype dtype, int64_t n,
                           int64_t naux, double eps, gf2_split_h** out, int64_t* nnzL, int64_t* wmax) {
  if (!KL) {
    if (ctx) ctx->err = "KL is null";
    return GF2_E_ARG;
  }
  return split_impl(ctx, B, KL, dtype, n, naux, eps, out, nnzL, wmax);
}

void gf2_split_free(gf2_split_h* h) {
  if (!h) return;
  void* ps[] = {h->w, h->idx, h->blk, h->blk32, h->idx_t, h->blk_t, h->pat_ij, h->pat_off, h->pat_q, h->row_off, h->row_q,
                h->orb_off, h->orb_q, h->orb_cs};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  delete h;
}

gf2_status gf2_screen_ijA(gf2_ctx* ctx, int64_t n, int64_t naux, const void* ijA, gf2_dtype dtype,
                          double eps_prime, void* out, int64_t* nnz) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(n > 0 && naux > 0 && ijA && out, GF2_E_ARG, "bad screening arguments");
    GF2_REQUIRE(dtype == GF2_F64 || dtype == GF2_F32, GF2_E_ARG, "bad dtype");
    GF2_REQUIRE(eps_prime >= 0.0 && std::isfinite(eps_prime), GF2_E_ARG, "eps' must be finite and >= 0");
    auto* mb = (unsigned long long*)ctx_buf(ctx, "scr_max", (size_t)n * 8, true);
    auto* kept = (unsigned long long*)ctx_buf(ctx, "scr_cnt", 8, true);
    launch_screen_ija(ijA, dtype == GF2_F64, n, naux, eps_prime / (double)n, mb, out, kept, ctx->stream);
    GF2_HIP(hipGetLastError());
    unsigned long long k = 0;
    d2h(ctx, &k, kept, 1);
    if (nnz) *nnz = (int64_t)k;
  });
}

gf2_status gf2_split_export(gf2_ctx* ctx, const gf2_split_h* h, int32_t* w, int32_t* idx, double* blk,
                            double* kmax) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(h && h->owner == ctx, GF2_E_STATE, "split handle of another context");
    if (w) d2h(ctx, w, h->w, (size_t)h->naux);
    if (idx) d2h(ctx, idx, h->idx, (size_t)h->naux * kWMax);
    if (blk) d2h(ctx, blk, h->blk, (size_t)h->naux * kWMax * kWMax);
    if (kmax) *kmax = h->kmax;
  });
}

// ------------------------------------------------------------ G(tau) ------
gf2_status gf2_green_tau(gf2_ctx* ctx, int64_t n, const double* F, const double* S, double mu,
                         int64_t n_occ, double beta, int64_t ntau, const double* tau, double* G,
                         double* Gbar, double* mu_out) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(n > 0 && F && tau && G && Gbar && ntau > 0, GF2_E_ARG, "bad green_tau arguments");
    GF2_REQUIRE(beta > 0 && std::isfinite(beta), GF2_E_ARG, "beta must be positive");
    GF2_REQUIRE(n_occ < n, GF2_E_ARG, "n_occ must be < n");
    for (int64_t t = 0; t < ntau; ++t)
      GF2_REQUIRE(tau[t] >= 0 && tau[t] <= beta, GF2_E_ARG, "tau outside [0, beta]");
    std::vector<double> eps, c;
    orbitals_fs(n, F, S, eps, c);
    if (n_occ > 0) mu = 0.5 * (eps[n_occ - 1] + eps[n_occ]);
    if (mu_out) *mu_out = mu;
    GF2_REQUIRE(std::isfinite(mu), GF2_E_ARG, "mu is not finite");
    const int64_t np = pad_dim(n);
    std::vector<double> lw((size_t)(ntau * n)), lb((size_t)(ntau * n));
    for (int64_t t = 0; t < ntau; ++t)
      for (int64_t k = 0; k < n; ++k) {
        const double et = eps[k] - mu;
        lw[t * n + k] = -et * tau[t] - softplus(-beta * et);     // ln[(1-f) e^{-e~ tau}]
        lb[t * n + k] = et * tau[t] - softplus(beta * et);       // ln[f e^{e~ tau}]
      }
    std::vector<double> cp((size_t)(np * np), 0.0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = 0; k < n; ++k) cp[i * np + k] = c[i * n + k];
    auto* dc = (double*)ctx_buf(ctx, "g_c", (size_t)(n * n) * 8);
    auto* dcp = (double*)ctx_buf(ctx, "g_cp", (size_t)(np * np) * 8);
    auto* dlw = (double*)ctx_buf(ctx, "g_lw", (size_t)(ntau * n) * 8);
    auto* da = (double*)ctx_buf(ctx, "g_a", (size_t)(ntau * np * np) * 8);
    auto* dp = (double*)ctx_buf(ctx, "g_p", (size_t)(ntau * np * np) * 8);
    h2d(ctx, dc, c.data(), c.size());
    h2d(ctx, dcp, cp.data(), cp.size());
    Prob pb = prob0();
    pb.a[0] = opref(da, np * np);
    pb.b[0] = opref(dcp);
    pb.nout = 1;
    pb.out[0] = outspec(dp, 0, {1.0f}, 0, 0, np * np);
    auto* probs = (Prob*)ctx_buf(ctx, "g_prob", sizeof(Prob));
    h2d(ctx, probs, &pb, 1);
    std::vector<Unit> uh(ntau);
    for (int64_t t = 0; t < ntau; ++t) uh[t] = mk_unit(t, 0, 0, 0, 0);
    auto* units = (Unit*)ctx_buf(ctx, "g_units", (size_t)ntau * sizeof(Unit));
    h2d(ctx, units, uh.data(), uh.size());
    GemmLaunch L = chain_launch(probs, 1, units, (int32_t)ntau, n, np, 0);
    for (int which = 0; which < 2; ++which) {
      h2d(ctx, dlw, which == 0 ? lw.data() : lb.data(), lw.size());
      launch_scale_cols(dc, dlw, n, np, ntau, da, ctx->stream);
      GF2_HIP(hipGetLastError());
      launch_gemm(Prec::F64, L, tiles_of(pb, Prec::F64, n), ctx->stream);
      launch_unpad_sym(dp, n, np, ntau, -1.0, which == 0 ? G : Gbar, ctx->stream);
      GF2_HIP(hipGetLastError());
    }
    GF2_HIP(hipStreamSynchronize(ctx->stream));
  });
}

// ------------------------------------------------------------ Sigma -------
gf2_status gf2_sigma_det(gf2_ctx* ctx, const gf2_split_h* split, const double* G, const double* Gbar,
                         int64_t ntau, double* Sigma_det) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(split && split->owner == ctx, GF2_E_STATE, "split handle of another context");
    GF2_REQUIRE(G && Gbar && Sigma_det && ntau > 0 && ntau <= 65535, GF2_E_ARG, "bad sigma_det arguments");
    run_dd(ctx, split, G, Gbar, ntau, Sigma_det);
    GF2_HIP(hipStreamSynchronize(ctx->stream));
  });
}

namespace {

// Sigma[D,D] for every tau: the register strip form when supports are at
// most 8 orbitals wide, the LDS tile form otherwise.
void run_dd(gf2_ctx* ctx, const gf2_split_h* sp, const double* G, const double* Gb, int64_t ntau,
            double* out) {
  ProfScope ps(ctx, "dblock");
  if (sp->wmax <= 8) {
    const int64_t per = dd_strip_bytes(sp->n, sp->naux, sp->wmax, 1);
    const int64_t tb = std::max<int64_t>(1, std::min<int64_t>(ntau, (int64_t)2e9 / std::max<int64_t>(per, 1)));
    auto* strip = (double*)ctx_buf(ctx, "dd_strip", (size_t)(per * tb));
    launch_dd_strips(G, Gb, sp->n, sp->naux, ntau, sp->wmax, sp->span128, sp->w, sp->idx, sp->blk, sp->idx_t,
                     sp->blk_t, sp->orb_off, sp->orb_q, sp->orb_cs, sp->orb_ncs, strip, tb, out, ctx->stream);
  } else {
    launch_dblock(G, Gb, sp->n, ntau, sp->wmax, sp->w, sp->idx, sp->blk, sp->row_off, sp->row_q, out,
                  ctx->stream);
  }
}

struct ChainBufs {
  int64_t n, np, np2, plane;
  Prec prec;
  size_t sbytes, abytes;      // bytes of one storage / accumulator matrix
  int32_t slots;
};

// One instance's chain schedule: buffers, problem tables and unit lists,
// set up once; the chunks are then launched by chain_stage / chain_jk /
// chain_acc (one instance) or by the batch path (many instances at once).
struct ChainPlan {
  const gf2_split_h* sp = nullptr;
  Prec prec = Prec::F32;
  int64_t n = 0, np = 0, np2 = 0, naux = 0, ntau = 0, ns = 0, plane = 0;
  bool accf64 = false;
  size_t sb = 0, ab = 0;
  int64_t slots = 0, sc = 0, tcnt = 0;
  int mtiles = 0, ftiles = 0;
  int wideg[4] = {0, 0, 0, 0};    // per launch group: 0 the standard tile, else a 160-wide BF16 tile
  // launch groups of a BF16X3 chain that run as BF16 products on the
  // 160-wide tiles: every K segment A B^T becomes A_hi B_hi + A_hi B_lo +
  // A_lo B_hi, and storage outputs are written as hi and lo planes
  bool xsplit[4] = {false, false, false, false};
  double *mpart = nullptr, *epart = nullptr, *coef = nullptr, *gb64 = nullptr;
  char *wz = nullptr, *jw_l = nullptr, *jw_s = nullptr, *jz_st = nullptr, *jz_sum_t = nullptr, *jblk = nullptr;
  char* sig = nullptr;
  int64_t st_sl = 0, ac_sl = 0;
  std::vector<Prob> P;
  Prob* dprobs = nullptr;
  std::vector<Unit> uall;
  Unit* dunits = nullptr;
  std::vector<std::pair<int64_t, int64_t>> chunks;   // (offset, count) into uall
  std::vector<std::pair<int32_t, int32_t>> trange;   // tau range of each chunk
  double* Sigma_sum = nullptr;
  double* e_samples = nullptr;
  char* mst = nullptr;           // the four M matrices per slot (storage format)
  // estimator: 0 the paired L/S-resolved form, 1 the control-variate form,
  // 2 the double average over every (first-set, second-set) combination
  int variant = 0;
  int64_t npairs = 0;            // pairs of the unit list (ns, or ns^2 for the double average)
  int ngroups = 0;               // product launches per chunk and their problems
  int goff[4] = {0, 0, 0, 0}, gcnt[4] = {0, 0, 0, 0}, gprod[4] = {0, 0, 0, 0};
};

// The product launches of one chunk (first problem, problems, products per
// unit): s1 {U, V^T}, s2 {M_xL, M_xS, W, Z^T}, s3 {T, T}, s4; every problem
// of s1-s3 is a dual-A product.
constexpr int kGroups = 4;
constexpr int kStageOff[kGroups] = {0, 2, 6, 8};
constexpr int kStageCnt[kGroups] = {2, 4, 2, 1};
constexpr int kStageProducts[kGroups] = {4, 8, 4, 8};
constexpr int kProbsPerPlan = 9;
const char* const kGroupTag[kGroups] = {".s1", ".s2", ".s3", ".s4"};

const char* gemm_name(Prec prec) {
  return prec == Prec::F64 ? "gemm_f64" : prec == Prec::F32 ? "gemm_f32"
         : prec == Prec::BF16 ? "gemm_bf16" : "gemm_bf16x3";
}

// Slots (units per chunk) that keep the per-slot scratch near 4 GB.
int64_t auto_slots(int64_t n, Prec prec) {
  const int64_t np = pad_dim(n), np2 = np * np;
  const size_t sb = (size_t)st_planes(prec) * np2 * st_elem(prec);
  const size_t ab = (size_t)np2 * acc_elem(prec);
  const double per_slot = 30.0 * (double)std::max(sb, ab);
  return (int64_t)std::max(1.0, std::min(64.0, 4.0e9 / per_slot));
}

// Chunk length along tau (at most tmax) for chains on the 160-wide BF16
// tiles (BF16, and BF16X3 split into BF16 products).  A launch spreads its
// tiles evenly over the 8 XCDs and runs them on each XCD's CUs in rounds
// (one dual-A workgroup per CU for stages s1-s3, two single-tile workgroups
// for the deep-K stage s4); a round that is only partly filled takes about
// as long as a full one.  The length with the fewest estimated rounds over
// all chunks of the tau axis is taken (rounds of s4, about twice as long,
// counted twice; a small cost per chunk for its other launches); ties go to
// the longer chunk.  Other tiles keep tmax.
int64_t chunk_tau(const gf2_ctx* ctx, Prec prec, int64_t n, int64_t ntau, int64_t sc, int64_t tmax) {
  if (!((prec == Prec::BF16 || prec == Prec::BF16X3) && tile_mode(ctx, prec, n) >= 2 &&
        wide_pads_less(Prec::BF16, n)))
    return tmax;
  const int64_t tw = gemm_tile_n(Prec::BF16, 1);
  const int64_t tpu = ((n + tw - 1) / tw) * ((n + tw - 1) / tw);     // tiles per unit and stage
  int cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
    cus = prop.multiProcessorCount;
  const int64_t per_xcd = std::max(1, cus / 8);
  auto rounds = [&](int64_t units) {
    const int64_t tx = (units * tpu + 7) / 8;                         // tiles on one XCD
    return 3.0 * (double)((tx + per_xcd - 1) / per_xcd) + 2.0 * (double)((tx + 2 * per_xcd - 1) / (2 * per_xcd)) + 0.2;
  };
  int64_t best = tmax;
  double best_cost = 0.0;
  for (int64_t t = tmax; t >= 1; --t) {
    const int64_t full = ntau / t, tail = ntau % t;
    const double cost = (double)full * rounds(sc * t) + (tail ? rounds(sc * tail) : 0.0);
    if (t == tmax || cost < best_cost * (1.0 - 1e-9)) {
      best = t;
      best_cost = cost;
    }
  }
  return best;
}

// Buffers (tags prefixed by pfx), G conversions, stochastic vectors, problem
// tables and unit lists of one instance.  sc / tcnt > 0 force the chunk shape.
void plan_chain(gf2_ctx* ctx, ChainPlan& c, const std::string& pfx, const gf2_split_h* sp, const void* B,
                const double* G, const double* Gbar, int64_t ntau, const gf2_sampling* smp, Prec prec,
                double* Sigma_sum, double* e_samples, int64_t force_sc = 0, int64_t force_tcnt = 0,
                int variant = 0) {
  c.sp = sp;
  c.prec = prec;
  c.variant = variant;
  for (bool& x : c.xsplit) x = false;
  c.n = sp->n;
  c.np = sp->np;
  c.np2 = c.np * c.np;
  c.naux = sp->naux;
  c.ntau = ntau;
  c.ns = smp->ns;
  c.Sigma_sum = Sigma_sum;
  c.e_samples = e_samples;
  const int64_t n = c.n, np = c.np, np2 = c.np2, naux = c.naux, ns = c.ns, s0 = smp->s0;
  const bool bf64 = sp->dtype == GF2_F64;
  const int planes = st_planes(prec);
  c.plane = np2;
  const int64_t plane = c.plane;
  c.sb = (size_t)planes * np2 * st_elem(prec);     // one storage matrix
  c.ab = (size_t)np2 * acc_elem(prec);             // one accumulator matrix
  const size_t sb = c.sb, ab = c.ab;
  c.accf64 = prec == Prec::F64;
  hipStream_t st = ctx->stream;

  // ---- chunking: units (tau, s), s outer so that every Sigma_sum[tau]
  // receives its pairs in increasing s; several pairs per tau in a chunk, so
  // each Sigma_sum[tau] is read and written once per chunk for all of them.
  const int64_t npairs = variant == 2 ? ns * ns : ns;
  c.npairs = npairs;
  int64_t slots = ctx->max_units > 0 ? ctx->max_units : auto_slots(n, prec);
  slots = std::min<int64_t>(slots, ntau * npairs);
  c.sc = force_sc > 0 ? std::min(force_sc, npairs) : std::min<int64_t>(npairs, std::min<int64_t>(8, slots));
  c.tcnt = force_tcnt > 0 ? std::min(force_tcnt, ntau) : std::max<int64_t>(1, std::min<int64_t>(ntau, slots / c.sc));
  if (force_tcnt <= 0 && ctx->max_units <= 0) c.tcnt = chunk_tau(ctx, prec, n, ntau, c.sc, c.tcnt);
  c.slots = slots = c.sc * c.tcnt;

  // The products run over the zero padding of every np x np matrix, and the
  // kernels write only the n x n part: every byte a chain buffer is used
  // with under the current layout (n, np, precision) must have been cleared
  // under that layout.  A change of layout forgets what was cleared; a later
  // call that uses more of a buffer (more slots or vectors) clears the rest.
  const std::string key = std::to_string(n) + ":" + std::to_string(np) + ":" + std::to_string((int)prec);
  std::string& prev = ctx->chain_keys[pfx];
  std::map<std::string, size_t>& cleared = ctx->chain_cleared[pfx];
  if (prev != key) cleared.clear();
  prev = key;
  auto zbuf = [&](const std::string& tag, size_t bytes) {
    if (bytes == 0) bytes = 16;
    const bool grows = ctx->bufs[tag].bytes < bytes;       // a new allocation comes back zeroed
    char* p = (char*)ctx_buf(ctx, tag, bytes);
    size_t& z = cleared[tag];
    if (grows) {
      z = bytes;
    } else if (bytes > z) {
      GF2_HIP(hipMemsetAsync(p + z, 0, bytes - z, ctx->stream));
      z = bytes;
    }
    return p;
  };
  auto CB = [&](const char* tag, size_t bytes) { return zbuf(pfx + tag, bytes); };

  // ---- G, Gbar in padded storage format and FP64
  char* gst = CB("c_gst", sb * ntau);
  char* gbst = CB("c_gbst", sb * ntau);
  c.gb64 = (double*)CB("c_gb64", (size_t)ntau * np2 * 8);
  const int64_t mstride = (int64_t)planes * np2;              // elements per storage matrix
  launch_pad_convert(G, n, np, ntau, prec, gst, plane, mstride, nullptr, st);
  launch_pad_convert(Gbar, n, np, ntau, prec, gbst, plane, mstride, c.gb64, st);
  GF2_HIP(hipGetLastError());

  // ---- stochastic vectors: [0, ns) first vertex (xi), [ns, 2ns) second (eta)
  const int64_t nvec = 2 * ns;
  char* xl = CB("c_xl", sb * nvec);
  char* xs = CB("c_xs", sb * nvec);
  if (smp->mode == GF2_SAMPLE_RADEMACHER) {
    auto* theta = (int8_t*)ctx_buf(ctx, pfx + "c_theta", (size_t)(nvec * naux));
    ProfScope ps(ctx, "rbuild", 4.0 * (double)nvec * naux * n * n, (double)naux * n * n * (bf64 ? 8 : 4));
    launch_theta(smp->seed, ns, s0, naux, theta, st);
    launch_rbuild(B, bf64, n, naux, sp->thresh, theta, nvec, prec, xl, xs, np, plane, mstride, st, nullptr,
                  sp->lsrc);
  } else if (smp->mode == GF2_SAMPLE_STRATIFIED) {
    // class probabilities and their CDF, sequential FP64 sums
    const int32_t nc = smp->k;
    std::vector<double> pi(nc, 0.0), cdf(nc);
    for (int64_t q = 0; q < naux; ++q) pi[q % nc] += smp->p[q];
    double tot = 0.0;
    for (int32_t c = 0; c < nc; ++c) tot += pi[c];
    double acc = 0.0;
    for (int32_t c = 0; c < nc; ++c) {
      pi[c] /= tot;
      acc += pi[c];
      cdf[c] = acc;
    }
    cdf[nc - 1] = 1.0;
    auto* dpi = (double*)ctx_buf(ctx, pfx + "c_pi", (size_t)nc * 8);
    auto* dcdf = (double*)ctx_buf(ctx, pfx + "c_ccdf", (size_t)nc * 8);
    auto* theta = (int8_t*)ctx_buf(ctx, pfx + "c_theta", (size_t)(nvec * naux));
    auto* vsc = (double*)ctx_buf(ctx, pfx + "c_vscale", (size_t)nvec * 8);
    h2d(ctx, dpi, pi.data(), pi.size());
    h2d(ctx, dcdf, cdf.data(), cdf.size());
    ProfScope ps(ctx, "rbuild", 4.0 * (double)nvec * naux * n * n, (double)naux * n * n * (bf64 ? 8 : 4));
    launch_theta_strat(smp->seed, ns, s0, naux, nc, dcdf, dpi, theta, vsc, st);
    launch_rbuild(B, bf64, n, naux, sp->thresh, theta, nvec, prec, xl, xs, np, plane, mstride, st, vsc, sp->lsrc);
  } else {
    std::vector<double> cdf(naux);
    double acc = 0.0;
    for (int64_t q = 0; q < naux; ++q) {
      acc += smp->p[q];
      cdf[q] = acc;
    }
    cdf[naux - 1] = 1.0;
    auto* dcdf = (double*)ctx_buf(ctx, pfx + "c_cdf", (size_t)naux * 8);
    auto* dp = (double*)ctx_buf(ctx, pfx + "c_p", (size_t)naux * 8);
    auto* dq = (int32_t*)ctx_buf(ctx, pfx + "c_q", (size_t)(nvec * smp->k) * 4);
    auto* dw = (double*)ctx_buf(ctx, pfx + "c_w", (size_t)(nvec * smp->k) * 8);
    h2d(ctx, dcdf, cdf.data(), cdf.size());
    h2d(ctx, dp, smp->p, (size_t)naux);
    launch_draws(smp->seed, ns, s0, smp->k, dcdf, naux, dp, dq, dw, st);
    launch_rimportance(B, bf64, n, sp->thresh, dq, dw, smp->k, nvec, prec, xl, xs, np, plane, mstride, st,
                       sp->lsrc);
  }
  GF2_HIP(hipGetLastError());

  // per-slot scratch
  auto S = [&](const char* tag, size_t bytes) { return zbuf(pfx + tag, bytes * slots); };
  char *ul_n = S("c_uln", sb), *ul_t = S("c_ult", sb), *us_n = S("c_usn", sb), *us_t = S("c_ust", sb);
  char *vl_n = S("c_vln", sb), *vs_n = S("c_vsn", sb), *vs_t = S("c_vst", sb), *vsum_t = S("c_vsumt", sb);
  char* mst = S("c_mst", 4 * sb);
  char* mct = S("c_mct", 4 * sb);
  c.wz = S("c_wz", 4 * ab);
  char* wz = c.wz;
  char* tq = S("c_t", 4 * sb);
  c.sig = S("c_sig", ab);
  char* sig = c.sig;
  // pattern-only outputs of JK: zeroed once here, only pattern entries are
  // written (each JK output array is [slot][plane][np][np])
  char* jk = (char*)ctx_buf(ctx, pfx + "c_jk", 4 * sb * slots, true);
  c.jw_l = jk;
  c.jw_s = jk + sb * slots;
  c.jz_st = jk + 2 * sb * slots;
  c.jz_sum_t = jk + 3 * sb * slots;
  char *jw_l = c.jw_l, *jw_s = c.jw_s, *jz_st = c.jz_st, *jz_sum_t = c.jz_sum_t;
  c.jblk = (char*)ctx_buf(ctx, pfx + "c_jblk", jk_block_bytes(c.accf64, slots, naux, sp->wmax));
  c.st_sl = (int64_t)(sb / st_elem(prec));        // elements per storage slot
  c.ac_sl = (int64_t)np2;
  const int64_t st_sl = c.st_sl, ac_sl = c.ac_sl;
  const OpRef g_op = opref(gst, planes * np2);      // G(tau), G(beta - tau): one matrix per tau
  const OpRef gb_op = opref(gbst, planes * np2);

  // ---- problem tables
  const int64_t vst = planes * np2;                            // one vector
  std::vector<Prob>& P = c.P;
  P.clear();
  if (variant == 1) {
    // Control-variate form: chain(R_xi, R_eta) - chain(R^L_xi, R^L_eta) per
    // pair, chain(a, b) = 2 Tr(T) M - T M with M = a G b and T = M Gbar.
    // Full vectors R = R^L + R^S next to the large parts.
    char* xt = CB("c_xt", sb * nvec);
    launch_vec_sum(xl, xs, xt, nvec * mstride, prec, plane, mstride, st);
    c.wideg[0] = c.wideg[1] = c.wideg[2] = c.wideg[3] = 0;
    if (wide_for(ctx, prec, n)) {
      c.wideg[3] = 1;
      if (tile_mode(ctx, prec, n) >= 2) c.wideg[0] = c.wideg[2] = 3;
    } else if (prec == Prec::BF16X3 && tile_mode(ctx, prec, n) >= 1 && wide_pads_less(Prec::BF16, n)) {
      c.wideg[3] = 1;
      c.xsplit[3] = true;
      if (tile_mode(ctx, prec, n) >= 2) {
        c.wideg[0] = c.wideg[2] = 3;
        c.xsplit[0] = c.xsplit[2] = true;
      }
    }
    Prob dual = prob0();
    dual.nA = 2;
    c.mtiles = tiles_of(dual, c.xsplit[2] ? Prec::BF16 : prec, n, c.wideg[2]);
    Prob single = prob0();
    c.ftiles = tiles_of(single, c.xsplit[3] ? Prec::BF16 : prec, n, c.wideg[3]);
    c.mpart = (double*)S("c_mpart", 4 * c.mtiles * 8);
    c.epart = (double*)S("c_epart", c.ftiles * 8);
    c.coef = (double*)S("c_coef", kCoefStride * 8);
    c.mst = mst;
    // s1: U_t = R_xi G, U_L = R^L_xi G (dual-A)
    {
      Prob p = prob0();
      p.nA = 2;
      p.a[0] = opref(xt, 0, vst);
      p.a[1] = opref(xl, 0, vst);
      p.b[0] = g_op;
      p.nout = 2;
      p.out[0] = outspec(ul_n, st_sl, {1, 0}, 0, 1);
      p.out[1] = outspec(us_n, st_sl, {0, 1}, 0, 1);
      P.push_back(p);
    }
    // s2: M_t = U_t R_eta, M_L = U_L R^L_eta, and -M_t^T, +M_L^T for the exchange
    for (int h = 0; h < 2; ++h) {
      Prob p = prob0();
      p.a[0] = opref(h == 0 ? ul_n : us_n, 0, 0, st_sl);
      p.b[0] = opref((h == 0 ? xt : xl) + sb * ns, 0, 0, 0, vst);
      p.nout = 2;
      p.out[0] = outspec(mst + h * sb, 4 * st_sl, {1}, 0, 1);
      p.out[1] = outspec(mct + h * sb, 4 * st_sl, {h == 0 ? -1.0f : 1.0f}, 1, 1);
      P.push_back(p);
    }
    // s3: T = M Gbar for (M_t, M_L) with their traces into mpart[slot][0..1]
    {
      Prob p = prob0();
      p.nA = 2;
      p.a[0] = opref(mst + 0 * sb, 0, 0, 4 * st_sl);
      p.a[1] = opref(mst + 1 * sb, 0, 0, 4 * st_sl);
      p.b[0] = gb_op;
      p.nout = 2;
      p.out[0] = outspec(tq + 0 * sb, 4 * st_sl, {1, 0}, 0, 1);
      p.out[1] = outspec(tq + 1 * sb, 4 * st_sl, {0, 1}, 0, 1);
      p.nhad = 2;
      p.had_diag = 1;
      p.had_coef[0][0] = 1.0f; p.had_coef[0][1] = 0.0f;
      p.had_coef[1][0] = 0.0f; p.had_coef[1][1] = 1.0f;
      p.had_part = c.mpart;
      p.had_ntiles = c.mtiles;
      p.had_slot_stride = 4;
      P.push_back(p);
    }
    // s4: -T_t M_t + T_L M_L (the direct terms join in the accumulation)
    {
      Prob p = prob0();
      p.nseg = 2;
      for (int x = 0; x < 2; ++x) {
        p.a[x] = opref(tq + x * sb, 0, 0, 4 * st_sl);
        p.b[x] = opref(mct + x * sb, 0, 0, 4 * st_sl);
      }
      p.nout = 1;
      p.out[0] = outspec(sig, ac_sl, {1}, 0, 0);
      p.nhad = 1;
      p.had_h = opref(c.gb64, np2);
      p.had_coef[0][0] = 1.0f;
      p.had_part = c.epart;
      p.had_ntiles = c.ftiles;
      p.had_slot_stride = 1;
      P.push_back(p);
    }
    c.ngroups = 4;
    const int go[4] = {0, 1, 3, 4}, gc[4] = {1, 2, 1, 1}, gp[4] = {2, 2, 2, 2};
    for (int g = 0; g < 4; ++g) { c.goff[g] = go[g]; c.gcnt[g] = gc[g]; c.gprod[g] = gp[g]; }
  } else {
    // S1: U = X G (dual A), V = G Y (dual B)
    {
      Prob p = prob0();
      p.nA = 2;
      p.a[0] = opref(xl, 0, vst);
      p.a[1] = opref(xs, 0, vst);
      p.b[0] = g_op;
      p.nout = 4;
      p.out[0] = outspec(ul_n, st_sl, {1, 0}, 0, 1);
      p.out[1] = outspec(ul_t, st_sl, {1, 0}, 1, 1);
      p.out[2] = outspec(us_n, st_sl, {0, 1}, 0, 1);
      p.out[3] = outspec(us_t, st_sl, {0, 1}, 1, 1);
      P.push_back(p);
      // V_c = G Y_c as its transpose Y_c G (G and Y_c symmetric): a dual-A
      // product whose tile holds V_L^T and V_S^T at the same positions
      Prob q = prob0();
      q.nA = 2;
      q.a[0] = opref(xl + sb * ns, 0, 0, 0, vst);
      q.a[1] = opref(xs + sb * ns, 0, 0, 0, vst);
      q.b[0] = g_op;
      q.nout = 4;
      q.out[0] = outspec(vl_n, st_sl, {1, 0}, 1, 1);
      q.out[1] = outspec(vs_n, st_sl, {0, 1}, 1, 1);
      q.out[2] = outspec(vs_t, st_sl, {0, 1}, 0, 1);
      q.out[3] = outspec(vsum_t, st_sl, {1, 1}, 0, 1);
      P.push_back(q);
    }
    if (wide_for(ctx, prec, n)) {
      // 160-wide tiles where they pad n less: the deep-K stage s4 always, the
      // dual-A launches (s1, s2, s3) in the default mode 2
      c.wideg[3] = 1;
      if (tile_mode(ctx, prec, n) >= 2) c.wideg[0] = c.wideg[1] = c.wideg[2] = 3;
    } else if (prec == Prec::BF16X3 && tile_mode(ctx, prec, n) >= 1 && wide_pads_less(Prec::BF16, n)) {
      c.wideg[3] = 1;
      c.xsplit[3] = true;
      if (tile_mode(ctx, prec, n) >= 2) {
        c.wideg[0] = c.wideg[1] = c.wideg[2] = 3;
        c.xsplit[0] = c.xsplit[1] = c.xsplit[2] = true;
      }
    }
    Prob dual = prob0();
    dual.nA = 2;
    c.mtiles = tiles_of(dual, c.xsplit[2] ? Prec::BF16 : prec, n, c.wideg[2]);
    Prob single = prob0();
    c.ftiles = tiles_of(single, c.xsplit[3] ? Prec::BF16 : prec, n, c.wideg[3]);
    c.mpart = (double*)S("c_mpart", 4 * c.mtiles * 8);
    c.epart = (double*)S("c_epart", c.ftiles * 8);
    c.coef = (double*)S("c_coef", kCoefStride * 8);
    c.mst = mst;
    // Matrices of the exchange term, -sum over the nine (T_xy, M_zw) pairs of
    // S_xi x S_eta, grouped into four products whose factors each come from
    // one dual-A tile:
    //   T_SS (M_LL + M_SL) + (T_SL + T_SS)(M_LS + M_SS) + T_LS M_SL + (T_LL + T_LS) M_SS.
    // mst[x] = M_x (x = LL, LS, SL, SS; row-major, the A operands of s3 and
    // the direct terms); mct[x] = the x-th B factor above, negated and
    // transposed; tq[x] = the x-th A factor.
    // S2: M_xL = U_x Y_L and M_xS = U_x Y_S (dual-A over x), W = V Gb (dual-A),
    // Z = Gb U as Z^T = U^T Gb (dual-A)
    for (int y = 0; y < 2; ++y) {
      Prob p = prob0();
      p.nA = 2;
      p.a[0] = opref(ul_n, 0, 0, st_sl);
      p.a[1] = opref(us_n, 0, 0, st_sl);
      p.b[0] = opref((y == 0 ? xl : xs) + sb * ns, 0, 0, 0, vst);
      p.nout = 4;
      const int lx = y == 0 ? 0 : 1, sx = y == 0 ? 2 : 3;      // M_Ly and M_Sy in mst order
      p.out[0] = outspec(mst + lx * sb, 4 * st_sl, {1, 0}, 0, 1);
      p.out[1] = outspec(mst + sx * sb, 4 * st_sl, {0, 1}, 0, 1);
      if (y == 0) {
        p.out[2] = outspec(mct + 0 * sb, 4 * st_sl, {-1, -1}, 1, 1);     // -(M_LL + M_SL)^T
        p.out[3] = outspec(mct + 2 * sb, 4 * st_sl, {0, -1}, 1, 1);      // -M_SL^T
      } else {
        p.out[2] = outspec(mct + 1 * sb, 4 * st_sl, {-1, -1}, 1, 1);     // -(M_LS + M_SS)^T
        p.out[3] = outspec(mct + 3 * sb, 4 * st_sl, {0, -1}, 1, 1);      // -M_SS^T
      }
      P.push_back(p);
    }
    {
      Prob w = prob0();
      w.nA = 2;
      w.a[0] = opref(vl_n, 0, 0, st_sl);
      w.a[1] = opref(vs_n, 0, 0, st_sl);
      w.b[0] = gb_op;
      w.nout = 2;
      w.out[0] = outspec(wz + 0 * ab, 4 * ac_sl, {1, 0}, 0, 0);
      w.out[1] = outspec(wz + 1 * ab, 4 * ac_sl, {0, 1}, 0, 0);
      P.push_back(w);
      // Z_b = Gbar U_b as its transpose U_b^T Gbar (Gbar symmetric): dual-A
      Prob z = prob0();
      z.nA = 2;
      z.a[0] = opref(ul_t, 0, 0, st_sl);
      z.a[1] = opref(us_t, 0, 0, st_sl);
      z.b[0] = gb_op;
      z.nout = 2;
      z.out[0] = outspec(wz + 2 * ab, 4 * ac_sl, {1, 0}, 1, 0);
      z.out[1] = outspec(wz + 3 * ab, 4 * ac_sl, {0, 1}, 1, 0);
      P.push_back(z);
    }
    // S3: T = M Gb for the pairs (M_SS, M_SL) and (M_LS, M_LL), writing the A
    // factors of the exchange term and the traces Tr(T_x) (the diagonal of the
    // FP32 products) into mpart[slot][x][tile]
    for (int h = 0; h < 2; ++h) {
      Prob p = prob0();
      p.nA = 2;
      const int a0 = h == 0 ? 3 : 1, a1 = h == 0 ? 2 : 0;       // (SS, SL) and (LS, LL)
      p.a[0] = opref(mst + a0 * sb, 0, 0, 4 * st_sl);
      p.a[1] = opref(mst + a1 * sb, 0, 0, 4 * st_sl);
      p.b[0] = gb_op;
      p.nout = 2;
      p.out[0] = outspec(tq + (2 * h) * sb, 4 * st_sl, {1, 0}, 0, 1);       // T_SS, T_LS
      p.out[1] = outspec(tq + (2 * h + 1) * sb, 4 * st_sl, {1, 1}, 0, 1);   // T_SL + T_SS, T_LL + T_LS
      p.nhad = 2;
      p.had_diag = 1;
      p.had_coef[0][0] = 0.0f; p.had_coef[0][1] = 1.0f;                     // Tr(T_a1)
      p.had_coef[1][0] = 1.0f; p.had_coef[1][1] = 0.0f;                     // Tr(T_a0)
      p.had_part = c.mpart + (int64_t)std::min(a0, a1) * c.mtiles;         // h slots a1, a0 (a1 < a0)
      p.had_ntiles = c.mtiles;
      p.had_slot_stride = 4;
      P.push_back(p);
    }
    // S4: exchange + cross terms as one K-concatenated product, the trace of
    // that product in the epilogue (the direct terms 2 Tr(T) M join in the
    // accumulation)
    {
      Prob p = prob0();
      p.nseg = 8;
      for (int x = 0; x < 4; ++x) {
        p.a[x] = opref(tq + x * sb, 0, 0, 4 * st_sl);
        p.b[x] = opref(mct + x * sb, 0, 0, 4 * st_sl);
      }
      p.a[4] = opref(jw_l, 0, 0, st_sl);   p.b[4] = opref(vs_t, 0, 0, st_sl);
      p.a[5] = opref(jw_s, 0, 0, st_sl);   p.b[5] = opref(vsum_t, 0, 0, st_sl);
      p.a[6] = opref(ul_n, 0, 0, st_sl);   p.b[6] = opref(jz_st, 0, 0, st_sl);
      p.a[7] = opref(us_n, 0, 0, st_sl);   p.b[7] = opref(jz_sum_t, 0, 0, st_sl);
      p.nout = 1;
      p.out[0] = outspec(sig, ac_sl, {1}, 0, 0);
      p.nhad = 1;
      p.had_h = opref(c.gb64, np2);
      p.had_coef[0][0] = 1.0f;
      p.had_part = c.epart;
      p.had_ntiles = c.ftiles;
      p.had_slot_stride = 1;
      P.push_back(p);
    }
    c.ngroups = kGroups;
    for (int g = 0; g < kGroups; ++g) { c.goff[g] = kStageOff[g]; c.gcnt[g] = kStageCnt[g]; c.gprod[g] = kStageProducts[g]; }
  }
  // Launch groups of a BF16X3 chain on the 160-wide BF16 tiles: each K
  // segment A B^T becomes three BF16 segments A_hi B_hi, A_hi B_lo, A_lo B_hi
  // (a storage matrix's lo plane follows its hi plane at `plane` elements),
  // summed by the FP32 accumulator as the BF16X3 tile sums its products, in
  // another order; storage outputs are written as hi and lo planes (type 2)
  auto lo = [&](OpRef r) {
    r.base = (const char*)r.base + plane * (int64_t)sizeof(uint16_t);
    return r;
  };
  for (int g = 0; g < c.ngroups; ++g) {
    if (!c.xsplit[g]) continue;
    for (int j = 0; j < c.gcnt[g]; ++j) {
      Prob& q = P[c.goff[g] + j];
      const int ns0 = q.nseg;
      OpRef a0[kMaxSeg], b0[kMaxSeg];
      for (int x = 0; x < kMaxSeg; ++x) { a0[x] = q.a[x]; b0[x] = q.b[x]; }
      if (c.wideg[g] == 3) {
        // dual-A: segment x holds a[2x], a[2x + 1] against b[x]
        GF2_REQUIRE(q.nA == 2 && q.nB == 1 && ns0 == 1 && 6 <= kMaxSeg, GF2_E_STATE, "dual-A product to split");
        q.a[0] = a0[0];     q.a[1] = a0[1];     q.b[0] = b0[0];
        q.a[2] = a0[0];     q.a[3] = a0[1];     q.b[1] = lo(b0[0]);
        q.a[4] = lo(a0[0]); q.a[5] = lo(a0[1]); q.b[2] = b0[0];
        q.nseg = 3;
      } else {
        GF2_REQUIRE(q.nA == 1 && q.nB == 1 && 3 * ns0 <= kMaxSeg, GF2_E_STATE, "deep-K stage too long to split");
        for (int x = 0; x < ns0; ++x) {
          q.a[3 * x] = a0[x];         q.b[3 * x] = b0[x];
          q.a[3 * x + 1] = a0[x];     q.b[3 * x + 1] = lo(b0[x]);
          q.a[3 * x + 2] = lo(a0[x]); q.b[3 * x + 2] = b0[x];
        }
        q.nseg = 3 * ns0;
      }
      for (int o = 0; o < q.nout; ++o)
        if (q.out[o].type == 1) q.out[o].type = 2;
    }
  }
  for (int g = 0; g < c.ngroups; ++g)
    for (int j = 0; j < c.gcnt[g]; ++j)
      GF2_REQUIRE(gemm_wide_supports(c.wideg[g], P[c.goff[g] + j]), GF2_E_STATE, "product problem not supported by its tile");
  c.dprobs = (Prob*)ctx_buf(ctx, pfx + "c_probs", P.size() * sizeof(Prob));
  h2d(ctx, c.dprobs, P.data(), P.size());

  // ---- unit lists of all chunks (vector arrays are indexed by s - s0)
  c.uall.clear();
  c.chunks.clear();
  c.trange.clear();
  for (int64_t sbk = 0; sbk < npairs; sbk += c.sc)
    for (int64_t tb = 0; tb < ntau; tb += c.tcnt) {
      const int64_t off0 = (int64_t)c.uall.size();
      int32_t slot = 0;
      const int64_t t1 = std::min(ntau, tb + c.tcnt), s1 = std::min(npairs, sbk + c.sc);
      for (int64_t t = tb; t < t1; ++t)
        for (int64_t p = sbk; p < s1; ++p) {
          // pair p: vectors (p, p), or (p / ns, p mod ns) for the double average
          const int64_t a = variant == 2 ? p / ns : p, b2 = variant == 2 ? p % ns : p;
          c.uall.push_back(mk_unit(t, a, slot++, b2, p));
        }
      c.chunks.push_back({off0, (int64_t)c.uall.size() - off0});
      c.trange.push_back({(int32_t)tb, (int32_t)t1});
    }
  c.dunits = (Unit*)ctx_buf(ctx, pfx + "c_units", c.uall.size() * sizeof(Unit));
  h2d(ctx, c.dunits, c.uall.data(), c.uall.size());
}

void chain_stage(gf2_ctx* ctx, const ChainPlan& c, int stage, int64_t ci) {
  const int off = c.goff[stage], cnt = c.gcnt[stage];
  const int wide = c.wideg[stage];
  // a split BF16X3 launch group runs BF16 products (named as the chain's precision)
  const Prec lp = c.xsplit[stage] ? Prec::BF16 : c.prec;
  int mt = 0;
  for (int i = 0; i < cnt; ++i) mt = std::max(mt, tiles_of(c.P[off + i], lp, c.n, wide));
  const int nu = (int)c.chunks[ci].second;
  GemmLaunch L = chain_launch(c.dprobs + off, cnt, c.dunits + c.chunks[ci].first, nu, c.n, c.np, c.plane);
  L.wide = wide;
  const std::string nm = std::string(gemm_name(c.prec)) + kGroupTag[stage] + (wide ? "@160" : "");
  ProfScope ps(ctx, nm.c_str(), 2.0 * (double)c.n * c.n * c.n * c.gprod[stage] * nu);
  launch_gemm(lp, L, mt, ctx->stream);
}

void chain_jk(gf2_ctx* ctx, const ChainPlan& c, int64_t ci) {
  const gf2_split_h* sp = c.sp;
  const int nu = (int)c.chunks[ci].second;
  {
    ProfScope ps(ctx, "jk_blocks");
    launch_jk_blocks(c.accf64, c.wz, 4 * c.ac_sl, c.ac_sl, c.np, c.naux, nu, sp->wmax, sp->w, sp->idx,
                     c.accf64 ? (const void*)sp->blk : (const void*)sp->blk32, c.jblk, ctx->stream);
  }
  ProfScope ps(ctx, "jk_scatter");
  launch_jk_scatter(c.accf64, c.jblk, c.naux, nu, sp->wmax, sp->npat, sp->pat_ij, sp->pat_off, sp->pat_q, c.np, c.prec,
                    c.plane, c.jw_l, c.jw_s, c.jz_st, c.jz_sum_t, c.st_sl, ctx->stream);
}

void chain_acc(gf2_ctx* ctx, const ChainPlan& c, int64_t ci) {
  const Unit* du = c.dunits + c.chunks[ci].first;
  const int nu = (int)c.chunks[ci].second;
  const int64_t n = c.n;
  launch_trace_coef(c.mpart, c.mtiles, (int32_t)c.slots, c.coef, c.variant == 1 ? 1 : 0, ctx->stream);
  ProfScope ps(ctx, "accumulate", 0.0,
               (double)nu * n * n * (c.accf64 ? 8 : 4) + 2.0 * (c.trange[ci].second - c.trange[ci].first) * n * n * 8);
  launch_accumulate(du, nu, c.sig, c.accf64, c.ac_sl, n, c.np, c.Sigma_sum, c.trange[ci].first,
                    c.trange[ci].second, c.mst, c.prec, 4 * c.st_sl, c.st_sl, c.plane, c.coef, ctx->stream);
  if (c.e_samples) launch_esamples(du, nu, c.epart, c.ftiles, 0, c.ntau, c.e_samples, c.coef, ctx->stream);
}

void run_stoch(gf2_ctx* ctx, const gf2_split_h* sp, const void* B, const double* G, const double* Gbar,
               int64_t ntau, const gf2_sampling* smp, Prec prec, double* Sigma_sum, double* e_samples,
               int variant = 0) {
  ChainPlan c;
  plan_chain(ctx, c, "", sp, B, G, Gbar, ntau, smp, prec, Sigma_sum, e_samples, 0, 0, variant);
  for (size_t ci = 0; ci < c.chunks.size(); ++ci) {
    for (int g = 0; g < c.ngroups; ++g) {
      chain_stage(ctx, c, g, (int64_t)ci);
      if (g == 1 && c.variant != 1) chain_jk(ctx, c, (int64_t)ci);   // the control-variate form has no J/K
    }
    chain_acc(ctx, c, (int64_t)ci);
    GF2_HIP(hipGetLastError());
  }
  GF2_HIP(hipStreamSynchronize(ctx->stream));
}

// run_stoch at a gf2_precision: BF16C is the two-level estimator -- every
// pair in BF16, the first k = min(ns, kLevelProbe) pairs also in BF16X3, and
// Sigma_sum and the per-pair traces moved by the mean BF16X3 - BF16
// difference of those pairs (ns / k times their summed difference).
void run_stoch_prec(gf2_ctx* ctx, const gf2_split_h* sp, const void* B, const double* G, const double* Gbar,
                    int64_t ntau, const gf2_sampling* smp, gf2_precision prec, double* Sigma_sum,
                    double* e_samples) {
  if (prec != GF2_PREC_BF16C) {
    run_stoch(ctx, sp, B, G, Gbar, ntau, smp, to_prec(prec), Sigma_sum, e_samples);
    return;
  }
  const int64_t ns = smp->ns, k = std::min<int64_t>(ns, kLevelProbe);
  const size_t mat = (size_t)(ntau * sp->n * sp->n);
  auto* lo = (double*)ctx_buf(ctx, "l_lo", mat * 8, true);
  auto* hi = (double*)ctx_buf(ctx, "l_hi", mat * 8, true);
  auto* ehi = (double*)ctx_buf(ctx, "l_ehi", (size_t)(k * ntau) * 8);
  auto* elo = e_samples ? e_samples : (double*)ctx_buf(ctx, "l_elo", (size_t)(k * ntau) * 8);
  gf2_sampling part = *smp;
  part.ns = k;
  run_stoch(ctx, sp, B, G, Gbar, ntau, &part, Prec::BF16, lo, elo);
  run_stoch(ctx, sp, B, G, Gbar, ntau, &part, Prec::BF16X3, hi, ehi);
  if (ns > k) {
    part.s0 = smp->s0 + k;
    part.ns = ns - k;
    run_stoch(ctx, sp, B, G, Gbar, ntau, &part, Prec::BF16, Sigma_sum, e_samples ? e_samples + k * ntau : nullptr);
  }
  launch_level_correct(Sigma_sum, hi, lo, (int64_t)mat, (double)ns / (double)k, ctx->stream);
  if (e_samples) launch_level_shift(e_samples, ehi, k, ns, ntau, ctx->stream);
  GF2_HIP(hipGetLastError());
}

void check_sampling(const gf2_split_h* sp, const gf2_sampling* s) {
  GF2_REQUIRE(s, GF2_E_ARG, "sampling is null");
  GF2_REQUIRE(s->ns >= 1 && s->s0 >= 0 && s->s0 + s->ns <= (1 << 30), GF2_E_ARG, "bad ns / s0");
  GF2_REQUIRE(s->mode == GF2_SAMPLE_RADEMACHER || s->mode == GF2_SAMPLE_IMPORTANCE ||
                  s->mode == GF2_SAMPLE_STRATIFIED, GF2_E_ARG, "bad mode");
  if (s->mode == GF2_SAMPLE_STRATIFIED)
    GF2_REQUIRE(s->k >= 2 && s->k <= sp->naux, GF2_E_ARG, "stratified sampling needs 2 <= classes <= naux");
  if (s->mode != GF2_SAMPLE_RADEMACHER) {
    if (s->mode == GF2_SAMPLE_IMPORTANCE) GF2_REQUIRE(s->k >= 1 && s->k <= 64, GF2_E_ARG, "k must be in [1, 64]");
    GF2_REQUIRE(s->p, GF2_E_ARG, "importance mode needs p");
    double tot = 0.0;
    for (int64_t q = 0; q < sp->naux; ++q) {
      GF2_REQUIRE(s->p[q] > 0 && std::isfinite(s->p[q]), GF2_E_ARG, "proposal must be positive");
      tot += s->p[q];
    }
    GF2_REQUIRE(std::fabs(tot - 1.0) < 1e-6, GF2_E_ARG, "proposal must sum to 1");
  }
}

}  // namespace

gf2_status gf2_sigma_stoch(gf2_ctx* ctx, const gf2_split_h* split, const void* B, const double* G,
                           const double* Gbar, int64_t ntau, const gf2_sampling* sampling,
                           gf2_precision prec, double* Sigma_sum, double* e_samples) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(split && split->owner == ctx, GF2_E_STATE, "split handle of another context");
    GF2_REQUIRE(B == split->bsrc, GF2_E_STATE, "split handle belongs to a different B");
    GF2_REQUIRE(G && Gbar && Sigma_sum && ntau > 0 && ntau <= 4096, GF2_E_ARG, "bad sigma arguments");
    check_sampling(split, sampling);
    run_stoch_prec(ctx, split, B, G, Gbar, ntau, sampling, prec, Sigma_sum, e_samples);
  });
}

gf2_status gf2_sigma_stoch_cv(gf2_ctx* ctx, const gf2_split_h* split, const void* B, const double* G,
                              const double* Gbar, int64_t ntau, const gf2_sampling* sampling, gf2_precision prec,
                              double* Sigma_sum, double* e_samples) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(split && split->owner == ctx, GF2_E_STATE, "split handle of another context");
    GF2_REQUIRE(B == split->bsrc, GF2_E_STATE, "split handle belongs to a different B");
    GF2_REQUIRE(G && Gbar && Sigma_sum && ntau > 0 && ntau <= 4096, GF2_E_ARG, "bad sigma arguments");
    check_sampling(split, sampling);
    run_stoch(ctx, split, B, G, Gbar, ntau, sampling, to_prec(prec), Sigma_sum, e_samples, 1);
  });
}

gf2_status gf2_sigma_stoch_double(gf2_ctx* ctx, const gf2_split_h* split, const void* B, const double* G,
                                  const double* Gbar, int64_t ntau, const gf2_sampling* sampling,
                                  gf2_precision prec, double* Sigma_sum, double* e_samples) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(split && split->owner == ctx, GF2_E_STATE, "split handle of another context");
    GF2_REQUIRE(B == split->bsrc, GF2_E_STATE, "split handle belongs to a different B");
    GF2_REQUIRE(G && Gbar && Sigma_sum && ntau > 0 && ntau <= 4096, GF2_E_ARG, "bad sigma arguments");
    check_sampling(split, sampling);
    GF2_REQUIRE(sampling->ns <= 256, GF2_E_ARG, "the double average takes at most 256 vectors per set");
    run_stoch(ctx, split, B, G, Gbar, ntau, sampling, to_prec(prec), Sigma_sum, e_samples, 2);
  });
}

gf2_status gf2_energy_double(gf2_ctx* ctx, int64_t n, int64_t ntau, const double* w, const double* Sigma,
                             const double* Gbar, const double* e_samples, int64_t ns, double n_elec, double* E_tot,
                             double* E_per_e, double* stderr_tot) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(n > 0 && ntau > 0 && ntau <= 512 && w && Sigma && Gbar && e_samples, GF2_E_ARG,
                "bad energy arguments");
    GF2_REQUIRE(n_elec > 0 && ns >= 2 && ns <= 256, GF2_E_ARG, "n_elec > 0 and 2 <= ns <= 256");
    auto* tr = (double*)ctx_buf(ctx, "e_tr", (size_t)ntau * 8);
    auto* dw = (double*)ctx_buf(ctx, "e_w", (size_t)ntau * 8);
    auto* res = (double*)ctx_buf(ctx, "e_res", 4 * 8);
    h2d(ctx, dw, w, (size_t)ntau);
    launch_trace_prod(Sigma, Gbar, n, ntau, tr, ctx->stream);
    launch_double_stats(tr, dw, ntau, e_samples, ns, kGM, res, ctx->stream);
    GF2_HIP(hipGetLastError());
    double h[4];
    d2h(ctx, h, res, 3);
    GF2_REQUIRE(std::isfinite(h[0]) && std::isfinite(h[2]), GF2_E_NUMERIC, "non-finite energy");
    if (E_tot) *E_tot = h[0];
    if (E_per_e) *E_per_e = h[0] / n_elec;
    if (stderr_tot) *stderr_tot = h[2];
  });
}

gf2_status gf2_sigma_finalize(gf2_ctx* ctx, int64_t n, int64_t ntau, const double* Sigma_det,
                              const double* Sigma_sum, int64_t ns_total, double* Sigma) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(n > 0 && ntau > 0 && ns_total > 0 && Sigma_det && Sigma_sum && Sigma, GF2_E_ARG,
                "bad finalize arguments");
    launch_finalize(Sigma_det, Sigma_sum, n, ntau, 0.5 / (double)ns_total, Sigma, ctx->stream);
    GF2_HIP(hipGetLastError());
    check_finite(ctx, Sigma, ntau * n * n, "Sigma");
  });
}

gf2_status gf2_sigma_tau(gf2_ctx* ctx, const gf2_split_h* split, const void* B, const double* G,
                         const double* Gbar, int64_t ntau, const gf2_sampling* sampling, gf2_precision prec,
                         double* Sigma, double* e_samples) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(split && split->owner == ctx, GF2_E_STATE, "split handle of another context");
    GF2_REQUIRE(B == split->bsrc, GF2_E_STATE, "split handle belongs to a different B");
    GF2_REQUIRE(G && Gbar && Sigma && ntau > 0 && ntau <= 4096, GF2_E_ARG, "bad sigma arguments");
    check_sampling(split, sampling);
    const int64_t n = split->n;
    const size_t bytes = (size_t)(ntau * n * n) * 8;
    auto* det = (double*)ctx_buf(ctx, "t_det", bytes);
    auto* sum = (double*)ctx_buf(ctx, "t_sum", bytes, true);
    run_dd(ctx, split, G, Gbar, ntau, det);
    run_stoch_prec(ctx, split, B, G, Gbar, ntau, sampling, prec, sum, e_samples);
    launch_finalize(det, sum, n, ntau, 0.5 / (double)sampling->ns, Sigma, ctx->stream);
    GF2_HIP(hipGetLastError());
    check_finite(ctx, Sigma, ntau * n * n, "Sigma");
  });
}

// ------------------------------------------------------------ energy ------
gf2_status gf2_energy(gf2_ctx* ctx, int64_t n, int64_t ntau, const double* w, const double* Sigma,
                      const double* Gbar, const double* e_samples, int64_t ns, double n_elec, double* E_tot,
                      double* E_per_e, double* stderr_tot) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(n > 0 && ntau > 0 && ntau <= 512 && w && Sigma && Gbar, GF2_E_ARG, "bad energy arguments");
    GF2_REQUIRE(n_elec > 0, GF2_E_ARG, "n_elec must be positive");
    GF2_REQUIRE(!e_samples || ns >= 2, GF2_E_ARG, "a standard error needs ns >= 2");
    auto* tr = (double*)ctx_buf(ctx, "e_tr", (size_t)ntau * 8);
    auto* dw = (double*)ctx_buf(ctx, "e_w", (size_t)ntau * 8);
    auto* res = (double*)ctx_buf(ctx, "e_res", 4 * 8);
    h2d(ctx, dw, w, (size_t)ntau);
    launch_trace_prod(Sigma, Gbar, n, ntau, tr, ctx->stream);
    launch_energy_stats(tr, dw, ntau, e_samples, e_samples ? ns : 0, kGM, res, ctx->stream);
    GF2_HIP(hipGetLastError());
    double h[4];
    d2h(ctx, h, res, 3);
    GF2_REQUIRE(std::isfinite(h[0]) && std::isfinite(h[2]), GF2_E_NUMERIC, "non-finite energy");
    if (E_tot) *E_tot = h[0];
    if (E_per_e) *E_per_e = h[0] / n_elec;
    if (stderr_tot) *stderr_tot = h[2];
  });
}

// ------------------------------------------------------------ batch -------
namespace {

struct BatchShape {
  int32_t tcnt, persist;
};

// All instances' chunks in lockstep: step c runs chunk c of every instance
// that has one; the product stages of a step are single launches over the
// units of all instances (largest instances first).
struct BatchRun {
  std::vector<ChainPlan> plans;
  Prob* dprobs = nullptr;          // [ninst][kProbsPerPlan]
  InstGeo* dgeo = nullptr;         // [ninst]
  Unit* dunits = nullptr;          // all steps' merged unit lists
  std::vector<std::pair<int64_t, int64_t>> steps;   // (offset, count) into dunits
  int tiles[kGroups] = {0, 0, 0, 0};      // per launch group, max over instances
  BatchSeg* dsegs = nullptr;       // work lists of all (step, stage)
  std::vector<int64_t> segoff, nseg, nitems;         // per step * kGroups + group
  int64_t nsteps = 0;
  int32_t persist = 0;
};

void batch_plan(gf2_ctx* ctx, BatchRun& R, int32_t nitem, const gf2_batch_item* items, Prec prec,
                const std::vector<double*>& sums, BatchShape shape) {
  R.plans.assign(nitem, ChainPlan());
  for (int32_t i = 0; i < nitem; ++i) {
    const gf2_batch_item& it = items[i];
    plan_chain(ctx, R.plans[i], "b" + std::to_string(i) + ":", it.split, it.B, it.G, it.Gbar, it.ntau,
               &it.sampling, prec, sums[i], it.e_samples, 8, shape.tcnt);
  }
  std::vector<Prob> ph((size_t)nitem * kProbsPerPlan);
  std::vector<InstGeo> gh(nitem);
  for (int32_t i = 0; i < nitem; ++i) {
    const ChainPlan& c = R.plans[i];
    for (int j = 0; j < kProbsPerPlan; ++j) ph[(size_t)i * kProbsPerPlan + j] = c.P[j];
    gh[i] = InstGeo{c.n, c.n, c.np, c.np, c.plane};
    for (int st = 0; st < kGroups; ++st)
      for (int j = 0; j < kStageCnt[st]; ++j)
        R.tiles[st] = std::max(R.tiles[st], tiles_of(c.P[kStageOff[st] + j], prec, c.n));
  }
  R.dprobs = (Prob*)ctx_buf(ctx, "bt_probs", ph.size() * sizeof(Prob));
  R.dgeo = (InstGeo*)ctx_buf(ctx, "bt_geo", gh.size() * sizeof(InstGeo));
  h2d(ctx, R.dprobs, ph.data(), ph.size());
  h2d(ctx, R.dgeo, gh.data(), gh.size());
  // merged units, instances by decreasing size within each step
  std::vector<int32_t> order(nitem);
  for (int32_t i = 0; i < nitem; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return R.plans[a].n > R.plans[b].n; });
  R.nsteps = 0;
  for (const ChainPlan& c : R.plans) R.nsteps = std::max<int64_t>(R.nsteps, (int64_t)c.chunks.size());
  // per instance and stage: tiles of its largest problem of the stage
  std::vector<std::array<int32_t, kGroups>> itiles(nitem);
  for (int32_t i = 0; i < nitem; ++i)
    for (int st = 0; st < kGroups; ++st) {
      int32_t t = 0;
      for (int j = 0; j < kStageCnt[st]; ++j) t = std::max(t, tiles_of(R.plans[i].P[kStageOff[st] + j], prec, R.plans[i].n));
      itiles[i][st] = t;
    }
  std::vector<Unit> uh;
  std::vector<BatchSeg> sh;
  R.steps.clear();
  R.segoff.clear();
  R.nseg.clear();
  R.nitems.clear();
  for (int64_t st = 0; st < R.nsteps; ++st) {
    const int64_t off0 = (int64_t)uh.size();
    std::vector<std::pair<int32_t, std::pair<int32_t, int32_t>>> runs;   // (inst, (unit0, nunits))
    for (int32_t i : order) {
      const ChainPlan& c = R.plans[i];
      if (st >= (int64_t)c.chunks.size()) continue;
      const int32_t u0 = (int32_t)(uh.size() - off0);
      for (int64_t q = 0; q < c.chunks[st].second; ++q) {
        Unit u = c.uall[c.chunks[st].first + q];
        u.inst = i;
        uh.push_back(u);
      }
      runs.push_back({i, {u0, (int32_t)c.chunks[st].second}});
    }
    R.steps.push_back({off0, (int64_t)uh.size() - off0});
    for (int stage = 0; stage < kGroups; ++stage) {
      R.segoff.push_back((int64_t)sh.size());
      int64_t item = 0;
      for (const auto& r : runs) {
        if (R.plans[r.first].wideg[stage]) continue;   // launched on its own (wide tile)
        const int32_t t = itiles[r.first][stage];
        sh.push_back(BatchSeg{item, r.second.first, r.second.second, t, 0});
        item += (int64_t)r.second.second * kStageCnt[stage] * t;
      }
      R.nseg.push_back((int64_t)(sh.size() - R.segoff.back()));
      R.nitems.push_back(item);
    }
  }
  R.dsegs = (BatchSeg*)ctx_buf(ctx, "bt_segs", std::max<size_t>(1, sh.size()) * sizeof(BatchSeg));
  if (!sh.empty()) h2d(ctx, R.dsegs, sh.data(), sh.size());
  R.dunits = (Unit*)ctx_buf(ctx, "bt_units", uh.size() * sizeof(Unit));
  h2d(ctx, R.dunits, uh.data(), uh.size());
  R.persist = shape.persist;
}

// Launch steps [s0, s1) of the batch (kernels only: no allocation, copy or
// fill, so the sequence can be recorded into a graph).
void batch_steps(gf2_ctx* ctx, const BatchRun& R, Prec prec, int64_t s0, int64_t s1) {
  GF2_REQUIRE(0 <= s0 && s0 <= s1 && s1 <= R.nsteps && R.nsteps == (int64_t)R.steps.size(), GF2_E_STATE,
              "batch step range out of bounds");
  for (int64_t st = s0; st < s1; ++st) {
    const int nu = (int)R.steps[st].second;
    for (int stage = 0; stage < kGroups; ++stage) {
      const int64_t k = st * kGroups + stage;
      GemmLaunch L{R.dprobs + kStageOff[stage], kStageCnt[stage], kProbsPerPlan, R.dunits + R.steps[st].first, nu,
                   InstGeo{0, 0, 0, 0, 0}, R.dgeo, 0, R.persist, R.dsegs + R.segoff[k], (int32_t)R.nseg[k],
                   R.nitems[k]};
      double fl = 0.0;
      for (const ChainPlan& c : R.plans)
        if (st < (int64_t)c.chunks.size() && !c.wideg[stage])
          fl += 2.0 * (double)c.n * c.n * c.n * kStageProducts[stage] * c.chunks[st].second;
      {
        const std::string nm = std::string(gemm_name(prec)) + kGroupTag[stage];
        ProfScope ps(ctx, nm.c_str(), fl);
        launch_gemm(prec, L, R.tiles[stage], ctx->stream);
      }
      // instances whose launch group runs on a wide tile, one launch each
      for (const ChainPlan& c : R.plans)
        if (c.wideg[stage] && st < (int64_t)c.chunks.size()) chain_stage(ctx, c, stage, st);
      if (stage == 1)
        for (const ChainPlan& c : R.plans)
          if (st < (int64_t)c.chunks.size()) chain_jk(ctx, c, st);
    }
    for (const ChainPlan& c : R.plans)
      if (st < (int64_t)c.chunks.size()) chain_acc(ctx, c, st);
  }
}

std::string batch_signature(int32_t nitem, const gf2_batch_item* items, Prec prec) {
  std::string sig = std::to_string((int)prec);
  for (int32_t i = 0; i < nitem; ++i)
    sig += ";" + std::to_string(items[i].split->n) + "," + std::to_string(items[i].ntau) + "," +
           std::to_string(items[i].sampling.ns);
  return sig;
}

}  // namespace

gf2_status gf2_sigma_batch(gf2_ctx* ctx, int32_t nitem, const gf2_batch_item* items, gf2_precision prec,
                           int32_t flags) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(nitem >= 1 && items, GF2_E_ARG, "empty batch");
    const Prec p = to_prec(prec);
    for (int32_t i = 0; i < nitem; ++i) {
      const gf2_batch_item& it = items[i];
      GF2_REQUIRE(it.split && it.split->owner == ctx, GF2_E_STATE, "split handle of another context");
      GF2_REQUIRE(it.B == it.split->bsrc, GF2_E_STATE, "split handle belongs to a different B");
      GF2_REQUIRE(it.G && it.Gbar && it.Sigma && it.ntau > 0 && it.ntau <= 4096, GF2_E_ARG,
                  "bad batch item " + std::to_string(i));
      check_sampling(it.split, &it.sampling);
    }
    // deterministic blocks and zeroed sums
    std::vector<double*> dets(nitem), sums(nitem);
    for (int32_t i = 0; i < nitem; ++i) {
      const int64_t n = items[i].split->n;
      const size_t bytes = (size_t)(items[i].ntau * n * n) * 8;
      dets[i] = (double*)ctx_buf(ctx, "b" + std::to_string(i) + ":det", bytes);
      sums[i] = (double*)ctx_buf(ctx, "b" + std::to_string(i) + ":sum", bytes, true);
      run_dd(ctx, items[i].split, items[i].G, items[i].Gbar, items[i].ntau, dets[i]);
    }
    // launch shape: tuned (cached per signature) or the default
    BatchShape shape{8, 0};
    const std::string sig = batch_signature(nitem, items, p);
    auto hit = ctx->tuned.find(sig);
    if (hit != ctx->tuned.end()) {
      shape = BatchShape{hit->second.first, hit->second.second};
    } else if (flags & GF2_BATCH_AUTOTUNE) {
      int dev_cus = 256;
      hipDeviceProp_t prop;
      if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) dev_cus = prop.multiProcessorCount;
      const bool prof = ctx->prof;
      ctx->prof = false;
      // time per unit of a plan: warm with step 0, time steps [t0, t1)
      // (step 0 again if it is the only one)
      auto per_unit = [&](int32_t cnt, const gf2_batch_item* its, const std::vector<double*>& sm, BatchShape cs) {
        BatchRun R;
        batch_plan(ctx, R, cnt, its, p, sm, cs);
        const int64_t t0 = R.nsteps >= 2 ? 1 : 0;
        const int64_t t1 = R.nsteps >= 2 ? std::min<int64_t>(R.nsteps, 4) : 1;
        batch_steps(ctx, R, p, 0, 1);
        hipEvent_t a, b;
        GF2_HIP(hipEventCreate(&a));
        GF2_HIP(hipEventCreate(&b));
        GF2_HIP(hipEventRecord(a, ctx->stream));
        batch_steps(ctx, R, p, t0, t1);
        GF2_HIP(hipEventRecord(b, ctx->stream));
        GF2_HIP(hipEventSynchronize(b));
        float ms = 0.0f;
        GF2_HIP(hipEventElapsedTime(&ms, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        int64_t units = 0;
        for (int64_t st = t0; st < t1; ++st) units += R.steps[st].second;
        return units > 0 ? ms / (double)units : 1e300;
      };
      // 1. tile mode per chain size where it matters (BF16 sizes a 160-wide
      // tile pads less): each mode timed on the first chain of that size
      // alone, the fastest kept for the size
      std::map<int64_t, int32_t> first_of;
      for (int32_t i = 0; i < nitem; ++i)
        if (wide_pads_less(p, items[i].split->n)) first_of.emplace(items[i].split->n, i);
      for (const auto& fo : first_of) {
        const std::pair<int32_t, int64_t> key{(int32_t)p, fo.first};
        if (ctx->tiles_tuned.count(key)) continue;
        int32_t pick = ctx->gemm_wide;
        double tbest = 1e300;
        for (int32_t m = 0; m <= 2; ++m) {
          ctx->tiles_tuned[key] = m;
          const double t = per_unit(1, items + fo.second, {sums[fo.second]}, BatchShape{8, 0});
          if (t < tbest) {
            tbest = t;
            pick = m;
          }
        }
        ctx->tiles_tuned[key] = pick;
      }
      // 2. launch shape of the whole batch with those tiles
      const BatchShape cand[] = {{8, 0}, {4, 0}, {2, 0}, {8, 2 * dev_cus}, {4, 2 * dev_cus}};
      double best = 1e300;
      for (const BatchShape& cs : cand) {
        const double t = per_unit(nitem, items, sums, cs);
        if (t < best) {
          best = t;
          shape = cs;
        }
      }
      ctx->prof = prof;
      ctx->tuned[sig] = {shape.tcnt, shape.persist};
      // the trial steps added to the sums: start again from zero
      for (int32_t i = 0; i < nitem; ++i)
        sums[i] = (double*)ctx_buf(ctx, "b" + std::to_string(i) + ":sum",
                                   (size_t)(items[i].ntau * items[i].split->n * items[i].split->n) * 8, true);
    }
    BatchRun R;
    batch_plan(ctx, R, nitem, items, p, sums, shape);
    if (flags & GF2_BATCH_GRAPH) {
      // record on a stream of our own (the caller's may be the legacy
      // default stream, which cannot capture), launch on the caller's
      GF2_HIP(hipStreamSynchronize(ctx->stream));
      hipStream_t cap = nullptr;
      GF2_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      const bool prof = ctx->prof;
      hipStream_t user = ctx->stream;
      ctx->prof = false;                       // no event records inside the graph
      ctx->stream = cap;
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        try {
          batch_steps(ctx, R, p, 0, R.nsteps);
        } catch (...) {
          (void)hipStreamEndCapture(cap, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          ctx->stream = user;
          ctx->prof = prof;
          (void)hipStreamDestroy(cap);
          throw;
        }
        e = hipStreamEndCapture(cap, &graph);
      }
      ctx->stream = user;
      ctx->prof = prof;
      if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (e == hipSuccess) e = hipGraphLaunch(exec, ctx->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipStreamDestroy(cap);
      GF2_HIP(e);
    } else {
      batch_steps(ctx, R, p, 0, R.nsteps);
    }
    for (int32_t i = 0; i < nitem; ++i) {
      const int64_t n = items[i].split->n, ntau = items[i].ntau;
      launch_finalize(dets[i], sums[i], n, ntau, 0.5 / (double)items[i].sampling.ns, items[i].Sigma, ctx->stream);
      GF2_HIP(hipGetLastError());
      check_finite(ctx, items[i].Sigma, ntau * n * n, "Sigma");
    }
    GF2_HIP(hipStreamSynchronize(ctx->stream));
  });
}

// ------------------------------------------------------------ adaptive ----
namespace {
// One-sided 95% upper confidence bound of a standard error estimated from
// `pairs` samples: se * sqrt(k / chi2_{0.05}(k)), k = pairs - 1, with the
// chi-square quantile from the Wilson-Hilferty cube-root normal
// approximation (Wilson & Hilferty 1931): chi2_p(k) = k (1 - 2/(9k) +
// z_p sqrt(2/(9k)))^3, z_0.05 = -1.6448536.  At k = 7 it is 2.15 (tables:
// 2.17), so the bound is 1.80 se.
double stderr_upper(double se, int64_t pairs) {
  const double k = (double)(pairs - 1);
  const double a = 2.0 / (9.0 * k);
  const double c = 1.0 - a - 1.6448536269514722 * std::sqrt(a);
  if (c <= 0.0) return std::numeric_limits<double>::infinity();   // too few samples for a bound
  return se * std::sqrt(k / (k * c * c * c));
}
}  // namespace

namespace {

// Waits for the context's second stream when it goes out of scope, so that
// no work of a call is left running on it after the call returns or throws.
struct AuxJoin {
  gf2_ctx* ctx;
  bool on = false;
  hipEvent_t ev = nullptr;
  ~AuxJoin() {
    if (on) (void)hipStreamSynchronize(ctx->aux);
    if (ev) (void)hipEventDestroy(ev);
  }
};

// The adaptive loop.  With det_out, Sigma[D,D] is computed into det_out on
// the context's second stream while the first batch of pairs runs on the
// main stream; the main stream waits for it before its first read (the
// energy statistics), so the results equal gf2_sigma_det followed by the
// plain adaptive call.
void adaptive_core(gf2_ctx* ctx, const gf2_split_h* split, const void* B, const double* G, const double* Gbar,
                   int64_t ntau, const double* w, const double* Sigma_det_in, double* det_out, double n_elec,
                   const gf2_sampling* sampling, gf2_precision prec, double target, int64_t max_pairs,
                   double* Sigma, double* e_samples, gf2_adaptive_result* res) {
  const double* Sigma_det = det_out ? det_out : Sigma_det_in;
  {
    GF2_REQUIRE(split && split->owner == ctx, GF2_E_STATE, "split handle of another context");
    GF2_REQUIRE(B == split->bsrc, GF2_E_STATE, "split handle belongs to a different B");
    GF2_REQUIRE(G && Gbar && w && Sigma_det && Sigma && e_samples && res, GF2_E_ARG, "bad adaptive arguments");
    GF2_REQUIRE(ntau > 0 && ntau <= 512 && n_elec > 0 && target > 0 && max_pairs >= 2, GF2_E_ARG,
                "bad adaptive arguments (ntau <= 512, target > 0, max_pairs >= 2)");
    check_sampling(split, sampling);
    const bool autop = prec == GF2_PREC_AUTO;
    GF2_REQUIRE(!autop || sampling->ns >= 2, GF2_E_ARG, "AUTO needs batches of at least 2 pairs");
    Prec wp = autop ? Prec::BF16 : to_prec(prec);
    const int64_t n = split->n, batch = sampling->ns;
    const size_t mat = (size_t)(ntau * n * n);
    auto* sum = (double*)ctx_buf(ctx, "a_sum", mat * 8, true);
    auto* tr = (double*)ctx_buf(ctx, "a_tr", (size_t)ntau * 8);
    auto* dw = (double*)ctx_buf(ctx, "a_w", (size_t)ntau * 8);
    auto* stats = (double*)ctx_buf(ctx, "a_stats", 4 * 8);
    h2d(ctx, dw, w, (size_t)ntau);
    AuxJoin join{ctx};
    hipEvent_t det_done = nullptr;
    if (det_out) {
      if (!ctx->aux) GF2_HIP(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
      hipEvent_t ready = nullptr;
      GF2_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
      GF2_HIP(hipEventRecord(ready, ctx->stream));               // G, Gbar, split in place
      GF2_HIP(hipStreamWaitEvent(ctx->aux, ready, 0));
      (void)hipEventDestroy(ready);
      join.on = true;
      hipStream_t main = ctx->stream;
      ctx->stream = ctx->aux;
      try {
        run_dd(ctx, split, G, Gbar, ntau, det_out);
      } catch (...) {
        ctx->stream = main;
        throw;
      }
      ctx->stream = main;
      GF2_HIP(hipEventCreateWithFlags(&join.ev, hipEventDisableTiming));
      det_done = join.ev;
      GF2_HIP(hipEventRecord(det_done, ctx->aux));
    }
    bool have_tr = false;
    auto ensure_tr = [&] {                // Tr(Sigma_det Gbar) per tau
      if (have_tr) return;
      if (det_done) {
        GF2_HIP(hipStreamWaitEvent(ctx->stream, det_done, 0));
        det_done = nullptr;
      }
      launch_trace_prod(Sigma_det, Gbar, n, ntau, tr, ctx->stream);
      GF2_HIP(hipGetLastError());
      have_tr = true;
    };
    gf2_sampling smp = *sampling;
    auto run = [&](int64_t s0, int64_t cnt, Prec p) {
      smp.s0 = s0;
      smp.ns = cnt;
      run_stoch(ctx, split, B, G, Gbar, ntau, &smp, p, sum, e_samples + s0 * ntau);
    };
    auto stat = [&](int64_t pairs, double* h) {
      ensure_tr();
      launch_energy_stats(tr, dw, ntau, e_samples, pairs, kGM, stats, ctx->stream, true);
      GF2_HIP(hipGetLastError());
      d2h(ctx, h, stats, 3);
      GF2_HIP(hipStreamSynchronize(ctx->stream));
      GF2_REQUIRE(std::isfinite(h[0]) && std::isfinite(h[2]), GF2_E_NUMERIC, "non-finite energy");
    };
    // AUTO (two-level estimator): every pair runs in BF16; the first kp
    // pairs also run in BF16X3.  Their differences d_q = BF16X3 - BF16 (per
    // pair energy and per-tau trace) estimate the BF16 rounding bias, which
    // is removed from the final mean; the correction's own uncertainty is
    // std(d)/sqrt(kp).  The probe starts with kAutoProbe0 pairs and grows to
    // kLevelProbe only when the correction is not precise enough at the
    // error reached (loose targets stop after the small probe).
    const int64_t kmax = autop ? std::min<int64_t>(kLevelProbe, max_pairs) : 0;
    int64_t kp = autop ? std::min<int64_t>(kAutoProbe0, kmax) : 0;
    double* psum16 = nullptr;
    double* psum3 = nullptr;
    double* eprobe = nullptr;
    double* psum16x = nullptr;                // BF16 sums of probe pairs that also sit in `sum`
    std::vector<double> dE, de;              // per probe pair: energy, and [kp][ntau] traces
    std::vector<double> eh;                  // per probe pair: its BF16X3 energy
    double bias = 0.0;
    int64_t pairs = 0;
    // BF16X3 into psum3 for probe pairs [k0, k1) (and, with lo, BF16 into
    // lo; without, their BF16 traces are those the sampling already left in
    // e_samples); their trace differences appended to dE / de
    auto probe = [&](int64_t k0, int64_t k1, double* lo) {
      smp.s0 = k0;
      smp.ns = k1 - k0;
      if (lo) run_stoch(ctx, split, B, G, Gbar, ntau, &smp, Prec::BF16, lo, e_samples + k0 * ntau);
      run_stoch(ctx, split, B, G, Gbar, ntau, &smp, Prec::BF16X3, psum3, eprobe + k0 * ntau);
      const int64_t cnt = k1 - k0;
      std::vector<double> lv((size_t)(cnt * ntau)), hv((size_t)(cnt * ntau));
      d2h(ctx, lv.data(), e_samples + k0 * ntau, lv.size());
      d2h(ctx, hv.data(), eprobe + k0 * ntau, hv.size());
      dE.resize((size_t)k1, 0.0);
      eh.resize((size_t)k1, 0.0);
      de.resize((size_t)(k1 * ntau), 0.0);
      for (int64_t q = 0; q < cnt; ++q)
        for (int64_t t = 0; t < ntau; ++t) {
          de[(k0 + q) * ntau + t] = hv[q * ntau + t] - lv[q * ntau + t];
          dE[k0 + q] += -kGM * w[t] * de[(k0 + q) * ntau + t];
          eh[k0 + q] += -kGM * w[t] * hv[q * ntau + t];
        }
      double m = 0.0;
      for (int64_t q = 0; q < k1; ++q) m += dE[q];
      bias = std::fabs(m / (double)k1);
    };
    if (autop) {
      psum16 = (double*)ctx_buf(ctx, "a_probe_lo", mat * 8, true);
      psum3 = (double*)ctx_buf(ctx, "a_probe_hi", mat * 8, true);
      eprobe = (double*)ctx_buf(ctx, "a_probe_e", (size_t)(kmax * ntau) * 8);
      probe(0, kp, psum16);
      pairs = kp;
      // Early decision.  While the probe holds every pair, the correction's
      // uncertainty std(d)/sqrt(kp) and the standard error std(E)/sqrt(pairs)
      // fall together, so their ratio on the first probe (the spread of its
      // BF16X3 energies standing in for the error the batch will reach) is
      // what a larger probe would see too.  Far above the bar, BF16 would be
      // rejected after the batch anyway: the probe pairs' BF16X3 sums and
      // traces become the samples and the sampling goes on in BF16X3.
      if (kp >= 2) {
        auto sd = [&](const std::vector<double>& x) {
          double m = 0.0, v = 0.0;
          for (int64_t q = 0; q < kp; ++q) m += x[q];
          m /= (double)kp;
          for (int64_t q = 0; q < kp; ++q) v += (x[q] - m) * (x[q] - m);
          return std::sqrt(v / (double)(kp - 1));
        };
        const double unc2 = 2.0 * sd(dE);
        if (unc2 > 0.0 && unc2 > kAutoEarly * 0.1 * sd(eh)) {
          wp = Prec::BF16X3;
          GF2_HIP(hipMemcpyAsync(sum, psum3, mat * 8, hipMemcpyDeviceToDevice, ctx->stream));
          GF2_HIP(hipMemcpyAsync(e_samples, eprobe, (size_t)(kp * ntau) * 8, hipMemcpyDeviceToDevice,
                                 ctx->stream));
        }
      }
    }
    // sample mean and standard error of the mean of x[0..k)
    auto mean_se = [](const double* x, int64_t k, int64_t stride) {
      double m = 0.0, v = 0.0;
      for (int64_t q = 0; q < k; ++q) m += x[q * stride];
      m /= (double)k;
      for (int64_t q = 0; q < k; ++q) v += (x[q * stride] - m) * (x[q * stride] - m);
      return std::make_pair(m, k > 1 ? std::sqrt(v / (double)(k - 1) / (double)k) : INFINITY);
    };
    // The corrected BF16 mean is accepted if twice the correction's
    // uncertainty is below 0.1x the standard error of the total, and, for
    // every tau, below the larger of 0.1x the standard error of the mean
    // trace and 1e-5 of the trace Tr(Sigma(tau) Gbar(tau)) itself (the FP32
    // path's relative tolerance; at tau points where the stochastic part
    // vanishes its standard error does too).
    auto bf16_ok = [&](int64_t np_, double se_tot) {
      if (2.0 * mean_se(dE.data(), kp, 1).second >= 0.1 * se_tot) return false;
      ensure_tr();
      std::vector<double> es((size_t)(np_ * ntau)), trh((size_t)ntau);
      d2h(ctx, es.data(), e_samples, es.size());
      d2h(ctx, trh.data(), tr, trh.size());
      for (int64_t t = 0; t < ntau; ++t) {
        const auto st_ = mean_se(es.data() + t, np_, ntau);
        const double bar = std::max(0.1 * st_.second, 1e-5 * std::fabs(trh[t] + st_.first));
        if (2.0 * mean_se(de.data() + t, kp, ntau).second >= bar) return false;
      }
      return true;
    };
    double h[4] = {0, 0, 0, 0};
    const int64_t first = std::max<int64_t>(2, std::min(batch, max_pairs));   // the first test, as without AUTO
    while (true) {
      if (pairs >= first) {
        stat(pairs, h);
        bool done = stderr_upper(h[2], pairs) < target || pairs >= max_pairs;
        if (done && autop && wp == Prec::BF16 && !bf16_ok(pairs, h[2]) && kp < std::min(kmax, pairs)) {
          // a larger probe: pairs [kp, k1) ran in BF16 inside `sum` (their
          // traces are in e_samples), so only their BF16X3 level runs now;
          // their separate BF16 sums are made only if the correction is used
          const int64_t k1 = std::min(kmax, pairs);
          probe(kp, k1, nullptr);
          kp = k1;
        }
        if (done && autop && wp == Prec::BF16 && !bf16_ok(pairs, h[2])) {
          // the correction is not precise enough at this error: every pair
          // in BF16X3 (same theta) -- the probe pairs have their BF16X3 sums
          // and traces already, the others are redone -- and go on sampling
          // in BF16X3
          wp = Prec::BF16X3;
          GF2_HIP(hipMemcpyAsync(sum, psum3, mat * 8, hipMemcpyDeviceToDevice, ctx->stream));
          GF2_HIP(hipMemcpyAsync(e_samples, eprobe, (size_t)(kp * ntau) * 8, hipMemcpyDeviceToDevice, ctx->stream));
          for (int64_t s0 = kp; s0 < pairs; s0 += batch) run(s0, std::min(batch, pairs - s0), wp);
          stat(pairs, h);
          done = stderr_upper(h[2], pairs) < target || pairs >= max_pairs;
        }
        if (done) break;
      }
      // batches of `batch` pairs; the first one is filled up after the probe
      const int64_t cnt = std::min(pairs < batch ? batch - pairs : batch, max_pairs - pairs);
      if (cnt <= 0) break;
      run(pairs, cnt, wp);
      pairs += cnt;
    }
    if (autop && wp == Prec::BF16) {
      // Sigma_sum and the samples to the BF16X3 level: with lo the BF16 sums
      // of all kp probe pairs, sum += psum16 + (pairs/kp)(hi - lo); the
      // pairs the probe grew by (psum16x, their BF16 sums, made here) are
      // already in `sum`, so they enter only through lo
      const int64_t kp0 = std::min<int64_t>(kAutoProbe0, kmax);
      if (kp > kp0) {
        psum16x = (double*)ctx_buf(ctx, "a_probe_lox", mat * 8, true);
        smp.s0 = kp0;
        smp.ns = kp - kp0;
        run_stoch(ctx, split, B, G, Gbar, ntau, &smp, Prec::BF16, psum16x, e_samples + kp0 * ntau);
      }
      const double c = (double)pairs / (double)kp;
      launch_level_correct(sum, psum3, psum16, (int64_t)mat, c, ctx->stream);
      if (psum16x) {
        auto* zero = (double*)ctx_buf(ctx, "a_zero", mat * 8, true);
        launch_level_correct(sum, zero, psum16x, (int64_t)mat, 1.0 + c, ctx->stream);   // sum -= c psum16x
      }
      launch_level_shift(e_samples, eprobe, kp, pairs, ntau, ctx->stream);
      GF2_HIP(hipGetLastError());
      stat(pairs, h);
    } else if (autop) {
      bias = 0.0;                 // every pair ran in BF16X3: nothing corrected
    }
    ensure_tr();
    launch_finalize(Sigma_det, sum, n, ntau, 0.5 / (double)pairs, Sigma, ctx->stream);
    GF2_HIP(hipGetLastError());
    check_finite(ctx, Sigma, (int64_t)mat, "Sigma");
    res->e_corr = h[0];
    res->e_corr_per_e = h[0] / n_elec;
    res->stderr_tot = h[2];
    res->pairs = pairs;
    res->precision = wp == Prec::F64 ? GF2_PREC_FP64 : wp == Prec::F32 ? GF2_PREC_FP32
                     : wp == Prec::BF16 ? (autop ? GF2_PREC_BF16C : GF2_PREC_BF16) : GF2_PREC_BF16X3;
    res->bias_probe = bias;
  }
}

}  // namespace

gf2_status gf2_energy_adaptive(gf2_ctx* ctx, const gf2_split_h* split, const void* B, const double* G,
                               const double* Gbar, int64_t ntau, const double* w, const double* Sigma_det,
                               double n_elec, const gf2_sampling* sampling, gf2_precision prec, double target,
                               int64_t max_pairs, double* Sigma, double* e_samples, gf2_adaptive_result* res) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(Sigma_det, GF2_E_ARG, "bad adaptive arguments");
    adaptive_core(ctx, split, B, G, Gbar, ntau, w, Sigma_det, nullptr, n_elec, sampling, prec, target, max_pairs,
                  Sigma, e_samples, res);
  });
}

gf2_status gf2_energy_adaptive_det(gf2_ctx* ctx, const gf2_split_h* split, const void* B, const double* G,
                                   const double* Gbar, int64_t ntau, const double* w, double n_elec,
                                   const gf2_sampling* sampling, gf2_precision prec, double target,
                                   int64_t max_pairs, double* Sigma_det, double* Sigma, double* e_samples,
                                   gf2_adaptive_result* res) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(Sigma_det && G && Gbar && ntau > 0 && ntau <= 65535, GF2_E_ARG, "bad adaptive arguments");
    adaptive_core(ctx, split, B, G, Gbar, ntau, w, nullptr, Sigma_det, n_elec, sampling, prec, target, max_pairs,
                  Sigma, e_samples, res);
  });
}

gf2_status gf2_debug_gemm(gf2_ctx* ctx, gf2_precision prec, int64_t n, int64_t batch, const void* A,
                          const void* Bt, void* C) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(n > 0 && batch > 0 && batch <= 65535 && A && Bt && C, GF2_E_ARG, "bad gemm arguments");
    const Prec p = to_prec(prec);
    const int64_t ld = pad_dim(n), ld2 = ld * ld;
    const int64_t st = st_planes(p) * ld2;
    Prob pb = prob0();
    pb.a[0] = opref(A, 0, st);
    pb.b[0] = opref(Bt, 0, st);
    pb.nout = 1;
    pb.out[0] = outspec(C, 0, {1.0f}, 0, 0);
    pb.out[0].st_s = ld2;
    auto* probs = (Prob*)ctx_buf(ctx, "dbg_prob", sizeof(Prob));
    h2d(ctx, probs, &pb, 1);
    std::vector<Unit> uh(batch);
    for (int64_t b = 0; b < batch; ++b) uh[b] = mk_unit(0, b, 0, b, b);
    auto* units = (Unit*)ctx_buf(ctx, "dbg_units", uh.size() * sizeof(Unit));
    h2d(ctx, units, uh.data(), uh.size());
    GemmLaunch L = chain_launch(probs, 1, units, (int32_t)batch, n, ld, ld2);
    L.wide = wide_for(ctx, p, n);      // the tile the chain's single-product stage would use
    ProfScope ps(ctx, "debug_gemm", 2.0 * (double)n * n * n * batch);
    launch_gemm(p, L, tiles_of(pb, p, n, L.wide), ctx->stream);
  });
}

gf2_status gf2_set_profiling(gf2_ctx* ctx, int on) {
  if (!ctx) return GF2_E_ARG;
  ctx->prof = on != 0;
  return GF2_OK;
}

gf2_status gf2_profile_read(gf2_ctx* ctx, int32_t cap, char* names, int64_t* launches, double* total_ms,
                            double* flops, double* bytes, int32_t* count) {
  return guarded(ctx, [&] {
    GF2_HIP(hipStreamSynchronize(ctx->stream));
    std::vector<std::string> order;
    std::map<std::string, std::tuple<int64_t, double, double, double>> agg;
    for (auto& e : ctx->events) {
      float ms = 0.0f;
      GF2_HIP(hipEventElapsedTime(&ms, e.a, e.b));
      if (!agg.count(e.name)) order.push_back(e.name);
      auto& t = agg[e.name];
      std::get<0>(t) += 1;
      std::get<1>(t) += ms;
      std::get<2>(t) += e.flops;
      std::get<3>(t) += e.bytes;
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    ctx->events.clear();
    int32_t k = 0;
    for (auto& nm : order) {
      if (k >= cap) break;
      auto& t = agg[nm];
      if (names) {
        std::memset(names + 32 * k, 0, 32);
        std::strncpy(names + 32 * k, nm.c_str(), 31);
      }
      if (launches) launches[k] = std::get<0>(t);
      if (total_ms) total_ms[k] = std::get<1>(t);
      if (flops) flops[k] = std::get<2>(t);
      if (bytes) bytes[k] = std::get<3>(t);
      ++k;
    }
    if (count) *count = k;
  });
}

// ------------------------------------------------------------ proposal ----
gf2_status gf2_proposal_features(gf2_ctx* ctx, const gf2_split_h* split, const void* B, const double* x,
                                 const double* xq, const double* Gbeta, double* phi) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(split && split->owner == ctx, GF2_E_STATE, "split handle of another context");
    GF2_REQUIRE(B == split->bsrc, GF2_E_STATE, "split handle belongs to a different B");
    GF2_REQUIRE(x && xq && Gbeta && phi, GF2_E_ARG, "bad feature arguments");
    auto* dx = (double*)ctx_buf(ctx, "pf_x", (size_t)split->n * 8);
    auto* dq = (double*)ctx_buf(ctx, "pf_xq", (size_t)split->naux * 8);
    h2d(ctx, dx, x, (size_t)split->n);
    h2d(ctx, dq, xq, (size_t)split->naux);
    launch_features(B, split->dtype == GF2_F64, split->n, split->naux, split->thresh, dx, dq, Gbeta, phi,
                    ctx->stream);
    GF2_HIP(hipGetLastError());
    GF2_HIP(hipStreamSynchronize(ctx->stream));
  });
}

gf2_status gf2_proposal_targets(gf2_ctx* ctx, const gf2_split_h* split, const void* B, const double* G,
                                const double* Gbar, int64_t ntau, const double* w, double rel, double* t,
                                double* tables) {
  gf2_split_h* bt = nullptr;
  gf2_status st = guarded(ctx, [&] {
    GF2_REQUIRE(split && split->owner == ctx, GF2_E_STATE, "split handle of another context");
    GF2_REQUIRE(B == split->bsrc, GF2_E_STATE, "split handle belongs to a different B");
    GF2_REQUIRE(G && Gbar && w && t && ntau > 0 && rel > 0 && rel < 1, GF2_E_ARG, "bad target arguments");
    GF2_REQUIRE(split->naux <= 8192, GF2_E_ARG, "targets need naux <= 8192");
  });
  if (st != GF2_OK) return st;
  // truncated B on its numerical support, as a split with threshold rel
  int64_t nnz = 0, wb = 0;
  st = gf2_split(ctx, B, split->dtype, split->n, split->naux, rel, &bt, &nnz, &wb);
  if (st != GF2_OK) return st;
  st = guarded(ctx, [&] {
    const int64_t naux = split->naux;
    auto* dw = (double*)ctx_buf(ctx, "pt_w", (size_t)ntau * 8);
    h2d(ctx, dw, w, (size_t)ntau);
    double* tab = tables ? tables : (double*)ctx_buf(ctx, "pt_tab", (size_t)(4 * naux * naux) * 8);
    launch_pair_tables(std::max<int>((int)wb, split->wmax), G, Gbar, split->n, ntau, dw, naux, bt->w, bt->idx,
                       bt->blk, split->w, split->idx, split->blk, tab, ctx->stream);
    launch_targets(tab, naux, t, ctx->stream);
    GF2_HIP(hipGetLastError());
    GF2_HIP(hipStreamSynchronize(ctx->stream));
  });
  gf2_split_free(bt);
  return st;
}

gf2_status gf2_proposal_init(gf2_ctx* ctx, gf2_mlp* mlp, const double* phi, int64_t ntotal, uint64_t seed) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(mlp && phi && ntotal > 0, GF2_E_ARG, "bad init arguments");
    launch_mlp_init(phi, ntotal, seed, *mlp, ctx->stream);
    GF2_HIP(hipGetLastError());
    GF2_HIP(hipStreamSynchronize(ctx->stream));
    mlp->step = 0;
  });
}

namespace {
void mlp_run(gf2_ctx* ctx, const gf2_mlp* mlp, int32_t nchains, const int64_t* chain_off, const double* phi,
             const double* t_hat, int32_t steps, double lr, double* loss, double* grad) {
  GF2_REQUIRE(mlp && chain_off && phi && t_hat && nchains > 0 && nchains <= 1024, GF2_E_ARG,
              "bad network arguments (1 <= nchains <= 1024)");
  const int64_t ntotal = chain_off[nchains];
  GF2_REQUIRE(ntotal > 0, GF2_E_ARG, "empty training set");
  for (int32_t c = 0; c < nchains; ++c) GF2_REQUIRE(chain_off[c] <= chain_off[c + 1], GF2_E_ARG, "bad offsets");
  auto* coff = (int64_t*)ctx_buf(ctx, "mlp_off", (size_t)(nchains + 1) * 8);
  auto* z = (float*)ctx_buf(ctx, "mlp_z", (size_t)ntotal * 4);
  auto* dz = (float*)ctx_buf(ctx, "mlp_dz", (size_t)ntotal * 4);
  auto* g = (double*)ctx_buf(ctx, "mlp_g", (size_t)mlp_nparam() * 8);
  auto* l = (double*)ctx_buf(ctx, "mlp_l", (size_t)std::max(1, steps) * 8);
  h2d(ctx, coff, chain_off, (size_t)nchains + 1);
  {
    ProfScope ps(ctx, steps > 0 ? "mlp_train" : "mlp_grad");
    launch_mlp_train(*mlp, nchains, coff, phi, t_hat, steps, (float)lr, mlp->step, z, dz, g, l, ctx->stream);
  }
  GF2_HIP(hipGetLastError());
  if (loss) d2h(ctx, loss, l, (size_t)std::max(1, steps));
  if (grad) d2h(ctx, grad, g, (size_t)mlp_nparam());
  GF2_HIP(hipStreamSynchronize(ctx->stream));
}
}  // namespace

gf2_status gf2_proposal_grad(gf2_ctx* ctx, const gf2_mlp* mlp, int32_t nchains, const int64_t* chain_off,
                             const double* phi, const double* t_hat, double* loss, double* grad) {
  return guarded(ctx, [&] { mlp_run(ctx, mlp, nchains, chain_off, phi, t_hat, 0, 0.0, loss, grad); });
}

gf2_status gf2_proposal_train(gf2_ctx* ctx, gf2_mlp* mlp, int32_t nchains, const int64_t* chain_off,
                              const double* phi, const double* t_hat, int32_t steps, double lr, double* loss_hist) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(steps > 0 && lr > 0, GF2_E_ARG, "steps and lr must be positive");
    mlp_run(ctx, mlp, nchains, chain_off, phi, t_hat, steps, lr, loss_hist, nullptr);
    mlp->step += steps;
  });
}

gf2_status gf2_proposal_infer(gf2_ctx* ctx, const gf2_mlp* mlp, const double* phi, int64_t naux, double alpha,
                              int32_t bf16, double* p) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(mlp && phi && p && naux > 0 && alpha > 0 && alpha <= 1, GF2_E_ARG,
                "bad inference arguments (0 < alpha <= 1 keeps p > 0)");
    auto* z = (float*)ctx_buf(ctx, "mlp_zi", (size_t)naux * 4);
    ProfScope ps(ctx, "mlp_infer");
    launch_mlp_infer(*mlp, phi, naux, bf16, alpha, z, p, ctx->stream);
    GF2_HIP(hipGetLastError());
    GF2_HIP(hipStreamSynchronize(ctx->stream));
  });
}


// ------------------------------------------------------------ SCF --------
// The steps on either side of Sigma(tau) that make GF2 self-consistent
// (Section III), in the orthonormal eigenbasis of (F, S).
namespace {

struct ScfGrid {
  int64_t n = 0, np = 0, ntau = 0, nw = 0, nc = 0, ncp = 0, nchunk = 0, nto = 0, ntop = 0;
  double beta = 0.0;
  std::vector<double> eps, c, tau;
  double* sig = nullptr;     // Sigma~(tau) [ntau][np][np]
  double* ph = nullptr;      // [nchunk][ntau][ncp][2]: w_t (cos, sin)(w_f tau_t)
  double* cs = nullptr;      // [nchunk][ncp][ntop][2]: (cos, sin)(w_f tau_o), tau_ntau = beta
  double* om = nullptr;      // [nchunk][ncp]
  double* a = nullptr;       // [nc][2][np][np]
  double* colbuf = nullptr;  // [nc][2][np][32]
  double* pbuf = nullptr;    // [nc][2][32][32]
  double* tr = nullptr;      // [nchunk * nc][2]: trace of D and its mu-derivative
  double* shift = nullptr;   // [np]
  int* err = nullptr;
};

constexpr size_t kScfChunkBytes = size_t(1) << 31;   // Dyson matrices of one frequency chunk

// Upload C (padded) and C^T, transform Sigma(tau) to Sigma~ = C^T Sigma C on
// the FP64 MFMA GEMM, and tabulate the phases of both transforms.
void scf_prepare(gf2_ctx* ctx, ScfGrid& g, int64_t n, const double* F, const double* S, double beta, int64_t ntau,
                 const double* tau, const double* w, const double* Sigma, int64_t nw, bool need_back,
                 bool dyson = true) {
  GF2_REQUIRE(n > 0 && F && tau && w && Sigma && ntau > 0 && nw > 0, GF2_E_ARG, "bad Dyson arguments");
  GF2_REQUIRE(beta > 0 && std::isfinite(beta), GF2_E_ARG, "beta must be positive");
  for (int64_t t = 0; t < ntau; ++t)
    GF2_REQUIRE(tau[t] >= 0 && tau[t] <= beta, GF2_E_ARG, "tau outside [0, beta]");
  orbitals_fs(n, F, S, g.eps, g.c);
  g.n = n;
  g.np = pad_dim(n);
  g.ntau = ntau;
  g.nw = nw;
  g.beta = beta;
  g.tau.assign(tau, tau + ntau);
  const int64_t np = g.np, np2 = np * np, fg = scf_freq_group(), og = scf_time_group();
  // one chunk of all nw frequencies when no Dyson matrices are formed
  g.nc = dyson ? std::max<int64_t>(1, std::min<int64_t>({nw, 4096, (int64_t)(kScfChunkBytes / (size_t)(16 * np2))}))
               : nw;
  g.ncp = (g.nc + fg - 1) / fg * fg;
  g.nchunk = (nw + g.nc - 1) / g.nc;
  g.nto = ntau + 1;
  g.ntop = (g.nto + og - 1) / og * og;
  // eigenvectors, padded, and their transpose
  std::vector<double> cp((size_t)np2, 0.0), ctp((size_t)np2, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = 0; k < n; ++k) {
      cp[i * np + k] = g.c[i * n + k];
      ctp[k * np + i] = g.c[i * n + k];
    }
  auto* dcp = (double*)ctx_buf(ctx, "scf_cp", (size_t)np2 * 8);
  auto* dct = (double*)ctx_buf(ctx, "scf_ct", (size_t)np2 * 8);
  h2d(ctx, dcp, cp.data(), cp.size());
  h2d(ctx, dct, ctp.data(), ctp.size());
  // Sigma~ = C^T Sigma C: Y = C^T Sigma (A = C^T, B = Sigma, Sigma symmetric),
  // then Sigma~ = Y C (A = Y, B = C^T).  The GEMM writes only the n x n part
  // of its outputs: their padding is cleared first, since Y is read again as
  // an operand over the padded length and Sigma~ in full by the quadrature.
  auto* spad = (double*)ctx_buf(ctx, "scf_spad", (size_t)(ntau * np2) * 8);
  auto* y = (double*)ctx_buf(ctx, "scf_y", (size_t)(ntau * np2) * 8, true);
  g.sig = (double*)ctx_buf(ctx, "scf_sig", (size_t)(ntau * np2) * 8, true);
  launch_pad_convert(Sigma, n, np, ntau, Prec::F64, spad, 0, np2, nullptr, ctx->stream);
  GF2_HIP(hipGetLastError());
  Prob pb[2];
  pb[0] = prob0();
  pb[0].a[0] = opref(dct);
  pb[0].b[0] = opref(spad, np2);
  pb[0].nout = 1;
  pb[0].out[0] = outspec(y, 0, {1.0f}, 0, 0, np2);
  pb[1] = prob0();
  pb[1].a[0] = opref(y, np2);
  pb[1].b[0] = opref(dct);
  pb[1].nout = 1;
  pb[1].out[0] = outspec(g.sig, 0, {1.0f}, 0, 0, np2);
  auto* probs = (Prob*)ctx_buf(ctx, "scf_prob", 2 * sizeof(Prob));
  h2d(ctx, probs, pb, 2);
  std::vector<Unit> uh((size_t)ntau);
  for (int64_t t = 0; t < ntau; ++t) uh[t] = mk_unit(t, 0, 0, 0, 0);
  auto* units = (Unit*)ctx_buf(ctx, "scf_units", (size_t)ntau * sizeof(Unit));
  h2d(ctx, units, uh.data(), uh.size());
  {
    ProfScope ps(ctx, "scf_mo", 4.0 * (double)ntau * (double)n * n * n);
    for (int k = 0; k < 2; ++k) {
      GemmLaunch L = chain_launch(probs + k, 1, units, (int32_t)ntau, n, np, 0);
      launch_gemm(Prec::F64, L, tiles_of(pb[k], Prec::F64, n), ctx->stream);
    }
  }
  GF2_HIP(hipGetLastError());
  // phase tables (host, FP64): w_f = (2f + 1) pi / beta
  std::vector<double> ph((size_t)(g.nchunk * ntau * g.ncp * 2), 0.0), om((size_t)(g.nchunk * g.ncp), 0.0);
  std::vector<double> cs(need_back ? (size_t)(g.nchunk * g.ntop * g.ncp * 2) : 0, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t ch = 0; ch < g.nchunk; ++ch)
    for (int64_t f = 0; f < g.nc; ++f) {
      const int64_t fg_ = ch * g.nc + f;
      if (fg_ >= nw) break;
      const double wf = (2.0 * (double)fg_ + 1.0) * M_PI / beta;
      om[ch * g.ncp + f] = wf;
      for (int64_t t = 0; t < ntau; ++t) {
        const double x = wf * tau[t];
        double* p = &ph[((ch * ntau + t) * g.ncp + f) * 2];
        p[0] = w[t] * std::cos(x);
        p[1] = w[t] * std::sin(x);
      }
      if (need_back)
        for (int64_t o = 0; o < g.nto; ++o) {
          const double x = wf * (o < ntau ? tau[o] : beta);
          double* p = &cs[((ch * g.ncp + f) * g.ntop + o) * 2];
          p[0] = std::cos(x);
          p[1] = std::sin(x);
        }
    }
  g.ph = (double*)ctx_buf(ctx, "scf_ph", ph.size() * 8);
  g.om = (double*)ctx_buf(ctx, "scf_om", om.size() * 8);
  h2d(ctx, g.ph, ph.data(), ph.size());
  h2d(ctx, g.om, om.data(), om.size());
  if (need_back) {
    g.cs = (double*)ctx_buf(ctx, "scf_cs", cs.size() * 8);
    h2d(ctx, g.cs, cs.data(), cs.size());
  }
  if (!dyson) {
    GF2_HIP(hipStreamSynchronize(ctx->stream));
    return;
  }
  const int64_t nb = scf_panel();
  g.a = (double*)ctx_buf(ctx, "scf_a", (size_t)(g.nc * 2 * np2) * 8);
  g.colbuf = (double*)ctx_buf(ctx, "scf_col", (size_t)(g.nc * 2 * np * nb) * 8);
  g.pbuf = (double*)ctx_buf(ctx, "scf_piv", (size_t)(g.nc * 2 * nb * nb) * 8);
  g.tr = (double*)ctx_buf(ctx, "scf_tr", (size_t)(g.nchunk * g.nc * 2) * 8);
  g.shift = (double*)ctx_buf(ctx, "scf_shift", (size_t)np * 8);
  g.err = (int*)ctx_buf(ctx, "scf_err", sizeof(int), true);
  GF2_HIP(hipStreamSynchronize(ctx->stream));
}

// Dyson matrices of frequency chunk ch at chemical potential mu (shift
// already uploaded), inverted in place; returns the chunk's frequency count.
int64_t scf_chunk(gf2_ctx* ctx, const ScfGrid& g, int64_t ch) {
  const int64_t cnt = std::min(g.nc, g.nw - ch * g.nc);
  const double np = (double)g.np;
  {
    ProfScope ps(ctx, "scf_sig_iw", 4.0 * (double)cnt * (double)g.ntau * np * np);
    launch_sig_iw(g.sig, g.ntau, g.np, g.n, g.ph + ch * g.ntau * g.ncp * 2, (int32_t)cnt, (int32_t)g.ncp, g.shift,
                  g.om + ch * g.ncp, g.a, ctx->stream);
  }
  {
    ProfScope ps(ctx, "scf_invert", 8.0 * (double)cnt * np * np * np);
    launch_gj_invert(g.a, (int32_t)cnt, g.np, g.colbuf, g.pbuf, g.err, ctx->stream);
  }
  GF2_HIP(hipGetLastError());
  return cnt;
}

void scf_set_mu(gf2_ctx* ctx, const ScfGrid& g, double mu) {
  std::vector<double> sh((size_t)g.np, 0.0);
  for (int64_t i = 0; i < g.n; ++i) sh[i] = mu - g.eps[i];
  h2d(ctx, g.shift, sh.data(), sh.size());
}

void scf_check(gf2_ctx* ctx, const ScfGrid& g) {
  int e = 0;
  d2h(ctx, &e, g.err, 1);
  if (e) throw Gf2Error{GF2_E_NUMERIC, "Dyson matrix with a vanishing or non-finite pivot"};
}

// N_e(mu) = -2 Tr G~(beta-) = 2 sum_i f_i + (4 / beta) sum_w sum_i Re D_ii(i w),
// and dN_e/dmu = 2 beta sum_i f_i (1 - f_i) + (4 / beta) sum_w [sum_i Re G0~_ii^2
// - sum_ij Re G_ij^2] (dG/dmu = -G^2).
std::pair<double, double> scf_count(gf2_ctx* ctx, const ScfGrid& g, double mu) {
  scf_set_mu(ctx, g, mu);
  for (int64_t ch = 0; ch < g.nchunk; ++ch) {
    const int64_t cnt = scf_chunk(ctx, g, ch);
    launch_iw_diag(g.a, (int32_t)cnt, g.np, g.n, g.shift, g.om + ch * g.ncp, g.tr + ch * g.nc * 2, ctx->stream);
  }
  GF2_HIP(hipGetLastError());
  std::vector<double> tr((size_t)(2 * g.nw));
  d2h(ctx, tr.data(), g.tr, tr.size());
  scf_check(ctx, g);
  double s = 0.0, d = 0.0;
  for (int64_t k = 0; k < g.nw; ++k) {
    s += tr[2 * k];
    d += tr[2 * k + 1];
  }
  double fsum = 0.0, fder = 0.0;
  for (int64_t i = 0; i < g.n; ++i) {
    const double f = std::exp(-softplus(g.beta * (g.eps[i] - mu)));
    fsum += f;
    fder += f * (1.0 - f);
  }
  return {2.0 * fsum + 4.0 / g.beta * s, 2.0 * g.beta * fder + 4.0 / g.beta * d};
}

// Newton on N_e(mu) - n_elec (N_e grows with mu) from the middle of [lo, hi],
// the bracket narrowed by every evaluation and a bisection wherever the
// Newton step leaves it.
double scf_tune(gf2_ctx* ctx, const ScfGrid& g, double n_elec, double lo, double hi, double* ne_out) {
  GF2_REQUIRE(lo < hi && std::isfinite(lo) && std::isfinite(hi), GF2_E_ARG, "bad mu bracket");
  const double tol_n = 1e-11 * std::max(1.0, std::fabs(n_elec));
  const double lo0 = lo, hi0 = hi;
  double m = 0.5 * (lo + hi), fm = 0.0;
  for (int it = 0; it < 200; ++it) {
    const auto nd = scf_count(ctx, g, m);
    fm = nd.first - n_elec;
    if (std::fabs(fm) <= tol_n) break;
    if (fm < 0.0) lo = m; else hi = m;
    if (hi - lo <= 1e-15 * std::max(1.0, std::fabs(lo) + std::fabs(hi))) break;
    double next = nd.second > 0.0 && std::isfinite(nd.second) ? m - fm / nd.second : lo - 1.0;
    if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
    m = next;
  }
  if (std::fabs(fm) > tol_n)
    GF2_REQUIRE(!(fm < 0.0 && hi0 - m <= 1e-12 * std::max(1.0, std::fabs(hi0))) &&
                    !(fm > 0.0 && m - lo0 <= 1e-12 * std::max(1.0, std::fabs(lo0))),
                GF2_E_ARG, "the mu bracket does not contain N_e = n_elec");
  if (ne_out) *ne_out = fm + n_elec;
  return m;
}

// G(tau), G(beta - tau) and G(beta-) at mu: the back-transform sums over all
// chunks, G~ in the eigenbasis, then G = C G~ C^T on the FP64 MFMA GEMM.
void scf_dyson(gf2_ctx* ctx, const ScfGrid& g, double mu, double* G, double* Gbar, double* Gbeta) {
  const int64_t np = g.np, np2 = np * np, nt = g.ntau, nmo = 2 * nt + 1;
  scf_set_mu(ctx, g, mu);
  auto* pc = (double*)ctx_buf(ctx, "scf_pc", (size_t)(g.nto * np2) * 8, true);
  auto* ps = (double*)ctx_buf(ctx, "scf_ps", (size_t)(g.nto * np2) * 8, true);
  for (int64_t ch = 0; ch < g.nchunk; ++ch) {
    const int64_t cnt = scf_chunk(ctx, g, ch);
    ProfScope pr(ctx, "scf_back", 4.0 * (double)cnt * (double)g.nto * (double)np2);
    launch_iw_back(g.a, (int32_t)cnt, np, g.n, g.shift, g.om + ch * g.ncp, g.cs + ch * g.ntop * g.ncp * 2,
                   (int32_t)g.nto, (int32_t)g.ntop, pc, ps, ctx->stream);
  }
  GF2_HIP(hipGetLastError());
  scf_check(ctx, g);
  std::vector<double> emu((size_t)g.n);
  for (int64_t i = 0; i < g.n; ++i) emu[i] = g.eps[i] - mu;
  auto* demu = (double*)ctx_buf(ctx, "scf_emu", (size_t)g.n * 8);
  auto* dtau = (double*)ctx_buf(ctx, "scf_tau", (size_t)nt * 8);
  h2d(ctx, demu, emu.data(), emu.size());
  h2d(ctx, dtau, g.tau.data(), g.tau.size());
  auto* mo = (double*)ctx_buf(ctx, "scf_mo", (size_t)(nmo * np2) * 8);
  auto* y = (double*)ctx_buf(ctx, "scf_y2", (size_t)(nmo * np2) * 8, true);
  auto* out = (double*)ctx_buf(ctx, "scf_out", (size_t)(nmo * np2) * 8);
  launch_g_mo(pc, ps, np, g.n, nt, dtau, demu, g.beta, mo, ctx->stream);
  GF2_HIP(hipGetLastError());
  // G = C G~ C^T: Y = C G~ (A = C, B = G~, symmetric), then G = Y C^T (A = Y,
  // B = C); Y's padding is cleared (read as an operand over the padded length)
  const double* dcp = (const double*)ctx_buf(ctx, "scf_cp", (size_t)np2 * 8);
  Prob pb[2];
  pb[0] = prob0();
  pb[0].a[0] = opref(dcp);
  pb[0].b[0] = opref(mo, np2);
  pb[0].nout = 1;
  pb[0].out[0] = outspec(y, 0, {1.0f}, 0, 0, np2);
  pb[1] = prob0();
  pb[1].a[0] = opref(y, np2);
  pb[1].b[0] = opref(dcp);
  pb[1].nout = 1;
  pb[1].out[0] = outspec(out, 0, {1.0f}, 0, 0, np2);
  auto* probs = (Prob*)ctx_buf(ctx, "scf_prob2", 2 * sizeof(Prob));
  h2d(ctx, probs, pb, 2);
  std::vector<Unit> uh((size_t)nmo);
  for (int64_t t = 0; t < nmo; ++t) uh[t] = mk_unit(t, 0, 0, 0, 0);
  auto* units = (Unit*)ctx_buf(ctx, "scf_units2", (size_t)nmo * sizeof(Unit));
  h2d(ctx, units, uh.data(), uh.size());
  {
    ProfScope ps2(ctx, "scf_ao", 4.0 * (double)nmo * (double)g.n * g.n * g.n);
    for (int k = 0; k < 2; ++k) {
      GemmLaunch L = chain_launch(probs + k, 1, units, (int32_t)nmo, g.n, np, 0);
      launch_gemm(Prec::F64, L, tiles_of(pb[k], Prec::F64, g.n), ctx->stream);
    }
  }
  if (G) launch_unpad_sym(out, g.n, np, nt, 1.0, G, ctx->stream);
  if (Gbar) launch_unpad_sym(out + nt * np2, g.n, np, nt, 1.0, Gbar, ctx->stream);
  if (Gbeta) launch_unpad_sym(out + 2 * nt * np2, g.n, np, 1, 1.0, Gbeta, ctx->stream);
  GF2_HIP(hipGetLastError());
  GF2_HIP(hipStreamSynchronize(ctx->stream));
}

// F = h + J[P] - K[P]/2 with P = -2 G(beta-): J from c_Q = Tr(B^Q P), K as
// sums over groups of 8 auxiliary indices of (B^Q P) B^Q on the FP64 GEMM.
void scf_fock(gf2_ctx* ctx, int64_t n, int64_t naux, const void* B, gf2_dtype dtype, const double* h,
              const double* Gbeta, double* Fout) {
  GF2_REQUIRE(n > 0 && naux > 0 && B && h && Gbeta && Fout, GF2_E_ARG, "bad Fock arguments");
  GF2_REQUIRE(dtype == GF2_F64 || dtype == GF2_F32, GF2_E_ARG, "bad dtype");
  const bool f64 = dtype == GF2_F64;
  const int64_t np = pad_dim(n), np2 = np * np, nn = n * n;
  auto* p = (double*)ctx_buf(ctx, "fk_p", (size_t)nn * 8);
  auto* ppad = (double*)ctx_buf(ctx, "fk_ppad", (size_t)np2 * 8);
  auto* cq = (double*)ctx_buf(ctx, "fk_c", (size_t)naux * 8);
  auto* dh = (double*)ctx_buf(ctx, "fk_h", (size_t)nn * 8);
  auto* df = (double*)ctx_buf(ctx, "fk_f", (size_t)nn * 8);
  h2d(ctx, dh, h, (size_t)nn);
  launch_density(Gbeta, nn, p, ctx->stream);
  launch_pad_convert(p, n, np, 1, Prec::F64, ppad, 0, np2, nullptr, ctx->stream);
  launch_bq_dot(B, f64, n, naux, p, cq, ctx->stream);
  GF2_HIP(hipGetLastError());
  constexpr int64_t kSeg = 8;                 // B^Q of one group, K-concatenated
  const int64_t qc = std::min<int64_t>((naux + kSeg - 1) / kSeg * kSeg,
                                       std::max<int64_t>(kSeg, ((int64_t)1 << 30) / (16 * np2) / kSeg * kSeg));
  const int64_t nchunk = (naux + qc - 1) / qc, ngc = qc / kSeg, ng = nchunk * ngc;
  auto* bq = (double*)ctx_buf(ctx, "fk_bq", (size_t)(qc * np2) * 8);
  auto* x = (double*)ctx_buf(ctx, "fk_x", (size_t)(qc * np2) * 8, true);
  auto* kp = (double*)ctx_buf(ctx, "fk_kp", (size_t)(ng * np2) * 8, true);
  Prob pb[2];
  pb[0] = prob0();          // X^Q = B^Q P  (A = B^Q, B = P, symmetric)
  pb[0].a[0] = opref(bq, np2);
  pb[0].b[0] = opref(ppad);
  pb[0].nout = 1;
  pb[0].out[0] = outspec(x, 0, {1.0f}, 0, 0, np2);
  pb[1] = prob0();          // sum over a group of 8 of X^Q B^Q (B^Q symmetric)
  pb[1].nseg = (int32_t)kSeg;
  for (int s_ = 0; s_ < kSeg; ++s_) {
    pb[1].a[s_] = opref(x + s_ * np2, kSeg * np2);
    pb[1].b[s_] = opref(bq + s_ * np2, kSeg * np2);
  }
  pb[1].nout = 1;
  auto* probs = (Prob*)ctx_buf(ctx, "fk_prob", 2 * nchunk * sizeof(Prob));
  std::vector<Prob> ph((size_t)(2 * nchunk));
  for (int64_t ch = 0; ch < nchunk; ++ch) {
    ph[2 * ch] = pb[0];
    ph[2 * ch + 1] = pb[1];
    ph[2 * ch + 1].out[0] = outspec(kp + ch * ngc * np2, 0, {1.0f}, 0, 0, np2);
  }
  h2d(ctx, probs, ph.data(), ph.size());
  std::vector<Unit> uh((size_t)qc);
  for (int64_t t = 0; t < qc; ++t) uh[t] = mk_unit(t, 0, 0, 0, 0);
  auto* units = (Unit*)ctx_buf(ctx, "fk_units", (size_t)qc * sizeof(Unit));
  h2d(ctx, units, uh.data(), uh.size());
  {
    ProfScope ps(ctx, "fock_k", 4.0 * (double)naux * (double)n * n * n);
    for (int64_t ch = 0; ch < nchunk; ++ch) {
      launch_pad_bq(B, f64, n, naux, np, ch * qc, qc, bq, ctx->stream);
      GemmLaunch L0 = chain_launch(probs + 2 * ch, 1, units, (int32_t)qc, n, np, 0);
      launch_gemm(Prec::F64, L0, tiles_of(pb[0], Prec::F64, n), ctx->stream);
      GemmLaunch L1 = chain_launch(probs + 2 * ch + 1, 1, units, (int32_t)ngc, n, np, 0);
      launch_gemm(Prec::F64, L1, tiles_of(pb[1], Prec::F64, n), ctx->stream);
    }
  }
  launch_fock_final(B, f64, n, naux, cq, dh, kp, ng, np, df, ctx->stream);
  GF2_HIP(hipGetLastError());
  d2h(ctx, Fout, df, (size_t)nn);
}

}  // namespace

gf2_status gf2_dyson(gf2_ctx* ctx, int64_t n, const double* F, const double* S, double mu, double beta,
                     int64_t ntau, const double* tau, const double* w, const double* Sigma, int64_t nw, double* G,
                     double* Gbar, double* Gbeta) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(G || Gbar || Gbeta, GF2_E_ARG, "no output requested");
    GF2_REQUIRE(std::isfinite(mu), GF2_E_ARG, "mu is not finite");
    ScfGrid g;
    scf_prepare(ctx, g, n, F, S, beta, ntau, tau, w, Sigma, nw, true);
    scf_dyson(ctx, g, mu, G, Gbar, Gbeta);
  });
}

gf2_status gf2_electron_count(gf2_ctx* ctx, int64_t n, const double* F, const double* S, double mu, double beta,
                              int64_t ntau, const double* tau, const double* w, const double* Sigma, int64_t nw,
                              double* n_e) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(n_e && std::isfinite(mu), GF2_E_ARG, "bad electron-count arguments");
    ScfGrid g;
    scf_prepare(ctx, g, n, F, S, beta, ntau, tau, w, Sigma, nw, false);
    *n_e = scf_count(ctx, g, mu).first;
  });
}

gf2_status gf2_tune_mu(gf2_ctx* ctx, int64_t n, const double* F, const double* S, double beta, int64_t ntau,
                       const double* tau, const double* w, const double* Sigma, int64_t nw, double n_elec,
                       double mu_lo, double mu_hi, double* mu_out, double* n_e) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(mu_out, GF2_E_ARG, "mu_out is null");
    ScfGrid g;
    scf_prepare(ctx, g, n, F, S, beta, ntau, tau, w, Sigma, nw, false);
    *mu_out = scf_tune(ctx, g, n_elec, mu_lo, mu_hi, n_e);
  });
}

gf2_status gf2_qp_energies(gf2_ctx* ctx, int64_t n, const double* F, const double* S, double mu, double beta,
                           int64_t ntau, const double* tau, const double* w, const double* Sigma, int32_t n_pade,
                           double eta, int32_t max_iter, double* E, int32_t* converged) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(E && n_pade >= 1 && n_pade <= 4096 && max_iter >= 1 && std::isfinite(mu) && std::isfinite(eta),
                GF2_E_ARG, "bad quasiparticle arguments");
    ScfGrid g;
    scf_prepare(ctx, g, n, F, S, beta, ntau, tau, w, Sigma, n_pade, false, false);
    auto* deps = (double*)ctx_buf(ctx, "qp_eps", (size_t)n * 8);
    auto* work = ctx_buf(ctx, "qp_work", (size_t)(n * 2 * n_pade) * 16);
    auto* de = (double*)ctx_buf(ctx, "qp_e", (size_t)n * 8);
    auto* dc = (int32_t*)ctx_buf(ctx, "qp_conv", (size_t)n * 4);
    h2d(ctx, deps, g.eps.data(), g.eps.size());
    {
      ProfScope ps(ctx, "qp");
      launch_qp(g.sig, ntau, g.np, n, g.ph, n_pade, (int32_t)g.ncp, g.om, deps, mu, eta, max_iter, work, de, dc,
                ctx->stream);
    }
    GF2_HIP(hipGetLastError());
    std::vector<int32_t> ch((size_t)n);
    d2h(ctx, E, de, (size_t)n);
    d2h(ctx, ch.data(), dc, ch.size());
    if (converged) std::copy(ch.begin(), ch.end(), converged);
    for (int64_t k = 0; k < n; ++k)
      GF2_REQUIRE(std::isfinite(E[k]), GF2_E_NUMERIC, "non-finite quasiparticle energy");
  });
}

gf2_status gf2_fock(gf2_ctx* ctx, int64_t n, int64_t naux, const void* B, gf2_dtype dtype, const double* h,
                    const double* Gbeta, double* F_out) {
  return guarded(ctx, [&] { scf_fock(ctx, n, naux, B, dtype, h, Gbeta, F_out); });
}

gf2_status gf2_scf_step(gf2_ctx* ctx, int64_t n, int64_t naux, const void* B, gf2_dtype dtype, const double* h,
                        const double* F, const double* S, double beta, int64_t ntau, const double* tau,
                        const double* w, const double* Sigma, int64_t nw, double n_elec, double mu_lo, double mu_hi,
                        double* mu_out, double* G, double* Gbar, double* Gbeta, double* F_out) {
  return guarded(ctx, [&] {
    GF2_REQUIRE(mu_out && G && Gbar && Gbeta && F_out, GF2_E_ARG, "bad SCF-step outputs");
    ScfGrid g;
    scf_prepare(ctx, g, n, F, S, beta, ntau, tau, w, Sigma, nw, true);
    const double mu = scf_tune(ctx, g, n_elec, mu_lo, mu_hi, nullptr);
    scf_dyson(ctx, g, mu, G, Gbar, Gbeta);
    scf_fock(ctx, n, naux, B, dtype, h, Gbeta, F_out);
    *mu_out = mu;
  });
}

}  // extern "C"
