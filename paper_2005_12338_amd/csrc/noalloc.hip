// gf2_energy_noalloc: the energy of eq:corr for callers that cannot allocate
// device memory.  It runs the same kernels as gf2_energy; their scratch
// (the per-tau traces and the result slots) lives in a fixed file-scope
// device array instead of context buffers, and the inputs and outputs stay
// on the device, so a call makes no allocation and no host synchronisation.
#include <mutex>

#include "kernels.hpp"

namespace {

constexpr int64_t kNoAllocMaxTau = 512;                  // the energy kernels' own tau limit
constexpr int64_t kResultSlots = 8;
constexpr int64_t kScratchDoubles = kNoAllocMaxTau + kResultSlots;   // 4160 bytes

// One copy per GPU, held until the process ends.  Host code never names it
// except through hipGetSymbolAddress: the device address kept per device is
// what kernels and copies receive.
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

__global__ void k_energy_publish(const double* res, double n_elec, double* out) {
  if (threadIdx.x == 0) {
    out[0] = res[0];
    out[1] = res[0] / n_elec;
    out[2] = res[2];
  }
}

}  // namespace

// Resolves the device address of `scratch` on `device`, which must be the
// current device.  Called once per device by gf2_create.
gf2_status noalloc_attach(int device) {
  if (device < 0 || device >= kMaxDevices) return GF2_E_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return GF2_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GF2_E_DEVICE;
  g_scratch_ptr[device] = (double*)p;
  return GF2_OK;
}

extern "C" gf2_status gf2_energy_noalloc(gf2_ctx* ctx, int64_t n, int64_t ntau, const double* w,
                                         const double* Sigma, const double* Gbar, const double* e_samples,
                                         int64_t ns, double n_elec, double* out) {
  if (!ctx) return GF2_E_ARG;
  try {
    GF2_REQUIRE(n > 0 && ntau > 0 && w && Sigma && Gbar && out, GF2_E_ARG, "bad energy arguments");
    GF2_REQUIRE(ntau <= kNoAllocMaxTau, GF2_E_ARG,
                "gf2_energy_noalloc: ntau = " + std::to_string(ntau) + " exceeds its fixed scratch of " +
                    std::to_string(kNoAllocMaxTau) + " tau points");
    GF2_REQUIRE(n_elec > 0, GF2_E_ARG, "n_elec must be positive");
    GF2_REQUIRE(!e_samples || ns >= 2, GF2_E_ARG, "a standard error needs ns >= 2");
    GF2_REQUIRE(ctx->device >= 0 && ctx->device < kMaxDevices, GF2_E_STATE, "context device out of range");
    double* base = nullptr;
    {
      std::lock_guard<std::mutex> lock(g_scratch_mu);
      base = g_scratch_ptr[ctx->device];
    }
    GF2_REQUIRE(base, GF2_E_STATE, "fixed scratch not attached on this device");
    GF2_HIP(hipSetDevice(ctx->device));
    // every slot the kernels read is written first in the same call: the
    // traces for t < ntau by the trace kernel, the results by the statistics
    // kernel, so nothing needs clearing
    double* tr = base;
    double* res = base + kNoAllocMaxTau;
    launch_trace_prod(Sigma, Gbar, n, ntau, tr, ctx->stream);
    // E = -(1/2) sum_t w_t Tr(Sigma Gbar), the Galitskii-Migdal factor of gf2_energy
    launch_energy_stats(tr, w, ntau, e_samples, e_samples ? ns : 0, 0.5, res, ctx->stream);
    hipLaunchKernelGGL(k_energy_publish, dim3(1), dim3(64), 0, ctx->stream, res, n_elec, out);
    GF2_HIP(hipGetLastError());
    ctx->err.clear();
    return GF2_OK;
  } catch (const Gf2Error& e) {
    ctx->err = e.msg;
    return e.code;
  } catch (...) {
    ctx->err = "unexpected internal error";
    return GF2_E_DEVICE;
  }
}
