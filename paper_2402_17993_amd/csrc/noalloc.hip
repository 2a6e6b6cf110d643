// Allocation-free energy + gradient: the launch sequence of ucc_energy_grad with every per-call
// buffer (state vectors, stored forward states, cos/sin, per-tile partials) carved from one
// static device array instead of buffers the context allocates.  The context's read-only
// tables (built by ucc_build) are used as they are; theta, energy and grad are the caller's
// device buffers (the final reduction writes energy and grad in place).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "api_internal.h"

namespace ucc {
namespace {

constexpr size_t kScratchBytes = UCC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// One copy per GPU, held until the process ends.  In host code `scratch` names a host-side
// stand-in: its device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (the device must be current).
ucc_status scratch_of(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(UCC_EINVAL, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                               "hipGetSymbolAddress(scratch)");
    g_scratch[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch[dev]);
  return UCC_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace
}  // namespace ucc

using namespace ucc;

extern "C" ucc_status ucc_energy_grad_noalloc(ucc_ctx* c, const double* theta, int32_t B,
                                              double* energy, double* grad, void* stream) {
  g_last_error.clear();
  if (!c) return fail(UCC_EINVAL, "ctx is NULL");
  if (c->host_only) return fail(UCC_EINVAL, "context was built host_only");
  if (c->plan.launch_mode == 3)
    return fail(UCC_EINVAL, "the allocation-free call runs the per-pass launches; the context is in launch_mode 3");
  if (B < 1 || B > 65535) return fail(UCC_EINVAL, "B must be in [1, 65535]");
  if (!theta || !energy || !grad) return fail(UCC_EINVAL, "NULL output or input");
  if (c->busy) return fail(UCC_EBUSY, "context is in use by a server job");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if (!is_device_ptr(theta) || !is_device_ptr(energy) || !is_device_ptr(grad))
    return fail(UCC_EINVAL, "theta, energy and grad must be device pointers");
  const Plan& p = c->plan;
  const size_t S = size_t(1) << p.n;
  const size_t nte = size_t(1) << (p.n - p.ke);
  const size_t ntr = size_t(1) << (p.n - p.kr);
  const size_t vec = align256(size_t(B) * S * 16);
  const size_t ck_bytes = p.ckpt ? size_t(p.nfwd - 1) * vec : 0;
  const size_t cs_bytes = align256(size_t(B) * p.K * 16);
  const size_t ep_bytes = align256(size_t(B) * p.nexp * nte * 8);
  const size_t gp_bytes = align256(size_t(B) * p.seq.size() * ntr * 8);
  const size_t need = 2 * vec + ck_bytes + cs_bytes + ep_bytes + gp_bytes;
  if (need > kScratchBytes)
    return fail(UCC_ENOMEM, "needs " + std::to_string(need) + " bytes of scratch; the allocation-free "
                "path holds " + std::to_string(kScratchBytes) + " (use ucc_energy_grad)");
  unsigned char* base = nullptr;
  ucc_status s = scratch_of(c->device, &base);
  if (s != UCC_OK) return s;
  Buffers b;  // a view: nothing here is freed
  b.cap = B;
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    unsigned char* q = base + off;
    off += bytes;
    return q;
  };
  b.psi = reinterpret_cast<double2*>(carve(vec));
  b.lam = reinterpret_cast<double2*>(carve(vec));
  b.ck = ck_bytes ? reinterpret_cast<double2*>(carve(ck_bytes)) : nullptr;
  b.cs = reinterpret_cast<double2*>(carve(cs_bytes));
  b.epart = reinterpret_cast<double*>(carve(ep_bytes));
  b.gpart = reinterpret_cast<double*>(carve(gp_bytes));
  b.theta = nullptr;
  b.E = energy;
  b.G = grad;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // lambda is exactly zero outside the N / S_z sector and no kernel writes there; the array
  // keeps whatever the last call left, so clear it (a kernel, not a memset node).  psi, the
  // stored states and the partials are fully written by the passes before they are read.
  e = launch_fill_zero(b.lam, size_t(B) * S, st);
  if (e != hipSuccess) return hip_fail(e, "launch fill (lambda)");
  return enqueue_eval(c, b, theta, B, true, st, nullptr);
}
