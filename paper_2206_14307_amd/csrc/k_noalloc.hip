// nqs_eloc_noalloc: log psi and E_loc (Sec. 3.1 Eqs. (2), (6); Sec. 3.2
// Eq. (10)) for callers that cannot allocate device memory (code under HIP
// graph capture, serving loops, harnesses that forbid allocation).
//
// It runs the same kernels as nqs_eloc for models with a fused (K*M <= 128)
// or wide (K*M > 128) E_loc kernel; the per-(configuration, 16-image block)
// partials those kernels exchange, (G/16) x 6 doubles per configuration, live
// in `scratch`, a file-scope device array of kScratchBytes instead of a
// caller workspace.  Each GPU holds its own copy for the life of the process;
// its address on a device is resolved once, with that device current, by
// noalloc_scratch_init (called from nqs_create, and from the entry point if
// that failed), and host code uses only that address.  Every partial a
// finish kernel reads is written by the kernel before it in the same call,
// so nothing needs clearing between calls; calls that overlap on one GPU
// (several streams or host threads at once) share the array and race.
#include <mutex>
#include <string>

#include "nqs_internal.h"

namespace nqs {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;    // 64 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

}  // namespace nqs

using namespace nqs;

extern "C" nqs_status nqs_eloc_noalloc(nqs_ctx* c, const int8_t* spins, int64_t S,
                                       double* logpsi_out, double* eloc_out, hipStream_t st) {
  if (!c) return NQS_ERR_ARG;
  auto fail = [&](nqs_status s, const std::string& m) {
    c->last_error = "eloc_noalloc: " + m;
    return s;
  };
  if (S < 0) return fail(NQS_ERR_ARG, "S must be >= 0");
  if (S > 0 && (!spins || !eloc_out)) return fail(NQS_ERR_ARG, "spins or eloc_out is NULL");
  const bool fused = eloc_fused_supported(c);
  if (!fused && !eloc_wide_supported(c))
    return fail(NQS_ERR_ARG, "the model has no fused or wide E_loc kernel (use nqs_eloc)");
  const size_t per = (size_t)(c->G / 16) * 6 * sizeof(double);
  const int64_t max_s = (int64_t)(kScratchBytes / per);
  if (S > max_s)
    return fail(NQS_ERR_ARG, "S = " + std::to_string(S) + " exceeds the " + std::to_string(max_s) +
                                 " configurations its " + std::to_string(kScratchBytes >> 20) +
                                 " MiB scratch holds for this lattice");
  if (S == 0) return NQS_OK;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(NQS_ERR_DEVICE, hipGetErrorString(e));
  if (dev != c->device) return fail(NQS_ERR_ARG, "the context's device is not the current device");
  void* base = scratch_ptr(dev);
  if (!base) {
    if ((e = noalloc_scratch_init(dev)) != hipSuccess)
      return fail(NQS_ERR_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    base = scratch_ptr(dev);
  }
  double* part = static_cast<double*>(base);
  if (fused) {
    e = launch_eloc_fused(c, spins, S, part, logpsi_out, eloc_out, 2, st);
  } else {
    e = launch_eloc_wide(c, spins, S, part, st);
    if (e == hipSuccess) e = launch_fused_finish(c, spins, S, part, logpsi_out, eloc_out, 2, st);
  }
  if (e != hipSuccess) return fail(NQS_ERR_DEVICE, hipGetErrorString(e));
  return NQS_OK;
}
