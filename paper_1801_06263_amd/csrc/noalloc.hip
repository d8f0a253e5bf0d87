// osscir_mocca_iterate_noalloc: the MOCCA iteration of osscir_mocca_iterate
// with its workspace in a file-scope device array instead of caller memory,
// for callers that cannot allocate (graph capture, tight serving loops).
//
// In host code the array's name stands for a host-side shadow, not a device
// address: its device address is looked up once per device with
// hipGetSymbolAddress and only that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "osscir.h"
#include "plan.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // the 512^2, 720 x 1024 scan needs 50.5 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of scratch, per device

int scratch_of(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return osscir::fail(OSSCIR_EINVAL, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return osscir::hip_fail(e, "noalloc: looking up the static scratch");
    if (!ptr) return osscir::fail(OSSCIR_EDEVICE, "noalloc: static scratch has no device address");
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return OSSCIR_OK;
}

}  // namespace

extern "C" int osscir_mocca_iterate_noalloc(osscir_plan plan, const osscir_params *params, float *f, float *fbar,
                                            float *y, const float *c, int32_t n_iter, double *dtpl,
                                            osscir_stream stream) {
  int rc = osscir::check_plan(plan);
  if (rc) return rc;
  const size_t need = osscir::work_layout(plan->sd).total;
  if (need > kScratchBytes)
    return osscir::fail(OSSCIR_EINVAL, "noalloc: this scan needs %zu bytes of scratch, more than the static %zu",
                        need, kScratchBytes);
  void *ptr = nullptr;
  if ((rc = scratch_of(plan->device, &ptr))) return rc;
  osscir_state st{f, fbar, y, c, ptr, kScratchBytes};
  return osscir_mocca_iterate(plan, params, &st, n_iter, dtpl, stream);
}
