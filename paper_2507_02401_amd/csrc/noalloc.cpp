// Allocation-free variant of matern_cov_apply: the level arrays a_1 .. a_m live in a file-scope
// device array instead of a caller workspace.  Each device that runs the library holds its own
// copy of the array (allocated with the code object when the library is first used on that
// device, kept until the process ends).  Host code never uses the array's name as an address:
// the device address of each device's copy comes from hipGetSymbolAddress, taken once per device
// with that device current, and that address is what the kernels receive as their workspace.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/eswave.h"
#include "internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

es_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return es::report_error(ES_EDEVICE, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return es::report_error(ES_EUNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      char msg[256];
      snprintf(msg, sizeof msg, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return es::report_error(ES_EDEVICE, msg);
    }
    if (!ptr || ((uintptr_t)ptr & 255)) return es::report_error(ES_EDEVICE, "scratch is not 256-byte aligned");
    g_ptr[dev] = ptr;
  }
  *out = g_ptr[dev];
  return ES_OK;
}

}  // namespace

extern "C" {

size_t es_noalloc_scratch_bytes(void) { return kScratchBytes; }

es_status matern_cov_apply_noalloc(int ndim, const int64_t* shape, int64_t batch, int order, int levels, double s,
                                   const float* x, float* y, void* stream) {
  // argument errors are reported by matern_cov_apply itself; only the scratch size is checked here
  if (batch > 0 && ndim >= 1 && ndim <= 3 && shape && order >= 1 && order <= 8 && levels >= 0 && levels <= 30) {
    const size_t need = es_workspace_bytes(ndim, shape, batch, order, levels, ES_OP_COV);
    if (need > kScratchBytes) {
      char msg[256];
      snprintf(msg, sizeof msg,
               "matern_cov_apply_noalloc: this geometry and batch need %zu bytes of scratch, the library holds %zu "
               "(use matern_cov_apply with a workspace)",
               need, kScratchBytes);
      return es::report_error(ES_EWORKSPACE, msg);
    }
    if (need) {
      es_status st = es::device_check();
      if (st != ES_OK) return st;
      void* ws = nullptr;
      st = scratch_address(&ws);
      if (st != ES_OK) return st;
      return matern_cov_apply(ndim, shape, batch, order, levels, s, x, y, ws, kScratchBytes, stream);
    }
  }
  return matern_cov_apply(ndim, shape, batch, order, levels, s, x, y, nullptr, 0, stream);
}

}  // extern "C"
