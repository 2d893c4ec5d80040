// phiq_plan_execute_noalloc: a Gauss-rule plan execution whose intermediate
// tensors live in a fixed device array of the library instead of the
// handle's grow-only workspace, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// The array is a file-scope __device__ variable: every GPU the library runs
// on holds its own copy, at its own address, from module load until the
// process ends.  In host code its name is only a host-side stand-in, so the
// device address is looked up once per device (hipGetSymbolAddress, at
// phiq_create with that device current) and only that pointer is handed to
// the kernels.  No call here allocates or frees.
#include <hip/hip_runtime.h>

#include <mutex>

#include "phiq_internal.h"

static __device__ __align__(256) unsigned char scratch[PHIQ_NOALLOC_SCRATCH_BYTES];

namespace phiq {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

phiq_status noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return PHIQ_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return PHIQ_OK;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != device) return PHIQ_ERR_HIP;  // caller makes it current
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return PHIQ_ERR_HIP;
  }
  g_ptr[device] = ptr;
  return PHIQ_OK;
}

}  // namespace phiq

extern "C" phiq_status phiq_plan_execute_noalloc(phiq_plan plan, const double* v, double* out, size_t* need,
                                                 hipStream_t stream) {
  const int dev = phiq::plan_device(plan);
  if (dev < 0 || dev >= phiq::kMaxDevices) return PHIQ_ERR_INVALID_ARG;
  void* ptr;
  {
    std::lock_guard<std::mutex> lk(phiq::g_mu);
    ptr = phiq::g_ptr[dev];
  }
  if (!ptr) return PHIQ_ERR_HIP;  // phiq_create resolves it; a handle cannot exist without it
  return phiq::plan_execute_in(plan, v, out, ptr, PHIQ_NOALLOC_SCRATCH_BYTES, stream, need);
}
