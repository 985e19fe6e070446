// Allocation-free Tucker operator: kp_tucker whose intermediates live in a
// fixed device buffer that belongs to the library (include/kp.h,
// kp_tucker_noalloc). For callers that cannot allocate device memory.
//
// The buffer is a file-scope device array. On the host its name is only a
// stand-in for the symbol, never a device address: the address is obtained
// once per device with hipGetSymbolAddress (each device holds its own copy of
// the array) and only that address is handed to the kernels.
#include "kp.h"

#include <mutex>

#include "kp_common.h"
#include "kp_internal.h"

namespace kp {
namespace {

static_assert(KP_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size: whole 256-byte units");

// The Tucker chain's two ping-pong intermediates (no value needs to start at
// zero: every intermediate is written in full before it is read).
static __device__ __align__(256) char scratch[KP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];  // per device: the device address of `scratch`

// The device address of the current device's copy of `scratch` (looked up on
// the first call on each device, with that device current), or nullptr with
// *status set.
void* scratch_for_current_device(int* status) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *status = hip_status(e);
    return nullptr;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    *status = hip_status(hipErrorInvalidDevice);
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *status = hip_status(e != hipSuccess ? e : hipErrorInvalidSymbol);
      return nullptr;
    }
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace
}  // namespace kp

extern "C" size_t kp_noalloc_scratch_bytes(void) { return KP_NOALLOC_SCRATCH_BYTES; }

extern "C" int kp_tucker_noalloc(const kp_tensor* T, const kp_matrix* const* L, kp_tensor* S,
                                 int prec, hipStream_t stream) {
  // Shapes first: the same validation as kp_tucker, so an argument error is
  // reported as such (kp_tucker_workspace answers 0 for invalid arguments).
  const size_t need = kp_tucker_workspace(T, L, prec);
  if (need > KP_NOALLOC_SCRATCH_BYTES) return KP_ERR_SCRATCH;
  int st = KP_OK;
  void* ws = nullptr;
  if (need > 0) {
    ws = kp::scratch_for_current_device(&st);
    if (!ws) return st;
  }
  return kp_tucker(T, L, S, prec, ws, need > 0 ? KP_NOALLOC_SCRATCH_BYTES : 0, nullptr, 0,
                   stream);
}
