// Fused pairs of consecutive mu-mode products (pair_tile.h), FP32 and the
// BF16 split forms: the memory-bound products of short modes (m <= 16,
// n <= 32), on the strided layout (I_l > 1: workgroups stride over 64-fiber
// tiles, 16 fibers per wave) or on the two leading modes (I_l = 1: waves
// stride over fibers, one contiguous block each). One launch per piece of
// the outer index b that stays below 2^31 bytes.
#include <mutex>
#include <unordered_map>

#include "kp_common.h"
#include "kp_internal.h"
#include "pair_tile.h"

namespace kp {
namespace {

using namespace tile;

constexpr int kNB1 = 2, kNB2 = 2;
static_assert(kThreads == 64 * kPairWaves, "one fiber group per wave");
static_assert(16 * kNB1 * 16 * kNB2 <= kLeadLdsFloats, "a lead-layout output block fits its LDS");

template <int FORM>
__global__ __launch_bounds__(kThreads, 2) void pair_kernel(PairArgs a, int64_t ntiles) {
  __shared__ __attribute__((aligned(16))) char lds[kPairLdsBytes];
  pair_run<FORM, kNB1, kNB2>(a, blockIdx.x, gridDim.x, ntiles, lds);
}

template <int FORM>
__global__ __launch_bounds__(kThreads) void lead_pair_kernel(PairArgs a) {
  __shared__ __attribute__((aligned(16))) float lds[kThreads / 64][kLeadLdsFloats];
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (kThreads / 64);
  const int w = threadIdx.x >> 6;
  lead_pair_run<FORM, kNB1, kNB2>(a, static_cast<int64_t>(blockIdx.x) * (kThreads / 64) + w,
                                  waves, lds[w]);
}

// Resident workgroups of the lead-layout pair kernel of a form, over the device.
int lead_pair_slots(int form) {
  static std::mutex mu;
  static int slots[3] = {0, 0, 0};  // FP32, BF16x3, BF16x6
  const int f = form == FORM_F32 ? 0 : (form == FORM_BF16X3 ? 1 : 2);
  std::lock_guard<std::mutex> lock(mu);
  if (slots[f] == 0) {
    const void* kern = f == 0   ? reinterpret_cast<const void*>(lead_pair_kernel<FORM_F32>)
                       : f == 1 ? reinterpret_cast<const void*>(lead_pair_kernel<FORM_BF16X3>)
                                : reinterpret_cast<const void*>(lead_pair_kernel<FORM_BF16X6>);
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kThreads, 0) != hipSuccess ||
        per < 1)
      per = 1;
    slots[f] = cus * per;
  }
  return slots[f];
}

int pair_slots() {
  static std::mutex mu;
  static int slots = 0;
  std::lock_guard<std::mutex> lock(mu);
  if (slots == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, reinterpret_cast<const void*>(pair_kernel<FORM_F32>), kThreads, 0) !=
            hipSuccess ||
        per < 1)
      per = 1;
    slots = cus * per;
  }
  return slots;
}

}  // namespace

bool pair_eligible(int form, int64_t Il, int64_t m1, int64_t m2, int64_t n1, int64_t n2) {
  return (form == FORM_F32 || form == FORM_BF16X3 || form == FORM_BF16X6) && Il >= 1 &&
         m1 >= 1 && m2 >= 1 && m1 <= kPairK && m2 <= kPairK && n1 >= 1 && n2 >= 1 &&
         n1 <= 16 * kNB1 && n2 <= 16 * kNB2;
}

hipError_t launch_pair(int form, const PairArgs& a, hipStream_t stream) {
  if (!pair_eligible(form, a.Il, a.m1, a.m2, a.n1, a.n2)) return hipErrorInvalidValue;
  if (a.Il * a.Ir == 0) return hipSuccess;
  const int64_t es = 4;
  const int64_t mm = a.m1 * a.m2, nn = a.n1 * a.n2;
  const int64_t slab = a.Il * (mm > nn ? mm : nn) * es;  // bytes per b
  const int64_t limit = static_cast<int64_t>(1) << 31;
  if (slab >= limit) return hipErrorInvalidValue;
  const int64_t per = (limit - 1) / slab;
  for (int64_t b0 = 0; b0 < a.Ir; b0 += per) {
    PairArgs p = a;
    p.Ir = (a.Ir - b0 < per) ? a.Ir - b0 : per;
    p.X = static_cast<const char*>(a.X) + b0 * a.Il * mm * es;
    p.Y = static_cast<char*>(a.Y) + b0 * a.Il * nn * es;
    if (p.Il == 1) {
      // one fiber per wave at a time
      const int64_t per_group = kThreads / 64;
      int64_t grid = lead_pair_slots(form);
      const int64_t groups = (p.Ir + per_group - 1) / per_group;
      if (grid > groups) grid = groups;
      void (*kern)(PairArgs) = form == FORM_F32      ? lead_pair_kernel<FORM_F32>
                               : form == FORM_BF16X3 ? lead_pair_kernel<FORM_BF16X3>
                                                     : lead_pair_kernel<FORM_BF16X6>;
      hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, stream, p);
    } else {
      const int64_t per_tile = kPairWaves * kPairFibers;
      const int64_t ntiles = (p.Il * p.Ir + per_tile - 1) / per_tile;
      int64_t grid = pair_slots();
      if (grid > ntiles) grid = ntiles;
      void (*kern)(PairArgs, int64_t) = form == FORM_F32      ? pair_kernel<FORM_F32>
                                        : form == FORM_BF16X3 ? pair_kernel<FORM_BF16X3>
                                                              : pair_kernel<FORM_BF16X6>;
      hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(grid)), dim3(kThreads), 0, stream, p,
                         ntiles);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace kp
