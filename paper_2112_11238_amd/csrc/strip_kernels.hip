// Standalone strip kernels (strip_tile.h): mu-mode products with a short
// contraction, m <= KP. Grid (G, nby): workgroup (x, y) owns n block y and
// streams the fiber tiles x, x + G, x + 2G, ... G is sized from the kernel's
// occupancy so that the resident workgroups fill the chip once.
#include <mutex>
#include <unordered_map>

#include "kp_common.h"
#include "kp_internal.h"
#include "strip_tile.h"

namespace kp {
namespace {

using namespace tile;

template <int FORM, int NB, int FB, int KP, bool INNER, bool VEC>
__global__ __launch_bounds__(kThreads, 2) void strip_kernel(ModeArgs a, int64_t ntiles) {
  __shared__ __attribute__((aligned(16))) char lds[strip_lds_bytes<FORM, NB, FB, KP>()];
  strip_run<FORM, NB, FB, KP, INNER, VEC>(a, blockIdx.y, blockIdx.x, gridDim.x, ntiles, lds);
}

using StripFn = void (*)(ModeArgs, int64_t);

struct StripVariant {
  int form, nb, fb, kp;
  StripFn inner, lead, lead_vec;
};

#define KP_S(FORM, NB, FB, KP)                                                         \
  {FORM, NB, FB, KP, strip_kernel<FORM, NB, FB, KP, true, false>,                     \
   strip_kernel<FORM, NB, FB, KP, false, false>, strip_kernel<FORM, NB, FB, KP, false, true>}

// Fiber blocks per wave chosen per (form, KP) so that a workgroup's LDS
// (L block plus two fiber tiles) stays near 56 KB or less, except the FP64
// strips of 48 and 64 (58-101 KB: one or two workgroups per CU).
const StripVariant kStrips[] = {
    KP_S(FORM_F32, 1, 2, 16), KP_S(FORM_F32, 2, 2, 16), KP_S(FORM_F32, 4, 2, 16),
    KP_S(FORM_F32, 1, 2, 32), KP_S(FORM_F32, 2, 2, 32), KP_S(FORM_F32, 4, 2, 32),
    KP_S(FORM_F32, 1, 1, 64), KP_S(FORM_F32, 2, 1, 64), KP_S(FORM_F32, 4, 1, 64),
    KP_S(FORM_F64, 1, 2, 16), KP_S(FORM_F64, 2, 2, 16), KP_S(FORM_F64, 4, 2, 16),
    KP_S(FORM_F64, 1, 1, 32), KP_S(FORM_F64, 2, 1, 32), KP_S(FORM_F64, 4, 1, 32),
    KP_S(FORM_F64, 1, 1, 48), KP_S(FORM_F64, 2, 1, 48), KP_S(FORM_F64, 4, 1, 48),
    KP_S(FORM_F64, 1, 1, 64), KP_S(FORM_F64, 2, 1, 64), KP_S(FORM_F64, 4, 1, 64),
    KP_S(FORM_BF16X3, 1, 2, 32), KP_S(FORM_BF16X3, 2, 2, 32), KP_S(FORM_BF16X3, 4, 2, 32),
    KP_S(FORM_BF16X3, 1, 1, 64), KP_S(FORM_BF16X3, 2, 1, 64), KP_S(FORM_BF16X3, 4, 1, 64),
    KP_S(FORM_BF16X6, 1, 1, 32), KP_S(FORM_BF16X6, 2, 1, 32), KP_S(FORM_BF16X6, 4, 1, 32),
    KP_S(FORM_BF16X6, 1, 1, 64), KP_S(FORM_BF16X6, 2, 1, 64), KP_S(FORM_BF16X6, 4, 1, 64),
};

const StripVariant* find_strip(int form, const ModeTile& t) {
  for (const StripVariant& v : kStrips)
    if (v.form == form && v.nb == t.nb && v.kp == t.bk && (t.fb == 0 || v.fb == t.fb))
      return &v;
  return nullptr;
}

int max_strip(int) { return 64; }

// Resident workgroups per CU of a kernel (queried once per kernel).
int blocks_per_cu(StripFn fn) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  const auto it = cache.find(reinterpret_cast<const void*>(fn));
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(fn),
                                                   kThreads, 0) != hipSuccess ||
      nb < 1)
    nb = 1;
  cache[reinterpret_cast<const void*>(fn)] = nb;
  return nb;
}

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  return cus;
}

}  // namespace

bool strip_default(int form, int64_t Il, int64_t m, int64_t n, int64_t Ir, ModeTile* out) {
  if (m < 1 || m > max_strip(form)) return false;
  // Ir < 0: no adjustment for the problem size (the batched executor)
  const bool sized = Ir >= 0;
  const int64_t F = Il > 1 ? Il * Ir : Ir;
  // FP64 with 32 < m <= 64: the 48- and 64-long strips (one or two
  // workgroups per CU) beat the k-loop tile on the lead layout, and on the
  // inner layout only for small problems
  if (form == FORM_F64 && m > 32 && Il > 1 && (!sized || F > 65536)) return false;
  // Inner layout, more than 64K fibers, 16 < n <= 64 and 16 < m <= 32
  // (FP64) or 16 < m (FP32): the k-loop tiles measured 5-20 % faster (FP32
  // m = 40-48: 30-50 %); for n <= 16 the strip stays ahead
  if (sized && Il > 1 && F > 65536 && m > 16 && n > 16 && n <= 64 &&
      (form == FORM_F32 || form == FORM_F64))
    return false;
  // FP32 with m <= 16: the k-loop tile (one chunk, 16-byte loads) measured
  // faster than the strip, except for m < 16 and n <= 16 over many fibers
  // (strips 10-50 % faster from 512K fibers on)
  if (form == FORM_F32 && m <= 16 && !(sized && m < 16 && n <= 16 && F >= 524288))
    return false;
  const int kp = form == FORM_BF16X3 || form == FORM_BF16X6
                     ? (m <= 32 ? 32 : 64)
                     : (m <= 16 ? 16 : (m <= 32 ? 32 : (form == FORM_F64 && m <= 48 ? 48 : 64)));
  int nb = n <= 16 ? 1 : (n <= 32 ? 2 : 4);
  // small problems: fewer rows per workgroup, so that the workgroups (fiber
  // tiles times n blocks) still spread over the chip
  ModeTile t{nb, 0, kp, 0, 0, 1};
  ModeTile r;
  while (sized && strip_resolve(form, t, &r) && t.nb > 1 &&
         ((F + 64 * r.fb - 1) / (64 * r.fb)) * ((n + 16 * t.nb - 1) / (16 * t.nb)) < 512)
    t.nb /= 2;
  return strip_resolve(form, t, out);
}

bool strip_resolve(int form, const ModeTile& t, ModeTile* out) {
  if (t.kind != 1) return false;
  const StripVariant* v = find_strip(form, t);
  if (!v) return false;
  *out = ModeTile{v->nb, v->fb, v->kp, 0, 0, 1};
  return true;
}

int list_strip_variants(int form, int32_t* out, int cap) {
  int count = 0;
  for (const StripVariant& v : kStrips) {
    if (v.form != form) continue;
    if (count < cap) {
      int32_t* o = out + 6 * count;
      o[0] = v.nb;
      o[1] = v.fb;
      o[2] = v.kp;
      o[3] = 0;
      o[4] = 0;
      o[5] = 1;
    }
    ++count;
  }
  return count;
}

hipError_t launch_strip(int form, const ModeArgs& a, const ModeTile& t, hipStream_t stream) {
  const StripVariant* v = find_strip(form, t);
  if (!v || a.m > v->kp) return hipErrorInvalidValue;
  const bool inner = a.Il > 1;
  const int64_t F = inner ? a.Il * a.Ir : a.Ir;
  if (F == 0 || a.n == 0) return hipSuccess;
  const int64_t es = form == FORM_F64 ? 8 : 4;
  // lead layout: 16-byte loads when every fiber row starts 16-byte aligned
  const bool vec = !inner && ((a.m * es) % 16) == 0 &&
                   (reinterpret_cast<uintptr_t>(a.X) % 16) == 0;
  const StripFn fn = inner ? v->inner : (vec ? v->lead_vec : v->lead);
  const int64_t bf = 64 * v->fb, bn = 16 * v->nb;
  const int64_t ntiles = (F + bf - 1) / bf;
  const int64_t nby = (a.n + bn - 1) / bn;
  if (nby > 65535) return hipErrorInvalidConfiguration;
  const int64_t slots = static_cast<int64_t>(blocks_per_cu(fn)) * device_cus();
  int64_t gx = (slots + nby - 1) / nby;
  if (gx > ntiles) gx = ntiles;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(gx), static_cast<unsigned>(nby)),
                     dim3(kThreads), 0, stream, a, ntiles);
  return hipGetLastError();
}

}  // namespace kp
