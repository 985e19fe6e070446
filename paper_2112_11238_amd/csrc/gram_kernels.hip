// Factor-gradient contraction for the Tucker operator's backward pass.
//
// dL_mu(i, j) = sum over every fiber r of Q(r, i) * P(r, j), where Q is the
// cotangent swept back to mode mu (view (Il, n, Ir)) and P the forward partial
// product before mode mu (view (Il, m, Ir)); r = a + Il*b runs over the Il*Ir
// fibers. The gradient rule follows from the Kronecker form of the Tucker
// operator (Sec. 2, the Lemma on vec(S)) and the transpose rule of Appendix A
// (property 5); the paper itself does not treat derivatives.
//
// The fiber sum is long (up to ~10^8 terms) and the result small (n x m), so
// the sum is split: workgroup (ti, tj, s) accumulates a 64 x 64 tile of C over
// its share of fiber chunks with MFMA, writes the partial tile to a workspace,
// and a second kernel adds the shares in a fixed order (deterministic) and
// writes dL with its own strides.
#include <mutex>
#include <unordered_map>

#include "gram_strip.h"
#include "gram_tile.h"
#include "kp_common.h"
#include "kp_internal.h"

namespace kp {
namespace {

using namespace gram;

template <typename E, int BR, bool INNER>
__global__ __launch_bounds__(kThreads, 2) void gram_kernel(GramArgs g) {
  __shared__ __attribute__((aligned(16))) char lds[gram_lds_bytes<E, BR>()];
  gram_tile<E, BR, INNER>(g, blockIdx.x, blockIdx.y, blockIdx.z, lds);
}

// dL(i, j) = sum_s part[s][i][j] in a fixed order, written at dL[i*rs + j*cs];
// workgroup x handles outputs 16x .. 16x + 15.
template <typename E, int OPB>
__global__ __launch_bounds__(kThreads) void gram_reduce(const E* __restrict__ part, int64_t splits,
                                                        int64_t n, int64_t m, E* __restrict__ dL,
                                                        int64_t rs, int64_t cs) {
  __shared__ E sred[kThreads];
  gram_reduce_block<E, OPB>(part, splits, n, m, dL, rs, cs, blockIdx.x, sred);
}

// dL = the fixed-order sum of `splits` partial tiles.
hipError_t launch_reduce(int dtype, const void* part, int64_t splits, int64_t n, int64_t m,
                         void* dL, int64_t rs, int64_t cs, hipStream_t stream) {
  const int opb = reduce_outputs(splits, n * m);
  const unsigned blocks = static_cast<unsigned>((n * m + opb - 1) / opb);
  if (dtype == KP_F64) {
    const double* p = static_cast<const double*>(part);
    double* o = static_cast<double*>(dL);
    if (opb == 4)
      hipLaunchKernelGGL((gram_reduce<double, 4>), dim3(blocks), dim3(kThreads), 0, stream, p,
                         splits, n, m, o, rs, cs);
    else
      hipLaunchKernelGGL((gram_reduce<double, 16>), dim3(blocks), dim3(kThreads), 0, stream, p,
                         splits, n, m, o, rs, cs);
  } else {
    const float* p = static_cast<const float*>(part);
    float* o = static_cast<float*>(dL);
    if (opb == 4)
      hipLaunchKernelGGL((gram_reduce<float, 4>), dim3(blocks), dim3(kThreads), 0, stream, p,
                         splits, n, m, o, rs, cs);
    else
      hipLaunchKernelGGL((gram_reduce<float, 16>), dim3(blocks), dim3(kThreads), 0, stream, p,
                         splits, n, m, o, rs, cs);
  }
  return hipGetLastError();
}

constexpr int kBR = 32;

// Small factors (n, m <= 64): one partial tile per workgroup, each
// workgroup streaming a contiguous run of fiber chunks (gram_strip.h).
template <typename E>
constexpr int strip_br() { return sizeof(E) == 8 ? 32 : 64; }
constexpr int64_t kMaxStripSplits = 2048;

template <typename E, int NB, int MB, bool INNER, bool VEC = false>
__global__ __launch_bounds__(kThreads, 2) void gram_strip_kernel(GramArgs g, int64_t chunks,
                                                                 int64_t splits) {
  constexpr int BR = strip_br<E>();
  __shared__ __attribute__((aligned(16))) char lds[strip_lds_bytes<E, NB, MB, BR>()];
  const int64_t s = blockIdx.x;
  const int64_t cb = s * chunks / splits, ce = (s + 1) * chunks / splits;
  gram_strip<E, NB, MB, BR, INNER, VEC>(g, cb, ce, static_cast<E*>(g.part) + s * g.n * g.m,
                                        lds);
}

// The fused backward step: the gram's partial tiles and Y = the mu-mode
// product with L^T, from one read of Q (FP32, inner layout with 16-byte
// fiber groups, n <= 32, m <= 32; JB = 16-row blocks of m, also the P tile's:
// with m <= 16 the LDS footprint allows four workgroups per CU, whose
// chunks in flight keep HBM busy).
template <int PFORM, int JB>
__global__ __launch_bounds__(kThreads, 2) void gram_product_kernel(GramArgs g, GramProduct prod,
                                                                   int64_t chunks,
                                                                   int64_t splits) {
  constexpr int BR = strip_br<float>();
  __shared__ __attribute__((aligned(16))) char lds[strip_lds_bytes<float, 2, JB, BR, JB>()];
  const int64_t s = blockIdx.x;
  const int64_t cb = s * chunks / splits, ce = (s + 1) * chunks / splits;
  gram_strip<float, 2, JB, BR, true, true, JB, PFORM>(
      g, cb, ce, static_cast<float*>(g.part) + s * g.n * g.m, lds, &prod);
}

using StripGramFn = void (*)(GramArgs, int64_t, int64_t);

// vec: inner layout with fiber groups of 16 bytes (I_l a multiple of the
// group, Q and P 16-byte aligned)
template <typename E>
StripGramFn strip_gram_fn(int64_t n, int64_t m, bool inner, bool vec) {
  const bool n2 = n <= 32, m2 = m <= 32;
  if (inner && vec) {
    if (n2)
      return m2 ? gram_strip_kernel<E, 2, 2, true, true> : gram_strip_kernel<E, 2, 4, true, true>;
    return m2 ? gram_strip_kernel<E, 4, 2, true, true> : gram_strip_kernel<E, 4, 4, true, true>;
  }
  if (inner) {
    if (n2) return m2 ? gram_strip_kernel<E, 2, 2, true> : gram_strip_kernel<E, 2, 4, true>;
    return m2 ? gram_strip_kernel<E, 4, 2, true> : gram_strip_kernel<E, 4, 4, true>;
  }
  if (n2) return m2 ? gram_strip_kernel<E, 2, 2, false> : gram_strip_kernel<E, 2, 4, false>;
  return m2 ? gram_strip_kernel<E, 4, 2, false> : gram_strip_kernel<E, 4, 4, false>;
}

bool use_strip(int64_t Il, int64_t n, int64_t m, int64_t Ir, size_t esize) {
  const int64_t rows = n > m ? n : m;
  return n <= 64 && m <= 64 &&
         Il * Ir * rows * static_cast<int64_t>(esize) < (static_cast<int64_t>(1) << 31);
}

int64_t strip_chunks(int64_t Il, int64_t Ir, size_t esize) {
  const int64_t br = esize == 8 ? 32 : 64;
  return (Il * Ir + br - 1) / br;
}

int strip_slots(StripGramFn fn) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  const auto it = cache.find(reinterpret_cast<const void*>(fn));
  int nb = 1;
  if (it != cache.end()) {
    nb = it->second;
  } else {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(fn),
                                                     kThreads, 0) != hipSuccess ||
        nb < 1)
      nb = 1;
    cache[reinterpret_cast<const void*>(fn)] = nb;
  }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  return nb * cus;
}

}  // namespace

bool gram_product_eligible(int dtype, const void* Q, const void* P, const void* Y, int64_t Il,
                           int64_t n, int64_t m, int64_t Ir) {
  return dtype == KP_F32 && Il > 1 && Il % 4 == 0 && n >= 1 && m >= 1 && n <= 32 && m <= 32 &&
         use_strip(Il, n, m, Ir, 4) && reinterpret_cast<uintptr_t>(Q) % 16 == 0 &&
         reinterpret_cast<uintptr_t>(P) % 16 == 0 && reinterpret_cast<uintptr_t>(Y) % 16 == 0;
}

hipError_t launch_gram_product(int form, const void* Q, const void* P, int64_t Il, int64_t n,
                               int64_t m, int64_t Ir, void* part, void* dL, int64_t rs, int64_t cs,
                               const kp_matrix& L, void* Y, hipStream_t stream) {
  if (form != FORM_F32 && form != FORM_BF16X3 && form != FORM_BF16X6) return hipErrorInvalidValue;
  if (!gram_product_eligible(KP_F32, Q, P, Y, Il, n, m, Ir)) return hipErrorInvalidValue;
  GramArgs g{};
  g.Q = Q;
  g.P = P;
  g.part = part;
  g.Il = Il;
  g.n = n;
  g.m = m;
  g.Ir = Ir;
  GramProduct prod{};
  prod.L = static_cast<const float*>(L.data);
  prod.Y = static_cast<float*>(Y);
  prod.rs = L.rs;
  prod.cs = L.cs;
  const int64_t chunks = strip_chunks(Il, Ir, 4);
  using Fn = void (*)(GramArgs, GramProduct, int64_t, int64_t);
  const Fn fn = form == FORM_F32      ? (m <= 16 ? gram_product_kernel<FORM_F32, 1>
                                                 : gram_product_kernel<FORM_F32, 2>)
                : form == FORM_BF16X3 ? (m <= 16 ? gram_product_kernel<FORM_BF16X3, 1>
                                                 : gram_product_kernel<FORM_BF16X3, 2>)
                                      : (m <= 16 ? gram_product_kernel<FORM_BF16X6, 1>
                                                 : gram_product_kernel<FORM_BF16X6, 2>);
  int64_t splits = strip_slots(reinterpret_cast<StripGramFn>(fn));
  if (splits > chunks) splits = chunks;
  if (splits > kMaxStripSplits) splits = kMaxStripSplits;
  if (splits < 1) splits = 1;
  hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(splits)), dim3(kThreads), 0, stream, g, prod,
                     chunks, splits);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce(KP_F32, part, splits, n, m, dL, rs, cs, stream);
}

int64_t gram_splits(int64_t Il, int64_t n, int64_t m, int64_t Ir) {
  const int64_t tiles = ((n + 63) / 64) * ((m + 63) / 64);
  const int64_t chunks = Il > 1 ? Ir * ((Il + kBR - 1) / kBR) : (Ir + kBR - 1) / kBR;
  int64_t s = (1024 + tiles - 1) / tiles;
  if (s > chunks) s = chunks;
  if (s < 1) s = 1;
  if (s > 65535) s = 65535;
  return s;
}

size_t gram_workspace(int64_t Il, int64_t n, int64_t m, int64_t Ir, size_t esize) {
  if (use_strip(Il, n, m, Ir, esize)) {
    int64_t s = strip_chunks(Il, Ir, esize);
    if (s > kMaxStripSplits) s = kMaxStripSplits;
    if (s < 1) s = 1;
    return static_cast<size_t>(s * n * m) * esize;
  }
  return static_cast<size_t>(gram_splits(Il, n, m, Ir) * n * m) * esize;
}

hipError_t launch_gram(int dtype, const void* Q, const void* P, int64_t Il, int64_t n, int64_t m,
                       int64_t Ir, void* part, void* dL, int64_t rs, int64_t cs,
                       hipStream_t stream) {
  if (n == 0 || m == 0) return hipSuccess;
  const size_t es = dtype == KP_F64 ? 8 : 4;
  if (use_strip(Il, n, m, Ir, es)) {
    GramArgs g{};
    g.Q = Q;
    g.P = P;
    g.part = part;
    g.Il = Il;
    g.n = n;
    g.m = m;
    g.Ir = Ir;
    const bool inner = Il > 1;
    const int64_t kv = 16 / static_cast<int64_t>(es);
    const bool vec = inner && Il % kv == 0 && reinterpret_cast<uintptr_t>(Q) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(P) % 16 == 0;
    const int64_t chunks = strip_chunks(Il, Ir, es);
    const StripGramFn fn = dtype == KP_F64 ? strip_gram_fn<double>(n, m, inner, vec)
                                           : strip_gram_fn<float>(n, m, inner, vec);
    int64_t splits = strip_slots(fn);
    if (splits > chunks) splits = chunks;
    if (splits > kMaxStripSplits) splits = kMaxStripSplits;
    if (splits < 1) splits = 1;
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(splits)), dim3(kThreads), 0, stream, g,
                       chunks, splits);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce(dtype, part, splits, n, m, dL, rs, cs, stream);
  }
  GramArgs g;
  g.Q = Q;
  g.P = P;
  g.part = part;
  g.Il = Il;
  g.n = n;
  g.m = m;
  g.Ir = Ir;
  const bool inner = Il > 1;
  g.achunks = inner ? (Il + kBR - 1) / kBR : 1;
  g.chunks = inner ? Ir * g.achunks : (Ir + kBR - 1) / kBR;
  const int64_t splits = gram_splits(Il, n, m, Ir);
  g.per_split = (g.chunks + splits - 1) / splits;
  const dim3 grid(static_cast<unsigned>((n + 63) / 64), static_cast<unsigned>((m + 63) / 64),
                  static_cast<unsigned>(splits));
  if (dtype == KP_F64) {
    if (inner)
      hipLaunchKernelGGL((gram_kernel<double, kBR, true>), grid, dim3(kThreads), 0, stream, g);
    else
      hipLaunchKernelGGL((gram_kernel<double, kBR, false>), grid, dim3(kThreads), 0, stream, g);
  } else {
    if (inner)
      hipLaunchKernelGGL((gram_kernel<float, kBR, true>), grid, dim3(kThreads), 0, stream, g);
    else
      hipLaunchKernelGGL((gram_kernel<float, kBR, false>), grid, dim3(kThreads), 0, stream, g);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce(dtype, part, splits, n, m, dL, rs, cs, stream);
}

}  // namespace kp
