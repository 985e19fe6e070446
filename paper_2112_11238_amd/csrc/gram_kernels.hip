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

// dL(i, j) = sum_s part[s][i][j], written at dL[i*rs + j*cs].
template <typename E>
__global__ __launch_bounds__(kThreads) void gram_reduce(const E* __restrict__ part, int64_t splits,
                                                        int64_t n, int64_t m, E* __restrict__ dL,
                                                        int64_t rs, int64_t cs) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= n * m) return;
  const int64_t i = idx / m, j = idx - (idx / m) * m;
  E s = E(0);
  for (int64_t k = 0; k < splits; ++k) s += part[k * n * m + idx];
  dL[i * rs + j * cs] = s;
}

constexpr int kBR = 32;

}  // namespace

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
  return static_cast<size_t>(gram_splits(Il, n, m, Ir) * n * m) * esize;
}

hipError_t launch_gram(int dtype, const void* Q, const void* P, int64_t Il, int64_t n, int64_t m,
                       int64_t Ir, void* part, void* dL, int64_t rs, int64_t cs,
                       hipStream_t stream) {
  if (n == 0 || m == 0) return hipSuccess;
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
  const int64_t total = n * m;
  const unsigned blocks = static_cast<unsigned>((total + kThreads - 1) / kThreads);
  if (dtype == KP_F64)
    hipLaunchKernelGGL(gram_reduce<double>, dim3(blocks), dim3(kThreads), 0, stream,
                       static_cast<const double*>(part), splits, n, m, static_cast<double*>(dL),
                       rs, cs);
  else
    hipLaunchKernelGGL(gram_reduce<float>, dim3(blocks), dim3(kThreads), 0, stream,
                       static_cast<const float*>(part), splits, n, m, static_cast<float*>(dL), rs,
                       cs);
  return hipGetLastError();
}

}  // namespace kp
