// FP64 matrix exponential of small matrices: the 1-D factors exp(tau A_mu)
// of the exponential of a Kronecker sum (Sec. 3.3: exp(tau(A_d (+) ... (+)
// A_1)) v is the Tucker operator of V with the factors exp(tau A_mu)).
//
// Method: scaling and squaring with the diagonal [13/13] Pade approximant
// (N. J. Higham, "The scaling and squaring method for the matrix exponential
// revisited", SIAM J. Matrix Anal. Appl. 26(4), 2005). With B = tau A and
// s = max(0, ceil(log2(||B||_1 / theta_13))), theta_13 = 5.371920351148152:
//   B <- B / 2^s,  p(B) = V + U,  q(B) = V - U  (even / odd parts),
//   solve q(B) R = p(B),  exp(tau A) ~= R^(2^s).
// The scaling exponent depends on the data, and the library never
// synchronises with the host, so every step (norm, scaling, products, the
// LU solve with partial pivoting, the squarings) runs inside one persistent
// workgroup per matrix; `count` matrices run side by side in one launch.
// The products run on the FP64 matrix cores; for n <= 128 the LU factors of
// q(B) stay in LDS and each column of the right-hand side is solved in
// registers by one wave.
#include "kp.h"

#include <math.h>

#include "kp_common.h"
#include "kp_internal.h"

namespace kp {
namespace {

constexpr int kT = 1024;       // threads per workgroup
constexpr int kTile = 64;      // C tile edge of the block GEMM
constexpr int kKc = 64;        // k chunk of the block GEMM
constexpr double kTheta13 = 5.371920351148152;
constexpr int kSmallN = 128;   // largest n whose LU factors stay in LDS

struct PadeCoef {
  double c[14];
};

// C = A * B for n x n column-major matrices in global memory, computed by the
// whole workgroup through LDS tiles on the FP64 matrix cores: each of the 16
// waves owns one 16 x 16 block of a 64 x 64 tile of C and adds one 16x16x4
// MFMA product per 4 k values of each 64-wide k chunk staged in LDS
// (operand fragments: lane l holds A(row l mod 16, k l / 16) and
// B(k l / 16, column l mod 16); result item v of lane l is
// C(4v + l / 16, l mod 16)).
__device__ void block_gemm(const double* __restrict__ A, const double* __restrict__ B,
                           double* __restrict__ C, int n, double (*As)[kKc + 1],
                           double (*Bs)[kTile + 1]) {
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wr = w & 3, wc = w >> 2;  // this wave's 16 x 16 block of the tile
  const int c = lane & 15, g = lane >> 4;
  for (int i0 = 0; i0 < n; i0 += kTile)
    for (int j0 = 0; j0 < n; j0 += kTile) {
      d4_t acc = {0.0, 0.0, 0.0, 0.0};
      for (int k0 = 0; k0 < n; k0 += kKc) {
        // stage A[i0:i0+64, k0:k0+16] and B[k0:k0+16, j0:j0+64]
        for (int e = t; e < kTile * kKc; e += kT) {
          const int r = e % kTile, kk = e / kTile;
          const int i = i0 + r, k = k0 + kk;
          As[r][kk] = (i < n && k < n) ? A[i + static_cast<int64_t>(n) * k] : 0.0;
        }
        for (int e = t; e < kTile * kKc; e += kT) {
          const int kk = e % kKc, cc = e / kKc;
          const int k = k0 + kk, j = j0 + cc;
          Bs[kk][cc] = (k < n && j < n) ? B[k + static_cast<int64_t>(n) * j] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kKc; kk += 4)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(As[16 * wr + c][kk + g],
                                                    Bs[kk + g][16 * wc + c], acc, 0, 0, 0);
        __syncthreads();
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + 16 * wr + 4 * v + g, j = j0 + 16 * wc + c;
        if (i < n && j < n) C[i + static_cast<int64_t>(n) * j] = acc[v];
      }
    }
  __syncthreads();
}

__device__ double block_max(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (t < s) red[t] = fmax(red[t], red[t + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Index of the entry of largest magnitude among v over the block (ties: the
// smallest index), for partial pivoting: a butterfly within each wave, then
// one over the 16 wave results. The order (value descending, index
// ascending) is total, so every lane of a butterfly ends with the same pair.
__device__ __forceinline__ void argmax_step(double& v, int& idx, int off) {
  const double o = __shfl_xor(v, off);
  const int oi = __shfl_xor(idx, off);
  if (o > v || (o == v && oi < idx)) {
    v = o;
    idx = oi;
  }
}

__device__ int block_argmax(double v, int idx, double* red, int* redi) {
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  for (int off = 32; off >= 1; off >>= 1) argmax_step(v, idx, off);
  if (lane == 0) {
    red[w] = v;
    redi[w] = idx;
  }
  __syncthreads();
  if (w == 0) {
    constexpr int kWaves = kT / 64;
    v = lane < kWaves ? red[lane] : -1.0;
    idx = lane < kWaves ? redi[lane] : 0x7fffffff;
    for (int off = kWaves / 2; off >= 1; off >>= 1) argmax_step(v, idx, off);
    if (lane == 0) redi[kWaves] = idx;
  }
  __syncthreads();
  const int r = redi[kT / 64];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kT) void expm_pade13(const double* __restrict__ Ain, int n,
                                                  double tau, double* __restrict__ Eout,
                                                  double* __restrict__ ws, PadeCoef pc) {
  // LDS: the GEMM tiles, or (n <= kSmallN) the LU factors of the Pade
  // denominator during the solve
  __shared__ __attribute__((aligned(16))) double smem[kSmallN * kSmallN];
  __shared__ double red[kT];
  __shared__ int redi[kT];
  __shared__ int spiv[kSmallN], sperm[kSmallN];
  auto As = reinterpret_cast<double(*)[kKc + 1]>(smem);
  auto Bs = reinterpret_cast<double(*)[kTile + 1]>(smem + kTile * (kKc + 1));
  const int64_t nn = static_cast<int64_t>(n) * n;
  const double* A = Ain + blockIdx.x * nn;
  double* E = Eout + blockIdx.x * nn;
  double* W = ws + blockIdx.x * 8 * nn;
  double* B = W;
  double* B2 = W + nn;
  double* B4 = W + 2 * nn;
  double* B6 = W + 3 * nn;
  double* T1 = W + 4 * nn;
  double* T2 = W + 5 * nn;
  double* U = W + 6 * nn;
  double* V = W + 7 * nn;
  const int t = threadIdx.x;

  // B = tau A and its 1-norm (largest absolute column sum)
  double colmax = 0.0;
  for (int j = t; j < n; j += kT) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += fabs(tau * A[i + static_cast<int64_t>(n) * j]);
    colmax = fmax(colmax, s);
  }
  const double norm1 = block_max(colmax, red);
  int s = 0;  // non-finite norms keep s = 0 and propagate as NaN/Inf
  if (isfinite(norm1) && norm1 > kTheta13) s = static_cast<int>(ceil(log2(norm1 / kTheta13)));
  if (s < 0) s = 0;
  if (s > 1100) s = 1100;
  for (int64_t e = t; e < nn; e += kT) B[e] = ldexp(tau * A[e], -s);
  __syncthreads();

  block_gemm(B, B, B2, n, As, Bs);
  block_gemm(B2, B2, B4, n, As, Bs);
  block_gemm(B4, B2, B6, n, As, Bs);
  const double* c = pc.c;
  // odd part: U = B (B6 (c13 B6 + c11 B4 + c9 B2) + c7 B6 + c5 B4 + c3 B2 + c1 I)
  for (int64_t e = t; e < nn; e += kT) T1[e] = c[13] * B6[e] + c[11] * B4[e] + c[9] * B2[e];
  __syncthreads();
  block_gemm(B6, T1, T2, n, As, Bs);
  for (int64_t e = t; e < nn; e += kT) {
    const bool diag = (e % n) == (e / n);
    T2[e] += c[7] * B6[e] + c[5] * B4[e] + c[3] * B2[e] + (diag ? c[1] : 0.0);
  }
  __syncthreads();
  block_gemm(B, T2, U, n, As, Bs);
  // even part: V = B6 (c12 B6 + c10 B4 + c8 B2) + c6 B6 + c4 B4 + c2 B2 + c0 I
  for (int64_t e = t; e < nn; e += kT) T1[e] = c[12] * B6[e] + c[10] * B4[e] + c[8] * B2[e];
  __syncthreads();
  block_gemm(B6, T1, V, n, As, Bs);
  for (int64_t e = t; e < nn; e += kT) {
    const bool diag = (e % n) == (e / n);
    V[e] += c[6] * B6[e] + c[4] * B4[e] + c[2] * B2[e] + (diag ? c[0] : 0.0);
  }
  __syncthreads();
  // M = V - U (into T1), R = V + U (into T2); solve M X = R in place.
  double* M = T1;
  double* R = T2;
  for (int64_t e = t; e < nn; e += kT) {
    M[e] = V[e] - U[e];
    R[e] = V[e] + U[e];
  }
  __syncthreads();
  if (n <= kSmallN) {
    // LU with partial pivoting of M in LDS, then each column of R solved in
    // registers by one wave (lane l holds rows l and l + 64; the value of
    // row k is broadcast from its lane), so the sweeps need no block barrier
    double* sM = smem;
    for (int64_t e = t; e < nn; e += kT) sM[e] = M[e];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
      double best = -1.0;
      int bi = k;
      if (k + t < n) {
        best = fabs(sM[k + t + n * k]);
        bi = k + t;
      }
      const int p = block_argmax(best, bi, red, redi);
      if (t == 0) spiv[k] = p;
      if (p != k) {
        for (int j = t; j < n; j += kT) {
          const double tmp = sM[k + n * j];
          sM[k + n * j] = sM[p + n * j];
          sM[p + n * j] = tmp;
        }
        __syncthreads();
      }
      const double piv = sM[k + n * k];
      for (int i = k + 1 + t; i < n; i += kT) sM[i + n * k] /= piv;
      __syncthreads();
      const int rows = n - k - 1;
      for (int e = t; e < rows * rows; e += kT) {
        const int i = k + 1 + e % rows, j = k + 1 + e / rows;
        sM[i + n * j] -= sM[i + n * k] * sM[k + n * j];
      }
      __syncthreads();
    }
    // row i of the permuted system is row sperm[i] of the original one
    if (t == 0) {
      for (int i = 0; i < n; ++i) sperm[i] = i;
      for (int k = 0; k < n; ++k) {
        const int tmp = sperm[k];
        sperm[k] = sperm[spiv[k]];
        sperm[spiv[k]] = tmp;
      }
    }
    __syncthreads();
    const int lane = t & 63, wv = t >> 6;
    for (int j = wv; j < n; j += kT / 64) {
      double x0 = lane < n ? R[sperm[lane] + static_cast<int64_t>(n) * j] : 0.0;
      double x1 = lane + 64 < n ? R[sperm[lane + 64] + static_cast<int64_t>(n) * j] : 0.0;
      for (int k = 0; k < n - 1; ++k) {  // unit lower triangle
        const double xk = __shfl(k < 64 ? x0 : x1, k & 63);
        if (lane > k && lane < n) x0 -= sM[lane + n * k] * xk;
        if (lane + 64 > k && lane + 64 < n) x1 -= sM[lane + 64 + n * k] * xk;
      }
      for (int k = n - 1; k >= 0; --k) {  // upper triangle
        if (lane == (k & 63)) {
          if (k < 64) x0 /= sM[k + n * k];
          else x1 /= sM[k + n * k];
        }
        const double xk = __shfl(k < 64 ? x0 : x1, k & 63);
        if (lane < k) x0 -= sM[lane + n * k] * xk;
        if (lane + 64 < k) x1 -= sM[lane + 64 + n * k] * xk;
      }
      if (lane < n) R[lane + static_cast<int64_t>(n) * j] = x0;
      if (lane + 64 < n) R[lane + 64 + static_cast<int64_t>(n) * j] = x1;
    }
    __syncthreads();
  }
  if (n > kSmallN) {
    // larger matrices: the same elimination on M and R in global memory
    for (int k = 0; k < n; ++k) {
      double best = -1.0;
      int bi = k;
      for (int i = k + t; i < n; i += kT) {
        const double v = fabs(M[i + static_cast<int64_t>(n) * k]);
        if (v > best) {
          best = v;
          bi = i;
        }
      }
      const int p = block_argmax(best, bi, red, redi);
      if (p != k) {
        for (int j = t; j < 2 * n; j += kT) {
          double* X = (j < n) ? M : R;
          const int jj = (j < n) ? j : j - n;
          const int64_t a = k + static_cast<int64_t>(n) * jj, b = p + static_cast<int64_t>(n) * jj;
          const double tmp = X[a];
          X[a] = X[b];
          X[b] = tmp;
        }
        __syncthreads();
      }
      const double piv = M[k + static_cast<int64_t>(n) * k];
      // multipliers stored below the diagonal of column k
      for (int i = k + 1 + t; i < n; i += kT) M[i + static_cast<int64_t>(n) * k] /= piv;
      __syncthreads();
      const int rows = n - k - 1;
      const int cols = (n - k - 1) + n;  // remaining columns of M, then all of R
      for (int e = t; e < rows * cols; e += kT) {
        const int i = k + 1 + e % rows;
        const int jc = e / rows;
        const double l = M[i + static_cast<int64_t>(n) * k];
        if (jc < n - k - 1) {
          const int j = k + 1 + jc;
          M[i + static_cast<int64_t>(n) * j] -= l * M[k + static_cast<int64_t>(n) * j];
        } else {
          const int j = jc - (n - k - 1);
          R[i + static_cast<int64_t>(n) * j] -= l * R[k + static_cast<int64_t>(n) * j];
        }
      }
      __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
      const double piv = M[k + static_cast<int64_t>(n) * k];
      for (int j = t; j < n; j += kT) R[k + static_cast<int64_t>(n) * j] /= piv;
      __syncthreads();
      for (int e = t; e < k * n; e += kT) {
        const int i = e % k, j = e / k;
        R[i + static_cast<int64_t>(n) * j] -= M[i + static_cast<int64_t>(n) * k] *
                                              R[k + static_cast<int64_t>(n) * j];
      }
      __syncthreads();
    }
  }
  // squarings: R <- R^2, s times (ping-pong between T2 and U)
  double* cur = R;
  double* nxt = U;
  for (int it = 0; it < s; ++it) {
    block_gemm(cur, cur, nxt, n, As, Bs);
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  for (int64_t e = t; e < nn; e += kT) E[e] = cur[e];
}

// c_j = (2m - j)! m! / ((2m)! j! (m - j)!) for m = 13, j = 0..13 (the
// coefficients of the numerator of the diagonal Pade approximant of e^x).
PadeCoef pade13() {
  PadeCoef p;
  const int m = 13;
  double c = 1.0;
  p.c[0] = 1.0;
  for (int j = 1; j <= m; ++j) {
    c *= static_cast<double>(m - j + 1) / (static_cast<double>(2 * m - j + 1) * j);
    p.c[j] = c;
  }
  return p;
}

}  // namespace
}  // namespace kp

using namespace kp;

extern "C" {

size_t kp_expm_workspace(int64_t n, int64_t count) {
  if (n <= 0 || count <= 0) return 0;
  return static_cast<size_t>(8 * n * n * count) * sizeof(double);
}

int kp_expm_f64(const double* A, int64_t n, int64_t count, double tau, double* E, void* ws,
                size_t ws_bytes, hipStream_t stream) {
  if (n < 0 || count < 0) return KP_ERR_SHAPE;
  if (n > 256) return KP_ERR_SHAPE;
  if (n == 0 || count == 0) return KP_OK;
  if (!A || !E) return KP_ERR_NULL;
  if (!isfinite(tau)) return KP_ERR_VALUE;
  const size_t need = kp_expm_workspace(n, count);
  if (!ws || ws_bytes < need) return KP_ERR_WORKSPACE;
  const size_t mb = static_cast<size_t>(n * n * count) * sizeof(double);
  const char* a = reinterpret_cast<const char*>(A);
  const char* e = reinterpret_cast<const char*>(E);
  const char* w = static_cast<const char*>(ws);
  if ((e < a + mb && a < e + mb) || (e < w + need && w < e + mb)) return KP_ERR_ALIAS;
  hipLaunchKernelGGL(expm_pade13, dim3(static_cast<unsigned>(count)), dim3(kT), 0, stream, A,
                     static_cast<int>(n), tau, E, static_cast<double*>(ws), pade13());
  return hip_status(hipGetLastError());
}

}  // extern "C"
