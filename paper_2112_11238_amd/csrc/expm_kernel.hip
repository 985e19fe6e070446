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
// The library never synchronises with the host, so the data-dependent
// scaling exponent stays on the device. The steps are separate launches on
// the caller's stream (kernel boundaries order them; no workgroup ever waits
// for another):
//   expm_scale    one workgroup per matrix: 1-norm, s (kept in the
//                 workspace), B = tau A 2^-s;
//   expm_gemm     the products, spread over 32 x 32 output tiles of every
//                 matrix on the FP64 matrix cores: B^2, B^4, B^6, then the
//                 odd and even parts with their linear combinations folded
//                 into the operand staging and the epilogue;
//   expm_solve    one workgroup per matrix: q(B) R = p(B) by Gauss-Jordan
//                 elimination with partial pivoting, q(B) in LDS and R in
//                 registers (n <= 128); larger n eliminate in global memory;
//   expm_gemm     kSquareLaunches squarings, each skipped by matrices whose
//                 s is smaller;
//   expm_finish   one workgroup per matrix: any squarings beyond those
//                 launches (s > kSquareLaunches) and the copy to E.
#include "kp.h"

#include <math.h>

#include <initializer_list>
#include <utility>

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

// ---------------------------------------------------------------------------
// Workspace: per matrix 8 n^2 doubles in these slots, then one int per
// matrix (its scaling exponent s).
enum Slot { W_B = 0, W_B2, W_B4, W_B6, W_Q0, W_U, W_V, W_Q1, kSlots };

constexpr int kGT = 32;          // output tile edge of expm_gemm
constexpr int kGThreads = 256;   // four waves, one 16 x 16 block each
constexpr int kMaxN = 256;
constexpr int kSquareLaunches = 8;
constexpr int kScaleThreads = 256;

__device__ __forceinline__ double* slot(double* ws, int64_t nn, int mat, int k) {
  return ws + (static_cast<int64_t>(mat) * kSlots + k) * nn;
}

// B = tau A 2^-s with s from the 1-norm of tau A (largest absolute column
// sum); one workgroup per matrix, one thread per column.
__global__ __launch_bounds__(kScaleThreads) void expm_scale(const double* __restrict__ Ain, int n,
                                                            double tau, double* __restrict__ ws,
                                                            int* __restrict__ svec) {
  __shared__ double red[kScaleThreads];
  __shared__ int s_sh;
  const int64_t nn = static_cast<int64_t>(n) * n;
  const int mat = blockIdx.x;
  const double* A = Ain + mat * nn;
  const int t = threadIdx.x;
  double colsum = 0.0;
  if (t < n) {
    const double* col = A + static_cast<int64_t>(n) * t;
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    int i = 0;
    for (; i + 4 <= n; i += 4)
#pragma unroll
      for (int q = 0; q < 4; ++q) part[q] += fabs(tau * col[i + q]);
    for (; i < n; ++i) part[0] += fabs(tau * col[i]);
    colsum = (part[0] + part[1]) + (part[2] + part[3]);
  }
  red[t] = colsum;
  __syncthreads();
  for (int st = kScaleThreads / 2; st > 0; st >>= 1) {
    if (t < st) red[t] = fmax(red[t], red[t + st]);
    __syncthreads();
  }
  if (t == 0) {
    const double norm1 = red[0];
    int s = 0;  // non-finite norms keep s = 0 and propagate as NaN/Inf
    if (isfinite(norm1) && norm1 > kTheta13) s = static_cast<int>(ceil(log2(norm1 / kTheta13)));
    if (s < 0) s = 0;
    if (s > 1100) s = 1100;
    s_sh = s;
    svec[mat] = s;
  }
  __syncthreads();
  const int s = s_sh;
  double* B = slot(ws, nn, mat, W_B);
  for (int64_t e = t; e < nn; e += kScaleThreads) B[e] = ldexp(tau * A[e], -s);
}

// One product of the method: C = A (sum_i beta_i M_i) + sum_j eps_j N_j +
// diag I, every operand a workspace slot of the same matrix.
struct GemmJob {
  int a;            // slot of the left factor
  int nb;           // terms of the right factor (1..3)
  int b[3];
  double beta[3];
  int ne;           // added terms (0..3)
  int e[3];
  double eps[3];
  double diag;
  int c;            // output slot
  int square;       // >= 0: a squaring, skipped by matrices with s <= square
};
struct GemmJobs {
  GemmJob job[2];
  int njobs;
};

// The products over 32 x 32 output tiles of every matrix (and job): the
// tile's 32 rows of A and 32 columns of the combined right factor, all of k,
// are staged in LDS (the combination formed while staging), then each wave
// accumulates one 16 x 16 block with the FP64 16x16x4 MFMA (lane l holds
// A(row l mod 16, k l / 16) and B(k l / 16, column l mod 16); item v of lane
// l is C(4v + l / 16, l mod 16)), k ascending in steps of 4.
__global__ __launch_bounds__(kGThreads) void expm_gemm(double* __restrict__ ws, int n, int count,
                                                       GemmJobs jobs, const int* __restrict__ svec) {
  __shared__ double As[kGT][kMaxN + 1];
  __shared__ double Bs[kMaxN][kGT + 1];
  const int tps = (n + kGT - 1) / kGT;
  const int tiles = tps * tps;
  const int bid = blockIdx.x;
  const int tile = bid % tiles;
  const int mat = (bid / tiles) % count;
  const GemmJob& jb = jobs.job[bid / (tiles * count)];
  if (jb.square >= 0 && jb.square >= svec[mat]) return;  // uniform: this matrix is done
  const int64_t nn = static_cast<int64_t>(n) * n;
  const int i0 = (tile % tps) * kGT, j0 = (tile / tps) * kGT;
  const int npad = (n + 3) & ~3;
  const double* A = slot(ws, nn, mat, jb.a);
  const int t = threadIdx.x;
  // staging: every thread's loads are issued before its LDS stores
  constexpr int kPer = kGT * kMaxN / kGThreads;  // elements per thread, at most
  const int total = kGT * npad;
  double va[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = t + u * kGThreads;
    const int r = e % kGT, k = e / kGT;
    const int i = i0 + r;
    va[u] = (e < total && i < n && k < n) ? A[i + static_cast<int64_t>(n) * k] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = t + u * kGThreads;
    if (e < total) As[e % kGT][e / kGT] = va[u];
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = t + u * kGThreads;
    const int k = e % npad, cc = e / npad;
    const int j = j0 + cc;
    double v = 0.0;
    if (e < total && k < n && j < n) {
      const int64_t o = k + static_cast<int64_t>(n) * j;
      v = jb.beta[0] * slot(ws, nn, mat, jb.b[0])[o];
      if (jb.nb > 1) v += jb.beta[1] * slot(ws, nn, mat, jb.b[1])[o];
      if (jb.nb > 2) v += jb.beta[2] * slot(ws, nn, mat, jb.b[2])[o];
    }
    va[u] = v;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = t + u * kGThreads;
    if (e < total) Bs[e % npad][e / npad] = va[u];
  }
  __syncthreads();
  const int lane = t & 63, w = t >> 6;
  const int wr = w & 1, wc = w >> 1;
  const int c = lane & 15, g = lane >> 4;
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int kk = 0; kk < npad; kk += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(As[16 * wr + c][kk + g], Bs[kk + g][16 * wc + c],
                                               acc, 0, 0, 0);
  double* C = slot(ws, nn, mat, jb.c);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + 16 * wr + 4 * v + g, j = j0 + 16 * wc + c;
    if (i < n && j < n) {
      const int64_t o = i + static_cast<int64_t>(n) * j;
      double r = acc[v];
      for (int q = 0; q < jb.ne; ++q) r += jb.eps[q] * slot(ws, nn, mat, jb.e[q])[o];
      if (i == j) r += jb.diag;
      C[o] = r;
    }
  }
}

// q(B) R = p(B) with q(B) = V - U, p(B) = V + U, result R into slot Q0.
// n <= kSmallN: Gauss-Jordan elimination with partial pivoting, q(B) and R
// both in registers: thread t holds column t mod 128, rows t / 128 + 8 r, of
// each. Rows are never moved: step k picks, among the rows not yet used as
// pivots, the one of largest |q(B)(i, k)| (ties: the smallest i), scales it
// by its pivot and eliminates column k from every other row; row p_k then
// holds row k of the solution. Per step only column k and the scaled pivot
// row pass through LDS (double-buffered by the parity of k, so the writes
// of step k + 1 never meet the reads of step k). Larger n: elimination with
// partial pivoting (row swaps) and back substitution in global memory.
__global__ __launch_bounds__(kT) void expm_solve(double* __restrict__ ws, int n) {
  __shared__ double ccol[2][kSmallN], mrow[2][kSmallN], rrow[2][kSmallN];
  __shared__ double red[kT];
  __shared__ int redi[kT];
  __shared__ int used[kSmallN], pstep[kSmallN];
  __shared__ int sp[2];
  const int64_t nn = static_cast<int64_t>(n) * n;
  const int mat = blockIdx.x;
  const double* U = slot(ws, nn, mat, W_U);
  const double* V = slot(ws, nn, mat, W_V);
  double* R = slot(ws, nn, mat, W_Q0);
  const int t = threadIdx.x;
  if (n <= kSmallN) {
    constexpr int kRows = kT / kSmallN;  // 8 thread rows; thread row tr holds rows tr + 8 r
    constexpr int kPer = kSmallN / kRows;
    const int j = t % kSmallN, tr = t / kSmallN;
    double mr[kPer], rr[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int i = tr + kRows * r;
      const int64_t o = i + static_cast<int64_t>(n) * j;
      const bool in = i < n && j < n;
      mr[r] = in ? V[o] - U[o] : 0.0;
      rr[r] = in ? V[o] + U[o] : 0.0;
    }
    for (int i = t; i < kSmallN; i += kT) {
      used[i] = 0;
      ccol[0][i] = 0.0;  // rows past n stay zero: their updates are no-ops
      ccol[1][i] = 0.0;
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
      const int b = k & 1;
      // column k, from the threads holding it
      if (j == k) {
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
          const int i = tr + kRows * r;
          if (i < n) ccol[b][i] = mr[r];
        }
      }
      __syncthreads();
      // pivot among the unused rows (one wave; two rows per lane)
      if (t < 64) {
        double best = -1.0;
        int bi = 0x7fffffff;
        for (int i = t; i < n; i += 64) {
          const double v = used[i] ? -1.0 : fabs(ccol[b][i]);
          if (v > best || (v == best && i < bi)) {
            best = v;
            bi = i;
          }
        }
        for (int off = 32; off >= 1; off >>= 1) argmax_step(best, bi, off);
        if (t == 0) {
          sp[b] = bi;
          used[bi] = 1;
          pstep[bi] = k;
        }
      }
      __syncthreads();
      const int p = sp[b];
      const double piv = ccol[b][p];
      // the scaled pivot row, from the threads holding row p (selects, not
      // branches, so the register arrays stay in place)
      double mv = 0.0, rv = 0.0;
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        const bool hold = tr + kRows * r == p;
        mv = hold ? mr[r] : mv;
        rv = hold ? rr[r] : rv;
      }
      if (tr == p % kRows && j < n) {
        mrow[b][j] = mv / piv;
        rrow[b][j] = rv / piv;
      }
      __syncthreads();
      {
        const double mp = mrow[b][j], rp = rrow[b][j];
        const double mk = j > k ? 1.0 : 0.0;  // columns up to k of q(B) are done
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
          const bool isp = tr + kRows * r == p;
          const double l = ccol[b][tr + kRows * r];
          mr[r] = isp ? mp : mr[r] - (mk * l) * mp;
          rr[r] = isp ? rp : rr[r] - l * rp;
        }
      }
    }
    // row i holds row pstep[i] of the solution
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int i = tr + kRows * r;
      if (i < n && j < n) R[pstep[i] + static_cast<int64_t>(n) * j] = rr[r];
    }
    return;
  }
  // n > kSmallN: M = V - U into slot B (free), R = V + U in slot Q0
  double* M = slot(ws, nn, mat, W_B);
  for (int64_t e = t; e < nn; e += kT) {
    M[e] = V[e] - U[e];
    R[e] = V[e] + U[e];
  }
  __syncthreads();
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

// Squarings past the kSquareLaunches launches (s larger than that), one
// workgroup per matrix, then the copy of R^(2^s) to E.
__global__ __launch_bounds__(kT) void expm_finish(double* __restrict__ ws, int n,
                                                  const int* __restrict__ svec,
                                                  double* __restrict__ Eout) {
  __shared__ __attribute__((aligned(16))) double smem[kTile * (kKc + 1) + kKc * (kTile + 1)];
  auto As = reinterpret_cast<double(*)[kKc + 1]>(smem);
  auto Bs = reinterpret_cast<double(*)[kTile + 1]>(smem + kTile * (kKc + 1));
  const int64_t nn = static_cast<int64_t>(n) * n;
  const int mat = blockIdx.x;
  const int s = svec[mat];
  const int done = s < kSquareLaunches ? s : kSquareLaunches;
  double* cur = slot(ws, nn, mat, (done & 1) ? W_Q1 : W_Q0);
  double* nxt = slot(ws, nn, mat, (done & 1) ? W_Q0 : W_Q1);
  for (int it = done; it < s; ++it) {
    block_gemm(cur, cur, nxt, n, As, Bs);
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  double* E = Eout + mat * nn;
  for (int64_t e = threadIdx.x; e < nn; e += kT) E[e] = cur[e];
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
  // kSlots n^2 doubles per matrix, then one int (the scaling exponent) per matrix
  const size_t mats = static_cast<size_t>(kSlots * n * n * count) * sizeof(double);
  return mats + ((static_cast<size_t>(count) * sizeof(int) + 255) & ~static_cast<size_t>(255));
}

int kp_expm_f64(const double* A, int64_t n, int64_t count, double tau, double* E, void* ws,
                size_t ws_bytes, hipStream_t stream) {
  if (n < 0 || count < 0) return KP_ERR_SHAPE;
  if (n > kMaxN) return KP_ERR_SHAPE;
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
  double* W = static_cast<double*>(ws);
  int* svec = reinterpret_cast<int*>(static_cast<char*>(ws) +
                                     static_cast<size_t>(kSlots * n * n * count) * sizeof(double));
  const int ni = static_cast<int>(n), ci = static_cast<int>(count);
  const PadeCoef pc = pade13();
  const double* c = pc.c;
  hipLaunchKernelGGL(expm_scale, dim3(static_cast<unsigned>(count)), dim3(kScaleThreads), 0,
                     stream, A, ni, tau, W, svec);
  const int tps = (ni + kGT - 1) / kGT;
  auto gemm = [&](const GemmJobs& jobs) {
    const unsigned grid = static_cast<unsigned>(tps * tps * count * jobs.njobs);
    hipLaunchKernelGGL(expm_gemm, dim3(grid), dim3(kGThreads), 0, stream, W, ni, ci, jobs, svec);
  };
  auto job = [](int a_, std::initializer_list<std::pair<int, double>> b,
                std::initializer_list<std::pair<int, double>> e_, double diag, int c_, int sq) {
    GemmJob j{};
    j.a = a_;
    for (const auto& x : b) {
      j.b[j.nb] = x.first;
      j.beta[j.nb] = x.second;
      ++j.nb;
    }
    for (const auto& x : e_) {
      j.e[j.ne] = x.first;
      j.eps[j.ne] = x.second;
      ++j.ne;
    }
    j.diag = diag;
    j.c = c_;
    j.square = sq;
    return j;
  };
  auto one = [](const GemmJob& j) {
    GemmJobs js{};
    js.job[0] = j;
    js.njobs = 1;
    return js;
  };
  // B^2, B^4, B^6
  gemm(one(job(W_B, {{W_B, 1.0}}, {}, 0.0, W_B2, -1)));
  gemm(one(job(W_B2, {{W_B2, 1.0}}, {}, 0.0, W_B4, -1)));
  gemm(one(job(W_B4, {{W_B2, 1.0}}, {}, 0.0, W_B6, -1)));
  // odd part, inner factor: T = B6 (c13 B6 + c11 B4 + c9 B2) + c7 B6 + c5 B4 + c3 B2 + c1 I
  // (T in slot Q1, free until the squarings)
  gemm(one(job(W_B6, {{W_B6, c[13]}, {W_B4, c[11]}, {W_B2, c[9]}},
               {{W_B6, c[7]}, {W_B4, c[5]}, {W_B2, c[3]}}, c[1], W_Q1, -1)));
  // U = B T and V = B6 (c12 B6 + c10 B4 + c8 B2) + c6 B6 + c4 B4 + c2 B2 + c0 I
  GemmJobs uv{};
  uv.job[0] = job(W_B, {{W_Q1, 1.0}}, {}, 0.0, W_U, -1);
  uv.job[1] = job(W_B6, {{W_B6, c[12]}, {W_B4, c[10]}, {W_B2, c[8]}},
                  {{W_B6, c[6]}, {W_B4, c[4]}, {W_B2, c[2]}}, c[0], W_V, -1);
  uv.njobs = 2;
  gemm(uv);
  // q(B) R = p(B), R into slot Q0
  hipLaunchKernelGGL(expm_solve, dim3(static_cast<unsigned>(count)), dim3(kT), 0, stream, W, ni);
  // squarings: R <- R^2, Q0 and Q1 alternating; matrices with s <= it skip
  for (int it = 0; it < kSquareLaunches; ++it) {
    const int src = (it & 1) ? W_Q1 : W_Q0, dst = (it & 1) ? W_Q0 : W_Q1;
    gemm(one(job(src, {{src, 1.0}}, {}, 0.0, dst, it)));
  }
  hipLaunchKernelGGL(expm_finish, dim3(static_cast<unsigned>(count)), dim3(kT), 0, stream, W, ni,
                     svec, E);
  return hip_status(hipGetLastError());
}

}  // extern "C"
