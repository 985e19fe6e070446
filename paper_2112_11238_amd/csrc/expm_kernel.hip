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
//   expm_gemm     the products, spread over 16 x 16 output tiles of every
//                 matrix (k split over four waves) on the FP64 matrix
//                 cores: B^2, B^4, B^6, then the odd and even parts with
//                 their linear combinations folded into the operand loads
//                 and the epilogue;
//   expm_solve    one workgroup per matrix: q(B) R = p(B) by Gauss-Jordan
//                 elimination with partial pivoting, q(B) and R in
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

constexpr int kMaxN = 256;
constexpr int kGT = 16;          // output tile edge of expm_gemm
constexpr int kGWaves = 4;       // waves of an expm_gemm workgroup, splitting k
constexpr int kGThreads = 64 * kGWaves;
constexpr int kGSteps = kMaxN / 4 / kGWaves;  // k steps of 4 per wave, at most (n = 256)
constexpr int kSquareLaunches = 8;
constexpr int kScaleThreads = 1024;

__device__ __forceinline__ double* slot(double* ws, int64_t nn, int mat, int k) {
  return ws + (static_cast<int64_t>(mat) * kSlots + k) * nn;
}

// B = tau A 2^-s with s from the 1-norm of tau A (largest absolute column
// sum); one workgroup per matrix: wave w sums columns w, w + 16, ... (lane l
// rows l, l + 64, ...; all loads in flight together), a cross-lane sum per
// column, then the largest over the waves through LDS. NMAX: a multiple of
// 64, at least n.
template <int NMAX>
__global__ __launch_bounds__(kScaleThreads) void expm_scale(const double* __restrict__ Ain, int n,
                                                            double tau, double* __restrict__ ws,
                                                            int* __restrict__ svec) {
  constexpr int kWaves = kScaleThreads / 64;
  __shared__ double wmax[kWaves];
  __shared__ int s_sh;
  const int64_t nn = static_cast<int64_t>(n) * n;
  const int mat = blockIdx.x;
  const double* A = Ain + mat * nn;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // every load of the column sums is issued before the first is used
  constexpr int kCols = NMAX / kWaves, kRowsPer = NMAX / 64;
  double part[kCols];
#pragma unroll
  for (int c = 0; c < kCols; ++c) {
    const int j = w + kWaves * c;
    part[c] = 0.0;
#pragma unroll
    for (int q = 0; q < kRowsPer; ++q) {
      const int i = lane + 64 * q;
      // clamped, so that every load is unconditional and in bounds
      const double x = A[min(i, n - 1) + static_cast<int64_t>(n) * min(j, n - 1)];
      part[c] += j < n && i < n ? fabs(tau * x) : 0.0;
    }
  }
  double best = 0.0;
#pragma unroll
  for (int c = 0; c < kCols; ++c) {
    double v = part[c];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    best = fmax(best, v);
  }
  if (lane == 0) wmax[w] = best;
  __syncthreads();
  if (t == 0) {
    double norm1 = 0.0;
    for (int q = 0; q < kWaves; ++q) norm1 = fmax(norm1, wmax[q]);
    int s = 0;  // non-finite norms keep s = 0 and propagate as NaN/Inf
    if (isfinite(norm1) && norm1 > kTheta13) s = static_cast<int>(ceil(log2(norm1 / kTheta13)));
    if (s > 1100) s = 1100;
    s_sh = s;
    svec[mat] = s;
  }
  __syncthreads();
  const int s = s_sh;
  double* B = slot(ws, nn, mat, W_B);
#pragma unroll 8
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

// The products over 16 x 16 output tiles of every matrix (and job), the k
// range split over the four waves of a workgroup (wave w takes the k steps
// w, w + 4, ...): each lane loads its operand fragments straight from the
// workspace (the right factor's combination formed on load; every term is
// loaded and unused ones are masked, so all loads are in flight at once),
// the FP64 16x16x4 MFMA accumulates (lane l holds A(row l mod 16, k l / 16)
// and B(k l / 16, column l mod 16); item v of lane l is C(4v + l / 16,
// l mod 16)), and the four partial blocks are summed through LDS, wave w
// finishing item w (added terms and diagonal included). STEPS: k steps per
// wave, at least ceil(n / 16).
template <int STEPS>
__global__ __launch_bounds__(kGThreads) void expm_gemm(double* __restrict__ ws, int n, int count,
                                                       GemmJobs jobs, const int* __restrict__ svec) {
  __shared__ double part[kGWaves][4][64];
  const int tps = (n + kGT - 1) / kGT;
  const int tiles = tps * tps;
  const int bid = blockIdx.x;
  const int tile = bid % tiles;
  const int mat = (bid / tiles) % count;
  const GemmJob& jb = jobs.job[bid / (tiles * count)];
  const int64_t nn = static_cast<int64_t>(n) * n;
  const int i0 = (tile % tps) * kGT, j0 = (tile / tps) * kGT;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int ksteps = (n + 3) / 4;
  const double* A = slot(ws, nn, mat, jb.a);
  const double* B0 = slot(ws, nn, mat, jb.b[0]);
  const double* B1 = slot(ws, nn, mat, jb.nb > 1 ? jb.b[1] : jb.b[0]);
  const double* B2 = slot(ws, nn, mat, jb.nb > 2 ? jb.b[2] : jb.b[0]);
  const int ia = i0 + c, jbc = j0 + c;
  double av[STEPS], b0[STEPS], b1[STEPS], b2[STEPS];
#pragma unroll
  for (int u = 0; u < STEPS; ++u) {
    const int k = 4 * (w + kGWaves * u) + g;
    const bool kin = k < n;
    av[u] = kin && ia < n ? A[ia + static_cast<int64_t>(n) * k] : 0.0;
    const int64_t o = k + static_cast<int64_t>(n) * jbc;
    const bool bin = kin && jbc < n;
    b0[u] = bin ? B0[o] : 0.0;
    b1[u] = bin ? B1[o] : 0.0;
    b2[u] = bin ? B2[o] : 0.0;
  }
  // the element this wave finishes: item w of the block, row 4 w + g, column c
  const int io = i0 + 4 * w + g;
  const bool out = io < n && jbc < n;
  const int64_t oo = io + static_cast<int64_t>(n) * jbc;
  double ev[3];
#pragma unroll
  for (int q = 0; q < 3; ++q)
    ev[q] = out && q < jb.ne ? slot(ws, nn, mat, jb.e[q])[oo] : 0.0;
  if (jb.square >= 0 && jb.square >= svec[mat]) return;  // uniform: this matrix is done
  const double be0 = jb.beta[0];
  const double be1 = jb.nb > 1 ? jb.beta[1] : 0.0, be2 = jb.nb > 2 ? jb.beta[2] : 0.0;
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < STEPS; ++u) {
    if (w + kGWaves * u < ksteps) {  // uniform per wave
      double bv = be0 * b0[u];
      bv = jb.nb > 1 ? fma(be1, b1[u], bv) : bv;
      bv = jb.nb > 2 ? fma(be2, b2[u], bv) : bv;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) part[w][v][lane] = acc[v];
  __syncthreads();
  double r = (part[0][w][lane] + part[1][w][lane]) + (part[2][w][lane] + part[3][w][lane]);
  if (out) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
      if (q < jb.ne) r = fma(jb.eps[q], ev[q], r);
    if (io == jbc) r += jb.diag;
    slot(ws, nn, mat, jb.c)[oo] = r;
  }
}

// Cross-lane moves for the pivot search: a DPP move of a 64-bit value
// (CTRL: a quad permutation, a row mirror or a row broadcast; lanes in rows
// outside ROWS keep their own value) and a lane read.
template <int CTRL, int ROWS>
__device__ __forceinline__ long long dpp64(long long v) {
  const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(v), static_cast<int>(v), CTRL, ROWS,
                                             0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(v >> 32), static_cast<int>(v >> 32),
                                             CTRL, ROWS, 0xF, false);
  return (static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ void key_max(long long& key) {
  const long long o = dpp64<CTRL, ROWS>(key);
  key = o > key ? o : key;
}

constexpr int kPanel = 4;  // columns per panel: the k of one FP64 16x16x4 MFMA
constexpr int kPanStride = kSmallN + 4;  // staged panel column stride: no bank conflicts

// A wave's column block of [q(B) | p(B)], 128 rows, as two halves of 64
// rows: item 4 rb + v of half h, lane (g, cc) = (l / 16, l mod 16), is row
// 64 h + 16 rb + 4 v + g, column cc (the MFMA result layout). Vectors, so
// that a uniform index is a relative register move.
typedef double Half __attribute__((ext_vector_type(16)));

// Stages columns k1 .. k1 + 3 of q(B), held by the calling wave, into pan.
__device__ __forceinline__ void stage_panel(Half X0, Half X1, int k1, int cc, int g,
                                            double (*pan)[kPanStride]) {
  const int c = cc - (k1 & 15);
  if (c >= 0 && c < kPanel) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      pan[c][16 * (e >> 2) + 4 * (e & 3) + g] = X0[e];
      pan[c][64 + 16 * (e >> 2) + 4 * (e & 3) + g] = X1[e];
    }
  }
}

// Factors one panel of q(B), columns k0 .. k0 + 3 as staged in pan (row i
// of column c at pan[c][i]), by one wave: lane l holds rows l and l + 64.
// Each of the panel's steps picks, among the rows not yet used as pivots,
// a row p of largest |entry| in its column and gives every other row i the
// multiplier q(B)(i, c) / q(B)(p, c), updating the panel's later columns.
// The search compares one 64-bit integer per row: |x| read as an integer
// (IEEE order for non-negative values; a NaN above everything finite) with
// its low 7 bits replaced by 127 - row, so the maximum is found with plain
// integer maxima across the wave, and candidates within 2^-45 of each
// other go to the smaller row. Publishes the multipliers (Lb[s][i], zero in
// row p_s), the pivot rows (Pb[s]; 0 for steps past n) and
// Tb[s][q] = L(p_s, q), q < s, and records each pivot row's step and pivot.
__device__ void factor_panel(int k0, int n, const double (*pan)[kPanStride],
                             double (*Lb)[kSmallN], int* Pb, double (*Tb)[kPanel],
                             unsigned char* used, int* pstep, double* ppiv) {
  const int lane = threadIdx.x & 63;
  const int ns = min(kPanel, n - k0);
  double f[2][kPanel], L[2][kPanel];
  bool u[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = lane + 64 * h;
    u[h] = i >= n || used[i] != 0;
#pragma unroll
    for (int c = 0; c < kPanel; ++c) {
      f[h][c] = pan[c][i];
      L[h][c] = 0.0;
    }
  }
#pragma unroll
  for (int s = 0; s < kPanel; ++s) {
    if (s < ns) {  // uniform
      long long key = -1;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        const long long kk = u[h] ? -1LL
                                  : ((__double_as_longlong(f[h][s]) & 0x7fffffffffffff80LL) |
                                     (127 - i));
        key = kk > key ? kk : key;
      }
      key_max<0xB1, 0xF>(key);   // lanes xor 1
      key_max<0x4E, 0xF>(key);   // lanes xor 2
      key_max<0x141, 0xF>(key);  // the other quad of eight lanes
      key_max<0x140, 0xF>(key);  // the other eight of sixteen: every lane holds its row's maximum
      key_max<0x142, 0xA>(key);  // rows 1 and 3 take in rows 0 and 2
      key_max<0x143, 0xC>(key);  // rows 2 and 3 take in row 1: lane 63 holds the maximum
      const int p = 127 - (__builtin_amdgcn_readlane(static_cast<int>(key), 63) & 127);
      const int hp = p >> 6, lp = p & 63;
      double prow[kPanel];
#pragma unroll
      for (int c = s; c < kPanel; ++c) {
        // both halves read, then a scalar select: the register arrays stay
        // in registers
        const double r0 = readlane_f64(f[0][c], lp), r1 = readlane_f64(f[1][c], lp);
        prow[c] = hp ? r1 : r0;
      }
      double trow[kPanel];  // row p's earlier multipliers, uniform
#pragma unroll
      for (int q = 0; q < s; ++q) {
        const double r0 = readlane_f64(L[0][q], lp), r1 = readlane_f64(L[1][q], lp);
        trow[q] = hp ? r1 : r0;
      }
      // 1 / pivot: the reciprocal estimate and two Newton steps
      double inv = __builtin_amdgcn_rcp(prow[s]);
      inv = fma(inv, fma(-prow[s], inv, 1.0), inv);
      inv = fma(inv, fma(-prow[s], inv, 1.0), inv);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool isp = lane + 64 * h == p;
        const double l = isp ? 0.0 : f[h][s] * inv;
        L[h][s] = l;
#pragma unroll
        for (int c = s + 1; c < kPanel; ++c) f[h][c] = fma(-l, prow[c], f[h][c]);
        u[h] = u[h] || isp;
      }
      if (lane == 0) {
        pstep[p] = k0 + s;
        ppiv[p] = prow[s];
        Pb[s] = p;
#pragma unroll
        for (int q = 0; q < s; ++q) Tb[s][q] = trow[q];
      }
    } else if (lane == 0) {
      Pb[s] = 0;  // multipliers stay zero: the step changes nothing
#pragma unroll
      for (int q = 0; q < s; ++q) Tb[s][q] = 0.0;
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = lane + 64 * h;
    used[i] = u[h] ? 1 : 0;
#pragma unroll
    for (int c = 0; c < kPanel; ++c) Lb[c][i] = L[h][c];
  }
}

// q(B) R = p(B) with q(B) = V - U, p(B) = V + U, result R into slot Q0, for
// n <= kSmallN: blocked Gauss-Jordan elimination with partial pivoting, one
// workgroup per matrix, [q(B) | p(B)] (n x 2n, zero-padded to 128 x 256)
// held in registers as 16 x 16 MFMA result blocks (Half): wave w owns column block
// w mod 8 of q(B) (w < 8) or of p(B) (w >= 8), all eight row blocks. Rows are
// never moved or scaled in place. Per panel of four columns the wave owning
// them stages them in LDS and factors them (factor_panel); then every wave
// applies the panel to its columns x at once: with y_s the value of pivot
// row p_s when step s comes (y = T^-1 x[P], T unit lower triangular with
// T(s, s') = L(p_s, s'), published with the panel), x <- x - L y, one FP64
// 16x16x4 MFMA per block with
// A = -L and B = y. The wave owning the next panel runs at raised priority
// and factors it as soon as its own update is done; one barrier per panel,
// the multipliers double-buffered by panel parity. At the end row p_k
// divided by its pivot is row k of the solution.
__global__ __launch_bounds__(kT) void expm_solve_panel(double* __restrict__ ws, int n) {
  __shared__ double pan[kPanel][kPanStride];
  __shared__ double Ls[2][kPanel][kSmallN];
  __shared__ double Ts[2][kPanel][kPanel];
  __shared__ int Ps[2][kPanel];
  __shared__ double ppiv[kSmallN];
  __shared__ int pstep[kSmallN];
  __shared__ unsigned char used[kSmallN];
  const int64_t nn = static_cast<int64_t>(n) * n;
  const int mat = blockIdx.x;
  const double* U = slot(ws, nn, mat, W_U);
  const double* V = slot(ws, nn, mat, W_V);
  double* R = slot(ws, nn, mat, W_Q0);
  const int t = threadIdx.x, lane = t & 63;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int cb = w & 7;
  const bool isR = w >= 8;
  const int cc = lane & 15, g = lane >> 4;
  const int col = 16 * cb + cc;  // this lane's column of q(B) or p(B)
  Half X0, X1;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int i = 16 * (e >> 2) + 4 * (e & 3) + g;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t o = i + 64 * h + static_cast<int64_t>(n) * col;
      const bool in = i + 64 * h < n && col < n;
      const double x = in ? (isR ? V[o] + U[o] : V[o] - U[o]) : 0.0;
      if (h == 0)
        X0[e] = x;
      else
        X1[e] = x;
    }
  }
  for (int i = t; i < kSmallN; i += kT) used[i] = 0;
  __syncthreads();
  const int npan = (n + kPanel - 1) / kPanel;
  if (w == 0) {
    stage_panel(X0, X1, 0, cc, g, pan);
    factor_panel(0, n, pan, Ls[0], Ps[0], Ts[0], used, pstep, ppiv);
  }
  for (int P = 0; P < npan; ++P) {
    const int b = P & 1, k0 = kPanel * P;
    __syncthreads();  // panel P factored: the only barrier of the panel
    const bool next = P + 1 < npan && w == (P + 1) / 4;  // this wave holds panel P + 1
    if (next) __builtin_amdgcn_s_setprio(3);
    if (isR || 16 * cb + 15 >= k0 + kPanel) {  // columns past this panel (uniform)
      double x[kPanel];
      int ps[kPanel];
#pragma unroll
      for (int s = 0; s < kPanel; ++s) {
        ps[s] = __builtin_amdgcn_readfirstlane(Ps[b][s]);
        const int e = 4 * ((ps[s] >> 4) & 3) + ((ps[s] & 15) >> 2);
        const double xe = ps[s] >= 64 ? X1[e] : X0[e];
        x[s] = __shfl(xe, 16 * (ps[s] & 3) + cc);  // row p_s of this lane's column
      }
      double y[kPanel];
#pragma unroll
      for (int s = 0; s < kPanel; ++s) {
        double acc = x[s];
#pragma unroll
        for (int q = 0; q < s; ++q) acc = fma(-Ts[b][s][q], y[q], acc);
        y[s] = acc;
      }
      const double yb = g == 0 ? y[0] : g == 1 ? y[1] : g == 2 ? y[2] : y[3];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        d4_t c0 = {X0[4 * rb], X0[4 * rb + 1], X0[4 * rb + 2], X0[4 * rb + 3]};
        d4_t c1 = {X1[4 * rb], X1[4 * rb + 1], X1[4 * rb + 2], X1[4 * rb + 3]};
        c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(-Ls[b][g][16 * rb + cc], yb, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(-Ls[b][g][64 + 16 * rb + cc], yb, c1, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          X0[4 * rb + v] = c0[v];
          X1[4 * rb + v] = c1[v];
        }
      }
    }
    if (next) {
      stage_panel(X0, X1, k0 + kPanel, cc, g, pan);
      factor_panel(k0 + kPanel, n, pan, Ls[b ^ 1], Ps[b ^ 1], Ts[b ^ 1], used, pstep, ppiv);
      __builtin_amdgcn_s_setprio(0);
    }
  }
  __syncthreads();
  if (isR) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int i = 16 * (e >> 2) + 4 * (e & 3) + g;
      if (i < n && col < n) R[pstep[i] + static_cast<int64_t>(n) * col] = X0[e] / ppiv[i];
      if (i + 64 < n && col < n)
        R[pstep[i + 64] + static_cast<int64_t>(n) * col] = X1[e] / ppiv[i + 64];
    }
  }
}

// q(B) R = p(B) for kSmallN < n <= kMaxN: elimination with partial pivoting
// (row swaps) and back substitution in global memory, one workgroup per
// matrix.
__global__ __launch_bounds__(kT) void expm_solve(double* __restrict__ ws, int n) {
  __shared__ double red[kT];
  __shared__ int redi[kT];
  const int64_t nn = static_cast<int64_t>(n) * n;
  const int mat = blockIdx.x;
  const double* U = slot(ws, nn, mat, W_U);
  const double* V = slot(ws, nn, mat, W_V);
  double* R = slot(ws, nn, mat, W_Q0);
  const int t = threadIdx.x;
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
  if (ni <= kMaxN / 2)
    hipLaunchKernelGGL(expm_scale<kMaxN / 2>, dim3(static_cast<unsigned>(count)),
                       dim3(kScaleThreads), 0, stream, A, ni, tau, W, svec);
  else
    hipLaunchKernelGGL(expm_scale<kMaxN>, dim3(static_cast<unsigned>(count)), dim3(kScaleThreads),
                       0, stream, A, ni, tau, W, svec);
  const int tps = (ni + kGT - 1) / kGT;
  auto gemm = [&](const GemmJobs& jobs) {
    const unsigned grid = static_cast<unsigned>(tps * tps * count * jobs.njobs);
    if (ni <= 4 * kGWaves * kGSteps / 2)
      hipLaunchKernelGGL(expm_gemm<kGSteps / 2>, dim3(grid), dim3(kGThreads), 0, stream, W, ni, ci,
                         jobs, svec);
    else
      hipLaunchKernelGGL(expm_gemm<kGSteps>, dim3(grid), dim3(kGThreads), 0, stream, W, ni, ci,
                         jobs, svec);
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
  if (ni <= kSmallN)
    hipLaunchKernelGGL(expm_solve_panel, dim3(static_cast<unsigned>(count)), dim3(kT), 0, stream,
                       W, ni);
  else
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
