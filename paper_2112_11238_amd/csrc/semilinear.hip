// The semilinear diffusion-reaction experiment on the device, in FP64
// (Sec. 3.4, preconditioning of Kronecker-sum systems; Sec. 4.5):
//
//  * inverses of tridiagonal matrices (the ADI factors (I - tau A_mu)^{-1}),
//    one elimination per identity column;
//  * the preconditioned conjugate gradient method for
//    (M_d (+) ... (+) M_1) x = b, whose matrix action is the Kronecker-sum
//    action (d mu-mode products) and whose preconditioner action is a
//    Tucker operator with the factor inverses;
//  * backward-forward Euler steps of u_t = Laplacian(u) + 1/(1 + u^2) + Phi
//    with the source Phi that makes e^t prod_mu x_mu (1 - x_mu) the exact
//    solution, one PCG solve per step.
//
// The conjugate-gradient loop runs on the host and reads one scalar (the
// residual norm) back per iteration to decide whether to stop; all vector
// arithmetic and every reduction runs in the kernels below. Reductions are
// two-level and in a fixed order (per-block partial sums, then a fixed tree
// over the partials), so results do not depend on scheduling.
#include "kp.h"

#include <math.h>


#include "kp_common.h"
#include "kp_internal.h"

namespace kp {
namespace {

constexpr int kRB = 256;           // threads per block of the vector kernels
constexpr int kMaxParts = 1024;    // partial sums per reduction
constexpr int kTriT = 256;         // columns per workgroup of the inverse
constexpr int64_t kTriMaxN = 2048;

// ---- tridiagonal matrices -------------------------------------------------
// T_k given by diagonals lo, dg, up (n entries each, matrix k at k*n):
// T[i][i-1] = lo[i], T[i][i] = dg[i], T[i][i+1] = up[i]. The kernels work on
// P = shift I + scale T.

// E_k = P_k^{-1}, column-major. Thread j computes row j of P^{-1}, i.e. the
// solution y of P^T y = e_j (Gaussian elimination without pivoting, the
// Thomas algorithm), so at every step the threads of a wave touch consecutive
// addresses of E. The pivots and eliminated super-diagonal, shared by all
// columns, are computed once per workgroup into LDS. E's own column j is the
// scratch for the forward sweep of y.
__global__ __launch_bounds__(kTriT) void tridiag_inverse_kernel(
    const double* __restrict__ lo, const double* __restrict__ dg, const double* __restrict__ up,
    int n, double shift, double scale, double* __restrict__ E) {
  extern __shared__ double sh[];
  double* den = sh;          // pivots
  double* cp = sh + n;       // eliminated super-diagonal of P^T
  double* sub = sh + 2 * n;  // sub-diagonal of P^T: sub[i] = P[i-1][i]
  const int64_t k = blockIdx.y;
  lo += k * n;
  dg += k * n;
  up += k * n;
  E += k * static_cast<int64_t>(n) * n;
  if (threadIdx.x == 0) {
    for (int i = 0; i < n; ++i) {
      const double a = i > 0 ? scale * up[i - 1] : 0.0;
      const double b = shift + scale * dg[i];
      const double c = i < n - 1 ? scale * lo[i + 1] : 0.0;
      const double dn = i > 0 ? b - a * cp[i - 1] : b;
      sub[i] = a;
      den[i] = dn;
      cp[i] = c / dn;
    }
  }
  __syncthreads();
  const int j = blockIdx.x * kTriT + threadIdx.x;
  if (j >= n) return;
  // forward sweep: entries above j are zero
  double y = 1.0 / den[j];
  E[j + static_cast<int64_t>(j) * n] = y;
  for (int i = j + 1; i < n; ++i) {
    y = -sub[i] * y / den[i];
    E[j + static_cast<int64_t>(i) * n] = y;
  }
  // back substitution, in place
  for (int i = n - 2; i >= 0; --i) {
    const double di = i >= j ? E[j + static_cast<int64_t>(i) * n] : 0.0;
    y = di - cp[i] * y;
    E[j + static_cast<int64_t>(i) * n] = y;
  }
}

// M = shift I + scale T as a dense column-major n x n matrix.
__global__ __launch_bounds__(kRB) void tridiag_dense_kernel(
    const double* __restrict__ lo, const double* __restrict__ dg, const double* __restrict__ up,
    int n, double shift, double scale, double* __restrict__ M) {
  const int64_t nn = static_cast<int64_t>(n) * n;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kRB) + threadIdx.x; e < nn;
       e += static_cast<int64_t>(gridDim.x) * kRB) {
    const int i = static_cast<int>(e % n), j = static_cast<int>(e / n);
    double v = 0.0;
    if (i == j) v = shift + scale * dg[i];
    else if (i == j + 1) v = scale * lo[i];
    else if (j == i + 1) v = scale * up[i];
    M[e] = v;
  }
}

// ---- vector kernels of the conjugate-gradient loop -----------------------
// Block b of every vector kernel owns elements [b*chunk, min((b+1)*chunk, N));
// thread t visits b*chunk + t, + kRB, ... in order.

__device__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = kRB / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// the sum of `np` partials, the same bits in every block
__device__ double parts_sum(const double* __restrict__ part, int np, double* red) {
  double v = 0.0;
  for (int k = threadIdx.x; k < np; k += kRB) v += part[k];
  return block_sum(v, red);
}

struct Span {
  int64_t lo, hi;
};

__device__ Span my_span(int64_t N, int64_t chunk) {
  const int64_t lo = blockIdx.x * chunk;
  return {lo + threadIdx.x, lo + chunk < N ? lo + chunk : N};
}

// r = b - q; partials of <r, r> and <b, b>
__global__ __launch_bounds__(kRB) void residual_init_kernel(
    const double* __restrict__ b, const double* __restrict__ q, double* __restrict__ r,
    int64_t N, int64_t chunk, double* __restrict__ part_rr, double* __restrict__ part_bb) {
  __shared__ double red[kRB];
  const Span s = my_span(N, chunk);
  double rr = 0.0, bb = 0.0;
  for (int64_t i = s.lo; i < s.hi; i += kRB) {
    const double bi = b[i], ri = bi - q[i];
    r[i] = ri;
    rr += ri * ri;
    bb += bi * bi;
  }
  rr = block_sum(rr, red);
  bb = block_sum(bb, red);
  if (threadIdx.x == 0) {
    part_rr[blockIdx.x] = rr;
    part_bb[blockIdx.x] = bb;
  }
}

// partials of <x, y>
__global__ __launch_bounds__(kRB) void dot_kernel(const double* __restrict__ x,
                                                  const double* __restrict__ y, int64_t N,
                                                  int64_t chunk, double* __restrict__ part) {
  __shared__ double red[kRB];
  const Span s = my_span(N, chunk);
  double acc = 0.0;
  for (int64_t i = s.lo; i < s.hi; i += kRB) acc += x[i] * y[i];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// out = sum of the partials (one block)
__global__ __launch_bounds__(kRB) void finalize_kernel(const double* __restrict__ part, int np,
                                                       double* __restrict__ out) {
  __shared__ double red[kRB];
  const double v = parts_sum(part, np, red);
  if (threadIdx.x == 0) *out = v;
}

// Scalars kept on the device between kernels.
enum { kRho = 0, kRhoPrev = 1, kRR = 2, kBB = 3, kNumScalars = 8 };

// rho = <r, z> (from its partials); p = z on the first iteration, else
// p = z + (rho / rho_prev) p. Block 0 records rho.
__global__ __launch_bounds__(kRB) void update_p_kernel(
    const double* __restrict__ z, double* __restrict__ p, int64_t N, int64_t chunk,
    const double* __restrict__ part_rz, int np, double* __restrict__ sc, int first) {
  __shared__ double red[kRB];
  const double rho = parts_sum(part_rz, np, red);
  const Span s = my_span(N, chunk);
  if (first) {
    for (int64_t i = s.lo; i < s.hi; i += kRB) p[i] = z[i];
  } else {
    const double beta = rho / sc[kRhoPrev];
    for (int64_t i = s.lo; i < s.hi; i += kRB) p[i] = z[i] + beta * p[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[kRho] = rho;
}

// alpha = rho / <p, q> (from its partials); x += alpha p; r -= alpha q;
// partials of <r, r>. Block 0 moves rho to rho_prev.
__global__ __launch_bounds__(kRB) void update_xr_kernel(
    double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
    const double* __restrict__ q, int64_t N, int64_t chunk, const double* __restrict__ part_pq,
    int np, double* __restrict__ sc, double* __restrict__ part_rr) {
  __shared__ double red[kRB];
  const double pq = parts_sum(part_pq, np, red);
  const double rho = sc[kRho];
  const double alpha = rho / pq;
  const Span s = my_span(N, chunk);
  double rr = 0.0;
  for (int64_t i = s.lo; i < s.hi; i += kRB) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    rr += ri * ri;
  }
  rr = block_sum(rr, red);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = rr;
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[kRhoPrev] = rho;
}

// ---- the experiment's right-hand side -------------------------------------
struct GridArgs {
  int d;
  int64_t dims[KP_MAX_ORDER];
  double h[KP_MAX_ORDER];
};

// b = u + tau (1/(1 + u^2) + Phi(t, x)) with x_mu = (i_mu + 1) h_mu,
// q_mu = x_mu (1 - x_mu), u0 = prod q_mu, Laplacian(u0) = -2 sum_mu
// prod_{nu != mu} q_nu and Phi = e^t (u0 - Laplacian(u0)) - 1/(1 + e^{2t} u0^2).
__global__ __launch_bounds__(kRB) void semilinear_rhs_kernel(const double* __restrict__ u,
                                                             double* __restrict__ b, int64_t N,
                                                             GridArgs g, double t, double tau) {
  const double et = exp(t);
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kRB) + threadIdx.x; e < N;
       e += static_cast<int64_t>(gridDim.x) * kRB) {
    double q[KP_MAX_ORDER];
    int64_t rem = e;
    for (int k = 0; k < g.d; ++k) {
      const int64_t i = rem % g.dims[k];
      rem /= g.dims[k];
      const double x = static_cast<double>(i + 1) * g.h[k];
      q[k] = x * (1.0 - x);
    }
    double u0 = 1.0, lap = 0.0;
    for (int k = 0; k < g.d; ++k) {
      u0 *= q[k];
      double pr = 1.0;
      for (int j = 0; j < g.d; ++j)
        if (j != k) pr *= q[j];
      lap += pr;
    }
    lap *= -2.0;
    const double phi = et * (u0 - lap) - 1.0 / (1.0 + et * et * u0 * u0);
    const double ue = u[e];
    b[e] = ue + tau * (1.0 / (1.0 + ue * ue) + phi);
  }
}

// ---- host side -------------------------------------------------------------
int64_t tensor_numel(const kp_tensor& t) {
  int64_t s = 1;
  for (int k = 0; k < t.d; ++k) s *= t.dims[k];
  return s;
}

struct RedPlan {
  int np;
  int64_t chunk;
};

RedPlan red_plan(int64_t N) {
  int64_t np = (N + 1023) / 1024;
  if (np > kMaxParts) np = kMaxParts;
  if (np < 1) np = 1;
  int64_t chunk = (N + np - 1) / np;
  chunk = (chunk + kRB - 1) / kRB * kRB;
  np = (N + chunk - 1) / chunk;
  if (np < 1) np = 1;
  return {static_cast<int>(np), chunk};
}

// Workspace of the solver: r, z, p, q, the preconditioner's chain workspace,
// three partial-sum arrays and the scalars.
struct PcgLayout {
  size_t r, z, p, q, tws, tws_bytes, pa, pb, pc, sc, total;
};

PcgLayout pcg_layout(const kp_tensor& X, const kp_matrix* const* P) {
  PcgLayout l;
  const size_t vb = align_up(static_cast<size_t>(tensor_numel(X)) * sizeof(double));
  size_t off = 0;
  l.r = off; off += vb;
  l.z = off; off += vb;
  l.p = off; off += vb;
  l.q = off; off += vb;
  // the preconditioner's factors are square, so each of its intermediates
  // has the size of X: two ping-pong buffers of that size cover any chain
  l.tws = off;
  l.tws_bytes = P ? 2 * vb : 0;
  off += l.tws_bytes;
  l.pa = off; off += align_up(kMaxParts * sizeof(double));
  l.pb = off; off += align_up(kMaxParts * sizeof(double));
  l.pc = off; off += align_up(kMaxParts * sizeof(double));
  l.sc = off; off += align_up(kNumScalars * sizeof(double));
  l.total = off;
  return l;
}

int check_square_f64(const kp_matrix* A, int64_t n) {
  const int st = check_matrix(A, KP_F64);
  if (st) return st;
  if (A->rows != n || A->cols != n) return KP_ERR_SHAPE;
  return KP_OK;
}

int check_pcg_args(const kp_tensor* B, const kp_matrix* const* M, const kp_matrix* const* P,
                   const kp_tensor* X, double tol, int maxit) {
  int st = check_tensor(B, true);
  if (st) return st;
  if (!X || !M) return KP_ERR_NULL;
  st = check_tensor(X, true);
  if (st) return st;
  if (B->dtype != KP_F64 || X->dtype != KP_F64) return KP_ERR_DTYPE;
  if (X->d != B->d) return KP_ERR_SHAPE;
  for (int k = 0; k < B->d; ++k)
    if (X->dims[k] != B->dims[k]) return KP_ERR_SHAPE;
  for (int k = 0; k < B->d; ++k) {
    if (!M[k]) return KP_ERR_NULL;
    st = check_square_f64(M[k], B->dims[k]);
    if (st) return st;
    if (P && P[k]) {
      st = check_square_f64(P[k], B->dims[k]);
      if (st) return st;
    }
  }
  if (!(tol >= 0.0) || !isfinite(tol) || maxit < 0) return KP_ERR_VALUE;
  return KP_OK;
}

// The solver proper, on validated arguments; `w` is a workspace laid out by
// pcg_layout.
int pcg_run(const kp_tensor& B, const kp_matrix* const* M, const kp_matrix* const* P,
            kp_tensor& X, double tol, int maxit, char* w, int* iters, double* relres,
            hipStream_t stream) {
  const PcgLayout l = pcg_layout(X, P);
  const int64_t N = tensor_numel(X);
  int it = 0;
  double res = 0.0;
  if (N == 0) {
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return KP_OK;
  }
  const RedPlan rp = red_plan(N);
  double* r = reinterpret_cast<double*>(w + l.r);
  double* z = P ? reinterpret_cast<double*>(w + l.z) : r;
  double* p = reinterpret_cast<double*>(w + l.p);
  double* q = reinterpret_cast<double*>(w + l.q);
  double* pa = reinterpret_cast<double*>(w + l.pa);
  double* pb = reinterpret_cast<double*>(w + l.pb);
  double* pc = reinterpret_cast<double*>(w + l.pc);
  double* sc = reinterpret_cast<double*>(w + l.sc);
  double* x = static_cast<double*>(X.data);
  const double* b = static_cast<const double*>(B.data);
  kp_tensor tr = X, tz = X, tp = X, tq = X;
  tr.data = r;
  tz.data = z;
  tp.data = p;
  tq.data = q;
  const dim3 grid(rp.np), block(kRB);

  // r = b - M x0
  int st = kp_kronsum(&X, M, &tq, KP_PREC_NATIVE, stream);
  if (st) return st;
  hipLaunchKernelGGL(residual_init_kernel, grid, block, 0, stream, b, q, r, N, rp.chunk, pa, pb);
  hipLaunchKernelGGL(finalize_kernel, dim3(1), block, 0, stream, pa, rp.np, sc + kRR);
  hipLaunchKernelGGL(finalize_kernel, dim3(1), block, 0, stream, pb, rp.np, sc + kBB);
  st = hip_status(hipGetLastError());
  if (st) return st;
  double host[2];
  st = hip_status(hipMemcpyAsync(host, sc + kRR, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
  if (st) return st;
  st = hip_status(hipStreamSynchronize(stream));
  if (st) return st;
  const double nb = sqrt(host[1]);
  if (nb == 0.0) {
    // b = 0: the solution is x = 0
    st = hip_status(hipMemsetAsync(x, 0, static_cast<size_t>(N) * sizeof(double), stream));
    if (st) return st;
    st = hip_status(hipStreamSynchronize(stream));
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return st;
  }
  res = sqrt(host[0]) / nb;
  while (res > tol && it < maxit) {
    if (P) {
      st = kp_tucker(&tr, P, &tz, KP_PREC_NATIVE, w + l.tws, l.tws_bytes, nullptr, 0, stream);
      if (st) return st;
    }
    hipLaunchKernelGGL(dot_kernel, grid, block, 0, stream, r, z, N, rp.chunk, pa);
    hipLaunchKernelGGL(update_p_kernel, grid, block, 0, stream, z, p, N, rp.chunk, pa, rp.np, sc,
                       it == 0 ? 1 : 0);
    st = hip_status(hipGetLastError());
    if (st) return st;
    st = kp_kronsum(&tp, M, &tq, KP_PREC_NATIVE, stream);
    if (st) return st;
    hipLaunchKernelGGL(dot_kernel, grid, block, 0, stream, p, q, N, rp.chunk, pb);
    hipLaunchKernelGGL(update_xr_kernel, grid, block, 0, stream, x, r, p, q, N, rp.chunk, pb,
                       rp.np, sc, pc);
    hipLaunchKernelGGL(finalize_kernel, dim3(1), block, 0, stream, pc, rp.np, sc + kRR);
    st = hip_status(hipGetLastError());
    if (st) return st;
    st = hip_status(hipMemcpyAsync(host, sc + kRR, sizeof(double), hipMemcpyDeviceToHost, stream));
    if (st) return st;
    st = hip_status(hipStreamSynchronize(stream));
    if (st) return st;
    ++it;
    res = sqrt(host[0]) / nb;
  }
  if (iters) *iters = it;
  if (relres) *relres = res;
  return KP_OK;
}

// Workspace of the time stepper: M_mu and P_mu^{-1} (dense), b, the solver's.
struct ImexLayout {
  size_t mats[KP_MAX_ORDER], pinv[KP_MAX_ORDER], b, pcg, total;
};

ImexLayout imex_layout(int d, const int64_t* dims, const PcgLayout& pl) {
  ImexLayout l;
  size_t off = 0;
  int64_t N = 1;
  for (int k = 0; k < d; ++k) {
    l.mats[k] = off;
    off += align_up(static_cast<size_t>(dims[k] * dims[k]) * sizeof(double));
    N *= dims[k];
  }
  for (int k = 0; k < d; ++k) {
    l.pinv[k] = off;
    off += align_up(static_cast<size_t>(dims[k] * dims[k]) * sizeof(double));
  }
  l.b = off;
  off += align_up(static_cast<size_t>(N) * sizeof(double));
  l.pcg = off;
  off += pl.total;
  l.total = off;
  return l;
}

kp_matrix dense_desc(int64_t n, void* data) {
  kp_matrix m;
  m.rows = n;
  m.cols = n;
  m.rs = 1;   // column-major
  m.cs = n;
  m.dtype = KP_F64;
  m.pad_ = 0;
  m.data = data;
  return m;
}

bool valid_dims(int d, const int64_t* dims) {
  if (!dims || d < 1 || d > KP_MAX_ORDER) return false;
  for (int k = 0; k < d; ++k)
    if (dims[k] < 1 || dims[k] > kTriMaxN) return false;
  return true;
}

}  // namespace
}  // namespace kp

using namespace kp;

extern "C" {

int kp_tridiag_inverse_f64(const double* lower, const double* diag, const double* upper,
                           int64_t n, int64_t count, double shift, double scale, double* E,
                           hipStream_t stream) {
  if (n < 0 || count < 0 || n > kTriMaxN || count > 65535) return KP_ERR_SHAPE;
  if (n == 0 || count == 0) return KP_OK;
  if (!lower || !diag || !upper || !E) return KP_ERR_NULL;
  if (!isfinite(shift) || !isfinite(scale)) return KP_ERR_VALUE;
  const size_t eb = static_cast<size_t>(n * n * count) * sizeof(double);
  const size_t db = static_cast<size_t>(n * count) * sizeof(double);
  if (overlaps(E, eb, lower, db) || overlaps(E, eb, diag, db) || overlaps(E, eb, upper, db))
    return KP_ERR_ALIAS;
  const dim3 grid(static_cast<unsigned>((n + kTriT - 1) / kTriT), static_cast<unsigned>(count));
  hipLaunchKernelGGL(tridiag_inverse_kernel, grid, dim3(kTriT), 3 * n * sizeof(double), stream,
                     lower, diag, upper, static_cast<int>(n), shift, scale, E);
  return hip_status(hipGetLastError());
}

size_t kp_pcg_workspace(const kp_tensor* X, const kp_matrix* const* P) {
  if (check_tensor(X, false) || X->dtype != KP_F64) return 0;
  return pcg_layout(*X, P).total;
}

int kp_pcg_kronsum(const kp_tensor* B, const kp_matrix* const* M, const kp_matrix* const* P,
                   kp_tensor* X, double tol, int maxit, void* ws, size_t ws_bytes, int* iters,
                   double* relres, hipStream_t stream) {
  int st = check_pcg_args(B, M, P, X, tol, maxit);
  if (st) return st;
  const PcgLayout l = pcg_layout(*X, P);
  if (!ws || ws_bytes < l.total) return KP_ERR_WORKSPACE;
  const size_t vb = static_cast<size_t>(tensor_numel(*X)) * sizeof(double);
  if (overlaps(X->data, vb, B->data, vb) || overlaps(X->data, vb, ws, l.total) ||
      overlaps(B->data, vb, ws, l.total))
    return KP_ERR_ALIAS;
  for (int k = 0; k < X->d; ++k) {
    const size_t mb = matrix_span_bytes(*M[k]);
    if (overlaps(X->data, vb, M[k]->data, mb) || overlaps(ws, l.total, M[k]->data, mb))
      return KP_ERR_ALIAS;
    if (P && P[k]) {
      const size_t pb = matrix_span_bytes(*P[k]);
      if (overlaps(X->data, vb, P[k]->data, pb) || overlaps(ws, l.total, P[k]->data, pb))
        return KP_ERR_ALIAS;
    }
  }
  return pcg_run(*B, M, P, *X, tol, maxit, static_cast<char*>(ws), iters, relres, stream);
}

size_t kp_semilinear_workspace(int d, const int64_t* dims) {
  if (!valid_dims(d, dims)) return 0;
  kp_tensor X;
  X.d = d;
  X.dtype = KP_F64;
  for (int k = 0; k < d; ++k) X.dims[k] = dims[k];
  X.data = nullptr;
  kp_matrix pm[KP_MAX_ORDER];
  const kp_matrix* pp[KP_MAX_ORDER];
  for (int k = 0; k < d; ++k) {
    pm[k] = dense_desc(dims[k], nullptr);
    pp[k] = &pm[k];
  }
  const PcgLayout pl = pcg_layout(X, pp);
  return imex_layout(d, dims, pl).total;
}

int kp_semilinear_imex_f64(kp_tensor* U, const double* const* lower, const double* const* diag,
                           const double* const* upper, const double* h, double t0, double tau,
                           int steps, double tol, int maxit, int precondition, void* ws,
                           size_t ws_bytes, int* iters, hipStream_t stream) {
  int st = check_tensor(U, true);
  if (st) return st;
  if (U->dtype != KP_F64) return KP_ERR_DTYPE;
  if (!valid_dims(U->d, U->dims)) return KP_ERR_SHAPE;
  if (!lower || !diag || !upper || !h) return KP_ERR_NULL;
  const int d = U->d;
  for (int k = 0; k < d; ++k) {
    if (!lower[k] || !diag[k] || !upper[k]) return KP_ERR_NULL;
    if (!(h[k] > 0.0) || !isfinite(h[k])) return KP_ERR_VALUE;
  }
  if (!isfinite(t0) || !isfinite(tau) || steps < 0 || !(tol >= 0.0) || !isfinite(tol) ||
      maxit < 0)
    return KP_ERR_VALUE;
  const size_t need = kp_semilinear_workspace(d, U->dims);
  if (!ws || ws_bytes < need) return KP_ERR_WORKSPACE;
  const int64_t N = tensor_numel(*U);
  const size_t vb = static_cast<size_t>(N) * sizeof(double);
  if (overlaps(U->data, vb, ws, need)) return KP_ERR_ALIAS;
  for (int k = 0; k < d; ++k) {
    const size_t db = static_cast<size_t>(U->dims[k]) * sizeof(double);
    if (overlaps(U->data, vb, lower[k], db) || overlaps(U->data, vb, diag[k], db) ||
        overlaps(U->data, vb, upper[k], db) || overlaps(ws, need, lower[k], db) ||
        overlaps(ws, need, diag[k], db) || overlaps(ws, need, upper[k], db))
      return KP_ERR_ALIAS;
  }

  char* w = static_cast<char*>(ws);
  kp_matrix mm[KP_MAX_ORDER], pm[KP_MAX_ORDER];
  const kp_matrix* mp[KP_MAX_ORDER];
  const kp_matrix* pp[KP_MAX_ORDER];
  for (int k = 0; k < d; ++k) {
    mm[k] = dense_desc(U->dims[k], nullptr);
    pm[k] = dense_desc(U->dims[k], nullptr);
    mp[k] = &mm[k];
    pp[k] = &pm[k];
  }
  const PcgLayout pl = pcg_layout(*U, pp);
  const ImexLayout il = imex_layout(d, U->dims, pl);
  // factors: M_mu = I/d - tau A_mu (the Kronecker-sum terms of the step
  // matrix) and (I - tau A_mu)^{-1} (the ADI preconditioner factors)
  for (int k = 0; k < d; ++k) {
    const int64_t n = U->dims[k];
    mm[k].data = w + il.mats[k];
    pm[k].data = w + il.pinv[k];
    const int64_t nn = n * n;
    const unsigned gb = static_cast<unsigned>((nn + kRB - 1) / kRB < 1024 ? (nn + kRB - 1) / kRB : 1024);
    hipLaunchKernelGGL(tridiag_dense_kernel, dim3(gb), dim3(kRB), 0, stream, lower[k], diag[k],
                       upper[k], static_cast<int>(n), 1.0 / d, -tau,
                       static_cast<double*>(mm[k].data));
    st = hip_status(hipGetLastError());
    if (st) return st;
    if (precondition) {
      st = kp_tridiag_inverse_f64(lower[k], diag[k], upper[k], n, 1, 1.0, -tau,
                                  static_cast<double*>(pm[k].data), stream);
      if (st) return st;
    }
  }
  GridArgs g;
  g.d = d;
  for (int k = 0; k < d; ++k) {
    g.dims[k] = U->dims[k];
    g.h[k] = h[k];
  }
  kp_tensor tb = *U;
  tb.data = w + il.b;
  double* b = static_cast<double*>(tb.data);
  const int64_t blocks = (N + kRB - 1) / kRB;
  const unsigned gb = static_cast<unsigned>(blocks < 4096 ? blocks : 4096);
  for (int s = 0; s < steps; ++s) {
    hipLaunchKernelGGL(semilinear_rhs_kernel, dim3(gb), dim3(kRB), 0, stream,
                       static_cast<const double*>(U->data), b, N, g, t0 + s * tau, tau);
    st = hip_status(hipGetLastError());
    if (st) return st;
    int it = 0;
    st = pcg_run(tb, mp, precondition ? pp : nullptr, *U, tol, maxit, w + il.pcg, &it, nullptr,
                 stream);
    if (st) return st;
    if (iters) iters[s] = it;
  }
  return KP_OK;
}

}  // extern "C"
