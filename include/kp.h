/*
 * kp.h -- C-ABI of the MI355X (gfx950) mu-mode product / Tucker operator library.
 *
 * Operations (Caliari, Cassini, Zivcovich, "A mu-mode BLAS approach for
 * multidimensional tensor-structured problems"):
 *   - the mu-mode product   S = T x_mu L          (Sec. 2, Definition of the
 *     mu-mode product; S^(mu) = L T^(mu));
 *   - the Tucker operator   S = T x_1 L_1 ... x_d L_d  (Sec. 2, Definition of
 *     the Tucker operator);
 *   - its gradient (not in the paper; derived from the Lemma relating the
 *     Tucker operator to L_d (x) ... (x) L_1 and the Kronecker transpose rule,
 *     Appendix A property 5);
 *   - the action of a Kronecker sum (Sec. 2);
 *   - the complex Tucker operator and its conjugate-transpose form (Sec. 2
 *     over C; Sec. 3, spectral transforms);
 *   - the exponential of a small matrix, the 1-D factor of the exponential of
 *     a Kronecker sum (Sec. 3.3);
 *   - tridiagonal inverses, preconditioned conjugate gradients on a
 *     Kronecker-sum system with a Kronecker-product (ADI-type) preconditioner
 *     and the backward-forward Euler steps of the semilinear experiment
 *     (Sec. 3.4, Sec. 4.5).
 *
 * Memory layout
 *   A tensor is column-major: mode 1 is contiguous, exactly the linear order
 *   of vec (Appendix A). Element (j_1..j_d) (0-based here) sits at offset
 *   j_1 + m_1 (j_2 + m_2 (j_3 + ...)). A row-major array of shape
 *   (m_1..m_d) is the same bytes as a column-major tensor of dims
 *   (m_d..m_1); callers with row-major data reverse the dims and the factor
 *   list (the Python binding does this).
 *   A matrix L (rows x cols) is strided: L(i,j) at data[i*rs + j*cs]. Its
 *   transpose is the same data with rows/cols and rs/cs swapped (the backward
 *   pass uses that, without a copy).
 *
 * Ownership and synchronisation
 *   The caller owns every buffer (device memory for tensors, factors, outputs
 *   and workspaces). The library never allocates device memory and never
 *   frees caller memory. Every call except the two iterative solvers
 *   (kp_pcg_kronsum, kp_semilinear_imex_f64, which wait for `stream` once
 *   per iteration) only enqueues kernels on `stream` and returns; those
 *   calls may be captured into a HIP graph.
 *   Outputs must not overlap inputs (KP_ERR_ALIAS).
 *
 * Errors
 *   Every entry point returns KP_OK (0) or a negative kp_status. Argument
 *   errors are detected on the host before anything is enqueued; nothing is
 *   launched then. KP_ERR_HIP reports a failed launch; kp_last_hip_error()
 *   returns the hipError_t behind it. Faults inside kernels surface at the
 *   caller's next synchronisation, as with any HIP call. NaN and Inf propagate
 *   by IEEE rules; they are not checked.
 */
#ifndef KP_H_
#define KP_H_

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KP_MAX_ORDER 8
#define KP_VERSION 100 /* 1.0.0 */

typedef enum {
  KP_OK = 0,
  KP_ERR_NULL = -1,      /* a required pointer is NULL */
  KP_ERR_ORDER = -2,     /* d < 1 or d > KP_MAX_ORDER */
  KP_ERR_MODE = -3,      /* mu outside 1..d */
  KP_ERR_SHAPE = -4,     /* sizes do not match (L cols vs m_mu, output dims) */
  KP_ERR_DTYPE = -5,     /* dtype / precision combination not supported */
  KP_ERR_ALIAS = -6,     /* an output overlaps an input */
  KP_ERR_WORKSPACE = -7, /* workspace missing or smaller than required */
  KP_ERR_HIP = -8,       /* a HIP launch failed; see kp_last_hip_error() */
  KP_ERR_VALUE = -9,     /* a scalar argument is out of range */
  KP_ERR_SCRATCH = -10   /* kp_tucker_noalloc: the intermediates need more than
                            KP_NOALLOC_SCRATCH_BYTES */
} kp_status;

typedef enum { KP_F64 = 0, KP_F32 = 1 } kp_dtype;

/* Arithmetic used by the contractions.
 *   KP_PREC_NATIVE : FP64 MFMA for KP_F64 data, FP32 MFMA for KP_F32 data.
 *   KP_PREC_BF16X3 : KP_F32 data only. Each operand x is split by
 *                    round-to-nearest-even into x1 = bf16(x), x2 = bf16(x-x1);
 *                    a*b is formed as a1 b1 + a1 b2 + a2 b1 on BF16 MFMA with
 *                    FP32 accumulation (about 16 significant bits).
 *   KP_PREC_BF16X6 : KP_F32 data only. Three-way split (x3 = bf16(x-x1-x2));
 *                    adds a1 b3 + a2 b2 + a3 b1 (about FP32 accuracy).
 * Intermediates of a chain are stored in the data type (FP32 for the BF16
 * forms) and re-split when read. */
typedef enum {
  KP_PREC_NATIVE = 0,
  KP_PREC_BF16X3 = 3,
  KP_PREC_BF16X6 = 6
} kp_prec;

/* Order-d tensor, column-major (mode 1 contiguous), dims[0..d-1] = m_1..m_d.
 * dims[k] >= 0; a zero size gives an empty tensor (calls then launch nothing). */
typedef struct {
  int32_t d;
  int32_t dtype; /* kp_dtype */
  int64_t dims[KP_MAX_ORDER];
  void* data;    /* device pointer */
} kp_tensor;

/* rows x cols matrix, element (i,j) at data[i*rs + j*cs] (elements, not bytes).
 * rs, cs >= 0 (a negative stride is KP_ERR_VALUE); the span the strides
 * address must stay below 2^31 bytes (KP_ERR_SHAPE otherwise). */
typedef struct {
  int64_t rows, cols;
  int64_t rs, cs;
  int32_t dtype; /* kp_dtype */
  int32_t pad_;
  void* data;    /* device pointer */
} kp_matrix;

/* ---- mu-mode product (Sec. 2, Definition of the mu-mode product) --------------
 * S = T x_mu L: every mu-fiber of T is multiplied by L. L is n x m_mu;
 * S has the dims of T with m_mu replaced by n. mu is 1-based. No permutation
 * or unfolding is materialised: the kernel reads the fibers in place.
 * If accumulate != 0, S += T x_mu L (the building block of the Kronecker-sum
 * action, Sec. 2); otherwise S is overwritten.
 * T, L and S must share the dtype. No workspace is needed. */
int kp_mump(const kp_tensor* T, const kp_matrix* L, int mu, kp_tensor* S,
            int prec, int accumulate, hipStream_t stream);

/* ---- Kronecker-sum action (Sec. 2, the action of a Kronecker sum) ----------
 * S = T x_1 A_1 + T x_2 A_2 + ... + T x_d A_d, that is
 * vec(S) = (A_d (+) ... (+) A_1) vec(T): d mu-mode products on `stream`, the
 * first writing S, each later one adding to it. Every A_mu is m_mu x m_mu
 * (none may be NULL); S has the sizes of T and must not overlap T or any A.
 * prec as for kp_mump. Errors: as kp_mump, KP_ERR_NULL for a NULL A_mu,
 * KP_ERR_SHAPE for a non-square A_mu or mismatched S. */
int kp_kronsum(const kp_tensor* T, const kp_matrix* const A[], kp_tensor* S, int prec,
               hipStream_t stream);

/* ---- Tucker operator (Sec. 2, Definition of the Tucker operator) --------------
 * S = T x_1 L[0] x_2 L[1] ... x_d L[d-1]. L[k] is n_k x m_k; S has dims
 * n_1..n_d. A NULL L[k] is the identity (mode skipped, n_k = m_k).
 * The products are applied in an order chosen to minimise flops (the
 * operator does not depend on the order, Sec. 2); ties keep 1..d.
 * Intermediates live in the workspace `ws` (ws_bytes >= kp_tucker_workspace);
 * with a cache they are written into the cache instead and ws may be NULL.
 * For the BF16 split forms kp_tucker_workspace also counts the factors'
 * bf16 planes, split once per call for the products that run on wide tiles;
 * a workspace that holds only the intermediates is accepted (those products
 * then split their factor rows themselves; the result is the same bit for
 * bit).
 * If `cache` is non-NULL it receives the forward partial products
 * P_k = T x_1 L_1 ... x_k L_k for k = 1..d-1 in definition order, packed one
 * after another as column-major tensors (cache_bytes >= kp_tucker_cache_size);
 * kp_tucker_backward can reuse them. Requesting the cache forces the
 * definition order 1..d.
 * Errors: KP_ERR_SHAPE / KP_ERR_DTYPE / KP_ERR_NULL as kp_mump;
 * KP_ERR_WORKSPACE if ws (or the cache) is missing or too small;
 * KP_ERR_ALIAS if S overlaps T or a factor, if the part of ws the call uses
 * overlaps T, S or a factor, or if the cache overlaps T, S, a factor or ws. */
size_t kp_tucker_workspace(const kp_tensor* T, const kp_matrix* const* L, int prec);
/* The order kp_tucker applies the non-identity factors in (without a cache):
 * order[0..*count-1] receives 1-based modes. Host-only query. */
int kp_tucker_order(const kp_tensor* T, const kp_matrix* const* L, int* order, int* count);
size_t kp_tucker_cache_size(const kp_tensor* T, const kp_matrix* const* L);
int kp_tucker(const kp_tensor* T, const kp_matrix* const* L, kp_tensor* S,
              int prec, void* ws, size_t ws_bytes,
              void* cache, size_t cache_bytes, hipStream_t stream);

/* ---- Tucker operator without caller memory ------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same result
 * as kp_tucker without a cache, with the intermediates held in a buffer the
 * library owns instead of a caller workspace. The buffer is a fixed device
 * array of KP_NOALLOC_SCRATCH_BYTES per device, kept from the first call on
 * that device until the process ends; the first call on a device looks up
 * its address (hipGetSymbolAddress), later calls do no set-up at all. The
 * call itself allocates and frees nothing; it only enqueues the products on
 * `stream`.
 * Every call on one device shares that device's buffer: calls whose work
 * overlaps in time on one device (different streams, or host threads without
 * ordering) race on it and must be serialised by the caller. Nothing in the
 * buffer needs to start at zero; it keeps the last call's intermediates.
 * Errors: as kp_tucker (argument errors before anything is enqueued);
 * KP_ERR_SCRATCH if kp_tucker_workspace(T, L, prec) exceeds
 * KP_NOALLOC_SCRATCH_BYTES; KP_ERR_HIP if the address look-up fails. */
#define KP_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20) /* 128 MiB */
size_t kp_noalloc_scratch_bytes(void);
int kp_tucker_noalloc(const kp_tensor* T, const kp_matrix* const* L, kp_tensor* S, int prec,
                      hipStream_t stream);

/* ---- complex Tucker operator (Sec. 2 over C; Sec. 3 conjugate-transpose form) -
 * A complex tensor is stored as interleaved (real, imaginary) pairs: T is a
 * real kp_tensor (F64 or F32) of order d + 1 whose first mode has size 2;
 * its modes 2..d+1 are the complex tensor's modes 1..d (d <= 7). Factor mu is
 * L_mu = Lre[mu-1] + i Lim[mu-1], given as two real matrices of the same
 * size (any strides, so an interleaved complex matrix is two views, element
 * strides (2*cols, 2) offset by one element). Lre[k] == NULL together with
 * Lim[k] == NULL is the identity; Lim[k] == NULL alone is a real factor.
 *   conj == 0: S = T x_1 L_1 ... x_d L_d, L_mu is n_mu x m_mu;
 *   conj != 0: S = T x_1 L_1^* ... x_d L_d^*, ^* the conjugate transpose,
 *              L_mu is m_mu x n_mu.
 * S is (2, n_1, ..., n_d) in the same layout. Modes are applied in order
 * 1..d; each is two real mu-mode products on the real kernels, with the real
 * and then the imaginary part of the factor, the second adding i (or -i for
 * the conjugate transpose) times its result in its epilogue. prec as for
 * kp_mump (the split forms need F32).
 * The factor parts are first packed, as applied, into the workspace; for the
 * BF16 split forms the workspace also holds each part's pre-split bf16
 * planes (as for kp_tucker), read by the products that run on wide tiles.
 * ws_bytes >= kp_tucker_complex_workspace(...); a workspace without room
 * for the planes (the intermediates and packed parts only) gives the same
 * result, each tile then splitting its factor rows itself. Errors: as kp_tucker, and
 * KP_ERR_ORDER for order < 2, KP_ERR_SHAPE if T's first mode is not 2 or the
 * parts of a factor differ in size, KP_ERR_NULL for Lim[k] without Lre[k]. */
size_t kp_tucker_complex_workspace(const kp_tensor* T, const kp_matrix* const* Lre,
                                   const kp_matrix* const* Lim, int conj, int prec);
int kp_tucker_complex(const kp_tensor* T, const kp_matrix* const* Lre,
                      const kp_matrix* const* Lim, kp_tensor* S, int conj, int prec, void* ws,
                      size_t ws_bytes, hipStream_t stream);

/* ---- gradient of the Tucker operator ------------------------------------------
 * Given the cotangent G = dloss/dS (dims n_1..n_d):
 *   dT    = G x_1 L_1^T ... x_d L_d^T         (dims m_1..m_d)
 *   dL_mu = Q_mu^(mu) (P_{mu-1}^(mu))^T         (n_mu x m_mu)
 * with P_k = T x_1 L_1 ... x_k L_k (P_0 = T) and
 *      Q_mu = G x_d L_d^T ... x_{mu+1} L_{mu+1}^T (Q_d = G), so that Q_0 = dT.
 * dT may be NULL, and any dL[k] may be NULL, to skip that output. The dL[k]
 * are written with their own strides (dtype of T). `cache` is the forward
 * cache written by kp_tucker (or NULL: the P_k are recomputed).
 * Every L[k] must be non-NULL here. ws_bytes >= kp_tucker_backward_workspace.
 * Errors: as kp_tucker; KP_ERR_ALIAS if an output (dT, a dL[k]) overlaps an
 * input (G, T, a factor, the cache), ws or another output, or if ws overlaps
 * G, T, a factor or the cache. */
size_t kp_tucker_backward_workspace(const kp_tensor* T, const kp_matrix* const* L,
                                    int prec);
int kp_tucker_backward(const kp_tensor* G, const kp_tensor* T,
                       const kp_matrix* const* L, const void* cache,
                       size_t cache_bytes, kp_tensor* dT, kp_matrix* const* dL,
                       int prec, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- batched Tucker operator: persistent launches per dependency level -----
 * `count` independent problems of any orders and sizes (same dtype), each a
 * Tucker operator in definition order (Sec. 2) and optionally its gradient.
 * All tasks of all problems that sit at the same dependency level (the
 * forward product of mode s, a factor-gradient partial sum, ...) and share
 * a task type (tile or strip variant, gram, reduce) run in ONE persistent
 * launch of a kernel compiled for that type; levels are launched in order on
 * `stream`, so no workgroup waits for another. A forward pass of order-d
 * problems takes d levels, forward plus backward about d + 2 (the reverse
 * sweep does not wait for the forward); a HIP graph capturing
 * kp_tucker_batched replays the whole batch.
 * Per problem: S = T x_1 L[0] ... x_d L[d-1] (no identity factors here).
 * If G.data != NULL the backward runs too: dT (if dT.data != NULL) and every
 * dL[k] with dL[k].data != NULL, as kp_tucker_backward defines them; the
 * forward partial products are kept in the workspace for it.
 * Each problem's tensors must stay below 2^31 bytes.
 *
 * Use: (1) ws_bytes = kp_batch_workspace(), plan_bytes = kp_batch_plan_bytes();
 * (2) kp_batch_plan() writes the plan into HOST memory `plan`, with every
 *     device address (inputs, outputs, intermediates in `ws`) resolved;
 * (3) the caller copies the plan bytes to device memory `plan_dev`;
 * (4) kp_tucker_batched(plan_dev, plan, ws, ...) enqueues the launches; it can
 *     be called (or graph-replayed) any number of times while the buffers stay
 *     valid. Calls that share `ws` must not overlap in time.
 * Tile shapes per mode product come from the tuning table (kp_tune_set) or
 * the built-in defaults, restricted to the variants the executor carries.
 * Errors: KP_ERR_NULL, KP_ERR_ORDER, KP_ERR_DTYPE, KP_ERR_SHAPE (mismatched
 * sizes, NULL or identity factors, a tensor of 2^31 bytes or more),
 * KP_ERR_WORKSPACE (ws or plan too small, or ws not the planned one),
 * KP_ERR_VALUE (count < 0, plan bytes not a plan or with an inconsistent
 * launch group). */
typedef struct {
  kp_tensor T, S;
  kp_matrix L[KP_MAX_ORDER];
  kp_tensor G, dT;
  kp_matrix dL[KP_MAX_ORDER];
} kp_batch_item;

size_t kp_batch_workspace(int count, const kp_batch_item* items, int prec);
size_t kp_batch_plan_bytes(int count, const kp_batch_item* items, int prec);
int kp_batch_plan(int count, const kp_batch_item* items, int prec, void* ws, size_t ws_bytes,
                  void* plan, size_t plan_bytes);
int kp_batch_info(const void* plan, int64_t* ntasks, int* nstages, int* nlevels);
int kp_tucker_batched(const void* plan_dev, const void* plan, void* ws, size_t ws_bytes,
                      hipStream_t stream);

/* ---- exponential of small matrices in FP64 (Sec. 3.3 factor build) ----------
 * E_k = exp(tau * A_k) for `count` n x n column-major FP64 matrices stored one
 * after another in A (device memory); E receives them in the same layout.
 * n <= 256. Scaling and squaring with the degree-13 diagonal Pade approximant
 * (Higham 2005), all steps on the device as a fixed sequence of launches on
 * `stream` (the scaling exponent stays in the workspace; the products run
 * over 32 x 32 tiles of every matrix, the Pade solve and any squarings past
 * the eighth in one workgroup per matrix), so the call never synchronises.
 * ws_bytes >= kp_expm_workspace(n, count).
 * Errors: KP_ERR_SHAPE (n < 0, n > 256, count < 0), KP_ERR_NULL,
 * KP_ERR_VALUE (tau not finite), KP_ERR_WORKSPACE, KP_ERR_ALIAS (E overlaps
 * A or the workspace). A singular Pade denominator (impossible for finite
 * ||tau A||) would propagate Inf/NaN. */
size_t kp_expm_workspace(int64_t n, int64_t count);
int kp_expm_f64(const double* A, int64_t n, int64_t count, double tau, double* E, void* ws,
                size_t ws_bytes, hipStream_t stream);

/* ---- inverse of tridiagonal matrices in FP64 (Sec. 3.4, ADI factors) --------
 * E_k = (shift I + scale T_k)^{-1} for `count` tridiagonal n x n matrices T_k
 * given by their diagonals in device memory (n doubles each, matrix k at
 * offset k*n): T[i][i-1] = lower[i] (i >= 1), T[i][i] = diag[i],
 * T[i][i+1] = upper[i] (i <= n-2); lower[0] and upper[n-1] are not read.
 * E receives `count` column-major n x n matrices one after another. With
 * shift = 1, scale = -tau and T the second difference A_mu this is the
 * factor (I - tau A_mu)^{-1} of the ADI-type preconditioner.
 * Gaussian elimination without pivoting per column of the identity: the
 * matrix must be one for which that is stable (diagonally dominant, or
 * symmetric positive definite, as I - tau A_mu is); a zero pivot propagates
 * Inf/NaN. n <= 2048, count <= 65535. No workspace; never synchronises.
 * Errors: KP_ERR_SHAPE (n or count out of range), KP_ERR_NULL, KP_ERR_VALUE
 * (shift or scale not finite), KP_ERR_ALIAS (E overlaps a diagonal). */
int kp_tridiag_inverse_f64(const double* lower, const double* diag, const double* upper,
                           int64_t n, int64_t count, double shift, double scale, double* E,
                           hipStream_t stream);

/* ---- preconditioned conjugate gradients on a Kronecker sum (Sec. 3.4) -------
 * Solves (M_d (+) ... (+) M_1) vec(X) = vec(B) for symmetric positive definite
 * systems, FP64. The matrix action is the Kronecker-sum action (kp_kronsum)
 * with the square M[k] (m_k x m_k, none NULL). If P is non-NULL the
 * preconditioner action is the Tucker operator R x_1 P[0] ... x_d P[d-1]
 * (kp_tucker; a NULL P[k] is the identity), i.e. P[k] holds the inverse of
 * the k-th factor of a Kronecker-product preconditioner; P == NULL runs plain
 * conjugate gradients.
 * X holds the initial guess on entry and the solution on return. Iterations
 * stop when ||B - M X||_2 <= tol ||B||_2 (also before the first) or after
 * maxit; B == 0 returns X = 0. *iters and *relres (each may be NULL) receive
 * the iteration count and the final relative residual; not converging within
 * maxit is not an error (relres > tol tells).
 * The iteration loop runs on the host and waits for `stream` once per
 * iteration to read the residual norm, so this call blocks and cannot be
 * captured into a graph. ws_bytes >= kp_pcg_workspace(X, P).
 * Errors: KP_ERR_NULL, KP_ERR_ORDER, KP_ERR_DTYPE (not FP64), KP_ERR_SHAPE
 * (B, X, M[k], P[k] sizes), KP_ERR_VALUE (tol negative or not finite,
 * maxit < 0, a negative stride), KP_ERR_WORKSPACE, KP_ERR_ALIAS (X overlaps B,
 * a factor or ws; B or a factor overlaps ws). */
size_t kp_pcg_workspace(const kp_tensor* X, const kp_matrix* const* P);
int kp_pcg_kronsum(const kp_tensor* B, const kp_matrix* const* M, const kp_matrix* const* P,
                   kp_tensor* X, double tol, int maxit, void* ws, size_t ws_bytes, int* iters,
                   double* relres, hipStream_t stream);

/* ---- backward-forward Euler for the semilinear experiment (Sec. 4.5) -------
 * u_t = Laplacian(u) + 1/(1 + u^2) + Phi(t, x) on the interior grid points
 * x_mu = (i_mu + 1) h[mu] of [0,1]^d (column-major U, dims m_1..m_d), with
 * Phi(t, x) = e^t (u0 - Laplacian(u0)) - 1/(1 + e^{2t} u0^2) and
 * u0 = prod_mu x_mu (1 - x_mu), so that e^t u0 solves the problem.
 * The discrete Laplacian is the Kronecker sum of the tridiagonal A_mu given
 * by the device diagonals lower[mu], diag[mu], upper[mu] (m_mu doubles each,
 * layout as kp_tridiag_inverse_f64). Each of `steps` steps, from t0 on with
 * step tau, solves
 *   (M_d (+) ... (+) M_1) u_{k+1} = u_k + tau (1/(1 + u_k^2) + Phi(t_k)),
 *   M_mu = I/d - tau A_mu,
 * by kp_pcg_kronsum from u_k (relative tolerance tol, at most maxit
 * iterations), with the ADI preconditioner factors (I - tau A_mu)^{-1}
 * (built on the device) if `precondition` is non-zero. U is updated in
 * place; iters (host, `steps` ints, may be NULL) receives the iterations of
 * each step. Blocks like kp_pcg_kronsum. m_mu <= 2048.
 * ws_bytes >= kp_semilinear_workspace(d, dims).
 * Errors: KP_ERR_NULL, KP_ERR_ORDER, KP_ERR_DTYPE (U not FP64), KP_ERR_SHAPE,
 * KP_ERR_VALUE (h not positive, t0 / tau / tol not finite, steps, maxit or
 * tol negative), KP_ERR_WORKSPACE, KP_ERR_ALIAS (U overlaps ws or a
 * diagonal). */
size_t kp_semilinear_workspace(int d, const int64_t* dims);
int kp_semilinear_imex_f64(kp_tensor* U, const double* const* lower, const double* const* diag,
                           const double* const* upper, const double* h, double t0, double tau,
                           int steps, double tol, int maxit, int precondition, void* ws,
                           size_t ws_bytes, int* iters, hipStream_t stream);

/* ---- tuning ----------------------------------------------------------------
 * A tile is (nb, fb, bk, occ, pf, kind):
 *   kind 0  k-loop tile: nb 16-wide blocks along n per workgroup, fb 16-wide
 *           fiber blocks per wave (4 waves), bk the k-chunk staged in LDS
 *           per step (32 for the BF16 forms), occ the waves per SIMD the
 *           variant's register budget targets (0: any), pf the prefetch
 *           distance in k-chunks (1 or 2; 0: 1);
 *   kind 1  strip tile for short contractions (m <= bk): the workgroup keeps
 *           its nb blocks of L rows in LDS and streams many fiber tiles of
 *           64*fb fibers; bk is the padded contraction length, occ = pf = 0;
 *   kind 3  wide tile of the BF16 split forms: the 4 waves split 64*nb rows
 *           of n (nb 16-wide blocks each), each loading and splitting its
 *           own rows of L, and share 16*fb fibers staged in LDS; bk = 32,
 *           pf = 2 (two chunks of fibers in flight).
 * Kind 2 is not a tile: it names a fused pair of modes in launch reports.
 * kp_force_tile forces the tile of every later mode-product launch in this
 * process; nb <= 0 restores the table / default choice. KP_ERR_VALUE for a
 * negative or out-of-range field. A launch whose forced tile is not a
 * compiled variant (or a strip shorter than m) fails with KP_ERR_HIP
 * (hipErrorInvalidValue). Not thread-safe; meant for tests and the
 * tile-timing driver. */
int kp_force_tile(int nb, int fb, int bk, int occ, int pf, int kind);

/* Process-wide options (not thread-safe; set them before launching).
 *   KP_OPT_FUSE (default 1): kp_tucker without a cache, on FP32 data with
 *   the native precision, applies two consecutive modes mu, mu + 1 of its
 *   planned order in one pass when both are short (m <= 16, n <= 32) and
 *   I_l > 1, so the intermediate never reaches HBM; the result is the same
 *   as applying them one after the other (same sums, same rounding).
 * kp_set_option returns KP_ERR_VALUE for an unknown option or value;
 * kp_get_option returns the value, or KP_ERR_VALUE. */
#define KP_OPT_FUSE 1
int kp_set_option(int option, int value);
int kp_get_option(int option);

/* Tile table. Before its built-in defaults, the library looks the tile of
 * each mu-mode product up in a process-wide table keyed by the product's
 * form and exact 3-index view; kp_tucker, kp_tucker_backward, kp_mump and
 * the batched planner (when its executor compiles that tile) all consult it,
 * a tile forced by kp_force_tile takes precedence. The table is filled by a
 * tuning driver that times the compiled variants on the products of a
 * problem (the Python package's `tune` module) or from a saved table.
 * Thread-safe.
 *   form   0 FP64, 1 FP32, 3 BF16x3, 6 BF16x6 (the last two on FP32 data)
 *   Il, m, n, Ir   the view: X is (Il, m, Ir), Y = (Il, n, Ir), L is n x m
 *   nb, fb, bk, occ, pf, kind   the tile, as for kp_force_tile (occ, pf as
 *                               compiled) */
typedef struct {
  int32_t form, pad0_;
  int64_t Il, m, n, Ir;
  int32_t nb, fb, bk, occ, pf, kind;
} kp_tune_entry; /* 64 bytes */

/* Insert or replace the entry for e's key. KP_ERR_NULL if e is NULL;
 * KP_ERR_VALUE if the key is invalid (form not 0/1/3/6, a size < 1), no
 * compiled variant has that tile (occ 0 or pf 0 take the first compiled
 * match, which is what is stored), or a strip tile is shorter than m. */
int kp_tune_set(const kp_tune_entry* e);
/* The tile a product with this key gets when no tile is forced: returns 1
 * and fills *out (with the queried key) from the table if the key, or its
 * shape class, is tuned, 0 and fills *out with the built-in default
 * otherwise; KP_ERR_NULL / KP_ERR_VALUE on bad input. Shape class: a key
 * without an entry of its own takes the entry with the same form, layout
 * (Il = 1 or Il > 1), m and n whose fiber count Il*Ir is nearest in ratio
 * to its own, within a factor of two (ties: the smaller count). */
int kp_tune_lookup(int form, int64_t Il, int64_t m, int64_t n, int64_t Ir, kp_tune_entry* out);
/* Number of entries; kp_tune_list copies the first min(cap, count) entries
 * (in key order) to out (may be NULL when cap is 0) and returns the count. */
int kp_tune_count(void);
int kp_tune_list(kp_tune_entry* out, int cap);
/* Remove every entry. */
int kp_tune_clear(void);
/* The mu-mode products a call launches for these shapes, in launch order,
 * each as a table key with the tile it gets now (table or default):
 *   which 0  kp_tucker without a cache (planned minimum-flop order)
 *         1  kp_tucker with a cache, and the forward partials that
 *            kp_tucker_backward recomputes (definition order)
 *         2  kp_tucker_backward's cotangent sweep Q_{mu-1} = Q_mu x_mu L_mu^T
 *            (mu = d..1; when dT is not wanted the sweep stops early)
 *         3  kp_tucker without a cache, one entry per launch: a fused pass
 *            over modes mu, mu + 1 (KP_OPT_FUSE) is one entry with kind 2,
 *            the view of mode mu and the other tile fields 0
 * Writes min(cap, count) entries (out may be NULL if cap is 0) and returns
 * the count; argument errors as kp_tucker_workspace's validation
 * (KP_ERR_NULL for which = 2 with an identity factor, KP_ERR_VALUE for a
 * bad `which`). Data pointers are not read. */
int kp_tucker_products(const kp_tensor* T, const kp_matrix* const L[], int prec, int which,
                       kp_tune_entry* out, int cap);
/* The compiled tiles for a form: batch = 0 the standalone kernels, batch =
 * 1 the batched executor; 6 ints per tile (nb, fb, bk, occ, pf, kind).
 * Writes min(cap, count) tiles to out (NULL if cap is 0) and returns the
 * count; KP_ERR_VALUE for an unknown form. */
int kp_tile_variants(int form, int batch, int32_t* out, int cap);

/* ---- utilities ------------------------------------------------------------- */
const char* kp_strerror(int status);
int kp_version(void);
int kp_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KP_H_ */
