// Host-side helpers shared by the C-ABI translation units.
#pragma once

#include "kp.h"
#include "kp_common.h"

namespace kp {

// Tile forced by kp_force_tile (nullptr: use the tuned / default choice).
const ModeTile* tile_override();
// KP_OPT_FUSE: consecutive short modes fused in kp_tucker.
bool fusion_enabled();

int hip_status(hipError_t e);
// Three-index view arguments for the product of mode mu0 (0-based) of a
// column-major tensor with sizes dims[0..d-1] (kp_api.hip).
ModeArgs mode_args(const void* X, void* Y, const int64_t* dims, int d, int mu0,
                   const kp_matrix& L, int accumulate);
size_t elem_size(int dtype);
size_t align_up(size_t x);
// Argument checks shared by the entry points (kp_api.hip): KP_OK or an error.
int check_tensor(const kp_tensor* t, bool need_data);
int check_prec(int prec, int dtype);
int form_of(int prec, int dtype);
int64_t numel(const kp_tensor& t);
int check_matrix(const kp_matrix* L, int dtype);
bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes);
size_t matrix_span_bytes(const kp_matrix& L);

// Factor-gradient contraction (gram_kernels.hip): dL(i,j) = sum_r Q(r,i) P(r,j)
// over the fibers of the views Q (Il, n, Ir) and P (Il, m, Ir), written at
// dL[i*rs + j*cs]; `part` is a workspace of gram_workspace() bytes.
int64_t gram_splits(int64_t Il, int64_t n, int64_t m, int64_t Ir);
size_t gram_workspace(int64_t Il, int64_t n, int64_t m, int64_t Ir, size_t esize);
hipError_t launch_gram(int dtype, const void* Q, const void* P, int64_t Il, int64_t n, int64_t m,
                       int64_t Ir, void* part, void* dL, int64_t rs, int64_t cs,
                       hipStream_t stream);
// The same contraction fused with Y = Q x_mu L^T (L: n x m, Y viewed as
// (Il, m, Ir)), reading Q once: FP32 data, Il a multiple of 4, n, m <= 32, Q,
// P and Y 16-byte aligned (gram_product_eligible); the product in `form`
// (FP32 or a BF16 split form), the gradient in FP32; same `part` workspace.
bool gram_product_eligible(int dtype, const void* Q, const void* P, const void* Y, int64_t Il,
                           int64_t n, int64_t m, int64_t Ir);
hipError_t launch_gram_product(int form, const void* Q, const void* P, int64_t Il, int64_t n,
                               int64_t m, int64_t Ir, void* part, void* dL, int64_t rs, int64_t cs,
                               const kp_matrix& L, void* Y, hipStream_t stream);

// Pre-split factor planes of the BF16 split forms' wide tiles (wide_tile.h):
// bytes for an n x m factor, whether a product runs on a wide tile (and so
// can read planes), one launch splitting up to KP_MAX_ORDER FP32 factors,
// and a product launch reading a factor's planes (nullptr: the tile splits
// the factor itself).
struct SplitJob {
  const void* L;
  int64_t n, m, rs, cs;
  void* planes;
  int64_t begin;  // first task (one lane of one block and step) of this job
};
struct SplitJobs {
  SplitJob job[KP_MAX_ORDER];
  int count;
  int64_t total;
};
size_t split_planes_bytes(int form, int64_t n, int64_t m);
// Tasks (one lane of one 16-row block and 32-wide k step) of one factor.
int64_t split_planes_tasks(int64_t n, int64_t m);
bool mode_uses_wide(int form, const ModeArgs& a, const ModeTile* force);
hipError_t launch_split_planes(int form, const SplitJobs& jobs, hipStream_t stream);
hipError_t launch_mode_planes(int form, const ModeArgs& a, const ModeTile* force,
                              const void* planes, hipStream_t stream);

}  // namespace kp
