// The Tucker operator over the complex field and its conjugate-transpose
// form (Sec. 2 states the mu-mode product and the Tucker operator for complex
// tensors; Sec. 3 applies the conjugate-transposed basis matrices to evaluate
// spectral decompositions at their quadrature grid).
//
// A complex tensor is stored as interleaved (real, imaginary) pairs, i.e. as
// a real tensor with an extra first mode of size 2; the real and imaginary
// parts of a factor are two real matrices (two strided views of an
// interleaved complex matrix). Mode mu of the complex product is then
//   Y = X x_(mu+1) Re(L) + i s (X x_(mu+1) Im(L)),
// two real mu-mode products on the same real kernels (the size-2 mode sits
// in the fibers' leading index), s = +1 for L and -1 for the conjugate
// transpose. The second product's epilogue adds i s times its value: the
// parts of one complex output are adjacent fibers, held by neighbouring
// lanes, so each lane combines with its partner's value before the store.
#include "kp.h"

#include "kp_common.h"
#include "kp_internal.h"

namespace kp {
namespace {

constexpr int kPT = 256;

// One factor part to pack: dst[i * cols + j] = A(i, j) = src[i * rs + j * cs]
// for an rows x cols matrix (the part as applied, packed k-contiguous);
// begin: its first element in the launch's element range.
struct PackJob {
  const void* src;
  int64_t rows, cols, rs, cs;
  void* dst;
  int64_t begin;
};
struct PackJobs {
  PackJob job[2 * KP_MAX_ORDER];
  int count;
  int64_t total;
};

// Every part of a call in one launch: element e (grid-stride) belongs to
// the job whose range holds it.
template <typename E>
__global__ __launch_bounds__(kPT) void pack_kernel(PackJobs jobs) {
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kPT) + threadIdx.x; e < jobs.total;
       e += static_cast<int64_t>(gridDim.x) * kPT) {
    int j = 0;
    while (j + 1 < jobs.count && e >= jobs.job[j + 1].begin) ++j;
    const PackJob& J = jobs.job[j];
    const int64_t loc = e - J.begin;
    const int64_t i = loc / J.cols, c = loc - i * J.cols;
    static_cast<E*>(J.dst)[loc] = static_cast<const E*>(J.src)[i * J.rs + c * J.cs];
  }
}

int64_t count_of(const int64_t* dims, int d) {
  int64_t s = 1;
  for (int k = 0; k < d; ++k) s *= dims[k];
  return s;
}

// The factor applied at complex mode k: L, or its transpose for the
// conjugate-transpose form (the sign of the imaginary part is applied in
// the epilogue of the imaginary-part product).
kp_matrix applied(const kp_matrix& L, int conj) {
  if (!conj) return L;
  kp_matrix t = L;
  t.rows = L.cols;
  t.cols = L.rows;
  t.rs = L.cs;
  t.cs = L.rs;
  return t;
}

struct ComplexPlan {
  int d;                                    // complex order
  int64_t dims[KP_MAX_ORDER + 1][KP_MAX_ORDER];  // real dims before step s
  int steps;
  int mode[KP_MAX_ORDER];                   // complex mode (0-based) of step s
  int64_t big;                              // largest intermediate (real entries)
};

int validate(const kp_tensor* T, const kp_matrix* const* Lre, const kp_matrix* const* Lim,
             int conj, int prec, ComplexPlan* p) {
  int st = check_tensor(T, true);
  if (st) return st;
  if (!Lre || !Lim) return KP_ERR_NULL;
  if (T->d < 2) return KP_ERR_ORDER;
  if (T->dims[0] != 2) return KP_ERR_SHAPE;
  st = check_prec(prec, T->dtype);
  if (st) return st;
  p->d = T->d - 1;
  p->steps = 0;
  p->big = 0;
  int64_t cur[KP_MAX_ORDER];
  for (int k = 0; k < T->d; ++k) cur[k] = T->dims[k];
  for (int k = 0; k < p->d; ++k) {
    if (!Lre[k]) {
      if (Lim[k]) return KP_ERR_NULL;
      continue;
    }
    st = check_matrix(Lre[k], T->dtype);
    if (st) return st;
    const kp_matrix a = applied(*Lre[k], conj);
    if (a.cols != T->dims[k + 1]) return KP_ERR_SHAPE;
    if (Lim[k]) {
      st = check_matrix(Lim[k], T->dtype);
      if (st) return st;
      if (Lim[k]->rows != Lre[k]->rows || Lim[k]->cols != Lre[k]->cols) return KP_ERR_SHAPE;
    }
    for (int j = 0; j < T->d; ++j) p->dims[p->steps][j] = cur[j];
    p->mode[p->steps] = k;
    cur[k + 1] = a.rows;
    const int64_t out = count_of(cur, T->d);
    ++p->steps;
    if (out > p->big) p->big = out;
  }
  for (int j = 0; j < T->d; ++j) p->dims[p->steps][j] = cur[j];
  return KP_OK;
}

// Workspace of a validated call: `base` holds two ping-pong buffers for the
// intermediates (only with two or more steps), then every factor part
// packed k-contiguous; `planes` (BF16 split forms only) one set of
// pre-split bf16 planes per factor part, placed after them.
void complex_ws(const kp_tensor* T, const kp_matrix* const* Lre, const kp_matrix* const* Lim,
                int conj, int prec, const ComplexPlan& p, size_t* base, size_t* planes) {
  const size_t es = elem_size(T->dtype);
  const int form = form_of(prec, T->dtype);
  const bool split = form == FORM_BF16X3 || form == FORM_BF16X6;
  *base = p.steps > 1 ? 2 * align_up(static_cast<size_t>(p.big) * es) : 0;
  *planes = 0;
  for (int k = 0; k < p.d; ++k) {
    if (!Lre[k]) continue;
    const kp_matrix a = applied(*Lre[k], conj);
    const int parts = Lim[k] ? 2 : 1;
    *base += parts * align_up(static_cast<size_t>(a.rows * a.cols) * es);
    if (split) *planes += parts * align_up(split_planes_bytes(form, a.rows, a.cols));
  }
}

}  // namespace
}  // namespace kp

using namespace kp;

extern "C" {

size_t kp_tucker_complex_workspace(const kp_tensor* T, const kp_matrix* const* Lre,
                                   const kp_matrix* const* Lim, int conj, int prec) {
  ComplexPlan p;
  if (validate(T, Lre, Lim, conj, prec, &p)) return 0;
  size_t base = 0, planes = 0;
  complex_ws(T, Lre, Lim, conj, prec, p, &base, &planes);
  return base + planes;
}

int kp_tucker_complex(const kp_tensor* T, const kp_matrix* const* Lre,
                      const kp_matrix* const* Lim, kp_tensor* S, int conj, int prec, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
  ComplexPlan p;
  int st = validate(T, Lre, Lim, conj, prec, &p);
  if (st) return st;
  if (!S) return KP_ERR_NULL;
  st = check_tensor(S, true);
  if (st) return st;
  if (S->dtype != T->dtype) return KP_ERR_DTYPE;
  if (S->d != T->d) return KP_ERR_SHAPE;
  for (int j = 0; j < T->d; ++j)
    if (S->dims[j] != p.dims[p.steps][j]) return KP_ERR_SHAPE;
  const size_t es = elem_size(T->dtype);
  const size_t sb = static_cast<size_t>(numel(*S)) * es;
  const size_t tb = static_cast<size_t>(numel(*T)) * es;
  if (overlaps(S->data, sb, T->data, tb)) return KP_ERR_ALIAS;
  for (int k = 0; k < p.d; ++k) {
    if (Lre[k] && overlaps(S->data, sb, Lre[k]->data, matrix_span_bytes(*Lre[k])))
      return KP_ERR_ALIAS;
    if (Lim[k] && overlaps(S->data, sb, Lim[k]->data, matrix_span_bytes(*Lim[k])))
      return KP_ERR_ALIAS;
  }
  // the planes are used when the workspace has room for them (a workspace
  // of `base` bytes runs the products with in-register splits)
  size_t need = 0, planes_need = 0;
  complex_ws(T, Lre, Lim, conj, prec, p, &need, &planes_need);
  if (need > 0 && (!ws || ws_bytes < need)) return KP_ERR_WORKSPACE;
  const size_t planes_at = need;
  if (planes_need > 0 && ws_bytes >= need + planes_need)
    need += planes_need;
  else
    planes_need = 0;
  if (need > 0 && (overlaps(ws, need, S->data, sb) || overlaps(ws, need, T->data, tb)))
    return KP_ERR_ALIAS;
  for (int k = 0; k < p.d; ++k) {
    if (Lre[k] && overlaps(ws, need, Lre[k]->data, matrix_span_bytes(*Lre[k])))
      return KP_ERR_ALIAS;
    if (Lim[k] && overlaps(ws, need, Lim[k]->data, matrix_span_bytes(*Lim[k])))
      return KP_ERR_ALIAS;
  }
  if (numel(*S) == 0) return KP_OK;
  if (p.steps == 0)
    return hip_status(hipMemcpyAsync(S->data, T->data, sb, hipMemcpyDeviceToDevice, stream));
  if (!ws) return KP_ERR_WORKSPACE;

  const int form = form_of(prec, T->dtype);
  char* w = static_cast<char*>(ws);
  const size_t buf = align_up(static_cast<size_t>(p.big) * es);
  char* pp[2] = {w, w + buf};
  // Factor parts as applied (transposed for the conjugate form). A part
  // whose product runs on a wide tile with the workspace's room for planes
  // is split into bf16 planes straight from its strided view; every other
  // part is packed k-contiguous into its workspace slot, so its product
  // stages it with 16-byte loads. One launch packs all parts, one splits up
  // to KP_MAX_ORDER.
  char* fw = w + (p.steps > 1 ? 2 * buf : 0);
  char* at = w + planes_at;
  kp_matrix pre[KP_MAX_ORDER], pim[KP_MAX_ORDER];
  const void* planes_re[KP_MAX_ORDER] = {};
  const void* planes_im[KP_MAX_ORDER] = {};
  PackJobs packs{};
  SplitJobs splits{};
  // the view the product of part L reads (*out) and, with planes, where
  // they go (*slot); slots in the workspace's order (modes 1..d, real part
  // first)
  auto place = [&](const kp_matrix& L, bool planes, kp_matrix* out, const void** slot) -> int {
    const kp_matrix a = applied(L, conj);
    *out = a;
    const int64_t total = a.rows * a.cols;
    char* packed = fw;
    fw += align_up(static_cast<size_t>(total) * es);
    if (planes) {
      SplitJob& J = splits.job[splits.count++];
      J.L = a.data;
      J.n = a.rows;
      J.m = a.cols;
      J.rs = a.rs;
      J.cs = a.cs;
      J.planes = at;
      J.begin = splits.total;
      splits.total += split_planes_tasks(J.n, J.m);
      *slot = at;
      at += align_up(split_planes_bytes(form, a.rows, a.cols));
      if (splits.count < KP_MAX_ORDER) return KP_OK;
      const int r = hip_status(launch_split_planes(form, splits, stream));
      splits = SplitJobs{};
      return r;
    }
    out->rs = a.cols;
    out->cs = 1;
    out->data = packed;
    if (total == 0) return KP_OK;
    PackJob& J = packs.job[packs.count++];
    J.src = a.data;
    J.rows = a.rows;
    J.cols = a.cols;
    J.rs = a.rs;
    J.cs = a.cs;
    J.dst = packed;
    J.begin = packs.total;
    packs.total += total;
    return KP_OK;
  };
  for (int s = 0; s < p.steps; ++s) {
    const int k = p.mode[s];
    const ModeArgs shape =
        mode_args(nullptr, nullptr, p.dims[s], T->d, k + 1, applied(*Lre[k], conj), kAccNone);
    const bool planes = planes_need > 0 && mode_uses_wide(form, shape, tile_override());
    st = place(*Lre[k], planes, &pre[k], &planes_re[k]);
    if (st) return st;
    if (Lim[k]) {
      st = place(*Lim[k], planes, &pim[k], &planes_im[k]);
      if (st) return st;
    }
  }
  if (packs.count > 0) {
    const int64_t blocks = (packs.total + kPT - 1) / kPT;
    const unsigned grid = static_cast<unsigned>(blocks < 1024 ? blocks : 1024);
    if (T->dtype == KP_F64)
      hipLaunchKernelGGL(pack_kernel<double>, dim3(grid), dim3(kPT), 0, stream, packs);
    else
      hipLaunchKernelGGL(pack_kernel<float>, dim3(grid), dim3(kPT), 0, stream, packs);
    st = hip_status(hipGetLastError());
    if (st) return st;
  }
  if (splits.count > 0) {
    st = hip_status(launch_split_planes(form, splits, stream));
    if (st) return st;
  }
  const void* src = T->data;
  int cur = -1;
  for (int s = 0; s < p.steps; ++s) {
    const int k = p.mode[s];
    void* dst;
    if (s == p.steps - 1) {
      dst = S->data;
    } else {
      cur = cur == 0 ? 1 : 0;
      dst = pp[cur];
    }
    ModeArgs a = mode_args(src, dst, p.dims[s], T->d, k + 1, pre[k], kAccNone);
    st = hip_status(launch_mode_planes(form, a, tile_override(), planes_re[k], stream));
    if (st) return st;
    if (Lim[k]) {
      // dst += i s (src x Im(L)), combined in the product's epilogue
      ModeArgs b =
          mode_args(src, dst, p.dims[s], T->d, k + 1, pim[k], conj ? kAccSubI : kAccAddI);
      st = hip_status(launch_mode_planes(form, b, tile_override(), planes_im[k], stream));
      if (st) return st;
    }
    src = dst;
  }
  return KP_OK;
}

}  // extern "C"
