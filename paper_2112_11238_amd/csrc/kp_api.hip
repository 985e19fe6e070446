// Host runtime of the C-ABI declared in include/kp.h: argument validation,
// mode-order planning, workspace layout and kernel launches. No allocation,
// no synchronisation: every entry point only enqueues work on the caller's
// stream, so calls can be captured into a HIP graph.
#include "kp.h"

#include <string.h>

#include "kp_common.h"
#include "kp_internal.h"
#include "pair_tile.h"

namespace kp {

thread_local int g_last_hip_error = 0;

int hip_status(hipError_t e) {
  if (e == hipSuccess) return KP_OK;
  g_last_hip_error = static_cast<int>(e);
  return KP_ERR_HIP;
}

size_t elem_size(int dtype) { return dtype == KP_F64 ? 8 : 4; }

int64_t numel(const kp_tensor& t) {
  int64_t s = 1;
  for (int k = 0; k < t.d; ++k) s *= t.dims[k];
  return s;
}

int check_tensor(const kp_tensor* t, bool need_data) {
  if (!t) return KP_ERR_NULL;
  if (t->d < 1 || t->d > KP_MAX_ORDER) return KP_ERR_ORDER;
  if (t->dtype != KP_F64 && t->dtype != KP_F32) return KP_ERR_DTYPE;
  for (int k = 0; k < t->d; ++k)
    if (t->dims[k] < 0) return KP_ERR_SHAPE;
  if (need_data && !t->data && numel(*t) > 0) return KP_ERR_NULL;
  return KP_OK;
}

int check_matrix(const kp_matrix* L, int dtype) {
  if (L->rows < 0 || L->cols < 0) return KP_ERR_SHAPE;
  if (L->rs < 0 || L->cs < 0) return KP_ERR_VALUE;
  if (L->dtype != dtype) return KP_ERR_DTYPE;
  if (!L->data && L->rows > 0 && L->cols > 0) return KP_ERR_NULL;
  // the kernels address factors with 32-bit byte offsets
  if (L->rows > 0 && L->cols > 0 &&
      ((L->rows - 1) * L->rs + (L->cols - 1) * L->cs + 1) * static_cast<int64_t>(elem_size(dtype)) >=
          (static_cast<int64_t>(1) << 31))
    return KP_ERR_SHAPE;
  return KP_OK;
}

int check_prec(int prec, int dtype) {
  if (prec == KP_PREC_NATIVE) return KP_OK;
  if (prec == KP_PREC_BF16X3 || prec == KP_PREC_BF16X6)
    return dtype == KP_F32 ? KP_OK : KP_ERR_DTYPE;
  return KP_ERR_DTYPE;
}

int form_of(int prec, int dtype) {
  if (prec == KP_PREC_BF16X3) return FORM_BF16X3;
  if (prec == KP_PREC_BF16X6) return FORM_BF16X6;
  return dtype == KP_F64 ? FORM_F64 : FORM_F32;
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  if (!a || !b || abytes == 0 || bbytes == 0) return false;
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + bbytes && pb < pa + abytes;
}

size_t matrix_span_bytes(const kp_matrix& L) {
  if (L.rows == 0 || L.cols == 0) return 0;
  const int64_t last = (L.rows - 1) * L.rs + (L.cols - 1) * L.cs;
  return static_cast<size_t>(last + 1) * elem_size(L.dtype);
}

size_t align_up(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

ModeArgs mode_args(const void* X, void* Y, const int64_t* dims, int d, int mu0,
                   const kp_matrix& L, int accumulate) {
  ModeArgs a;
  a.X = X;
  a.Y = Y;
  a.L = L.data;
  a.Il = 1;
  for (int k = 0; k < mu0; ++k) a.Il *= dims[k];
  a.m = dims[mu0];
  a.n = L.rows;
  a.Ir = 1;
  for (int k = mu0 + 1; k < d; ++k) a.Ir *= dims[k];
  a.rs = L.rs;
  a.cs = L.cs;
  a.accumulate = accumulate;
  return a;
}

// Minimum-flop order of the d products (dynamic programming over the set of
// modes already applied). Applying mode mu costs 2 n_mu times the current
// number of entries; ties keep the definition order.
void plan_order(const int64_t* m, const int64_t* n, const bool* active, int d, int* order,
                int* count) {
  const int full = 1 << d;
  double best[1 << KP_MAX_ORDER];
  int choice[1 << KP_MAX_ORDER];
  int target = 0;
  for (int k = 0; k < d; ++k)
    if (active[k]) target |= 1 << k;
  for (int s = 0; s < full; ++s) best[s] = 1e300;
  best[target] = 0.0;
  // best[s] = minimal cost to finish from state s (s = applied set)
  for (int s = full - 1; s >= 0; --s) {
    if ((s & ~target) != 0 || s == target) continue;
    double size = 1.0;
    for (int k = 0; k < d; ++k) size *= static_cast<double>((s >> k) & 1 ? n[k] : m[k]);
    for (int k = 0; k < d; ++k) {
      if (!((target >> k) & 1) || ((s >> k) & 1)) continue;
      const double c = 2.0 * static_cast<double>(n[k]) * size + best[s | (1 << k)];
      if (c < best[s] * (1.0 - 1e-12)) {
        best[s] = c;
        choice[s] = k;
      }
    }
  }
  int s = 0, c = 0;
  while (s != target) {
    order[c++] = choice[s];
    s |= 1 << choice[s];
  }
  *count = c;
}

struct ChainPlan {
  int count;
  int order[KP_MAX_ORDER];       // mode index (0-based) of each step
  int64_t dims[KP_MAX_ORDER + 1][KP_MAX_ORDER];  // dims before step s (and after last)
  int64_t size[KP_MAX_ORDER + 1];                // entries before step s
};

void make_chain(const kp_tensor& T, const kp_matrix* const* L, bool definition_order,
                ChainPlan* p) {
  const int d = T.d;
  int64_t m[KP_MAX_ORDER], n[KP_MAX_ORDER];
  bool active[KP_MAX_ORDER];
  for (int k = 0; k < d; ++k) {
    m[k] = T.dims[k];
    active[k] = L[k] != nullptr;
    n[k] = L[k] ? L[k]->rows : m[k];
  }
  if (definition_order) {
    p->count = 0;
    for (int k = 0; k < d; ++k)
      if (active[k]) p->order[p->count++] = k;
  } else {
    plan_order(m, n, active, d, p->order, &p->count);
    // FP32 data whose two leading modes fit a fused pair (m <= 16, n <= 32)
    // and grow the tensor: when it costs no more flops, those modes go last,
    // so that the pass writing the final (largest) tensor is the lead-layout
    // pair, which reads and writes each fiber as one contiguous block. The
    // order does not depend on whether fusion is enabled.
    if (T.dtype == KP_F32 && d > 2 && active[0] && active[1] && n[0] * n[1] > m[0] * m[1] &&
        pair_eligible(FORM_F32, 1, m[0], m[1], n[0], n[1])) {
      auto flops = [&](const int* ord, int cnt) {
        double size = 1.0, f = 0.0;
        for (int k = 0; k < d; ++k) size *= static_cast<double>(m[k]);
        for (int s = 0; s < cnt; ++s) {
          const int k = ord[s];
          f += 2.0 * static_cast<double>(n[k]) * size;
          size = size / static_cast<double>(m[k]) * static_cast<double>(n[k]);
        }
        return f;
      };
      bool rest[KP_MAX_ORDER];
      for (int k = 0; k < d; ++k) rest[k] = active[k] && k > 1;
      int alt[KP_MAX_ORDER], cnt = 0;
      plan_order(m, n, rest, d, alt, &cnt);
      alt[cnt++] = 0;
      alt[cnt++] = 1;
      if (flops(alt, cnt) <= flops(p->order, p->count) * (1.0 + 1e-12))
        for (int s = 0; s < cnt; ++s) p->order[s] = alt[s];
    }
  }
  int64_t cur[KP_MAX_ORDER];
  for (int k = 0; k < d; ++k) cur[k] = m[k];
  for (int s = 0; s <= p->count; ++s) {
    int64_t e = 1;
    for (int k = 0; k < d; ++k) {
      p->dims[s][k] = cur[k];
      e *= cur[k];
    }
    p->size[s] = e;
    if (s < p->count) cur[p->order[s]] = n[p->order[s]];
  }
}

// Workspace for a chain: two ping-pong buffers, each holding the largest
// intermediate (a fused pass skips a step, so either buffer may receive any
// intermediate); a launch always writes the buffer its input is not in.
void chain_ws(const ChainPlan& p, size_t esize, size_t* off1, size_t* total) {
  size_t big = 0;
  for (int s = 1; s < p.count; ++s) {
    const size_t bytes = static_cast<size_t>(p.size[s]) * esize;
    if (bytes > big) big = bytes;
  }
  *off1 = align_up(big);
  // one intermediate needs one buffer (the first launch writes buffer 0)
  *total = (p.count > 2 ? 2 : (p.count > 1 ? 1 : 0)) * align_up(big);
}

// Bytes of the pre-split factor planes a chain may use (the BF16 split
// forms: one plane set per non-identity factor, whichever tile its product
// runs on), placed after the chain's intermediates.
size_t chain_planes_bytes(const ChainPlan& p, const kp_matrix* const* L, int form) {
  if (form != FORM_BF16X3 && form != FORM_BF16X6) return 0;
  size_t total = 0;
  for (int s = 0; s < p.count; ++s) {
    const kp_matrix& f = *L[p.order[s]];
    total += align_up(split_planes_bytes(form, f.rows, f.cols));
  }
  return total;
}

// Whether steps s and s + 1 of a chain without a cache run as one fused pass
// (modes k and k + 1 in that order, both short; the strided pair for
// I_l > 1, the lead-layout pair for I_l = 1); fills the pass's arguments
// except the tensors.
bool fuse_step(const ChainPlan& p, int s, int d, const kp_matrix* const* L, int form,
               tile::PairArgs* pa) {
  if (!fusion_enabled() || tile_override() || s + 1 >= p.count) return false;
  const int k = p.order[s];
  if (p.order[s + 1] != k + 1) return false;
  const kp_matrix& L1 = *L[k];
  const kp_matrix& L2 = *L[k + 1];
  int64_t Il = 1, Ir = 1;
  for (int j = 0; j < k; ++j) Il *= p.dims[s][j];
  for (int j = k + 2; j < d; ++j) Ir *= p.dims[s][j];
  if (!pair_eligible(form, Il, L1.cols, L2.cols, L1.rows, L2.rows)) return false;
  pa->L1 = L1.data;
  pa->L2 = L2.data;
  pa->Il = Il;
  pa->m1 = L1.cols;
  pa->m2 = L2.cols;
  pa->n1 = L1.rows;
  pa->n2 = L2.rows;
  pa->Ir = Ir;
  pa->rs1 = L1.rs;
  pa->cs1 = L1.cs;
  pa->rs2 = L2.rs;
  pa->cs2 = L2.cs;
  return true;
}

// Which steps of a chain without a cache start a fused pass (fused[s]: steps
// s and s + 1 in one launch). Among the eligible pairs (fuse_step), the
// non-overlapping set that moves the fewest tensor elements through HBM: an
// unfused step reads its input and writes its output, a fused pair skips the
// intermediate between its two steps. Ties keep the plan with more fused
// passes, then the earlier ones.
void plan_fusion(const ChainPlan& p, int d, const kp_matrix* const* L, int form, bool* fused) {
  int64_t best[KP_MAX_ORDER + 2];
  bool pick[KP_MAX_ORDER + 1];
  best[p.count] = 0;
  best[p.count + 1] = 0;
  for (int s = p.count - 1; s >= 0; --s) {
    fused[s] = false;
    pick[s] = false;
    best[s] = p.size[s] + p.size[s + 1] + best[s + 1];
    tile::PairArgs pa;
    if (s + 1 < p.count && fuse_step(p, s, d, L, form, &pa)) {
      const int64_t c = p.size[s] + p.size[s + 2] + best[s + 2];
      if (c <= best[s]) {
        best[s] = c;
        pick[s] = true;
      }
    }
  }
  for (int s = 0; s < p.count;) {
    if (pick[s]) {
      fused[s] = true;
      s += 2;
    } else {
      ++s;
    }
  }
}

int validate_tucker_args(const kp_tensor* T, const kp_matrix* const* L, int prec) {
  int st = check_tensor(T, true);
  if (st) return st;
  if (!L) return KP_ERR_NULL;
  for (int k = 0; k < T->d; ++k) {
    if (!L[k]) continue;
    st = check_matrix(L[k], T->dtype);
    if (st) return st;
    if (L[k]->cols != T->dims[k]) return KP_ERR_SHAPE;
  }
  return check_prec(prec, T->dtype);
}

size_t cache_bytes_for(const kp_tensor& T, const kp_matrix* const* L) {
  ChainPlan p;
  make_chain(T, L, true, &p);
  size_t total = 0;
  for (int s = 1; s < p.count; ++s) total += align_up(static_cast<size_t>(p.size[s]) * elem_size(T.dtype));
  return total;
}

// Layout of the backward workspace: [P recompute region][Q ping][Q pong][gram partials]
struct BackwardLayout {
  size_t p_off, p_bytes;
  size_t q_off[2], q_bytes[2];
  size_t g_off, g_bytes;
  size_t total;
};

void backward_layout(const kp_tensor& T, const kp_matrix* const* L, bool need_p,
                     BackwardLayout* b) {
  const int d = T.d;
  const size_t es = elem_size(T.dtype);
  int64_t m[KP_MAX_ORDER], n[KP_MAX_ORDER];
  for (int k = 0; k < d; ++k) {
    m[k] = T.dims[k];
    n[k] = L[k]->rows;
  }
  b->p_bytes = need_p ? cache_bytes_for(T, L) : 0;
  // Q_mu (mu = d-1 .. 1) has dims n_1..n_mu, m_{mu+1}..m_d; Q_mu goes to
  // buffer (d - 1 - mu) & 1.
  b->q_bytes[0] = b->q_bytes[1] = 0;
  for (int mu = d - 1; mu >= 1; --mu) {
    int64_t e = 1;
    for (int k = 0; k < d; ++k) e *= (k < mu) ? n[k] : m[k];
    const size_t bytes = static_cast<size_t>(e) * es;
    size_t& slot = b->q_bytes[(d - 1 - mu) & 1];
    if (bytes > slot) slot = bytes;
  }
  b->g_bytes = 0;
  for (int mu = 1; mu <= d; ++mu) {
    int64_t Il = 1, Ir = 1;
    for (int k = 0; k < mu - 1; ++k) Il *= n[k];
    for (int k = mu; k < d; ++k) Ir *= m[k];
    const size_t g = gram_workspace(Il, n[mu - 1], m[mu - 1], Ir, es);
    if (g > b->g_bytes) b->g_bytes = g;
  }
  b->p_off = 0;
  b->q_off[0] = align_up(b->p_bytes);
  b->q_off[1] = b->q_off[0] + align_up(b->q_bytes[0]);
  b->g_off = b->q_off[1] + align_up(b->q_bytes[1]);
  b->total = b->g_off + align_up(b->g_bytes);
}

}  // namespace kp

using namespace kp;

extern "C" {

int kp_version(void) { return KP_VERSION; }
int kp_last_hip_error(void) { return g_last_hip_error; }

const char* kp_strerror(int status) {
  switch (status) {
    case KP_OK: return "ok";
    case KP_ERR_NULL: return "required pointer is NULL";
    case KP_ERR_ORDER: return "tensor order outside 1..KP_MAX_ORDER";
    case KP_ERR_MODE: return "mode outside 1..d";
    case KP_ERR_SHAPE: return "sizes do not match";
    case KP_ERR_DTYPE: return "unsupported dtype / precision combination";
    case KP_ERR_ALIAS: return "output overlaps an input";
    case KP_ERR_WORKSPACE: return "workspace missing or too small";
    case KP_ERR_HIP: return "HIP launch failed";
    case KP_ERR_VALUE: return "scalar argument out of range";
    case KP_ERR_SCRATCH: return "intermediates exceed the library's fixed scratch buffer";
    default: return "unknown status";
  }
}

int kp_mump(const kp_tensor* T, const kp_matrix* L, int mu, kp_tensor* S, int prec,
            int accumulate, hipStream_t stream) {
  int st = check_tensor(T, true);
  if (st) return st;
  if (!L || !S) return KP_ERR_NULL;
  if (mu < 1 || mu > T->d) return KP_ERR_MODE;
  st = check_matrix(L, T->dtype);
  if (st) return st;
  st = check_tensor(S, true);
  if (st) return st;
  if (S->dtype != T->dtype) return KP_ERR_DTYPE;
  st = check_prec(prec, T->dtype);
  if (st) return st;
  if (L->cols != T->dims[mu - 1] || S->d != T->d) return KP_ERR_SHAPE;
  for (int k = 0; k < T->d; ++k) {
    const int64_t want = (k == mu - 1) ? L->rows : T->dims[k];
    if (S->dims[k] != want) return KP_ERR_SHAPE;
  }
  const size_t es = elem_size(T->dtype);
  const size_t sb = static_cast<size_t>(numel(*S)) * es;
  if (overlaps(S->data, sb, T->data, static_cast<size_t>(numel(*T)) * es) ||
      overlaps(S->data, sb, L->data, matrix_span_bytes(*L)))
    return KP_ERR_ALIAS;
  if (numel(*S) == 0) return KP_OK;
  const ModeArgs a =
      mode_args(T->data, S->data, T->dims, T->d, mu - 1, *L, accumulate ? kAccAdd : kAccNone);
  return hip_status(launch_mode(form_of(prec, T->dtype), a, tile_override(), stream));
}

int kp_kronsum(const kp_tensor* T, const kp_matrix* const* A, kp_tensor* S, int prec,
               hipStream_t stream) {
  int st = check_tensor(T, true);
  if (st) return st;
  if (!A || !S) return KP_ERR_NULL;
  st = check_tensor(S, true);
  if (st) return st;
  const int d = T->d;
  for (int k = 0; k < d; ++k) {
    if (!A[k]) return KP_ERR_NULL;
    st = check_matrix(A[k], T->dtype);
    if (st) return st;
    if (A[k]->rows != T->dims[k] || A[k]->cols != T->dims[k]) return KP_ERR_SHAPE;
  }
  st = check_prec(prec, T->dtype);
  if (st) return st;
  if (S->dtype != T->dtype) return KP_ERR_DTYPE;
  if (S->d != d) return KP_ERR_SHAPE;
  for (int k = 0; k < d; ++k)
    if (S->dims[k] != T->dims[k]) return KP_ERR_SHAPE;
  const size_t es = elem_size(T->dtype);
  const size_t sb = static_cast<size_t>(numel(*S)) * es;
  if (overlaps(S->data, sb, T->data, sb)) return KP_ERR_ALIAS;
  for (int k = 0; k < d; ++k)
    if (overlaps(S->data, sb, A[k]->data, matrix_span_bytes(*A[k]))) return KP_ERR_ALIAS;
  if (numel(*S) == 0) return KP_OK;
  const int form = form_of(prec, T->dtype);
  for (int k = 0; k < d; ++k) {
    const ModeArgs a = mode_args(T->data, S->data, T->dims, d, k, *A[k], k > 0 ? 1 : 0);
    st = hip_status(launch_mode(form, a, tile_override(), stream));
    if (st) return st;
  }
  return KP_OK;
}

size_t kp_tucker_workspace(const kp_tensor* T, const kp_matrix* const* L, int prec) {
  if (validate_tucker_args(T, L, prec)) return 0;
  // the intermediates (what kp_tucker requires on its workspace path, no
  // cache) and, for the BF16 split forms, the factors' pre-split planes
  // (used when the workspace has room for them)
  ChainPlan p;
  make_chain(*T, L, false, &p);
  size_t off1, total;
  chain_ws(p, elem_size(T->dtype), &off1, &total);
  return total + chain_planes_bytes(p, L, form_of(prec, T->dtype));
}

int kp_tucker_order(const kp_tensor* T, const kp_matrix* const* L, int* order, int* count) {
  const int st = validate_tucker_args(T, L, KP_PREC_NATIVE);
  if (st) return st;
  if (!order || !count) return KP_ERR_NULL;
  ChainPlan p;
  make_chain(*T, L, false, &p);
  for (int s = 0; s < p.count; ++s) order[s] = p.order[s] + 1;
  *count = p.count;
  return KP_OK;
}

size_t kp_tucker_cache_size(const kp_tensor* T, const kp_matrix* const* L) {
  if (validate_tucker_args(T, L, KP_PREC_NATIVE)) return 0;
  return cache_bytes_for(*T, L);
}

int kp_tucker(const kp_tensor* T, const kp_matrix* const* L, kp_tensor* S, int prec, void* ws,
              size_t ws_bytes, void* cache, size_t cache_bytes, hipStream_t stream) {
  int st = validate_tucker_args(T, L, prec);
  if (st) return st;
  if (!S) return KP_ERR_NULL;
  st = check_tensor(S, true);
  if (st) return st;
  if (S->dtype != T->dtype) return KP_ERR_DTYPE;
  if (S->d != T->d) return KP_ERR_SHAPE;
  for (int k = 0; k < T->d; ++k)
    if (S->dims[k] != (L[k] ? L[k]->rows : T->dims[k])) return KP_ERR_SHAPE;
  const size_t es = elem_size(T->dtype);
  const size_t sb = static_cast<size_t>(numel(*S)) * es;
  if (overlaps(S->data, sb, T->data, static_cast<size_t>(numel(*T)) * es)) return KP_ERR_ALIAS;
  for (int k = 0; k < T->d; ++k)
    if (L[k] && overlaps(S->data, sb, L[k]->data, matrix_span_bytes(*L[k]))) return KP_ERR_ALIAS;

  ChainPlan p;
  make_chain(*T, L, cache != nullptr, &p);
  const size_t need_cache = cache ? cache_bytes_for(*T, L) : 0;
  if (cache && cache_bytes < need_cache) return KP_ERR_WORKSPACE;
  size_t off1 = 0, need = 0;
  const int form = form_of(prec, T->dtype);
  // pre-split factor planes after the intermediates, when the workspace has
  // room for them (kp_tucker_workspace counts them; a smaller workspace that
  // holds the intermediates runs the products with in-register splits)
  size_t planes_at = 0, planes_need = 0;
  if (!cache) {
    chain_ws(p, es, &off1, &need);
    if (need > 0 && (!ws || ws_bytes < need)) return KP_ERR_WORKSPACE;
    const size_t pb = chain_planes_bytes(p, L, form);
    if (pb > 0 && ws && ws_bytes >= align_up(need) + pb) {
      planes_at = align_up(need);
      planes_need = pb;
      need = planes_at + pb;
    }
  }
  // Buffers the chain writes (the used part of ws, the cache) must not
  // overlap anything it reads or writes elsewhere.
  const size_t Tb = static_cast<size_t>(numel(*T)) * es;
  auto hits_inputs = [&](const void* buf, size_t bytes) {
    if (overlaps(buf, bytes, T->data, Tb) || overlaps(buf, bytes, S->data, sb)) return true;
    for (int k = 0; k < T->d; ++k)
      if (L[k] && overlaps(buf, bytes, L[k]->data, matrix_span_bytes(*L[k]))) return true;
    return false;
  };
  if (need > 0 && hits_inputs(ws, need)) return KP_ERR_ALIAS;
  if (need_cache > 0 &&
      (hits_inputs(cache, need_cache) || overlaps(cache, need_cache, ws, ws ? ws_bytes : 0)))
    return KP_ERR_ALIAS;
  if (numel(*S) == 0) return KP_OK;
  if (p.count == 0) {
    // every factor is the identity: S = T
    return hip_status(hipMemcpyAsync(S->data, T->data, sb, hipMemcpyDeviceToDevice, stream));
  }
  const void* src = T->data;
  size_t cache_off = 0;
  int cur = -1;  // ping-pong buffer holding src (-1: src is T or a cache slot)
  // the launch that ends at step s writes S (last step), its cache slot, or
  // the ping-pong buffer that does not hold its input
  auto dst_of = [&](int s) -> void* {
    if (s == p.count - 1) return S->data;
    if (cache) return static_cast<char*>(cache) + cache_off;
    cur = cur == 0 ? 1 : 0;
    return static_cast<char*>(ws) + (cur ? off1 : 0);
  };
  // steps s and s + 1 on modes k and k + 1 run as one fused pass where the
  // fusion plan says so (never with a cache, which must hold every partial)
  bool fused[KP_MAX_ORDER] = {};
  if (!cache) plan_fusion(p, T->d, L, form, fused);
  // products on wide tiles read their factor's planes, split by one launch
  // before the chain
  const void* planes[KP_MAX_ORDER] = {};
  if (planes_need > 0) {
    // the steps that run as single products (as the loop below pairs them)
    bool single[KP_MAX_ORDER] = {};
    for (int s = 0; s < p.count; ++s) {
      tile::PairArgs probe;
      if (fused[s] && fuse_step(p, s, T->d, L, form, &probe)) {
        ++s;
        continue;
      }
      single[s] = true;
    }
    SplitJobs jobs{};
    size_t at = planes_at;
    for (int s = 0; s < p.count; ++s) {
      const int k = p.order[s];
      void* dst = static_cast<char*>(ws) + at;
      at += align_up(split_planes_bytes(form, L[k]->rows, L[k]->cols));
      if (!single[s]) continue;
      const ModeArgs a = mode_args(nullptr, nullptr, p.dims[s], T->d, k, *L[k], 0);
      if (!mode_uses_wide(form, a, tile_override())) continue;
      SplitJob& J = jobs.job[jobs.count++];
      J.L = L[k]->data;
      J.n = L[k]->rows;
      J.m = L[k]->cols;
      J.rs = L[k]->rs;
      J.cs = L[k]->cs;
      J.planes = dst;
      J.begin = jobs.total;
      jobs.total += split_planes_tasks(J.n, J.m);
      planes[s] = dst;
    }
    st = hip_status(launch_split_planes(form, jobs, stream));
    if (st) return st;
  }
  for (int s = 0; s < p.count; ++s) {
    const int k = p.order[s];
    tile::PairArgs pa;
    if (fused[s] && fuse_step(p, s, T->d, L, form, &pa)) {
      pa.X = src;
      pa.Y = dst_of(s + 1);
      st = hip_status(launch_pair(form, pa, stream));
      if (st) return st;
      src = pa.Y;
      ++s;
      continue;
    }
    void* dst = dst_of(s);
    if (cache && s < p.count - 1) cache_off += align_up(static_cast<size_t>(p.size[s + 1]) * es);
    const ModeArgs a = mode_args(src, dst, p.dims[s], T->d, k, *L[k], 0);
    st = hip_status(launch_mode_planes(form, a, tile_override(), planes[s], stream));
    if (st) return st;
    src = dst;
  }
  return KP_OK;
}

size_t kp_tucker_backward_workspace(const kp_tensor* T, const kp_matrix* const* L, int prec) {
  if (validate_tucker_args(T, L, prec)) return 0;
  for (int k = 0; k < T->d; ++k)
    if (!L[k]) return 0;
  BackwardLayout b;
  backward_layout(*T, L, true, &b);
  return b.total;
}

int kp_tucker_backward(const kp_tensor* G, const kp_tensor* T, const kp_matrix* const* L,
                       const void* cache, size_t cache_bytes, kp_tensor* dT,
                       kp_matrix* const* dL, int prec, void* ws, size_t ws_bytes,
                       hipStream_t stream) {
  int st = validate_tucker_args(T, L, prec);
  if (st) return st;
  const int d = T->d;
  for (int k = 0; k < d; ++k)
    if (!L[k]) return KP_ERR_NULL;
  st = check_tensor(G, true);
  if (st) return st;
  if (G->dtype != T->dtype) return KP_ERR_DTYPE;
  if (G->d != d) return KP_ERR_SHAPE;
  for (int k = 0; k < d; ++k)
    if (G->dims[k] != L[k]->rows) return KP_ERR_SHAPE;
  const size_t es = elem_size(T->dtype);
  if (dT) {
    st = check_tensor(dT, true);
    if (st) return st;
    if (dT->dtype != T->dtype) return KP_ERR_DTYPE;
    if (dT->d != d) return KP_ERR_SHAPE;
    for (int k = 0; k < d; ++k)
      if (dT->dims[k] != T->dims[k]) return KP_ERR_SHAPE;
  }
  bool want_dl = false;
  if (dL) {
    for (int k = 0; k < d; ++k) {
      if (!dL[k]) continue;
      want_dl = true;
      st = check_matrix(dL[k], T->dtype);
      if (st) return st;
      if (dL[k]->rows != L[k]->rows || dL[k]->cols != L[k]->cols) return KP_ERR_SHAPE;
    }
  }
  const size_t need_cache = cache_bytes_for(*T, L);
  const bool have_cache = cache != nullptr;
  if (have_cache && cache_bytes < need_cache) return KP_ERR_WORKSPACE;
  BackwardLayout b;
  backward_layout(*T, L, !have_cache && want_dl, &b);
  if (b.total > 0 && (!ws || ws_bytes < b.total)) return KP_ERR_WORKSPACE;
  // outputs must not overlap inputs or the workspace
  const size_t Tb = static_cast<size_t>(numel(*T)) * es;
  const size_t Gb = static_cast<size_t>(numel(*G)) * es;
  if (dT) {
    const size_t db = static_cast<size_t>(numel(*dT)) * es;
    if (overlaps(dT->data, db, T->data, Tb) || overlaps(dT->data, db, G->data, Gb) ||
        overlaps(dT->data, db, ws, b.total) || overlaps(dT->data, db, cache, need_cache))
      return KP_ERR_ALIAS;
    for (int k = 0; k < d; ++k)
      if (overlaps(dT->data, db, L[k]->data, matrix_span_bytes(*L[k]))) return KP_ERR_ALIAS;
  }
  if (dL) {
    for (int k = 0; k < d; ++k) {
      if (!dL[k]) continue;
      const size_t lb = matrix_span_bytes(*dL[k]);
      if (overlaps(dL[k]->data, lb, T->data, Tb) || overlaps(dL[k]->data, lb, G->data, Gb) ||
          overlaps(dL[k]->data, lb, ws, b.total) ||
          overlaps(dL[k]->data, lb, cache, have_cache ? need_cache : 0))
        return KP_ERR_ALIAS;
      if (dT && overlaps(dL[k]->data, lb, dT->data, static_cast<size_t>(numel(*dT)) * es))
        return KP_ERR_ALIAS;
      for (int j = 0; j < d; ++j) {
        if (overlaps(dL[k]->data, lb, L[j]->data, matrix_span_bytes(*L[j]))) return KP_ERR_ALIAS;
        if (j != k && dL[j] && overlaps(dL[k]->data, lb, dL[j]->data, matrix_span_bytes(*dL[j])))
          return KP_ERR_ALIAS;
      }
    }
  }
  // the workspace is written: it must not overlap an input or the cache
  if (b.total > 0) {
    if (overlaps(ws, b.total, T->data, Tb) || overlaps(ws, b.total, G->data, Gb) ||
        overlaps(ws, b.total, cache, have_cache ? need_cache : 0))
      return KP_ERR_ALIAS;
    for (int k = 0; k < d; ++k)
      if (overlaps(ws, b.total, L[k]->data, matrix_span_bytes(*L[k]))) return KP_ERR_ALIAS;
  }
  const int form = form_of(prec, T->dtype);
  char* wsb = static_cast<char*>(ws);

  // Forward partials P_1..P_{d-1} (definition order), packed like the cache.
  const void* Pk[KP_MAX_ORDER];
  Pk[0] = T->data;
  ChainPlan chain;
  make_chain(*T, L, true, &chain);
  if (want_dl && d > 1) {
    const char* base = have_cache ? static_cast<const char*>(cache) : wsb + b.p_off;
    size_t off = 0;
    for (int k = 1; k < d; ++k) {
      Pk[k] = base + off;
      off += align_up(static_cast<size_t>(chain.size[k]) * es);
    }
    if (!have_cache) {
      for (int k = 1; k < d; ++k) {
        const ModeArgs a = mode_args(Pk[k - 1], const_cast<void*>(Pk[k]), chain.dims[k - 1], d,
                                     k - 1, *L[k - 1], 0);
        st = hip_status(launch_mode(form, a, tile_override(), stream));
        if (st) return st;
      }
    }
  }

  // Reverse sweep: Q_d = G, Q_{mu-1} = Q_mu x_mu L_mu^T.
  int last_needed = 1;  // smallest mu whose Q_mu is needed
  if (!dT) {
    last_needed = d + 1;
    for (int k = 0; k < d; ++k)
      if (dL && dL[k] && k + 1 < last_needed) last_needed = k + 1;
  }
  const void* Qmu = G->data;
  int64_t qdims[KP_MAX_ORDER];  // dims of Q_mu
  for (int k = 0; k < d; ++k) qdims[k] = L[k]->rows;
  for (int mu = d; mu >= 1 && mu >= last_needed; --mu) {
    const int k = mu - 1;
    int64_t Il = 1, Ir = 1;
    for (int j = 0; j < k; ++j) Il *= qdims[j];
    for (int j = k + 1; j < d; ++j) Ir *= qdims[j];
    const bool sweep = (mu > last_needed || (mu == 1 && dT)) && !(mu == 1 && !dT);
    void* dst = sweep ? ((mu == 1) ? dT->data : wsb + b.q_off[(d - mu) & 1]) : nullptr;
    // FP32 data with both the factor gradient and the next cotangent needed,
    // on a short mode: one pass over Q_mu computes both
    if (dL && dL[k] && sweep && form != FORM_F64 && fusion_enabled() && !tile_override() &&
        gram_product_eligible(T->dtype, Qmu, Pk[k], dst, Il, L[k]->rows, L[k]->cols, Ir)) {
      st = hip_status(launch_gram_product(form, Qmu, Pk[k], Il, L[k]->rows, L[k]->cols, Ir,
                                          wsb + b.g_off, dL[k]->data, dL[k]->rs, dL[k]->cs,
                                          *L[k], dst, stream));
      if (st) return st;
      Qmu = dst;
      qdims[k] = L[k]->cols;
      continue;
    }
    if (dL && dL[k]) {
      st = hip_status(launch_gram(T->dtype, Qmu, Pk[k], Il, L[k]->rows, L[k]->cols, Ir,
                                  wsb + b.g_off, dL[k]->data, dL[k]->rs, dL[k]->cs, stream));
      if (st) return st;
    }
    if (mu == 1 && !dT) break;
    if (sweep) {
      kp_matrix Lt = *L[k];
      Lt.rows = L[k]->cols;
      Lt.cols = L[k]->rows;
      Lt.rs = L[k]->cs;
      Lt.cs = L[k]->rs;
      const ModeArgs a = mode_args(Qmu, dst, qdims, d, k, Lt, 0);
      st = hip_status(launch_mode(form, a, tile_override(), stream));
      if (st) return st;
      Qmu = dst;
      qdims[k] = L[k]->cols;
    }
  }
  return KP_OK;
}

int kp_tucker_products(const kp_tensor* T, const kp_matrix* const* L, int prec, int which,
                       kp_tune_entry* out, int cap) {
  int st = validate_tucker_args(T, L, prec);
  if (st) return st;
  if (which < 0 || which > 3) return KP_ERR_VALUE;
  if (cap > 0 && !out) return KP_ERR_NULL;
  const int d = T->d;
  if (which == 2)
    for (int k = 0; k < d; ++k)
      if (!L[k]) return KP_ERR_NULL;
  const int form = form_of(prec, T->dtype);
  int count = 0;
  auto emit = [&](const ModeArgs& a) {
    if (count < cap) {
      const ModeTile t = default_mode_tile(form, a);
      ModeTile r;
      if (!resolve_mode_tile(form, t, &r)) r = t;
      kp_tune_entry& e = out[count];
      e.form = form;
      e.pad0_ = 0;
      e.Il = a.Il;
      e.m = a.m;
      e.n = a.n;
      e.Ir = a.Ir;
      e.nb = r.nb;
      e.fb = r.fb;
      e.bk = r.bk;
      e.occ = r.occ;
      e.pf = r.pf;
      e.kind = r.kind;
    }
    ++count;
  };
  if (which < 2 || which == 3) {
    ChainPlan p;
    make_chain(*T, L, which == 1, &p);
    bool fused[KP_MAX_ORDER] = {};
    if (which == 3) plan_fusion(p, d, L, form, fused);
    for (int s = 0; s < p.count; ++s) {
      const int k = p.order[s];
      const ModeArgs a = mode_args(nullptr, nullptr, p.dims[s], d, k, *L[k], 0);
      tile::PairArgs pa;
      if (fused[s] && fuse_step(p, s, d, L, form, &pa)) {
        if (count < cap) {
          kp_tune_entry& e = out[count];
          memset(&e, 0, sizeof(e));
          e.form = form;
          e.Il = a.Il;
          e.m = a.m;
          e.n = a.n;
          e.Ir = a.Ir;
          e.kind = 2;
        }
        ++count;
        ++s;
        continue;
      }
      emit(a);
    }
  } else {
    int64_t qdims[KP_MAX_ORDER];
    for (int k = 0; k < d; ++k) qdims[k] = L[k]->rows;
    for (int k = d - 1; k >= 0; --k) {
      kp_matrix Lt = *L[k];
      Lt.rows = L[k]->cols;
      Lt.cols = L[k]->rows;
      Lt.rs = L[k]->cs;
      Lt.cs = L[k]->rs;
      emit(mode_args(nullptr, nullptr, qdims, d, k, Lt, 0));
      qdims[k] = L[k]->cols;
    }
  }
  return count;
}

}  // extern "C"
