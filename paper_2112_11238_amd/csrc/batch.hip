// Batched Tucker operator: many independent problems (uneven sizes), forward
// and optionally backward, in a few persistent launches.
//
// Every mu-mode product, factor-gradient partial sum and partial-sum
// reduction of every problem is a "stage" made of independent tiles. A
// stage's level is one more than the deepest level among the stages it
// depends on (the forward product of mode s depends on mode s-1, a factor
// gradient on the forward partial and on the reverse sweep, ...). All stages
// of one level, across all problems, run in ONE persistent launch whose
// workgroups stride over the level's tiles; the next level is the next launch
// on the same stream, so kernel boundaries order the dependencies and no
// workgroup ever waits for another. A forward pass of order-d problems takes
// d launches; with the backward about 2d + 2. Capturing kp_tucker_batched in
// a HIP graph turns the whole batch into one graph of that many nodes.
#include "kp.h"

#include <string.h>

#include <algorithm>
#include <vector>

#include "gram_tile.h"
#include "kp_common.h"
#include "kp_internal.h"
#include "mode_tile.h"

namespace kp {
namespace {

constexpr int kThreads = 256;
constexpr uint64_t kMagic = 0x6b70626174636802ULL;  // "kpbatch" v2
constexpr int kGramBR = 32;

enum StageKind { ST_MODE = 0, ST_GRAM = 1, ST_REDUCE = 2 };

struct BStage {
  int32_t kind;
  int32_t variant;        // mode: batch variant id; gram: 1 = inner layout
  int32_t tx, ty, tz;     // tile grid; tiles = tx * ty * tz
  int32_t dep0, dep1;     // stages that must be complete (-1: none)
  int32_t problem;
  int64_t begin;          // first global task number of this stage
  ModeArgs m;             // ST_MODE
  gram::GramArgs g;       // ST_GRAM (and n, m, part for ST_REDUCE)
  int64_t splits;         // ST_REDUCE
  void* dL;               // ST_REDUCE output
  int64_t rs, cs;
};

// Plan layout: [BHeader][BStage x nstages][int64 level_begin x (nlevels + 1)]
// level_begin[l] is the first task number of level l.
struct BHeader {
  uint64_t magic;
  int32_t nstages;
  int32_t form;
  int64_t ntasks;
  int32_t nlevels;
  int32_t pad_;
  const void* ws_base;
  size_t ws_bytes;
};

// Tile variants available to the executor, per form: (nb, fb, bk).
struct BVar {
  int nb, fb, bk;
};
constexpr BVar kBVarF64[] = {{1, 4, 16}, {2, 2, 16}, {4, 1, 16}, {7, 1, 16}, {8, 1, 16}};
constexpr BVar kBVarF32[] = {{1, 4, 16}, {2, 2, 16}, {4, 1, 16}, {8, 1, 16}, {2, 4, 16},
                             {4, 2, 16}};
constexpr BVar kBVarB16[] = {{1, 2, 32}, {2, 2, 32}, {4, 1, 32}, {2, 1, 32}};

template <int FORM>
struct BVars;
template <>
struct BVars<FORM_F64> {
  static constexpr const BVar* v = kBVarF64;
  static constexpr int n = 5;
};
template <>
struct BVars<FORM_F32> {
  static constexpr const BVar* v = kBVarF32;
  static constexpr int n = 6;
};
template <>
struct BVars<FORM_BF16X3> {
  static constexpr const BVar* v = kBVarB16;
  static constexpr int n = 4;
};
template <>
struct BVars<FORM_BF16X6> {
  static constexpr const BVar* v = kBVarB16;
  static constexpr int n = 4;
};

const BVar* host_vars(int form, int* count) {
  switch (form) {
    case FORM_F64: *count = 5; return kBVarF64;
    case FORM_F32: *count = 6; return kBVarF32;
    default: *count = 4; return kBVarB16;
  }
}

template <int FORM, int I>
constexpr size_t max_mode_lds() {
  if constexpr (I == BVars<FORM>::n) {
    return 0;
  } else {
    constexpr BVar b = BVars<FORM>::v[I];
    constexpr size_t here = tile::mode_lds_bytes<FORM, b.nb, b.fb, b.bk>();
    constexpr size_t rest = max_mode_lds<FORM, I + 1>();
    return here > rest ? here : rest;
  }
}

template <int FORM>
constexpr size_t batch_lds() {
  using E = typename tile::FormT<FORM>::G;
  constexpr size_t a = max_mode_lds<FORM, 0>();
  constexpr size_t b = gram::gram_lds_bytes<E, kGramBR>();
  return a > b ? a : b;
}

// Variant id = 2 * index + inner.
template <int FORM, int I>
__device__ __forceinline__ void run_mode_variant(int id, const ModeArgs& a, int64_t bx,
                                                 int64_t by, char* lds) {
  if constexpr (I < BVars<FORM>::n) {
    constexpr BVar b = BVars<FORM>::v[I];
    if (id == 2 * I) {
      tile::mode_tile<FORM, b.nb, b.fb, b.bk, false>(a, bx, by, lds);
    } else if (id == 2 * I + 1) {
      tile::mode_tile<FORM, b.nb, b.fb, b.bk, true>(a, bx, by, lds);
    } else {
      run_mode_variant<FORM, I + 1>(id, a, bx, by, lds);
    }
  }
}

// Runs the tiles [task_begin, task_end) of one level; workgroup b takes tasks
// task_begin + b, task_begin + b + gridDim.x, ... No task of a level depends
// on another task of the same level.
template <int FORM>
__global__ __launch_bounds__(kThreads) void batch_level_kernel(const BStage* __restrict__ st,
                                                               int nstages, int64_t task_begin,
                                                               int64_t task_end) {
  using E = typename tile::FormT<FORM>::G;
  __shared__ __attribute__((aligned(16))) char lds[batch_lds<FORM>()];
  const int t = threadIdx.x;
  for (int64_t task = task_begin + blockIdx.x; task < task_end; task += gridDim.x) {
    // stage of this task: the last stage whose begin <= task
    int lo = 0, hi = nstages - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (st[mid].begin <= task)
        lo = mid;
      else
        hi = mid - 1;
    }
    const BStage& S = st[lo];
    const int64_t tile_id = task - S.begin;
    __syncthreads();  // the previous tile's LDS reads are complete
    if (S.kind == ST_MODE) {
      const int64_t bx = tile_id % S.tx;
      const int64_t by = tile_id / S.tx;
      run_mode_variant<FORM, 0>(S.variant, S.m, bx, by, lds);
    } else if (S.kind == ST_GRAM) {
      const int64_t bx = tile_id % S.tx;
      const int64_t by = (tile_id / S.tx) % S.ty;
      const int64_t bz = tile_id / (static_cast<int64_t>(S.tx) * S.ty);
      if (S.variant)
        gram::gram_tile<E, kGramBR, true>(S.g, bx, by, bz, lds);
      else
        gram::gram_tile<E, kGramBR, false>(S.g, bx, by, bz, lds);
    } else {
      const int64_t nm = S.g.n * S.g.m;
      const int64_t idx = tile_id * kThreads + t;
      if (idx < nm) {
        const E* part = static_cast<const E*>(S.g.part);
        E s = E(0);
        for (int64_t k = 0; k < S.splits; ++k) s += part[k * nm + idx];
        const int64_t i = idx / S.g.m, j = idx - (idx / S.g.m) * S.g.m;
        static_cast<E*>(S.dL)[i * S.rs + j * S.cs] = s;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Host planning
// ---------------------------------------------------------------------------

int64_t numel_t(const kp_tensor& t) {
  int64_t s = 1;
  for (int k = 0; k < t.d; ++k) s *= t.dims[k];
  return s;
}

struct Plan {
  std::vector<BStage> stages;
  std::vector<int> level;
  std::vector<int64_t> level_begin;  // after finalize
  size_t ws_total = 0;
};

// Batch variant for a mode product: the tuned / default tile if the executor
// has it, else the executor's variant with the closest n coverage.
int pick_batch_variant(int form, const ModeArgs& a) {
  const ModeTile want = default_mode_tile(form, a);
  int nv;
  const BVar* vs = host_vars(form, &nv);
  int best = 0;
  int64_t best_cost = -1;
  for (int i = 0; i < nv; ++i) {
    if (want.kind == 0 && vs[i].nb == want.nb && vs[i].fb == want.fb && vs[i].bk == want.bk) {
      best = i;
      best_cost = 0;
      break;
    }
    // padding waste of n, then prefer larger fiber tiles for small n
    const int64_t bn = 16 * vs[i].nb;
    const int64_t padded = ((a.n + bn - 1) / bn) * bn;
    const int64_t cost = (padded - a.n) * 8 + (vs[i].nb == want.nb ? 0 : 1);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = i;
    }
  }
  return 2 * best + (a.Il > 1 ? 1 : 0);
}

size_t aligned(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

int check_item(const kp_batch_item& it, int prec, bool* has_bwd) {
  const kp_tensor& T = it.T;
  if (T.d < 1 || T.d > KP_MAX_ORDER) return KP_ERR_ORDER;
  if (T.dtype != KP_F64 && T.dtype != KP_F32) return KP_ERR_DTYPE;
  if (prec != KP_PREC_NATIVE && T.dtype != KP_F32) return KP_ERR_DTYPE;
  if (prec != KP_PREC_NATIVE && prec != KP_PREC_BF16X3 && prec != KP_PREC_BF16X6)
    return KP_ERR_DTYPE;
  const size_t es = elem_size(T.dtype);
  if (!T.data || !it.S.data) return KP_ERR_NULL;
  if (it.S.d != T.d || it.S.dtype != T.dtype) return KP_ERR_SHAPE;
  int64_t big = numel_t(T);
  for (int k = 0; k < T.d; ++k) {
    const kp_matrix& L = it.L[k];
    if (T.dims[k] < 1) return KP_ERR_SHAPE;
    if (!L.data) return KP_ERR_NULL;
    if (L.dtype != T.dtype) return KP_ERR_DTYPE;
    if (L.cols != T.dims[k] || L.rows < 1 || it.S.dims[k] != L.rows) return KP_ERR_SHAPE;
  }
  // every intermediate must fit the 32-bit offsets of the tile code
  int64_t cur = numel_t(T);
  for (int k = 0; k < T.d; ++k) {
    cur = cur / T.dims[k] * it.L[k].rows;
    if (cur > big) big = cur;
  }
  if (static_cast<size_t>(big) * es >= (static_cast<size_t>(1) << 31)) return KP_ERR_SHAPE;
  *has_bwd = it.G.data != nullptr;
  if (*has_bwd) {
    if (it.G.d != T.d || it.G.dtype != T.dtype) return KP_ERR_SHAPE;
    for (int k = 0; k < T.d; ++k)
      if (it.G.dims[k] != it.L[k].rows) return KP_ERR_SHAPE;
    if (it.dT.data) {
      if (it.dT.d != T.d || it.dT.dtype != T.dtype) return KP_ERR_SHAPE;
      for (int k = 0; k < T.d; ++k)
        if (it.dT.dims[k] != T.dims[k]) return KP_ERR_SHAPE;
    }
    for (int k = 0; k < T.d; ++k) {
      const kp_matrix& D = it.dL[k];
      if (!D.data) continue;
      if (D.dtype != T.dtype || D.rows != it.L[k].rows || D.cols != it.L[k].cols)
        return KP_ERR_SHAPE;
    }
  }
  return KP_OK;
}

int64_t batch_gram_splits(int64_t chunks) {
  int64_t s = chunks / 16;
  if (s < 1) s = 1;
  if (s > 4096) s = 4096;
  return s;
}

// Builds the stage list and the workspace layout. With ws_base == nullptr
// only sizes are computed (addresses are offsets from 0).
int build_plan(int count, const kp_batch_item* items, int prec, char* ws_base, Plan* pl) {
  if (count < 0) return KP_ERR_VALUE;
  if (count > 0 && !items) return KP_ERR_NULL;
  int dtype = -1;
  for (int q = 0; q < count; ++q) {
    bool hb;
    const int st = check_item(items[q], prec, &hb);
    if (st) return st;
    if (dtype >= 0 && items[q].T.dtype != dtype) return KP_ERR_DTYPE;
    dtype = items[q].T.dtype;
  }
  if (dtype < 0) dtype = KP_F32;
  const int form = (prec == KP_PREC_BF16X3) ? FORM_BF16X3
                   : (prec == KP_PREC_BF16X6) ? FORM_BF16X6
                   : (dtype == KP_F64 ? FORM_F64 : FORM_F32);
  const size_t es = elem_size(dtype);
  size_t off = 0;
  std::vector<BStage>& S = pl->stages;
  std::vector<int>& lev = pl->level;
  auto add = [&](const BStage& s, int level) {
    S.push_back(s);
    lev.push_back(level);
    return static_cast<int>(S.size()) - 1;
  };
  auto region = [&](size_t bytes) {
    char* p = ws_base ? ws_base + off : reinterpret_cast<char*>(off);
    off += aligned(bytes);
    return p;
  };
  for (int q = 0; q < count; ++q) {
    const kp_batch_item& it = items[q];
    const int d = it.T.d;
    bool bwd = it.G.data != nullptr;
    int64_t dims[KP_MAX_ORDER + 1][KP_MAX_ORDER];
    int64_t cur[KP_MAX_ORDER];
    for (int k = 0; k < d; ++k) cur[k] = it.T.dims[k];
    const void* P[KP_MAX_ORDER + 1];
    P[0] = it.T.data;
    int fstage[KP_MAX_ORDER + 1];
    int flev[KP_MAX_ORDER + 1];
    fstage[0] = -1;
    flev[0] = -1;
    for (int s = 1; s <= d; ++s) {
      for (int k = 0; k < d; ++k) dims[s - 1][k] = cur[k];
      const kp_matrix& L = it.L[s - 1];
      void* Y;
      if (s == d) {
        Y = it.S.data;
      } else {
        int64_t e = 1;
        for (int k = 0; k < d; ++k) e *= (k == s - 1) ? L.rows : cur[k];
        Y = region(static_cast<size_t>(e) * es);
      }
      BStage b{};
      b.kind = ST_MODE;
      b.m = mode_args(P[s - 1], Y, dims[s - 1], d, s - 1, L, 0);
      b.variant = pick_batch_variant(form, b.m);
      int nv;
      const BVar* vs = host_vars(form, &nv);
      const BVar& bv = vs[b.variant / 2];
      const int64_t F = b.m.Il > 1 ? b.m.Il * b.m.Ir : b.m.Ir;
      b.tx = static_cast<int32_t>((F + 64 * bv.fb - 1) / (64 * bv.fb));
      b.ty = static_cast<int32_t>((b.m.n + 16 * bv.nb - 1) / (16 * bv.nb));
      b.tz = 1;
      b.dep0 = fstage[s - 1];
      b.dep1 = -1;
      b.problem = q;
      flev[s] = flev[s - 1] + 1;
      fstage[s] = add(b, flev[s]);
      P[s] = Y;
      cur[s - 1] = L.rows;
    }
    if (!bwd) continue;
    // reverse sweep
    int lowest = it.dT.data ? 1 : d + 1;
    for (int k = 0; k < d; ++k)
      if (it.dL[k].data && k + 1 < lowest) lowest = k + 1;
    const void* Qmu = it.G.data;
    int qstage = -1, qlev = -1;
    int64_t qd[KP_MAX_ORDER];
    for (int k = 0; k < d; ++k) qd[k] = it.L[k].rows;
    for (int mu = d; mu >= lowest; --mu) {
      const int k = mu - 1;
      const kp_matrix& L = it.L[k];
      if (it.dL[k].data) {
        int64_t Il = 1, Ir = 1;
        for (int j = 0; j < k; ++j) Il *= qd[j];
        for (int j = k + 1; j < d; ++j) Ir *= qd[j];
        const bool inner = Il > 1;
        gram::GramArgs g{};
        g.Q = Qmu;
        g.P = P[k];
        g.Il = Il;
        g.n = L.rows;
        g.m = L.cols;
        g.Ir = Ir;
        g.achunks = inner ? (Il + kGramBR - 1) / kGramBR : 1;
        g.chunks = inner ? Ir * g.achunks : (Ir + kGramBR - 1) / kGramBR;
        const int64_t splits = batch_gram_splits(g.chunks);
        g.per_split = (g.chunks + splits - 1) / splits;
        g.part = region(static_cast<size_t>(splits * g.n * g.m) * es);
        BStage b{};
        b.kind = ST_GRAM;
        b.variant = inner ? 1 : 0;
        b.g = g;
        b.tx = static_cast<int32_t>((g.n + 63) / 64);
        b.ty = static_cast<int32_t>((g.m + 63) / 64);
        b.tz = static_cast<int32_t>(splits);
        b.dep0 = qstage;
        b.dep1 = fstage[k];
        b.problem = q;
        const int gl = 1 + std::max(qlev, flev[k]);
        const int gs = add(b, gl);
        BStage r{};
        r.kind = ST_REDUCE;
        r.g = g;
        r.splits = splits;
        r.dL = it.dL[k].data;
        r.rs = it.dL[k].rs;
        r.cs = it.dL[k].cs;
        r.tx = static_cast<int32_t>((g.n * g.m + kThreads - 1) / kThreads);
        r.ty = r.tz = 1;
        r.dep0 = gs;
        r.dep1 = -1;
        r.problem = q;
        add(r, gl + 1);
      }
      if (mu > lowest || (mu == 1 && it.dT.data)) {
        kp_matrix Lt = L;
        Lt.rows = L.cols;
        Lt.cols = L.rows;
        Lt.rs = L.cs;
        Lt.cs = L.rs;
        void* Y;
        if (mu == 1) {
          Y = it.dT.data;
        } else {
          int64_t e = 1;
          for (int j = 0; j < d; ++j) e *= (j == k) ? L.cols : qd[j];
          Y = region(static_cast<size_t>(e) * es);
        }
        BStage b{};
        b.kind = ST_MODE;
        b.m = mode_args(Qmu, Y, qd, d, k, Lt, 0);
        b.variant = pick_batch_variant(form, b.m);
        int nv;
        const BVar* vs = host_vars(form, &nv);
        const BVar& bv = vs[b.variant / 2];
        const int64_t F = b.m.Il > 1 ? b.m.Il * b.m.Ir : b.m.Ir;
        b.tx = static_cast<int32_t>((F + 64 * bv.fb - 1) / (64 * bv.fb));
        b.ty = static_cast<int32_t>((b.m.n + 16 * bv.nb - 1) / (16 * bv.nb));
        b.tz = 1;
        b.dep0 = qstage;
        b.dep1 = -1;
        b.problem = q;
        qlev = qlev + 1;
        qstage = add(b, qlev);
        Qmu = Y;
        qd[k] = L.cols;
      }
    }
  }
  pl->ws_total = off > 0 ? off : 256;
  return form;
}

// Orders stages by (level, problem) keeping dependencies earlier, rewrites
// the dependency indices and numbers the tasks.
int64_t finalize(Plan* pl) {
  const int n = static_cast<int>(pl->stages.size());
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (pl->level[a] != pl->level[b]) return pl->level[a] < pl->level[b];
    return pl->stages[a].problem < pl->stages[b].problem;
  });
  std::vector<int> pos(n);
  for (int i = 0; i < n; ++i) pos[idx[i]] = i;
  std::vector<BStage> out(n);
  int64_t task = 0;
  pl->level_begin.clear();
  int cur_level = -1;
  for (int i = 0; i < n; ++i) {
    BStage s = pl->stages[idx[i]];
    const int lv = pl->level[idx[i]];
    while (cur_level < lv) {  // levels are consecutive from 0
      pl->level_begin.push_back(task);
      ++cur_level;
    }
    if (s.dep0 >= 0) s.dep0 = pos[s.dep0];
    if (s.dep1 >= 0) s.dep1 = pos[s.dep1];
    s.begin = task;
    task += static_cast<int64_t>(s.tx) * s.ty * s.tz;
    out[i] = s;
  }
  pl->level_begin.push_back(task);
  pl->stages.swap(out);
  return task;
}

// Persistent workgroups for a form: all that fit on the device at once.
template <int FORM>
int batch_blocks() {
  static int blocks = 0;
  if (blocks == 0) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_level_kernel<FORM>, kThreads,
                                                     0) !=
            hipSuccess ||
        per <= 0)
      per = 1;
    blocks = cus * per;
  }
  return blocks;
}

}  // namespace

int list_batch_variants(int form, int32_t* out, int cap) {
  int nv;
  const BVar* vs = host_vars(form, &nv);
  for (int i = 0; i < nv && i < cap; ++i) {
    int32_t* o = out + 6 * i;
    o[0] = vs[i].nb;
    o[1] = vs[i].fb;
    o[2] = vs[i].bk;
    o[3] = 0;
    o[4] = 0;
    o[5] = 0;
  }
  return nv;
}

}  // namespace kp

using namespace kp;

extern "C" {

size_t kp_batch_workspace(int count, const kp_batch_item* items, int prec) {
  Plan pl;
  if (build_plan(count, items, prec, nullptr, &pl) < 0) return 0;
  return pl.ws_total;
}

size_t kp_batch_plan_bytes(int count, const kp_batch_item* items, int prec) {
  Plan pl;
  if (build_plan(count, items, prec, nullptr, &pl) < 0) return 0;
  finalize(&pl);
  return sizeof(BHeader) + pl.stages.size() * sizeof(BStage) +
         pl.level_begin.size() * sizeof(int64_t);
}

int kp_batch_plan(int count, const kp_batch_item* items, int prec, void* ws, size_t ws_bytes,
                  void* plan, size_t plan_bytes) {
  if (!plan || !ws) return KP_ERR_NULL;
  Plan pl;
  const int form = build_plan(count, items, prec, static_cast<char*>(ws), &pl);
  if (form < 0) return form;
  if (ws_bytes < pl.ws_total) return KP_ERR_WORKSPACE;
  const int64_t ntasks = finalize(&pl);
  const size_t need = sizeof(BHeader) + pl.stages.size() * sizeof(BStage) +
                      pl.level_begin.size() * sizeof(int64_t);
  if (plan_bytes < need) return KP_ERR_WORKSPACE;
  BHeader h{};
  h.magic = kMagic;
  h.nstages = static_cast<int32_t>(pl.stages.size());
  h.form = form;
  h.ntasks = ntasks;
  h.nlevels = static_cast<int32_t>(pl.level_begin.size()) - 1;
  h.ws_base = ws;
  h.ws_bytes = ws_bytes;
  char* p = static_cast<char*>(plan);
  memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  if (!pl.stages.empty()) memcpy(p, pl.stages.data(), pl.stages.size() * sizeof(BStage));
  p += pl.stages.size() * sizeof(BStage);
  memcpy(p, pl.level_begin.data(), pl.level_begin.size() * sizeof(int64_t));
  return KP_OK;
}

int kp_batch_info(const void* plan, int64_t* ntasks, int* nstages, int* nlevels) {
  if (!plan) return KP_ERR_NULL;
  BHeader h;
  memcpy(&h, plan, sizeof(h));
  if (h.magic != kMagic) return KP_ERR_VALUE;
  if (ntasks) *ntasks = h.ntasks;
  if (nstages) *nstages = h.nstages;
  if (nlevels) *nlevels = h.nlevels;
  return KP_OK;
}

int kp_tucker_batched(const void* plan_dev, const void* plan, void* ws, size_t ws_bytes,
                      hipStream_t stream) {
  if (!plan_dev || !plan || !ws) return KP_ERR_NULL;
  BHeader h;
  memcpy(&h, plan, sizeof(h));
  if (h.magic != kMagic) return KP_ERR_VALUE;
  if (h.ws_base != ws || ws_bytes < h.ws_bytes) return KP_ERR_WORKSPACE;
  if (h.nstages == 0) return KP_OK;
  const BStage* sd = reinterpret_cast<const BStage*>(static_cast<const char*>(plan_dev) +
                                                     sizeof(BHeader));
  const int64_t* lb = reinterpret_cast<const int64_t*>(
      static_cast<const char*>(plan) + sizeof(BHeader) + h.nstages * sizeof(BStage));
  int blocks;
  switch (h.form) {
    case FORM_F64: blocks = batch_blocks<FORM_F64>(); break;
    case FORM_F32: blocks = batch_blocks<FORM_F32>(); break;
    case FORM_BF16X3: blocks = batch_blocks<FORM_BF16X3>(); break;
    default: blocks = batch_blocks<FORM_BF16X6>(); break;
  }
  for (int l = 0; l < h.nlevels; ++l) {
    const int64_t b = lb[l], e = lb[l + 1];
    if (e <= b) continue;
    const unsigned grid = static_cast<unsigned>(e - b < blocks ? e - b : blocks);
    switch (h.form) {
      case FORM_F64:
        hipLaunchKernelGGL(batch_level_kernel<FORM_F64>, dim3(grid), dim3(kThreads), 0, stream,
                           sd, h.nstages, b, e);
        break;
      case FORM_F32:
        hipLaunchKernelGGL(batch_level_kernel<FORM_F32>, dim3(grid), dim3(kThreads), 0, stream,
                           sd, h.nstages, b, e);
        break;
      case FORM_BF16X3:
        hipLaunchKernelGGL(batch_level_kernel<FORM_BF16X3>, dim3(grid), dim3(kThreads), 0,
                           stream, sd, h.nstages, b, e);
        break;
      default:
        hipLaunchKernelGGL(batch_level_kernel<FORM_BF16X6>, dim3(grid), dim3(kThreads), 0,
                           stream, sd, h.nstages, b, e);
        break;
    }
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return hip_status(err);
  }
  return KP_OK;
}

}  // extern "C"
