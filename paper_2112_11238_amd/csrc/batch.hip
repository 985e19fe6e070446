// Batched Tucker operator: many independent problems (uneven sizes), forward
// and optionally backward, in a few launches.
//
// Every mu-mode product, factor-gradient partial sum and partial-sum
// reduction of every problem is a "stage" made of independent tasks. A
// stage's level is one more than the deepest level among the stages it
// depends on (the forward product of mode s depends on mode s-1, a factor
// gradient on the forward partial and on the reverse sweep, ...). The stages
// of one level that share a task type (k-loop tile or strip of one variant,
// gram tile, streaming gram, reduce) form a group; each group is one
// persistent launch whose workgroups stride over its tasks with a kernel
// compiled for that task type alone (so its registers and LDS are sized for
// it). Groups are launched level by level on one stream, so kernel
// boundaries order the dependencies and no workgroup ever waits for another.
// Capturing kp_tucker_batched in a HIP graph turns the whole batch into one
// graph.
#include "kp.h"

#include <string.h>

#include <algorithm>
#include <array>
#include <mutex>
#include <unordered_map>
#include <utility>
#include <vector>

#include "gram_strip.h"
#include "gram_tile.h"
#include "kp_common.h"
#include "kp_internal.h"
#include "mode_tile.h"
#include "strip_tile.h"

namespace kp {
namespace {

constexpr int kThreads = 256;
constexpr uint64_t kMagic = 0x6b70626174636803ULL;  // "kpbatch" v3
constexpr int kGramBR = 32;
constexpr int64_t kStripTiles = 16;   // fiber tiles per strip task
constexpr int64_t kGramChunks = 8;    // fiber chunks per streaming gram task

// ST_MODE: k-loop tiles; ST_STRIP: strip tasks (a run of fiber tiles of one
// n block, strip_tile.h); ST_GRAM: 64 x 64 gram tiles of one split;
// ST_GSTRIP: one streaming gram partial (gram_strip.h; variant bit 3: 16-byte
// fiber groups on the inner layout); ST_REDUCE: 16
// outputs of the fixed-order sum of a gram's partial tiles.
enum StageKind { ST_MODE = 0, ST_GRAM = 1, ST_REDUCE = 2, ST_STRIP = 3, ST_GSTRIP = 4 };

struct BStage {
  int32_t kind;
  int32_t variant;        // mode: batch variant id; gram: 1 = inner layout
  int32_t tx, ty, tz;     // tile grid; tiles = tx * ty * tz
  int32_t dep0, dep1;     // stages that must be complete (-1: none)
  int32_t problem;
  int64_t begin;          // first global task number of this stage
  ModeArgs m;             // ST_MODE
  gram::GramArgs g;       // ST_GRAM (and n, m, part for ST_REDUCE)
  int64_t splits;         // ST_REDUCE, ST_GSTRIP: number of partial tiles
  void* dL;               // ST_REDUCE output
  int64_t rs, cs;
  int64_t ntiles;         // ST_STRIP: fiber tiles; ST_GSTRIP: fiber chunks
};

// Plan layout: [BHeader][BStage x nstages][int64 level_begin x (nlevels + 1)]
// [BGroup x ngroups]; level_begin[l] is the first task number of level l.
struct BHeader {
  uint64_t magic;
  int32_t nstages;
  int32_t form;
  int64_t ntasks;
  int32_t nlevels;
  int32_t ngroups;
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

// Strip variants of the executor, per form: (nb, fb, kp); fb per kp as in
// the standalone strip kernels.
struct SVar {
  int nb, fb, kp;
};
constexpr SVar kSVarF32[] = {{1, 2, 16}, {2, 2, 16}, {4, 2, 16}, {1, 2, 32}, {2, 2, 32},
                             {4, 2, 32}, {1, 1, 64}, {2, 1, 64}, {4, 1, 64}};
constexpr SVar kSVarF64[] = {{2, 2, 16}, {4, 2, 16}, {2, 1, 32}, {4, 1, 32}};
constexpr SVar kSVarB3[] = {{2, 2, 32}, {4, 2, 32}, {2, 1, 64}, {4, 1, 64}};
constexpr SVar kSVarB6[] = {{2, 1, 32}, {4, 1, 32}, {2, 1, 64}, {4, 1, 64}};

template <int FORM>
struct SVars;
template <>
struct SVars<FORM_F32> {
  static constexpr const SVar* v = kSVarF32;
  static constexpr int n = 9;
};
template <>
struct SVars<FORM_F64> {
  static constexpr const SVar* v = kSVarF64;
  static constexpr int n = 4;
};
template <>
struct SVars<FORM_BF16X3> {
  static constexpr const SVar* v = kSVarB3;
  static constexpr int n = 4;
};
template <>
struct SVars<FORM_BF16X6> {
  static constexpr const SVar* v = kSVarB6;
  static constexpr int n = 4;
};

const SVar* host_svars(int form, int* count) {
  switch (form) {
    case FORM_F32: *count = 9; return kSVarF32;
    case FORM_F64: *count = 4; return kSVarF64;
    case FORM_BF16X3: *count = 4; return kSVarB3;
    default: *count = 4; return kSVarB6;
  }
}

template <typename E>
constexpr int gstrip_br() { return sizeof(E) == 8 ? 32 : 64; }

const BVar* host_vars(int form, int* count) {
  switch (form) {
    case FORM_F64: *count = 5; return kBVarF64;
    case FORM_F32: *count = 6; return kBVarF32;
    default: *count = 4; return kBVarB16;
  }
}

// LDS of one (kind, variant) task type.
template <int FORM, int KIND, int VAR>
constexpr size_t task_lds() {
  using E = typename tile::FormT<FORM>::G;
  if constexpr (KIND == ST_MODE) {
    constexpr BVar v = BVars<FORM>::v[VAR / 2];
    return tile::mode_lds_bytes<FORM, v.nb, v.fb, v.bk>();
  } else if constexpr (KIND == ST_STRIP) {
    constexpr SVar v = SVars<FORM>::v[VAR / 2];
    return tile::strip_lds_bytes<FORM, v.nb, v.fb, v.kp>();
  } else if constexpr (KIND == ST_GRAM) {
    return gram::gram_lds_bytes<E, kGramBR>();
  } else if constexpr (KIND == ST_GSTRIP) {
    return gram::strip_lds_bytes<E, (VAR & 4) ? 4 : 2, (VAR & 2) ? 4 : 2, gstrip_br<E>()>();
  } else {
    return kThreads * sizeof(E);
  }
}

// One task of a stage; the task type is fixed at compile time.
template <int FORM, int KIND, int VAR>
__device__ __forceinline__ void run_task(const BStage& S, int64_t tile_id, char* lds) {
  using E = typename tile::FormT<FORM>::G;
  constexpr bool INNER = (VAR & 1) != 0;
  if constexpr (KIND == ST_MODE) {
    constexpr BVar v = BVars<FORM>::v[VAR / 2];
    const int64_t bx = tile_id % S.tx;
    const int64_t by = tile_id / S.tx;
    tile::mode_tile<FORM, v.nb, v.fb, v.bk, INNER>(S.m, bx, by, lds);
  } else if constexpr (KIND == ST_STRIP) {
    constexpr SVar v = SVars<FORM>::v[VAR / 2];
    const int64_t sx = tile_id % S.tx;
    const int64_t by = tile_id / S.tx;
    const int64_t t0 = sx * S.ntiles / S.tx, t1 = (sx + 1) * S.ntiles / S.tx;
    tile::strip_run<FORM, v.nb, v.fb, v.kp, INNER, false>(S.m, by, t0, 1, t1, lds);
  } else if constexpr (KIND == ST_GRAM) {
    const int64_t bx = tile_id % S.tx;
    const int64_t by = (tile_id / S.tx) % S.ty;
    const int64_t bz = tile_id / (static_cast<int64_t>(S.tx) * S.ty);
    gram::gram_tile<E, kGramBR, INNER>(S.g, bx, by, bz, lds);
  } else if constexpr (KIND == ST_GSTRIP) {
    const int64_t cb = tile_id * S.ntiles / S.splits;
    const int64_t ce = (tile_id + 1) * S.ntiles / S.splits;
    gram::gram_strip<E, (VAR & 4) ? 4 : 2, (VAR & 2) ? 4 : 2, gstrip_br<E>(), INNER,
                     INNER && (VAR & 8) != 0>(
        S.g, cb, ce, static_cast<E*>(S.g.part) + tile_id * S.g.n * S.g.m, lds);
  } else {
    gram::gram_reduce_block<E, 16>(static_cast<const E*>(S.g.part), S.splits, S.g.n, S.g.m,
                                   static_cast<E*>(S.dL), S.rs, S.cs, tile_id,
                                   reinterpret_cast<E*>(lds));
  }
}

// Runs the tasks [task_begin, task_end) of one group: the stages
// [s_begin, s_end) of one level that share a task type. Workgroup b takes
// tasks task_begin + b, task_begin + b + gridDim.x, ...; no task of a level
// depends on another task of the same level.
template <int FORM, int KIND, int VAR>
__global__ __launch_bounds__(kThreads, 2) void batch_group_kernel(const BStage* __restrict__ st,
                                                                  int s_begin, int s_end,
                                                                  int64_t task_begin,
                                                                  int64_t task_end) {
  __shared__ __attribute__((aligned(16))) char lds[task_lds<FORM, KIND, VAR>()];
  for (int64_t task = task_begin + blockIdx.x; task < task_end; task += gridDim.x) {
    // stage of this task: the last stage whose begin <= task (the same in
    // every lane, so its fields are read with scalar loads)
    int lo = s_begin, hi = s_end - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (st[mid].begin <= task)
        lo = mid;
      else
        hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const BStage& S = st[lo];
    __syncthreads();  // the previous task's LDS reads are complete
    run_task<FORM, KIND, VAR>(S, task - S.begin, lds);
  }
}

using GroupFn = void (*)(const BStage*, int, int, int64_t, int64_t);

// Kernel table of a form: index = kind-specific offset + variant.
template <int FORM, int KIND, int... V>
constexpr std::array<GroupFn, sizeof...(V)> group_fns(std::integer_sequence<int, V...>) {
  return {{batch_group_kernel<FORM, KIND, V>...}};
}

template <int FORM>
struct GroupTable {
  static constexpr int NM = 2 * BVars<FORM>::n, NS = 2 * SVars<FORM>::n;
  static constexpr auto mode = group_fns<FORM, ST_MODE>(std::make_integer_sequence<int, NM>{});
  static constexpr auto strip = group_fns<FORM, ST_STRIP>(std::make_integer_sequence<int, NS>{});
  static constexpr auto gram = group_fns<FORM, ST_GRAM>(std::make_integer_sequence<int, 2>{});
  static constexpr auto gstrip = group_fns<FORM, ST_GSTRIP>(std::make_integer_sequence<int, 16>{});
  static constexpr auto reduce = group_fns<FORM, ST_REDUCE>(std::make_integer_sequence<int, 1>{});
  static GroupFn get(int kind, int var) {
    switch (kind) {
      case ST_MODE: return var >= 0 && var < NM ? mode[var] : nullptr;
      case ST_STRIP: return var >= 0 && var < NS ? strip[var] : nullptr;
      case ST_GRAM: return var >= 0 && var < 2 ? gram[var] : nullptr;
      case ST_GSTRIP: return var >= 0 && var < 16 ? gstrip[var] : nullptr;
      case ST_REDUCE: return var == 0 ? reduce[0] : nullptr;
      default: return nullptr;
    }
  }
};

GroupFn group_fn(int form, int kind, int var) {
  switch (form) {
    case FORM_F64: return GroupTable<FORM_F64>::get(kind, var);
    case FORM_F32: return GroupTable<FORM_F32>::get(kind, var);
    case FORM_BF16X3: return GroupTable<FORM_BF16X3>::get(kind, var);
    default: return GroupTable<FORM_BF16X6>::get(kind, var);
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

// One launch: stages [s_begin, s_end) of one level and one task type,
// tasks [t_begin, t_end).
struct BGroup {
  int32_t kind, variant, s_begin, s_end, level, pad_;
  int64_t t_begin, t_end;
};

struct Plan {
  std::vector<BStage> stages;
  std::vector<int> level;
  std::vector<int64_t> level_begin;  // after finalize
  std::vector<BGroup> groups;        // after finalize
  size_t ws_total = 0;
};

// Batch variant for a mode product: the tuned / default tile if the executor
// has it, else the executor's variant with the closest n coverage.
int pick_batch_variant(int form, const ModeArgs& a) {
  const ModeTile want = default_mode_tile(form, a, false);
  // n blocks per workgroup of the wanted tile (a wide tile has 4 waves of nb)
  const int want_nb = want.kind == 3 ? 4 * want.nb : want.nb;
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
    const int64_t cost = (padded - a.n) * 8 + (vs[i].nb == want_nb ? 0 : 1);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = i;
    }
  }
  return 2 * best + (a.Il > 1 ? 1 : 0);
}

// Strip variant of the executor for a product whose tuned / default tile is
// a strip: the same (nb, kp) if the executor has it, else the shortest strip
// covering m with the least n padding; -1 if no strip covers m.
int pick_strip_variant(int form, const ModeArgs& a, const ModeTile& want) {
  int nv;
  const SVar* vs = host_svars(form, &nv);
  int best = -1;
  int64_t best_cost = 0;
  for (int i = 0; i < nv; ++i) {
    if (vs[i].kp < a.m) continue;
    if (vs[i].nb == want.nb && vs[i].kp == want.bk) return i;
    const int64_t bn = 16 * vs[i].nb;
    const int64_t padded = ((a.n + bn - 1) / bn) * bn;
    const int64_t cost = static_cast<int64_t>(vs[i].kp) * 4096 + (padded - a.n);
    if (best < 0 || cost < best_cost) {
      best = i;
      best_cost = cost;
    }
  }
  return best;
}

// Kind, variant and task grid of a mode-product stage (b.m set).
void set_mode_stage(int form, BStage& b) {
  const ModeTile want = default_mode_tile(form, b.m, false);
  const bool inner = b.m.Il > 1;
  const int64_t F = inner ? b.m.Il * b.m.Ir : b.m.Ir;
  if (want.kind == 1) {
    const int sv = pick_strip_variant(form, b.m, want);
    if (sv >= 0) {
      int nv;
      const SVar& v = host_svars(form, &nv)[sv];
      b.kind = ST_STRIP;
      b.variant = 2 * sv + (inner ? 1 : 0);
      b.ntiles = (F + 64 * v.fb - 1) / (64 * v.fb);
      b.tx = static_cast<int32_t>((b.ntiles + kStripTiles - 1) / kStripTiles);
      b.ty = static_cast<int32_t>((b.m.n + 16 * v.nb - 1) / (16 * v.nb));
      b.tz = 1;
      return;
    }
  }
  b.kind = ST_MODE;
  b.variant = pick_batch_variant(form, b.m);
  int nv;
  const BVar& bv = host_vars(form, &nv)[b.variant / 2];
  b.tx = static_cast<int32_t>((F + 64 * bv.fb - 1) / (64 * bv.fb));
  b.ty = static_cast<int32_t>((b.m.n + 16 * bv.nb - 1) / (16 * bv.nb));
  b.tz = 1;
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
    if (L.rs < 0 || L.cs < 0) return KP_ERR_VALUE;
    if (((L.rows - 1) * L.rs + (L.cols - 1) * L.cs + 1) * static_cast<int64_t>(es) >=
        (static_cast<int64_t>(1) << 31))
      return KP_ERR_SHAPE;
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
      if (D.rs < 0 || D.cs < 0) return KP_ERR_VALUE;
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
      b.m = mode_args(P[s - 1], Y, dims[s - 1], d, s - 1, L, 0);
      set_mode_stage(form, b);
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
        BStage b{};
        int64_t splits;
        if (g.n <= 64 && g.m <= 64) {
          // streaming partials: each task a contiguous run of fiber chunks
          const int64_t br = es == 8 ? 32 : 64;
          const int64_t chunks = (Il * Ir + br - 1) / br;
          splits = (chunks + kGramChunks - 1) / kGramChunks;
          if (splits > 1024) splits = 1024;
          if (splits < 1) splits = 1;
          g.part = region(static_cast<size_t>(splits * g.n * g.m) * es);
          b.kind = ST_GSTRIP;
          // + 8: inner fibers staged in 16-byte groups (I_l a multiple of
          // the group, Q and P 16-byte aligned)
          const bool gv = inner && Il % static_cast<int64_t>(16 / es) == 0 &&
                          reinterpret_cast<uintptr_t>(g.Q) % 16 == 0 &&
                          reinterpret_cast<uintptr_t>(g.P) % 16 == 0;
          b.variant = (inner ? 1 : 0) + (g.m > 32 ? 2 : 0) + (g.n > 32 ? 4 : 0) + (gv ? 8 : 0);
          b.ntiles = chunks;
          b.splits = splits;
          b.tx = static_cast<int32_t>(splits);
          b.ty = b.tz = 1;
        } else {
          g.achunks = inner ? (Il + kGramBR - 1) / kGramBR : 1;
          g.chunks = inner ? Ir * g.achunks : (Ir + kGramBR - 1) / kGramBR;
          splits = batch_gram_splits(g.chunks);
          g.per_split = (g.chunks + splits - 1) / splits;
          g.part = region(static_cast<size_t>(splits * g.n * g.m) * es);
          b.kind = ST_GRAM;
          b.variant = inner ? 1 : 0;
          b.tx = static_cast<int32_t>((g.n + 63) / 64);
          b.ty = static_cast<int32_t>((g.m + 63) / 64);
          b.tz = static_cast<int32_t>(splits);
        }
        b.g = g;
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
        r.tx = static_cast<int32_t>((g.n * g.m + 15) / 16);
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
        b.m = mode_args(Qmu, Y, qd, d, k, Lt, 0);
        set_mode_stage(form, b);
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

// Orders stages by (level, task type, problem) keeping dependencies
// earlier, rewrites the dependency indices, numbers the tasks and forms the
// launch groups: runs of stages of one level with one task type.
int64_t finalize(Plan* pl) {
  const int n = static_cast<int>(pl->stages.size());
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    const BStage& x = pl->stages[a];
    const BStage& y = pl->stages[b];
    if (pl->level[a] != pl->level[b]) return pl->level[a] < pl->level[b];
    if (x.kind != y.kind) return x.kind < y.kind;
    if (x.variant != y.variant) return x.variant < y.variant;
    return x.problem < y.problem;
  });
  std::vector<int> pos(n);
  for (int i = 0; i < n; ++i) pos[idx[i]] = i;
  std::vector<BStage> out(n);
  int64_t task = 0;
  pl->level_begin.clear();
  pl->groups.clear();
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
    const int64_t nt = static_cast<int64_t>(s.tx) * s.ty * s.tz;
    BGroup* g = pl->groups.empty() ? nullptr : &pl->groups.back();
    if (!g || g->level != lv || g->kind != s.kind || g->variant != s.variant) {
      BGroup ng{};
      ng.kind = s.kind;
      ng.variant = s.variant;
      ng.s_begin = i;
      ng.level = lv;
      ng.t_begin = task;
      pl->groups.push_back(ng);
      g = &pl->groups.back();
    }
    g->s_end = i + 1;
    g->t_end = task + nt;
    task += nt;
    out[i] = s;
  }
  pl->level_begin.push_back(task);
  pl->stages.swap(out);
  return task;
}

// Resident workgroups of a kernel on the device (queried once per kernel).
int group_blocks(GroupFn fn) {
  static std::mutex mu;
  static std::unordered_map<const void*, int> cache;
  std::lock_guard<std::mutex> lock(mu);
  const auto it = cache.find(reinterpret_cast<const void*>(fn));
  if (it != cache.end()) return it->second;
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(fn),
                                                   kThreads, 0) != hipSuccess ||
      per <= 0)
    per = 1;
  cache[reinterpret_cast<const void*>(fn)] = cus * per;
  return cus * per;
}

}  // namespace

int list_batch_variants(int form, int32_t* out, int cap) {
  int nv, ns;
  const BVar* vs = host_vars(form, &nv);
  const SVar* ss = host_svars(form, &ns);
  for (int i = 0; i < nv + ns && i < cap; ++i) {
    int32_t* o = out + 6 * i;
    const bool strip = i >= nv;
    o[0] = strip ? ss[i - nv].nb : vs[i].nb;
    o[1] = strip ? ss[i - nv].fb : vs[i].fb;
    o[2] = strip ? ss[i - nv].kp : vs[i].bk;
    o[3] = 0;
    o[4] = 0;
    o[5] = strip ? 1 : 0;
  }
  return nv + ns;
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
         pl.level_begin.size() * sizeof(int64_t) + pl.groups.size() * sizeof(BGroup);
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
                      pl.level_begin.size() * sizeof(int64_t) + pl.groups.size() * sizeof(BGroup);
  if (plan_bytes < need) return KP_ERR_WORKSPACE;
  BHeader h{};
  h.magic = kMagic;
  h.nstages = static_cast<int32_t>(pl.stages.size());
  h.form = form;
  h.ntasks = ntasks;
  h.nlevels = static_cast<int32_t>(pl.level_begin.size()) - 1;
  h.ngroups = static_cast<int32_t>(pl.groups.size());
  h.ws_base = ws;
  h.ws_bytes = ws_bytes;
  char* p = static_cast<char*>(plan);
  memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  if (!pl.stages.empty()) memcpy(p, pl.stages.data(), pl.stages.size() * sizeof(BStage));
  p += pl.stages.size() * sizeof(BStage);
  memcpy(p, pl.level_begin.data(), pl.level_begin.size() * sizeof(int64_t));
  p += pl.level_begin.size() * sizeof(int64_t);
  if (!pl.groups.empty()) memcpy(p, pl.groups.data(), pl.groups.size() * sizeof(BGroup));
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
  const BGroup* gr = reinterpret_cast<const BGroup*>(
      static_cast<const char*>(plan) + sizeof(BHeader) + h.nstages * sizeof(BStage) +
      (h.nlevels + 1) * sizeof(int64_t));
  // one launch per group, in plan order (levels ascending): kernel
  // boundaries on the stream order the levels
  for (int q = 0; q < h.ngroups; ++q) {
    const BGroup& g = gr[q];
    if (g.s_begin < 0 || g.s_end > h.nstages || g.s_begin >= g.s_end) return KP_ERR_VALUE;
    if (g.t_end <= g.t_begin) continue;
    const GroupFn fn = group_fn(h.form, g.kind, g.variant);
    if (!fn) return KP_ERR_VALUE;
    const int64_t blocks = group_blocks(fn);
    const int64_t tasks = g.t_end - g.t_begin;
    const unsigned grid = static_cast<unsigned>(tasks < blocks ? tasks : blocks);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kThreads), 0, stream, sd, g.s_begin, g.s_end,
                       g.t_begin, g.t_end);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return hip_status(err);
  }
  return KP_OK;
}

}  // extern "C"
