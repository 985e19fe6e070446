// mu-mode product kernels for gfx950 (CDNA4).
//
// S = T x_mu L (Sec. 2, Definition of the mu-mode product): every mu-fiber of
// the input is multiplied by L. With the column-major layout of vec
// (Appendix A) the input is read in place as the three-index view
// (Il, m, Ir): no permutation or unfolding is ever materialised.
//
// Two layouts of the same contraction, chosen by whether mode mu has a
// contiguous run of earlier modes in front of it:
//   lead  (Il == 1): fibers are contiguous columns X[j + m*b]; the output
//                    run Y[i + n*b] is contiguous along i.
//   inner (Il  > 1): consecutive fibers are adjacent in memory,
//                    X[a + Il*(j + m*b)]; the output is contiguous along the
//                    fiber index r = a + Il*b (piecewise: runs of Il).
// In both, MFMA columns (the lane-contiguous index of the 16x16 output block)
// are the memory-contiguous output index, so stores from the accumulators are
// coalesced rows.
//
// Forms: FP64 MFMA (v_mfma_f64_16x16x4), FP32 MFMA (v_mfma_f32_16x16x4),
// and the BF16 split forms on v_mfma_f32_16x16x32_bf16: each FP32 operand is
// split on load into 2 (x3) or 3 (x6) BF16 planes by round-to-nearest-even,
// and the partial products are accumulated in FP32, the leading product in
// its own accumulator and all correction products in a second one.
#include "kp_common.h"
#include "kp_internal.h"
#include "mode_tile.h"
#include "wide_tile.h"

namespace kp {
namespace {

using namespace tile;

// Workgroups are dealt to the XCDs round-robin (workgroup id mod kXcds), each
// XCD with its own L2. The launch is one-dimensional and the id is remapped
// so that each XCD receives a contiguous range of logical tiles (logical =
// bx * gy + by), in order: the n tiles of one fiber tile are adjacent and
// read the same input fibers from that XCD's L2. TAIL_LAST (k-loop tiles):
// within its range an XCD takes the tiles of the last n tile (by = gy - 1,
// which holds the rows up to n and can be shorter) after all the others, so
// the tail of the launch, when fewer workgroups than slots are left, runs
// the shorter tiles (cube200 FP64: 69.3 -> 67.3 us per mode). The wide tiles
// keep the adjacent order (BF16x3 lost 6 % without it). Either way each
// range is permuted, not changed.
constexpr int kXcds = 8;

template <bool TAIL_LAST>
__device__ __forceinline__ void xcd_tile(int64_t gx, int64_t gy, int64_t* bx, int64_t* by) {
  const int64_t total = gx * gy;
  const int64_t id = blockIdx.x;
  const int64_t xcd = id % kXcds, local = id / kXcds;
  const int64_t per = total / kXcds, rem = total % kXcds;
  const int64_t start = xcd * per + (xcd < rem ? xcd : rem);
  const int64_t cnt = per + (xcd < rem ? 1 : 0);
  int64_t logical;
  if (!TAIL_LAST || gy < 2) {
    logical = start + local;
  } else {
    // last-n-tile entries of the range: (q0 + k) gy + gy - 1, k = 0 .. nlast-1
    const int64_t q0 = start / gy, r0 = start - q0 * gy;
    const int64_t e = start + cnt - 1 - (gy - 1) - q0 * gy;
    const int64_t nlast = e >= 0 ? e / gy + 1 : 0;
    const int64_t nfirst = cnt - nlast;
    if (local >= nfirst) {
      logical = (q0 + (local - nfirst)) * gy + gy - 1;
    } else {
      // the other entries in order: first those of fiber tile q0 from r0 on
      const int64_t head = gy - 1 - r0;
      if (local < head) {
        logical = start + local;
      } else {
        const int64_t j = local - head;
        logical = (q0 + 1 + j / (gy - 1)) * gy + j % (gy - 1);
      }
    }
  }
  *by = logical % gy;
  *bx = logical / gy;
}

template <int FORM, int NB, int FB, int BK, int OCC, int PF, bool INNER, bool VEC>
__global__ __launch_bounds__(kThreads, OCC) void mode_kernel(ModeArgs a, int64_t gx,
                                                             int64_t gy) {
  __shared__ __attribute__((aligned(16))) char lds[mode_lds_bytes<FORM, NB, FB, BK>()];
  int64_t bx, by;
  xcd_tile<true>(gx, gy, &bx, &by);
  mode_tile<FORM, NB, FB, BK, INNER, PF, VEC>(a, bx, by, lds);
}

// Wide tiles of the BF16 split forms (wide_tile.h): the four waves split the
// n rows (NBW 16-row blocks each) and share FBW 16-fiber blocks; 32-wide k
// steps.
// PRE: a.L points at the factor's pre-split planes (split_planes_kernel).
template <int FORM, int NBW, int FBW, int OCC, bool INNER, bool VEC, bool PRE = false>
__global__ __launch_bounds__(kThreads, OCC) void wide_kernel(ModeArgs a, int64_t gx,
                                                             int64_t gy) {
  __shared__ __attribute__((aligned(16))) char lds[wide_lds_bytes<FORM, FBW, 4, 32>()];
  int64_t bx, by;
  xcd_tile<false>(gx, gy, &bx, &by);
  wide_tile<FORM, NBW, FBW, 4, 32, INNER, VEC, PRE>(a, bx, by, lds);
}

// The bf16 planes of up to KP_MAX_ORDER factors in one launch; thread t
// (grid-stride) writes one lane's fragments of one (block, step) of the
// factor whose task range holds it.
template <int FORM>
__global__ __launch_bounds__(kThreads) void split_planes_kernel(SplitJobs jobs) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; t < jobs.total;
       t += stride) {
    int j = 0;
    while (j + 1 < jobs.count && t >= jobs.job[j + 1].begin) ++j;
    const SplitJob& J = jobs.job[j];
    const int64_t r = t - J.begin;
    const int lane = static_cast<int>(r & 63);
    const int64_t steps = (J.m + 31) / 32;
    const int64_t s = (r >> 6) % steps, b = (r >> 6) / steps;
    split_planes_lane<FORM>(static_cast<const float*>(J.L), J.n, J.m, J.rs, J.cs, b, s, lane,
                            static_cast<bf16x8_t*>(J.planes));
  }
}

// ---------------------------------------------------------------------------
// Dispatch over the compiled tile variants.
// ---------------------------------------------------------------------------
using KernelFn = void (*)(ModeArgs, int64_t, int64_t);

// kernel[inner][vec]
struct Variant {
  int form, nb, fb, bk, occ, pf;
  KernelFn kernel[2][2];
};

#define KP_VP(FORM, NB, FB, BK, OCC, PF)                                           \
  {FORM, NB, FB, BK, OCC, PF,                                                       \
   {{mode_kernel<FORM, NB, FB, BK, OCC, PF, false, false>,                          \
     mode_kernel<FORM, NB, FB, BK, OCC, PF, false, true>},                          \
    {mode_kernel<FORM, NB, FB, BK, OCC, PF, true, false>,                           \
     mode_kernel<FORM, NB, FB, BK, OCC, PF, true, true>}}}
#define KP_V(FORM, NB, FB, BK, OCC) KP_VP(FORM, NB, FB, BK, OCC, 1)

const Variant kVariants[] = {
    // FP64
    KP_V(FORM_F64, 1, 4, 16, 1), KP_V(FORM_F64, 2, 2, 16, 2), KP_V(FORM_F64, 4, 1, 16, 2),
    KP_V(FORM_F64, 7, 1, 16, 2), KP_V(FORM_F64, 8, 1, 16, 2), KP_V(FORM_F64, 13, 1, 16, 2),
    KP_V(FORM_F64, 7, 1, 8, 2), KP_V(FORM_F64, 7, 1, 8, 3), KP_V(FORM_F64, 4, 1, 8, 3),
    KP_V(FORM_F64, 8, 1, 8, 3), KP_V(FORM_F64, 2, 2, 8, 3), KP_V(FORM_F64, 13, 1, 8, 2),
    KP_VP(FORM_F64, 7, 1, 16, 2, 2), KP_VP(FORM_F64, 7, 1, 8, 2, 2),
    KP_VP(FORM_F64, 4, 1, 16, 2, 2),
    // FP32
    KP_V(FORM_F32, 1, 4, 16, 2), KP_V(FORM_F32, 2, 4, 16, 2), KP_V(FORM_F32, 2, 2, 16, 2),
    KP_V(FORM_F32, 4, 2, 16, 2), KP_V(FORM_F32, 4, 1, 16, 2), KP_V(FORM_F32, 8, 1, 16, 2),
    KP_V(FORM_F32, 7, 2, 16, 2), KP_V(FORM_F32, 13, 1, 16, 2),
    KP_VP(FORM_F32, 4, 1, 16, 2, 2), KP_VP(FORM_F32, 7, 1, 16, 2, 2),
    KP_VP(FORM_F32, 8, 1, 16, 2, 2),
    // BF16 x3
    KP_V(FORM_BF16X3, 1, 4, 32, 2), KP_V(FORM_BF16X3, 2, 4, 32, 2), KP_V(FORM_BF16X3, 2, 2, 32, 2),
    KP_V(FORM_BF16X3, 4, 2, 32, 2), KP_V(FORM_BF16X3, 4, 1, 32, 2), KP_V(FORM_BF16X3, 8, 1, 32, 2),
    KP_V(FORM_BF16X3, 7, 1, 32, 2), KP_V(FORM_BF16X3, 1, 2, 32, 2), KP_V(FORM_BF16X3, 2, 1, 32, 2),
    KP_VP(FORM_BF16X3, 4, 1, 32, 2, 2),
    // BF16 x6
    KP_V(FORM_BF16X6, 1, 4, 32, 2), KP_V(FORM_BF16X6, 2, 4, 32, 2), KP_V(FORM_BF16X6, 2, 2, 32, 2),
    KP_V(FORM_BF16X6, 4, 2, 32, 2), KP_V(FORM_BF16X6, 4, 1, 32, 2), KP_V(FORM_BF16X6, 8, 1, 32, 2),
    KP_V(FORM_BF16X6, 1, 2, 32, 2), KP_V(FORM_BF16X6, 2, 1, 32, 2),
    KP_VP(FORM_BF16X6, 4, 1, 32, 2, 2),
};

// Wide tiles (kind 3): nb = NBW, fb = FBW, bk = 32, pf = 2 (two chunks of
// fibers in flight).
#define KP_W(FORM, NBW, FBW, OCC)                                                   \
  {FORM, NBW, FBW, 32, OCC, 2,                                                      \
   {{wide_kernel<FORM, NBW, FBW, OCC, false, false>,                                \
     wide_kernel<FORM, NBW, FBW, OCC, false, true>},                                \
    {wide_kernel<FORM, NBW, FBW, OCC, true, false>,                                 \
     wide_kernel<FORM, NBW, FBW, OCC, true, true>}}}

const Variant kWide[] = {
    KP_W(FORM_BF16X3, 2, 4, 2), KP_W(FORM_BF16X3, 4, 2, 2), KP_W(FORM_BF16X3, 4, 4, 1),
    KP_W(FORM_BF16X6, 2, 4, 2), KP_W(FORM_BF16X6, 4, 2, 2), KP_W(FORM_BF16X6, 4, 4, 1),
};
// The same tiles reading pre-split planes, in the same order: kernel[inner][vec].
#define KP_WP(FORM, NBW, FBW, OCC)                                                  \
  {FORM, NBW, FBW, 32, OCC, 2,                                                      \
   {{wide_kernel<FORM, NBW, FBW, OCC, false, false, true>,                          \
     wide_kernel<FORM, NBW, FBW, OCC, false, true, true>},                          \
    {wide_kernel<FORM, NBW, FBW, OCC, true, false, true>,                           \
     wide_kernel<FORM, NBW, FBW, OCC, true, true, true>}}}
const Variant kWidePre[] = {
    KP_WP(FORM_BF16X3, 2, 4, 2), KP_WP(FORM_BF16X3, 4, 2, 2), KP_WP(FORM_BF16X3, 4, 4, 1),
    KP_WP(FORM_BF16X6, 2, 4, 2), KP_WP(FORM_BF16X6, 4, 2, 2), KP_WP(FORM_BF16X6, 4, 4, 1),
};
static_assert(sizeof(kWide) == sizeof(kWidePre), "one planes kernel per wide tile");

const Variant* find_wide(int form, const ModeTile& t) {
  if (t.kind != 3) return nullptr;
  for (const Variant& v : kWide)
    if (v.form == form && v.nb == t.nb && v.fb == t.fb && v.bk == t.bk &&
        (t.occ == 0 || v.occ == t.occ) && (t.pf == 0 || v.pf == t.pf))
      return &v;
  return nullptr;
}

const Variant* find_variant(int form, const ModeTile& t) {
  if (t.kind != 0) return nullptr;
  for (const Variant& v : kVariants)
    if (v.form == form && v.nb == t.nb && v.fb == t.fb && v.bk == t.bk &&
        (t.occ == 0 || v.occ == t.occ) && (t.pf == 0 ? v.pf == 1 : v.pf == t.pf))
      return &v;
  return nullptr;
}

// Default tiles, chosen from tile sweeps on cubes with n = 128..324 (cube200
// among them) and small modes: FP64 favours 7 (or, at 112 < n <= 184, 4)
// blocks along n with 8-wide k chunks (small LDS and register footprint),
// with two chunks of loads in flight once m >= 160; FP32 7 blocks (8 at
// n <= 128, 4 at 128 < n <= 184) with two chunks of loads in flight; the
// BF16 split forms 4 blocks (BF16x6 with two chunks in flight), or the wide
// tile above n = 176 (see the end of pick_tile). Short
// contractions (m <= 64; FP64: m <= 32, or m <= 64 on the lead layout)
// take strip tiles.
// 16-row blocks left empty in the last n tile when n is covered by tiles of
// nb blocks.
int64_t idle_blocks(int64_t n, int nb) {
  const int64_t b = (n + 15) / 16;
  return nb * ((b + nb - 1) / nb) - b;
}

ModeTile pick_tile(int form, int64_t Il, int64_t m, int64_t n, int64_t Ir) {
  ModeTile t{};
  if (strip_default(form, Il, m, n, Ir, &t)) return t;
  t.occ = 0;
  t.pf = 0;
  if (form == FORM_F64) {
    t.bk = 16;
    if (n <= 16) { t.nb = 1; t.fb = 4; }
    else if (n <= 32) {
      t.nb = 2;
      t.fb = 2;
      // contractions of 17-24: 8-wide chunks waste less of the last chunk
      if (m > 16 && m <= 24) {
        t.bk = 8;
        t.occ = 3;
      }
    }
    else {
      t.bk = 8;
      t.occ = 3;
      t.fb = 1;
      t.nb = (n <= 64 || (n > 112 && n <= 184)) ? 4 : 7;
      // long contractions keep two chunks of loads in flight
      if (t.nb == 7 && m >= 160) {
        t.occ = 2;
        t.pf = 2;
      }
      // n > 184 whose last 7-block tile would be at least 4 blocks emptier
      // than with 4-block tiles (n = 240, 256, 352, 384: 8-14 % faster)
      if (n > 184 && idle_blocks(n, 7) - idle_blocks(n, 4) >= 4) {
        t.nb = 4;
        t.bk = 16;
        t.occ = 2;
        t.pf = 2;
      }
    }
  } else if (form == FORM_F32) {
    t.bk = 16;
    if (n <= 16) { t.nb = 1; t.fb = 4; }
    else if (n <= 32) { t.nb = 2; t.fb = 2; }
    else if (n <= 64) { t.nb = 4; t.fb = 1; }
    else {
      t.nb = n <= 128 ? 8 : (n <= 184 ? 4 : 7);
      t.fb = 1;
      t.pf = 2;
      // the same for 8-block tiles (n = 240, 256, 352, 384: 10-18 % faster)
      if (n > 184 && idle_blocks(n, 7) - idle_blocks(n, 8) >= 4) t.nb = 8;
    }
  } else {
    t.bk = 32;
    if (n <= 16) { t.nb = 1; t.fb = 4; }
    else if (n <= 32) { t.nb = 2; t.fb = 2; }
    else { t.nb = 4; t.fb = 1; t.pf = form == FORM_BF16X6 ? 2 : 0; }
  }
  // Small problems (64 < n <= 184): when the tile above gives too few
  // workgroups to fill the chip, the smaller tiles the sweeps favoured there
  // (Ir < 0: no size adjustment)
  if (Ir < 0) return t;
  const int64_t F = Il > 1 ? Il * Ir : Ir;
  const int64_t tiles = ((F + 64 * t.fb - 1) / (64 * t.fb)) * ((n + 16 * t.nb - 1) / (16 * t.nb));
  const bool split = form == FORM_BF16X3 || form == FORM_BF16X6;
  if (n > 64 && n <= 184 && tiles < (split ? 512 : 1024)) {
    t.occ = 0;
    t.pf = 0;
    if (split) {
      if (n <= 112) { t.nb = 2; t.fb = 1; t.bk = 32; }
    } else if (n <= 112) {
      t.nb = 2; t.fb = 2; t.bk = 16;
    } else {
      t.nb = 4; t.fb = 1; t.bk = 16; t.pf = 2;
    }
  }
  // The split forms with n > 176 on the large-problem tile: the wide tile
  // (32 x 64 outputs per wave, each wave with its own factor rows). Cube
  // sweeps, us per mode, k-loop -> wide with the rows split in registers
  // (kp_mump): BF16x6 n = 200 50 -> 35, 256 87 -> 61, 324 252 -> 179;
  // BF16x3 n = 200 31 -> 29, 324 158 -> 129, 256 52 -> 56. us per Tucker
  // step with the factor planes split once (kp_tucker): BF16x3 n = 256
  // 159 -> 138, 324 504 -> 387; BF16x6 256 271 -> 176. At n = 160 the
  // k-loop tile stays ahead (BF16x3 43 against 54 us per step).
  if ((form == FORM_BF16X6 || form == FORM_BF16X3) && t.kind == 0 && t.nb == 4 && t.fb == 1 &&
      n > 176)
    t = ModeTile{2, 4, 32, 2, 2, 3};
  return t;
}

}  // namespace

ModeTile builtin_mode_tile(int form, int64_t Il, int64_t m, int64_t n, int64_t Ir) {
  return pick_tile(form, Il, m, n, Ir);
}

ModeTile default_mode_tile(int form, const ModeArgs& a, bool alone) {
  ModeTile t;
  if (tuned_tile(form, a.Il, a.m, a.n, a.Ir, &t)) return t;
  return pick_tile(form, a.Il, a.m, a.n, alone ? a.Ir : -1);
}

bool resolve_mode_tile(int form, const ModeTile& t, ModeTile* out) {
  if (t.kind == 1) return strip_resolve(form, t, out);
  const Variant* v = t.kind == 3 ? find_wide(form, t) : find_variant(form, t);
  if (!v) return false;
  *out = ModeTile{v->nb, v->fb, v->bk, v->occ, v->pf, t.kind};
  return true;
}

bool mode_tile_supported(int form, const ModeArgs& a, const ModeTile& t) {
  ModeTile r;
  if (!resolve_mode_tile(form, t, &r)) return false;
  return r.kind == 0 || a.m <= r.bk;
}

int list_mode_variants(int form, int32_t* out, int cap) {
  int count = 0;
  for (const Variant& v : kVariants) {
    if (v.form != form) continue;
    if (count < cap) {
      int32_t* o = out + 6 * count;
      o[0] = v.nb;
      o[1] = v.fb;
      o[2] = v.bk;
      o[3] = v.occ;
      o[4] = v.pf;
      o[5] = 0;
    }
    ++count;
  }
  for (const Variant& v : kWide) {
    if (v.form != form) continue;
    if (count < cap) {
      int32_t* o = out + 6 * count;
      o[0] = v.nb;
      o[1] = v.fb;
      o[2] = v.bk;
      o[3] = v.occ;
      o[4] = v.pf;
      o[5] = 3;
    }
    ++count;
  }
  const int ns = list_strip_variants(form, count < cap ? out + 6 * count : nullptr,
                                     count < cap ? cap - count : 0);
  return count + ns;
}

size_t split_planes_bytes(int form, int64_t n, int64_t m) {
  if (n <= 0 || m <= 0) return 0;
  const int64_t frags = form == FORM_BF16X6 ? split_plane_frags<FORM_BF16X6>(n, m)
                                            : split_plane_frags<FORM_BF16X3>(n, m);
  return static_cast<size_t>(frags) * sizeof(bf16x8_t);
}

int64_t split_planes_tasks(int64_t n, int64_t m) {
  return n > 0 && m > 0 ? ((n + 15) / 16) * ((m + 31) / 32) * 64 : 0;
}

bool mode_uses_wide(int form, const ModeArgs& a, const ModeTile* force) {
  if (form != FORM_BF16X3 && form != FORM_BF16X6) return false;
  const ModeTile t = force ? *force : default_mode_tile(form, a);
  return t.kind == 3 && find_wide(form, t) != nullptr;
}

hipError_t launch_split_planes(int form, const SplitJobs& jobs, hipStream_t stream) {
  if (jobs.count <= 0 || jobs.total <= 0) return hipSuccess;
  if (form != FORM_BF16X3 && form != FORM_BF16X6) return hipErrorInvalidValue;
  int64_t blocks = (jobs.total + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(form == FORM_BF16X6 ? split_planes_kernel<FORM_BF16X6>
                                         : split_planes_kernel<FORM_BF16X3>,
                     dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0, stream, jobs);
  return hipGetLastError();
}

hipError_t launch_mode(int form, const ModeArgs& a, const ModeTile* force,
                       hipStream_t stream) {
  return launch_mode_planes(form, a, force, nullptr, stream);
}

hipError_t launch_mode_planes(int form, const ModeArgs& a, const ModeTile* force,
                              const void* planes, hipStream_t stream) {
  const ModeTile t = force ? *force : default_mode_tile(form, a);
  const bool strip = t.kind == 1;
  const bool wide = t.kind == 3;
  const Variant* v = strip ? nullptr : (wide ? find_wide(form, t) : find_variant(form, t));
  // a wide tile with the factor's pre-split planes runs their kernel
  if (wide && v && planes) v = &kWidePre[v - kWide];
  ModeTile st{};
  if (strip && (!strip_resolve(form, t, &st) || a.m > st.bk)) return hipErrorInvalidValue;
  if (!strip && !v) return hipErrorInvalidValue;
  const bool inner = a.Il > 1;
  if (a.Il * a.Ir == 0 || a.n == 0) return hipSuccess;
  // The kernels address each launch's tensors with 32-bit byte offsets:
  // split the launch along the outer index b so every piece stays below
  // 2^31 bytes (pieces are independent: fibers never mix).
  const int64_t es = (form == FORM_F64) ? 8 : 4;
  const int64_t slab = a.Il * (a.m > a.n ? a.m : a.n) * es;  // bytes per b
  const int64_t limit = static_cast<int64_t>(1) << 31;
  if (slab >= limit) return hipErrorInvalidValue;
  const int64_t lspan = ((a.n - 1) * a.rs + (a.m > 0 ? a.m - 1 : 0) * a.cs + 1) * es;
  if (lspan >= limit) return hipErrorInvalidValue;
  const int64_t per = (limit - 1) / (slab > 0 ? slab : 1);
  // workgroup tile: k-loop tiles 16 nb rows x 64 fb fibers; wide tiles
  // 64 nb rows x 16 fb fibers
  const int64_t bf = strip ? 0 : (wide ? 16 * v->fb : 64 * v->fb);
  const int64_t bn = strip ? 0 : (wide ? 64 * v->nb : 16 * v->nb);
  // 16-byte group loads: L k-contiguous with 16-byte aligned rows, m a
  // multiple of 16 bytes' worth of elements (so the k tail is whole 16-byte
  // pieces), and for the lead layout X rows (m elements) 16-byte aligned too
  const bool vec_l = a.cs == 1 && (a.rs * es) % 16 == 0 && (a.m * es) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(a.L) % 16 == 0;
  const bool xrow16 = (a.m * es) % 16 == 0;
  for (int64_t b0 = 0; b0 < a.Ir; b0 += per) {
    ModeArgs p = a;
    p.Ir = (a.Ir - b0 < per) ? a.Ir - b0 : per;
    p.X = static_cast<const char*>(a.X) + b0 * a.Il * a.m * es;
    p.Y = static_cast<char*>(a.Y) + b0 * a.Il * a.n * es;
    if (strip) {
      const hipError_t e = launch_strip(form, p, st, stream);
      if (e != hipSuccess) return e;
      continue;
    }
    const int64_t F = inner ? p.Il * p.Ir : p.Ir;
    const int64_t gx = (F + bf - 1) / bf;
    const int64_t gy = (p.n + bn - 1) / bn;
    // one-dimensional grid: its size in work-items must fit 32 bits
    if (gx * gy > 0xffffffffLL / kThreads) return hipErrorInvalidConfiguration;
    const bool vec = vec_l && (inner || (xrow16 && reinterpret_cast<uintptr_t>(p.X) % 16 == 0));
    if (wide && planes) p.L = planes;
    hipLaunchKernelGGL(v->kernel[inner ? 1 : 0][vec ? 1 : 0],
                       dim3(static_cast<unsigned>(gx * gy)), dim3(kThreads), 0, stream, p, gx,
                       gy);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace kp
