// Device-side tile of the mu-mode product for gfx950 (Sec. 2, Definition of
// the mu-mode product), shared by the standalone mode kernels and the batched
// persistent executor. The input is read in place as the (Il, m, Ir) view of
// the column-major tensor; see mode_kernels.hip for the layouts and forms.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kp_common.h"

namespace kp {
namespace tile {

constexpr int kThreads = 256;  // threads per workgroup (4 waves)

// ---------------------------------------------------------------------------
// MFMA operand layouts (checked on the device):
//   16x16x4 (f64, f32): lane l feeds A[l%16][l/16] and B[l/16][l%16];
//     accumulator item v of lane l is D[4v + l/16][l%16] for FP64 and
//     D[4(l/16) + v][l%16] for FP32.
//   16x16x32 bf16: lane l feeds A[l%16][8(l/16) .. +7] and
//     B[8(l/16) .. +7][l%16]; item v of lane l is D[4(l/16) + v][l%16].
// ---------------------------------------------------------------------------
// Offset of fiber r = a + Il*b of a (Il, len, Ir) view: a + Il*len*b.
__device__ __forceinline__ uint32_t fiber_offset(uint32_t r, uint32_t Il, uint32_t len) {
  const uint32_t b = r / Il;
  return (r - b * Il) + Il * len * b;
}

// Round-to-nearest-even split of x into P bf16 terms: x1 = bf16(x),
// x2 = bf16(x - x1), x3 = bf16(x - x1 - x2). Each difference is exact in FP32.
template <int P>
__device__ __forceinline__ void split_bf16(float x, __bf16 (&o)[P]) {
  float r = x;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const __bf16 h = static_cast<__bf16>(r);
    o[p] = h;
    r = r - static_cast<float>(h);
  }
}

// The same split for KV consecutive values at once, two per conversion
// (each pair of bf16 terms is one round-to-nearest-even packed conversion),
// written as the P bf16 planes of one k group.
template <int P, int KV, typename V8>
__device__ __forceinline__ void split_bf16_group(const float (&x)[KV], V8 (&pl)[P]) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef __bf16 b2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int e = 0; e < KV; e += 2) {
    f2 r = {x[e], x[e + 1]};
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const b2 h = __builtin_convertvector(r, b2);
      pl[p][e] = h[0];
      pl[p][e + 1] = h[1];
      if (p + 1 < P) r = r - __builtin_convertvector(h, f2);
    }
  }
}

// Epilogue store of one output value y at byte offset off (past the
// resource: dropped) by the lane holding fiber column c: overwrite, add, or
// (inner layout only) add +-i times the value on interleaved complex data.
// The parts of one complex entry are the adjacent fibers held by lanes c and
// c ^ 1, so each lane takes its partner's value: re += -s im(v),
// im += s re(v). acc is uniform across the wave, so every lane shuffles.
template <bool INNER, typename G>
__device__ __forceinline__ void store_out(G y, __amdgpu_buffer_rsrc_t rs, uint32_t off, int acc,
                                          int c);

// Buffer resource word 3 for raw (unformatted, unswizzled) buffers on the
// gfx9 family; loads at offsets at or past the resource's size return zero.
constexpr int kBufferFlags = 0x00020000;

// off: per-lane byte offset; soff: a wave-uniform byte offset added to it.
template <typename G>
__device__ __forceinline__ G buffer_load(__amdgpu_buffer_rsrc_t rs, uint32_t off,
                                         uint32_t soff = 0) {
  if constexpr (sizeof(G) == 8) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, static_cast<int>(off),
                                                         static_cast<int>(soff), 0);
    return __builtin_bit_cast(G, v);
  } else {
    const unsigned int v = __builtin_amdgcn_raw_buffer_load_b32(rs, static_cast<int>(off),
                                                                static_cast<int>(soff), 0);
    return __builtin_bit_cast(G, v);
  }
}

template <typename G>
__device__ __forceinline__ void buffer_store(G v, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
  if constexpr (sizeof(G) == 8) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs,
                                          static_cast<int>(off), 0, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), rs,
                                          static_cast<int>(off), 0, 0);
  }
}

template <bool INNER, typename G>
__device__ __forceinline__ void store_out(G y, __amdgpu_buffer_rsrc_t rs, uint32_t off, int acc,
                                          int c) {
  if constexpr (INNER) {
    if (acc >= kAccAddI) {
      const G other = __shfl_xor(y, 1);
      const G s = acc == kAccAddI ? G(1) : G(-1);
      y = (c & 1) ? s * other : -s * other;
    }
  }
  if (acc != kAccNone) y += buffer_load<G>(rs, off);
  buffer_store<G>(y, rs, off);
}

// Per-form constants. The LDS tiles hold rows (an n index or a fiber) whose
// k values are contiguous; every lane reads 16 bytes = KV consecutive k of
// one row. Because the contraction is a plain sum over k, lane group
// g = lane/16 may own k values [KV*g, KV*g + KV) of each macro step of
// MK = 4*KV values: MFMA step s then pairs A[row][KV*g + s] with
// B[KV*g + s][col] in every lane group, the same k on both operands.
template <int FORM>
struct FormT;

template <>
struct FormT<FORM_F64> {
  using G = double;   // global element
  using S = double;   // LDS element
  static constexpr int P = 1, KV = 2, MK = 8;
  using acc_t = d4_t;
  static __device__ __forceinline__ int row(int l, int v) { return 4 * v + (l >> 4); }
};
template <>
struct FormT<FORM_F32> {
  using G = float;
  using S = float;
  static constexpr int P = 1, KV = 4, MK = 16;
  using acc_t = f4_t;
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};
template <int FORM>
struct FormBf16 {
  using G = float;
  using S = __bf16;
  static constexpr int P = FORM == FORM_BF16X3 ? 2 : 3, KV = 8, MK = 32;
  using acc_t = f4_t;
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};
template <>
struct FormT<FORM_BF16X3> : FormBf16<FORM_BF16X3> {};
template <>
struct FormT<FORM_BF16X6> : FormBf16<FORM_BF16X6> {};

template <int FORM>
using Frag = typename std::conditional<FORM == FORM_F64, d2_t,
             typename std::conditional<FORM == FORM_F32, f4v_t, bf16x8_t>::type>::type;

// One macro step of MFMAs for one (row block, column block) pair.
// A: KV k values of the MFMA row operand (per plane), B: same for the column
// operand. hi/lo: accumulators (lo is unused by the native forms).
template <int FORM>
__device__ __forceinline__ void macro_step(const Frag<FORM> (&A)[FormT<FORM>::P],
                                           const Frag<FORM> (&B)[FormT<FORM>::P],
                                           typename FormT<FORM>::acc_t& hi,
                                           typename FormT<FORM>::acc_t& lo) {
  if constexpr (FORM == FORM_F64) {
    hi = __builtin_amdgcn_mfma_f64_16x16x4f64(A[0][0], B[0][0], hi, 0, 0, 0);
    hi = __builtin_amdgcn_mfma_f64_16x16x4f64(A[0][1], B[0][1], hi, 0, 0, 0);
    (void)lo;
  } else if constexpr (FORM == FORM_F32) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
      hi = __builtin_amdgcn_mfma_f32_16x16x4f32(A[0][s], B[0][s], hi, 0, 0, 0);
    (void)lo;
  } else {
    // correction products (smallest first) into lo, the leading one into hi
    if constexpr (FORM == FORM_BF16X6) {
      lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[2], lo, 0, 0, 0);
      lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[1], lo, 0, 0, 0);
      lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2], B[0], lo, 0, 0, 0);
    }
    lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[1], lo, 0, 0, 0);
    lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[0], lo, 0, 0, 0);
    hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[0], hi, 0, 0, 0);
  }
}

// One macro step for an R x C grid of output blocks at once: A[r] feeds
// block row r, B[c] block column c. The products are issued slot by slot
// across all blocks (slot = one of the per-block MFMAs of macro_step, in the
// same order), so consecutive MFMAs never write the same accumulator and
// each accumulator still receives its products in macro_step's order (the
// results are bitwise those of R x C separate macro steps).
template <int FORM, int R, int C>
__device__ __forceinline__ void macro_step_grid(
    const Frag<FORM> (&A)[R][FormT<FORM>::P], const Frag<FORM> (&B)[C][FormT<FORM>::P],
    typename FormT<FORM>::acc_t (&hi)[R][C], typename FormT<FORM>::acc_t (&lo)[R][C]) {
  auto each = [&](auto&& f) {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < C; ++c) f(r, c);
  };
  if constexpr (FORM == FORM_F64) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
      each([&](int r, int c) {
        hi[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[r][0][s], B[c][0][s], hi[r][c], 0, 0, 0);
      });
  } else if constexpr (FORM == FORM_F32) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
      each([&](int r, int c) {
        hi[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[r][0][s], B[c][0][s], hi[r][c], 0, 0, 0);
      });
  } else {
    // correction products (smallest first) into lo, the leading one into hi
    auto slot = [&](int pa, int pb, auto& acc) {
      each([&](int r, int c) {
        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[r][pa], B[c][pb], acc[r][c], 0, 0, 0);
      });
    };
    if constexpr (FORM == FORM_BF16X6) {
      slot(0, 2, lo);
      slot(1, 1, lo);
      slot(2, 0, lo);
    }
    slot(0, 1, lo);
    slot(1, 0, lo);
    slot(0, 0, hi);
  }
}

// NB: 16-blocks along n per workgroup (every wave covers all of them).
// FB: 16-blocks of fibers per wave; 4 waves split the fibers, so a workgroup
//     covers 64*FB fibers.
// BK: k values staged through LDS per chunk (double buffered, one barrier
//     per chunk). OCC: waves per SIMD the register budget is sized for.
// LDS bytes one tile of a variant needs (double-buffered L and X tiles).
template <int FORM, int NB, int FB, int BK>
constexpr size_t mode_lds_bytes() {
  using FT = FormT<FORM>;
  constexpr int LDK = BK + 16 / sizeof(typename FT::S);
  return 2 * FT::P * (16 * NB + 64 * FB) * LDK * sizeof(typename FT::S);
}

// One output tile (fiber block bx, n block by) of a mu-mode product,
// computed by the 256 threads of a workgroup; `lds` holds
// mode_lds_bytes<...>() bytes, 16-byte aligned.
// PF: prefetch distance in k-chunks (1 or 2). With 2, two register sets
// alternate so the global loads of chunk c+2 are in flight while chunk c
// computes (LDS stays double buffered).
// VEC: L is k-contiguous (cs = 1) and, in the lead layout, so is X; every
// KV-element group then starts 16-byte aligned and m is a multiple of 16
// bytes' worth of elements, so each group is loaded with 16-byte loads (the
// host checks these conditions).
template <int FORM, int NB, int FB, int BK, bool INNER, int PF = 1, bool VEC = false>
__device__ __forceinline__ void mode_tile(const ModeArgs& a, int64_t bx, int64_t by,
                                          char* __restrict__ lds) {
  using FT = FormT<FORM>;
  using G = typename FT::G;
  using SE = typename FT::S;
  using acc_t = typename FT::acc_t;
  using FragT = Frag<FORM>;
  constexpr int P = FT::P, KV = FT::KV, MK = FT::MK;
  constexpr bool SPLIT = FORM == FORM_BF16X3 || FORM == FORM_BF16X6;
  constexpr int BN = 16 * NB;
  constexpr int BF = 64 * FB;
  constexpr int KG = BK / KV;                 // k groups per row and chunk
  constexpr int LDK = BK + 16 / sizeof(SE);   // row stride: +16 bytes
  constexpr int XT = (BF * KG + kThreads - 1) / kThreads;  // X tasks / thread
  constexpr int LT = (BN * KG + kThreads - 1) / kThreads;  // L tasks / thread
  constexpr int QB = INNER ? NB : FB;  // MFMA row blocks
  constexpr int PB = INNER ? FB : NB;  // MFMA column blocks
  static_assert(BK % MK == 0, "BK must be a multiple of the macro step");
  static_assert(!INNER || kThreads % BF == 0, "BF must divide the block size");

  typedef SE LTile[P][BN][LDK];
  typedef SE XTile[P][BF][LDK];
  LTile* sL = reinterpret_cast<LTile*>(lds);
  XTile* sX = reinterpret_cast<XTile*>(lds + 2 * sizeof(LTile));

  const G* __restrict__ X = static_cast<const G*>(a.X);
  const G* __restrict__ L = static_cast<const G*>(a.L);
  G* __restrict__ Y = static_cast<G*>(a.Y);
  const int64_t Il = a.Il, m = a.m, n = a.n;
  const int64_t F = INNER ? a.Il * a.Ir : a.Ir;
  const int64_t f0 = bx * BF;
  const int64_t i0 = by * BN;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;

  // Staging tasks: one row and one group of KV consecutive k.
  //   X, inner: row = id % BF (consecutive threads walk adjacent fibers),
  //             kg = id / BF.
  //   X, lead : kg = id % KG, row = id / KG (threads walk along k).
  //   L       : kg = id % KG, row = id / KG.
  // Every element's byte offset from the chunk's uniform base pointer is
  // fixed for the whole k loop, so it is computed once here (32-bit: the
  // host splits launches so that each stays below 2^31 bytes). Rows past
  // the end are clamped to the last row: they only feed accumulator rows
  // or columns that are never stored. Only the k tail needs zeros.
  // Offsets of each task's first element; element e of the group sits e
  // element strides further (X: Il or 1 elements, L: cs elements), a
  // uniform step passed as the loads' scalar offset.
  uint32_t xo[XT], lo_[LT];
  int xkg[XT], lkg[LT];
  // 32-bit index math: every element offset of X, Y and the span of L are
  // below 2^31 bytes (the host splits launches and checks factor spans)
  const uint32_t Il32 = static_cast<uint32_t>(Il), m32 = static_cast<uint32_t>(m);
  const uint32_t n32 = static_cast<uint32_t>(n), F32 = static_cast<uint32_t>(F);
  const uint32_t f032 = static_cast<uint32_t>(f0), i032 = static_cast<uint32_t>(i0);
  const uint32_t xkstep = INNER ? Il32 : 1;  // elements per unit of k in X
#pragma unroll
  for (int s = 0; s < XT; ++s) {
    const int id = t + s * kThreads;
    uint32_t rowoff;
    int kg;
    if (INNER) {
      kg = (id / BF) % KG;
      uint32_t r = f032 + id % BF;
      r = r < F32 ? r : F32 - 1;
      rowoff = fiber_offset(r, Il32, m32);
    } else {
      kg = id % KG;
      uint32_t f = f032 + (id / KG) % BF;
      f = f < F32 ? f : F32 - 1;
      rowoff = f * m32;
    }
    xkg[s] = kg;
    xo[s] = (rowoff + static_cast<uint32_t>(kg * KV) * xkstep) * static_cast<uint32_t>(sizeof(G));
  }
  const uint32_t rs32 = static_cast<uint32_t>(a.rs), cs32 = static_cast<uint32_t>(a.cs);
#pragma unroll
  for (int s = 0; s < LT; ++s) {
    const int id = t + s * kThreads;
    const int kg = id % KG;
    uint32_t i = i032 + (id / KG) % BN;
    i = i < n32 ? i : n32 - 1;
    lkg[s] = kg;
    // offsets of k past m (tail chunk only) may wrap; they are replaced by
    // an out-of-range offset before use
    lo_[s] = (i * rs32 + static_cast<uint32_t>(kg * KV) * cs32) * static_cast<uint32_t>(sizeof(G));
  }
  static_assert(PF == 1 || PF == 2, "prefetch distance 1 or 2");
  G xr[PF][XT][KV], lr[PF][LT][KV];

  // CHECK: the chunk reaches past k = m; those k read as zero.
  // SET: the register set the chunk is loaded into.
  // Chunk loads go through buffer resources (base and size in scalar
  // registers, built per chunk): each load is the fixed 32-bit per-thread
  // offset, with no per-load address arithmetic. A k past m (CHECK, the last
  // chunk) gets an offset beyond the resource's size, which the hardware
  // answers with zero, so no value is ever selected after it is loaded. The
  // host keeps each launch's operands below 2^31 bytes.
  const uint32_t x_bytes = static_cast<uint32_t>(a.Il * a.m * a.Ir * sizeof(G));
  const uint32_t l_bytes =
      static_cast<uint32_t>(((n - 1) * a.rs + (m - 1) * a.cs + 1) * sizeof(G));
  // byte steps between the KV elements of one task's group
  const uint32_t xes = xkstep * static_cast<uint32_t>(sizeof(G));
  const uint32_t les = cs32 * static_cast<uint32_t>(sizeof(G));
  auto load_chunk = [&](int64_t k0, auto check, auto set) {
    constexpr bool CHECK = decltype(check)::value;
    constexpr int SET = decltype(set)::value;
    constexpr uint32_t kOut = 0x80000000u;  // >= any resource size here
    const uint32_t xk = static_cast<uint32_t>(k0 * xkstep * sizeof(G));
    const uint32_t lk = static_cast<uint32_t>(k0 * a.cs * sizeof(G));
    const auto xrs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(reinterpret_cast<const char*>(X)) + xk, 0, x_bytes - xk, kBufferFlags);
    const auto lrs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(reinterpret_cast<const char*>(L)) + lk, 0, l_bytes - lk, kBufferFlags);
    // a group of KV k values (first k = kb) as 16-byte loads; m is a multiple
    // of 16 bytes' worth of elements, so each 16-byte piece is wholly inside
    // or wholly past k = m (checked on the tail chunk only)
    auto load_group = [&](__amdgpu_buffer_rsrc_t rs, uint32_t off, int64_t kb, G (&dst)[KV]) {
      typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
      constexpr int NQ = KV * sizeof(G) / 16;
      constexpr int PER = 16 / sizeof(G);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        uint32_t o = off + 16 * q;
        if constexpr (CHECK) o = kb + q * PER < m ? o : kOut;
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, static_cast<int>(o), 0, 0);
        typedef G g16 __attribute__((ext_vector_type(16 / sizeof(G))));
        const g16 gv = __builtin_bit_cast(g16, v);
#pragma unroll
        for (int e = 0; e < static_cast<int>(16 / sizeof(G)); ++e)
          dst[q * (16 / sizeof(G)) + e] = gv[e];
      }
    };
#pragma unroll
    for (int s = 0; s < XT; ++s) {
      if constexpr (VEC && !INNER) {
        load_group(xrs, xo[s], k0 + xkg[s] * KV, xr[SET][s]);
      } else {
#pragma unroll
        for (int e = 0; e < KV; ++e) {
          if constexpr (CHECK) {
            const uint32_t off = k0 + xkg[s] * KV + e < m ? xo[s] + e * xes : kOut;
            xr[SET][s][e] = buffer_load<G>(xrs, off);
          } else {
            xr[SET][s][e] = buffer_load<G>(xrs, xo[s], e * xes);
          }
        }
      }
    }
#pragma unroll
    for (int s = 0; s < LT; ++s) {
      if constexpr (VEC) {
        load_group(lrs, lo_[s], k0 + lkg[s] * KV, lr[SET][s]);
      } else {
#pragma unroll
        for (int e = 0; e < KV; ++e) {
          if constexpr (CHECK) {
            const uint32_t off = k0 + lkg[s] * KV + e < m ? lo_[s] + e * les : kOut;
            lr[SET][s][e] = buffer_load<G>(lrs, off);
          } else {
            lr[SET][s][e] = buffer_load<G>(lrs, lo_[s], e * les);
          }
        }
      }
    }
  };
  // Registers -> LDS; the split forms write P bf16 planes.
  auto store_rows = [&](auto& tile, int row, int kg, const G (&v)[KV]) {
    if constexpr (SPLIT) {
      bf16x8_t pl[P];
      split_bf16_group<P, KV>(v, pl);
#pragma unroll
      for (int p = 0; p < P; ++p) *reinterpret_cast<bf16x8_t*>(&tile[p][row][kg * KV]) = pl[p];
    } else {
      FragT f;
#pragma unroll
      for (int e = 0; e < KV; ++e) f[e] = v[e];
      *reinterpret_cast<FragT*>(&tile[0][row][kg * KV]) = f;
    }
  };
  auto store_chunk = [&](int buf, auto set) {
    constexpr int SET = decltype(set)::value;
#pragma unroll
    for (int s = 0; s < XT; ++s) {
      const int id = t + s * kThreads;
      const int row = INNER ? id % BF : id / KG;
      const int kg = INNER ? id / BF : id % KG;
      if (row < BF && kg < KG) store_rows(sX[buf], row, kg, xr[SET][s]);
    }
#pragma unroll
    for (int s = 0; s < LT; ++s) {
      const int id = t + s * kThreads;
      const int row = id / KG;
      const int kg = id % KG;
      if (row < BN) store_rows(sL[buf], row, kg, lr[SET][s]);
    }
  };

  acc_t hi[QB][PB], lo[QB][PB];
#pragma unroll
  for (int q = 0; q < QB; ++q)
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      hi[q][p] = acc_t{};
      lo[q][p] = acc_t{};
    }

  const int c = lane & 15;
  const int g = lane >> 4;
  const int64_t nchunks = (m + BK - 1) / BK;
  const int64_t nfull = m / BK;  // chunks with no k past m
  using Checked = std::true_type;
  using Unchecked = std::false_type;
  using Set0 = std::integral_constant<int, 0>;
  using Set1 = std::integral_constant<int, PF - 1>;
  // load chunk `ch` (k0 = ch*BK) into register set SET, checked only at the tail
  auto load = [&](int64_t ch, auto set) {
    if (ch < nfull)
      load_chunk(ch * BK, Unchecked{}, set);
    else
      load_chunk(ch * BK, Checked{}, set);
  };
  // n blocks of this tile that hold rows below n. A tile computes either all
  // NB blocks or, when at most the first NH hold rows below n (the last n
  // tile), only those NH; the blocks past them hold no output row. NH is
  // NB - 1 for tall tiles (n = 200 with 7-block tiles: 7 + 6 blocks), else
  // half of NB.
  const int nbu = static_cast<int>((n - i0 + 15) / 16);
  constexpr int NH = NB >= 5 ? NB - 1 : (NB + 1) / 2;
  // One chunk's macro steps over the first NBC n blocks: every fragment of a
  // macro step is read from LDS first, then its MFMAs are issued across all
  // blocks (macro_step_grid).
  auto compute_n = [&](int buf, auto nbc) {
    constexpr int NBC = decltype(nbc)::value;
#pragma unroll
    for (int kk = 0; kk < BK; kk += MK) {
      FragT xa[FB][P];
      FragT la[NBC][P];
#pragma unroll
      for (int fb = 0; fb < FB; ++fb)
#pragma unroll
        for (int p = 0; p < P; ++p)
          xa[fb][p] = *reinterpret_cast<const FragT*>(
              &sX[buf][p][w * 16 * FB + fb * 16 + c][kk + KV * g]);
#pragma unroll
      for (int nb = 0; nb < NBC; ++nb)
#pragma unroll
        for (int p = 0; p < P; ++p)
          la[nb][p] = *reinterpret_cast<const FragT*>(&sL[buf][p][nb * 16 + c][kk + KV * g]);
      // A operand = MFMA rows, B = MFMA (memory-contiguous) columns; the
      // accumulators of the first NBC blocks are passed as a grid of their own
      if constexpr (INNER) {
        typename FT::acc_t h[NBC][FB], l[NBC][FB];
#pragma unroll
        for (int nb = 0; nb < NBC; ++nb)
#pragma unroll
          for (int fb = 0; fb < FB; ++fb) {
            h[nb][fb] = hi[nb][fb];
            l[nb][fb] = lo[nb][fb];
          }
        macro_step_grid<FORM, NBC, FB>(la, xa, h, l);
#pragma unroll
        for (int nb = 0; nb < NBC; ++nb)
#pragma unroll
          for (int fb = 0; fb < FB; ++fb) {
            hi[nb][fb] = h[nb][fb];
            lo[nb][fb] = l[nb][fb];
          }
      } else {
        // hi[fb][nb] with NB columns: the first NBC of each row
        typename FT::acc_t h[FB][NBC], l[FB][NBC];
#pragma unroll
        for (int fb = 0; fb < FB; ++fb)
#pragma unroll
          for (int nb = 0; nb < NBC; ++nb) {
            h[fb][nb] = hi[fb][nb];
            l[fb][nb] = lo[fb][nb];
          }
        macro_step_grid<FORM, FB, NBC>(xa, la, h, l);
#pragma unroll
        for (int fb = 0; fb < FB; ++fb)
#pragma unroll
          for (int nb = 0; nb < NBC; ++nb) {
            hi[fb][nb] = h[fb][nb];
            lo[fb][nb] = l[fb][nb];
          }
      }
    }
  };
  // The whole k loop for tiles computing the first NBC n blocks (NBC = NB,
  // or NH for a last n tile with at most NH blocks below n): the two loops
  // are separate code, so each keeps its own register allocation.
  auto kloop = [&](auto nbc) {
  auto compute = [&](int buf) { compute_n(buf, nbc); };
  if constexpr (PF == 1) {
    if (nchunks > 0) {
      load(0, Set0{});
      store_chunk(0, Set0{});
    }
    __syncthreads();
    for (int64_t ch = 0; ch < nchunks; ++ch) {
      const int buf = static_cast<int>(ch & 1);
      if (ch + 1 < nchunks) load(ch + 1, Set0{});
      compute(buf);
      if (ch + 1 < nchunks) store_chunk(buf ^ 1, Set0{});
      __syncthreads();
    }
  } else {
    // set 0 carries even chunks, set 1 odd ones; chunk c is loaded two
    // chunks before it is computed and stored to LDS one chunk before
    if (nchunks > 0) {
      load(0, Set0{});
      if (nchunks > 1) load(1, Set1{});
      store_chunk(0, Set0{});
    }
    __syncthreads();
    int64_t ch = 0;
    // Steady state: the two chunks loaded per pass (ch + 2, ch + 3) are full,
    // so their loads carry no k check and sit in no branch; each LDS store
    // then waits only for its own register set while the other set's loads
    // stay in flight. Entry and exit state: LDS buffer 0 holds chunk ch and
    // set 1 holds chunk ch + 1.
    for (; ch + 3 < nfull; ch += 2) {
      load_chunk((ch + 2) * BK, Unchecked{}, Set0{});
      compute(0);
      store_chunk(1, Set1{});
      __syncthreads();
      load_chunk((ch + 3) * BK, Unchecked{}, Set1{});
      compute(1);
      store_chunk(0, Set0{});
      __syncthreads();
    }
    for (; ch < nchunks; ch += 2) {
      if (ch + 2 < nchunks) load(ch + 2, Set0{});
      compute(0);
      if (ch + 1 < nchunks) store_chunk(1, Set1{});
      __syncthreads();
      if (ch + 1 >= nchunks) break;
      if (ch + 3 < nchunks) load(ch + 3, Set1{});
      compute(1);
      if (ch + 2 < nchunks) store_chunk(0, Set0{});
      __syncthreads();
    }
  }
  };
  if (NH < NB && nbu <= NH)
    kloop(std::integral_constant<int, NH>{});
  else
    kloop(std::integral_constant<int, NB>{});

  // Store: MFMA column = lane & 15 is the memory-contiguous output index.
  // Through a buffer resource over Y: rows past n and fibers past F get an
  // offset past the resource, and the hardware drops the store.
  constexpr uint32_t kDrop = 0x80000000u;  // >= any resource size here
  const auto yrs = __builtin_amdgcn_make_buffer_rsrc(
      Y, 0, static_cast<int>(a.Il * a.n * a.Ir * sizeof(G)), kBufferFlags);
  constexpr uint32_t ES = static_cast<uint32_t>(sizeof(G));
#pragma unroll
  for (int q = 0; q < QB; ++q)
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      acc_t val = hi[q][p];
      if constexpr (SPLIT) val = hi[q][p] + lo[q][p];
      uint32_t off[4];
      if constexpr (INNER) {
        const uint32_t r = f032 + w * 16 * FB + p * 16 + c;
        const uint32_t yb = fiber_offset(r < F32 ? r : 0, Il32, n32);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const uint32_t i = i032 + q * 16 + FT::row(lane, v);
          off[v] = (r < F32 && i < n32) ? (yb + Il32 * i) * ES : kDrop;
        }
      } else {
        const uint32_t i = i032 + p * 16 + c;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const uint32_t f = f032 + w * 16 * FB + q * 16 + FT::row(lane, v);
          off[v] = (f < F32 && i < n32) ? (i + n32 * f) * ES : kDrop;
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) store_out<INNER, G>(val[v], yrs, off[v], a.accumulate, c);
    }
}

}  // namespace tile
}  // namespace kp
