// Strip tile of the mu-mode product for short contractions (m <= KP <= 64),
// the HBM-bound regime (Sec. 2, Definition of the mu-mode product; the
// small-factor products of the interpolation and batched workloads).
//
// The whole contraction fits one LDS chunk, so instead of a k loop a
// workgroup keeps its block of BN rows of L (all m columns) in LDS for its
// whole life and streams a sequence of fiber tiles through double-buffered
// LDS: the global loads of the next tile are in flight while the current
// tile computes and its outputs are stored. One barrier per tile.
#pragma once

#include "mode_tile.h"

namespace kp {
namespace tile {

template <int FORM, int NB, int FB, int KP>
constexpr size_t strip_lds_bytes() {
  using FT = FormT<FORM>;
  constexpr int LDK = KP + 16 / sizeof(typename FT::S);
  return FT::P * (16 * NB + 2 * 64 * FB) * LDK * sizeof(typename FT::S);
}

// Fiber tiles bx = t0, t0 + tstep, ... < ntiles of n block `by`.
// VEC (lead layout only): every fiber row starts 16-byte aligned (m is a
// multiple of 16 bytes' worth of elements), so each staging task is a few
// 16-byte loads.
template <int FORM, int NB, int FB, int KP, bool INNER, bool VEC>
__device__ __forceinline__ void strip_run(const ModeArgs& a, int64_t by, int64_t t0,
                                          int64_t tstep, int64_t ntiles,
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
  constexpr int KG = KP / KV;
  constexpr int LDK = KP + 16 / sizeof(SE);
  constexpr int XT = (BF * KG + kThreads - 1) / kThreads;
  constexpr int LT = (BN * KG + kThreads - 1) / kThreads;
  constexpr int QB = INNER ? NB : FB;
  constexpr int PB = INNER ? FB : NB;
  static_assert(KP % MK == 0, "KP must be a multiple of the macro step");
  static_assert(!INNER || kThreads % BF == 0, "BF must divide the block size");
  static_assert(!(INNER && VEC), "vector loads are for the lead layout");

  typedef SE LTile[P][BN][LDK];
  typedef SE XTile[P][BF][LDK];
  LTile& sL = *reinterpret_cast<LTile*>(lds);
  XTile* sX = reinterpret_cast<XTile*>(lds + sizeof(LTile));

  const G* __restrict__ L = static_cast<const G*>(a.L);
  // 32-bit index math: the host keeps every launch below 2^31 bytes
  const uint32_t Il = static_cast<uint32_t>(a.Il), m = static_cast<uint32_t>(a.m);
  const uint32_t n = static_cast<uint32_t>(a.n);
  const uint32_t F = static_cast<uint32_t>(INNER ? a.Il * a.Ir : a.Ir);
  const uint32_t i0 = static_cast<uint32_t>(by) * BN;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int c = lane & 15;
  const int g = lane >> 4;

  // Staging tasks (row, k group), fixed for the workgroup's life:
  //   X inner: row = id % BF, kg = id / BF;  X lead and L: kg = id % KG, row = id / KG.
  int xrow[XT], xkg[XT];
#pragma unroll
  for (int s = 0; s < XT; ++s) {
    const int id = t + s * kThreads;
    xrow[s] = INNER ? id % BF : (id / KG) % BF;
    xkg[s] = INNER ? (id / BF) % KG : id % KG;
  }

  // L block -> LDS once (k >= m and rows >= n read as zero).
  {
    G lr[LT][KV];
#pragma unroll
    for (int s = 0; s < LT; ++s) {
      const int id = t + s * kThreads;
      const uint32_t i = i0 + (id / KG) % BN;
      const int kg = id % KG;
#pragma unroll
      for (int e = 0; e < KV; ++e) {
        const uint32_t k = kg * KV + e;
        lr[s][e] = (i < n && k < m) ? L[static_cast<int64_t>(i) * a.rs + k * a.cs] : G(0);
      }
    }
#pragma unroll
    for (int s = 0; s < LT; ++s) {
      const int id = t + s * kThreads;
      const int row = id / KG, kg = id % KG;
      if (row >= BN) continue;
      if constexpr (SPLIT) {
        bf16x8_t pl[P];
        split_bf16_group<P, KV>(lr[s], pl);
#pragma unroll
        for (int p = 0; p < P; ++p) *reinterpret_cast<bf16x8_t*>(&sL[p][row][kg * KV]) = pl[p];
      } else {
        FragT f;
#pragma unroll
        for (int e = 0; e < KV; ++e) f[e] = lr[s][e];
        *reinterpret_cast<FragT*>(&sL[0][row][kg * KV]) = f;
      }
    }
  }

  // BF16x6 (the most arithmetic per tile): two register sets, the loads of
  // tile bx + 2 tstep in flight while tile bx is computed and tile
  // bx + tstep waits in the other set; the other forms keep one set (the
  // second one measured no faster, FP64 slower)
  constexpr bool PF2 = FORM == FORM_BF16X6;
  G xr[PF2 ? 2 : 1][XT][KV];
  // Global -> registers for fiber tile bx, through a buffer resource over
  // the launch's X (32-bit offsets, no per-load address arithmetic). Fibers
  // past F are clamped to the last one (their outputs are never stored); a
  // k at or past m gets an offset past the resource and reads as zero.
  constexpr uint32_t kOut = 0x80000000u;  // >= any resource size here
  const auto xrs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.X), 0, static_cast<int>(a.Il * a.m * a.Ir * sizeof(G)), kBufferFlags);
  const auto yrs = __builtin_amdgcn_make_buffer_rsrc(
      a.Y, 0, static_cast<int>(a.Il * a.n * a.Ir * sizeof(G)), kBufferFlags);
  auto load_x = [&](int64_t bx, auto set) {
    constexpr int SET = decltype(set)::value;
    const uint32_t f0 = static_cast<uint32_t>(bx) * BF;
#pragma unroll
    for (int s = 0; s < XT; ++s) {
      uint32_t r = f0 + xrow[s];
      r = r < F ? r : F - 1;
      uint32_t base;
      if constexpr (INNER) {
        const uint32_t b = r / Il;
        base = (r - b * Il) + Il * m * b;
      } else {
        base = r * m;
      }
      const uint32_t kb = xkg[s] * KV;
      if constexpr (VEC) {
        typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
        typedef G g16 __attribute__((ext_vector_type(16 / sizeof(G))));
        constexpr int NQ = KV * sizeof(G) / 16;
        constexpr int PER = 16 / sizeof(G);
        // each 16-byte piece lies wholly inside or wholly past k = m
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const uint32_t off = kb + q * PER < m ? (base + kb) * sizeof(G) + 16 * q : kOut;
          const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(xrs, static_cast<int>(off), 0, 0);
          const g16 gv = __builtin_bit_cast(g16, v);
#pragma unroll
          for (int e = 0; e < PER; ++e) xr[SET][s][q * PER + e] = gv[e];
        }
      } else {
        const uint32_t ks = INNER ? Il : 1;
#pragma unroll
        for (int e = 0; e < KV; ++e) {
          const uint32_t k = kb + e;
          xr[SET][s][e] = buffer_load<G>(xrs, k < m ? (base + k * ks) * sizeof(G) : kOut);
        }
      }
    }
  };
  auto store_x = [&](int buf, auto set) {
    constexpr int SET = decltype(set)::value;
#pragma unroll
    for (int s = 0; s < XT; ++s) {
      const int id = t + s * kThreads;
      if (id >= BF * KG) continue;
      const int row = xrow[s], kg = xkg[s];
      if constexpr (SPLIT) {
        bf16x8_t pl[P];
        split_bf16_group<P, KV>(xr[SET][s], pl);
#pragma unroll
        for (int p = 0; p < P; ++p)
          *reinterpret_cast<bf16x8_t*>(&sX[buf][p][row][kg * KV]) = pl[p];
      } else {
        FragT f;
#pragma unroll
        for (int e = 0; e < KV; ++e) f[e] = xr[SET][s][e];
        *reinterpret_cast<FragT*>(&sX[buf][0][row][kg * KV]) = f;
      }
    }
  };

  using Set0 = std::integral_constant<int, 0>;
  using Set1 = std::integral_constant<int, 1>;
  if (t0 < ntiles) {
    load_x(t0, Set0{});
    if constexpr (PF2)
      if (t0 + tstep < ntiles) load_x(t0 + tstep, Set1{});
    store_x(0, Set0{});
  }
  __syncthreads();
  int buf = 0;
  // tile bx from LDS buffer `buf`. PF2: set CUR is free (its tile is in
  // LDS) and takes tile bx + 2 tstep, set NXT holds tile bx + tstep; else
  // the one set takes tile bx + tstep
  auto step = [&](int64_t bx, auto cur, auto nxt) {
    const int64_t nx = bx + tstep;
    if constexpr (PF2) {
      if (nx + tstep < ntiles) load_x(nx + tstep, cur);
    } else {
      if (nx < ntiles) load_x(nx, nxt);
    }
    acc_t hi[QB][PB], lo[QB][PB];
#pragma unroll
    for (int q = 0; q < QB; ++q)
#pragma unroll
      for (int p = 0; p < PB; ++p) {
        hi[q][p] = acc_t{};
        lo[q][p] = acc_t{};
      }
#pragma unroll
    for (int kk = 0; kk < KP; kk += MK) {
      FragT xa[FB][P];
#pragma unroll
      for (int fb = 0; fb < FB; ++fb)
#pragma unroll
        for (int p = 0; p < P; ++p)
          xa[fb][p] = *reinterpret_cast<const FragT*>(
              &sX[buf][p][w * 16 * FB + fb * 16 + c][kk + KV * g]);
      FragT la[NB][P];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int p = 0; p < P; ++p)
          la[nb][p] = *reinterpret_cast<const FragT*>(&sL[p][nb * 16 + c][kk + KV * g]);
      // products issued slot by slot across the blocks (macro_step_grid)
      if constexpr (INNER)
        macro_step_grid<FORM, NB, FB>(la, xa, hi, lo);
      else
        macro_step_grid<FORM, FB, NB>(xa, la, hi, lo);
    }
    // outputs of this tile (MFMA column = memory-contiguous index), through a
    // buffer resource over Y: rows past n and fibers past F get an offset
    // past the resource and the hardware drops the store
#pragma unroll
    for (int q = 0; q < QB; ++q)
#pragma unroll
      for (int p = 0; p < PB; ++p) {
        acc_t val = hi[q][p];
        if constexpr (SPLIT) val = hi[q][p] + lo[q][p];
        const uint32_t f0 = static_cast<uint32_t>(bx) * BF;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          uint32_t off;
          if constexpr (INNER) {
            const uint32_t r = f0 + w * 16 * FB + p * 16 + c;
            const uint32_t i = i0 + q * 16 + FT::row(lane, v);
            const uint32_t b = r / Il;
            off = (r < F && i < n) ? ((r - b * Il) + Il * n * b + Il * i) * sizeof(G) : kOut;
          } else {
            const uint32_t i = i0 + p * 16 + c;
            const uint32_t f = f0 + w * 16 * FB + q * 16 + FT::row(lane, v);
            off = (f < F && i < n) ? (i + n * f) * sizeof(G) : kOut;
          }
          store_out<INNER, G>(val[v], yrs, off, a.accumulate, c);
        }
      }
    if (nx < ntiles) store_x(buf ^ 1, nxt);
    __syncthreads();
    buf ^= 1;
  };
  int64_t bx = t0;
  if constexpr (PF2) {
    for (; bx + tstep < ntiles; bx += 2 * tstep) {
      step(bx, Set0{}, Set1{});
      step(bx + tstep, Set1{}, Set0{});
    }
    if (bx < ntiles) step(bx, Set0{}, Set1{});
  } else {
    for (; bx < ntiles; bx += tstep) step(bx, Set0{}, Set0{});
  }
}

}  // namespace tile
}  // namespace kp
