// Wide tile of the mu-mode product for the BF16 split forms (Sec. 2,
// Definition of the mu-mode product), gfx950.
//
// A v_mfma_f32_16x16x32_bf16 product of two 16 x 32 operand fragments takes
// 16 cycles, and each split product needs P = 2 (BF16x3) or 3 (BF16x6) bf16
// planes of both fragments: a wave whose output block is small spends far
// more time fetching operands than multiplying them. Here each wave owns a
// 64 x 64 output block (16 MFMA blocks, hi and lo accumulators), and the two
// operands take different paths so that neither path carries both:
//   * the factor rows a wave multiplies belong to that wave alone (the four
//     waves split the n rows of the workgroup tile), so each wave loads its
//     rows of L straight from global memory (L is small and stays in L2)
//     and splits them in registers, one 32-wide k step ahead;
//   * the input fibers are shared by the four waves, so they are staged once
//     per workgroup through LDS as bf16 planes (split at staging), double
//     buffered, with two chunks of global loads in flight.
// The products per accumulator are issued in the same order as in
// mode_tile.h (same k steps, same split, same slot order), so the result
// equals that of the k-loop tile with 32-wide chunks bit for bit.
#pragma once

#include "mode_tile.h"

namespace kp {
namespace tile {

// NBW: 16-row blocks of n per wave; WN: waves along n (the workgroup covers
// 16*NBW*WN rows); FBW: 16-fiber blocks per wave; the 4/WN wave columns
// split the fibers (the workgroup covers 16*FBW*(4/WN) fibers). BK: k values
// per LDS chunk (a multiple of 32).
template <int FORM, int FBW, int WN, int BK>
constexpr size_t wide_lds_bytes() {
  return 2 * FormT<FORM>::P * (16 * FBW * (4 / WN)) * (BK + 8) * sizeof(__bf16);
}

template <int FORM, int NBW, int FBW, int WN, int BK, bool INNER, bool VEC>
__device__ __forceinline__ void wide_tile(const ModeArgs& a, int64_t bx, int64_t by,
                                          char* __restrict__ lds) {
  static_assert(FORM == FORM_BF16X3 || FORM == FORM_BF16X6, "split forms only");
  using FT = FormT<FORM>;
  using acc_t = f4_t;
  constexpr int P = FT::P, KV = 8, MK = 32;
  constexpr int WF = 4 / WN;
  constexpr int BN = 16 * NBW * WN;
  constexpr int BF = 16 * FBW * WF;
  constexpr int KG = BK / KV;          // k groups per fiber and chunk
  constexpr int KS = BK / MK;          // k steps per chunk
  constexpr int LDK = BK + 8;          // row stride: +16 bytes
  constexpr int XT = (BF * KG + kThreads - 1) / kThreads;
  static_assert(WN * WF == 4 && BK % MK == 0, "tile shape");
  static_assert(!INNER || kThreads % BF == 0, "BF must divide the block size");

  typedef __bf16 XTile[P][BF][LDK];
  XTile* sX = reinterpret_cast<XTile*>(lds);

  const float* __restrict__ X = static_cast<const float*>(a.X);
  const float* __restrict__ L = static_cast<const float*>(a.L);
  float* __restrict__ Y = static_cast<float*>(a.Y);
  const int64_t m = a.m, n = a.n;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int wn = w % WN, wf = w / WN;
  const int c = lane & 15;
  const int g = lane >> 4;

  // 32-bit offsets: every operand of a launch is below 2^31 bytes (the host
  // splits launches and checks factor spans)
  const uint32_t Il32 = static_cast<uint32_t>(a.Il), m32 = static_cast<uint32_t>(m);
  const uint32_t n32 = static_cast<uint32_t>(n);
  const uint32_t F32 = static_cast<uint32_t>(INNER ? a.Il * a.Ir : a.Ir);
  const uint32_t f032 = static_cast<uint32_t>(bx * BF), i032 = static_cast<uint32_t>(by * BN);

  // X staging tasks (as in mode_tile): inner: row = id % BF, kg = id / BF;
  // lead: kg = id % KG, row = id / KG; rows past the end read the last one.
  const uint32_t xkstep = INNER ? Il32 : 1;
  uint32_t xo[XT];
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
    xo[s] = (rowoff + static_cast<uint32_t>(kg * KV) * xkstep) * 4u;
  }
  auto xkg = [&](int s) {
    const int id = t + s * kThreads;
    return INNER ? (id / BF) % KG : id % KG;
  };
  // This wave's factor rows: row nb*16 + c of its n blocks, k values
  // 8g .. 8g+7 of each step (the MFMA fragment layout of both operands).
  const uint32_t rs32 = static_cast<uint32_t>(a.rs), cs32 = static_cast<uint32_t>(a.cs);
  uint32_t lofs[NBW];
#pragma unroll
  for (int nb = 0; nb < NBW; ++nb) {
    uint32_t i = i032 + (wn * NBW + nb) * 16 + c;
    i = i < n32 ? i : n32 - 1;
    lofs[nb] = (i * rs32 + static_cast<uint32_t>(KV * g) * cs32) * 4u;
  }

  constexpr uint32_t kOut = 0x80000000u;  // >= any resource size here
  const uint32_t x_bytes = static_cast<uint32_t>(a.Il * m * a.Ir * 4);
  const uint32_t l_bytes = static_cast<uint32_t>(((n - 1) * a.rs + (m - 1) * a.cs + 1) * 4);
  const uint32_t xes = xkstep * 4u;  // bytes between consecutive k of a fiber
  const uint32_t les = cs32 * 4u;    // bytes between consecutive k of a row of L
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  typedef float f4v __attribute__((ext_vector_type(4)));

  float xr[2][XT][KV];
  float lv[NBW][KV];

  // Chunk ch of X (k0 = ch*BK) into register set SET; CHECK: the chunk
  // reaches past k = m (those k read as zero through the resource bound).
  auto load_x = [&](int64_t ch, auto set, auto check) {
    constexpr int SET = decltype(set)::value;
    constexpr bool CHECK = decltype(check)::value;
    const int64_t k0 = ch * BK;
    const uint32_t xk = static_cast<uint32_t>(k0 * xkstep * 4);
    const auto rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(reinterpret_cast<const char*>(X)) + xk, 0, x_bytes - xk, kBufferFlags);
#pragma unroll
    for (int s = 0; s < XT; ++s) {
      const int64_t kb = k0 + xkg(s) * KV;
      if constexpr (VEC && !INNER) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          uint32_t o = xo[s] + 16 * q;
          if constexpr (CHECK) o = kb + 4 * q < m ? o : kOut;
          const f4v v = __builtin_bit_cast(
              f4v, __builtin_amdgcn_raw_buffer_load_b128(rs, static_cast<int>(o), 0, 0));
#pragma unroll
          for (int e = 0; e < 4; ++e) xr[SET][s][4 * q + e] = v[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < KV; ++e) {
          if constexpr (CHECK)
            xr[SET][s][e] = buffer_load<float>(rs, kb + e < m ? xo[s] + e * xes : kOut);
          else
            xr[SET][s][e] = buffer_load<float>(rs, xo[s], e * xes);
        }
      }
    }
  };
  // Register set SET -> LDS buffer BUF as P bf16 planes.
  auto store_x = [&](int buf, auto set) {
    constexpr int SET = decltype(set)::value;
#pragma unroll
    for (int s = 0; s < XT; ++s) {
      const int id = t + s * kThreads;
      const int row = INNER ? id % BF : id / KG;
      const int kg = INNER ? id / BF : id % KG;
      if (XT * kThreads == BF * KG || (row < BF && kg < KG)) {
        bf16x8_t pl[P];
        split_bf16_group<P, KV>(xr[SET][s], pl);
#pragma unroll
        for (int p = 0; p < P; ++p)
          *reinterpret_cast<bf16x8_t*>(&sX[buf][p][row][kg * KV]) = pl[p];
      }
    }
  };
  // k step s (k0 = 32 s) of this wave's factor rows into lv.
  auto load_l = [&](int64_t s, auto check) {
    constexpr bool CHECK = decltype(check)::value;
    const int64_t k0 = s * MK;
    const uint32_t lk = static_cast<uint32_t>(k0 * a.cs * 4);
    const auto rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(reinterpret_cast<const char*>(L)) + lk, 0, l_bytes - lk, kBufferFlags);
    const int64_t kb = k0 + KV * g;
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) {
      if constexpr (VEC) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          uint32_t o = lofs[nb] + 16 * q;
          if constexpr (CHECK) o = kb + 4 * q < m ? o : kOut;
          const f4v v = __builtin_bit_cast(
              f4v, __builtin_amdgcn_raw_buffer_load_b128(rs, static_cast<int>(o), 0, 0));
#pragma unroll
          for (int e = 0; e < 4; ++e) lv[nb][4 * q + e] = v[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < KV; ++e) {
          if constexpr (CHECK)
            lv[nb][e] = buffer_load<float>(rs, kb + e < m ? lofs[nb] + e * les : kOut);
          else
            lv[nb][e] = buffer_load<float>(rs, lofs[nb], e * les);
        }
      }
    }
  };

  acc_t hi[INNER ? NBW : FBW][INNER ? FBW : NBW], lo[INNER ? NBW : FBW][INNER ? FBW : NBW];
#pragma unroll
  for (int q = 0; q < (INNER ? NBW : FBW); ++q)
#pragma unroll
    for (int p = 0; p < (INNER ? FBW : NBW); ++p) {
      hi[q][p] = acc_t{};
      lo[q][p] = acc_t{};
    }

  const int64_t nchunks = (m + BK - 1) / BK;
  const int64_t nfull = m / BK;   // chunks with no k past m
  const int64_t nsteps = (m + MK - 1) / MK;
  const int64_t lfull = m / MK;   // k steps with no k past m
  using Checked = std::true_type;
  using Unchecked = std::false_type;
  using Set0 = std::integral_constant<int, 0>;
  using Set1 = std::integral_constant<int, 1>;

  // One k step from LDS buffer buf at chunk offset kk: split this step's
  // factor rows, start loading the next step's, read the fibers' planes and
  // issue the products. STEADY: the next step is full (no check, no branch).
  auto step = [&](int buf, int kk, int64_t s, auto steady) {
    constexpr bool STEADY = decltype(steady)::value;
    bf16x8_t la[NBW][P];
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) split_bf16_group<P, KV>(lv[nb], la[nb]);
    if constexpr (STEADY) {
      load_l(s + 1, Unchecked{});
    } else if (s + 1 < nsteps) {
      if (s + 1 < lfull)
        load_l(s + 1, Unchecked{});
      else
        load_l(s + 1, Checked{});
    }
    bf16x8_t xa[FBW][P];
#pragma unroll
    for (int fb = 0; fb < FBW; ++fb)
#pragma unroll
      for (int p = 0; p < P; ++p)
        xa[fb][p] = *reinterpret_cast<const bf16x8_t*>(
            &sX[buf][p][wf * 16 * FBW + fb * 16 + c][kk + KV * g]);
    if constexpr (INNER)
      macro_step_grid<FORM, NBW, FBW>(la, xa, hi, lo);
    else
      macro_step_grid<FORM, FBW, NBW>(xa, la, hi, lo);
  };
  // Chunk ch (parity PAR = ch % 2: LDS buffer and the register set it was
  // loaded into). STEADY: chunk ch + 2 is full and exists, so every load of
  // the iteration is unconditional and unchecked.
  auto iter = [&](int64_t ch, auto par, auto steady) {
    constexpr int PAR = decltype(par)::value;
    constexpr bool STEADY = decltype(steady)::value;
    using SetP = std::integral_constant<int, PAR>;
    using SetQ = std::integral_constant<int, PAR ^ 1>;
    if constexpr (STEADY) {
      load_x(ch + 2, SetP{}, Unchecked{});
    } else if (ch + 2 < nchunks) {
      if (ch + 2 < nfull)
        load_x(ch + 2, SetP{}, Unchecked{});
      else
        load_x(ch + 2, SetP{}, Checked{});
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int64_t s = ch * KS + ks;
      if constexpr (STEADY)
        step(PAR, ks * MK, s, std::true_type{});
      else if (s < nsteps)
        step(PAR, ks * MK, s, std::false_type{});
    }
    if constexpr (STEADY)
      store_x(PAR ^ 1, SetQ{});
    else if (ch + 1 < nchunks)
      store_x(PAR ^ 1, SetQ{});
    __syncthreads();
  };

  if (nchunks > 0) {
    if (nfull > 0)
      load_x(0, Set0{}, Unchecked{});
    else
      load_x(0, Set0{}, Checked{});
    if (nchunks > 1) {
      if (nfull > 1)
        load_x(1, Set1{}, Unchecked{});
      else
        load_x(1, Set1{}, Checked{});
    }
    if (lfull > 0)
      load_l(0, Unchecked{});
    else
      load_l(0, Checked{});
    store_x(0, Set0{});
  }
  __syncthreads();
  int64_t ch = 0;
  for (; ch + 3 < nfull; ch += 2) {
    iter(ch, Set0{}, std::true_type{});
    iter(ch + 1, Set1{}, std::true_type{});
  }
  for (; ch < nchunks; ch += 2) {
    iter(ch, Set0{}, std::false_type{});
    if (ch + 1 < nchunks) iter(ch + 1, Set1{}, std::false_type{});
  }

  // Store (as mode_tile): the MFMA column lane & 15 is the memory-contiguous
  // output index; rows past n and fibers past F get an offset past the
  // resource and the hardware drops the store.
  constexpr uint32_t kDrop = 0x80000000u;
  const auto yrs = __builtin_amdgcn_make_buffer_rsrc(
      Y, 0, static_cast<int>(a.Il * n * a.Ir * 4), kBufferFlags);
#pragma unroll
  for (int q = 0; q < (INNER ? NBW : FBW); ++q)
#pragma unroll
    for (int p = 0; p < (INNER ? FBW : NBW); ++p) {
      const acc_t val = hi[q][p] + lo[q][p];
      uint32_t off[4];
      if constexpr (INNER) {
        const uint32_t r = f032 + wf * 16 * FBW + p * 16 + c;
        const uint32_t yb = fiber_offset(r < F32 ? r : 0, Il32, n32);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const uint32_t i = i032 + (wn * NBW + q) * 16 + FT::row(lane, v);
          off[v] = (r < F32 && i < n32) ? (yb + Il32 * i) * 4u : kDrop;
        }
      } else {
        const uint32_t i = i032 + (wn * NBW + p) * 16 + c;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const uint32_t f = f032 + wf * 16 * FBW + q * 16 + FT::row(lane, v);
          off[v] = (f < F32 && i < n32) ? (i + n32 * f) * 4u : kDrop;
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) store_out<INNER, float>(val[v], yrs, off[v], a.accumulate, c);
    }
}

}  // namespace tile
}  // namespace kp
