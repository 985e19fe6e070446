// Wide tile of the mu-mode product (Sec. 2, Definition of the mu-mode
// product), gfx950, all forms.
//
// The k-loop tile (mode_tile.h) stages both operands through LDS and lets
// every wave read every factor row of the workgroup. Here the four waves
// split the n rows instead, so the two operands take different paths:
//   * the factor rows a wave multiplies belong to that wave alone, so each
//     wave loads its rows of L straight from global memory (L is small and
//     stays in L2), one k step ahead, and builds its MFMA fragments in
//     registers (the BF16 split forms split them there);
//   * the input fibers are shared by the four waves, so they are staged once
//     per workgroup through LDS (as bf16 planes for the split forms), double
//     buffered, with two chunks of global loads in flight.
// A Tucker call may split every factor once instead (split_planes below):
// the wave then loads its rows' fragments as bf16 planes (PRE), the same
// values the in-register split gives.
// No factor chunk is written to or read from LDS, and each wave issues more
// products per barrier. This pays for the split forms, whose products are
// short next to their operand fetches; the FP64 and FP32 forms, compiled
// from the same code, measured no faster than the k-loop tile and are not
// instantiated. The products per accumulator are issued in the same
// order as in mode_tile.h (same k steps and lane-group k ownership, same
// split, same slot order), so the result equals that of the k-loop tile
// with the same chunk width bit for bit.
#pragma once

#include "mode_tile.h"

namespace kp {
namespace tile {

// NBW: 16-row blocks of n per wave; WN: waves along n (the workgroup covers
// 16*NBW*WN rows); FBW: 16-fiber blocks per wave; the 4/WN wave columns
// split the fibers (the workgroup covers 16*FBW*(4/WN) fibers). BK: k values
// per LDS chunk (a multiple of the form's macro step: 8 FP64, 16 FP32, 32
// BF16).
template <int FORM, int FBW, int WN, int BK>
constexpr size_t wide_lds_bytes() {
  using SE = typename FormT<FORM>::S;
  return 2 * FormT<FORM>::P * (16 * FBW * (4 / WN)) * (BK + 16 / sizeof(SE)) * sizeof(SE);
}

// Store of one value at per-lane byte offset off plus the wave-uniform
// byte offset soff (the instruction's scalar offset).
template <typename G>
__device__ __forceinline__ void buffer_store_at(G v, __amdgpu_buffer_rsrc_t rs, uint32_t off,
                                                uint32_t soff) {
  if constexpr (sizeof(G) == 8) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, static_cast<int>(off),
                                          static_cast<int>(soff), 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), rs,
                                          static_cast<int>(off), static_cast<int>(soff), 0);
  }
}

// Pre-split factor planes (split forms): for every 16-row block of L
// (ceil(n/16) blocks), every 32-wide k step (ceil(m/32)) and every plane,
// the 64 lanes' MFMA fragments, lane l holding rows 16 b + l % 16 and k
// values 32 s + 8 (l / 16) .. + 7 (zero past k = m): 1 KB per (block,
// step, plane), stored in that order.
template <int FORM>
__host__ __device__ constexpr int64_t split_plane_frags(int64_t n, int64_t m) {
  return ((n + 15) / 16) * ((m + 31) / 32) * FormT<FORM>::P * 64;
}

// One lane's fragments (all planes) of block b, step s of L (FP32, element
// (i, k) at L[i rs + k cs], n x m), written to planes.
template <int FORM>
__device__ __forceinline__ void split_planes_lane(const float* __restrict__ L, int64_t n, int64_t m,
                                                  int64_t rs, int64_t cs, int64_t b, int64_t s,
                                                  int lane, bf16x8_t* __restrict__ planes) {
  constexpr int P = FormT<FORM>::P;
  int64_t i = 16 * b + (lane & 15);
  i = i < n ? i : n - 1;
  float v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t k = 32 * s + 8 * (lane >> 4) + e;
    v[e] = k < m ? L[i * rs + k * cs] : 0.0f;
  }
  bf16x8_t pl[P];
  split_bf16_group<P, 8>(v, pl);
  const int64_t steps = (m + 31) / 32;
#pragma unroll
  for (int p = 0; p < P; ++p) planes[((b * steps + s) * P + p) * 64 + lane] = pl[p];
}

template <int FORM, int NBW, int FBW, int WN, int BK, bool INNER, bool VEC, bool PRE = false>
__device__ __forceinline__ void wide_tile(const ModeArgs& a, int64_t bx, int64_t by,
                                          char* __restrict__ lds) {
  using FT = FormT<FORM>;
  using G = typename FT::G;
  using SE = typename FT::S;
  using acc_t = typename FT::acc_t;
  using FragT = Frag<FORM>;
  constexpr bool SPLIT = FORM == FORM_BF16X3 || FORM == FORM_BF16X6;
  constexpr int P = FT::P, KV = FT::KV, MK = FT::MK;
  constexpr uint32_t ES = sizeof(G);
  constexpr int PER = 16 / sizeof(G);  // elements per 16-byte piece
  constexpr int WF = 4 / WN;
  constexpr int BN = 16 * NBW * WN;
  constexpr int BF = 16 * FBW * WF;
  constexpr int KG = BK / KV;          // k groups per fiber and chunk
  constexpr int KS = BK / MK;          // k steps per chunk
  constexpr int LDK = BK + 16 / static_cast<int>(sizeof(SE));  // row stride: +16 bytes
  constexpr int XT = (BF * KG + kThreads - 1) / kThreads;
  static_assert(WN * WF == 4 && BK % MK == 0, "tile shape");
  static_assert(!PRE || SPLIT, "pre-split planes are for the split forms");
  static_assert(!INNER || kThreads % BF == 0, "BF must divide the block size");

  typedef SE XTile[P][BF][LDK];
  XTile* sX = reinterpret_cast<XTile*>(lds);

  const G* __restrict__ X = static_cast<const G*>(a.X);
  const G* __restrict__ L = static_cast<const G*>(a.L);
  G* __restrict__ Y = static_cast<G*>(a.Y);
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
    xo[s] = (rowoff + static_cast<uint32_t>(kg * KV) * xkstep) * ES;
  }
  auto xkg = [&](int s) {
    const int id = t + s * kThreads;
    return INNER ? (id / BF) % KG : id % KG;
  };
  // This wave's factor rows: row nb*16 + c of its n blocks, k values
  // KV*g .. KV*g + KV-1 of each macro step (the MFMA fragment layout of
  // both operands).
  const uint32_t rs32 = static_cast<uint32_t>(a.rs), cs32 = static_cast<uint32_t>(a.cs);
  uint32_t lofs[NBW];
#pragma unroll
  for (int nb = 0; nb < NBW; ++nb) {
    uint32_t i = i032 + (wn * NBW + nb) * 16 + c;
    i = i < n32 ? i : n32 - 1;
    lofs[nb] = (i * rs32 + static_cast<uint32_t>(KV * g) * cs32) * ES;
  }

  constexpr uint32_t kOut = 0x80000000u;  // >= any resource size here
  const uint32_t x_bytes = static_cast<uint32_t>(a.Il * m * a.Ir * ES);
  const uint32_t l_bytes = static_cast<uint32_t>(((n - 1) * a.rs + (m - 1) * a.cs + 1) * ES);
  const uint32_t xes = xkstep * ES;  // bytes between consecutive k of a fiber
  const uint32_t les = cs32 * ES;    // bytes between consecutive k of a row of L
  typedef G g16 __attribute__((ext_vector_type(PER)));
  constexpr int NQ = KV / PER;       // 16-byte pieces per group of KV values

  G xr[2][XT][KV];
  G lv[NBW][KV];       // the next step's factor values (in-register split)
  FragT lnext[NBW][P];  // the next step's factor fragments (PRE: a.L holds the planes)
  const int64_t lblocks = (n + 15) / 16;

  // Chunk ch of X (k0 = ch*BK) into register set SET; CHECK: the chunk
  // reaches past k = m (those k read as zero through the resource bound).
  auto load_x = [&](int64_t ch, auto set, auto check) {
    constexpr int SET = decltype(set)::value;
    constexpr bool CHECK = decltype(check)::value;
    const int64_t k0 = ch * BK;
    const uint32_t xk = static_cast<uint32_t>(k0 * xkstep * ES);
    const auto rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(reinterpret_cast<const char*>(X)) + xk, 0, x_bytes - xk, kBufferFlags);
#pragma unroll
    for (int s = 0; s < XT; ++s) {
      const int64_t kb = k0 + xkg(s) * KV;
      if constexpr (VEC && !INNER) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          uint32_t o = xo[s] + 16 * q;
          if constexpr (CHECK) o = kb + PER * q < m ? o : kOut;
          const g16 v = __builtin_bit_cast(
              g16, __builtin_amdgcn_raw_buffer_load_b128(rs, static_cast<int>(o), 0, 0));
#pragma unroll
          for (int e = 0; e < PER; ++e) xr[SET][s][PER * q + e] = v[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < KV; ++e) {
          if constexpr (CHECK)
            xr[SET][s][e] = buffer_load<G>(rs, kb + e < m ? xo[s] + e * xes : kOut);
          else
            xr[SET][s][e] = buffer_load<G>(rs, xo[s], e * xes);
        }
      }
    }
  };
  // KV values of one row -> the P fragment planes (split forms: the bf16
  // split; native forms: the values themselves).
  auto to_frag = [&](const G (&v)[KV], FragT (&f)[P]) {
    if constexpr (SPLIT) {
      split_bf16_group<P, KV>(v, f);
    } else {
#pragma unroll
      for (int e = 0; e < KV; ++e) f[0][e] = v[e];
    }
  };
  // Register set SET -> LDS buffer BUF (P planes).
  auto store_x = [&](int buf, auto set) {
    constexpr int SET = decltype(set)::value;
#pragma unroll
    for (int s = 0; s < XT; ++s) {
      const int id = t + s * kThreads;
      const int row = INNER ? id % BF : id / KG;
      const int kg = INNER ? id / BF : id % KG;
      if (XT * kThreads == BF * KG || (row < BF && kg < KG)) {
        FragT pl[P];
        to_frag(xr[SET][s], pl);
#pragma unroll
        for (int p = 0; p < P; ++p) *reinterpret_cast<FragT*>(&sX[buf][p][row][kg * KV]) = pl[p];
      }
    }
  };
  // Macro step s (k0 = MK s) of this wave's factor rows into lv.
  auto load_l = [&](int64_t s, auto check) {
    constexpr bool CHECK = decltype(check)::value;
    if constexpr (PRE) {
      // the planes hold zeros past k = m: no check; blocks past the last one
      // (rows past n, never stored) read the last block
      const FragT* __restrict__ Lp = static_cast<const FragT*>(a.L);
      const int64_t steps = (m + MK - 1) / MK;
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) {
        int64_t b = i032 / 16 + wn * NBW + nb;
        b = b < lblocks ? b : lblocks - 1;
#pragma unroll
        for (int p = 0; p < P; ++p) lnext[nb][p] = Lp[((b * steps + s) * P + p) * 64 + lane];
      }
      return;
    }
    const int64_t k0 = s * MK;
    const uint32_t lk = static_cast<uint32_t>(k0 * a.cs * ES);
    const auto rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(reinterpret_cast<const char*>(L)) + lk, 0, l_bytes - lk, kBufferFlags);
    const int64_t kb = k0 + KV * g;
#pragma unroll
    for (int nb = 0; nb < NBW; ++nb) {
      if constexpr (VEC) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          uint32_t o = lofs[nb] + 16 * q;
          if constexpr (CHECK) o = kb + PER * q < m ? o : kOut;
          const g16 v = __builtin_bit_cast(
              g16, __builtin_amdgcn_raw_buffer_load_b128(rs, static_cast<int>(o), 0, 0));
#pragma unroll
          for (int e = 0; e < PER; ++e) lv[nb][PER * q + e] = v[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < KV; ++e) {
          if constexpr (CHECK)
            lv[nb][e] = buffer_load<G>(rs, kb + e < m ? lofs[nb] + e * les : kOut);
          else
            lv[nb][e] = buffer_load<G>(rs, lofs[nb], e * les);
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
  const int64_t lfull = m / MK;   // macro steps with no k past m
  using Checked = std::true_type;
  using Unchecked = std::false_type;
  using Set0 = std::integral_constant<int, 0>;
  using Set1 = std::integral_constant<int, 1>;

  // One macro step from LDS buffer buf at chunk offset kk: turn this step's
  // factor rows into fragments, start loading the next step's, read the
  // fibers' planes and issue the products. STEADY: the next step is full
  // (no check, no branch).
  // A wave whose n blocks all lie past n (the same in every lane) reads no
  // fragments and issues no products; it still stages fibers and meets
  // every barrier, and leaves its SIMD's matrix core to the other waves.
  const bool idle = __builtin_amdgcn_readfirstlane(
      static_cast<int>(static_cast<int64_t>(i032) + wn * NBW * 16 >= n));
  auto step = [&](int buf, int kk, int64_t s, auto steady) {
    constexpr bool STEADY = decltype(steady)::value;
    FragT la[NBW][P];
    if constexpr (PRE) {
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb)
#pragma unroll
        for (int p = 0; p < P; ++p) la[nb][p] = lnext[nb][p];
    } else {
#pragma unroll
      for (int nb = 0; nb < NBW; ++nb) to_frag(lv[nb], la[nb]);
    }
    if constexpr (STEADY) {
      load_l(s + 1, Unchecked{});
    } else if (s + 1 < nsteps) {
      if (s + 1 < lfull)
        load_l(s + 1, Unchecked{});
      else
        load_l(s + 1, Checked{});
    }
    if (idle) return;
    FragT xa[FBW][P];
#pragma unroll
    for (int fb = 0; fb < FBW; ++fb)
#pragma unroll
      for (int p = 0; p < P; ++p)
        xa[fb][p] = *reinterpret_cast<const FragT*>(
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
  // resource and the hardware drops the store. A plain store (no
  // accumulation) of a block that lies wholly inside the output takes one
  // per-lane offset per block: accumulator items v step the row (inner) or
  // the fiber (lead) by RV*v, a uniform byte step passed as the scalar
  // offset, so the stores need no per-item address arithmetic.
  constexpr uint32_t kDrop = 0x80000000u;
  constexpr uint32_t RV = FORM == FORM_F64 ? 4 : 1;  // row(lane, v) - row(lane, 0) = RV v
  const auto yrs = __builtin_amdgcn_make_buffer_rsrc(
      Y, 0, static_cast<int>(a.Il * n * a.Ir * ES), kBufferFlags);
  const bool plain = a.accumulate == kAccNone;
#pragma unroll
  for (int q = 0; q < (INNER ? NBW : FBW); ++q)
#pragma unroll
    for (int p = 0; p < (INNER ? FBW : NBW); ++p) {
      acc_t val = hi[q][p];
      if constexpr (SPLIT) val = hi[q][p] + lo[q][p];
      uint32_t off[4];
      if constexpr (INNER) {
        const uint32_t r = f032 + wf * 16 * FBW + p * 16 + c;
        const uint32_t yb = fiber_offset(r < F32 ? r : 0, Il32, n32);
        const uint32_t rowb = i032 + (wn * NBW + q) * 16;  // the block's first row
        if (rowb >= n32) continue;                          // wholly past n
        if (plain && rowb + 16 <= n32 && f032 + BF <= F32) {
          const uint32_t vb = (yb + Il32 * (rowb + FT::row(lane, 0))) * ES;
#pragma unroll
          for (int v = 0; v < 4; ++v) buffer_store_at<G>(val[v], yrs, vb, Il32 * ES * RV * v);
          continue;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const uint32_t i = i032 + (wn * NBW + q) * 16 + FT::row(lane, v);
          off[v] = (r < F32 && i < n32) ? (yb + Il32 * i) * ES : kDrop;
        }
      } else {
        if (i032 + (wn * NBW + p) * 16 >= n32) continue;  // wholly past n
        const uint32_t i = i032 + (wn * NBW + p) * 16 + c;
        const uint32_t fb0 = f032 + wf * 16 * FBW + q * 16;  // the block's first fiber
        if (plain && i032 + (wn * NBW + p) * 16 + 16 <= n32 && fb0 + 16 <= F32) {
          const uint32_t vb = (i + n32 * (fb0 + FT::row(lane, 0))) * ES;
#pragma unroll
          for (int v = 0; v < 4; ++v) buffer_store_at<G>(val[v], yrs, vb, n32 * ES * RV * v);
          continue;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const uint32_t f = f032 + wf * 16 * FBW + q * 16 + FT::row(lane, v);
          off[v] = (f < F32 && i < n32) ? (i + n32 * f) * ES : kDrop;
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) store_out<INNER, G>(val[v], yrs, off[v], a.accumulate, c);
    }
}

}  // namespace tile
}  // namespace kp
