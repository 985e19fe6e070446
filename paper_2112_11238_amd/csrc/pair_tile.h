// Two consecutive mu-mode products in one pass (Sec. 2: the Tucker operator
// applies its modes one after another, in any order; modes mu and mu + 1
// are applied here back to back without writing the intermediate to HBM).
//
// View: X as (Il, m1, m2, Ir), Y as (Il, n1, n2, Ir), fiber r = a + Il*b,
//   Z[r; i1, j2] = sum_j1 L1(i1, j1) X[r; j1, j2]          (mode mu)
//   Y[r; i1, i2] = sum_j2 L2(i2, j2) Z[r; i1, j2]          (mode mu + 1)
// X[r; j1, j2] sits at base(r, m1*m2) + Il*(j1 + m1*j2) with
// base(r, len) = (r % Il) + Il*len*(r / Il); Y likewise with n1, n2.
//
// A workgroup keeps L1 and L2 in LDS and streams tiles of 16 fibers: the
// tile's X goes to LDS (the next tile's global loads are in flight meanwhile),
// stage 1 writes Z to LDS (the waves split the j2 values), stage 2 reads it
// and writes Y straight to HBM (the waves split the i1 values). Fibers are
// the MFMA columns, so every store is a run of consecutive fibers; the
// kernel is meant for Il > 1, where consecutive fibers are contiguous.
// Each output element is summed over j1, then j2, in the same order and
// precision as two separate mu-mode products, with Z rounded to the
// element type in between (FP32 for the split forms, re-split on use).
#pragma once

#include "mode_tile.h"

namespace kp {
namespace tile {

constexpr int kPairFibers = 16;

// KP1 >= m1, KP2 >= m2 (multiples of the macro step), NB1*16 >= n1,
// NB2*16 >= n2.
template <int FORM, int KP1, int KP2, int NB1, int NB2>
struct PairLayout {
  using FT = FormT<FORM>;
  using SE = typename FT::S;
  static constexpr int P = FT::P;
  static constexpr int BF = kPairFibers;
  static constexpr int LD1 = KP1 + 16 / sizeof(SE);   // sX rows: j1 contiguous
  static constexpr int LD2 = KP2 + 16 / sizeof(SE);   // sZ rows: j2 contiguous
  static constexpr size_t l1 = sizeof(SE) * P * (16 * NB1) * LD1;
  static constexpr size_t l2 = sizeof(SE) * P * (16 * NB2) * LD2;
  static constexpr size_t x = sizeof(SE) * P * KP2 * BF * LD1;        // [p][j2][f][j1]
  static constexpr size_t z = sizeof(SE) * P * (16 * NB1) * BF * LD2; // [p][i1][f][j2]
  static constexpr size_t bytes = l1 + l2 + x + z;
};

template <int FORM, int KP1, int KP2, int NB1, int NB2>
constexpr size_t pair_lds_bytes() {
  return PairLayout<FORM, KP1, KP2, NB1, NB2>::bytes;
}

struct PairArgs {
  const void* X;
  void* Y;
  const void* L1;  // n1 x m1, L1(i, j) = L1[i*rs1 + j*cs1]
  const void* L2;  // n2 x m2
  int64_t Il, m1, m2, n1, n2, Ir;
  int64_t rs1, cs1, rs2, cs2;
};

// Fiber tiles t0, t0 + tstep, ... < ntiles (16 fibers each).
template <int FORM, int KP1, int KP2, int NB1, int NB2>
__device__ __forceinline__ void pair_run(const PairArgs& a, int64_t t0, int64_t tstep,
                                         int64_t ntiles, char* __restrict__ lds) {
  using LY = PairLayout<FORM, KP1, KP2, NB1, NB2>;
  using FT = FormT<FORM>;
  using G = typename FT::G;
  using SE = typename FT::S;
  using acc_t = typename FT::acc_t;
  using FragT = Frag<FORM>;
  constexpr int P = FT::P, KV = FT::KV, MK = FT::MK;
  constexpr bool SPLIT = FORM == FORM_BF16X3 || FORM == FORM_BF16X6;
  constexpr int BF = LY::BF, LD1 = LY::LD1, LD2 = LY::LD2;
  constexpr int R1 = 16 * NB1, R2 = 16 * NB2;
  constexpr int KG1 = KP1 / KV;
  // X staging tasks: (fiber, j1 group, j2); lanes walk along fibers
  constexpr int XTASKS = BF * KG1 * KP2;
  constexpr int XT = (XTASKS + kThreads - 1) / kThreads;
  static_assert(KP1 % MK == 0 && KP2 % MK == 0, "contraction lengths need whole macro steps");

  typedef SE L1T[P][R1][LD1];
  typedef SE L2T[P][R2][LD2];
  typedef SE XTl[P][KP2][BF][LD1];
  typedef SE ZTl[P][R1][BF][LD2];
  L1T& sL1 = *reinterpret_cast<L1T*>(lds);
  L2T& sL2 = *reinterpret_cast<L2T*>(lds + LY::l1);
  XTl& sX = *reinterpret_cast<XTl*>(lds + LY::l1 + LY::l2);
  ZTl& sZ = *reinterpret_cast<ZTl*>(lds + LY::l1 + LY::l2 + LY::x);

  const G* __restrict__ L1 = static_cast<const G*>(a.L1);
  const G* __restrict__ L2 = static_cast<const G*>(a.L2);
  // 32-bit index math: the host keeps every launch below 2^31 bytes
  const uint32_t Il = static_cast<uint32_t>(a.Il);
  const uint32_t m1 = static_cast<uint32_t>(a.m1), m2 = static_cast<uint32_t>(a.m2);
  const uint32_t n1 = static_cast<uint32_t>(a.n1), n2 = static_cast<uint32_t>(a.n2);
  const uint32_t F = static_cast<uint32_t>(a.Il * a.Ir);
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int c = lane & 15;
  const int g = lane >> 4;

  auto put = [&](SE* dst0, size_t plane, const G (&v)[KV]) {
    // KV consecutive k values of one row into every plane (16 bytes each)
    if constexpr (SPLIT) {
      bf16x8_t pl[P];
#pragma unroll
      for (int e = 0; e < KV; ++e) {
        __bf16 o[P];
        split_bf16<P>(v[e], o);
#pragma unroll
        for (int p = 0; p < P; ++p) pl[p][e] = o[p];
      }
#pragma unroll
      for (int p = 0; p < P; ++p) *reinterpret_cast<bf16x8_t*>(dst0 + p * plane) = pl[p];
    } else {
      FragT f;
#pragma unroll
      for (int e = 0; e < KV; ++e) f[e] = v[e];
      *reinterpret_cast<FragT*>(dst0) = f;
    }
  };

  // factors -> LDS once (k >= m and rows >= n read as zero)
  for (int id = t; id < R1 * KG1; id += kThreads) {
    const int i = id / KG1, kg = id % KG1;
    G v[KV];
#pragma unroll
    for (int e = 0; e < KV; ++e) {
      const uint32_t k = kg * KV + e;
      v[e] = (static_cast<uint32_t>(i) < n1 && k < m1) ? L1[i * a.rs1 + k * a.cs1] : G(0);
    }
    put(&sL1[0][i][kg * KV], R1 * LD1, v);
  }
  for (int id = t; id < R2 * (KP2 / KV); id += kThreads) {
    const int i = id / (KP2 / KV), kg = id % (KP2 / KV);
    G v[KV];
#pragma unroll
    for (int e = 0; e < KV; ++e) {
      const uint32_t k = kg * KV + e;
      v[e] = (static_cast<uint32_t>(i) < n2 && k < m2) ? L2[i * a.rs2 + k * a.cs2] : G(0);
    }
    put(&sL2[0][i][kg * KV], R2 * LD2, v);
  }

  G xr[XT][KV];
  // X tile -> registers through a buffer resource (32-bit offsets): task =
  // (fiber f, j1 group kg, j2); a j1 or j2 past m1, m2 gets an offset past the
  // resource and reads as zero; fibers past F are clamped (their outputs are
  // never stored). Y is written through a resource too.
  constexpr uint32_t kOut = 0x80000000u;
  const auto xrs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.X), 0, static_cast<int>(a.Il * a.m1 * a.m2 * a.Ir * sizeof(G)),
      kBufferFlags);
  const auto yrs = __builtin_amdgcn_make_buffer_rsrc(
      a.Y, 0, static_cast<int>(a.Il * a.n1 * a.n2 * a.Ir * sizeof(G)), kBufferFlags);
  auto load_x = [&](int64_t bx) {
    const uint32_t f0 = static_cast<uint32_t>(bx) * BF;
#pragma unroll
    for (int s = 0; s < XT; ++s) {
      const int id = t + s * kThreads;
      const int f = id % BF;
      const int kg = (id / BF) % KG1;
      const uint32_t j2 = id / (BF * KG1);
      uint32_t r = f0 + f;
      r = r < F ? r : F - 1;
      const uint32_t b = r / Il;
      const uint32_t base = (r - b * Il) + Il * m1 * m2 * b + Il * m1 * j2;
#pragma unroll
      for (int e = 0; e < KV; ++e) {
        const uint32_t j1 = kg * KV + e;
        xr[s][e] = buffer_load<G>(
            xrs, (id < XTASKS && j1 < m1 && j2 < m2) ? (base + Il * j1) * sizeof(G) : kOut);
      }
    }
  };
  auto store_x = [&]() {
#pragma unroll
    for (int s = 0; s < XT; ++s) {
      const int id = t + s * kThreads;
      if (id >= XTASKS) continue;
      const int f = id % BF;
      const int kg = (id / BF) % KG1;
      const int j2 = id / (BF * KG1);
      put(&sX[0][j2][f][kg * KV], KP2 * BF * LD1, xr[s]);
    }
  };

  if (t0 < ntiles) {
    load_x(t0);
    store_x();
  }
  __syncthreads();
  for (int64_t bx = t0; bx < ntiles; bx += tstep) {
    const int64_t nx = bx + tstep;
    if (nx < ntiles) load_x(nx);
    // stage 1: Z[i1][f][j2] for the j2 of this wave (w, w + 4, ...)
    for (int j2 = w; j2 < KP2; j2 += 4) {
      acc_t hi[NB1][1], lo[NB1][1];
#pragma unroll
      for (int q = 0; q < NB1; ++q) {
        hi[q][0] = acc_t{};
        lo[q][0] = acc_t{};
      }
#pragma unroll
      for (int kk = 0; kk < KP1; kk += MK) {
        FragT xb[1][P];
        FragT la[NB1][P];
#pragma unroll
        for (int p = 0; p < P; ++p)
          xb[0][p] = *reinterpret_cast<const FragT*>(&sX[p][j2][c][kk + KV * g]);
#pragma unroll
        for (int q = 0; q < NB1; ++q)
#pragma unroll
          for (int p = 0; p < P; ++p)
            la[q][p] = *reinterpret_cast<const FragT*>(&sL1[p][q * 16 + c][kk + KV * g]);
        macro_step_grid<FORM, NB1, 1>(la, xb, hi, lo);
      }
      // rows i1 = q*16 + row(lane, v), column f = c; Z rounded to G, split
      // into the planes when the form has them
#pragma unroll
      for (int q = 0; q < NB1; ++q) {
        acc_t val = hi[q][0];
        if constexpr (SPLIT) val = hi[q][0] + lo[q][0];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i1 = q * 16 + FT::row(lane, v);
          const G z = static_cast<G>(val[v]);
          if constexpr (SPLIT) {
            __bf16 o[P];
            split_bf16<P>(z, o);
#pragma unroll
            for (int p = 0; p < P; ++p) sZ[p][i1][c][j2] = o[p];
          } else {
            sZ[0][i1][c][j2] = z;
          }
        }
      }
    }
    __syncthreads();  // Z complete, X reads done
    if (nx < ntiles) store_x();
    // stage 2: Y for the i1 of this wave (w, w + 4, ...)
    const uint32_t f0 = static_cast<uint32_t>(bx) * BF;
    const uint32_t r = f0 + c;
    const uint32_t rb = r / Il;
    const uint32_t ybase = (r - rb * Il) + Il * n1 * n2 * rb;
    for (int i1 = w; i1 < static_cast<int>(n1); i1 += 4) {
      acc_t hi[NB2][1], lo[NB2][1];
#pragma unroll
      for (int q = 0; q < NB2; ++q) {
        hi[q][0] = acc_t{};
        lo[q][0] = acc_t{};
      }
#pragma unroll
      for (int kk = 0; kk < KP2; kk += MK) {
        FragT zb[1][P];
        FragT la[NB2][P];
#pragma unroll
        for (int p = 0; p < P; ++p)
          zb[0][p] = *reinterpret_cast<const FragT*>(&sZ[p][i1][c][kk + KV * g]);
#pragma unroll
        for (int q = 0; q < NB2; ++q)
#pragma unroll
          for (int p = 0; p < P; ++p)
            la[q][p] = *reinterpret_cast<const FragT*>(&sL2[p][q * 16 + c][kk + KV * g]);
        macro_step_grid<FORM, NB2, 1>(la, zb, hi, lo);
      }
#pragma unroll
      for (int q = 0; q < NB2; ++q) {
        acc_t val = hi[q][0];
        if constexpr (SPLIT) val = hi[q][0] + lo[q][0];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const uint32_t i2 = q * 16 + FT::row(lane, v);
          buffer_store<G>(val[v], yrs,
                          (r < F && i2 < n2) ? (ybase + Il * (i1 + n1 * i2)) * sizeof(G) : kOut);
        }
      }
    }
    __syncthreads();  // Z reads done; the next tile's X is in LDS
  }
}

}  // namespace tile
}  // namespace kp
