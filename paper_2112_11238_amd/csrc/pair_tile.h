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
// FP32 (v_mfma_f32_16x16x4, four per 16-long macro step) and the BF16 split
// forms (v_mfma_f32_16x16x16_bf16 on the two or three bf16 planes of each
// operand, split in registers by round-to-nearest-even, the leading product
// in one FP32 accumulator and the correction products in another). Every
// wave works alone on 16 consecutive fibers at a time (the MFMA columns), so
// no barrier is ever needed:
//   - the MFMA operands of L1 and L2 are loaded once into registers;
//   - a wave's X values go straight from global memory into the stage-1
//     operand registers (each X value feeds exactly one product, so staging
//     through LDS would buy nothing); the next fiber group's values are
//     loaded while the current one is computed;
//   - stage 1 writes Z for 16 rows i1 at a time into the wave's own LDS
//     block, stage 2 reads it back as its operand and stores Y directly.
// The four waves of a workgroup take four adjacent fiber groups, so each
// row of X and Y is read and written in runs of 64 consecutive fibers.
// Each output element is summed over j1, then j2, with Z rounded to FP32 in
// between as in two separate mu-mode products. In FP32 the products and
// their order are those of the unfused kernels (one 16-long macro step), so
// fused and unfused results are equal; the BF16 forms take the 16-long bf16
// MFMA here where the unfused kernels zero-pad a 32-long one, so their sums
// agree to rounding, within the same error bound.
#pragma once

#include "mode_tile.h"

namespace kp {
namespace tile {

constexpr int kPairK = 16;        // m1, m2 <= 16
constexpr int kPairFibers = 16;   // fibers per wave group
constexpr int kPairWaves = 4;     // waves per workgroup
// LDS: per wave, Z for 16 rows i1 x 16 fibers x 16 j2 (FP32), no padding:
// the four 16-byte j2 slots of a (row, fiber) are XOR-swizzled by the fiber
constexpr size_t kPairLdsBytes = kPairWaves * 16 * kPairFibers * kPairK * sizeof(float);

struct PairArgs {
  const void* X;
  void* Y;
  const void* L1;  // n1 x m1, L1(i, j) = L1[i*rs1 + j*cs1]
  const void* L2;  // n2 x m2
  int64_t Il, m1, m2, n1, n2, Ir;
  int64_t rs1, cs1, rs2, cs2;
};

// NB1*16 >= n1, NB2*16 >= n2. Workgroup tiles tile0, tile0 + tstep, ... <
// ntiles; tile k covers fibers 64k .. 64k + 63, wave w of the workgroup the
// 16 fibers 64k + 16w .. 64k + 16w + 15.
// bf16 operand of the 16x16x16 MFMA: lane l holds k = 4 (l / 16) .. + 3 of
// row (A) or column (B) l mod 16
typedef short pair_s4_t __attribute__((ext_vector_type(4)));
typedef __bf16 pair_b4_t __attribute__((ext_vector_type(4)));

template <int FORM>
struct PairPlanes {
  static constexpr int P = FORM == FORM_BF16X6 ? 3 : 2;
  pair_s4_t p[P];
};

// The P bf16 planes of four consecutive k values.
template <int FORM>
__device__ __forceinline__ PairPlanes<FORM> pair_split(const f4v_t& v) {
  PairPlanes<FORM> out;
  const float x[4] = {v[0], v[1], v[2], v[3]};
  pair_b4_t pl[PairPlanes<FORM>::P];
  split_bf16_group<PairPlanes<FORM>::P, 4>(x, pl);
#pragma unroll
  for (int q = 0; q < PairPlanes<FORM>::P; ++q) out.p[q] = __builtin_bit_cast(pair_s4_t, pl[q]);
  return out;
}

// One 16-long macro step of the split products into (hi, lo): the
// correction products (smallest first) into lo, the leading one into hi.
template <int FORM>
__device__ __forceinline__ void pair_mma(const PairPlanes<FORM>& A, const PairPlanes<FORM>& B,
                                         f4_t& hi, f4_t& lo) {
  if constexpr (FORM == FORM_BF16X6) {
    lo = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.p[0], B.p[2], lo, 0, 0, 0);
    lo = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.p[1], B.p[1], lo, 0, 0, 0);
    lo = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.p[2], B.p[0], lo, 0, 0, 0);
  }
  lo = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.p[0], B.p[1], lo, 0, 0, 0);
  lo = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.p[1], B.p[0], lo, 0, 0, 0);
  hi = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A.p[0], B.p[0], hi, 0, 0, 0);
}

template <int FORM, int NB1, int NB2>
__device__ __forceinline__ void pair_run(const PairArgs& a, int64_t tile0, int64_t tstep,
                                         int64_t ntiles, char* __restrict__ lds) {
  using acc_t = f4_t;
  using FragT = f4v_t;
  constexpr bool SPLIT = FORM != FORM_F32;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int c = lane & 15;  // MFMA column: fiber within the group
  const int g = lane >> 4;  // lane group: k values 4g .. 4g + 3 of a macro step
  float* __restrict__ zw = reinterpret_cast<float*>(lds) + w * (16 * kPairFibers * kPairK);

  // 32-bit index math: the host keeps every launch below 2^31 bytes
  const uint32_t Il = static_cast<uint32_t>(a.Il);
  const uint32_t m1 = static_cast<uint32_t>(a.m1), m2 = static_cast<uint32_t>(a.m2);
  const uint32_t n1 = static_cast<uint32_t>(a.n1), n2 = static_cast<uint32_t>(a.n2);
  const uint32_t F = static_cast<uint32_t>(a.Il * a.Ir);
  constexpr uint32_t kOut = 0x80000000u;  // >= any resource size here

  // Operands of L1 (rows i1 = 16 q + c, k = j1 = 4g + s) and L2 (rows
  // i2 = 16 q + c, k = j2 = 4g + s), zero past n or m: fixed for the kernel.
  FragT l1f[NB1], l2f[NB2];
  const float* L1 = static_cast<const float*>(a.L1);
  const float* L2 = static_cast<const float*>(a.L2);
#pragma unroll
  for (int q = 0; q < NB1; ++q)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const uint32_t i = 16 * q + c, k = 4 * g + s;
      l1f[q][s] = (i < n1 && k < m1) ? L1[i * a.rs1 + k * a.cs1] : 0.0f;
    }
#pragma unroll
  for (int q = 0; q < NB2; ++q)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const uint32_t i = 16 * q + c, k = 4 * g + s;
      l2f[q][s] = (i < n2 && k < m2) ? L2[i * a.rs2 + k * a.cs2] : 0.0f;
    }

  PairPlanes<FORM> l1p[NB1], l2p[NB2];
  if constexpr (SPLIT) {
#pragma unroll
    for (int q = 0; q < NB1; ++q) l1p[q] = pair_split<FORM>(l1f[q]);
#pragma unroll
    for (int q = 0; q < NB2; ++q) l2p[q] = pair_split<FORM>(l2f[q]);
  }

  const auto xrs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.X), 0, static_cast<int>(a.Il * a.m1 * a.m2 * a.Ir * sizeof(float)),
      kBufferFlags);
  const auto yrs = __builtin_amdgcn_make_buffer_rsrc(
      a.Y, 0, static_cast<int>(a.Il * a.n1 * a.n2 * a.Ir * sizeof(float)), kBufferFlags);
  const uint32_t xstep = Il * 4;  // bytes per unit of j1

  // Stage-1 operand of X for j2 and step s: X[r; j1 = 4g + s, j2] of this
  // lane's fiber r (zero past m1, m2; fibers past F read the last fiber,
  // whose outputs are never stored).
  // Full modes (m1 = m2 = 16): one per-lane offset, the (s, j2) step as the
  // loads' scalar offset; otherwise per-element offsets, k past m reading zero.
  const bool full = m1 == kPairK && m2 == kPairK;
  auto load_x = [&](int64_t tile, float (&xr)[kPairK][4]) {
    uint32_t r = static_cast<uint32_t>(tile) * (kPairWaves * kPairFibers) + w * kPairFibers + c;
    r = r < F ? r : F - 1;
    const uint32_t b = r / Il;
    const uint32_t base = ((r - b * Il) + Il * m1 * m2 * b) * 4 + xstep * (4 * g);
    if (full) {
      uint32_t vj = base;  // offset of (j1 = 4g, j2)
#pragma unroll
      for (int j2 = 0; j2 < kPairK; ++j2, vj += kPairK * xstep)
#pragma unroll
        for (int s = 0; s < 4; ++s) xr[j2][s] = buffer_load<float>(xrs, vj, xstep * s);
    } else {
      uint32_t vj = base;
#pragma unroll
      for (int j2 = 0; j2 < kPairK; ++j2, vj += m1 * xstep) {
        if (static_cast<uint32_t>(j2) >= m2) {
#pragma unroll
          for (int s = 0; s < 4; ++s) xr[j2][s] = 0.0f;
          continue;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
          xr[j2][s] = buffer_load<float>(
              xrs, 4 * g + s < static_cast<int>(m1) ? vj + s * xstep : kOut);
      }
    }
  };
  // Z of (row i1 local, fiber c) holds 16 j2 values as four 16-byte slots;
  // slot u sits at position u ^ (c >> 2 & 3), so the 16 fibers of one lane
  // group read 16 different bank groups
  auto zslot = [&](int row, int u) {
    return zw + (row * kPairFibers + c) * kPairK + 4 * (u ^ ((c >> 2) & 3));
  };

  float xa[kPairK][4], xb[kPairK][4];
  auto run = [&](int64_t tile, float (&xr)[kPairK][4]) {
    const uint32_t r = static_cast<uint32_t>(tile) * (kPairWaves * kPairFibers) +
                       w * kPairFibers + c;
    const uint32_t rr = r < F ? r : 0;
    const uint32_t rb = rr / Il;
    const uint32_t ybase = (rr - rb * Il) + Il * n1 * n2 * rb;
#pragma unroll
    for (int q = 0; q < NB1; ++q) {
      if (16u * q >= n1) break;
      // stage 1: Z[i1 = 16q + 4g + v][c][j2] for all 16 j2 (4 at a time)
#pragma unroll
      for (int u = 0; u < kPairK / 4; ++u) {
        acc_t z[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) z[e] = acc_t{};
        if constexpr (SPLIT) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const FragT xv = {xr[4 * u + e][0], xr[4 * u + e][1], xr[4 * u + e][2],
                              xr[4 * u + e][3]};
            acc_t lo = acc_t{};
            pair_mma<FORM>(l1p[q], pair_split<FORM>(xv), z[e], lo);
            z[e] = z[e] + lo;
          }
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int e = 0; e < 4; ++e)
              z[e] = __builtin_amdgcn_mfma_f32_16x16x4f32(l1f[q][s], xr[4 * u + e][s], z[e], 0,
                                                          0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const f4v_t val = {z[0][v], z[1][v], z[2][v], z[3][v]};
          *reinterpret_cast<f4v_t*>(zslot(4 * g + v, u)) = val;
        }
      }
      // the wave's own LDS writes above precede its reads below
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // stage 2: Y[r; i1, i2] for the rows i1 of this block
      const uint32_t rows = n1 - 16 * q < 16 ? n1 - 16 * q : 16;
      for (uint32_t il = 0; il < rows; ++il) {
        const FragT zf = *reinterpret_cast<const FragT*>(zslot(il, g));
        acc_t y[NB2];
#pragma unroll
        for (int q2 = 0; q2 < NB2; ++q2) y[q2] = acc_t{};
        if constexpr (SPLIT) {
          const PairPlanes<FORM> zp = pair_split<FORM>(zf);
#pragma unroll
          for (int q2 = 0; q2 < NB2; ++q2) {
            acc_t lo = acc_t{};
            pair_mma<FORM>(l2p[q2], zp, y[q2], lo);
            y[q2] = y[q2] + lo;
          }
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int q2 = 0; q2 < NB2; ++q2)
              y[q2] = __builtin_amdgcn_mfma_f32_16x16x4f32(l2f[q2][s], zf[s], y[q2], 0, 0, 0);
        }
        const uint32_t i1 = 16 * q + il;
#pragma unroll
        for (int q2 = 0; q2 < NB2; ++q2)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const uint32_t i2 = 16 * q2 + 4 * g + v;
            buffer_store<float>(y[q2][v], yrs,
                                (r < F && i2 < n2) ? (ybase + Il * (i1 + n1 * i2)) * 4 : kOut);
          }
      }
      // the reads above precede the next block's writes
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  };
  // workgroup tiles tile0, tile0 + tstep, ...; in FP32 two register sets
  // alternate so the next tile's X is in flight while the current one is
  // computed; the split forms (whose operand splits need the registers) load
  // each tile's X before computing it
  int64_t tile = tile0;
  if constexpr (SPLIT) {
    for (; tile < ntiles; tile += tstep) {
      load_x(tile, xa);
      run(tile, xa);
    }
    return;
  }
  if (tile < ntiles) load_x(tile, xa);
  while (tile < ntiles) {
    const int64_t nx = tile + tstep;
    if (nx < ntiles) load_x(nx, xb);
    run(tile, xa);
    if (nx >= ntiles) break;
    const int64_t nx2 = nx + tstep;
    if (nx2 < ntiles) load_x(nx2, xa);
    run(nx, xb);
    tile = nx2;
  }
}

// Two consecutive mu-mode products on the two leading modes (I_l = 1):
// fiber r, the index over the remaining modes, is the contiguous m1 x m2
// block X[r; j1, j2] at r*m1*m2 + j1 + m1*j2, and its result the contiguous
// n1 x n2 block Y[r; i1, i2] at r*n1*n2 + i1 + n1*i2.
//   stage 1: Z(i1, j2) = sum_j1 L1(i1, j1) X(j1, j2), computed transposed
//            (A = X: rows j2, k = j1; B = L1^T: k = j1, columns i1), so that
//            each lane's result items (rows j2 = 4g + v, column i1 = c) are
//            its own A operand of stage 2 (row i1 = c, k = j2 = 4g + v):
//            Z never leaves the registers;
//   stage 2: Y(i1, i2) = sum_j2 L2(i2, j2) Z(i1, j2) (A = Z, B = L2^T); each
//            lane's result items are four consecutive i1 of one i2. They go
//            through the wave's own LDS block (n1*n2 floats) and leave as
//            lane-linear 16-byte stores: each store instruction writes 1 KB
//            of contiguous output (storing the MFMA layout directly writes
//            runs of 64 bytes, a slower pattern for HBM).
// One wave per fiber at a time (its X block is one 16-byte load per lane
// when m1 is a multiple of 4), no barrier; the waves of the grid take
// consecutive fibers, so reads and writes stream through contiguous
// memory. The k grouping of every product is that of the unfused kernels
// (lane group g owns k = 4g .. 4g + 3 of a 16-long macro step), so in FP32
// fused and unfused results are equal; the split forms use the 16-long
// bf16 MFMA as the strided pair does.
constexpr int kLeadLdsFloats = 32 * 32;  // per wave: one n1 x n2 output block

template <int FORM, int NB1, int NB2>
__device__ __forceinline__ void lead_pair_run(const PairArgs& a, int64_t wave0, int64_t wstep,
                                              float* __restrict__ yw) {
  using acc_t = f4_t;
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  constexpr bool SPLIT = FORM != FORM_F32;
  const int lane = threadIdx.x & 63;
  const int c = lane & 15;  // MFMA row (A) or column (B)
  const int g = lane >> 4;  // lane group: k values 4g .. 4g + 3 of a macro step
  // 32-bit index math: the host keeps every launch below 2^31 bytes
  const uint32_t m1 = static_cast<uint32_t>(a.m1), m2 = static_cast<uint32_t>(a.m2);
  const uint32_t n1 = static_cast<uint32_t>(a.n1), n2 = static_cast<uint32_t>(a.n2);
  const int64_t F = a.Ir;
  constexpr uint32_t kOut = 0x80000000u;  // >= any resource size here

  // B operands, fixed for the kernel: L1^T (k = j1 = 4g + s, column
  // i1 = 16 q + c) and L2^T (k = j2 = 4g + s, column i2 = 16 q + c), zero
  // past n or m
  f4v_t l1b[NB1], l2b[NB2];
  const float* L1 = static_cast<const float*>(a.L1);
  const float* L2 = static_cast<const float*>(a.L2);
#pragma unroll
  for (int q = 0; q < NB1; ++q)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const uint32_t i = 16 * q + c, k = 4 * g + s;
      l1b[q][s] = (i < n1 && k < m1) ? L1[i * a.rs1 + k * a.cs1] : 0.0f;
    }
#pragma unroll
  for (int q = 0; q < NB2; ++q)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const uint32_t i = 16 * q + c, k = 4 * g + s;
      l2b[q][s] = (i < n2 && k < m2) ? L2[i * a.rs2 + k * a.cs2] : 0.0f;
    }
  PairPlanes<FORM> l1p[NB1], l2p[NB2];
  if constexpr (SPLIT) {
#pragma unroll
    for (int q = 0; q < NB1; ++q) l1p[q] = pair_split<FORM>(l1b[q]);
#pragma unroll
    for (int q = 0; q < NB2; ++q) l2p[q] = pair_split<FORM>(l2b[q]);
  }

  const auto xrs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(a.X), 0, static_cast<int>(F * a.m1 * a.m2 * sizeof(float)), kBufferFlags);
  const auto yrs = __builtin_amdgcn_make_buffer_rsrc(
      a.Y, 0, static_cast<int>(F * a.n1 * a.n2 * sizeof(float)), kBufferFlags);
  const bool vin = (m1 & 3u) == 0, vout = (n1 & 3u) == 0;
  const uint32_t nn = n1 * n2;             // floats per output block
  const bool vstore = (nn & 3u) == 0;      // every block starts 16-byte aligned

  // A operand of stage 1: X(j1 = 4g + s, j2 = c) of fiber r, zero past m
  auto load = [&](int64_t r, f4v_t& x) {
    const uint32_t base = static_cast<uint32_t>(r) * m1 * m2 * 4u;
    if (vin) {
      const uint32_t off = (4u * g < m1 && static_cast<uint32_t>(c) < m2)
                               ? base + (4u * g + m1 * c) * 4u
                               : kOut;
      x = __builtin_bit_cast(f4v_t,
                             __builtin_amdgcn_raw_buffer_load_b128(xrs, static_cast<int>(off), 0, 0));
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        x[s] = buffer_load<float>(xrs, (4u * g + s < m1 && static_cast<uint32_t>(c) < m2)
                                           ? base + (4u * g + s + m1 * c) * 4u
                                           : kOut);
    }
  };
  auto run = [&](int64_t r, const f4v_t& x) {
    // stage 1: z[q] item v = Z(i1 = 16 q + c, j2 = 4g + v)
    acc_t z[NB1];
    if constexpr (SPLIT) {
      const PairPlanes<FORM> xp = pair_split<FORM>(x);
#pragma unroll
      for (int q = 0; q < NB1; ++q) {
        acc_t hi = acc_t{}, lo = acc_t{};
        pair_mma<FORM>(xp, l1p[q], hi, lo);
        z[q] = hi + lo;
      }
    } else {
#pragma unroll
      for (int q = 0; q < NB1; ++q) {
        z[q] = acc_t{};
#pragma unroll
        for (int s = 0; s < 4; ++s)
          z[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[s], l1b[q][s], z[q], 0, 0, 0);
      }
    }
    // stage 2 into the LDS block: y item v = Y(i1 = 16 q + 4g + v, i2 = 16 q2 + c)
#pragma unroll
    for (int q = 0; q < NB1; ++q) {
      if (16u * q >= n1) break;
      const f4v_t za = {z[q][0], z[q][1], z[q][2], z[q][3]};
      PairPlanes<FORM> zp;
      if constexpr (SPLIT) zp = pair_split<FORM>(za);
#pragma unroll
      for (int q2 = 0; q2 < NB2; ++q2) {
        if (16u * q2 >= n2) break;
        acc_t y;
        if constexpr (SPLIT) {
          acc_t lo = acc_t{};
          y = acc_t{};
          pair_mma<FORM>(zp, l2p[q2], y, lo);
          y = y + lo;
        } else {
          y = acc_t{};
#pragma unroll
          for (int v = 0; v < 4; ++v)
            y = __builtin_amdgcn_mfma_f32_16x16x4f32(za[v], l2b[q2][v], y, 0, 0, 0);
        }
        const uint32_t i1 = 16 * q + 4 * g, i2 = 16 * q2 + c;
        if (i2 < n2) {
          if (vout) {
            if (i1 < n1) *reinterpret_cast<f4v_t*>(yw + i1 + n1 * i2) = y;
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v)
              if (i1 + v < n1) yw[i1 + v + n1 * i2] = y[v];
          }
        }
      }
    }
    // the wave's LDS writes above precede its reads below
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t ybase = static_cast<uint32_t>(r) * nn * 4u;
    if (vstore) {
      for (uint32_t e = lane; e < nn / 4; e += 64) {
        const f4v_t v = *reinterpret_cast<const f4v_t*>(yw + 4 * e);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), yrs,
                                               static_cast<int>(ybase + 16 * e), 0, 0);
      }
    } else {
      for (uint32_t e = lane; e < nn; e += 64) buffer_store<float>(yw[e], yrs, ybase + 4 * e);
    }
    // the reads above precede the next fiber's writes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  // fibers wave0, wave0 + wstep, ...: the X blocks of the next kLeadDepth
  // fibers are in flight while one is computed (a wave's compute per fiber
  // is short against the memory latency)
  constexpr int kLeadDepth = 4;
  f4v_t xb[kLeadDepth];
#pragma unroll
  for (int i = 0; i < kLeadDepth; ++i)
    if (wave0 + i * wstep < F) load(wave0 + i * wstep, xb[i]);
  for (int64_t r = wave0; r < F; r += kLeadDepth * wstep) {
#pragma unroll
    for (int i = 0; i < kLeadDepth; ++i) {
      const int64_t ri = r + i * wstep;
      if (ri >= F) break;
      const f4v_t x = xb[i];
      const int64_t rn = ri + kLeadDepth * wstep;
      if (rn < F) load(rn, xb[i]);
      run(ri, x);
    }
  }
}

}  // namespace tile
}  // namespace kp
