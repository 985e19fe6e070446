// Device-side tile of the factor-gradient contraction, shared by the
// standalone gram kernels and the batched persistent executor.
#pragma once

#include <hip/hip_runtime.h>

#include "kp_common.h"

namespace kp {
namespace gram {

constexpr int kThreads = 256;


template <typename E>
struct GramT;
template <>
struct GramT<double> {
  static constexpr int KV = 2;
  using frag = d2_t;
  using acc_t = d4_t;
  static __device__ __forceinline__ int row(int l, int v) { return 4 * v + (l >> 4); }
  static __device__ __forceinline__ void step(const frag& a, const frag& b, acc_t& c) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], c, 0, 0, 0);
  }
};
template <>
struct GramT<float> {
  static constexpr int KV = 4;
  using frag = f4v_t;
  using acc_t = f4_t;
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
  static __device__ __forceinline__ void step(const frag& a, const frag& b, acc_t& c) {
#pragma unroll
    for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], c, 0, 0, 0);
  }
};

struct GramArgs {
  const void* Q;   // view (Il, n, Ir)
  const void* P;   // view (Il, m, Ir)
  void* part;      // [splits][n][m] partial sums, element type E
  int64_t Il, n, m, Ir;
  int64_t chunks;      // number of fiber chunks
  int64_t per_split;   // chunks per split
  int64_t achunks;     // inner: chunks per b (ceil(Il / BR))
};

template <typename E, int BR>
constexpr size_t gram_lds_bytes() {
  return 2 * 64 * (BR + 16 / sizeof(E)) * sizeof(E);
}

// One 64 x 64 tile (bx, by) of the partial sum of split bz.
// BR fibers per chunk. INNER: Il > 1 (a chunk is a run of BR consecutive a at
// one b, contiguous in memory); lead: Il == 1 (a chunk is BR consecutive b).
template <typename E, int BR, bool INNER>
__device__ __forceinline__ void gram_tile(const GramArgs& g, int64_t bx, int64_t by, int64_t bz,
                                          char* __restrict__ lds) {
  using GT = GramT<E>;
  constexpr int KV = GT::KV;
  constexpr int RG = BR / KV;            // r groups per row
  constexpr int LDR = BR + 16 / sizeof(E);
  constexpr int T = 64 * RG / kThreads;  // tasks per thread per operand
  static_assert(T >= 1 && (64 * RG) % kThreads == 0, "tile/threads mismatch");
  typedef E Tile[64][LDR];
  Tile& sQ = *reinterpret_cast<Tile*>(lds);
  Tile& sP = *reinterpret_cast<Tile*>(lds + sizeof(Tile));

  const E* __restrict__ Q = static_cast<const E*>(g.Q);
  const E* __restrict__ P = static_cast<const E*>(g.P);
  const int64_t Il = g.Il, n = g.n, m = g.m;
  const int64_t i0 = bx * 64;
  const int64_t j0 = by * 64;
  const int64_t c_begin = bz * g.per_split;
  int64_t c_end = c_begin + g.per_split;
  if (c_end > g.chunks) c_end = g.chunks;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int wi = w >> 1, wj = w & 1;

  // Task: (row, r group). INNER: threads walk along r (contiguous);
  // lead: threads walk along the row index (contiguous).
  int trow[T], trg[T];
#pragma unroll
  for (int s = 0; s < T; ++s) {
    const int id = t + s * kThreads;
    if (INNER) {
      trg[s] = id % RG;
      trow[s] = id / RG;
    } else {
      trow[s] = id % 64;
      trg[s] = id / 64;
    }
  }
  // Element (row, rr) of a chunk sits at base + rr*rstride + row*istride.
  const int64_t q_istride = INNER ? Il : 1;
  const int64_t p_istride = INNER ? Il : 1;
  const int64_t q_rstride = INNER ? 1 : n;
  const int64_t p_rstride = INNER ? 1 : m;

  using acc_t = typename GT::acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{};

  const int c = lane & 15;
  const int gq = lane >> 4;
  for (int64_t ch = c_begin; ch < c_end; ++ch) {
    int64_t qbase, pbase, valid;
    if (INNER) {
      const int64_t b = ch / g.achunks;
      const int64_t a0 = (ch - b * g.achunks) * BR;
      qbase = a0 + Il * n * b;
      pbase = a0 + Il * m * b;
      valid = Il - a0 < BR ? Il - a0 : BR;
    } else {
      const int64_t b0 = ch * BR;
      qbase = n * b0;
      pbase = m * b0;
      valid = g.Ir - b0 < BR ? g.Ir - b0 : BR;
    }
    E qv[T][KV], pv[T][KV];
#pragma unroll
    for (int s = 0; s < T; ++s) {
      const int64_t iq = i0 + trow[s];
      const int64_t jp = j0 + trow[s];
#pragma unroll
      for (int e = 0; e < KV; ++e) {
        const int rr = trg[s] * KV + e;
        const bool okr = rr < valid;
        const bool okq = okr && iq < n;
        const bool okp = okr && jp < m;
        const E a = Q[okq ? qbase + rr * q_rstride + iq * q_istride : 0];
        const E b = P[okp ? pbase + rr * p_rstride + jp * p_istride : 0];
        qv[s][e] = okq ? a : E(0);
        pv[s][e] = okp ? b : E(0);
      }
    }
    __syncthreads();  // previous chunk's fragments (or the caller's LDS use) are done
#pragma unroll
    for (int s = 0; s < T; ++s) {
      typename GT::frag fq, fp;
#pragma unroll
      for (int e = 0; e < KV; ++e) {
        fq[e] = qv[s][e];
        fp[e] = pv[s][e];
      }
      *reinterpret_cast<typename GT::frag*>(&sQ[trow[s]][trg[s] * KV]) = fq;
      *reinterpret_cast<typename GT::frag*>(&sP[trow[s]][trg[s] * KV]) = fp;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BR; kk += 4 * KV) {
      typename GT::frag fa[2], fb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        fa[a] = *reinterpret_cast<const typename GT::frag*>(
            &sQ[wi * 32 + a * 16 + c][kk + KV * gq]);
#pragma unroll
      for (int b = 0; b < 2; ++b)
        fb[b] = *reinterpret_cast<const typename GT::frag*>(
            &sP[wj * 32 + b * 16 + c][kk + KV * gq]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) GT::step(fa[a], fb[b], acc[a][b]);
    }
  }

  E* part = static_cast<E*>(g.part) + bz * n * m;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t j = j0 + wj * 32 + b * 16 + c;
      if (j >= m) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + wi * 32 + a * 16 + GT::row(lane, v);
        if (i < n) part[i * m + j] = acc[a][b][v];
      }
    }
}

}  // namespace gram
}  // namespace kp
