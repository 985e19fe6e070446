// Factor-gradient contraction for small factors (n, m <= 64):
// C(i, j) = sum over fibers r of Q(r, i) P(r, j), Q viewed as (Il, n, Ir),
// P as (Il, m, Ir), r = a + Il*b (the rule is derived from the Kronecker
// form of the Tucker operator, Sec. 2, and the transpose rule of
// Appendix A, property 5).
//
// The whole n x m output fits one workgroup's registers, so a workgroup
// streams a contiguous run of BR-fiber chunks: both operands of a chunk go
// through double-buffered LDS with the next chunk's global loads in flight,
// and the four waves split each chunk's fibers (the MFMA k dimension), each
// accumulating the full output. At the end the waves' partial sums are
// added in LDS in a fixed order and written as this workgroup's partial
// tile; a separate pass adds the workgroups' tiles in a fixed order.
#pragma once

#include "gram_tile.h"
#include "mode_tile.h"
#include "pair_tile.h"

namespace kp {
namespace gram {

template <typename E, int NB, int MB, int BR>
constexpr size_t strip_stage_bytes() {
  return 2 * static_cast<size_t>(16 * (NB + MB)) * (BR + 16 / sizeof(E)) * sizeof(E);
}
// JB > 0: the fused variant's output staging (two buffers of 16*JB rows of
// BR fibers) follows the operand staging
template <typename E, int NB, int MB, int BR, int JB = 0>
constexpr size_t strip_lds_bytes() {
  constexpr size_t stage = strip_stage_bytes<E, NB, MB, BR>() +
                           2 * static_cast<size_t>(16 * JB) * BR * sizeof(E);
  constexpr size_t reduce = static_cast<size_t>(16 * NB) * (16 * MB) * sizeof(E);
  return stage > reduce ? stage : reduce;
}

// The fused backward step (gram_strip with JB > 0, FP32, inner layout with
// 16-byte fiber groups): from the same staged chunks of Q, besides the
// factor gradient's partial tile, the cotangent of the next mode down,
// Y(r, j) = sum_i L(i, j) Q(r, i) (the mu-mode product with L^T, Y viewed
// as (Il, m, Ir)), so Q is read from HBM once for both.
struct GramProduct {
  const float* L;  // n x m, L(i, j) = L[i*rs + j*cs]
  float* Y;
  int64_t rs, cs;
};

// Chunks [c_begin, c_end) of BR consecutive fibers; writes the partial n x m
// tile to out[i*m + j]. At the end the waves' sums are added in LDS in
// wave order, ((w0 + w1) + w2) + w3.
// INNER (Il > 1): a staging task is one fiber and KV consecutive rows, lanes
// walk along fibers (contiguous in memory). Lead (Il == 1): a task is one
// row and KV consecutive fibers, lanes walk along rows. INNER with VEC
// (Il a multiple of KV, Q and P 16-byte aligned): a task is one row and KV
// consecutive fibers, which are adjacent in memory, so it is one 16-byte
// load and one 16-byte LDS store; lanes walk along the fiber groups.
// JB > 0 (fused step): wave w also computes Y for fibers 16w .. 16w + 15 of
// each chunk (MFMA rows = fibers, k = i in 16-long macro steps with lane
// group g owning i = 4g .. 4g + 3, as in the unfused products; columns = j)
// into an LDS block of 16*JB rows of BR fibers, and after the chunk's
// barrier every thread stores 16 contiguous bytes of it (rows of BR fibers
// leave as runs of 4*BR bytes). PFORM: the product's form, FP32 MFMA or a
// BF16 split form (16-long bf16 MFMAs on the operands' planes, the leading
// product in one accumulator, the corrections in another).
template <typename E, int NB, int MB, int BR, bool INNER, bool VEC = false, int JB = 0,
          int PFORM = FORM_F32>
__device__ __forceinline__ void gram_strip(const GramArgs& g, int64_t c_begin, int64_t c_end,
                                           E* __restrict__ out, char* __restrict__ lds,
                                           const GramProduct* prod = nullptr) {
  using GT = GramT<E>;
  using frag = typename GT::frag;
  using acc_t = typename GT::acc_t;
  constexpr int KV = GT::KV;
  constexpr int MK = 4 * KV;
  constexpr int RQ = 16 * NB, RP = 16 * MB;      // staged rows of Q and P
  constexpr int LDR = BR + 16 / sizeof(E);
  constexpr int KW = BR / 4;                     // fibers per wave and chunk
  static_assert(KW % MK == 0, "each wave needs whole macro steps");
  // tasks: INNER (fiber, row group of KV), lead (row, fiber group of KV)
  constexpr int TQ = (RQ / KV) * BR;
  constexpr int TP = (RP / KV) * BR;
  constexpr int NQ = (TQ + kThreads - 1) / kThreads;
  constexpr int NP = (TP + kThreads - 1) / kThreads;
  typedef E QTile[RQ][LDR];
  typedef E PTile[RP][LDR];
  QTile* sQ = reinterpret_cast<QTile*>(lds);
  PTile* sP = reinterpret_cast<PTile*>(lds + 2 * sizeof(QTile));
  constexpr bool PROD = JB > 0;
  static_assert(!PROD || (sizeof(E) == 4 && INNER && VEC && NB <= 2 && BR == 64),
                "the fused step: FP32, inner layout with fiber groups, n <= 32, 64-fiber chunks");
  typedef E OTile[16 * (JB > 0 ? JB : 1)][BR];
  OTile* sO = reinterpret_cast<OTile*>(lds + strip_stage_bytes<E, NB, MB, BR>());

  // 32-bit index math: the host keeps each operand below 2^31 bytes
  const uint32_t Il = static_cast<uint32_t>(g.Il), n = static_cast<uint32_t>(g.n);
  const uint32_t m = static_cast<uint32_t>(g.m);
  const uint32_t F = static_cast<uint32_t>(g.Il * g.Ir);
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int c = lane & 15;
  const int gq = lane >> 4;

  // two register sets (PF2): the loads of chunk ch + 2 are in flight while
  // chunk ch is computed and chunk ch + 1 waits in the other set; the
  // largest tiles (4 x 4 blocks) keep one set, the next chunk in flight
  constexpr bool PF2 = !(NB == 4 && MB == 4);
  E qv[PF2 ? 2 : 1][NQ][KV], pv[PF2 ? 2 : 1][NP][KV];
  // loads through buffer resources over Q and P (32-bit offsets); elements
  // past F, n or m get an offset past the resource and read as zero
  constexpr uint32_t kOut = 0x80000000u;
  const auto qrs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(g.Q), 0, static_cast<int>(g.Il * g.n * g.Ir * sizeof(E)),
      tile::kBufferFlags);
  const auto prs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<void*>(g.P), 0, static_cast<int>(g.Il * g.m * g.Ir * sizeof(E)),
      tile::kBufferFlags);
  constexpr bool GV = INNER && VEC;   // grouped fibers on the inner layout
  constexpr int FG = BR / KV;          // fiber groups per chunk
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  auto load_vec = [&](__amdgpu_buffer_rsrc_t rs, uint32_t r, uint32_t i, uint32_t rows,
                      uint32_t len, E (&dst)[KV]) {
    const uint32_t b = r / Il;
    const uint32_t off = (r < F && i < rows) ? ((r - b * Il) + Il * len * b + Il * i) * sizeof(E)
                                            : kOut;
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, static_cast<int>(off), 0, 0);
    const frag f = __builtin_bit_cast(frag, v);
#pragma unroll
    for (int e = 0; e < KV; ++e) dst[e] = f[e];
  };
  auto load = [&](int64_t ch, auto set) {
    constexpr int SET = decltype(set)::value;
    const uint32_t r0 = static_cast<uint32_t>(ch) * BR;
    if constexpr (GV) {
#pragma unroll
      for (int s = 0; s < NQ; ++s) {
        const int id = t + s * kThreads;
        const uint32_t row = id / FG, r = r0 + (id % FG) * KV;
        load_vec(qrs, r, id < TQ ? row : n, n, n, qv[SET][s]);
      }
#pragma unroll
      for (int s = 0; s < NP; ++s) {
        const int id = t + s * kThreads;
        const uint32_t row = id / FG, r = r0 + (id % FG) * KV;
        load_vec(prs, r, id < TP ? row : m, m, m, pv[SET][s]);
      }
      return;
    }
    // INNER: one fiber per task (its base offset computed once, rows at
    // stride Il); lead: one row per task, fibers at stride len
#pragma unroll
    for (int s = 0; s < NQ; ++s) {
      const int id = t + s * kThreads;
      const int fr = INNER ? id % BR : (id / RQ) * KV;   // first fiber of the task
      const int row = INNER ? (id / BR) * KV : id % RQ;  // first row of the task
      uint32_t base = 0;
      if constexpr (INNER) {
        const uint32_t r = r0 + fr;
        const uint32_t b = r / Il;
        base = (r - b * Il) + Il * n * b;
      }
#pragma unroll
      for (int e = 0; e < KV; ++e) {
        const uint32_t r = r0 + fr + (INNER ? 0 : e);
        const uint32_t i = row + (INNER ? e : 0);
        const bool ok = id < TQ && r < F && i < n;
        const uint32_t off = INNER ? base + Il * i : i + n * r;
        qv[SET][s][e] = tile::buffer_load<E>(qrs, ok ? off * sizeof(E) : kOut);
      }
    }
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      const int id = t + s * kThreads;
      const int fr = INNER ? id % BR : (id / RP) * KV;
      const int row = INNER ? (id / BR) * KV : id % RP;
      uint32_t base = 0;
      if constexpr (INNER) {
        const uint32_t r = r0 + fr;
        const uint32_t b = r / Il;
        base = (r - b * Il) + Il * m * b;
      }
#pragma unroll
      for (int e = 0; e < KV; ++e) {
        const uint32_t r = r0 + fr + (INNER ? 0 : e);
        const uint32_t j = row + (INNER ? e : 0);
        const bool ok = id < TP && r < F && j < m;
        const uint32_t off = INNER ? base + Il * j : j + m * r;
        pv[SET][s][e] = tile::buffer_load<E>(prs, ok ? off * sizeof(E) : kOut);
      }
    }
  };
  auto store = [&](int buf, auto set) {
    constexpr int SET = decltype(set)::value;
    if constexpr (GV) {
#pragma unroll
      for (int s = 0; s < NQ; ++s) {
        const int id = t + s * kThreads;
        if (id >= TQ) continue;
        frag f;
#pragma unroll
        for (int e = 0; e < KV; ++e) f[e] = qv[SET][s][e];
        *reinterpret_cast<frag*>(&sQ[buf][id / FG][(id % FG) * KV]) = f;
      }
#pragma unroll
      for (int s = 0; s < NP; ++s) {
        const int id = t + s * kThreads;
        if (id >= TP) continue;
        frag f;
#pragma unroll
        for (int e = 0; e < KV; ++e) f[e] = pv[SET][s][e];
        *reinterpret_cast<frag*>(&sP[buf][id / FG][(id % FG) * KV]) = f;
      }
      return;
    }
#pragma unroll
    for (int s = 0; s < NQ; ++s) {
      const int id = t + s * kThreads;
      if (id >= TQ) continue;
      if constexpr (INNER) {
        const int fr = id % BR, row = (id / BR) * KV;
#pragma unroll
        for (int e = 0; e < KV; ++e) sQ[buf][row + e][fr] = qv[SET][s][e];
      } else {
        const int fr = (id / RQ) * KV, row = id % RQ;
        frag f;
#pragma unroll
        for (int e = 0; e < KV; ++e) f[e] = qv[SET][s][e];
        *reinterpret_cast<frag*>(&sQ[buf][row][fr]) = f;
      }
    }
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      const int id = t + s * kThreads;
      if (id >= TP) continue;
      if constexpr (INNER) {
        const int fr = id % BR, row = (id / BR) * KV;
#pragma unroll
        for (int e = 0; e < KV; ++e) sP[buf][row + e][fr] = pv[SET][s][e];
      } else {
        const int fr = (id / RP) * KV, row = id % RP;
        frag f;
#pragma unroll
        for (int e = 0; e < KV; ++e) f[e] = pv[SET][s][e];
        *reinterpret_cast<frag*>(&sP[buf][row][fr]) = f;
      }
    }
  };

  acc_t acc[NB][MB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < MB; ++b) acc[a][b] = acc_t{};
  // row blocks past n / column blocks past m hold no output: skip them
  const int nbu = static_cast<int>((n + 15) / 16), mbu = static_cast<int>((m + 15) / 16);

  // fused step: B operands of the product, L(i = 16 h + 4 gq + s, j = 16 jb + c),
  // zero past n or m; Y through a buffer resource (offsets past it dropped)
  f4v_t lb[NB > 0 ? NB : 1][JB > 0 ? JB : 1];
  constexpr bool PSPLIT = PFORM != FORM_F32;
  tile::PairPlanes<PSPLIT ? PFORM : FORM_BF16X3> lp[PSPLIT ? NB : 1][PSPLIT ? JB : 1];
  const auto yrs = __builtin_amdgcn_make_buffer_rsrc(
      PROD ? static_cast<void*>(prod->Y) : nullptr, 0,
      PROD ? static_cast<int>(g.Il * g.m * g.Ir * sizeof(E)) : 0, tile::kBufferFlags);
  if constexpr (PROD) {
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
      for (int jb = 0; jb < JB; ++jb)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const uint32_t i = 16 * h + 4 * gq + s4, j = 16 * jb + c;
          lb[h][jb][s4] = (i < n && j < m) ? prod->L[i * prod->rs + j * prod->cs] : 0.0f;
        }
    if constexpr (PSPLIT) {
#pragma unroll
      for (int h = 0; h < NB; ++h)
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) lp[h][jb] = tile::pair_split<PFORM>(lb[h][jb]);
    }
  }
  // Y rows of this lane's fibers 16w + 4gq .. + 3 for chunk buffer `buf`
  auto product = [&](int buf) {
    f4_t o[JB > 0 ? JB : 1];
#pragma unroll
    for (int jb = 0; jb < JB; ++jb) o[jb] = f4_t{};
    if constexpr (PSPLIT) {
      f4_t lo[JB > 0 ? JB : 1];
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) lo[jb] = f4_t{};
#pragma unroll
      for (int h = 0; h < NB; ++h) {
        if (h >= nbu) break;
        f4v_t xv;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) xv[s4] = sQ[buf][16 * h + 4 * gq + s4][16 * w + c];
        const auto xp = tile::pair_split<PFORM>(xv);
#pragma unroll
        for (int jb = 0; jb < JB; ++jb) tile::pair_mma<PFORM>(xp, lp[h][jb], o[jb], lo[jb]);
      }
#pragma unroll
      for (int jb = 0; jb < JB; ++jb) o[jb] = o[jb] + lo[jb];
    } else {
#pragma unroll
      for (int h = 0; h < NB; ++h) {
        if (h >= nbu) break;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const E x = sQ[buf][16 * h + 4 * gq + s4][16 * w + c];
#pragma unroll
          for (int jb = 0; jb < JB; ++jb)
            o[jb] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, lb[h][jb][s4], o[jb], 0, 0, 0);
        }
      }
    }
    // o[jb] item v: Y(fiber 16w + 4gq + v, j = 16 jb + c)
#pragma unroll
    for (int jb = 0; jb < JB; ++jb)
      *reinterpret_cast<f4v_t*>(&sO[buf][16 * jb + c][16 * w + 4 * gq]) =
          f4v_t{o[jb][0], o[jb][1], o[jb][2], o[jb][3]};
  };
  // every thread stores 16 contiguous bytes (4 fibers of one row j) per pass
  auto store_y = [&](int buf, int64_t ch) {
    const uint32_t r0 = static_cast<uint32_t>(ch) * BR;
#pragma unroll
    for (int e = t; e < 16 * JB * (BR / 4); e += kThreads) {
      const uint32_t j = e / (BR / 4), r = r0 + 4 * (e % (BR / 4));
      const uint32_t b = r / Il;
      const uint32_t off = (r < F && j < m) ? ((r - b * Il) + Il * m * b + Il * j) * sizeof(E)
                                           : kOut;
      const f4v_t v = *reinterpret_cast<const f4v_t*>(&sO[buf][j][4 * (e % (BR / 4))]);
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), yrs,
                                             static_cast<int>(off), 0, 0);
    }
  };

  using Set0 = std::integral_constant<int, 0>;
  using Set1 = std::integral_constant<int, 1>;
  if (c_begin < c_end) {
    load(c_begin, Set0{});
    if constexpr (PF2)
      if (c_begin + 1 < c_end) load(c_begin + 1, Set1{});
    store(0, Set0{});
  }
  __syncthreads();
  int buf = 0;
  // chunk ch from LDS buffer `buf`. PF2: set CUR is free (its chunk is in
  // LDS) and takes chunk ch + 2, set NXT holds chunk ch + 1; else the one
  // set takes chunk ch + 1
  auto step = [&](int64_t ch, auto cur, auto nxt) {
    if constexpr (PF2) {
      if (ch + 2 < c_end) load(ch + 2, cur);
    } else {
      if (ch + 1 < c_end) load(ch + 1, nxt);
    }
#pragma unroll
    for (int kk = w * KW; kk < (w + 1) * KW; kk += MK) {
      frag fa[NB], fb[MB];
#pragma unroll
      for (int a = 0; a < NB; ++a)
        if (a < nbu) fa[a] = *reinterpret_cast<const frag*>(&sQ[buf][a * 16 + c][kk + KV * gq]);
#pragma unroll
      for (int b = 0; b < MB; ++b)
        if (b < mbu) fb[b] = *reinterpret_cast<const frag*>(&sP[buf][b * 16 + c][kk + KV * gq]);
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < MB; ++b)
          if (a < nbu && b < mbu) GT::step(fa[a], fb[b], acc[a][b]);
    }
    if constexpr (PROD) product(buf);
    if (ch + 1 < c_end) store(buf ^ 1, nxt);
    __syncthreads();
    if constexpr (PROD) store_y(buf, ch);
    buf ^= 1;
  };
  int64_t ch = c_begin;
  if constexpr (PF2) {
    for (; ch + 1 < c_end; ch += 2) {
      step(ch, Set0{}, Set1{});
      step(ch + 1, Set1{}, Set0{});
    }
    if (ch < c_end) step(ch, Set0{}, Set1{});
  } else {
    for (; ch < c_end; ++ch) step(ch, Set0{}, Set0{});
  }

  // wave sums added into one LDS tile in wave order
  typedef E Red[RQ][RP];
  Red& red = *reinterpret_cast<Red*>(lds);
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww) {
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < MB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            E& dst = red[a * 16 + GT::row(lane, v)][b * 16 + c];
            dst = ww == 0 ? acc[a][b][v] : dst + acc[a][b][v];
          }
    }
    __syncthreads();
  }
  for (int idx = t; idx < RQ * RP; idx += kThreads) {
    const int i = idx / RP, j = idx % RP;
    if (static_cast<uint32_t>(i) < n && static_cast<uint32_t>(j) < m) out[i * m + j] = red[i][j];
  }
  __syncthreads();  // the caller may reuse the LDS
}

// Outputs per 256-thread block of the partial-tile reduction: 4 (64
// threads per output) when many partial tiles meet few outputs (a narrow
// reduction would run on few CUs, each thread walking a long sum), else 16.
__host__ __device__ constexpr int reduce_outputs(int64_t splits, int64_t outputs) {
  return splits >= 256 && outputs < 4096 ? 4 : 16;
}

// part holds `splits` partial n x m tiles; dL(i, j) = their sum, written at
// dL[i*rs + j*cs]. A block handles OPB outputs with G = 256 / OPB threads
// each: thread q adds splits q, q + G, ... and the G partial sums are then
// added by a fixed pairwise tree (q + h into q for h = G/2, ..., 1), so the
// result does not depend on scheduling.
template <typename E, int OPB>
__device__ __forceinline__ void gram_reduce_block(const E* __restrict__ part, int64_t splits,
                                                  int64_t n, int64_t m, E* __restrict__ dL,
                                                  int64_t rs, int64_t cs, int64_t blk,
                                                  E* __restrict__ sred) {
  constexpr int G = kThreads / OPB;
  const int t = threadIdx.x;
  const int o = t % OPB, q = t / OPB;
  const int64_t idx = blk * OPB + o;
  const int64_t nm = n * m;
  E s = E(0);
  if (idx < nm)
    for (int64_t k = q; k < splits; k += G) s += part[k * nm + idx];
  sred[t] = s;
  __syncthreads();
  for (int h = G / 2; h >= 1; h /= 2) {
    if (q < h) sred[t] += sred[t + h * OPB];
    __syncthreads();
  }
  if (q == 0 && idx < nm) {
    const int64_t i = idx / m, j = idx - (idx / m) * m;
    dL[i * rs + j * cs] = sred[o];
  }
  __syncthreads();
}

}  // namespace gram
}  // namespace kp
