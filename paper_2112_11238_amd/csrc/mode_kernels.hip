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

#include <hip/hip_bf16.h>

namespace kp {
namespace {

constexpr int kThreads = 256;

// ---------------------------------------------------------------------------
// FP64 / FP32 MFMA, 16x16x4. Lane l feeds A[l%16][l/16] and B[l/16][l%16].
// Accumulator item v of lane l is D[row(l,v)][l%16]; the row map differs
// between the FP64 and FP32 instructions (checked on the device).
// ---------------------------------------------------------------------------
template <typename E>
struct Mfma4;

template <>
struct Mfma4<double> {
  using acc_t = d4_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * v + (l >> 4); }
};

template <>
struct Mfma4<float> {
  using acc_t = f4_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// Offset of fiber r = a + Il*b of a (Il, len, Ir) view: a + Il*len*b.
__device__ __forceinline__ int64_t fiber_offset(int64_t r, int64_t Il, int64_t len) {
  const int64_t b = r / Il;
  return (r - b * Il) + Il * len * b;
}

// NB: 16-blocks along n per workgroup (every wave covers all of them).
// FB: 16-blocks of fibers per wave; 4 waves split the fibers, so a workgroup
//     covers 64*FB fibers.
// BK: k-chunk staged through LDS (double buffered, one barrier per chunk).
template <typename E, int NB, int FB, int BK, bool INNER>
__global__ __launch_bounds__(kThreads) void mode_mfma4(ModeArgs a) {
  using Op = Mfma4<E>;
  using acc_t = typename Op::acc_t;
  constexpr int BN = 16 * NB;
  constexpr int BF = 64 * FB;
  constexpr int LDN = BN + 1;  // odd row lengths spread LDS banks
  constexpr int LDF = BF + 1;
  static_assert(kThreads % BK == 0, "BK must divide the block size");
  static_assert(!INNER || kThreads % BF == 0, "BF must divide the block size");
  constexpr int XPT = (BF * BK + kThreads - 1) / kThreads;
  constexpr int LPT = (BN * BK + kThreads - 1) / kThreads;
  constexpr int QB = INNER ? NB : FB;  // MFMA row blocks
  constexpr int PB = INNER ? FB : NB;  // MFMA column blocks

  __shared__ E sL[2][BK][LDN];
  __shared__ E sX[2][BK][LDF];

  const E* __restrict__ X = static_cast<const E*>(a.X);
  E* __restrict__ Y = static_cast<E*>(a.Y);
  const E* __restrict__ L = static_cast<const E*>(a.L);
  const int64_t Il = a.Il, m = a.m, n = a.n;
  const int64_t F = INNER ? a.Il * a.Ir : a.Ir;
  const int64_t f0 = static_cast<int64_t>(blockIdx.x) * BF;
  const int64_t i0 = static_cast<int64_t>(blockIdx.y) * BN;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;

  // This thread's staging assignment (fixed across chunks).
  //   lead : X element (k, f) with k = t % BK,  f = t / BK + s*(256/BK)
  //   inner: X element (k, f) with f = t % BF,  k = t / BF + s*(256/BF)
  //   L    : element (k, i)   with k = t % BK,  i = t / BK + s*(256/BK)
  int64_t xbase;  // offset of the thread's first element at k0 = 0
  bool xf_ok;     // inner: the thread's single fiber is in range
  if (INNER) {
    const int64_t r = f0 + (t % BF);
    xf_ok = r < F;
    xbase = xf_ok ? fiber_offset(r, Il, m) : 0;
  } else {
    xf_ok = true;
    xbase = (f0 + t / BK) * m + (t % BK);
  }
  E xr[XPT], lr[LPT];

  auto load_chunk = [&](int64_t k0) {
#pragma unroll
    for (int s = 0; s < XPT; ++s) {
      E v = E(0);
      if (INNER) {
        const int k = t / BF + s * (kThreads / BF);
        if (k < BK && xf_ok && k0 + k < m) v = X[xbase + Il * (k0 + k)];
      } else {
        const int k = t % BK;
        const int64_t f = f0 + t / BK + s * (kThreads / BK);
        if (t + s * kThreads < BF * BK && f < F && k0 + k < m)
          v = X[xbase + static_cast<int64_t>(s) * (kThreads / BK) * m + k0];
      }
      xr[s] = v;
    }
#pragma unroll
    for (int s = 0; s < LPT; ++s) {
      const int k = t % BK;
      const int i = t / BK + s * (kThreads / BK);
      E v = E(0);
      if (i < BN && i0 + i < n && k0 + k < m) v = L[(i0 + i) * a.rs + (k0 + k) * a.cs];
      lr[s] = v;
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int s = 0; s < XPT; ++s) {
      if (INNER) {
        const int k = t / BF + s * (kThreads / BF);
        if (k < BK) sX[buf][k][t % BF] = xr[s];
      } else {
        const int idx = t + s * kThreads;
        if (idx < BF * BK) sX[buf][t % BK][idx / BK] = xr[s];
      }
    }
#pragma unroll
    for (int s = 0; s < LPT; ++s) {
      const int i = t / BK + s * (kThreads / BK);
      if (i < BN) sL[buf][t % BK][i] = lr[s];
    }
  };

  acc_t acc[QB][PB];
#pragma unroll
  for (int q = 0; q < QB; ++q)
#pragma unroll
    for (int p = 0; p < PB; ++p) acc[q][p] = acc_t{};

  const int64_t nchunks = (m + BK - 1) / BK;
  if (nchunks > 0) {
    load_chunk(0);
    store_chunk(0);
  }
  __syncthreads();
  const int c = lane & 15;
  const int kr0 = lane >> 4;
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    const int buf = static_cast<int>(ch & 1);
    if (ch + 1 < nchunks) load_chunk((ch + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      E xf[FB], lf[NB];
#pragma unroll
      for (int fb = 0; fb < FB; ++fb) xf[fb] = sX[buf][kk + kr0][w * 16 * FB + fb * 16 + c];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) lf[nb] = sL[buf][kk + kr0][nb * 16 + c];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int fb = 0; fb < FB; ++fb) {
          if constexpr (INNER)
            acc[nb][fb] = Op::run(lf[nb], xf[fb], acc[nb][fb]);
          else
            acc[fb][nb] = Op::run(xf[fb], lf[nb], acc[fb][nb]);
        }
    }
    if (ch + 1 < nchunks) store_chunk(buf ^ 1);
    __syncthreads();
  }

  // Store: MFMA column = lane & 15 is the memory-contiguous output index.
#pragma unroll
  for (int q = 0; q < QB; ++q)
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      if (INNER) {
        const int64_t r = f0 + w * 16 * FB + p * 16 + c;
        if (r >= F) continue;
        const int64_t yb = fiber_offset(r, Il, n);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t i = i0 + q * 16 + Op::row(lane, v);
          if (i < n) {
            E* dst = Y + yb + Il * i;
            *dst = a.accumulate ? *dst + acc[q][p][v] : acc[q][p][v];
          }
        }
      } else {
        const int64_t i = i0 + p * 16 + c;
        if (i >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t f = f0 + w * 16 * FB + q * 16 + Op::row(lane, v);
          if (f < F) {
            E* dst = Y + i + n * f;
            *dst = a.accumulate ? *dst + acc[q][p][v] : acc[q][p][v];
          }
        }
      }
    }
}

// ---------------------------------------------------------------------------
// BF16 split forms on v_mfma_f32_16x16x32_bf16. Lane l feeds
// A[l%16][8*(l/16) .. +7] and B[8*(l/16) .. +7][l%16]: both operands are read
// from LDS rows that are contiguous along k (16-byte reads). Accumulator item
// v of lane l is D[4*(l/16) + v][l%16].
// ---------------------------------------------------------------------------

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

// Partial products of the split form: the leading a1*b1 into `hi`, the
// correction products (smallest first) into `lo`.
template <int S, int P>
__device__ __forceinline__ void split_products(const bf16x8_t (&A)[P], const bf16x8_t (&B)[P],
                                               f4_t& hi, f4_t& lo) {
  if constexpr (S == 6) {
    lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[2], lo, 0, 0, 0);
    lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[1], lo, 0, 0, 0);
    lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[2], B[0], lo, 0, 0, 0);
  }
  lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[1], lo, 0, 0, 0);
  lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[1], B[0], lo, 0, 0, 0);
  hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[0], B[0], hi, 0, 0, 0);
}

template <int S, int NB, int FB, bool INNER>
__global__ __launch_bounds__(kThreads) void mode_bf16(ModeArgs a) {
  constexpr int P = (S == 3) ? 2 : 3;  // split planes
  constexpr int BK = 32;
  constexpr int KG = BK / 8;  // 8-wide k groups per row
  constexpr int BN = 16 * NB;
  constexpr int BF = 64 * FB;
  constexpr int LDK = BK + 8;  // 80-byte rows: conflict-free 16-byte reads
  constexpr int XT = (BF * KG + kThreads - 1) / kThreads;  // X tasks/thread
  constexpr int LT = (BN * KG + kThreads - 1) / kThreads;  // L tasks/thread
  constexpr int QB = INNER ? NB : FB;
  constexpr int PB = INNER ? FB : NB;
  static_assert(!INNER || kThreads % BF == 0, "BF must divide the block size");

  __shared__ __attribute__((aligned(16))) __bf16 sL[P][BN][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 sX[P][BF][LDK];

  const float* __restrict__ X = static_cast<const float*>(a.X);
  float* __restrict__ Y = static_cast<float*>(a.Y);
  const float* __restrict__ L = static_cast<const float*>(a.L);
  const int64_t Il = a.Il, m = a.m, n = a.n;
  const int64_t F = INNER ? a.Il * a.Ir : a.Ir;
  const int64_t f0 = static_cast<int64_t>(blockIdx.x) * BF;
  const int64_t i0 = static_cast<int64_t>(blockIdx.y) * BN;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;

  // X task: one row (fiber) and one 8-wide k group.
  //   lead : kg = id % KG, f = id / KG   (consecutive threads walk along k)
  //   inner: f = id % BF,  kg = id / BF  (consecutive threads walk fibers)
  int64_t xbase = 0;
  bool xf_ok = true;
  if (INNER) {
    const int64_t r = f0 + (t % BF);
    xf_ok = r < F;
    xbase = xf_ok ? fiber_offset(r, Il, m) : 0;
  }
  float xr[XT][8], lr[LT][8];

  auto load_chunk = [&](int64_t k0) {
#pragma unroll
    for (int s = 0; s < XT; ++s) {
      const int id = t + s * kThreads;
      if (INNER) {
        const int kg = id / BF;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t k = k0 + kg * 8 + e;
          xr[s][e] = (kg < KG && xf_ok && k < m) ? X[xbase + Il * k] : 0.f;
        }
      } else {
        const int kg = id % KG;
        const int64_t f = f0 + id / KG;
        const bool ok = id < BF * KG && f < F;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t k = k0 + kg * 8 + e;
          xr[s][e] = (ok && k < m) ? X[f * m + k] : 0.f;
        }
      }
    }
#pragma unroll
    for (int s = 0; s < LT; ++s) {
      const int id = t + s * kThreads;
      const int kg = id % KG;
      const int i = id / KG;
      const bool ok = i < BN && i0 + i < n;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t k = k0 + kg * 8 + e;
        lr[s][e] = (ok && k < m) ? L[(i0 + i) * a.rs + k * a.cs] : 0.f;
      }
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int s = 0; s < XT; ++s) {
      const int id = t + s * kThreads;
      int row, kg;
      if (INNER) {
        row = id % BF;
        kg = id / BF;
      } else {
        row = id / KG;
        kg = id % KG;
      }
      if (row < BF && kg < KG) {
        bf16x8_t v[P];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 o[P];
          split_bf16<P>(xr[s][e], o);
#pragma unroll
          for (int p = 0; p < P; ++p) v[p][e] = o[p];
        }
#pragma unroll
        for (int p = 0; p < P; ++p) *reinterpret_cast<bf16x8_t*>(&sX[p][row][kg * 8]) = v[p];
      }
    }
#pragma unroll
    for (int s = 0; s < LT; ++s) {
      const int id = t + s * kThreads;
      const int i = id / KG;
      const int kg = id % KG;
      if (i < BN) {
        bf16x8_t v[P];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          __bf16 o[P];
          split_bf16<P>(lr[s][e], o);
#pragma unroll
          for (int p = 0; p < P; ++p) v[p][e] = o[p];
        }
#pragma unroll
        for (int p = 0; p < P; ++p) *reinterpret_cast<bf16x8_t*>(&sL[p][i][kg * 8]) = v[p];
      }
    }
  };

  f4_t hi[QB][PB], lo[QB][PB];
#pragma unroll
  for (int q = 0; q < QB; ++q)
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      hi[q][p] = f4_t{};
      lo[q][p] = f4_t{};
    }

  const int c = lane & 15;
  const int g = lane >> 4;
  const int64_t nchunks = (m + BK - 1) / BK;
  if (nchunks > 0) load_chunk(0);
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    store_chunk();
    __syncthreads();
    if (ch + 1 < nchunks) load_chunk((ch + 1) * BK);
    bf16x8_t xa[FB][P];
#pragma unroll
    for (int fb = 0; fb < FB; ++fb)
#pragma unroll
      for (int p = 0; p < P; ++p)
        xa[fb][p] = *reinterpret_cast<const bf16x8_t*>(&sX[p][w * 16 * FB + fb * 16 + c][g * 8]);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      bf16x8_t la[P];
#pragma unroll
      for (int p = 0; p < P; ++p)
        la[p] = *reinterpret_cast<const bf16x8_t*>(&sL[p][nb * 16 + c][g * 8]);
#pragma unroll
      for (int fb = 0; fb < FB; ++fb) {
        // A operand holds the MFMA rows, B the (memory-contiguous) columns.
        if constexpr (INNER)
          split_products<S>(la, xa[fb], hi[nb][fb], lo[nb][fb]);
        else
          split_products<S>(xa[fb], la, hi[fb][nb], lo[fb][nb]);
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int q = 0; q < QB; ++q)
#pragma unroll
    for (int p = 0; p < PB; ++p) {
      if (INNER) {
        const int64_t r = f0 + w * 16 * FB + p * 16 + c;
        if (r >= F) continue;
        const int64_t yb = fiber_offset(r, Il, n);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t i = i0 + q * 16 + 4 * g + v;
          if (i < n) {
            float* dst = Y + yb + Il * i;
            const float val = hi[q][p][v] + lo[q][p][v];
            *dst = a.accumulate ? *dst + val : val;
          }
        }
      } else {
        const int64_t i = i0 + p * 16 + c;
        if (i >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t f = f0 + w * 16 * FB + q * 16 + 4 * g + v;
          if (f < F) {
            float* dst = Y + i + n * f;
            const float val = hi[q][p][v] + lo[q][p][v];
            *dst = a.accumulate ? *dst + val : val;
          }
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Dispatch over the compiled tile variants.
// ---------------------------------------------------------------------------
using KernelFn = void (*)(ModeArgs);

struct Variant {
  int form, nb, fb, bk;
  KernelFn lead, inner;
};

#define KP_V4(E, FORM, NB, FB, BK) \
  {FORM, NB, FB, BK, mode_mfma4<E, NB, FB, BK, false>, mode_mfma4<E, NB, FB, BK, true>}
#define KP_VB(S, NB, FB) {S, NB, FB, 32, mode_bf16<S, NB, FB, false>, mode_bf16<S, NB, FB, true>}

const Variant kVariants[] = {
    KP_V4(double, FORM_F64, 1, 4, 16), KP_V4(double, FORM_F64, 2, 4, 16),
    KP_V4(double, FORM_F64, 2, 2, 16), KP_V4(double, FORM_F64, 4, 2, 16),
    KP_V4(double, FORM_F64, 4, 1, 16), KP_V4(double, FORM_F64, 8, 1, 16),
    KP_V4(double, FORM_F64, 8, 2, 8),  KP_V4(double, FORM_F64, 13, 1, 8),
    KP_V4(double, FORM_F64, 16, 1, 8),
    KP_V4(float, FORM_F32, 1, 4, 16),  KP_V4(float, FORM_F32, 2, 4, 16),
    KP_V4(float, FORM_F32, 2, 2, 16),  KP_V4(float, FORM_F32, 4, 2, 16),
    KP_V4(float, FORM_F32, 4, 1, 16),  KP_V4(float, FORM_F32, 8, 1, 16),
    KP_V4(float, FORM_F32, 8, 2, 16),  KP_V4(float, FORM_F32, 13, 1, 16),
    KP_V4(float, FORM_F32, 16, 1, 16),
    KP_VB(3, 1, 4), KP_VB(3, 2, 4), KP_VB(3, 2, 2), KP_VB(3, 4, 2), KP_VB(3, 4, 1),
    KP_VB(3, 8, 1), KP_VB(3, 8, 2), KP_VB(3, 13, 1), KP_VB(3, 16, 1),
    KP_VB(6, 1, 4), KP_VB(6, 2, 4), KP_VB(6, 2, 2), KP_VB(6, 4, 2), KP_VB(6, 4, 1),
    KP_VB(6, 8, 1), KP_VB(6, 8, 2), KP_VB(6, 13, 1), KP_VB(6, 16, 1),
};

const Variant* find_variant(int form, const ModeTile& t) {
  for (const Variant& v : kVariants)
    if (v.form == form && v.nb == t.nb && v.fb == t.fb && v.bk == t.bk) return &v;
  return nullptr;
}

int nb_for(int64_t n) {
  if (n <= 16) return 1;
  if (n <= 32) return 2;
  if (n <= 64) return 4;
  if (n <= 128) return 8;
  if (n <= 208) return 13;
  return 16;
}

}  // namespace

ModeTile default_mode_tile(int form, const ModeArgs& a) {
  ModeTile t;
  t.nb = nb_for(a.n);
  t.fb = t.nb <= 2 ? 4 : (t.nb <= 4 ? 2 : 1);
  if (form == FORM_F64)
    t.bk = t.nb >= 13 ? 8 : (t.nb == 8 && t.fb == 2 ? 8 : 16);
  else if (form == FORM_F32)
    t.bk = 16;
  else
    t.bk = 32;
  return t;
}

bool mode_tile_supported(int form, const ModeArgs& a, const ModeTile& t) {
  (void)a;
  return find_variant(form, t) != nullptr;
}

hipError_t launch_mode(int form, const ModeArgs& a, const ModeTile* force,
                       hipStream_t stream) {
  const ModeTile t = force ? *force : default_mode_tile(form, a);
  const Variant* v = find_variant(form, t);
  if (!v) return hipErrorInvalidValue;
  const bool inner = a.Il > 1;
  const int64_t F = inner ? a.Il * a.Ir : a.Ir;
  if (F == 0 || a.n == 0) return hipSuccess;
  const int64_t bf = 64 * t.fb;
  const int64_t bn = 16 * t.nb;
  const int64_t gx = (F + bf - 1) / bf;
  const int64_t gy = (a.n + bn - 1) / bn;
  if (gx > 0x7fffffffLL || gy > 65535) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(inner ? v->inner : v->lead, dim3(static_cast<unsigned>(gx),
                     static_cast<unsigned>(gy)), dim3(kThreads), 0, stream, a);
  return hipGetLastError();
}

}  // namespace kp
