// Internal definitions shared by the gfx950 kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kp {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef float f4v_t __attribute__((ext_vector_type(4)));

// Arithmetic form of a contraction (values match kp_prec / kp_dtype use).
enum Form { FORM_F64 = 0, FORM_F32 = 1, FORM_BF16X3 = 3, FORM_BF16X6 = 6 };

// One mu-mode product on the three-index view of a column-major tensor:
//   X viewed as (Il, m, Ir), Y as (Il, n, Ir),
//   Y[a, i, b] (+)= sum_j L(i, j) X[a, j, b],   L(i, j) = L[i*rs + j*cs].
// Il = product of the sizes before mode mu (contiguous run), Ir = product
// of the sizes after it. Offsets: X[a + Il*(j + m*b)], Y[a + Il*(i + n*b)].
struct ModeArgs {
  const void* X;
  void* Y;
  const void* L;
  int64_t Il, m, n, Ir;
  int64_t rs, cs;
  int accumulate;  // an Acc value
};

// What the epilogue does with a computed value v at its output y:
// overwrite, add, or add i v / -i v on interleaved complex data, where the
// real and imaginary parts of one complex entry are adjacent fibers (I_l
// even, the pair index fastest).
enum Acc { kAccNone = 0, kAccAdd = 1, kAccAddI = 2, kAccSubI = 3 };

// Tile choice for the mode kernels. nb = 16-wide blocks along n per
// workgroup, fb = 16-wide fiber blocks per wave (4 waves per workgroup),
// bk = k-chunk staged in LDS per step, occ = waves per SIMD the variant's
// register budget targets (0: any), pf = prefetch distance in chunks (0: 1).
// kind 0: k-loop tile (mode_tile.h); kind 1: strip tile (strip_tile.h) for
// m <= bk, where bk is the padded contraction length and occ, pf are 0.
struct ModeTile {
  int nb, fb, bk, occ, pf, kind;
};

// Launch one mu-mode product; returns a hipError_t.
hipError_t launch_mode(int form, const ModeArgs& a, const ModeTile* force,
                       hipStream_t stream);
// Default tile for a problem (what launch_mode uses when force == nullptr).
// alone: a standalone launch (small problems then take tiles that spread
// over the chip); false inside the batched executor, whose launches are
// filled by many problems at once.
ModeTile default_mode_tile(int form, const ModeArgs& a, bool alone = true);
// Whether a tile is one of the compiled variants for this form/layout.
bool mode_tile_supported(int form, const ModeArgs& a, const ModeTile& t);
// The compiled variant matching t (occ 0 / pf 0: first match), written to
// *out with its occ and pf filled in; false if none.
bool resolve_mode_tile(int form, const ModeTile& t, ModeTile* out);
// Built-in default tile by form and the mode's sizes.
// Ir < 0: no adjustment for the problem size.
ModeTile builtin_mode_tile(int form, int64_t Il, int64_t m, int64_t n, int64_t Ir);
// Tile-table lookup (kp_tune.hip); false if the key has no entry.
bool tuned_tile(int form, int64_t Il, int64_t m, int64_t n, int64_t Ir, ModeTile* out);
// Compiled tiles as (nb, fb, bk, occ, pf, kind) sextuples; returns the count.
int list_mode_variants(int form, int32_t* out, int cap);
int list_batch_variants(int form, int32_t* out, int cap);
// Strip tiles (strip_kernels.hip): default choice for m <= the form's
// largest strip (false otherwise), resolution against the compiled list,
// listing, and the launch of one piece (< 2^31 bytes) of a product.
bool strip_default(int form, int64_t Il, int64_t m, int64_t n, int64_t Ir, ModeTile* out);
bool strip_resolve(int form, const ModeTile& t, ModeTile* out);
int list_strip_variants(int form, int32_t* out, int cap);
hipError_t launch_strip(int form, const ModeArgs& a, const ModeTile& t, hipStream_t stream);

// Fused pair of consecutive products, modes mu and mu + 1 (pair_tile.h,
// pair_kernels.hip): whether a form and shape have a pair kernel, and the
// launch. The product of mode mu has the sizes (Il, m1) -> n1, that of
// mode mu + 1 then (Il*n1, m2) -> n2.
namespace tile {
struct PairArgs;
}
bool pair_eligible(int form, int64_t Il, int64_t m1, int64_t m2, int64_t n1, int64_t n2);
hipError_t launch_pair(int form, const tile::PairArgs& a, hipStream_t stream);

}  // namespace kp
