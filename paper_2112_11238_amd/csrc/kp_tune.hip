// Tile selection: a process-wide forced tile (tests cover every compiled
// variant with it; the tuning driver times candidates with it) and the tile
// table, keyed by the exact product shape, that the tuning driver fills; a
// view without an entry of its own takes the entry of its shape class.
#include <map>
#include <mutex>
#include <tuple>

#include "kp.h"
#include "kp_internal.h"

namespace kp {
namespace {
ModeTile g_forced;
bool g_force = false;

using Key = std::tuple<int, int64_t, int64_t, int64_t, int64_t>;  // form, Il, m, n, Ir
std::mutex g_mu;
std::map<Key, ModeTile>& table() {
  static std::map<Key, ModeTile> t;
  return t;
}

bool valid_form(int form) {
  return form == FORM_F64 || form == FORM_F32 || form == FORM_BF16X3 || form == FORM_BF16X6;
}

bool valid_key(int form, int64_t Il, int64_t m, int64_t n, int64_t Ir) {
  return valid_form(form) && Il >= 1 && m >= 1 && n >= 1 && Ir >= 1;
}

void fill(kp_tune_entry* e, const Key& k, const ModeTile& t) {
  e->form = std::get<0>(k);
  e->pad0_ = 0;
  e->Il = std::get<1>(k);
  e->m = std::get<2>(k);
  e->n = std::get<3>(k);
  e->Ir = std::get<4>(k);
  e->nb = t.nb;
  e->fb = t.fb;
  e->bk = t.bk;
  e->occ = t.occ;
  e->pf = t.pf;
  e->kind = t.kind;
}
}  // namespace

const ModeTile* tile_override() { return g_force ? &g_forced : nullptr; }

namespace {
bool g_fuse = true;
}  // namespace

bool fusion_enabled() { return g_fuse; }

// Exact view first; otherwise the entry of the same shape class: same form,
// same layout (I_l = 1 or I_l > 1), same m and n, and a fiber count within
// a factor of two (the nearest in ratio; ties: the smaller count). A tile
// tuned on one size of a product thus also serves its neighbours.
bool tuned_tile(int form, int64_t Il, int64_t m, int64_t n, int64_t Ir, ModeTile* out) {
  std::lock_guard<std::mutex> lock(g_mu);
  const auto& t = table();
  if (t.empty()) return false;
  const auto it = t.find(Key{form, Il, m, n, Ir});
  if (it != t.end()) {
    *out = it->second;
    return true;
  }
  const bool lead = Il == 1;
  const double F = static_cast<double>(Il) * static_cast<double>(Ir);
  const ModeTile* best = nullptr;
  double best_ratio = 2.0 + 1e-9, best_F = 0.0;
  for (const auto& kv : t) {
    const Key& k = kv.first;
    if (std::get<0>(k) != form || std::get<2>(k) != m || std::get<3>(k) != n) continue;
    if ((std::get<1>(k) == 1) != lead) continue;
    const double Fk = static_cast<double>(std::get<1>(k)) * static_cast<double>(std::get<4>(k));
    const double ratio = Fk > F ? Fk / F : F / Fk;
    if (ratio < best_ratio || (ratio == best_ratio && Fk < best_F)) {
      best_ratio = ratio;
      best_F = Fk;
      best = &kv.second;
    }
  }
  if (!best) return false;
  *out = *best;
  return true;
}

}  // namespace kp

extern "C" int kp_force_tile(int nb, int fb, int bk, int occ, int pf, int kind) {
  if (nb <= 0) {
    kp::g_force = false;
    return KP_OK;
  }
  // kinds: 0 k-loop tile, 1 strip tile, 3 wide tile (2 names a fused pair in
  // launch reports and is not a tile)
  if (fb <= 0 || bk <= 0 || occ < 0 || pf < 0 || pf > 2 || kind < 0 || kind > 3 || kind == 2)
    return KP_ERR_VALUE;
  kp::g_forced.kind = kind;
  kp::g_forced.nb = nb;
  kp::g_forced.fb = fb;
  kp::g_forced.bk = bk;
  kp::g_forced.occ = occ;
  kp::g_forced.pf = pf;
  kp::g_force = true;
  return KP_OK;
}

extern "C" int kp_set_option(int option, int value) {
  if (option == KP_OPT_FUSE) {
    if (value != 0 && value != 1) return KP_ERR_VALUE;
    kp::g_fuse = value != 0;
    return KP_OK;
  }
  return KP_ERR_VALUE;
}

extern "C" int kp_get_option(int option) {
  if (option == KP_OPT_FUSE) return kp::g_fuse ? 1 : 0;
  return KP_ERR_VALUE;
}

extern "C" int kp_tune_set(const kp_tune_entry* e) {
  if (!e) return KP_ERR_NULL;
  if (!kp::valid_key(e->form, e->Il, e->m, e->n, e->Ir)) return KP_ERR_VALUE;
  if (e->nb <= 0 || e->fb <= 0 || e->bk <= 0 || e->occ < 0 || e->pf < 0 || e->pf > 2 ||
      e->kind < 0 || e->kind > 3 || e->kind == 2)
    return KP_ERR_VALUE;
  kp::ModeTile t{e->nb, e->fb, e->bk, e->occ, e->pf, e->kind};
  kp::ModeTile r;
  if (!kp::resolve_mode_tile(e->form, t, &r)) return KP_ERR_VALUE;
  if (r.kind == 1 && e->m > r.bk) return KP_ERR_VALUE;
  std::lock_guard<std::mutex> lock(kp::g_mu);
  kp::table()[kp::Key{e->form, e->Il, e->m, e->n, e->Ir}] = r;
  return KP_OK;
}

extern "C" int kp_tune_lookup(int form, int64_t Il, int64_t m, int64_t n, int64_t Ir,
                              kp_tune_entry* out) {
  if (!out) return KP_ERR_NULL;
  if (!kp::valid_key(form, Il, m, n, Ir)) return KP_ERR_VALUE;
  kp::ModeTile t;
  const bool tuned = kp::tuned_tile(form, Il, m, n, Ir, &t);
  if (!tuned) t = kp::builtin_mode_tile(form, Il, m, n, Ir);
  kp::ModeTile r;
  if (!kp::resolve_mode_tile(form, t, &r)) r = t;
  kp::fill(out, kp::Key{form, Il, m, n, Ir}, r);
  return tuned ? 1 : 0;
}

extern "C" int kp_tune_count(void) {
  std::lock_guard<std::mutex> lock(kp::g_mu);
  return static_cast<int>(kp::table().size());
}

extern "C" int kp_tune_list(kp_tune_entry* out, int cap) {
  std::lock_guard<std::mutex> lock(kp::g_mu);
  const auto& t = kp::table();
  if (cap > 0 && !out) return KP_ERR_NULL;
  int i = 0;
  for (const auto& kv : t) {
    if (i >= cap) break;
    kp::fill(out + i, kv.first, kv.second);
    ++i;
  }
  return static_cast<int>(t.size());
}

extern "C" int kp_tune_clear(void) {
  std::lock_guard<std::mutex> lock(kp::g_mu);
  kp::table().clear();
  return KP_OK;
}

extern "C" int kp_tile_variants(int form, int batch, int32_t* out, int cap) {
  // six ints per tile: nb, fb, bk, occ, pf, kind
  if (!kp::valid_form(form) || (batch != 0 && batch != 1)) return KP_ERR_VALUE;
  if (cap > 0 && !out) return KP_ERR_NULL;
  if (cap < 0) cap = 0;
  return batch ? kp::list_batch_variants(form, out, cap) : kp::list_mode_variants(form, out, cap);
}
