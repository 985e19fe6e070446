// Tile selection hooks: a process-wide forced tile used by the tests (to cover
// every compiled variant) and by the tuning driver (to time candidates).
#include "kp.h"
#include "kp_internal.h"

namespace kp {
namespace {
ModeTile g_forced;
bool g_force = false;
}  // namespace

const ModeTile* tile_override() { return g_force ? &g_forced : nullptr; }

}  // namespace kp

extern "C" int kp_force_tile(int nb, int fb, int bk, int occ, int pf) {
  if (nb <= 0) {
    kp::g_force = false;
    return KP_OK;
  }
  if (fb <= 0 || bk <= 0 || occ < 0 || pf < 0 || pf > 2) return KP_ERR_VALUE;
  kp::g_forced.nb = nb;
  kp::g_forced.fb = fb;
  kp::g_forced.bk = bk;
  kp::g_forced.occ = occ;
  kp::g_forced.pf = pf;
  kp::g_force = true;
  return KP_OK;
}
