// Host-side helpers shared by the C-ABI translation units.
#pragma once

#include "kp.h"
#include "kp_common.h"

namespace kp {

// Tile forced by kp_force_tile (nullptr: use the tuned / default choice).
const ModeTile* tile_override();

int hip_status(hipError_t e);
size_t elem_size(int dtype);
size_t align_up(size_t x);

}  // namespace kp
