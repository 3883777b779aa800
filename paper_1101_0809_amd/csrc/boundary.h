// boundary.h -- launchers of the open x boundary (pic_grid_desc.xbc = 1) that
// live outside the field kernels: the absorption of particles near the walls.
#pragma once

#include "pic_internal.h"

namespace pic {

// Zero the weight of every particle of sp whose x cell is < PIC_ABSORB or
// >= nx - 1 - PIC_ABSORB (its current of the step is already deposited).
hipError_t launch_absorb(const Ctx& c, const Species& sp, hipStream_t s);

}  // namespace pic
