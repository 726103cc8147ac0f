// Internal declarations shared by the host plan builder and the device code.
#pragma once

#include "life.h"

namespace life {

constexpr int32_t kMaxTheta = 1024;
constexpr int64_t kMaxNnz = 2147483646;  // int32 positions, with room for nnz itself

life_status validate_dims(const life_dims *d);
life_status validate_indices(const life_dims *d, const int16_t *atom, const int32_t *voxel,
                             const int32_t *fascicle);
life_status plan_host(const life_dims *d, const int16_t *atom, const int32_t *voxel,
                      const int32_t *fascicle, int32_t *dsc_perm, int32_t *vox_ptr,
                      int32_t *wc_perm, int32_t *fas_ptr);

}  // namespace life
