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

namespace life {

// Work decomposition of the chunked (LDS-tiled) kernels, computed on the host.
//   The dictionary is staged in shared memory one atom tile at a time: n_tiles
//   tiles of tile_atoms atoms, each row padded to row_floats (a multiple of 32).
//   Voxels are cut into chunks of kChunkVoxels consecutive voxels; a chunk is one
//   workgroup of kChunkWaves waves and each wave owns up to kWaveVoxels voxels.
constexpr int kChunkWaves = 16;
constexpr int kWaveVoxels = 4;
constexpr int kChunkVoxels = kChunkWaves * kWaveVoxels;
constexpr int kMaxTileRowFloats = 128;      // chunked kernels handle n_theta <= 128
constexpr int kLdsBudget = 160 * 1024 - 1024;

struct TileGeom {
    int row_floats = 0;   // LDS row length (floats), 0 = chunked kernels not applicable
    int tile_atoms = 0;
    int n_tiles = 0;
};

TileGeom tile_geometry(int n_theta, int n_atoms);

// tile_ptr[v*(n_tiles+1) + t]: first DSC position of voxel v whose atom is >= t*tile_atoms
// (the segment's atoms are ascending); tile_ptr[v*(n_tiles+1) + n_tiles] = end of segment.
// chunk_vox[c*kChunkVoxels + wave*kWaveVoxels + j]: voxel owned by slot j of a wave in chunk c
// (-1 = empty), balanced inside each chunk by longest-processing-time assignment.
void chunk_plan(const life_dims *d, const TileGeom &tg, const int32_t *vox_ptr, const int16_t *atom_sorted,
                int32_t *tile_ptr, int32_t *chunk_vox);

}  // namespace life
