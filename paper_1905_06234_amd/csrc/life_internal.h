// Internal declarations shared by the host plan builder and the device code.
#pragma once

#include <vector>

#include "life.h"

namespace life {

constexpr int32_t kMaxTheta = 1024;
constexpr int64_t kMaxNnz = 2147483646;  // int32 positions, with room for nnz itself

life_status validate_dims(const life_dims *d);
life_status validate_indices(const life_dims *d, const int16_t *atom, const int32_t *voxel,
                             const int32_t *fascicle);
life_status validate_coords(const life_dims *d, const int16_t *voxel_xyz);

// Batched plans: n_inst independent problems sharing D, concatenated into one
// block-diagonal problem; instance k owns voxels [vox_off[k], vox_off[k+1]) and
// fascicles [fas_off[k], fas_off[k+1]), and each nonzero lies in one instance.
life_status validate_instances(const life_dims *d, int n_inst, const int32_t *vox_off, const int32_t *fas_off,
                               const int32_t *voxel, const int32_t *fascicle);

// Number of voxel processing positions: n_voxels for one instance; with several,
// each instance's block is padded to whole chunks so no chunk spans two
// instances.  -1 if it exceeds the 32-bit limit.
int32_t padded_positions(const life_dims *d, int n_inst, const int32_t *vox_off);

// Voxel processing order: instance by instance (n_inst <= 1: one instance, no
// padding); inside an instance voxel id order, or, given grid coordinates, the
// Morton (Z-order) sequence of the coordinates (ties by id), so that consecutive
// voxels form compact blocks.  proc_pos[v] = position of voxel v; proc_vox[k] =
// voxel at position k, -1 for padding (padded_positions entries).
void voxel_order(const life_dims *d, const int16_t *voxel_xyz, int n_inst, const int32_t *vox_off,
                 int32_t *proc_pos, int32_t *proc_vox);

// Host restructuring (see life_plan_host in life.h); proc_pos may be NULL (id
// order); n_pos = number of processing positions; fas_inst (batched plans, else
// NULL) gives each fascicle's instance, the major key of the fascicle ranks, so
// that each instance's fascicles take one contiguous block of ranks.
life_status plan_host(const life_dims *d, const int16_t *atom, const int32_t *voxel, const int32_t *fascicle,
                      const int32_t *proc_pos, int32_t n_pos, const int32_t *fas_inst, int32_t *dsc_perm,
                      int32_t *vox_ptr, int32_t *fas_rank, int32_t *wc_perm, int32_t *fas_ptr);

// Work decomposition of the chunked (LDS-tiled) kernels, computed on the host.
//   The dictionary is staged in shared memory one atom tile at a time: n_tiles
//   tiles of tile_atoms atoms (at most kMaxTileAtoms), each row padded to
//   row_floats (a multiple of 32).
//   Voxels are cut into chunks of kChunkVoxels consecutive voxels of the
//   processing order; a chunk is one workgroup of kChunkWaves waves and each
//   wave owns up to kWaveVoxels voxels.
constexpr int kChunkWaves = 16;
constexpr int kWaveVoxels = 4;
constexpr int kChunkVoxels = kChunkWaves * kWaveVoxels;
constexpr int kMaxTileRowFloats = 128;      // chunked kernels handle n_theta <= 128
constexpr int kLdsBudget = 160 * 1024 - 1024;
// Default size of a staged dictionary tile (4 tiles of 265 atoms at N_theta = 96:
// fewer restagings of D per chunk than 80 KB tiles, measured 4% faster per SBB
// step on the full connectome); a plan may ask for other tile sizes
// (life_plan_flags, life_plan_autotune).
constexpr int kTileBytes = 104 * 1024;
// Dictionary-gradient kernel: per tile, a dense (atom x voxel slot) block of the
// chunk and the chunk's (theta x voxel slot) signal block in LDS, rows of
// kPsiStride floats (64 slots + 4 to spread the banks); a tile has at most
// kMaxTileAtoms atoms so that both fit the LDS budget for every N_theta <= 128.
constexpr int kPsiStride = 68;
constexpr int kMaxTileAtoms = 512;

struct TileGeom {
    int row_floats = 0;   // LDS row length (floats), 0 = chunked kernels not applicable
    int tile_atoms = 0;
    int n_tiles = 0;
    int fas_cap = 0;      // distinct fascicles a chunk may cross (DSC keeps their weights in LDS beside a tile)
};

// Tiles of at most tile_atoms atoms (0: as many as kTileBytes holds), balanced;
// row_floats = 0 when N_theta > 128 or the requested tile leaves no LDS for the
// chunk's weights.
TileGeom tile_geometry(int n_theta, int n_atoms, int tile_atoms = 0);

// Chunks.  Processing positions are cut into groups of kChunkVoxels consecutive
// positions (instance blocks of batched plans are whole groups, so no group spans
// two instances).  A group becomes one chunk, or, when its nonzeros cross more
// than kChunkFasCap distinct fascicles, is halved (recursively) into chunks that
// cross at most that many: the chunked kernels keep one value per distinct
// fascicle of their chunk in LDS (the DSC weights, the WC partial sums).  A
// single voxel that crosses more fascicles makes the plan fall back to the
// generic kernels.  A chunk is one workgroup of kChunkWaves waves; each wave owns
// up to kWaveVoxels voxel slots, balanced inside the chunk by longest-processing-
// time assignment (ties keep processing order).
constexpr int kChunkFasCap = 16384;   // at most (kChunkFasCap is also the 16-bit local index's bound)
constexpr uint16_t kRunStart = 0x8000;

// Chunked layout: for every (chunk c, tile t, wave w) one contiguous range of the
// padded arrays holds the tile-t sub-ranges of the wave's voxel slots j = 0..3,
// each padded with zero-valued entries to a multiple of kStepEntries (one step of
// the wave's lane groups never mixes voxels); chunks are laid out one after the
// other.  Inside a slot's sub-range the atoms never decrease: entries follow the
// DSC order and the pads repeat the last atom.
// wave_work[((c*T + t)*kChunkWaves + w)*kWorkInts + k]:
//   k = 0: first position of the range; k = 1..4: cumulative step counts E1..E4
//   (slot j owns steps [E_j, E_{j+1}), E_0 = 0; kStepEntries entries per step).
constexpr int kStepEntries = 4;
constexpr int kWorkInts = 5;

struct ChunkLayout {
    int n_chunks = 0;
    int64_t n_pad = 0;                  // padded entries
    bool fas_overflow = false;          // a single voxel crosses more than kChunkFasCap fascicles
    int max_fas = 0;                    // largest number of distinct fascicles of a chunk
    std::vector<int32_t> bounds;        // [n_chunks + 1] processing-position range of each chunk
    std::vector<int32_t> chunk_vox;     // [n_chunks * kChunkVoxels] voxel of each slot, -1 = empty
    std::vector<int32_t> wave_work;     // [n_chunks * T * kChunkWaves * kWorkInts]
    std::vector<int64_t> work;          // [n_chunks] padded entries of each chunk
    // padded DSC-order copies: atom, fascicle rank, local fascicle index, value
    std::vector<int16_t> atom_c;
    std::vector<int32_t> fas_c;
    std::vector<uint16_t> loc_c;
    std::vector<float> phi_c;
    // chunk fascicle lists: chunk c crosses the ranks cfas[cfas_ptr[c] .. cfas_ptr[c+1])
    // (ascending); an entry's local index is its rank's place in that list
    std::vector<int32_t> cfas_ptr, cfas;
    // WC pass 1: the nonzeros of each (chunk, tile) bucket ct = c T + t, in WC order
    // (rank, voxel position, atom, ...), at [wc_ent[ct], wc_ent[ct + 1]):
    //   wkey = kRunStart (first entry of a run of one fascicle) | (atom - t TA) << 6
    //          | voxel slot;   wphi = value.
    // Runs are numbered in entry order.  Wave w of the bucket's workgroup takes the
    // entries [wc_wave[ct W + w], wc_wave[ct W + w + 1]) (W = kChunkWaves; the cuts
    // fall on run starts, so no run is split), whose first run is wc_wrun[ct W + w].
    std::vector<int32_t> wc_ent;
    std::vector<uint16_t> wkey;
    std::vector<float> wphi;
    std::vector<int32_t> wc_wave, wc_wrun;
    int64_t n_runs = 0;
    // WC pass 2: the fascicle of rank r sums the run values of runs
    // rr[rr_ptr[r] .. rr_ptr[r+1]) (ascending)
    std::vector<int32_t> rr_ptr, rr;
};

// Voxel slots of chunks with the given position bounds (longest voxel first, ties
// in processing order, each to the least loaded wave with a free slot):
// chunk_vox [n_chunks * kChunkVoxels] (-1 = empty), and for every voxel its chunk
// and slot (vox_chunk, vox_slot: -1 for voxels in no chunk).
void chunk_slots(const life_dims *d, const int32_t *vox_ptr, const int32_t *proc_vox, const std::vector<int32_t> &bounds,
                 std::vector<int32_t> &chunk_vox, std::vector<int32_t> &vox_chunk, std::vector<int32_t> &vox_slot);

// The same restructuring on the device (life_plan_gpu.hip), from device COO arrays.
// Produces the canonical DSC and WC orders and the chunked layout of ChunkLayout
// (bit for bit what plan_host and chunk_layout give), in device memory that the
// caller takes over.  With n_chunks = 0 on return (tile geometry not chunked, or a
// voxel crossing more than kChunkFasCap fascicles) only the canonical orders are
// built.
struct DevLayout {
    int32_t *vox_ptr = nullptr, *fas_v = nullptr, *fas_rank = nullptr, *fas_ext = nullptr, *fas_ptr = nullptr,
            *wc_perm = nullptr, *vox_dsc = nullptr;
    int16_t *atom_v = nullptr;
    float *phi_v = nullptr;
    int n_chunks = 0;
    int64_t n_pad = 0, n_runs = 0;
    int max_fas = 0;
    bool fas_overflow = false;
    std::vector<int32_t> bounds;
    std::vector<int64_t> work;
    int32_t *chunk_vox = nullptr, *wave_work = nullptr, *fas_c = nullptr, *cfas_ptr = nullptr, *cfas = nullptr,
            *wc_wave = nullptr, *wc_wrun = nullptr, *rr_ptr = nullptr, *rr = nullptr;
    int16_t *atom_c = nullptr;
    uint16_t *loc_c = nullptr, *wkey = nullptr;
    float *phi_c = nullptr, *wphi = nullptr;
};
void free_dev_layout(DevLayout *L);
life_status plan_gpu(const life_dims *d, const TileGeom &tg, const int16_t *atom, const int32_t *voxel,
                     const int32_t *fascicle, const float *phi, const int32_t *proc_pos, const int32_t *proc_vox,
                     int32_t n_pos, const int32_t *fas_inst, const int32_t *vox_off, int n_inst, DevLayout *out);

// The chunked layout from the canonical DSC-order arrays (atom_v, fas_v = ranks,
// phi_v, voxel of each DSC position), the WC permutation (wc_perm), the segment
// offsets vox_ptr and the processing order (proc_pos / proc_vox over n_pos
// positions).  Returns LIFE_ERANGE if a padded length exceeds the 32-bit limit.
life_status chunk_layout(const life_dims *d, const TileGeom &tg, const int32_t *vox_ptr, const int16_t *atom_v,
                         const int32_t *fas_v, const float *phi_v, const int32_t *voxel_of_dsc,
                         const int32_t *wc_perm, const int32_t *proc_pos, const int32_t *proc_vox, int32_t n_pos,
                         ChunkLayout *out);

// Workgroup-to-chunk map of the chunked kernels (chunk or -1 per workgroup).
// Consecutive workgroups are dispatched to the 8 XCDs in turn, so workgroup i
// runs on XCD i % 8.  Policies: index order (workgroup i = chunk i); equal
// counts (XCD x gets one contiguous run of n/8 chunks); equal work (XCD x gets
// one contiguous run of chunks holding about 1/8 of the padded entries; the
// runs' lengths differ, shorter ones are filled with -1).  Contiguous runs keep
// neighbouring chunks, which gather nearby weights, on one L2.
enum SchedulePolicy { kScheduleIndex = 0, kScheduleXcdCount = 1, kScheduleXcdWork = 2 };
constexpr SchedulePolicy kScheduleDefault = kScheduleIndex;
constexpr int kXcds = 8;
std::vector<int32_t> chunk_schedule(const std::vector<int64_t> &work, SchedulePolicy policy);

}  // namespace life
