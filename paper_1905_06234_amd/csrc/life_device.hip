// HIP (gfx950) kernels and the C ABI of the LiFE sparse-Tucker products.
//
// DSC  y = M w   (eq. 1, M_v = D Phi_v of eq. 3): a voxel-segmented reduction
//      over the voxel-sorted nonzeros; every y column is accumulated in
//      registers and written exactly once (no atomics).
// WC   g = M^T y  (the transpose product of eq. 6), in two deterministic passes:
//      (1) voxel-major: each nonzero c gets z_c = phi_c <D[:,atom_c], y[:,v]>
//          (the chunked path keeps one sum per run of a fascicle's nonzeros);
//      (2) fascicle-major: g[f] = sum of those values over the fascicle, read
//          through the fascicle-sorted permutation, in a fixed tree order.
// SBB  one SBB-NNLS iteration (Algorithm 1) chains these with a mask kernel, a
//      one-block step-length kernel and an update kernel; every scalar stays on
//      the device and every reduction has a fixed order.
//
// Two implementations of DSC and WC pass 1 exist:
//   chunked (n_theta <= 128): a 1024-thread workgroup owns 64 voxels and works
//     one atom tile at a time (by default a tile of D takes at most 104 KB: 4
//     tiles of 265 atoms for N_theta = 96; a plan may be built with other tile
//     sizes, and life_plan_autotune picks one by timing).
//     DSC stages the tile in LDS; inside a wave, four 16-lane groups each take one
//     nonzero per step, lane l of a group holding theta = 4l .. 4l + 3 and
//     64 + 2l, 65 + 2l, so a step is one ds_read_b128 (the 16 lanes of a group
//     read 256 contiguous bytes), one ds_read_b64 and 6 FMA per lane.  The per-nonzero scalars are loaded
//     coalesced once per 64 nonzeros and broadcast inside each group with a DPP
//     row broadcast (a VALU move, leaving the LDS pipe to the D reads).  This
//     replaces the paper's one-warp-per-sub-vector mapping, which on a 64-wide
//     wavefront with N_theta = 96 would idle lanes and read D through the cache
//     hierarchy at 384 B per nonzero.
//     WC pass 1 forms all the tile's projections of the chunk at once, as the
//     dense block D_tile^T Y_chunk on the matrix cores (exact 8-bit digit
//     products), then each nonzero is one lookup, and a segmented scan leaves one
//     value per run of a fascicle's nonzeros.
//   generic (any n_theta <= 1024): 32 lanes per voxel, D read through L1/L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <utility>
#include <vector>

#include "life_internal.h"

using life::kChunkVoxels;
using life::kChunkWaves;
using life::kWaveVoxels;

namespace {

// Launch gate of the products that only some SBB iterations need: with st set,
// the kernel runs only when the iteration count's parity equals par, decided on
// the device so a whole iteration is enqueued without a host round trip.
struct Gate {
    const life_sbb_state *st;
    int par;
};
__device__ inline bool gated_off(const Gate &g) { return g.st && (int)(g.st->iter & 1) != g.par; }

// Work item of this workgroup.  Consecutive workgroups are dispatched to the 8
// XCDs in turn; this gives each XCD one contiguous range of items, so that
// neighbouring chunks (or fascicle ranks) share that XCD's L2.  A bijection on
// [0, gridDim.x).
__device__ __forceinline__ int xcd_item()
{
    const int n = (int)gridDim.x, i = (int)blockIdx.x;
    const int per = n >> 3, rem = n & 7, x = i & 7, k = i >> 3;
    return x * per + (x < rem ? x : rem) + k;
}

constexpr int kBlock = 256;                  // threads per block of the generic / glue kernels
constexpr int kSeg = 32;                     // lanes per voxel segment (generic kernels)
constexpr int kSegPerBlock = kBlock / kSeg;  // voxels per block (generic kernels)
constexpr int kFasLanes = 16;                // lanes per fascicle in the WC sum
constexpr int kSumBlock = 512;               // threads per block of the WC sum (measured best)
constexpr int kFasPerBlock = kSumBlock / kFasLanes;
constexpr int kWG = kChunkWaves * 64;        // threads per chunk workgroup
constexpr int kAlphaThreads = 1024;

// ----------------------------------------------------------------------------- device helpers

// Sum a double over the block in a fixed order and store it at out[slot].
template <int NT>
__device__ __forceinline__ void block_sum_store(double v, double *out, int slot)
{
    __shared__ double sh[NT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) s += sh[i];
        out[slot] = s;
    }
}

// Fixed-order sum of n doubles by one block of kAlphaThreads; valid in every thread.
__device__ double block_sum_array(const double *a, int n)
{
    __shared__ double sh[kAlphaThreads];
    // four independent running sums per thread (four loads in flight), combined in a fixed order
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * kAlphaThreads < n; i += 4 * kAlphaThreads) {
        s0 += a[i];
        s1 += a[i + kAlphaThreads];
        s2 += a[i + 2 * kAlphaThreads];
        s3 += a[i + 3 * kAlphaThreads];
    }
    for (; i < n; i += kAlphaThreads) s0 += a[i];
    sh[threadIdx.x] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    for (int w = kAlphaThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// ----------------------------------------------------------------------------- chunked kernels

// Stage atoms [a0, a0 + nrow) of D into LDS rows of ROW floats (zero padded).
// vec: rows are contiguous (ROW == nth) and D is 16-byte aligned.
template <int ROW>
__device__ __forceinline__ void stage_tile(float *lds, const float *__restrict__ D, int a0, int nrow, int nth,
                                           bool vec)
{
    if (vec) {
        // rows are contiguous in D: plain float4 copy
        const float4 *src = reinterpret_cast<const float4 *>(D + (size_t)a0 * nth);
        float4 *dst = reinterpret_cast<float4 *>(lds);
        const int n4 = nrow * (ROW / 4);
        for (int i = threadIdx.x; i < n4; i += kWG) dst[i] = src[i];
    } else {
        const int n = nrow * ROW;
        for (int i = threadIdx.x; i < n; i += kWG) {
            const int r = i / ROW, c = i - r * ROW;
            lds[i] = c < nth ? D[(size_t)(a0 + r) * nth + c] : 0.f;
        }
    }
}

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// DPP moves inside 16-lane rows (VALU only, no LDS traffic).
template <int CTRL>
__device__ __forceinline__ float dppf(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, true));
}
// One step of a wave-wide inclusive segmented scan of (v, f) (f: a segment starts
// in the lane's range) on DPP moves: the partial from the lane CTRL selects (row
// shift or row broadcast; lanes without a source, or outside ROW_MASK, get the
// neutral (0, 0)) is added unless a segment starts in the lane's own range.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void seg_scan_step(float &v, int &f)
{
    const float vu = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
    const int fu = __builtin_amdgcn_update_dpp(0, f, CTRL, ROW_MASK, 0xf, true);
    if (!f) {
        v += vu;
        f |= fu;
    }
}
// broadcast lane K of every row to the row (row_newbcast)
template <int K>
__device__ __forceinline__ int bcast16(int x)
{
    return __builtin_amdgcn_mov_dpp(x, 0x150 + K, 0xf, 0xf, true);
}
template <int K>
__device__ __forceinline__ float bcast16f(float x) { return dppf<0x150 + K>(x); }
constexpr int kSE = life::kStepEntries;      // entries per step (= lane groups per wave)
constexpr int kGL = 64 / kSE;                // lanes per group (16)
constexpr int kBatch = 64;                   // entries per batch: kGL steps

// Work range of this wave in tile t (see life::chunk_layout): slot j owns entries
// [q0 + kSE*E_j, q0 + kSE*E_{j+1}).
struct WaveRange {
    int p[kWaveVoxels + 1];
    __device__ __forceinline__ WaveRange(const int32_t *__restrict__ wave_work, int chunk, int t, int T, int wave)
    {
        const int32_t *ww = wave_work + ((size_t)(chunk * T + t) * kChunkWaves + wave) * life::kWorkInts;
        const int q0 = uni(ww[0]);
        p[0] = q0;
#pragma unroll
        for (int j = 1; j <= kWaveVoxels; ++j) p[j] = q0 + kSE * uni(ww[j]);
    }
    // start of the batch that follows the batch starting at b (p[kWaveVoxels] = none):
    // the next 64 entries of the same slot, else the start of the next non-empty slot
    __device__ __forceinline__ int next(int b) const
    {
        if (b >= p[kWaveVoxels]) return p[kWaveVoxels];
        const int e = b < p[1] ? p[1] : b < p[2] ? p[2] : b < p[3] ? p[3] : p[4];
        return b + kBatch < e ? b + kBatch : e;
    }
    // in-bounds entry index for this lane in the batch starting at b (clamped)
    __device__ __forceinline__ int entry(int b, int mypos) const
    {
        return b + mypos < p[kWaveVoxels] ? b + mypos : p[0];
    }
};

// Lane layout of the chunked DSC: a wave is kSE groups of kGL = 16 lanes; at step
// k of a batch, group g handles entry kSE*k + g, and lane l of a group holds
// theta = 64q + 4l + {0..3} for q < NC/2 (a float4 read per 64-float block of the
// LDS row) and, for odd NC, theta = 64 (NC/2) + 2l + {0, 1} (a float2 read).
// The lane that loads the scalars of entry kSE*k + g is lane kGL*g + k, so a row
// broadcast of lane k hands every group its entry.  Batches never span two voxel
// slots; full batches run 16 branch-free steps, the last batch of a slot is
// guarded per step.

// DSC: y[:, v] = sum_{c in seg(v)} D[:, atom_c] * (phi_c * w[fas_c])   (minus b[:, v] if bsub)
// NC = 32-float chunks per LDS row (N_theta <= 32 NC).
// The weights of the chunk's fascicles are first gathered into LDS (wl, after the
// dictionary tile: one value per distinct fascicle of the chunk, in rank order, so
// the gather reads ascending addresses), and every nonzero reads its weight there
// through its local index.
template <int NC>
__global__ __launch_bounds__(kWG) void k_dsc_chunk(const int32_t *__restrict__ chunk_map,
                                                   const int32_t *__restrict__ chunk_vox,
                                                   const int32_t *__restrict__ wave_work,
                                                   const uint2 *__restrict__ rec,
                                                   const int32_t *__restrict__ cfas_ptr,
                                                   const int32_t *__restrict__ cfas,
                                                   const float *__restrict__ w,
                                                   const float *__restrict__ D,
                                                   const float *__restrict__ bsub,
                                                   float *__restrict__ y, double *__restrict__ part,
                                                   int nth, int na, int T, int TA, bool vec)
{
    extern __shared__ float4 lds4[];
    float *lds = reinterpret_cast<float *>(lds4);
    constexpr int ROW = NC * 32;
    constexpr int PER = NC * 2;
    constexpr int NQ = NC / 2, NR = NC % 2;   // 64-float blocks of a row (16-byte reads), 32-float tail
    const int chunk = chunk_map[blockIdx.x];   // -1: no chunk for this workgroup (uniform exit)
    if (chunk < 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float *wl = lds + TA * ROW;
    __shared__ int zero_w[kChunkWaves];   // zero weights among the chunk's fascicles, per wave
    const int f0 = cfas_ptr[chunk], nl = cfas_ptr[chunk + 1] - f0;
    {
        int nz = 0;
        for (int i = threadIdx.x; i < nl; i += kWG) {
            const float wv = w[cfas[f0 + i]];
            wl[i] = wv;
            nz += wv == 0.f;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) nz += __shfl_xor(nz, o, 64);
        if (lane == 0) zero_w[wave] = nz;
    }
    // group g of the wave writes slot g at the end; its b values are requested now
    const int g = lane / kGL, l16 = lane % kGL;
    const int vme = chunk_vox[chunk * kChunkVoxels + wave * kWaveVoxels + g];
    float bme[PER];
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int th = e < 4 * NQ ? 64 * (e / 4) + 4 * l16 + e % 4 : 64 * NQ + 2 * l16 + (e - 4 * NQ);
        bme[e] = bsub && vme >= 0 && th < nth ? bsub[(size_t)vme * nth + th] : 0.f;
    }
    // the first tile (its LDS region is not the weights')
    stage_tile<ROW>(lds, D, 0, min(na, TA), nth, vec);
    __syncthreads();
    // zero-weight skip (Sec. 2.2) where at least 1/8 of the chunk's weights are zero:
    // a batch without a nonzero product then costs nothing, and one with few moves
    // them to its first steps; denser chunks run the plain loop (no per-batch test)
    int n_zero = 0;
#pragma unroll
    for (int i = 0; i < kChunkWaves; ++i) n_zero += zero_w[i];
    const bool skip = uni(8 * n_zero >= nl ? 1 : 0) != 0;
    const int mypos = kSE * l16 + g;       // entry of a batch whose scalars this lane loads
    float acc[kWaveVoxels][PER];
#pragma unroll
    for (int j = 0; j < kWaveVoxels; ++j)
#pragma unroll
        for (int e = 0; e < PER; ++e) acc[j][e] = 0.f;

    auto tiles = [&](auto skip_tag) {
        constexpr bool SKIP = decltype(skip_tag)::value;
        for (int t = 0; t < T; ++t) {
            const int a0 = t * TA;
            // two-stage prefetch over batch starts: the scalars of batch i+2 and the
            // w gather of batch i+1 are in flight while batch i is computed; the first
            // two batches of a tile are requested before its staging
            const WaveRange R(wave_work, chunk, t, T, wave);
            const bool any = R.p[kWaveVoxels] != R.p[0];
            int bq = R.next(R.p[0]);
            uint2 r = make_uint2(0u, 0u), r1 = make_uint2(0u, 0u);
            if (any) {
                r = rec[R.entry(R.p[0], mypos)];
                r1 = rec[R.entry(bq, mypos)];
            }
            if (t > 0) {   // (tile 0 is staged above)
                __syncthreads();
                stage_tile<ROW>(lds, D, a0, min(na, a0 + TA) - a0, nth, vec);
                __syncthreads();
            }
            if (!any) continue;   // nothing for this wave in this tile
            int ix;
            int a_0 = (int)(r.x & 0xffffu), f_0 = (int)(r.x >> 16);
            float ph_0 = __uint_as_float(r.y);
            r = r1;
            int a_1 = (int)(r.x & 0xffffu), f_1 = (int)(r.x >> 16);
            float ph_1 = __uint_as_float(r.y);
            float w_0 = wl[f_0];
#pragma unroll
            for (int j = 0; j < kWaveVoxels; ++j) {
                for (int b = R.p[j]; b < R.p[j + 1]; b += kBatch) {
                    const int m = min(kBatch, R.p[j + 1] - b);
                    const int a_c = a_0;
                    const float ph_c = ph_0, w_c = w_0;
                    const float w_1 = wl[f_1];
                    bq = R.next(bq);
                    ix = R.entry(bq, mypos);
                    a_0 = a_1;
                    ph_0 = ph_1;
                    w_0 = w_1;
                    r = rec[ix];
                    a_1 = (int)(r.x & 0xffffu);
                    f_1 = (int)(r.x >> 16);
                    ph_1 = __uint_as_float(r.y);
                    const bool valid = mypos < m;
                    int aoff = valid ? (a_c - a0) * ROW : 0;
                    float s = valid ? ph_c * w_c : 0.f;   // loop-invariant product hoisted (Sec. 4.1)
                    // (SKIP: a batch without a nonzero product costs nothing; one with few
                    // nonzero products moves them to its first steps)
#define LIFE_DSC_STEP(K)                                                                  \
        {                                                                                     \
            const int ak = bcast16<K>(aoff);                                                  \
            const float sk = bcast16f<K>(s);                                                  \
            _Pragma("unroll") for (int q = 0; q < NQ; ++q) {                                  \
                const float4 d = *reinterpret_cast<const float4 *>(lds + ak + 4 * l16 + 64 * q); \
                acc[j][4 * q + 0] = fmaf(d.x, sk, acc[j][4 * q + 0]);                         \
                acc[j][4 * q + 1] = fmaf(d.y, sk, acc[j][4 * q + 1]);                         \
                acc[j][4 * q + 2] = fmaf(d.z, sk, acc[j][4 * q + 2]);                         \
                acc[j][4 * q + 3] = fmaf(d.w, sk, acc[j][4 * q + 3]);                         \
            }                                                                                 \
            if constexpr (NR) {                                                               \
                const float2 d = *reinterpret_cast<const float2 *>(lds + ak + 2 * l16 + 64 * NQ); \
                acc[j][4 * NQ + 0] = fmaf(d.x, sk, acc[j][4 * NQ + 0]);                       \
                acc[j][4 * NQ + 1] = fmaf(d.y, sk, acc[j][4 * NQ + 1]);                       \
            }                                                                                 \
        }
                    int n = m;   // entries to cover (the rest carry zero products)
                    if constexpr (SKIP) {
                        const uint64_t nzm = __ballot(s != 0.f);
                        const int cnt = __popcll(nzm);
                        if (cnt == 0) n = 0;
                        else if ((cnt + 15) / 16 < (m + 15) / 16) {
                        // compaction, when it saves steps: the r-th nonzero product (in lane
                        // order) goes to position r = kSE k + g of the batch (step k, group g),
                        // the zero products after them; every lane sends one value, so every
                        // lane receives one (a permutation of the wave)
                        const uint64_t below = (1ull << lane) - 1;
                        const int r = s != 0.f ? __popcll(nzm & below) : cnt + __popcll(~nzm & below);
                        const int dst = kGL * (r % kSE) + r / kSE;
                        aoff = __builtin_amdgcn_ds_permute(4 * dst, aoff);
                        s = __int_as_float(__builtin_amdgcn_ds_permute(4 * dst, __float_as_int(s)));
                        n = cnt;
                        }
                    }
                    if (n == kBatch) {
                        LIFE_DSC_STEP(0) LIFE_DSC_STEP(1) LIFE_DSC_STEP(2) LIFE_DSC_STEP(3)
                        LIFE_DSC_STEP(4) LIFE_DSC_STEP(5) LIFE_DSC_STEP(6) LIFE_DSC_STEP(7)
                        LIFE_DSC_STEP(8) LIFE_DSC_STEP(9) LIFE_DSC_STEP(10) LIFE_DSC_STEP(11)
                        LIFE_DSC_STEP(12) LIFE_DSC_STEP(13) LIFE_DSC_STEP(14) LIFE_DSC_STEP(15)
                    } else if (SKIP && n > 0) {
                        // blocks of four steps (16 entries); entries past n have zero products
                        LIFE_DSC_STEP(0) LIFE_DSC_STEP(1) LIFE_DSC_STEP(2) LIFE_DSC_STEP(3)
                        if (n > 16) { LIFE_DSC_STEP(4) LIFE_DSC_STEP(5) LIFE_DSC_STEP(6) LIFE_DSC_STEP(7) }
                        if (n > 32) { LIFE_DSC_STEP(8) LIFE_DSC_STEP(9) LIFE_DSC_STEP(10) LIFE_DSC_STEP(11) }
                        if (n > 48) { LIFE_DSC_STEP(12) LIFE_DSC_STEP(13) LIFE_DSC_STEP(14) LIFE_DSC_STEP(15) }
                    } else if (!SKIP) {
                        const int ns = m / kSE;     // sub-ranges are padded to whole steps
#define LIFE_DSC_GSTEP(K) if (K < ns) LIFE_DSC_STEP(K)
                        LIFE_DSC_GSTEP(0) LIFE_DSC_GSTEP(1) LIFE_DSC_GSTEP(2) LIFE_DSC_GSTEP(3)
                        LIFE_DSC_GSTEP(4) LIFE_DSC_GSTEP(5) LIFE_DSC_GSTEP(6) LIFE_DSC_GSTEP(7)
                        LIFE_DSC_GSTEP(8) LIFE_DSC_GSTEP(9) LIFE_DSC_GSTEP(10) LIFE_DSC_GSTEP(11)
                        LIFE_DSC_GSTEP(12) LIFE_DSC_GSTEP(13) LIFE_DSC_GSTEP(14)
#undef LIFE_DSC_GSTEP
                    }
#undef LIFE_DSC_STEP
                }
            }
        }
    };
    if (skip)
        tiles(std::true_type{});
    else
        tiles(std::false_type{});

    // combine the group partials (fixed butterfly: every group gets the sums) and
    // write each column once, group g writing slot g
    double sq = 0.0;
    float mine[PER];
#pragma unroll
    for (int j = 0; j < kWaveVoxels; ++j) {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            float x = acc[j][e];
            x += __shfl_xor(x, 16, 64);
            x += __shfl_xor(x, 32, 64);
            if (j == 0 || g == j) mine[e] = x;
        }
    }
    if (vme >= 0) {
        float *yv = y + (size_t)vme * nth;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int th = e < 4 * NQ ? 64 * (e / 4) + 4 * l16 + e % 4 : 64 * NQ + 2 * l16 + (e - 4 * NQ);
            if (th < nth) {
                const float r = mine[e] - bme[e];
                yv[th] = r;
                sq += (double)r * (double)r;
            }
        }
    }
    if (part) block_sum_store<kWG>(sq, part, chunk);
}

// ----------------------------------------------------------------------------- WC pass 1 on the matrix cores
// For one chunk and one atom tile every needed projection <D[:, a], y[:, v]> is an
// entry of the dense block P = D_tile^T Y_chunk (atoms x 64 voxel slots), formed on
// v_mfma_i32_32x32x32_i8; each nonzero then costs one LDS lookup.
// Exact integer products: a column (an atom of D, a voxel slot of y) is scaled by
// a power of two 2^k that puts its largest magnitude in [2^29, 2^30) and rounded
// to an integer q (|q| <= 2^30, to 2^-31 of the column maximum), written as four
// balanced 8-bit digits q = q3 2^24 + q2 2^16 + q1 2^8 + q0 (q0..q2 in [-128, 127],
// |q3| <= 64).  The matrix cores sum the digit products exactly in 32-bit
// integers, grouped by weight: C6 = S33, C5 = S32 + S23, C4 = S31 + S22 + S13,
// C3 = S30 + S21 + S12 + S03 (S_ij = sum over theta of digit i of D times digit j
// of y); the terms of weight 2^16 and below are dropped (about 2^-30 of the
// largest possible product sum, and symmetric about zero).  Then
// P = (2^24 C6 + 2^16 C5 + 2^8 C4 + C3) 2^(24 - k_a - k_v), formed exactly in
// double and rounded once to float: no accumulation bias (FP32 accumulation on the
// matrix cores rounds toward zero), and about 2^-24 relative error per projection.
// Every element of P depends only on its own atom column and voxel column, so
// results do not depend on the chunking.
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

constexpr int kPS = 64;     // LDS row stride of P (floats): one row per atom, one column per slot
constexpr int kQ8Pad = 16;  // bytes after each slot's digits in LDS (spreads the banks)
constexpr int kDigits = 4;

// exponent k with m 2^k in [2^29, 2^30) (0 when m is zero or not finite), clamped so
// that 2^(24-k) and 2^-k stay normal floats
__device__ __forceinline__ int q30_exp(float m)
{
    if (!(m > 0.f) || !(m <= 3.4028234e38f)) return 0;
    int e;
    (void)frexpf(m, &e);
    return min(100, max(-100, 30 - e));
}

// balanced base-256 digits of the integer nearest x (|x| <= 2^30)
__device__ __forceinline__ void q30_digits(float x, int8_t *d, int stride)
{
    int q = (int)rintf(x);
#pragma unroll
    for (int g = 0; g < kDigits - 1; ++g) {
        const int dg = ((q + 128) & 255) - 128;
        d[g * stride] = (int8_t)dg;
        q = (q - dg) >> 8;
    }
    d[(kDigits - 1) * stride] = (int8_t)q;
}

// A operands of P = D_tile^T Y: one wave per (tile t, atom block ab of 32, row r);
// for a = t TA + 32 ab + r and theta = 32 ks + 16 hf + i, byte i of
// frag[(((t AB + ab) KS + ks) kDigits + g) 64 + 32 hf + r] is digit g of
// 2^{k_a} D[theta][a] (zero outside the tile, the dictionary or N_theta), and
// dscale[(t AB + ab) 32 + r] = 2^{24 - k_a}.  N_theta <= 128 (KS <= 4).
__global__ __launch_bounds__(kBlock) void k_split_dt(const float *__restrict__ D, i32x4 *__restrict__ frag,
                                                      float *__restrict__ dscale, int nth, int na, int T, int TA,
                                                      int AB, int KS, Gate gate)
{
    if (gated_off(gate)) return;
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (i >= T * AB * 32) return;   // uniform per wave
    const int t = i / (AB * 32), rem = i - t * AB * 32, ab = rem / 32, r = rem % 32;
    const int al = 32 * ab + r, a = t * TA + al;
    const bool ok = al < TA && a < na;
    const float x0 = (ok && lane < nth) ? D[(size_t)a * nth + lane] : 0.f;
    const float x1 = (ok && lane + 64 < nth) ? D[(size_t)a * nth + lane + 64] : 0.f;
    float m = fmaxf(fabsf(x0), fabsf(x1));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    const int e = q30_exp(m);
    if (lane == 0) dscale[i] = ldexpf(1.f, 24 - e);
    int8_t *f = reinterpret_cast<int8_t *>(frag);
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        const int th = lane + 64 * hh;
        if (th < 32 * KS) {
            const int ks = th / 32, hf = (th % 32) / 16, q = th % 16;
            const size_t base = ((size_t)((t * AB + ab) * KS + ks) * kDigits * 64 + 32 * hf + r) * 16 + q;
            q30_digits(ldexpf(hh ? x1 : x0, e), f + base, 64 * 16);
        }
    }
}

// WC pass 1: one value per run of one fascicle's nonzeros in one (chunk, tile):
// zrun[r] = sum over the run's entries e of phi_e * <D[:, atom_e], y[:, v_e]>.
// Per tile, the waves first form P = D_tile^T Y_chunk in LDS (units of one 32-atom
// block and one 32-slot half, dealt round-robin); then every wave walks its own
// entry range of the (chunk, tile) bucket (cut at run starts) in batches of 64
// consecutive entries, four batches requested at once: each lane looks up its
// entry's projection in P, and a segmented scan over the batch (DPP row shifts and
// row broadcasts with run-start flags, fixed order) sums each run; the lane at a
// run's end writes it, a run that crosses into the next batch carries its partial
// sum there.
// LDS: P [32 AB][kPS] floats, the digits of Y [4 digits][64 slots][YS] bytes
// (YS = 32 KS + kQ8Pad), the 64 slot scales.
template <int KS>
__global__ __launch_bounds__(kWG) void k_wcr_mfma(const int32_t *__restrict__ chunk_map,
                                                  const int32_t *__restrict__ chunk_vox,
                                                  const uint2 *__restrict__ wrec,
                                                  const int32_t *__restrict__ wc_wave,
                                                  const int32_t *__restrict__ wc_wrun,
                                                  const i32x4 *__restrict__ frag,
                                                  const float *__restrict__ dscale,
                                                  const float *__restrict__ y,
                                                  float *__restrict__ zrun, int nth, int T, int AB, Gate gate)
{
    if (gated_off(gate)) return;   // uniform over the grid
    extern __shared__ float4 lds4[];
    float *P = reinterpret_cast<float *>(lds4);
    const int YS = 32 * KS + kQ8Pad;   // bytes per slot and digit
    int8_t *Yq = reinterpret_cast<int8_t *>(P + AB * 32 * kPS);   // [kDigits][64 slots][YS]
    float *yscale = reinterpret_cast<float *>(Yq + kDigits * kChunkVoxels * YS);
    const int chunk = chunk_map[blockIdx.x];   // -1: no chunk for this workgroup (uniform exit)
    if (chunk < 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    // this wave's bucket range in a tile and its first two batches of records (for
    // tile 0 requested before the y columns, for the others before P is formed)
    int eb = 0, ee = 0;
    uint2 r0 = make_uint2(0u, 0u), r1 = make_uint2(0u, 0u);
    auto first_records = [&](int t) {
        const int wi = (chunk * T + t) * kChunkWaves + wave;
        eb = uni(wc_wave[wi]);
        ee = uni(wc_wave[wi + 1]);
        if (eb < ee) {
            r0 = wrec[eb + lane < ee ? eb + lane : ee - 1];
            r1 = wrec[eb + 64 + lane < ee ? eb + 64 + lane : ee - 1];
        }
    };
    first_records(0);

    // the chunk's y columns (all requested at once), each scaled by its own power of
    // two and cut into digits
    float xs0[kWaveVoxels], xs1[kWaveVoxels];
#pragma unroll
    for (int j = 0; j < kWaveVoxels; ++j) {
        const int v = uni(chunk_vox[chunk * kChunkVoxels + wave * kWaveVoxels + j]);
        xs0[j] = v >= 0 && lane < nth ? y[(size_t)v * nth + lane] : 0.f;
        xs1[j] = v >= 0 && lane + 64 < nth ? y[(size_t)v * nth + lane + 64] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kWaveVoxels; ++j) {
        const int slot = wave * kWaveVoxels + j;
        const float x0 = xs0[j], x1 = xs1[j];
        float m = fmaxf(fabsf(x0), fabsf(x1));
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
        const int e = q30_exp(m);
        if (lane == 0) yscale[slot] = ldexpf(1.f, -e);
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int th = lane + 64 * hh;
            if (th < 32 * KS) q30_digits(ldexpf(hh ? x1 : x0, e), Yq + slot * YS + th, kChunkVoxels * YS);
        }
    }

    for (int t = 0; t < T; ++t) {
        if (t > 0) first_records(t);   // (their latency hides behind the matrix-core phase)
        __syncthreads();   // Y is staged / the previous tile's lookups are done with P
        // units (32-atom block, 32-slot half) dealt round-robin to the 16 waves: the
        // matrix cores bound this phase, so the units are spread over all four SIMDs
        // (with one unit per block the busiest SIMD would run a third more of them)
#pragma unroll 1
        for (int u = wave; u < 2 * AB; u += kChunkWaves) {
            const int ab = u >> 1, h = u & 1;
            const i32x4 *fa = frag + (size_t)(t * AB + ab) * KS * kDigits * 64 + lane;
            const int col = lane & 31, kh = 16 * (lane >> 5);
            const float *ds = dscale + (size_t)(t * AB + ab) * 32;
            i32x16 c6 = {}, c5 = {}, c4 = {}, c3 = {};
            const int8_t *yb = Yq + (32 * h + col) * YS + kh;
            for (int ks = 0; ks < KS; ++ks) {
                i32x4 a[kDigits];
#pragma unroll
                for (int g = 0; g < kDigits; ++g) a[g] = fa[(ks * kDigits + g) * 64];
                // one B digit at a time (fewer live registers): digit j meets A digits
                // i >= 3 - j, and the product goes to the class of weight i + j
                const int8_t *yk = yb + 32 * ks;
                i32x4 b = *reinterpret_cast<const i32x4 *>(yk + 3 * kChunkVoxels * YS);
                c6 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[3], b, c6, 0, 0, 0);
                c5 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[2], b, c5, 0, 0, 0);
                c4 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[1], b, c4, 0, 0, 0);
                c3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[0], b, c3, 0, 0, 0);
                b = *reinterpret_cast<const i32x4 *>(yk + 2 * kChunkVoxels * YS);
                c5 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[3], b, c5, 0, 0, 0);
                c4 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[2], b, c4, 0, 0, 0);
                c3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[1], b, c3, 0, 0, 0);
                b = *reinterpret_cast<const i32x4 *>(yk + kChunkVoxels * YS);
                c4 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[3], b, c4, 0, 0, 0);
                c3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[2], b, c3, 0, 0, 0);
                b = *reinterpret_cast<const i32x4 *>(yk);
                c3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[3], b, c3, 0, 0, 0);
            }
            // accumulator r of lane l holds (atom row 8 (r/4) + 4 (l/32) + r%4, slot 32 h + l%32)
            const float sv = yscale[32 * h + col];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
                // |C6| <= 2^19, |C5| <= 2^21, |C4| <= 2^22, |C3| < 2^22.6 for K <= 128, so both
                // halves are exact in 32-bit integers and their combination in double
                const int hi = c6[r] * 256 + c5[r], lo = c4[r] * 256 + c3[r];
                const double exact = fma((double)hi, 65536.0, (double)lo);
                P[(32 * ab + row) * kPS + 32 * h + col] = ((float)exact * ds[row]) * sv;
            }
        }
        __syncthreads();
        if (eb >= ee) continue;
        int run = uni(wc_wrun[(chunk * T + t) * kChunkWaves + wave]);      // index of the run open before the current batch, plus one
        float carry = 0.f;
        for (int b0 = eb; b0 < ee; b0 += 4 * 64) {
            // four batches of keys and values requested at once, and the key after them
            int kk[4];
            float pp[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = b0 + 64 * u + lane;
                uint2 r = u == 0 ? r0 : r1;
                if (u > 1 || b0 != eb) r = wrec[e < ee ? e : ee - 1];
                kk[u] = e < ee ? (int)r.x : (int)life::kRunStart;
                pp[u] = e < ee ? __uint_as_float(r.y) : 0.f;
            }
            const int after = b0 + 256 < ee ? (int)wrec[b0 + 256].x : (int)life::kRunStart;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int b = b0 + 64 * u;
                if (b >= ee) break;   // uniform
                const int key = kk[u];
                const float ph = pp[u];
                const bool in = b + lane < ee;
                const bool st = (key & life::kRunStart) != 0;
                float v = in ? ph * P[((key >> 6) & 0x1ff) * kPS + (key & 63)] : 0.f;
                if (lane == 0 && !st) v += carry;
                // inclusive segmented scan (a run start stops the sums from the left)
                int f = st ? 1 : 0;
                seg_scan_step<0x111, 0xf>(v, f);   // row_shr:1, 2, 4, 8 inside 16-lane rows
                seg_scan_step<0x112, 0xf>(v, f);
                seg_scan_step<0x114, 0xf>(v, f);
                seg_scan_step<0x118, 0xf>(v, f);
                seg_scan_step<0x142, 0xa>(v, f);   // row_bcast:15 into rows 1 and 3
                seg_scan_step<0x143, 0xc>(v, f);   // row_bcast:31 into rows 2 and 3
                const uint64_t starts = __ballot(st);
                // the entry after this batch (a start past the range)
                const int next_key0 = u < 3 ? __shfl(kk[u < 3 ? u + 1 : 3], 0, 64) : after;
                const bool nxt = lane < 63 ? ((starts >> (lane + 1)) & 1) != 0 : (next_key0 & life::kRunStart) != 0;
                const int before = __popcll(starts & (lane == 63 ? ~0ull : ((2ull << lane) - 1)));
                if (in && nxt) zrun[run + before - 1] = v;
                run += __popcll(starts & __ballot(in));
                carry = __shfl(v, 63, 64);   // used only if the next batch does not start a run
            }
        }
    }
}

// ----------------------------------------------------------------------------- generic kernels

// y[:, v] = sum_{c in seg(v)} D[:, atom_c] * (phi_c * w[fas_c])   (minus b[:, v] if bsub)
// NT = accumulator slots per lane: lane l covers theta = l + 32 t, t < NT.
template <int NT>
__global__ __launch_bounds__(kBlock) void k_dsc(const int32_t *__restrict__ vptr,
                                                 const int16_t *__restrict__ atom,
                                                 const int32_t *__restrict__ fas,
                                                 const float *__restrict__ phi,
                                                 const float *__restrict__ w,
                                                 const float *__restrict__ D,
                                                 const float *__restrict__ bsub,
                                                 float *__restrict__ y, double *__restrict__ part,
                                                 int nth, int nv)
{
    const int lane = threadIdx.x & (kSeg - 1);
    const int v = blockIdx.x * kSegPerBlock + (threadIdx.x / kSeg);
    float acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = 0.f;
    if (v < nv) {
        const int beg = vptr[v], end = vptr[v + 1];
        for (int base = beg; base < end; base += kSeg) {
            const int j = base + lane;
            int a = 0;
            float s = 0.f;
            if (j < end) {
                a = atom[j];
                s = phi[j] * w[fas[j]];
            }
            const int cnt = min(kSeg, end - base);
            for (int k = 0; k < cnt; ++k) {
                const float sk = __shfl(s, k, kSeg);
                const int ak = __shfl(a, k, kSeg);
                if (sk != 0.f) {
                    const float *__restrict__ d = D + (size_t)ak * nth + lane;
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        if (lane + kSeg * t < nth) acc[t] = fmaf(d[kSeg * t], sk, acc[t]);
                }
            }
        }
    }
    double sq = 0.0;
    if (v < nv) {
        float *yv = y + (size_t)v * nth;
        const float *bv = bsub ? bsub + (size_t)v * nth : nullptr;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int th = lane + kSeg * t;
            if (th < nth) {
                float r = acc[t];
                if (bv) r -= bv[th];
                yv[th] = r;
                sq += (double)r * (double)r;
            }
        }
    }
    if (part) block_sum_store<kBlock>(sq, part, blockIdx.x);
}

// WC pass 1 (generic): z[c] = phi_c * <D[:, atom_c], y[:, v]>, 32 lanes per voxel.
template <int NT>
__global__ __launch_bounds__(kBlock) void k_wc_z(const int32_t *__restrict__ vptr,
                                                  const int16_t *__restrict__ atom,
                                                  const float *__restrict__ phi,
                                                  const float *__restrict__ D,
                                                  const float *__restrict__ y,
                                                  float *__restrict__ z, int nth, int nv, Gate gate)
{
    if (gated_off(gate)) return;
    const int lane = threadIdx.x & (kSeg - 1);
    const int v = blockIdx.x * kSegPerBlock + (threadIdx.x / kSeg);
    if (v >= nv) return;
    float yv[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int th = lane + kSeg * t;
        yv[t] = th < nth ? y[(size_t)v * nth + th] : 0.f;
    }
    const int beg = vptr[v], end = vptr[v + 1];
    for (int base = beg; base < end; base += kSeg) {
        const int j = base + lane;
        int a = 0;
        float p = 0.f;
        if (j < end) {
            a = atom[j];
            p = phi[j];
        }
        const int cnt = min(kSeg, end - base);
        float mine = 0.f;
        for (int k = 0; k < cnt; ++k) {
            const int ak = __shfl(a, k, kSeg);
            const float *__restrict__ d = D + (size_t)ak * nth + lane;
            float q = 0.f;
#pragma unroll
            for (int t = 0; t < NT; ++t)
                if (lane + kSeg * t < nth) q = fmaf(d[kSeg * t], yv[t], q);
#pragma unroll
            for (int o = kSeg / 2; o > 0; o >>= 1) q += __shfl_xor(q, o, kSeg);
            if (lane == k) mine = q;
        }
        if (j < end) z[j] = p * mine;
    }
}

// WC pass 2: g[out(r)] = sum_{j in seg(r)} z[wperm[j]] for the fascicle of rank r
// (16 lanes per fascicle; each lane keeps 4 index loads and 4 gathers in flight;
// fixed summation tree); out(r) = gmap[r] (caller order) or r.
__global__ __launch_bounds__(kSumBlock) void k_wc_sum(const int32_t *__restrict__ fptr,
                                                       const int32_t *__restrict__ wperm,
                                                       const float *__restrict__ z,
                                                       const int32_t *__restrict__ gmap,
                                                       float *__restrict__ g, double *__restrict__ part,
                                                       int nf, Gate gate)
{
    if (gated_off(gate)) return;   // uniform over the grid
    const int lane = threadIdx.x & (kFasLanes - 1);
    const int f = xcd_item() * kFasPerBlock + threadIdx.x / kFasLanes;
    float s = 0.f;
    if (f < nf) {
        const int beg = fptr[f], end = fptr[f + 1];
        for (int j = beg + lane; j < end; j += 4 * kFasLanes) {
            const int j1 = j + kFasLanes, j2 = j + 2 * kFasLanes, j3 = j + 3 * kFasLanes;
            const int i0 = wperm[j];
            const int i1 = wperm[j1 < end ? j1 : j];
            const int i2 = wperm[j2 < end ? j2 : j];
            const int i3 = wperm[j3 < end ? j3 : j];
            const float z0 = z[i0];
            const float z1 = j1 < end ? z[i1] : 0.f;
            const float z2 = j2 < end ? z[i2] : 0.f;
            const float z3 = j3 < end ? z[i3] : 0.f;
            s += (z0 + z1) + (z2 + z3);
        }
    }
#pragma unroll
    for (int o = kFasLanes / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kFasLanes);
    double sq = 0.0;
    if (f < nf && lane == 0) {
        g[gmap ? gmap[f] : f] = s;
        sq = (double)s * (double)s;
    }
    if (part) block_sum_store<kSumBlock>(sq, part, blockIdx.x);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------------------- dictionary gradient

constexpr int kPsiStride = life::kPsiStride;

// dD = d<ybar, M(D) w>/dD:  dD[:, a] = sum over nonzeros c with atom_c = a of
// (phi_c w[f_c]) * ybar[:, voxel_c].  Per (chunk, atom tile) the nonzeros are
// first merged into a dense block Psi[a][slot] = sum of phi_c w[f_c] over the
// nonzeros of (voxel of slot, a) (LDS, fixed-order segmented sums); then
// dD_tile += Ybar_chunk * Psi^T is a dense product over the chunk's 64 voxel slots
// on the matrix cores (v_mfma_f32_16x16x4_f32, FP32 in, FP32 accumulate), with
// Ybar_chunk staged in LDS as [theta][slot].
// One workgroup owns one span of S consecutive atom tiles of the plan (a "dd
// tile" of up to S TA atoms: fewer, larger blocks than the DSC tiles, so the
// chunk's Ybar staging and the block's zeroing are shared by S tiles) and one
// contiguous group of chunks; it keeps its share of dD in the accumulators and
// writes it once to part (layout [dd tile][group][atom of dd tile][theta, padded
// to 16]); k_dd_reduce sums the groups.
//   MFMA operands (16 x 16 x 4 per instruction, 16 steps per chunk): lane l has
//   row = l % 16, kq = l / 16; at step s the reduction index kq stands for voxel
//   slot 16 kq + s, so the 16 steps cover the 64 slots once:
//     A[row][kq] = Ybar[16 i + row][16 kq + s]   (theta block i)
//     B[kq][row] = Psi[16 m + row][16 kq + s]    (atom block m)
//   and the accumulator element r of lane l is (theta 16 i + 4 kq + r, atom 16 m + row).
template <int NBW>
__global__ __launch_bounds__(kWG) void k_dd_chunk(const int32_t *__restrict__ chunk_vox,
                                                  const int32_t *__restrict__ wave_work,
                                                  const int16_t *__restrict__ atom,
                                                  const int32_t *__restrict__ fas,
                                                  const float *__restrict__ phi,
                                                  const float *__restrict__ w,
                                                  const float *__restrict__ ybar,
                                                  float *__restrict__ part, int nth, int T, int TA, int TAP,
                                                  int S, int n_chunks, int G)
{
    extern __shared__ float4 lds4[];
    float *psi = reinterpret_cast<float *>(lds4);
    const int NTB = (nth + 15) / 16, NT16 = 16 * NTB;
    float *ylds = psi + TAP * kPsiStride;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int item = xcd_item();
    const int DT = (T + S - 1) / S;
    const int u = item % DT, grp = item / DT;
    const int c0 = (int)((int64_t)grp * n_chunks / G), c1 = (int)((int64_t)(grp + 1) * n_chunks / G);
    const int a0 = u * S * TA, t_end = min(T, (u + 1) * S);
    const int MB = TAP / 16, NB = NTB * MB;
    const int b_lo = wave * NB / kChunkWaves, b_hi = (wave + 1) * NB / kChunkWaves;   // this wave's blocks
    const int row = lane & 15, kq = lane >> 4;
    f32x4 acc[NBW];
#pragma unroll
    for (int k = 0; k < NBW; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int n4 = TAP * kPsiStride / 4;

    for (int c = c0; c < c1; ++c) {
        __syncthreads();                          // the previous chunk's products are done with the LDS
        for (int i = threadIdx.x; i < n4; i += kWG) lds4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        // the chunk's ybar block (at most 64 x 128 values: 8 per thread, 4 in flight)
        for (int i0 = threadIdx.x; i0 < kChunkVoxels * NT16; i0 += 4 * kWG) {
            int vv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int i = i0 + k * kWG;
                vv[k] = i < kChunkVoxels * NT16 ? chunk_vox[(size_t)c * kChunkVoxels + i / NT16] : -1;
            }
            float yv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int th = (i0 + k * kWG) % NT16;
                yv[k] = (vv[k] >= 0 && th < nth) ? ybar[(size_t)vv[k] * nth + th] : 0.f;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int i = i0 + k * kWG, slot = i / NT16, th = i - slot * NT16;
                if (i < kChunkVoxels * NT16) ylds[th * kPsiStride + slot] = yv[k];
            }
        }
        __syncthreads();
        // Psi of this chunk and dd tile: one nonzero per lane, four batches of 64 in
        // flight over the wave's whole range (its 4 slots in turn); atoms never
        // decrease inside a slot's sub-range, so runs of equal (slot, atom) are summed
        // by a segmented scan
        for (int t = u * S; t < t_end; ++t) {
            const WaveRange R(wave_work, c, t, T, wave);
            const int p1 = R.p[1], p2 = R.p[2], p3 = R.p[3], pe = R.p[kWaveVoxels];
            for (int b = R.p[0]; b < pe; b += 4 * 64) {
                int aa[4], ff[4];
                float ph[4], sv[4];
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const int idx = b + 64 * h + lane;
                    const int ix = idx < pe ? idx : R.p[0];
                    aa[h] = atom[ix];
                    ff[h] = fas[ix];
                    ph[h] = phi[ix];
                }
#pragma unroll
                for (int h = 0; h < 4; ++h) sv[h] = ph[h] * w[ff[h]];
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const int idx = b + 64 * h + lane;
                    if (b + 64 * h < pe) {   // uniform
                        const bool valid = idx < pe;
                        const int j = (idx >= p1) + (idx >= p2) + (idx >= p3);
                        const int key = valid ? (j << 16) | aa[h] : -1;
                        float v = valid ? sv[h] : 0.f;
                        // a run of equal keys starts where the previous lane's key differs
                        // (wave_shr:1; lane 0 keeps -2, no key); segmented scan on DPP
                        const int kp = __builtin_amdgcn_update_dpp(-2, key, 0x138, 0xf, 0xf, false);
                        int f = kp != key ? 1 : 0;
                        seg_scan_step<0x111, 0xf>(v, f);
                        seg_scan_step<0x112, 0xf>(v, f);
                        seg_scan_step<0x114, 0xf>(v, f);
                        seg_scan_step<0x118, 0xf>(v, f);
                        seg_scan_step<0x142, 0xa>(v, f);
                        seg_scan_step<0x143, 0xc>(v, f);
                        // the run's last lane adds it (wave_shl:1; lane 63 keeps -2)
                        const int kn = __builtin_amdgcn_update_dpp(-2, key, 0x130, 0xf, 0xf, false);
                        if (valid && kn != key) psi[(aa[h] - a0) * kPsiStride + wave * kWaveVoxels + j] += v;
                    }
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NBW; ++k) {
            const int bb = b_lo + k;
            if (bb < b_hi) {
                const int i = bb / MB, mb = bb - i * MB;
                const float4 *ap = reinterpret_cast<const float4 *>(ylds + (16 * i + row) * kPsiStride + 16 * kq);
                const float4 *bp = reinterpret_cast<const float4 *>(psi + (16 * mb + row) * kPsiStride + 16 * kq);
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const float4 A = ap[h], B = bp[h];
                    acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.x, B.x, acc[k], 0, 0, 0);
                    acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.y, B.y, acc[k], 0, 0, 0);
                    acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.z, B.z, acc[k], 0, 0, 0);
                    acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.w, B.w, acc[k], 0, 0, 0);
                }
            }
        }
    }
    float *out = part + (size_t)(u * G + grp) * TAP * NT16;
#pragma unroll
    for (int k = 0; k < NBW; ++k) {
        const int bb = b_lo + k;
        if (bb < b_hi) {
            const int i = bb / MB, mb = bb - i * MB;
#pragma unroll
            for (int r = 0; r < 4; ++r) out[(size_t)(16 * mb + row) * NT16 + 16 * i + 4 * kq + r] = acc[k][r];
        }
    }
}

// dD[theta + nth a] = sum over groups g (fixed order) of the partial of a's tile.
__global__ __launch_bounds__(kBlock) void k_dd_reduce(const float *__restrict__ part, float *__restrict__ dD,
                                                       int nth, int na, int TA, int TAP, int G)
{
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (int64_t)na * nth) return;
    const int a = (int)(idx / nth), th = (int)(idx - (int64_t)a * nth);
    const int t = a / TA, al = a - t * TA;
    const int NT16 = ((nth + 15) / 16) * 16;
    const float *p = part + ((size_t)t * G * TAP + al) * NT16 + th;
    const size_t stride = (size_t)TAP * NT16;
    float s = 0.f;
    for (int g = 0; g < G; ++g) s += p[g * stride];
    dD[idx] = s;
}

// Generic dictionary gradient (any N_theta): one block per atom over the atom's
// nonzeros (atom-major copy), 8 segments of 32 lanes, NT theta slots per lane,
// fixed-order combination of the segments.
template <int NT>
__global__ __launch_bounds__(kBlock) void k_dd_atom(const int32_t *__restrict__ aptr,
                                                     const int32_t *__restrict__ avox,
                                                     const int32_t *__restrict__ afas,
                                                     const float *__restrict__ aphi,
                                                     const float *__restrict__ w,
                                                     const float *__restrict__ ybar, float *__restrict__ dD,
                                                     int nth, int na)
{
    __shared__ float sh[kBlock / kSeg][kSeg * NT];
    const int a = blockIdx.x;
    const int lane = threadIdx.x & (kSeg - 1), seg = threadIdx.x / kSeg;
    float acc[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) acc[i] = 0.f;
    const int beg = aptr[a], end = aptr[a + 1];
    for (int e = beg + seg; e < end; e += kBlock / kSeg) {
        const float sv = aphi[e] * w[afas[e]];
        const float *yv = ybar + (size_t)avox[e] * nth;
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            const int th = lane + kSeg * i;
            if (th < nth) acc[i] = fmaf(sv, yv[th], acc[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < NT; ++i) sh[seg][lane + kSeg * i] = acc[i];
    __syncthreads();
    for (int th = threadIdx.x; th < nth; th += kBlock) {
        float sum = 0.f;
        for (int k = 0; k < kBlock / kSeg; ++k) sum += sh[k][th];
        dD[(size_t)a * nth + th] = sum;
    }
}

// ----------------------------------------------------------------------------- SBB glue

// g~_f = g_f unless w_f = 0 and g_f > 0 (the bound is active); partial ||g~||^2.
__global__ __launch_bounds__(kBlock) void k_mask(const float *__restrict__ w, const float *__restrict__ g,
                                                  float *__restrict__ gt, double *__restrict__ part, int nf)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double sq = 0.0;
    if (i < nf) {
        const float gi = g[i];
        const float v = (w[i] > 0.f || gi < 0.f) ? gi : 0.f;
        gt[i] = v;
        sq = (double)v * (double)v;
    }
    block_sum_store<kBlock>(sq, part, blockIdx.x);
}

// alpha from the partial sums; records the state; i += 1.
//   Algorithm 1 (lagged = 0): odd i  alpha = <g~,g~> / <Mg~,Mg~>
//                             even i alpha = <Mg~,Mg~> / <M^T M g~, M^T M g~>
//   eqs. 7-8 (lagged = 1), q = g~ of the previous iterate (the current one at i = 0):
//                             even i alpha = <q,q> / <Mq,Mq>
//                             odd i  alpha = <Mq,Mq> / <M^T M q, M^T M q>
// p_vp / p_vpp hold the partial squared norms of M q and M^T M q (q = g~ in
// Algorithm 1); p_q those of q (NULL: q = g~).
__global__ __launch_bounds__(kAlphaThreads) void k_alpha(const double *__restrict__ p_r, int n_r,
                                                          const double *__restrict__ p_gt, int n_gt,
                                                          const double *__restrict__ p_q, int n_q,
                                                          const double *__restrict__ p_vp, int n_vp,
                                                          const double *__restrict__ p_vpp, int n_vpp,
                                                          life_sbb_state *__restrict__ st, int lagged)
{
    const int64_t it = st->iter;
    const bool odd = (it & 1) != 0;
    const bool first_form = lagged ? !odd : odd;      // <q,q> / <Mq,Mq>
    const double r2 = block_sum_array(p_r, n_r);
    const double gt2 = block_sum_array(p_gt, n_gt);
    const double q2 = p_q ? block_sum_array(p_q, n_q) : gt2;
    const double vp2 = block_sum_array(p_vp, n_vp);
    const double vpp2 = first_form ? 0.0 : block_sum_array(p_vpp, n_vpp);
    if (threadIdx.x == 0) {
        const double num = first_form ? q2 : vp2;
        const double den = first_form ? vp2 : vpp2;
        st->alpha = den > 0.0 ? num / den : 0.0;
        st->obj = 0.5 * r2;
        st->gt_norm2 = gt2;
        st->num = num;
        st->den = den;
        st->iter = it + 1;
    }
}

// q for the lagged step: q[r] = g~ of the previous iterate (caller order, in
// gt_prev) or, at i = 0, the current g~; partial ||q||^2.
__global__ __launch_bounds__(kBlock) void k_lag_q(const float *__restrict__ gt_prev, const int32_t *__restrict__ ext,
                                                   const float *__restrict__ gt, float *__restrict__ q,
                                                   double *__restrict__ part, const life_sbb_state *__restrict__ st,
                                                   int nf)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const bool first = st->iter == 0;
    double sq = 0.0;
    if (i < nf) {
        const float v = first ? gt[i] : gt_prev[ext[i]];
        q[i] = v;
        sq = (double)v * (double)v;
    }
    block_sum_store<kBlock>(sq, part, blockIdx.x);
}

// Batched plans: the SBB scalars of every instance (one block per instance, all
// instances at the same iteration; Algorithm 1).  y-space sums come from the
// per-chunk partials of the instance's chunks, w-space sums are taken from the
// vectors over the instance's rank range; every sum has a fixed order.
__device__ double block_sum_range(const double *a, int lo, int hi)
{
    __shared__ double sh[kAlphaThreads];
    double s = 0.0;
    for (int i = lo + threadIdx.x; i < hi; i += kAlphaThreads) s += a[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kAlphaThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ double block_sumsq_range(const float *x, int lo, int hi)
{
    __shared__ double sh[kAlphaThreads];
    double s = 0.0;
    for (int i = lo + threadIdx.x; i < hi; i += kAlphaThreads) s += (double)x[i] * (double)x[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kAlphaThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kAlphaThreads) void k_alpha_batch(const double *__restrict__ p_r,
                                                                const double *__restrict__ p_vp,
                                                                const int32_t *__restrict__ inst_chunk,
                                                                const float *__restrict__ gt,
                                                                const float *__restrict__ vpp,
                                                                const int32_t *__restrict__ inst_rank,
                                                                life_sbb_state *__restrict__ states)
{
    const int k = blockIdx.x;
    life_sbb_state *st = states + k;
    const int64_t it = st->iter;
    const bool odd = (it & 1) != 0;
    const int c0 = inst_chunk[k], c1 = inst_chunk[k + 1], r0 = inst_rank[k], r1 = inst_rank[k + 1];
    const double r2 = block_sum_range(p_r, c0, c1);
    const double vp2 = block_sum_range(p_vp, c0, c1);
    const double gt2 = block_sumsq_range(gt, r0, r1);
    const double vpp2 = odd ? 0.0 : block_sumsq_range(vpp, r0, r1);
    if (threadIdx.x == 0) {
        const double num = odd ? gt2 : vp2;
        const double den = odd ? vp2 : vpp2;
        st->alpha = den > 0.0 ? num / den : 0.0;
        st->obj = 0.5 * r2;
        st->gt_norm2 = gt2;
        st->num = num;
        st->den = den;
        st->iter = it + 1;
    }
}

// w <- [w - alpha_k g~]_+ with the step length of each rank's instance k.
__global__ __launch_bounds__(kBlock) void k_update_batch(float *__restrict__ w_out, const float *__restrict__ w_rank,
                                                          const float *__restrict__ gt,
                                                          const int32_t *__restrict__ ext,
                                                          const life_sbb_state *__restrict__ states,
                                                          const int32_t *__restrict__ inst_rank, int n_inst, int nf)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nf) return;
    int lo = 0, hi = n_inst;               // instance k with inst_rank[k] <= i < inst_rank[k+1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (inst_rank[mid] <= i) lo = mid; else hi = mid;
    }
    const double x = (double)w_rank[i] - states[lo].alpha * (double)gt[i];
    w_out[ext[i]] = x > 0.0 ? (float)x : 0.0f;
}

// w <- [w - alpha g~]_+  (eq. 5), evaluated in double and rounded once.  The
// iterate and g~ are in fascicle-rank order; w_out is in the caller's order.
__global__ __launch_bounds__(kBlock) void k_update(float *__restrict__ w_out, const float *__restrict__ w_rank,
                                                    const float *__restrict__ gt, const int32_t *__restrict__ ext,
                                                    const life_sbb_state *__restrict__ st, float *__restrict__ gt_out,
                                                    int nf)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= nf) return;
    const double x = (double)w_rank[i] - st->alpha * (double)gt[i];
    w_out[ext[i]] = x > 0.0 ? (float)x : 0.0f;
    if (gt_out) gt_out[ext[i]] = gt[i];
}

// w_rank[r] = w[ext[r]]: weights into fascicle-rank order.
__global__ __launch_bounds__(kBlock) void k_gather(const float *__restrict__ w, const int32_t *__restrict__ ext,
                                                    float *__restrict__ w_rank, int nf)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < nf) w_rank[i] = w[ext[i]];
}

int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// rec[i] = (key, bits of phi): the WC pass-1 bucket stream in one record
__global__ __launch_bounds__(kBlock) void k_pack_wc(const uint16_t *__restrict__ key, const float *__restrict__ phi,
                                                     int64_t n, uint2 *__restrict__ rec)
{
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i < n) rec[i] = make_uint2((uint32_t)key[i], __float_as_uint(phi[i]));
}

// rec[i] = (atom | local index << 16, bits of phi): the chunked DSC stream in one record
__global__ __launch_bounds__(kBlock) void k_pack_dsc(const int16_t *__restrict__ atom, const uint16_t *__restrict__ loc,
                                                      const float *__restrict__ phi, int64_t n, uint2 *__restrict__ rec)
{
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i < n) rec[i] = make_uint2((uint32_t)(uint16_t)atom[i] | (uint32_t)loc[i] << 16, __float_as_uint(phi[i]));
}

}  // namespace

// ============================================================================= plan object

// Everything the enqueue calls write besides their outputs.  One contiguous block
// (life_plan_scratch_bytes) carved into regions of 256-byte aligned arrays; the
// plan owns one, and the *_ws calls take the caller's, so that one plan can serve
// several streams at once.
struct Workspace {
    float *w_rank = nullptr;      // [Nf] weights (or g~) in fascicle-rank order
    i32x4 *dt_frag = nullptr;     // [n_tiles][dt_ab][dt_ks][kDigits][64] digits of D^T, the A operands of WC pass 1
    float *dt_scale = nullptr;    // [n_tiles][dt_ab][32]
    float *z = nullptr;           // WC pass-1 values: one per run (chunked plans) or per nonzero
    float *r = nullptr, *vp = nullptr;                                // [Nt*Nv] SBB residual, M q
    float *g = nullptr, *gt = nullptr, *vpp = nullptr, *q = nullptr;  // [Nf] SBB vectors
    double *part = nullptr;       // 5 regions of part_stride partial sums
    float *dd_part = nullptr;     // dictionary-gradient partials
};

// Regions of the workspace a call needs.
enum : unsigned { kWsDsc = 1u, kWsWc = 2u, kWsSbb = 4u, kWsDd = 8u, kWsAll = 15u };

struct life_plan_s {
    life_dims dims{};
    int device = 0;
    int slots = 1;                // generic kernels: theta slots per lane
    life::TileGeom tile;          // chunked kernels: LDS tiling (row_floats = 0: not used)
    int n_chunks = 0;
    // DSC order (voxel, atom, fascicle, input position)
    int32_t *vox_ptr = nullptr;   // [Nv + 1]
    int16_t *atom_v = nullptr;    // [nnz]
    int32_t *fas_v = nullptr;     // [nnz]
    float *phi_v = nullptr;       // [nnz]
    // chunked layout (see life::chunk_layout): padded copies of the DSC-order arrays
    int64_t n_pad = 0;
    int32_t *chunk_vox = nullptr; // [n_chunks * kChunkVoxels]
    int32_t *chunk_map = nullptr; // [chunk_grid] chunk of each workgroup of the chunk kernels, -1 = none
    int chunk_grid = 0;
    int schedule = life::kScheduleDefault;
    std::vector<int64_t> chunk_work;   // host: padded entries per chunk (for re-scheduling)
    int32_t *wave_work = nullptr; // [n_chunks * n_tiles * kChunkWaves * kWorkInts]
    int16_t *atom_c = nullptr;    // [n_pad]
    int32_t *fas_c = nullptr;     // [n_pad] fascicle rank
    uint16_t *loc_c = nullptr;    // [n_pad] place of the fascicle in its chunk's list
    float *phi_c = nullptr;       // [n_pad]
    uint2 *dsc_rec = nullptr;     // [n_pad] the DSC stream packed: (atom | local index << 16, phi)
    int32_t *cfas_ptr = nullptr;  // [n_chunks + 1] chunk fascicle lists (see life::ChunkLayout)
    int32_t *cfas = nullptr;
    int max_fas = 0;              // longest chunk fascicle list
    size_t dsc_lds = 0;
    // WC pass 1 buckets (see life::ChunkLayout) and pass 2 run lists
    uint16_t *wkey = nullptr;     // [nnz]
    float *wphi = nullptr;        // [nnz]
    uint2 *wc_rec = nullptr;      // [nnz] (wkey, bits of wphi): WC pass 1 reads one record per entry
    int32_t *wc_wave = nullptr;   // [n_chunks * n_tiles * kChunkWaves + 1]
    int32_t *wc_wrun = nullptr;   // [n_chunks * n_tiles * kChunkWaves]
    int64_t n_runs = 0;
    int32_t *rr_ptr = nullptr;    // [Nf + 1]
    int32_t *rr = nullptr;        // [n_runs]
    // WC pass 1 on the matrix cores: split D^T operands (k_split_dt) and the LDS size
    int dt_ab = 0, dt_ks = 0;     // atom blocks of 32 per tile, k-steps of 32 theta
    size_t wcr_lds = 0;
    // fascicles are processed in rank order (fas_v holds ranks)
    int32_t *fas_rank = nullptr;  // [Nf] rank of each fascicle
    int32_t *fas_ext = nullptr;   // [Nf] fascicle of each rank
    // WC order (rank, voxel, atom, input position) as DSC positions
    int32_t *fas_ptr = nullptr;   // [Nf + 1]
    int32_t *wc_perm = nullptr;   // [nnz]
    // the plan's own workspace (calls given no caller scratch use it)
    Workspace ws;
    void *ws_base = nullptr;
    int64_t part_stride = 0;      // doubles per partial-sum region of the workspace
    // dictionary gradient: chunked (per tile and chunk group partials) ...
    int dd_groups = 0, dd_tap = 0, dd_nbw = 0, dd_span = 1;   // dd tile = dd_span plan tiles
    int64_t dd_floats = 0;        // [T][groups][dd_tap][16 ceil(Nt/16)] partials in the workspace
    // ... or generic (atom-major copy of the nonzeros)
    int32_t *a_ptr = nullptr;     // [Na + 1]
    int32_t *a_vox = nullptr, *a_fas = nullptr;   // [nnz] voxel, fascicle rank
    float *a_phi = nullptr;       // [nnz]
    // instances of a batched plan (one for other plans): chunk and rank ranges
    int n_inst = 1;
    int32_t *inst_chunk = nullptr; // [n_inst + 1] first chunk of each instance
    int32_t *inst_rank = nullptr;  // [n_inst + 1] first fascicle rank (= fascicle) of each instance
    // profiling
    bool profile = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> events;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

template <class T>
hipError_t dalloc(T **p, int64_t n)
{
    *p = nullptr;
    if (n <= 0) return hipSuccess;
    return hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * (size_t)n);
}

void free_plan(life_plan_s *p)
{
    void *ptrs[] = {p->vox_ptr, p->atom_v, p->fas_v, p->phi_v, p->chunk_vox, p->chunk_map, p->wave_work, p->atom_c,
                    p->dsc_rec,
                    p->fas_c, p->loc_c, p->phi_c, p->cfas_ptr, p->cfas, p->wkey, p->wphi, p->wc_wave, p->wc_wrun,
                    p->wc_rec,
                    p->rr_ptr, p->rr, p->fas_rank, p->fas_ext, p->fas_ptr,
                    p->wc_perm, p->ws_base, p->a_ptr, p->a_vox, p->a_fas, p->a_phi, p->inst_chunk, p->inst_rank};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    for (auto &e : p->events) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    delete p;
}

// Carve the regions a call needs (mask of kWs*) out of base (NULL: sizes only);
// returns the bytes they take.  Every region starts on a 256-byte boundary.
size_t workspace_layout(const life_plan_s *p, unsigned need, char *base, Workspace *ws)
{
    const life_dims &d = p->dims;
    const int64_t nf = d.n_fascicles, nsig = (int64_t)d.n_theta * d.n_voxels;
    size_t off = 0;
    auto take = [&](auto **ptr, int64_t n, size_t elem) {
        off = (off + 255) / 256 * 256;
        using T = std::remove_reference_t<decltype(**ptr)>;
        *ptr = (base && n > 0) ? reinterpret_cast<T *>(base + off) : nullptr;
        off += (size_t)std::max<int64_t>(n, 0) * elem;
    };
    Workspace w;
    if (need & (kWsDsc | kWsSbb | kWsDd)) take(&w.w_rank, nf, sizeof(float));
    if (need & (kWsWc | kWsSbb)) {
        if (p->n_chunks > 0) {
            take(&w.dt_frag, (int64_t)p->tile.n_tiles * p->dt_ab * p->dt_ks * kDigits * 64, sizeof(i32x4));
            take(&w.dt_scale, (int64_t)p->tile.n_tiles * p->dt_ab * 32, sizeof(float));
        }
        take(&w.z, p->n_chunks > 0 ? p->n_runs : d.nnz, sizeof(float));
    }
    if (need & kWsSbb) {
        take(&w.r, nsig, sizeof(float));
        take(&w.vp, nsig, sizeof(float));
        take(&w.g, nf, sizeof(float));
        take(&w.gt, nf, sizeof(float));
        take(&w.vpp, nf, sizeof(float));
        take(&w.q, nf, sizeof(float));
        take(&w.part, 5 * p->part_stride, sizeof(double));
    }
    if (need & kWsDd) take(&w.dd_part, p->dd_floats, sizeof(float));
    if (ws) *ws = w;
    return (off + 255) / 256 * 256;
}

int slots_for(int nth)
{
    const int need = (nth + kSeg - 1) / kSeg;
    static const int variants[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
    for (int v : variants)
        if (v >= need) return v;
    return 32;
}

// The last HIP runtime error a call of this thread ran into (life_hip_error).
thread_local const char *t_hip_error = "";
void note_hip_error(hipError_t e) { t_hip_error = hipGetErrorString(e); }

// Set while a call that must not create events enqueues its launches.
thread_local bool t_no_events = false;
struct NoEvents {
    bool prev;
    NoEvents() : prev(t_no_events) { t_no_events = true; }
    ~NoEvents() { t_no_events = prev; }
};

// Launch with optional event bracketing; returns the launch status.
template <class F>
life_status launch(life_plan_s *p, int kind, hipStream_t s, F &&f)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool prof = p->profile && !t_no_events;
    if (prof) {
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LIFE_EDEVICE;
        if (hipEventRecord(e0, s) != hipSuccess) return LIFE_EDEVICE;
    }
    f();
    const hipError_t err = hipGetLastError();
    if (prof) {
        if (hipEventRecord(e1, s) != hipSuccess) return LIFE_EDEVICE;
        p->events.push_back({kind, {e0, e1}});
    }
    if (err != hipSuccess) note_hip_error(err);
    return err == hipSuccess ? LIFE_OK : LIFE_EDEVICE;
}

#define LIFE_DISPATCH_SLOTS(SLOTS, KERNEL, ...)                                      \
    switch (SLOTS) {                                                                 \
    case 1: KERNEL<1><<<__VA_ARGS__; break;                                          \
    case 2: KERNEL<2><<<__VA_ARGS__; break;                                          \
    case 3: KERNEL<3><<<__VA_ARGS__; break;                                          \
    case 4: KERNEL<4><<<__VA_ARGS__; break;                                          \
    case 6: KERNEL<6><<<__VA_ARGS__; break;                                          \
    case 8: KERNEL<8><<<__VA_ARGS__; break;                                          \
    case 12: KERNEL<12><<<__VA_ARGS__; break;                                        \
    case 16: KERNEL<16><<<__VA_ARGS__; break;                                        \
    case 24: KERNEL<24><<<__VA_ARGS__; break;                                        \
    default: KERNEL<32><<<__VA_ARGS__; break;                                        \
    }

// accumulator blocks per wave of the dictionary-gradient kernel (at most 10 for
// the tile geometries of N_theta <= 128: e.g. 6 theta blocks x 26 atom blocks
// over 16 waves)
int dd_nbw_variant(int need)
{
    static const int variants[] = {1, 2, 3, 5, 9, 12};
    for (int v : variants)
        if (v >= need) return v;
    return -1;
}

#define LIFE_DISPATCH_NBW(NBWV, KERNEL, ...)                                         \
    switch (NBWV) {                                                                  \
    case 1: KERNEL<1><<<__VA_ARGS__; break;                                          \
    case 2: KERNEL<2><<<__VA_ARGS__; break;                                          \
    case 3: KERNEL<3><<<__VA_ARGS__; break;                                          \
    case 5: KERNEL<5><<<__VA_ARGS__; break;                                          \
    case 9: KERNEL<9><<<__VA_ARGS__; break;                                          \
    default: KERNEL<12><<<__VA_ARGS__; break;                                        \
    }

#define LIFE_DISPATCH_NC(NCV, KERNEL, ...)                                           \
    switch (NCV) {                                                                   \
    case 1: KERNEL<1><<<__VA_ARGS__; break;                                          \
    case 2: KERNEL<2><<<__VA_ARGS__; break;                                          \
    case 3: KERNEL<3><<<__VA_ARGS__; break;                                          \
    default: KERNEL<4><<<__VA_ARGS__; break;                                         \
    }

bool chunked(const life_plan_s *p) { return p->tile.row_floats > 0 && p->n_chunks > 0; }

bool vec_tile(const life_plan_s *p, const float *D)
{
    return p->tile.row_floats == p->dims.n_theta && (reinterpret_cast<uintptr_t>(D) & 15) == 0;
}

size_t tile_lds_bytes(const life_plan_s *p) { return (size_t)p->tile.tile_atoms * p->tile.row_floats * sizeof(float); }

// The chunked kernels may use up to the full LDS budget; set once per process so
// that plans with different tilings never lower each other's limit.
hipError_t allow_lds()
{
    const int bytes = life::kLdsBudget;
    const void *fns[] = {(const void *)k_dsc_chunk<1>, (const void *)k_dsc_chunk<2>, (const void *)k_dsc_chunk<3>,
                         (const void *)k_dsc_chunk<4>, (const void *)k_wcr_mfma<1>, (const void *)k_wcr_mfma<2>,
                         (const void *)k_wcr_mfma<3>, (const void *)k_wcr_mfma<4>, (const void *)k_dd_chunk<1>,
                         (const void *)k_dd_chunk<2>, (const void *)k_dd_chunk<3>, (const void *)k_dd_chunk<5>,
                         (const void *)k_dd_chunk<9>, (const void *)k_dd_chunk<12>};
    for (const void *f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int dsc_partials(const life_plan_s *p)
{
    return chunked(p) ? p->n_chunks : cdiv(p->dims.n_voxels, kSegPerBlock);
}

life_status enqueue_dsc(life_plan_s *p, const float *D, const float *w, const float *bsub, float *y,
                        double *part, hipStream_t s)
{
    const int nv = p->dims.n_voxels, nth = p->dims.n_theta;
    if (nv == 0) return LIFE_OK;
    if (chunked(p)) {
        const int nc = p->tile.row_floats / 32;
        return launch(p, LIFE_K_DSC, s, [&] {
            LIFE_DISPATCH_NC(nc, k_dsc_chunk, p->chunk_grid, kWG, p->dsc_lds, s>>>(p->chunk_map, p->chunk_vox,
                                                                                  p->wave_work, p->dsc_rec,
                                                                                  p->cfas_ptr, p->cfas, w, D,
                                                                                  bsub, y, part, nth,
                                                                                  p->dims.n_atoms, p->tile.n_tiles,
                                                                                  p->tile.tile_atoms, vec_tile(p, D)))
        });
    }
    const int grid = cdiv(nv, kSegPerBlock);
    return launch(p, LIFE_K_DSC, s, [&] {
        LIFE_DISPATCH_SLOTS(p->slots, k_dsc, grid, kBlock, 0, s>>>(p->vox_ptr, p->atom_v, p->fas_v, p->phi_v, w, D,
                                                                   bsub, y, part, nth, nv))
    });
}

life_status enqueue_wc(life_plan_s *p, const Workspace &ws, const float *D, const float *y, float *g,
                       const int32_t *gmap, double *part, Gate gate, hipStream_t s, bool split_d = true)
{
    const int nv = p->dims.n_voxels, nf = p->dims.n_fascicles, nth = p->dims.n_theta;
    life_status st = LIFE_OK;
    if (nv > 0 && p->dims.nnz > 0) {
        const int kind = gate.st ? LIFE_K_WC_Z_2ND : LIFE_K_WC_Z;
        if (chunked(p)) {
            // split_d = false: D was split by an earlier call of the same enqueue sequence
            const int T = p->tile.n_tiles, AB = p->dt_ab, KS = p->dt_ks, TA = p->tile.tile_atoms;
            st = launch(p, kind, s, [&] {
                if (split_d)
                    k_split_dt<<<cdiv((int64_t)T * AB * 32, kBlock / 64), kBlock, 0, s>>>(D, ws.dt_frag, ws.dt_scale,
                                                                                         nth, p->dims.n_atoms, T, TA,
                                                                                         AB, KS, gate);
#define LIFE_WCR(K)                                                                                        \
    k_wcr_mfma<K><<<p->chunk_grid, kWG, p->wcr_lds, s>>>(p->chunk_map, p->chunk_vox, p->wc_rec, p->wc_wave,     \
                                                         p->wc_wrun, ws.dt_frag, ws.dt_scale, y, ws.z, nth, T, AB, gate)
                // the k-steps as a compile-time count: the A digits of the next k-step
                // can then be requested while the matrix cores work on this one
                switch (KS) {   // N_theta <= 128
                case 1: LIFE_WCR(1); break;
                case 2: LIFE_WCR(2); break;
                case 3: LIFE_WCR(3); break;
                default: LIFE_WCR(4); break;
                }
#undef LIFE_WCR
            });
        } else {
            const int grid = cdiv(nv, kSegPerBlock);
            st = launch(p, kind, s, [&] {
                LIFE_DISPATCH_SLOTS(p->slots, k_wc_z, grid, kBlock, 0, s>>>(p->vox_ptr, p->atom_v, p->phi_v, D, y,
                                                                            ws.z, nth, nv, gate))
            });
        }
        if (st != LIFE_OK) return st;
    }
    if (nf > 0) {
        const int grid = cdiv(nf, kFasPerBlock);
        st = launch(p, gate.st ? LIFE_K_WC_SUM_2ND : LIFE_K_WC_SUM, s, [&] {
            k_wc_sum<<<grid, kSumBlock, 0, s>>>(chunked(p) ? p->rr_ptr : p->fas_ptr,
                                                chunked(p) ? p->rr : p->wc_perm, ws.z, gmap, g, part, nf, gate);
        });
    }
    return st;
}

life_status enqueue_gather(life_plan_s *p, const Workspace &ws, const float *w, hipStream_t s)
{
    const int nf = p->dims.n_fascicles;
    if (nf == 0) return LIFE_OK;
    return launch(p, LIFE_K_PERMUTE, s, [&] {
        k_gather<<<cdiv(nf, kBlock), kBlock, 0, s>>>(w, p->fas_ext, ws.w_rank, nf);
    });
}

// dD from w_rank (weights already in rank order) and ybar.
life_status enqueue_dd(life_plan_s *p, const Workspace &ws, const float *ybar, float *dD, hipStream_t s)
{
    const life_dims &d = p->dims;
    const int nth = d.n_theta, na = d.n_atoms;
    if (chunked(p)) {
        const int T = p->tile.n_tiles, TA = p->tile.tile_atoms, TAP = p->dd_tap, G = p->dd_groups;
        const int S = p->dd_span, DT = (T + S - 1) / S;
        const size_t lds = (size_t)(TAP + (nth + 15) / 16 * 16) * kPsiStride * sizeof(float);
        life_status st = launch(p, LIFE_K_DD, s, [&] {
            LIFE_DISPATCH_NBW(p->dd_nbw, k_dd_chunk, DT * G, kWG, lds, s>>>(p->chunk_vox, p->wave_work, p->atom_c,
                                                                          p->fas_c, p->phi_c, ws.w_rank, ybar,
                                                                          ws.dd_part, nth, T, TA, TAP, S,
                                                                          p->n_chunks, G))
        });
        if (st != LIFE_OK) return st;
        // a dd tile holds S TA atoms
        return launch(p, LIFE_K_DD_REDUCE, s, [&] {
            k_dd_reduce<<<cdiv((int64_t)na * nth, kBlock), kBlock, 0, s>>>(ws.dd_part, dD, nth, na, S * TA, TAP, G);
        });
    }
    return launch(p, LIFE_K_DD, s, [&] {
        LIFE_DISPATCH_SLOTS(p->slots, k_dd_atom, na, kBlock, 0, s>>>(p->a_ptr, p->a_vox, p->a_fas, p->a_phi,
                                                                     ws.w_rank, ybar, dD, nth, na))
    });
}

}  // namespace

// ============================================================================= C ABI

extern "C" life_status life_plan(const life_dims *dims, const int16_t *atom, const int32_t *voxel,
                                 const int32_t *fascicle, const float *phi, life_plan_t *out)
{
    return life_plan_ex(dims, atom, voxel, fascicle, phi, nullptr, out);
}

namespace {

// Whether the chunked kernels' LDS layouts fit a tiling: the WC pass-1 block
// (the P tile of tile_atoms rows plus the chunk's Y digits), the dictionary
// gradient's Psi block for a span of one tile, and the DSC tile beside a
// fascicle list of at least 1024 weights (tile_geometry checks the last).
bool tiling_fits(int n_theta, const life::TileGeom &tg)
{
    if (tg.row_floats == 0) return false;   // tile_geometry found no room for the DSC's fascicle list
    const int ab = (tg.tile_atoms + 31) / 32, ks = (n_theta + 31) / 32;
    const size_t wcr = (size_t)ab * 32 * kPS * sizeof(float) + (size_t)kDigits * kChunkVoxels * (32 * ks + kQ8Pad) +
                       kChunkVoxels * sizeof(float);
    const int64_t dd = (int64_t)((tg.tile_atoms + 15) / 16 * 16 + (n_theta + 15) / 16 * 16) * kPsiStride * 4;
    return ab <= kChunkWaves && wcr <= (size_t)life::kLdsBudget && dd <= life::kLdsBudget;
}

// Plan construction shared by life_plan, life_plan_ex, life_plan_batch and
// life_plan_flags (n_inst <= 1: a single problem).  The restructuring runs on the
// device (life::plan_gpu) unless LIFE_PLAN_HOST_BUILD asks for the host builder,
// the tile geometry is not chunked (N_theta > 128), or a voxel crosses more
// fascicles than a chunk holds; both builders give the same plan bit for bit.
life_status build_plan(const life_dims *dims, const int16_t *atom_in, const int32_t *voxel_in,
                       const int32_t *fascicle_in, const float *phi_in, const int16_t *voxel_xyz, int n_inst,
                       const int32_t *vox_off, const int32_t *fas_off, uint32_t flags, int tile_atoms,
                       life_plan_t *out)
{
    if (!out) return LIFE_EINVAL;
    *out = nullptr;
    life_status st = life::validate_dims(dims);
    if (st != LIFE_OK) return st;
    if ((st = life::validate_coords(dims, voxel_xyz)) != LIFE_OK) return st;
    const life_dims d = *dims;
    if (d.nnz > 0 && (!phi_in || !atom_in || !voxel_in || !fascicle_in)) return LIFE_EINVAL;
    const bool dev_in = (flags & LIFE_PLAN_DEVICE_INPUT) != 0;
    const bool batched = n_inst > 1;
    const int32_t one_v[2] = {0, d.n_voxels}, one_f[2] = {0, d.n_fascicles};
    if (!batched) {
        n_inst = 1;
        vox_off = one_v;
        fas_off = one_f;
    } else {
        if (vox_off[0] != 0 || fas_off[0] != 0 || vox_off[n_inst] != d.n_voxels || fas_off[n_inst] != d.n_fascicles)
            return LIFE_EINVAL;
        for (int k = 0; k < n_inst; ++k)
            if (vox_off[k + 1] < vox_off[k] || fas_off[k + 1] < fas_off[k]) return LIFE_EINVAL;
    }
    if (tile_atoms < 0) return LIFE_EINVAL;
    const life::TileGeom tg = life::tile_geometry(d.n_theta, d.n_atoms, tile_atoms);
    if (batched && tg.row_floats == 0) return LIFE_EINVAL;   // batched plans need N_theta <= 128
    // an explicit tiling the chunked kernels cannot hold (ignored when N_theta > 128)
    if (tile_atoms > 0 && d.n_theta <= life::kMaxTileRowFloats && !tiling_fits(d.n_theta, tg)) return LIFE_EINVAL;
    const int32_t n_pos = life::padded_positions(&d, n_inst, vox_off);
    if (n_pos < 0) return LIFE_ERANGE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        // no device: still report bad host input as such
        if (!dev_in && (st = life::validate_indices(&d, atom_in, voxel_in, fascicle_in)) != LIFE_OK) return st;
        return LIFE_EDEVICE;
    }

    std::vector<int32_t> perm, vptr, wperm, fptr, rank, ext, ppos, pvox, vdsc, fas_inst;
    std::vector<int32_t> aptr, avox, afas, cmap;
    std::vector<float> aphi;
    std::vector<int16_t> atom_v;
    std::vector<int32_t> fas_v;
    std::vector<float> phi_v;
    std::vector<int32_t> ichunk((size_t)n_inst + 1, 0);
    life::ChunkLayout L;
    life::DevLayout G;   // device-built arrays (owned here until the plan takes them)
    struct GFree {
        life::DevLayout *g;
        ~GFree() { life::free_dev_layout(g); }
    } gfree{&G};
    bool on_gpu = false;
    int n_chunks = 0;
    std::vector<int32_t> bounds;
    std::vector<int64_t> work;
    int max_fas = 0;
    int64_t n_pad = 0, n_runs = 0;
    try {
        ppos.resize((size_t)d.n_voxels);
        pvox.resize((size_t)n_pos);
        life::voxel_order(&d, voxel_xyz, n_inst, vox_off, ppos.data(), pvox.data());
        if (batched) {
            // each instance's fascicles take one contiguous block of ranks
            fas_inst.resize((size_t)d.n_fascicles);
            for (int k = 0; k < n_inst; ++k)
                for (int32_t f = fas_off[k]; f < fas_off[k + 1]; ++f) fas_inst[(size_t)f] = k;
        }
        const int32_t *ppos_used = (voxel_xyz || batched) ? ppos.data() : nullptr;
        if (!(flags & LIFE_PLAN_HOST_BUILD) && tg.row_floats > 0) {
            // the COO arrays on the device
            const int16_t *atom = atom_in;
            const int32_t *voxel = voxel_in, *fascicle = fascicle_in;
            const float *phi = phi_in;
            void *stage[4] = {nullptr, nullptr, nullptr, nullptr};
            struct SFree {
                void **s;
                ~SFree() { for (int i = 0; i < 4; ++i) if (s[i]) (void)hipFree(s[i]); }
            } sfree{stage};
            if (!dev_in && d.nnz > 0) {
                const size_t sz[4] = {sizeof(int16_t), sizeof(int32_t), sizeof(int32_t), sizeof(float)};
                const void *src[4] = {atom_in, voxel_in, fascicle_in, phi_in};
                for (int i = 0; i < 4; ++i) {
                    hipError_t e = hipMalloc(&stage[i], sz[i] * (size_t)d.nnz);
                    if (e == hipSuccess) e = hipMemcpy(stage[i], src[i], sz[i] * (size_t)d.nnz, hipMemcpyHostToDevice);
                    if (e != hipSuccess) return e == hipErrorOutOfMemory ? LIFE_ENOMEM : LIFE_EDEVICE;
                }
                atom = static_cast<const int16_t *>(stage[0]);
                voxel = static_cast<const int32_t *>(stage[1]);
                fascicle = static_cast<const int32_t *>(stage[2]);
                phi = static_cast<const float *>(stage[3]);
            }
            st = life::plan_gpu(&d, tg, atom, voxel, fascicle, phi, ppos_used, pvox.data(), n_pos,
                                batched ? fas_inst.data() : nullptr, vox_off, n_inst, &G);
            if (st == LIFE_OK && hipGetLastError() != hipSuccess) st = LIFE_EDEVICE;
            if (st != LIFE_OK) return st;
            if (G.fas_overflow) {
                if (batched) return LIFE_EINVAL;
                life::free_dev_layout(&G);   // the host builder makes the generic plan below
            } else {
                on_gpu = true;
                n_chunks = G.n_chunks;
                bounds = G.bounds;
                work = G.work;
                max_fas = G.max_fas;
                n_pad = G.n_pad;
                n_runs = G.n_runs;
            }
        }
        if (!on_gpu) {
            // host builder: host copies of the COO arrays when they are on the device
            std::vector<int16_t> atom_h;
            std::vector<int32_t> voxel_h, fascicle_h;
            std::vector<float> phi_h;
            const int16_t *atom = atom_in;
            const int32_t *voxel = voxel_in, *fascicle = fascicle_in;
            const float *phi = phi_in;
            if (dev_in && d.nnz > 0) {
                atom_h.resize((size_t)d.nnz);
                voxel_h.resize((size_t)d.nnz);
                fascicle_h.resize((size_t)d.nnz);
                phi_h.resize((size_t)d.nnz);
                hipError_t e = hipMemcpy(atom_h.data(), atom_in, sizeof(int16_t) * d.nnz, hipMemcpyDeviceToHost);
                if (e == hipSuccess) e = hipMemcpy(voxel_h.data(), voxel_in, sizeof(int32_t) * d.nnz, hipMemcpyDeviceToHost);
                if (e == hipSuccess)
                    e = hipMemcpy(fascicle_h.data(), fascicle_in, sizeof(int32_t) * d.nnz, hipMemcpyDeviceToHost);
                if (e == hipSuccess) e = hipMemcpy(phi_h.data(), phi_in, sizeof(float) * d.nnz, hipMemcpyDeviceToHost);
                if (e != hipSuccess) return LIFE_EDEVICE;
                atom = atom_h.data();
                voxel = voxel_h.data();
                fascicle = fascicle_h.data();
                phi = phi_h.data();
            }
            if (batched) {
                if ((st = life::validate_indices(&d, atom, voxel, fascicle)) != LIFE_OK) return st;
                if ((st = life::validate_instances(&d, n_inst, vox_off, fas_off, voxel, fascicle)) != LIFE_OK)
                    return st;
            }
            perm.resize((size_t)d.nnz);
            wperm.resize((size_t)d.nnz);
            vptr.resize((size_t)d.n_voxels + 1);
            fptr.resize((size_t)d.n_fascicles + 1);
            rank.resize((size_t)d.n_fascicles);
            ext.resize((size_t)d.n_fascicles);
            st = life::plan_host(&d, atom, voxel, fascicle, ppos_used, n_pos, batched ? fas_inst.data() : nullptr,
                                 perm.data(), vptr.data(), rank.data(), wperm.data(), fptr.data());
            if (st != LIFE_OK) return st;
            for (int32_t f = 0; f < d.n_fascicles; ++f) ext[(size_t)rank[(size_t)f]] = f;
            atom_v.resize((size_t)d.nnz);
            fas_v.resize((size_t)d.nnz);
            phi_v.resize((size_t)d.nnz);
            vdsc.resize((size_t)d.nnz);
            for (int64_t q = 0; q < d.nnz; ++q) {
                const int32_t c = perm[(size_t)q];
                atom_v[(size_t)q] = atom[c];
                fas_v[(size_t)q] = rank[(size_t)fascicle[c]];
                phi_v[(size_t)q] = phi[c];
                vdsc[(size_t)q] = voxel[c];
            }
            if (tg.row_floats > 0) {
                st = life::chunk_layout(&d, tg, vptr.data(), atom_v.data(), fas_v.data(), phi_v.data(), vdsc.data(),
                                        wperm.data(), ppos.data(), pvox.data(), n_pos, &L);
                if (st != LIFE_OK) return st;
                if (L.fas_overflow) {
                    // a voxel crosses more fascicles than a chunk can hold: generic kernels
                    if (batched) return LIFE_EINVAL;
                    L = life::ChunkLayout();
                }
                n_chunks = L.n_chunks;
                bounds = L.bounds;
                work = L.work;
                max_fas = L.max_fas;
                n_pad = L.n_pad;
                n_runs = L.n_runs;
            }
            if (n_chunks == 0 && d.nnz > 0) {
                // atom-major copy of the nonzeros for the generic dictionary gradient
                aptr.assign((size_t)d.n_atoms + 1, 0);
                for (int64_t q = 0; q < d.nnz; ++q) ++aptr[(size_t)atom_v[(size_t)q] + 1];
                for (int32_t a = 0; a < d.n_atoms; ++a) aptr[(size_t)a + 1] += aptr[(size_t)a];
                std::vector<int32_t> fill(aptr.begin(), aptr.end() - 1);
                avox.resize((size_t)d.nnz);
                afas.resize((size_t)d.nnz);
                aphi.resize((size_t)d.nnz);
                for (int64_t q = 0; q < d.nnz; ++q) {
                    const int32_t e = fill[(size_t)atom_v[(size_t)q]]++;
                    avox[(size_t)e] = vdsc[(size_t)q];
                    afas[(size_t)e] = fas_v[(size_t)q];
                    aphi[(size_t)e] = phi_v[(size_t)q];
                }
            }
        }
        if (batched) {
            // first chunk of each instance: instance blocks are whole groups of positions
            int32_t base = 0;
            size_t c = 0;
            for (int k = 0; k < n_inst; ++k) {
                base += cdiv(vox_off[k + 1] - vox_off[k], kChunkVoxels) * kChunkVoxels;
                while (c < bounds.size() && bounds[c] < base) ++c;
                ichunk[(size_t)k + 1] = static_cast<int32_t>(c);
            }
        } else {
            ichunk[1] = n_chunks;
        }
        if (n_chunks > 0) {
            // one grid length for every schedule policy (the longest map, the others
            // padded with -1), so that re-scheduling keeps the map's address and the
            // grid of launches already captured in a graph
            size_t grid = 0;
            for (int pol : {life::kScheduleIndex, life::kScheduleXcdCount, life::kScheduleXcdWork})
                grid = std::max(grid, life::chunk_schedule(work, (life::SchedulePolicy)pol).size());
            cmap = life::chunk_schedule(work, life::kScheduleDefault);
            cmap.resize(grid, -1);
        }
    } catch (const std::bad_alloc &) {
        return LIFE_ENOMEM;
    }

    life_plan_s *p = new (std::nothrow) life_plan_s;
    if (!p) return LIFE_ENOMEM;
    p->dims = d;
    p->device = dev;
    p->slots = slots_for(d.n_theta);
    p->tile = tg;
    p->n_chunks = n_chunks;
    p->n_pad = n_pad;
    p->chunk_grid = (int)cmap.size();
    p->chunk_work = work;
    p->max_fas = max_fas;
    p->n_runs = n_runs;
    const int64_t nb = std::max<int64_t>({cdiv(d.n_voxels, kSegPerBlock), (int64_t)n_chunks,
                                          cdiv(d.n_fascicles, kFasPerBlock), cdiv(d.n_fascicles, kBlock), 1});
    p->part_stride = nb;
    if (n_chunks > 0) {
        const int T = tg.n_tiles;
        // the widest span of tiles whose block fits the LDS and the accumulator variants
        const int nt16 = (d.n_theta + 15) / 16 * 16;
        p->dd_span = 1;
        for (int sp = 2; sp <= T; ++sp) {
            const int tap = (sp * tg.tile_atoms + 15) / 16 * 16;
            const int blocks = nt16 / 16 * (tap / 16);
            if (sp * tg.tile_atoms > life::kMaxTileAtoms || (int64_t)(tap + nt16) * kPsiStride * 4 > life::kLdsBudget ||
                dd_nbw_variant((blocks + kChunkWaves - 1) / kChunkWaves) < 0)
                break;
            p->dd_span = sp;
        }
        const int DT = (T + p->dd_span - 1) / p->dd_span;
        p->dd_tap = (p->dd_span * tg.tile_atoms + 15) / 16 * 16;
        p->dd_groups = std::max(1, std::min(n_chunks, 512 / DT));
        const int nb_blocks = nt16 / 16 * (p->dd_tap / 16);
        p->dd_nbw = dd_nbw_variant((nb_blocks + kChunkWaves - 1) / kChunkWaves);
        p->dd_floats = (int64_t)DT * p->dd_groups * p->dd_tap * nt16;
        p->dt_ab = (tg.tile_atoms + 31) / 32;
        p->dt_ks = (d.n_theta + 31) / 32;
        p->wcr_lds = (size_t)p->dt_ab * 32 * kPS * sizeof(float) +
                     (size_t)kDigits * kChunkVoxels * (32 * p->dt_ks + kQ8Pad) +
                     kChunkVoxels * sizeof(float);
        // DSC: the dictionary tile, then one weight per fascicle of the chunk
        p->dsc_lds = tile_lds_bytes(p) + (size_t)p->max_fas * sizeof(float);
        if (p->dd_nbw < 0 ||
            (int64_t)(p->dd_tap + (d.n_theta + 15) / 16 * 16) * kPsiStride * 4 > life::kLdsBudget ||
            p->dt_ab > kChunkWaves || p->dt_ks > 4 || p->wcr_lds > (size_t)life::kLdsBudget ||
            p->dsc_lds > (size_t)life::kLdsBudget) {
            delete p;
            return LIFE_EINVAL;   // cannot happen: tiles hold at most kMaxTileAtoms atoms, N_theta <= 128
        }
    }
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
    auto up = [&](void *dst, const void *src, size_t bytes) {
        if (bytes) chk(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    };
    // dst <- the device-built array (taken over), or a new copy of the host array
    auto take = [&](auto **dst, auto *&dev_src, const auto &host_src) {
        if (on_gpu) {
            *dst = dev_src;
            dev_src = nullptr;
        } else {
            chk(dalloc(dst, (int64_t)host_src.size()));
            up(*dst, host_src.data(), sizeof(host_src[0]) * host_src.size());
        }
    };
    take(&p->vox_ptr, G.vox_ptr, vptr);
    take(&p->atom_v, G.atom_v, atom_v);
    take(&p->fas_v, G.fas_v, fas_v);
    take(&p->phi_v, G.phi_v, phi_v);
    take(&p->fas_rank, G.fas_rank, rank);
    take(&p->fas_ext, G.fas_ext, ext);
    take(&p->fas_ptr, G.fas_ptr, fptr);
    take(&p->wc_perm, G.wc_perm, wperm);
    take(&p->chunk_vox, G.chunk_vox, L.chunk_vox);
    take(&p->wave_work, G.wave_work, L.wave_work);
    take(&p->atom_c, G.atom_c, L.atom_c);
    take(&p->fas_c, G.fas_c, L.fas_c);
    take(&p->loc_c, G.loc_c, L.loc_c);
    take(&p->phi_c, G.phi_c, L.phi_c);
    take(&p->cfas_ptr, G.cfas_ptr, L.cfas_ptr);
    take(&p->cfas, G.cfas, L.cfas);
    take(&p->wkey, G.wkey, L.wkey);
    take(&p->wphi, G.wphi, L.wphi);
    take(&p->wc_wave, G.wc_wave, L.wc_wave);
    take(&p->wc_wrun, G.wc_wrun, L.wc_wrun);
    take(&p->rr_ptr, G.rr_ptr, L.rr_ptr);
    take(&p->rr, G.rr, L.rr);
    if (n_chunks > 0) {
        // the DSC reads its stream as one 8-byte record per entry
        chk(dalloc(&p->dsc_rec, n_pad));
        if (e == hipSuccess && n_pad > 0)
            k_pack_dsc<<<cdiv(n_pad, kBlock), kBlock>>>(p->atom_c, p->loc_c, p->phi_c, n_pad, p->dsc_rec);
        chk(dalloc(&p->wc_rec, d.nnz));
        if (e == hipSuccess && d.nnz > 0)
            k_pack_wc<<<cdiv(d.nnz, kBlock), kBlock>>>(p->wkey, p->wphi, d.nnz, p->wc_rec);
    }
    chk(dalloc(&p->chunk_map, (int64_t)cmap.size()));
    up(p->chunk_map, cmap.data(), sizeof(int32_t) * cmap.size());
    {
        char *base = nullptr;
        chk(dalloc(&base, (int64_t)workspace_layout(p, kWsAll, nullptr, nullptr)));
        p->ws_base = base;
        workspace_layout(p, kWsAll, base, &p->ws);
    }
    chk(dalloc(&p->a_ptr, (int64_t)aptr.size()));
    chk(dalloc(&p->a_vox, (int64_t)avox.size()));
    chk(dalloc(&p->a_fas, (int64_t)afas.size()));
    chk(dalloc(&p->a_phi, (int64_t)aphi.size()));
    p->n_inst = n_inst;
    chk(dalloc(&p->inst_chunk, (int64_t)n_inst + 1));
    chk(dalloc(&p->inst_rank, (int64_t)n_inst + 1));
    if (e == hipSuccess && n_chunks > 0) e = allow_lds();
    if (e != hipSuccess) {
        free_plan(p);
        return e == hipErrorOutOfMemory ? LIFE_ENOMEM : LIFE_EDEVICE;
    }
    up(p->a_ptr, aptr.data(), sizeof(int32_t) * aptr.size());
    up(p->a_vox, avox.data(), sizeof(int32_t) * avox.size());
    up(p->a_fas, afas.data(), sizeof(int32_t) * afas.size());
    up(p->a_phi, aphi.data(), sizeof(float) * aphi.size());
    up(p->inst_chunk, ichunk.data(), sizeof(int32_t) * ichunk.size());
    up(p->inst_rank, fas_off, sizeof(int32_t) * ((size_t)n_inst + 1));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_plan(p);
        return LIFE_EDEVICE;
    }
    *out = p;
    return LIFE_OK;
}

}  // namespace

extern "C" life_status life_plan_ex(const life_dims *dims, const int16_t *atom, const int32_t *voxel,
                                    const int32_t *fascicle, const float *phi, const int16_t *voxel_xyz,
                                    life_plan_t *out)
{
    return build_plan(dims, atom, voxel, fascicle, phi, voxel_xyz, 1, nullptr, nullptr, 0, 0, out);
}

extern "C" life_status life_plan_batch(const life_dims *dims, int32_t n_inst, const int32_t *vox_off,
                                       const int32_t *fas_off, const int16_t *atom, const int32_t *voxel,
                                       const int32_t *fascicle, const float *phi, const int16_t *voxel_xyz,
                                       life_plan_t *out)
{
    if (n_inst < 1 || !vox_off || !fas_off) return LIFE_EINVAL;
    return build_plan(dims, atom, voxel, fascicle, phi, voxel_xyz, n_inst, vox_off, fas_off, 0, 0, out);
}

extern "C" life_status life_plan_flags(const life_dims *dims, int32_t n_inst, const int32_t *vox_off,
                                       const int32_t *fas_off, const int16_t *atom, const int32_t *voxel,
                                       const int32_t *fascicle, const float *phi, const int16_t *voxel_xyz,
                                       uint32_t flags, int32_t tile_atoms, life_plan_t *out)
{
    if (n_inst < 1 || (n_inst > 1 && (!vox_off || !fas_off))) return LIFE_EINVAL;
    if (flags & ~(uint32_t)(LIFE_PLAN_DEVICE_INPUT | LIFE_PLAN_HOST_BUILD)) return LIFE_EINVAL;
    return build_plan(dims, atom, voxel, fascicle, phi, voxel_xyz, n_inst, vox_off, fas_off, flags, tile_atoms,
                      out);
}

extern "C" life_status life_plan_tile_atoms(life_plan_t plan, int32_t *tile_atoms)
{
    if (!plan || !tile_atoms) return LIFE_EINVAL;
    *tile_atoms = chunked(plan) ? plan->tile.tile_atoms : 0;
    return LIFE_OK;
}

namespace {

// x[i] = a deterministic pseudo-random value in [lo, lo + span) (inputs of the timing runs)
__global__ void k_fill_hash(float *x, int64_t n, uint32_t seed, float lo, float span)
{
    const int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (i >= n) return;
    uint32_t h = (uint32_t)i * 2654435761u ^ seed;
    h ^= h >> 16;
    h *= 2246822519u;
    h ^= h >> 13;
    h *= 3266489917u;
    h ^= h >> 16;
    x[i] = lo + span * (float)(h >> 8) * (1.0f / 16777216.0f);
}

// Milliseconds of reps DSC + WC pairs of a plan on (D, w, y) (one warm-up pair first).
life_status time_pairs(life_plan_s *p, const float *D, const float *w, const float *y, float *yo, float *go, int reps,
                       float *ms)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LIFE_EDEVICE;
    life_status st = LIFE_OK;
    for (int i = -1; i < reps && st == LIFE_OK; ++i) {
        if (i == 0 && hipEventRecord(e0, nullptr) != hipSuccess) st = LIFE_EDEVICE;
        if (st == LIFE_OK) st = life_dsc(p, D, w, yo, nullptr);
        if (st == LIFE_OK) st = life_wc(p, D, y, go, nullptr);
    }
    if (st == LIFE_OK && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(ms, e0, e1) != hipSuccess))
        st = LIFE_EDEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

}  // namespace

extern "C" life_status life_plan_autotune(const life_dims *dims, int32_t n_inst, const int32_t *vox_off,
                                          const int32_t *fas_off, const int16_t *atom, const int32_t *voxel,
                                          const int32_t *fascicle, const float *phi, const int16_t *voxel_xyz,
                                          uint32_t flags, const float *D, int32_t reps, int32_t *tile_atoms_out,
                                          int32_t *policy_out, life_plan_t *out)
{
    if (!out || !dims || reps < 1 || (dims->n_theta > 0 && dims->n_atoms > 0 && !D)) return LIFE_EINVAL;
    *out = nullptr;
    if (n_inst < 1 || (n_inst > 1 && (!vox_off || !fas_off))) return LIFE_EINVAL;
    if (flags & ~(uint32_t)LIFE_PLAN_DEVICE_INPUT) return LIFE_EINVAL;
    life_status st = life::validate_dims(dims);
    if (st != LIFE_OK) return st;
    const life_dims d = *dims;
    // candidate tiles: 3, 4, 5, 6 and 8 tiles of the dictionary (those the LDS holds)
    std::vector<int> cands;
    for (int nt : {5, 4, 6, 3, 8}) {
        const int ta = (d.n_atoms + nt - 1) / nt;
        const life::TileGeom tg = life::tile_geometry(d.n_theta, d.n_atoms, ta);
        if (tiling_fits(d.n_theta, tg) && std::find(cands.begin(), cands.end(), tg.tile_atoms) == cands.end())
            cands.push_back(tg.tile_atoms);
    }
    if (cands.empty()) {   // N_theta > 128: one (generic) plan, nothing to choose
        st = build_plan(dims, atom, voxel, fascicle, phi, voxel_xyz, n_inst, vox_off, fas_off, flags, 0, out);
        if (st == LIFE_OK && tile_atoms_out) *tile_atoms_out = 0;
        if (st == LIFE_OK && policy_out) *policy_out = (*out)->schedule;
        return st;
    }
    // the COO arrays on the device once; every candidate is built from them
    void *coo[4] = {nullptr, nullptr, nullptr, nullptr};
    float *buf[4] = {nullptr, nullptr, nullptr, nullptr};   // w, y, y out, g out
    life_plan_t best = nullptr;
    float best_ms = 0.f;
    int best_ta = 0;
    st = LIFE_OK;
    auto cleanup = [&]() {
        for (void *q : coo)
            if (q) (void)hipFree(q);
        for (float *q : buf)
            if (q) (void)hipFree(q);
    };
    const int16_t *a_d = atom;
    const int32_t *v_d = voxel, *f_d = fascicle;
    const float *p_d = phi;
    if (!(flags & LIFE_PLAN_DEVICE_INPUT) && d.nnz > 0) {
        const size_t sz[4] = {sizeof(int16_t), sizeof(int32_t), sizeof(int32_t), sizeof(float)};
        const void *src[4] = {atom, voxel, fascicle, phi};
        for (int i = 0; i < 4 && st == LIFE_OK; ++i) {
            if (!src[i] || hipMalloc(&coo[i], sz[i] * (size_t)d.nnz) != hipSuccess ||
                hipMemcpy(coo[i], src[i], sz[i] * (size_t)d.nnz, hipMemcpyHostToDevice) != hipSuccess)
                st = src[i] ? LIFE_EDEVICE : LIFE_EINVAL;
        }
        a_d = static_cast<const int16_t *>(coo[0]);
        v_d = static_cast<const int32_t *>(coo[1]);
        f_d = static_cast<const int32_t *>(coo[2]);
        p_d = static_cast<const float *>(coo[3]);
    }
    const int64_t nsig = (int64_t)d.n_theta * d.n_voxels, nw = d.n_fascicles;
    const int64_t lens[4] = {nw, nsig, nsig, nw};
    for (int i = 0; i < 4 && st == LIFE_OK; ++i)
        if (lens[i] > 0 && hipMalloc(&buf[i], sizeof(float) * (size_t)lens[i]) != hipSuccess) st = LIFE_ENOMEM;
    if (st == LIFE_OK && nw > 0) k_fill_hash<<<cdiv(nw, kBlock), kBlock>>>(buf[0], nw, 12345u, 0.f, 1.f);
    if (st == LIFE_OK && nsig > 0) k_fill_hash<<<cdiv(nsig, kBlock), kBlock>>>(buf[1], nsig, 777u, -1.f, 2.f);
    for (size_t k = 0; k < cands.size() && st == LIFE_OK; ++k) {
        life_plan_t p = nullptr;
        st = build_plan(dims, a_d, v_d, f_d, p_d, voxel_xyz, n_inst, vox_off, fas_off, LIFE_PLAN_DEVICE_INPUT,
                        cands[k], &p);
        if (st != LIFE_OK) break;
        float ms = 0.f;
        st = time_pairs(p, D, buf[0], buf[1], buf[2], buf[3], reps, &ms);
        if (st != LIFE_OK) {
            (void)life_plan_destroy(p);
            break;
        }
        if (!best || ms < best_ms) {
            if (best) (void)life_plan_destroy(best);
            best = p;
            best_ms = ms;
            best_ta = cands[k];
        } else {
            (void)life_plan_destroy(p);
        }
    }
    int32_t pol = 0;
    if (st == LIFE_OK && best) st = life_plan_tune(best, D, buf[0], buf[1], reps, &pol);
    cleanup();
    if (st != LIFE_OK) {
        if (best) (void)life_plan_destroy(best);
        return st;
    }
    *out = best;
    if (tile_atoms_out) *tile_atoms_out = chunked(best) ? best_ta : 0;
    if (policy_out) *policy_out = pol;
    return LIFE_OK;
}

namespace {

// FNV-1a over bytes, continued from h
uint64_t fnv1a(uint64_t h, const void *data, size_t bytes)
{
    const unsigned char *b = static_cast<const unsigned char *>(data);
    for (size_t i = 0; i < bytes; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

}  // namespace

extern "C" life_status life_plan_digest(life_plan_t plan, uint64_t *digest)
{
    if (!plan || !digest) return LIFE_EINVAL;
    DeviceGuard g(plan->device);
    if (!g.ok) return LIFE_EDEVICE;
    const life_plan_s &p = *plan;
    const life_dims &d = p.dims;
    const int T = p.tile.n_tiles;
    const int64_t nct = (int64_t)p.n_chunks * T;
    struct Arr {
        const void *ptr;
        int64_t bytes;
    };
    const Arr arrs[LIFE_DIGEST_WORDS - 1] = {
        {p.vox_ptr, 4 * ((int64_t)d.n_voxels + 1)},
        {p.atom_v, 2 * d.nnz},
        {p.fas_v, 4 * d.nnz},
        {p.phi_v, 4 * d.nnz},
        {p.fas_rank, 4 * (int64_t)d.n_fascicles},
        {p.fas_ext, 4 * (int64_t)d.n_fascicles},
        {p.fas_ptr, 4 * ((int64_t)d.n_fascicles + 1)},
        {p.wc_perm, 4 * d.nnz},
        {p.chunk_vox, 4 * (int64_t)p.n_chunks * kChunkVoxels},
        {p.wave_work, 4 * nct * kChunkWaves * life::kWorkInts},
        {p.atom_c, 2 * p.n_pad},
        {p.fas_c, 4 * p.n_pad},
        {p.loc_c, 2 * p.n_pad},
        {p.phi_c, 4 * p.n_pad},
        {p.cfas_ptr, p.n_chunks > 0 ? 4 * ((int64_t)p.n_chunks + 1) : 0},
        {p.cfas, 0},   // length from cfas_ptr below
        {p.wkey, p.n_chunks > 0 ? 2 * d.nnz : 0},
        {p.wphi, p.n_chunks > 0 ? 4 * d.nnz : 0},
        {p.wc_wave, p.n_chunks > 0 ? 4 * (nct * kChunkWaves + 1) : 0},
        {p.wc_wrun, 4 * nct * kChunkWaves},
        {p.rr_ptr, p.n_chunks > 0 ? 4 * ((int64_t)d.n_fascicles + 1) : 0},
        {p.rr, 4 * p.n_runs},
        {p.chunk_map, 4 * (int64_t)p.chunk_grid},
    };
    int64_t n_cfas = 0;
    if (p.n_chunks > 0 && p.cfas_ptr) {
        int32_t last = 0;
        if (hipMemcpy(&last, p.cfas_ptr + p.n_chunks, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
            return LIFE_EDEVICE;
        n_cfas = last;
    }
    std::vector<unsigned char> buf;
    for (int i = 0; i < LIFE_DIGEST_WORDS - 1; ++i) {
        const int64_t bytes = i == 15 ? 4 * n_cfas : arrs[i].bytes;
        uint64_t h = 1469598103934665603ull;
        if (bytes > 0 && arrs[i].ptr) {
            try {
                buf.resize((size_t)bytes);
            } catch (const std::bad_alloc &) {
                return LIFE_ENOMEM;
            }
            if (hipMemcpy(buf.data(), arrs[i].ptr, (size_t)bytes, hipMemcpyDeviceToHost) != hipSuccess)
                return LIFE_EDEVICE;
            h = fnv1a(h, buf.data(), (size_t)bytes);
        }
        digest[i] = h;
    }
    const int64_t scal[5] = {p.n_chunks, p.n_pad, p.n_runs, p.max_fas, p.chunk_grid};
    digest[LIFE_DIGEST_WORDS - 1] = fnv1a(1469598103934665603ull, scal, sizeof(scal));
    return LIFE_OK;
}

extern "C" life_status life_plan_destroy(life_plan_t plan)
{
    if (!plan) return LIFE_OK;
    DeviceGuard g(plan->device);
    (void)hipDeviceSynchronize();
    free_plan(plan);
    return g.ok ? LIFE_OK : LIFE_EDEVICE;
}

extern "C" life_status life_plan_dims(life_plan_t plan, life_dims *out)
{
    if (!plan || !out) return LIFE_EINVAL;
    *out = plan->dims;
    return LIFE_OK;
}

extern "C" life_status life_plan_export(life_plan_t plan, int32_t *vox_ptr, int16_t *atom_v, int32_t *fas_v,
                                        float *phi_v, int32_t *fas_rank, int32_t *fas_ptr, int32_t *wc_perm)
{
    if (!plan) return LIFE_EINVAL;
    DeviceGuard g(plan->device);
    if (!g.ok) return LIFE_EDEVICE;
    const life_dims &d = plan->dims;
    hipError_t e = hipSuccess;
    auto down = [&](void *dst, const void *src, size_t bytes) {
        if (dst && bytes && e == hipSuccess) e = hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
    };
    down(vox_ptr, plan->vox_ptr, sizeof(int32_t) * (size_t)(d.n_voxels + 1));
    down(atom_v, plan->atom_v, sizeof(int16_t) * (size_t)d.nnz);
    down(fas_v, plan->fas_v, sizeof(int32_t) * (size_t)d.nnz);
    down(phi_v, plan->phi_v, sizeof(float) * (size_t)d.nnz);
    down(fas_rank, plan->fas_rank, sizeof(int32_t) * (size_t)d.n_fascicles);
    down(fas_ptr, plan->fas_ptr, sizeof(int32_t) * (size_t)(d.n_fascicles + 1));
    down(wc_perm, plan->wc_perm, sizeof(int32_t) * (size_t)d.nnz);
    return e == hipSuccess ? LIFE_OK : LIFE_EDEVICE;
}

static bool need(const void *ptr, int64_t n) { return n == 0 || ptr != nullptr; }

namespace {

// The workspace of a call: the caller's scratch (at least life_plan_scratch_bytes,
// 256-byte aligned) carved like the plan's own, or the plan's own when scratch is NULL.
life_status call_workspace(life_plan_s *p, void *scratch, uint64_t bytes, Workspace *ws)
{
    if (!scratch) {
        *ws = p->ws;
        return LIFE_OK;
    }
    const size_t want = workspace_layout(p, kWsAll, nullptr, nullptr);
    if (bytes < want || (reinterpret_cast<uintptr_t>(scratch) & 255) != 0) return LIFE_EINVAL;
    workspace_layout(p, kWsAll, static_cast<char *>(scratch), ws);
    return LIFE_OK;
}

life_status dsc_call(life_plan_s *plan, const Workspace &ws, const float *D, const float *w, float *y,
                     hipStream_t s)
{
    life_status st = enqueue_gather(plan, ws, w, s);
    if (st != LIFE_OK) return st;
    return enqueue_dsc(plan, D, ws.w_rank, nullptr, y, nullptr, s);
}

bool dsc_args_ok(const life_plan_s *plan, const float *D, const float *w, const float *y)
{
    const life_dims &d = plan->dims;
    return need(D, (int64_t)d.n_theta * d.n_atoms) && need(w, d.n_fascicles) && need(y, (int64_t)d.n_theta * d.n_voxels);
}

}  // namespace

extern "C" life_status life_plan_scratch_bytes(life_plan_t plan, uint64_t *bytes)
{
    if (!plan || !bytes) return LIFE_EINVAL;
    *bytes = workspace_layout(plan, kWsAll, nullptr, nullptr);
    return LIFE_OK;
}

extern "C" life_status life_dsc_ws(life_plan_t plan, const float *D, const float *w, float *y, void *scratch,
                                   uint64_t scratch_bytes, void *stream)
{
    if (!plan || !dsc_args_ok(plan, D, w, y)) return LIFE_EINVAL;
    Workspace ws;
    life_status st = call_workspace(plan, scratch, scratch_bytes, &ws);
    if (st != LIFE_OK) return st;
    DeviceGuard g(plan->device);
    if (!g.ok) return LIFE_EDEVICE;
    return dsc_call(plan, ws, D, w, y, static_cast<hipStream_t>(stream));
}

extern "C" life_status life_dsc(life_plan_t plan, const float *D, const float *w, float *y, void *stream)
{
    return life_dsc_ws(plan, D, w, y, nullptr, 0, stream);
}

extern "C" life_status life_wc_ws(life_plan_t plan, const float *D, const float *y, float *g, void *scratch,
                                  uint64_t scratch_bytes, void *stream)
{
    if (!plan) return LIFE_EINVAL;
    const life_dims &d = plan->dims;
    if (!need(D, (int64_t)d.n_theta * d.n_atoms) || !need(y, (int64_t)d.n_theta * d.n_voxels) ||
        !need(g, d.n_fascicles))
        return LIFE_EINVAL;
    Workspace ws;
    life_status st = call_workspace(plan, scratch, scratch_bytes, &ws);
    if (st != LIFE_OK) return st;
    DeviceGuard gd(plan->device);
    if (!gd.ok) return LIFE_EDEVICE;
    return enqueue_wc(plan, ws, D, y, g, plan->fas_ext, nullptr, Gate{nullptr, 0}, static_cast<hipStream_t>(stream));
}

extern "C" life_status life_wc(life_plan_t plan, const float *D, const float *y, float *g, void *stream)
{
    return life_wc_ws(plan, D, y, g, nullptr, 0, stream);
}

namespace {

// One SBB-NNLS iteration; gt_prev != NULL selects the lagged (eqs. 7-8) step.
life_status enqueue_sbb(life_plan_s *plan, const Workspace &ws, const float *D, const float *b, float *w,
                        float *gt_prev, life_sbb_state *state, hipStream_t s)
{
    const life_dims &d = plan->dims;
    const bool lagged = gt_prev != nullptr;
    const int64_t ps = plan->part_stride;
    double *p_r = ws.part, *p_gt = ws.part + ps, *p_vp = ws.part + 2 * ps, *p_vpp = ws.part + 3 * ps;
    double *p_q = ws.part + 4 * ps;
    const int nv = d.n_voxels, nf = d.n_fascicles;
    const int nb_dsc = nv > 0 ? dsc_partials(plan) : 0;
    const int nb_mask = nf > 0 ? cdiv(nf, kBlock) : 0;
    const int nb_sum = nf > 0 ? cdiv(nf, kFasPerBlock) : 0;
    life_status st;
    // weights into fascicle-rank order (every vector of the step below stays in it)
    if ((st = enqueue_gather(plan, ws, w, s)) != LIFE_OK) return st;
    // r = M w - b, partial ||r||^2
    if ((st = enqueue_dsc(plan, D, ws.w_rank, b, ws.r, p_r, s)) != LIFE_OK) return st;
    // g = M^T r
    if ((st = enqueue_wc(plan, ws, D, ws.r, ws.g, nullptr, nullptr, Gate{nullptr, 0}, s)) != LIFE_OK) return st;
    // g~ and ||g~||^2
    if (nf > 0) {
        st = launch(plan, LIFE_K_MASK, s, [&] {
            k_mask<<<nb_mask, kBlock, 0, s>>>(ws.w_rank, ws.g, ws.gt, p_gt, nf);
        });
        if (st != LIFE_OK) return st;
    }
    // q: g~ (Algorithm 1) or the previous iterate's g~ (eqs. 7-8), and ||q||^2
    const float *q = ws.gt;
    if (lagged && nf > 0) {
        st = launch(plan, LIFE_K_MASK, s, [&] {
            k_lag_q<<<nb_mask, kBlock, 0, s>>>(gt_prev, plan->fas_ext, ws.gt, ws.q, p_q, state, nf);
        });
        if (st != LIFE_OK) return st;
        q = ws.q;
    }
    // v' = M q, ||v'||^2
    if ((st = enqueue_dsc(plan, D, q, nullptr, ws.vp, p_vp, s)) != LIFE_OK) return st;
    // v'' = M^T v', ||v''||^2, on the iterations of the second alpha form (even i
    // in Algorithm 1, odd i in eqs. 7-8); the kernels test the parity on the device
    if ((st = enqueue_wc(plan, ws, D, ws.vp, ws.vpp, nullptr, p_vpp, Gate{state, lagged ? 1 : 0}, s, false)) !=
        LIFE_OK)
        return st;
    st = launch(plan, LIFE_K_ALPHA, s, [&] {
        k_alpha<<<1, kAlphaThreads, 0, s>>>(p_r, nb_dsc, p_gt, nb_mask, lagged ? p_q : nullptr, nb_mask, p_vp, nb_dsc,
                                            p_vpp, nb_sum, state, lagged ? 1 : 0);
    });
    if (st != LIFE_OK) return st;
    if (nf > 0) {
        st = launch(plan, LIFE_K_UPDATE, s, [&] {
            k_update<<<cdiv(nf, kBlock), kBlock, 0, s>>>(w, ws.w_rank, ws.gt, plan->fas_ext, state,
                                                         lagged ? gt_prev : nullptr, nf);
        });
    }
    return st;
}

}  // namespace

namespace {

// One SBB-NNLS iteration (Algorithm 1) of every instance of a batched plan.
life_status enqueue_sbb_batch(life_plan_s *plan, const Workspace &ws, const float *D, const float *b, float *w,
                              life_sbb_state *states, hipStream_t s)
{
    const life_dims &d = plan->dims;
    const int64_t ps = plan->part_stride;
    double *p_r = ws.part, *p_gt = ws.part + ps, *p_vp = ws.part + 2 * ps;
    const int nf = d.n_fascicles;
    const int nb_mask = nf > 0 ? cdiv(nf, kBlock) : 0;
    life_status st;
    if ((st = enqueue_gather(plan, ws, w, s)) != LIFE_OK) return st;
    if ((st = enqueue_dsc(plan, D, ws.w_rank, b, ws.r, p_r, s)) != LIFE_OK) return st;
    if ((st = enqueue_wc(plan, ws, D, ws.r, ws.g, nullptr, nullptr, Gate{nullptr, 0}, s)) != LIFE_OK) return st;
    if (nf > 0) {
        st = launch(plan, LIFE_K_MASK, s, [&] {
            k_mask<<<nb_mask, kBlock, 0, s>>>(ws.w_rank, ws.g, ws.gt, p_gt, nf);
        });
        if (st != LIFE_OK) return st;
    }
    if ((st = enqueue_dsc(plan, D, ws.gt, nullptr, ws.vp, p_vp, s)) != LIFE_OK) return st;
    // instances advance together: the first instance's parity gates the second WC
    if ((st = enqueue_wc(plan, ws, D, ws.vp, ws.vpp, nullptr, nullptr, Gate{states, 0}, s, false)) != LIFE_OK)
        return st;
    st = launch(plan, LIFE_K_ALPHA, s, [&] {
        k_alpha_batch<<<plan->n_inst, kAlphaThreads, 0, s>>>(p_r, p_vp, plan->inst_chunk, ws.gt, ws.vpp,
                                                             plan->inst_rank, states);
    });
    if (st != LIFE_OK) return st;
    if (nf > 0) {
        st = launch(plan, LIFE_K_UPDATE, s, [&] {
            k_update_batch<<<cdiv(nf, kBlock), kBlock, 0, s>>>(w, ws.w_rank, ws.gt, plan->fas_ext, states,
                                                               plan->inst_rank, plan->n_inst, nf);
        });
    }
    return st;
}

}  // namespace

extern "C" life_status life_plan_tune(life_plan_t plan, const float *D, const float *w, const float *y, int32_t reps,
                                      int32_t *policy)
{
    if (!plan || reps < 1) return LIFE_EINVAL;
    const life_dims &d = plan->dims;
    if (!need(D, (int64_t)d.n_theta * d.n_atoms) || !need(w, d.n_fascicles) ||
        !need(y, (int64_t)d.n_theta * d.n_voxels))
        return LIFE_EINVAL;
    if (!chunked(plan)) {
        if (policy) *policy = plan->schedule;
        return LIFE_OK;
    }
    DeviceGuard gd(plan->device);
    if (!gd.ok) return LIFE_EDEVICE;
    const bool prof = plan->profile;
    plan->profile = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LIFE_EDEVICE;
    // install the schedule of policy pol: the workgroup map is overwritten in place
    // (same address, same grid length: every map is padded with -1 to chunk_grid)
    auto install = [&](int pol) -> hipError_t {
        std::vector<int32_t> map = life::chunk_schedule(plan->chunk_work, (life::SchedulePolicy)pol);
        if (map.size() > (size_t)plan->chunk_grid) return hipErrorInvalidValue;   // cannot happen
        map.resize((size_t)plan->chunk_grid, -1);
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
        e = hipMemcpy(plan->chunk_map, map.data(), sizeof(int32_t) * map.size(), hipMemcpyHostToDevice);
        plan->schedule = pol;
        return e;
    };
    const int pols[] = {life::kScheduleIndex, life::kScheduleXcdCount, life::kScheduleXcdWork};
    float best = 0.f;
    int best_pol = plan->schedule;
    life_status st = LIFE_OK;
    for (int pol : pols) {
        if (install(pol) != hipSuccess) { st = LIFE_EDEVICE; break; }
        auto run = [&]() {
            const Workspace &ws = plan->ws;
            if (enqueue_gather(plan, ws, w, nullptr) != LIFE_OK) return false;
            if (enqueue_dsc(plan, D, ws.w_rank, nullptr, ws.r, nullptr, nullptr) != LIFE_OK) return false;
            return enqueue_wc(plan, ws, D, y, ws.g, nullptr, nullptr, Gate{nullptr, 0}, nullptr) == LIFE_OK;
        };
        if (!run()) { st = LIFE_EDEVICE; break; }                 // warm-up
        float ms = 0.f;
        bool ok = hipEventRecord(e0, nullptr) == hipSuccess;
        for (int i = 0; ok && i < reps; ++i) ok = run();
        ok = ok && hipEventRecord(e1, nullptr) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (!ok) { st = LIFE_EDEVICE; break; }
        if (best_pol < 0 || pol == pols[0] || ms < best) {
            best = ms;
            best_pol = pol;
        }
    }
    if (st == LIFE_OK && install(best_pol) != hipSuccess) st = LIFE_EDEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan->profile = prof;
    if (st == LIFE_OK && policy) *policy = best_pol;
    return st;
}

extern "C" life_status life_plan_instances(life_plan_t plan, int32_t *n_inst)
{
    if (!plan || !n_inst) return LIFE_EINVAL;
    *n_inst = plan->n_inst;
    return LIFE_OK;
}

extern "C" life_status life_sbbnnls_step_batch(life_plan_t plan, const float *D, const float *b, float *w,
                                               life_sbb_state *states, void *stream)
{
    if (!plan || !states) return LIFE_EINVAL;
    const life_dims &d = plan->dims;
    if (!chunked(plan) && plan->n_inst > 1) return LIFE_EINVAL;
    if (!need(D, (int64_t)d.n_theta * d.n_atoms) || !need(b, (int64_t)d.n_theta * d.n_voxels) ||
        !need(w, d.n_fascicles))
        return LIFE_EINVAL;
    if (!chunked(plan)) return life_sbbnnls_step(plan, D, b, w, states, stream);   // one instance
    DeviceGuard gd(plan->device);
    if (!gd.ok) return LIFE_EDEVICE;
    return enqueue_sbb_batch(plan, plan->ws, D, b, w, states, static_cast<hipStream_t>(stream));
}

extern "C" life_status life_sbbnnls_step_ws(life_plan_t plan, const float *D, const float *b, float *w,
                                            life_sbb_state *state, void *scratch, uint64_t scratch_bytes,
                                            void *stream)
{
    if (!plan || !state) return LIFE_EINVAL;
    const life_dims &d = plan->dims;
    if (!need(D, (int64_t)d.n_theta * d.n_atoms) || !need(b, (int64_t)d.n_theta * d.n_voxels) ||
        !need(w, d.n_fascicles))
        return LIFE_EINVAL;
    Workspace ws;
    life_status st = call_workspace(plan, scratch, scratch_bytes, &ws);
    if (st != LIFE_OK) return st;
    DeviceGuard gd(plan->device);
    if (!gd.ok) return LIFE_EDEVICE;
    return enqueue_sbb(plan, ws, D, b, w, nullptr, state, static_cast<hipStream_t>(stream));
}

extern "C" life_status life_sbbnnls_step(life_plan_t plan, const float *D, const float *b, float *w,
                                         life_sbb_state *state, void *stream)
{
    return life_sbbnnls_step_ws(plan, D, b, w, state, nullptr, 0, stream);
}

extern "C" life_status life_sbbnnls_step_lagged(life_plan_t plan, const float *D, const float *b, float *w,
                                                float *gt_prev, life_sbb_state *state, void *stream)
{
    if (!plan || !state) return LIFE_EINVAL;
    const life_dims &d = plan->dims;
    if (!need(D, (int64_t)d.n_theta * d.n_atoms) || !need(b, (int64_t)d.n_theta * d.n_voxels) ||
        !need(w, d.n_fascicles) || !need(gt_prev, d.n_fascicles))
        return LIFE_EINVAL;
    DeviceGuard gd(plan->device);
    if (!gd.ok) return LIFE_EDEVICE;
    return enqueue_sbb(plan, plan->ws, D, b, w, gt_prev, state, static_cast<hipStream_t>(stream));
}

extern "C" life_status life_dict_grad(life_plan_t plan, const float *w, const float *ybar, float *dD, void *stream)
{
    if (!plan) return LIFE_EINVAL;
    const life_dims &d = plan->dims;
    if (!need(w, d.n_fascicles) || !need(ybar, (int64_t)d.n_theta * d.n_voxels) ||
        !need(dD, (int64_t)d.n_theta * d.n_atoms))
        return LIFE_EINVAL;
    DeviceGuard gd(plan->device);
    if (!gd.ok) return LIFE_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Workspace &ws = plan->ws;
    life_status st = enqueue_gather(plan, ws, w, s);
    if (st != LIFE_OK) return st;
    return enqueue_dd(plan, ws, ybar, dD, s);
}

extern "C" life_status life_profile_enable(life_plan_t plan, int enable)
{
    if (!plan) return LIFE_EINVAL;
    plan->profile = enable != 0;
    return LIFE_OK;
}

extern "C" life_status life_profile_read(life_plan_t plan, double *ms, int64_t *count)
{
    if (!plan) return LIFE_EINVAL;
    DeviceGuard gd(plan->device);
    if (!gd.ok) return LIFE_EDEVICE;
    double acc[LIFE_K_COUNT] = {0};
    int64_t cnt[LIFE_K_COUNT] = {0};
    life_status st = LIFE_OK;
    for (auto &e : plan->events) {
        float t = 0.f;
        if (hipEventSynchronize(e.second.second) != hipSuccess ||
            hipEventElapsedTime(&t, e.second.first, e.second.second) != hipSuccess)
            st = LIFE_EDEVICE;
        acc[e.first] += t;
        cnt[e.first] += 1;
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    plan->events.clear();
    for (int k = 0; k < LIFE_K_COUNT; ++k) {
        if (ms) ms[k] = acc[k];
        if (count) count[k] = cnt[k];
    }
    return st;
}

// ============================================================================= allocation-free DSC

namespace {

// Scratch of life_dsc_noalloc: a file-scope device array, one copy per device,
// held from the first use until the process ends.  Host code never passes this
// symbol itself to a kernel (on the host it names a stand-in, not device memory);
// it uses the device address hipGetSymbolAddress returns for each device.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) char noalloc_scratch[kNoAllocScratchBytes];

std::mutex g_noalloc_mu;
char *g_noalloc_ptr[kMaxDevices] = {};

// Device address of noalloc_scratch on device dev (the current device), looked up
// once per device.
life_status noalloc_base(int dev, char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return LIFE_EDEVICE;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc_scratch)) != hipSuccess || !ptr) return LIFE_EDEVICE;
        g_noalloc_ptr[dev] = static_cast<char *>(ptr);
    }
    *out = g_noalloc_ptr[dev];
    return LIFE_OK;
}

}  // namespace

extern "C" life_status life_dsc_noalloc(life_plan_t plan, const float *D, const float *w, float *y, void *stream)
{
    if (!plan || !dsc_args_ok(plan, D, w, y)) return LIFE_EINVAL;
    if (workspace_layout(plan, kWsDsc, nullptr, nullptr) > kNoAllocScratchBytes) return LIFE_ERANGE;
    DeviceGuard g(plan->device);
    if (!g.ok) return LIFE_EDEVICE;
    char *base = nullptr;
    life_status st = noalloc_base(plan->device, &base);
    if (st != LIFE_OK) return st;
    Workspace ws;
    workspace_layout(plan, kWsDsc, base, &ws);
    NoEvents quiet;   // the profiling hooks would create events: not on this path
    return dsc_call(plan, ws, D, w, y, static_cast<hipStream_t>(stream));
}

extern "C" const char *life_hip_error(void) { return t_hip_error; }
