// The data restructuring of the LiFE sparse-Tucker products on the device.
//
// The same plan as the host builder (life_plan.cpp: plan_host, chunk_layout), bit
// for bit, built from device COO arrays: the restructuring step of Sec. 4.1 (sort
// the nonzeros by voxel for DSC and by fascicle for WC) as stable radix sorts, the
// chunked layout (padded per (chunk, tile, wave) ranges, chunk fascicle lists, WC
// buckets and runs, per-fascicle run lists) as gathers, scatters and scans.  The
// paper amortizes its restructuring over the SBB-NNLS iterations (3-5% of their
// time); on the host, single-threaded, this took longer than a 500-iteration solve.
//
// Every step is deterministic: sorts are stable, per-key counts use integer adds
// whose totals do not depend on their order, and min/max reductions are exact.
// The few O(voxels) and O(chunks) steps whose result the next step needs on the
// host (chunk splitting, the slot assignment, the schedule) run on the host over
// small downloaded arrays.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <vector>

#include "life_internal.h"

namespace life {
namespace {

constexpr int kT = 256;   // threads per block

int blocks(int64_t n) { return (int)std::max<int64_t>(1, (n + kT - 1) / kT); }

int bits_for(int64_t n)   // bits to hold 0 .. n - 1
{
    int b = 0;
    while (b < 62 && (int64_t(1) << b) < n) ++b;
    return b;
}

// Device allocations of one build: freed on destruction unless released to the plan.
struct Arena {
    std::vector<void *> ptrs;
    hipError_t err = hipSuccess;
    template <class T>
    T *get(int64_t n)
    {
        if (err != hipSuccess || n <= 0) return nullptr;
        void *p = nullptr;
        err = hipMalloc(&p, sizeof(T) * (size_t)n);
        if (err != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return static_cast<T *>(p);
    }
    template <class T>
    T *keep(T *p)   // ownership moves to the caller
    {
        ptrs.erase(std::remove(ptrs.begin(), ptrs.end(), static_cast<void *>(p)), ptrs.end());
        return p;
    }
    ~Arena()
    {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

// ------------------------------------------------------------------------------ kernels

__global__ void k_validate(const int16_t *atom, const int32_t *voxel, const int32_t *fascicle, int64_t n, int na,
                           int nv, int nf, const int32_t *fas_inst, const int32_t *vox_off, int *bad)
{
    const int64_t c = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (c >= n) return;
    const int a = atom[c], v = voxel[c], f = fascicle[c];
    bool b = a < 0 || a >= na || v < 0 || v >= nv || f < 0 || f >= nf;
    if (!b && fas_inst) {
        const int k = fas_inst[f];
        b = v < vox_off[k] || v >= vox_off[k + 1];
    }
    if (b) atomicOr(bad, 1);
}

// DSC sort key (voxel, atom, fascicle) in one 64-bit word, or only its voxel-atom
// part (fascicle pass first) when the three do not fit.
__global__ void k_dsc_keys(const int16_t *atom, const int32_t *voxel, const int32_t *fascicle, int64_t n, int bf,
                           bool with_fas, uint64_t *key, int32_t *val)
{
    const int64_t c = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (c >= n) return;
    const uint64_t va = (uint64_t)(uint32_t)voxel[c] << 15 | (uint64_t)(uint16_t)atom[c];
    key[c] = with_fas ? (va << bf | (uint64_t)(uint32_t)fascicle[c]) : va;
    val[c] = (int32_t)c;
}

__global__ void k_fas_keys32(const int32_t *fascicle, int64_t n, uint32_t *key, int32_t *val)
{
    const int64_t c = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (c >= n) return;
    key[c] = (uint32_t)fascicle[c];
    val[c] = (int32_t)c;
}

// with_fas = false: the voxel-atom keys of the nonzeros in the order of perm
__global__ void k_dsc_keys_perm(const int16_t *atom, const int32_t *voxel, const int32_t *perm, int64_t n,
                                uint64_t *key)
{
    const int64_t p = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (p >= n) return;
    const int32_t c = perm[p];
    key[p] = (uint64_t)(uint32_t)voxel[c] << 15 | (uint64_t)(uint16_t)atom[c];
}

__global__ void k_gather_dsc(const int32_t *perm, const int16_t *atom, const int32_t *voxel,
                             const int32_t *fascicle, const float *phi, int64_t n, int16_t *atom_v, int32_t *vox_v,
                             int32_t *fas_o, float *phi_v)
{
    const int64_t p = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (p >= n) return;
    const int32_t c = perm[p];
    atom_v[p] = atom[c];
    vox_v[p] = voxel[c];
    fas_o[p] = fascicle[c];
    phi_v[p] = phi[c];
}

// ptr[s] = first position whose key is >= s, for s = 0 .. nseg (keys ascending)
template <class K>
__global__ void k_seg_ptr(const K *keys, int64_t n, int64_t nseg, int shift, int32_t *ptr)
{
    const int64_t s = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (s > nseg) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)(keys[mid] >> shift) < s) lo = mid + 1;
        else hi = mid;
    }
    ptr[s] = (int32_t)lo;
}

__global__ void k_fill_i32(int32_t *a, int64_t n, int32_t v)
{
    const int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ void k_lohi(const int32_t *voxel, const int32_t *fascicle, const int32_t *proc_pos, int64_t n,
                       int32_t *lo, int32_t *hi)
{
    const int64_t c = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (c >= n) return;
    const int32_t p = proc_pos ? proc_pos[voxel[c]] : voxel[c];
    atomicMin(&lo[fascicle[c]], p);
    atomicMax(&hi[fascicle[c]], p);
}

__device__ uint64_t interleave2(uint32_t a, uint32_t b)
{
    uint64_t k = 0;
    for (int i = 0; i < 32; ++i) k |= (uint64_t)((a >> i) & 1u) << (2 * i) | (uint64_t)((b >> i) & 1u) << (2 * i + 1);
    return k;
}

__global__ void k_rank_keys(const int32_t *lo, const int32_t *hi, int nf, uint64_t *key, int32_t *val)
{
    const int f = blockIdx.x * kT + threadIdx.x;
    if (f >= nf) return;
    key[f] = hi[f] >= 0 ? interleave2((uint32_t)lo[f], (uint32_t)hi[f]) : UINT64_MAX;
    val[f] = f;
}

__global__ void k_inst_keys(const int32_t *fas_inst, const int32_t *order, int nf, uint32_t *key)
{
    const int r = blockIdx.x * kT + threadIdx.x;
    if (r < nf) key[r] = (uint32_t)fas_inst[order[r]];
}

__global__ void k_rank_scatter(const int32_t *order, int nf, int32_t *rank, int32_t *ext)
{
    const int r = blockIdx.x * kT + threadIdx.x;
    if (r >= nf) return;
    rank[order[r]] = r;
    ext[r] = order[r];
}

// ranks of the DSC-order nonzeros and the WC sort keys (rank, processing position)
__global__ void k_wc_keys(const int32_t *fas_o, const int32_t *rank, const int32_t *vox_v, const int32_t *proc_pos,
                          int64_t n, int bp, int32_t *fas_v, uint64_t *key, int32_t *val)
{
    const int64_t p = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (p >= n) return;
    const int32_t r = rank[fas_o[p]];
    fas_v[p] = r;
    const int32_t pp = proc_pos ? proc_pos[vox_v[p]] : vox_v[p];
    key[p] = (uint64_t)(uint32_t)r << bp | (uint64_t)(uint32_t)pp;
    val[p] = (int32_t)p;
}

// distinct (rank, chunk) pairs of the WC order: count per chunk, or flag each pair's first entry
__global__ void k_pair_count(const uint64_t *wkey, int64_t n, int bp, const int32_t *chunk_of_pos, int32_t *cnt,
                             int32_t *flag)
{
    const int64_t j = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (j >= n) return;
    const uint64_t mask = (uint64_t(1) << bp) - 1;
    const uint64_t k = wkey[j];
    const int32_t c = chunk_of_pos[(int64_t)(k & mask)];
    bool first = j == 0;
    if (!first) {
        const uint64_t kp = wkey[j - 1];
        first = (k >> bp) != (kp >> bp) || chunk_of_pos[(int64_t)(kp & mask)] != c;
    }
    if (cnt && first) atomicAdd(&cnt[c], 1);
    if (flag) flag[j] = first ? 1 : 0;
}

__global__ void k_tile_ptr(const int32_t *vox_ptr, const int16_t *atom_v, int nv, int T, int TA, int32_t *tile_ptr)
{
    const int v = blockIdx.x * kT + threadIdx.x;
    if (v >= nv) return;
    const int32_t b = vox_ptr[v], e = vox_ptr[v + 1];
    for (int t = 0; t < T; ++t) {
        int32_t lo = b, hi = e;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (atom_v[mid] < t * TA) lo = mid + 1;
            else hi = mid;
        }
        tile_ptr[(int64_t)v * (T + 1) + t] = lo;
    }
    tile_ptr[(int64_t)v * (T + 1) + T] = e;
}

// per (chunk, tile, wave) i: the slots' cumulative step counts and the padded length
__global__ void k_wave_counts(const int32_t *chunk_vox, const int32_t *tile_ptr, int64_t nitems, int T,
                              int32_t *wave_work, int64_t *len)
{
    const int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i >= nitems) return;
    const int64_t ct = i / kChunkWaves;
    const int w = (int)(i % kChunkWaves);
    const int64_t c = ct / T;
    const int t = (int)(ct % T);
    int steps = 0;
    for (int j = 0; j < kWaveVoxels; ++j) {
        const int v = chunk_vox[c * kChunkVoxels + w * kWaveVoxels + j];
        if (v >= 0) {
            const int32_t n = tile_ptr[(int64_t)v * (T + 1) + t + 1] - tile_ptr[(int64_t)v * (T + 1) + t];
            steps += (n + kStepEntries - 1) / kStepEntries;
        }
        wave_work[i * kWorkInts + 1 + j] = steps;
    }
    len[i] = (int64_t)kStepEntries * steps;
}

// first padded position of the range of item i, and of each (voxel, tile) sub-range
__global__ void k_wave_base(const int64_t *base, const int32_t *chunk_vox, int64_t nitems, int T, int32_t *wave_work,
                            int32_t *vt_base)
{
    const int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i >= nitems) return;
    const int64_t ct = i / kChunkWaves;
    const int w = (int)(i % kChunkWaves);
    const int64_t c = ct / T;
    const int t = (int)(ct % T);
    const int32_t b = (int32_t)base[i];
    wave_work[i * kWorkInts] = b;
    for (int j = 0; j < kWaveVoxels; ++j) {
        const int v = chunk_vox[c * kChunkVoxels + w * kWaveVoxels + j];
        if (v >= 0) vt_base[(int64_t)v * T + t] = b + kStepEntries * (j ? wave_work[i * kWorkInts + j] : 0);
    }
}

__global__ void k_fill_chunked(const int32_t *vox_v, const int16_t *atom_v, const int32_t *fas_v, const float *phi_v,
                               const int32_t *tile_ptr, const int32_t *vt_base, int64_t n, int T, int TA,
                               int16_t *atom_c, int32_t *fas_c, float *phi_c, int32_t *cpos)
{
    const int64_t p = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (p >= n) return;
    const int32_t v = vox_v[p];
    const int t = atom_v[p] / TA;
    const int32_t q = vt_base[(int64_t)v * T + t] + (int32_t)(p - tile_ptr[(int64_t)v * (T + 1) + t]);
    atom_c[q] = atom_v[p];
    fas_c[q] = fas_v[p];
    phi_c[q] = phi_v[p];
    cpos[p] = q;
}

// pads of each (voxel, tile) sub-range: value 0, the last real atom, rank and local index 0
__global__ void k_fill_pads(const int32_t *tile_ptr, const int32_t *vt_base, const int16_t *atom_v,
                            const int32_t *vox_chunk, int nv, int T, int16_t *atom_c, int32_t *fas_c, float *phi_c,
                            uint16_t *loc_c)
{
    const int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i >= (int64_t)nv * T) return;
    const int64_t v = i / T;
    const int t = (int)(i % T);
    if (vox_chunk[v] < 0) return;
    const int32_t b = tile_ptr[v * (T + 1) + t], e = tile_ptr[v * (T + 1) + t + 1], real = e - b;
    if (real == 0) return;
    const int32_t q0 = vt_base[v * T + t] + real;
    const int32_t pad = (real + kStepEntries - 1) / kStepEntries * kStepEntries - real;
    for (int32_t k = 0; k < pad; ++k) {
        atom_c[q0 + k] = atom_v[e - 1];
        fas_c[q0 + k] = 0;
        phi_c[q0 + k] = 0.f;
        loc_c[q0 + k] = 0;
    }
}

__global__ void k_pair_emit(const int32_t *flag, const int32_t *incl, const uint64_t *wkey, int64_t n, int bp,
                            const int32_t *chunk_of_pos, uint32_t *pair_chunk, int32_t *pair_rank, int32_t *iota)
{
    const int64_t j = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (j >= n || !flag[j]) return;
    const uint64_t mask = (uint64_t(1) << bp) - 1;
    const int32_t id = incl[j] - 1;
    pair_chunk[id] = (uint32_t)chunk_of_pos[(int64_t)(wkey[j] & mask)];
    pair_rank[id] = (int32_t)(wkey[j] >> bp);
    iota[id] = id;
}

__global__ void k_cfas(const int32_t *order, const int32_t *pair_rank, int64_t np, int32_t *cfas, int32_t *pos_of_pair)
{
    const int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i >= np) return;
    cfas[i] = pair_rank[order[i]];
    pos_of_pair[order[i]] = (int32_t)i;
}

__global__ void k_loc(const int32_t *incl, const int32_t *pos_of_pair, const uint64_t *wkey, const int32_t *wc_perm,
                      const int32_t *cpos, const int32_t *chunk_of_pos, const int32_t *cfas_ptr, int64_t n, int bp,
                      uint16_t *loc_c)
{
    const int64_t j = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (j >= n) return;
    const uint64_t mask = (uint64_t(1) << bp) - 1;
    const int32_t c = chunk_of_pos[(int64_t)(wkey[j] & mask)];
    loc_c[cpos[wc_perm[j]]] = (uint16_t)(pos_of_pair[incl[j] - 1] - cfas_ptr[c]);
}

__global__ void k_bucket_keys(const uint64_t *wkey, const int32_t *wc_perm, const int16_t *atom_v,
                              const int32_t *chunk_of_pos, int64_t n, int bp, int T, int TA, uint32_t *bkey,
                              int32_t *val)
{
    const int64_t j = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (j >= n) return;
    const uint64_t mask = (uint64_t(1) << bp) - 1;
    const int32_t c = chunk_of_pos[(int64_t)(wkey[j] & mask)];
    bkey[j] = (uint32_t)((int64_t)c * T + atom_v[wc_perm[j]] / TA);
    val[j] = (int32_t)j;
}

__global__ void k_wc_entries(const int32_t *border, const uint32_t *bkey, const int32_t *wc_perm, const uint64_t *wkey,
                             const int16_t *atom_v, const float *phi_v, const int32_t *vox_v, const int32_t *vox_slot,
                             int64_t n, int bp, int TA, uint16_t *wk, float *wphi, int32_t *erank, int32_t *flag)
{
    const int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (e >= n) return;
    const int32_t j = border[e], p = wc_perm[j];
    const int32_t r = (int32_t)(wkey[j] >> bp);
    const int a = atom_v[p], t = a / TA;
    erank[e] = r;
    bool start = e == 0 || bkey[e] != bkey[e - 1];
    if (!start) start = (int32_t)(wkey[border[e - 1]] >> bp) != r;
    wk[e] = (uint16_t)(((a - t * TA) << 6) | vox_slot[vox_v[p]] | (start ? kRunStart : 0));
    wphi[e] = phi_v[p];
    flag[e] = start ? 1 : 0;
}

__global__ void k_run_beg(const int32_t *flag, const int32_t *incl, int64_t n, int32_t *run_beg, int32_t *run_rank,
                          const int32_t *erank, int32_t *iota)
{
    const int64_t e = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (e >= n || !flag[e]) return;
    const int32_t r = incl[e] - 1;
    run_beg[r] = (int32_t)e;
    run_rank[r] = erank[e];
    iota[r] = r;
}

// wave w of bucket ct starts at the first run start e with (e - e0) 16 >= w n
__global__ void k_wave_ranges(const int32_t *wc_ent, const int32_t *run_beg, const int32_t *incl, int64_t nct,
                              int64_t n, int64_t n_runs, int32_t *wc_wave, int32_t *wc_wrun)
{
    const int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x;
    if (i >= nct * kChunkWaves) return;
    const int64_t ct = i / kChunkWaves;
    const int w = (int)(i % kChunkWaves);
    const int32_t e0 = wc_ent[ct], e1 = wc_ent[ct + 1];
    const int64_t nn = e1 - e0;
    const int32_t r0 = e0 < n ? incl[e0] - 1 : (int32_t)n_runs;   // e0, e1 start runs (bucket starts)
    const int32_t r1 = e1 < n ? incl[e1] - 1 : (int32_t)n_runs;
    int32_t lo = r0, hi = r1;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if ((int64_t)(run_beg[mid] - e0) * kChunkWaves >= (int64_t)w * nn) hi = mid;
        else lo = mid + 1;
    }
    wc_wave[i] = lo < r1 ? run_beg[lo] : e1;
    wc_wrun[i] = lo;
}

// ------------------------------------------------------------------------------ helpers

struct Sorter {
    Arena &ar;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    hipError_t err = hipSuccess;
    template <class K>
    void pairs(const K *kin, K *kout, const int32_t *vin, int32_t *vout, int64_t n, int end_bit)
    {
        if (err != hipSuccess || n == 0) return;
        size_t need = 0;
        err = hipcub::DeviceRadixSort::SortPairs(nullptr, need, kin, kout, vin, vout, (int)n, 0, end_bit, nullptr);
        if (err != hipSuccess) return;
        if (need > tmp_bytes) {
            tmp = ar.get<char>((int64_t)need);
            if (!tmp) { err = ar.err; return; }
            tmp_bytes = need;
        }
        err = hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, vin, vout, (int)n, 0, end_bit, nullptr);
    }
    // inclusive prefix sum of int32 flags
    void incl_sum(const int32_t *in, int32_t *out, int64_t n)
    {
        if (err != hipSuccess || n == 0) return;
        size_t need = 0;
        err = hipcub::DeviceScan::InclusiveSum(nullptr, need, in, out, (int)n, nullptr);
        if (err != hipSuccess) return;
        if (need > tmp_bytes) {
            tmp = ar.get<char>((int64_t)need);
            if (!tmp) { err = ar.err; return; }
            tmp_bytes = need;
        }
        err = hipcub::DeviceScan::InclusiveSum(tmp, tmp_bytes, in, out, (int)n, nullptr);
    }
    void excl_sum64(const int64_t *in, int64_t *out, int64_t n)
    {
        if (err != hipSuccess || n == 0) return;
        size_t need = 0;
        err = hipcub::DeviceScan::ExclusiveSum(nullptr, need, in, out, (int)n, nullptr);
        if (err != hipSuccess) return;
        if (need > tmp_bytes) {
            tmp = ar.get<char>((int64_t)need);
            if (!tmp) { err = ar.err; return; }
            tmp_bytes = need;
        }
        err = hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, in, out, (int)n, nullptr);
    }
};

template <class T>
hipError_t down(std::vector<T> &dst, const T *src, int64_t n)
{
    dst.resize((size_t)std::max<int64_t>(n, 0));
    return n > 0 ? hipMemcpy(dst.data(), src, sizeof(T) * (size_t)n, hipMemcpyDeviceToHost) : hipSuccess;
}

template <class T>
hipError_t up(T *dst, const std::vector<T> &src)
{
    return src.empty() ? hipSuccess : hipMemcpy(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

}  // namespace

void free_dev_layout(DevLayout *L)
{
    void *ptrs[] = {L->vox_ptr, L->fas_v, L->fas_rank, L->fas_ext, L->fas_ptr, L->wc_perm, L->vox_dsc, L->atom_v,
                    L->phi_v, L->chunk_vox, L->wave_work, L->fas_c, L->cfas_ptr, L->cfas, L->wc_wave, L->wc_wrun,
                    L->rr_ptr, L->rr, L->atom_c, L->loc_c, L->wkey, L->phi_c, L->wphi};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    *L = DevLayout();
}

life_status plan_gpu(const life_dims *d, const TileGeom &tg, const int16_t *atom, const int32_t *voxel,
                     const int32_t *fascicle, const float *phi, const int32_t *proc_pos_h, const int32_t *proc_vox,
                     int32_t n_pos, const int32_t *fas_inst_h, const int32_t *vox_off_h, int n_inst, DevLayout *out)
{
    // built in L, handed to *out only on success: the arena frees L's arrays on
    // every other return
    *out = DevLayout();
    DevLayout L;
    const int64_t n = d->nnz;
    const int nv = d->n_voxels, nf = d->n_fascicles, T = tg.n_tiles, TA = tg.tile_atoms;
    Arena ar;
    Sorter so{ar};
    hipError_t e = hipSuccess;
    auto ok = [&]() { return e == hipSuccess && ar.err == hipSuccess && so.err == hipSuccess; };
    auto fail = [&]() -> life_status {
        const hipError_t x = e != hipSuccess ? e : ar.err != hipSuccess ? ar.err : so.err;
        return x == hipErrorOutOfMemory ? LIFE_ENOMEM : LIFE_EDEVICE;
    };
    // small host inputs on the device
    int32_t *proc_pos = nullptr, *fas_inst = nullptr, *vox_off = nullptr;
    if (proc_pos_h) {
        proc_pos = ar.get<int32_t>(nv);
        if (ok() && nv) e = hipMemcpy(proc_pos, proc_pos_h, sizeof(int32_t) * nv, hipMemcpyHostToDevice);
    }
    if (fas_inst_h) {
        fas_inst = ar.get<int32_t>(nf);
        vox_off = ar.get<int32_t>(n_inst + 1);
        if (ok() && nf) e = hipMemcpy(fas_inst, fas_inst_h, sizeof(int32_t) * nf, hipMemcpyHostToDevice);
        if (ok()) e = hipMemcpy(vox_off, vox_off_h, sizeof(int32_t) * (n_inst + 1), hipMemcpyHostToDevice);
    }
    if (!ok()) return fail();
    // index checks
    {
        int *bad = ar.get<int>(1);
        if (!ok()) return fail();
        e = hipMemset(bad, 0, sizeof(int));
        if (ok() && n) k_validate<<<blocks(n), kT>>>(atom, voxel, fascicle, n, d->n_atoms, nv, nf, fas_inst, vox_off, bad);
        int hbad = 0;
        if (ok()) e = hipMemcpy(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost);
        if (!ok()) return fail();
        if (hbad) return LIFE_ERANGE;
    }
    // DSC order: stable sort by (voxel, atom, fascicle); ties keep the input order
    const int bf = bits_for(nf), bvox = bits_for(nv);
    int32_t *perm = ar.get<int32_t>(n), *vtmp = ar.get<int32_t>(n);
    uint64_t *k64a = ar.get<uint64_t>(n), *k64b = ar.get<uint64_t>(n);
    if (!ok()) return fail();
    if (n) {
        if (bvox + 15 + bf <= 64) {
            k_dsc_keys<<<blocks(n), kT>>>(atom, voxel, fascicle, n, bf, true, k64a, vtmp);
            so.pairs(k64a, k64b, vtmp, perm, n, bvox + 15 + bf);
        } else {
            uint32_t *k32a = ar.get<uint32_t>(n), *k32b = ar.get<uint32_t>(n);
            int32_t *p1 = ar.get<int32_t>(n);
            if (!ok()) return fail();
            k_fas_keys32<<<blocks(n), kT>>>(fascicle, n, k32a, vtmp);
            so.pairs(k32a, k32b, vtmp, p1, n, bf);
            k_dsc_keys_perm<<<blocks(n), kT>>>(atom, voxel, p1, n, k64a);
            so.pairs(k64a, k64b, p1, perm, n, bvox + 15);
        }
    }
    L.atom_v = ar.get<int16_t>(n);
    L.vox_dsc = ar.get<int32_t>(n);
    L.phi_v = ar.get<float>(n);
    int32_t *fas_o = ar.get<int32_t>(n);
    L.vox_ptr = ar.get<int32_t>((int64_t)nv + 1);
    if (!ok()) return fail();
    if (n) k_gather_dsc<<<blocks(n), kT>>>(perm, atom, voxel, fascicle, phi, n, L.atom_v, L.vox_dsc, fas_o, L.phi_v);
    k_seg_ptr<int32_t><<<blocks((int64_t)nv + 1), kT>>>(L.vox_dsc, n, nv, 0, L.vox_ptr);
    // fascicle ranks: Z-order of the first and last processing positions (ties by
    // index, fascicles without nonzeros last), the instance as the major key
    L.fas_rank = ar.get<int32_t>(nf);
    L.fas_ext = ar.get<int32_t>(nf);
    {
        int32_t *lo = ar.get<int32_t>(nf), *hi = ar.get<int32_t>(nf), *fv = ar.get<int32_t>(nf),
                *ord = ar.get<int32_t>(nf);
        uint64_t *rk = ar.get<uint64_t>(nf), *rk2 = ar.get<uint64_t>(nf);
        if (!ok()) return fail();
        if (nf) {
            k_fill_i32<<<blocks(nf), kT>>>(lo, nf, INT32_MAX);
            k_fill_i32<<<blocks(nf), kT>>>(hi, nf, -1);
            if (n) k_lohi<<<blocks(n), kT>>>(voxel, fascicle, proc_pos, n, lo, hi);
            k_rank_keys<<<blocks(nf), kT>>>(lo, hi, nf, rk, fv);
            so.pairs(rk, rk2, fv, ord, nf, 64);
            if (fas_inst) {
                uint32_t *ik = ar.get<uint32_t>(nf), *ik2 = ar.get<uint32_t>(nf);
                int32_t *ord2 = ar.get<int32_t>(nf);
                if (!ok()) return fail();
                k_inst_keys<<<blocks(nf), kT>>>(fas_inst, ord, nf, ik);
                so.pairs(ik, ik2, ord, ord2, nf, bits_for(n_inst));
                ord = ord2;
            }
            k_rank_scatter<<<blocks(nf), kT>>>(ord, nf, L.fas_rank, L.fas_ext);
        }
    }
    // WC order: stable sort of the DSC positions by (rank, voxel position)
    const int bp = bits_for(std::max<int64_t>(n_pos, nv));
    L.fas_v = ar.get<int32_t>(n);
    L.wc_perm = ar.get<int32_t>(n);
    L.fas_ptr = ar.get<int32_t>((int64_t)nf + 1);
    if (!ok()) return fail();
    uint64_t *wkey = k64a;   // sorted WC keys
    if (n) {
        k_wc_keys<<<blocks(n), kT>>>(fas_o, L.fas_rank, L.vox_dsc, proc_pos, n, bp, L.fas_v, k64b, vtmp);
        so.pairs(k64b, k64a, vtmp, L.wc_perm, n, bf + bp);
    }
    k_seg_ptr<uint64_t><<<blocks((int64_t)nf + 1), kT>>>(wkey, n, nf, bp, L.fas_ptr);
    if (!ok()) return fail();
    if (tg.row_floats == 0) {   // generic kernels: the canonical orders only
        L.n_chunks = 0;
        e = hipDeviceSynchronize();
        if (!ok()) return fail();
        for (void **p : {(void **)&L.vox_ptr, (void **)&L.fas_v, (void **)&L.fas_rank, (void **)&L.fas_ext,
                         (void **)&L.fas_ptr, (void **)&L.wc_perm, (void **)&L.vox_dsc, (void **)&L.atom_v,
                         (void **)&L.phi_v})
            ar.keep(*p);
        *out = L;
        return LIFE_OK;
    }

    // ---- chunks: groups of kChunkVoxels positions, halved while they cross more than
    // tg.fas_cap distinct fascicles (counted as distinct (rank, chunk) pairs of the
    // WC order, where they are adjacent)
    std::vector<int32_t> bounds;
    for (int32_t g0 = 0; g0 < n_pos; g0 += kChunkVoxels) bounds.push_back(g0);
    bounds.push_back(n_pos);
    std::vector<int32_t> chunk_of_pos_h((size_t)std::max(n_pos, 1));
    int32_t *chunk_of_pos = ar.get<int32_t>(std::max(n_pos, 1));
    int32_t *cnt = nullptr;
    std::vector<int32_t> cnt_h;
    L.fas_overflow = false;
    for (;;) {
        const int nc = (int)bounds.size() - 1;
        for (int c = 0; c < nc; ++c)
            for (int32_t k = bounds[c]; k < bounds[c + 1]; ++k) chunk_of_pos_h[(size_t)k] = c;
        cnt = ar.get<int32_t>(std::max(nc, 1));
        if (!ok()) return fail();
        e = up(chunk_of_pos, chunk_of_pos_h);
        if (ok()) e = hipMemset(cnt, 0, sizeof(int32_t) * std::max(nc, 1));
        if (ok() && n) k_pair_count<<<blocks(n), kT>>>(wkey, n, bp, chunk_of_pos, cnt, nullptr);
        if (ok()) e = down(cnt_h, cnt, nc);
        if (!ok()) return fail();
        std::vector<int32_t> nb;
        bool split = false;
        for (int c = 0; c < nc; ++c) {
            nb.push_back(bounds[c]);
            if (cnt_h[(size_t)c] > tg.fas_cap) {
                if (bounds[c + 1] - bounds[c] > 1) {
                    nb.push_back(bounds[c] + (bounds[c + 1] - bounds[c]) / 2);
                    split = true;
                } else {
                    L.fas_overflow = true;
                }
            }
        }
        nb.push_back(bounds[(size_t)nc]);
        if (L.fas_overflow) {   // the caller falls back to the generic kernels
            e = hipDeviceSynchronize();
            if (!ok()) return fail();
            out->fas_overflow = true;
            return LIFE_OK;
        }
        if (!split) break;
        bounds.swap(nb);
    }
    const int nc = (int)bounds.size() - 1;
    L.n_chunks = nc;
    L.bounds = bounds;
    // voxel slots (host; O(voxels))
    std::vector<int32_t> vox_ptr_h, chunk_vox_h, vox_chunk_h, vox_slot_h;
    e = down(vox_ptr_h, L.vox_ptr, (int64_t)nv + 1);
    if (!ok()) return fail();
    chunk_slots(d, vox_ptr_h.data(), proc_vox, bounds, chunk_vox_h, vox_chunk_h, vox_slot_h);
    L.chunk_vox = ar.get<int32_t>((int64_t)nc * kChunkVoxels);
    int32_t *vox_chunk = ar.get<int32_t>(nv), *vox_slot = ar.get<int32_t>(nv);
    int32_t *tile_ptr = ar.get<int32_t>((int64_t)nv * (T + 1));
    int32_t *vt_base = ar.get<int32_t>((int64_t)nv * T);
    const int64_t nitems = (int64_t)nc * T * kChunkWaves;
    L.wave_work = ar.get<int32_t>(nitems * kWorkInts);
    int64_t *len = ar.get<int64_t>(nitems), *base = ar.get<int64_t>(nitems);
    if (!ok()) return fail();
    e = up(L.chunk_vox, chunk_vox_h);
    if (ok()) e = up(vox_chunk, vox_chunk_h);
    if (ok()) e = up(vox_slot, vox_slot_h);
    if (!ok()) return fail();
    if (nv) k_tile_ptr<<<blocks(nv), kT>>>(L.vox_ptr, L.atom_v, nv, T, TA, tile_ptr);
    if (nitems) k_wave_counts<<<blocks(nitems), kT>>>(L.chunk_vox, tile_ptr, nitems, T, L.wave_work, len);
    so.excl_sum64(len, base, nitems);
    if (nitems) k_wave_base<<<blocks(nitems), kT>>>(base, L.chunk_vox, nitems, T, L.wave_work, vt_base);
    std::vector<int64_t> base_h, len_h;
    if (ok()) e = down(base_h, base, nitems);
    if (ok()) e = down(len_h, len, nitems);
    if (!ok()) return fail();
    L.n_pad = nitems ? base_h.back() + len_h.back() : 0;
    if (L.n_pad > kMaxNnz) return LIFE_ERANGE;
    L.work.assign((size_t)nc, 0);
    for (int c = 0; c < nc; ++c) {
        const int64_t b0 = base_h[(size_t)c * T * kChunkWaves];
        const int64_t b1 = c + 1 < nc ? base_h[(size_t)(c + 1) * T * kChunkWaves] : L.n_pad;
        L.work[(size_t)c] = b1 - b0;
    }
    // padded copies
    L.atom_c = ar.get<int16_t>(L.n_pad);
    L.fas_c = ar.get<int32_t>(L.n_pad);
    L.loc_c = ar.get<uint16_t>(L.n_pad);
    L.phi_c = ar.get<float>(L.n_pad);
    int32_t *cpos = ar.get<int32_t>(n);
    if (!ok()) return fail();
    if (n) k_fill_chunked<<<blocks(n), kT>>>(L.vox_dsc, L.atom_v, L.fas_v, L.phi_v, tile_ptr, vt_base, n, T, TA,
                                             L.atom_c, L.fas_c, L.phi_c, cpos);
    if ((int64_t)nv * T) k_fill_pads<<<blocks((int64_t)nv * T), kT>>>(tile_ptr, vt_base, L.atom_v, vox_chunk, nv, T,
                                                                       L.atom_c, L.fas_c, L.phi_c, L.loc_c);
    // chunk fascicle lists: the distinct (rank, chunk) pairs of the WC order, stably
    // grouped by chunk (ranks ascend inside a chunk); local index of every nonzero
    int32_t *flag = ar.get<int32_t>(n), *incl = ar.get<int32_t>(n);
    if (!ok()) return fail();
    if (n) k_pair_count<<<blocks(n), kT>>>(wkey, n, bp, chunk_of_pos, nullptr, flag);
    so.incl_sum(flag, incl, n);
    int32_t np = 0;
    if (ok() && n) e = hipMemcpy(&np, incl + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (!ok()) return fail();
    uint32_t *pck = ar.get<uint32_t>(np), *pck2 = ar.get<uint32_t>(np);
    int32_t *prank = ar.get<int32_t>(np), *piota = ar.get<int32_t>(np), *pord = ar.get<int32_t>(np),
            *ppos = ar.get<int32_t>(np);
    L.cfas = ar.get<int32_t>(np);
    L.cfas_ptr = ar.get<int32_t>((int64_t)nc + 1);
    if (!ok()) return fail();
    if (n) k_pair_emit<<<blocks(n), kT>>>(flag, incl, wkey, n, bp, chunk_of_pos, pck, prank, piota);
    so.pairs(pck, pck2, piota, pord, np, bits_for(nc));
    if (np) k_cfas<<<blocks(np), kT>>>(pord, prank, np, L.cfas, ppos);
    k_seg_ptr<uint32_t><<<blocks((int64_t)nc + 1), kT>>>(pck2, np, nc, 0, L.cfas_ptr);
    if (n) k_loc<<<blocks(n), kT>>>(incl, ppos, wkey, L.wc_perm, cpos, chunk_of_pos, L.cfas_ptr, n, bp, L.loc_c);
    std::vector<int32_t> cfas_ptr_h;
    if (ok()) e = down(cfas_ptr_h, L.cfas_ptr, (int64_t)nc + 1);
    if (!ok()) return fail();
    L.max_fas = 0;
    for (int c = 0; c < nc; ++c) L.max_fas = std::max(L.max_fas, cfas_ptr_h[(size_t)c + 1] - cfas_ptr_h[(size_t)c]);
    // WC pass 1: the WC order bucketed stably by (chunk, tile), runs of one fascicle
    const int64_t nct = (int64_t)nc * T;
    uint32_t *bk = ar.get<uint32_t>(n), *bk2 = ar.get<uint32_t>(n);
    int32_t *border = ar.get<int32_t>(n), *erank = ar.get<int32_t>(n);
    int32_t *wc_ent = ar.get<int32_t>(nct + 1);
    L.wkey = ar.get<uint16_t>(n);
    L.wphi = ar.get<float>(n);
    if (!ok()) return fail();
    if (n) {
        k_bucket_keys<<<blocks(n), kT>>>(wkey, L.wc_perm, L.atom_v, chunk_of_pos, n, bp, T, TA, bk, vtmp);
        so.pairs(bk, bk2, vtmp, border, n, bits_for(nct));
        k_wc_entries<<<blocks(n), kT>>>(border, bk2, L.wc_perm, wkey, L.atom_v, L.phi_v, L.vox_dsc, vox_slot, n, bp,
                                        TA, L.wkey, L.wphi, erank, flag);
    }
    k_seg_ptr<uint32_t><<<blocks(nct + 1), kT>>>(bk2, n, nct, 0, wc_ent);
    so.incl_sum(flag, incl, n);
    int32_t nr = 0;
    if (ok() && n) e = hipMemcpy(&nr, incl + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (!ok()) return fail();
    L.n_runs = nr;
    int32_t *run_beg = ar.get<int32_t>((int64_t)nr + 1), *run_rank = ar.get<int32_t>(nr),
            *riota = ar.get<int32_t>(nr);
    L.wc_wave = ar.get<int32_t>(nct * kChunkWaves + 1);
    L.wc_wrun = ar.get<int32_t>(nct * kChunkWaves);
    if (!ok()) return fail();
    if (n) k_run_beg<<<blocks(n), kT>>>(flag, incl, n, run_beg, run_rank, erank, riota);
    {
        const int32_t nn = (int32_t)n;
        e = hipMemcpy(run_beg + nr, &nn, sizeof(int32_t), hipMemcpyHostToDevice);
        if (ok()) e = hipMemcpy(L.wc_wave + nct * kChunkWaves, &nn, sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (nct) k_wave_ranges<<<blocks(nct * kChunkWaves), kT>>>(wc_ent, run_beg, incl, nct, n, nr, L.wc_wave, L.wc_wrun);
    // WC pass 2: each rank's runs in run order
    uint32_t *rrk = ar.get<uint32_t>(nr), *rrk2 = ar.get<uint32_t>(nr);
    L.rr = ar.get<int32_t>(nr);
    L.rr_ptr = ar.get<int32_t>((int64_t)nf + 1);
    if (!ok()) return fail();
    if (nr) {
        e = hipMemcpy(rrk, run_rank, sizeof(int32_t) * nr, hipMemcpyDeviceToDevice);
        so.pairs(rrk, rrk2, riota, L.rr, nr, bf);
    }
    k_seg_ptr<uint32_t><<<blocks((int64_t)nf + 1), kT>>>(rrk2, nr, nf, 0, L.rr_ptr);
    if (ok()) e = hipGetLastError();
    if (ok()) e = hipDeviceSynchronize();
    if (!ok()) return fail();
    for (void **p : {(void **)&L.vox_ptr, (void **)&L.fas_v, (void **)&L.fas_rank, (void **)&L.fas_ext,
                     (void **)&L.fas_ptr, (void **)&L.wc_perm, (void **)&L.vox_dsc, (void **)&L.atom_v,
                     (void **)&L.phi_v, (void **)&L.chunk_vox, (void **)&L.wave_work, (void **)&L.fas_c,
                     (void **)&L.cfas_ptr, (void **)&L.cfas, (void **)&L.wc_wave, (void **)&L.wc_wrun,
                     (void **)&L.rr_ptr, (void **)&L.rr, (void **)&L.atom_c, (void **)&L.loc_c, (void **)&L.wkey,
                     (void **)&L.phi_c, (void **)&L.wphi})
        ar.keep(*p);
    *out = L;
    return LIFE_OK;
}

}  // namespace life
