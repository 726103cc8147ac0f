// Host-side data restructuring for the LiFE sparse-Tucker products.
//
// The paper restructures the Phi tensor once, before SBB-NNLS, by sorting its
// nonzeros on one of the index vectors (Sec. 4.1, "Data Restructuring"): by
// voxel, so that every voxel's nonzeros form one contiguous "sub-vector"
// (Sec. 4, sub-vectors of a sorted indirection vector), and - the variant the
// paper sets aside and this library uses for WC because it needs no atomics -
// by fiber (fascicle).  Both orders here are total orders, so a plan is unique:
//   DSC order: (voxel, atom, fascicle, input position)
//   WC order : (fascicle rank, voxel position, atom, fascicle, input position)
// where the voxel position is the voxel's place in the processing order (id
// order, or Morton order of its grid coordinates when they are given) and the
// fascicle rank orders fascicles by the Z-order of the (first, last) positions of
// their voxels.  They are built with stable LSD counting sorts, O(nnz + N) per key.
//
// Pure C++17: no HIP, so it can be checked on the host alone.
#include "life_internal.h"

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

namespace life {

life_status validate_dims(const life_dims *d)
{
    if (!d) return LIFE_EINVAL;
    if (d->n_theta < 1 || d->n_theta > kMaxTheta) return LIFE_EINVAL;
    if (d->n_atoms < 1 || d->n_atoms > 32767) return LIFE_EINVAL;
    if (d->n_voxels < 0 || d->n_fascicles < 0 || d->nnz < 0) return LIFE_EINVAL;
    if (d->nnz > kMaxNnz) return LIFE_ERANGE;
    return LIFE_OK;
}

life_status validate_indices(const life_dims *d, const int16_t *atom, const int32_t *voxel,
                             const int32_t *fascicle)
{
    const int64_t n = d->nnz;
    if (n > 0 && (!atom || !voxel || !fascicle)) return LIFE_EINVAL;
    const int32_t na = d->n_atoms, nv = d->n_voxels, nf = d->n_fascicles;
    int bad = 0;
    for (int64_t c = 0; c < n; ++c) {
        bad |= (atom[c] < 0) | (atom[c] >= na);
        bad |= (voxel[c] < 0) | (voxel[c] >= nv);
        bad |= (fascicle[c] < 0) | (fascicle[c] >= nf);
    }
    return bad ? LIFE_ERANGE : LIFE_OK;
}

life_status validate_coords(const life_dims *d, const int16_t *voxel_xyz)
{
    if (!voxel_xyz) return LIFE_OK;
    for (int64_t i = 0; i < 3 * (int64_t)d->n_voxels; ++i)
        if (voxel_xyz[i] < 0) return LIFE_ERANGE;
    return LIFE_OK;
}

namespace {

// Stable counting sort of the items in `in` by key(item) in [0, nkeys).
template <class Key>
void counting_sort(const int32_t *in, int32_t *out, int64_t n, int64_t nkeys, Key key,
                   std::vector<int64_t> &cnt)
{
    cnt.assign(static_cast<size_t>(nkeys) + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++cnt[static_cast<size_t>(key(in[i])) + 1];
    for (int64_t k = 0; k < nkeys; ++k) cnt[k + 1] += cnt[k];
    for (int64_t i = 0; i < n; ++i) out[cnt[static_cast<size_t>(key(in[i]))]++] = in[i];
}

void segment_offsets(const int32_t *keys_in_order, int64_t n, int32_t nkeys, int32_t *ptr)
{
    // keys_in_order is sorted ascending; ptr[k] = first position with key >= k
    int64_t pos = 0;
    for (int32_t k = 0; k <= nkeys; ++k) {
        while (pos < n && keys_in_order[pos] < k) ++pos;
        ptr[k] = static_cast<int32_t>(pos);
    }
}

// Morton (Z-order) key: bit b of x, y, z goes to bit 3b, 3b+1, 3b+2.
uint64_t morton_key(const int16_t *c)
{
    uint64_t key = 0;
    for (int b = 0; b < 16; ++b)
        for (int axis = 0; axis < 3; ++axis)
            key |= (uint64_t)(((uint16_t)c[axis] >> b) & 1u) << (3 * b + axis);
    return key;
}

// Bits of a and b interleaved (bit i of a -> bit 2i, bit i of b -> bit 2i+1).
uint64_t interleave2(uint32_t a, uint32_t b)
{
    uint64_t k = 0;
    for (int i = 0; i < 32; ++i)
        k |= (uint64_t)((a >> i) & 1u) << (2 * i) | (uint64_t)((b >> i) & 1u) << (2 * i + 1);
    return k;
}

// Fascicle rank: fascicles in Z-order of (lo, hi), the first and last processing
// positions of the voxels they cross (ties by index).  A chunk of voxels gathers
// the weights of the fascicles crossing it; fascicles with nearby (lo, hi) cross
// mostly the same chunks, so this order puts them in the same cache lines of w
// (on the full synthetic connectome it halves the distinct (chunk, 128-byte line)
// pairs against ordering by the mean position).  Fascicles without nonzeros rank
// last.  With fas_inst (batched plans) the instance of each fascicle is the major
// key, so every instance's fascicles take one contiguous block of ranks (its
// empty fascicles at the end of the block).
void fascicle_ranks(const life_dims *d, const int32_t *voxel, const int32_t *fascicle, const int32_t *proc_pos,
                    const int32_t *fas_inst, int32_t *rank)
{
    const int32_t nf = d->n_fascicles;
    std::vector<int32_t> lo(static_cast<size_t>(nf), INT32_MAX), hi(static_cast<size_t>(nf), -1);
    for (int64_t c = 0; c < d->nnz; ++c) {
        const int32_t p = proc_pos ? proc_pos[voxel[c]] : voxel[c];
        lo[fascicle[c]] = std::min(lo[fascicle[c]], p);
        hi[fascicle[c]] = std::max(hi[fascicle[c]], p);
    }
    std::vector<uint64_t> key(static_cast<size_t>(nf));
    for (int32_t f = 0; f < nf; ++f)
        key[f] = hi[f] >= 0 ? interleave2(static_cast<uint32_t>(lo[f]), static_cast<uint32_t>(hi[f])) : UINT64_MAX;
    std::vector<int32_t> order(static_cast<size_t>(nf));
    for (int32_t f = 0; f < nf; ++f) order[f] = f;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const int32_t ia = fas_inst ? fas_inst[a] : 0, ib = fas_inst ? fas_inst[b] : 0;
        return ia != ib ? ia < ib : key[a] < key[b];
    });
    for (int32_t r = 0; r < nf; ++r) rank[order[r]] = r;
}

}  // namespace

life_status validate_instances(const life_dims *d, int n_inst, const int32_t *vox_off, const int32_t *fas_off,
                               const int32_t *voxel, const int32_t *fascicle)
{
    if (n_inst < 1 || !vox_off || !fas_off) return LIFE_EINVAL;
    if (vox_off[0] != 0 || fas_off[0] != 0 || vox_off[n_inst] != d->n_voxels || fas_off[n_inst] != d->n_fascicles)
        return LIFE_EINVAL;
    for (int k = 0; k < n_inst; ++k)
        if (vox_off[k + 1] < vox_off[k] || fas_off[k + 1] < fas_off[k]) return LIFE_EINVAL;
    // every nonzero's voxel and fascicle lie in one instance (block-diagonal M)
    std::vector<int32_t> fas_inst(static_cast<size_t>(d->n_fascicles));
    for (int k = 0; k < n_inst; ++k)
        for (int32_t f = fas_off[k]; f < fas_off[k + 1]; ++f) fas_inst[f] = k;
    for (int64_t c = 0; c < d->nnz; ++c) {
        const int k = fas_inst[fascicle[c]];
        if (voxel[c] < vox_off[k] || voxel[c] >= vox_off[k + 1]) return LIFE_ERANGE;
    }
    return LIFE_OK;
}

int32_t padded_positions(const life_dims *d, int n_inst, const int32_t *vox_off)
{
    if (n_inst <= 1) return d->n_voxels;
    int64_t n = 0;
    for (int k = 0; k < n_inst; ++k) n += (vox_off[k + 1] - vox_off[k] + kChunkVoxels - 1) / kChunkVoxels * kChunkVoxels;
    return n > kMaxNnz ? -1 : static_cast<int32_t>(n);
}

void voxel_order(const life_dims *d, const int16_t *voxel_xyz, int n_inst, const int32_t *vox_off,
                 int32_t *proc_pos, int32_t *proc_vox)
{
    const int32_t nv = d->n_voxels;
    const int32_t one[2] = {0, nv};
    if (n_inst <= 1) vox_off = one;
    const int ni = n_inst <= 1 ? 1 : n_inst;
    int32_t base = 0;
    std::vector<int32_t> order;
    std::vector<uint64_t> key;
    for (int k = 0; k < ni; ++k) {
        const int32_t v0 = vox_off[k], v1 = vox_off[k + 1], n = v1 - v0;
        order.resize(static_cast<size_t>(n));
        for (int32_t i = 0; i < n; ++i) order[i] = v0 + i;
        if (voxel_xyz) {
            key.resize(static_cast<size_t>(n));
            for (int32_t i = 0; i < n; ++i) key[i] = morton_key(voxel_xyz + 3 * (int64_t)(v0 + i));
            std::stable_sort(order.begin(), order.end(),
                             [&](int32_t a, int32_t b) { return key[a - v0] < key[b - v0]; });
        }
        const int32_t span = ni == 1 ? n : (n + kChunkVoxels - 1) / kChunkVoxels * kChunkVoxels;
        for (int32_t i = 0; i < span; ++i) {
            if (proc_vox) proc_vox[base + i] = i < n ? order[i] : -1;
            if (proc_pos && i < n) proc_pos[order[i]] = base + i;
        }
        base += span;
    }
}

life_status plan_host(const life_dims *d, const int16_t *atom, const int32_t *voxel, const int32_t *fascicle,
                      const int32_t *proc_pos, int32_t n_pos, const int32_t *fas_inst, int32_t *dsc_perm,
                      int32_t *vox_ptr, int32_t *fas_rank, int32_t *wc_perm, int32_t *fas_ptr)
{
    life_status st = validate_dims(d);
    if (st != LIFE_OK) return st;
    st = validate_indices(d, atom, voxel, fascicle);
    if (st != LIFE_OK) return st;
    const int64_t n = d->nnz;
    try {
        std::vector<int32_t> a(static_cast<size_t>(n)), b(static_cast<size_t>(n));
        std::vector<int64_t> cnt;
        for (int64_t i = 0; i < n; ++i) a[i] = static_cast<int32_t>(i);
        // LSD: least significant key first; ties keep input order.
        counting_sort(a.data(), b.data(), n, d->n_fascicles, [&](int32_t i) { return fascicle[i]; }, cnt);
        counting_sort(b.data(), a.data(), n, d->n_atoms, [&](int32_t i) { return atom[i]; }, cnt);
        counting_sort(a.data(), b.data(), n, d->n_voxels, [&](int32_t i) { return voxel[i]; }, cnt);
        // b = DSC order (voxel, atom, fascicle, input position)
        if (vox_ptr) {
            std::vector<int32_t> keys(static_cast<size_t>(n));
            for (int64_t p = 0; p < n; ++p) keys[p] = voxel[b[p]];
            segment_offsets(keys.data(), n, d->n_voxels, vox_ptr);
        }
        std::vector<int32_t> rank(static_cast<size_t>(d->n_fascicles));
        fascicle_ranks(d, voxel, fascicle, proc_pos, fas_inst, rank.data());
        if (fas_rank && d->n_fascicles)
            std::memcpy(fas_rank, rank.data(), sizeof(int32_t) * static_cast<size_t>(d->n_fascicles));
        if (wc_perm || fas_ptr) {
            // Stable sorts of DSC positions: by voxel position (a no-op in id order),
            // then by fascicle rank; the DSC order supplies (atom, fascicle, position).
            std::vector<int32_t> w(static_cast<size_t>(n));
            for (int64_t p = 0; p < n; ++p) a[p] = static_cast<int32_t>(p);
            if (proc_pos) {
                counting_sort(a.data(), w.data(), n, std::max(n_pos, d->n_voxels),
                              [&](int32_t p) { return proc_pos[voxel[b[p]]]; }, cnt);
                std::swap(a, w);
            }
            counting_sort(a.data(), w.data(), n, d->n_fascicles, [&](int32_t p) { return rank[fascicle[b[p]]]; },
                          cnt);
            if (fas_ptr) {
                std::vector<int32_t> keys(static_cast<size_t>(n));
                for (int64_t j = 0; j < n; ++j) keys[j] = rank[fascicle[b[w[j]]]];
                segment_offsets(keys.data(), n, d->n_fascicles, fas_ptr);
            }
            if (wc_perm && n) std::memcpy(wc_perm, w.data(), sizeof(int32_t) * static_cast<size_t>(n));
        }
        if (dsc_perm && n) std::memcpy(dsc_perm, b.data(), sizeof(int32_t) * static_cast<size_t>(n));
    } catch (const std::bad_alloc &) {
        return LIFE_ENOMEM;
    }
    return LIFE_OK;
}

TileGeom tile_geometry(int n_theta, int n_atoms, int tile_atoms)
{
    TileGeom g;
    const int row = ((n_theta + 31) / 32) * 32;
    if (row > kMaxTileRowFloats) return g;
    const int max_atoms = std::min(tile_atoms > 0 ? tile_atoms : kTileBytes / (row * 4), kMaxTileAtoms);
    const int n_tiles = (n_atoms + max_atoms - 1) / max_atoms;
    const int ta = (n_atoms + n_tiles - 1) / n_tiles;   // balanced tiles
    // the LDS left beside one tile holds the chunk's weights (at least 1024 of them)
    const int cap = std::min(kChunkFasCap, (kLdsBudget - ta * row * 4) / 4);
    if (cap < 1024) return g;
    g.row_floats = row;
    g.n_tiles = n_tiles;
    g.tile_atoms = ta;
    g.fas_cap = cap;
    return g;
}

namespace {

// Distinct fascicle ranks of the nonzeros of processing positions [pb, pe);
// stamp[rank] == tag marks a rank already counted (tags never repeat).
int distinct_fascicles(const int32_t *vox_ptr, const int32_t *fas_v, const int32_t *proc_vox, int32_t pb, int32_t pe,
                       std::vector<int64_t> &stamp, int64_t tag)
{
    int n = 0;
    for (int32_t k = pb; k < pe; ++k) {
        const int32_t v = proc_vox ? proc_vox[k] : k;
        if (v < 0) continue;
        for (int32_t q = vox_ptr[v]; q < vox_ptr[v + 1]; ++q)
            if (stamp[(size_t)fas_v[q]] != tag) {
                stamp[(size_t)fas_v[q]] = tag;
                ++n;
            }
    }
    return n;
}

}  // namespace

void chunk_slots(const life_dims *d, const int32_t *vox_ptr, const int32_t *proc_vox, const std::vector<int32_t> &bounds,
                 std::vector<int32_t> &chunk_vox, std::vector<int32_t> &vox_chunk, std::vector<int32_t> &vox_slot)
{
    const int nc = (int)bounds.size() - 1;
    chunk_vox.assign((size_t)nc * kChunkVoxels, -1);
    vox_chunk.assign((size_t)d->n_voxels, -1);
    vox_slot.assign((size_t)d->n_voxels, -1);
    std::vector<int> ids;
    for (int c = 0; c < nc; ++c) {
        ids.clear();
        for (int32_t k = bounds[c]; k < bounds[c + 1]; ++k) {
            const int v = proc_vox ? proc_vox[k] : k;
            if (v >= 0) ids.push_back(v);
        }
        std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) {
            return vox_ptr[a + 1] - vox_ptr[a] > vox_ptr[b + 1] - vox_ptr[b];
        });
        int64_t load[kChunkWaves] = {0};
        int fill[kChunkWaves] = {0};
        int32_t *slots = chunk_vox.data() + (size_t)c * kChunkVoxels;
        for (int v : ids) {
            int best = -1;
            for (int wv = 0; wv < kChunkWaves; ++wv)
                if (fill[wv] < kWaveVoxels && (best < 0 || load[wv] < load[best])) best = wv;
            const int slot = best * kWaveVoxels + fill[best]++;
            slots[slot] = v;
            vox_chunk[(size_t)v] = c;
            vox_slot[(size_t)v] = slot;
            load[best] += vox_ptr[v + 1] - vox_ptr[v];
        }
    }
}

life_status chunk_layout(const life_dims *d, const TileGeom &tg, const int32_t *vox_ptr, const int16_t *atom_v,
                         const int32_t *fas_v, const float *phi_v, const int32_t *voxel_of_dsc,
                         const int32_t *wc_perm, const int32_t *proc_pos, const int32_t *proc_vox, int32_t n_pos,
                         ChunkLayout *out)
{
    ChunkLayout &L = *out;
    const int nv = d->n_voxels, nf = d->n_fascicles, T = tg.n_tiles, TA = tg.tile_atoms;
    const int64_t nnz = d->nnz;
    // per voxel: first DSC position of each tile (atoms ascend inside a segment)
    std::vector<int32_t> tile_ptr((size_t)nv * (T + 1));
    for (int v = 0; v < nv; ++v) {
        int p = vox_ptr[v];
        const int end = vox_ptr[v + 1];
        for (int t = 0; t < T; ++t) {
            while (p < end && atom_v[p] < t * TA) ++p;
            tile_ptr[(size_t)v * (T + 1) + t] = p;
        }
        tile_ptr[(size_t)v * (T + 1) + T] = end;
    }
    // chunk bounds: groups of kChunkVoxels positions, halved while they cross too
    // many distinct fascicles
    std::vector<int64_t> stamp((size_t)nf, -1);
    int64_t tag = 0;
    L.bounds.assign(1, 0);
    L.fas_overflow = false;
    std::vector<std::pair<int32_t, int32_t>> todo;
    for (int32_t g0 = 0; g0 < n_pos; g0 += kChunkVoxels) {
        todo.assign(1, {g0, std::min(n_pos, g0 + kChunkVoxels)});
        while (!todo.empty()) {
            const auto r = todo.back();
            todo.pop_back();
            const int n = distinct_fascicles(vox_ptr, fas_v, proc_vox, r.first, r.second, stamp, tag++);
            if (n > tg.fas_cap && r.second - r.first > 1) {
                const int32_t mid = r.first + (r.second - r.first) / 2;
                todo.push_back({mid, r.second});   // LIFO: the lower half is cut first
                todo.push_back({r.first, mid});
                continue;
            }
            if (n > tg.fas_cap) L.fas_overflow = true;
            L.bounds.push_back(r.second);
        }
    }
    const int nc = (int)L.bounds.size() - 1;
    L.n_chunks = nc;
    std::vector<int32_t> vox_chunk, vox_slot;
    chunk_slots(d, vox_ptr, proc_vox, L.bounds, L.chunk_vox, vox_chunk, vox_slot);
    // padded positions of the DSC entries and the wave ranges
    L.wave_work.assign((size_t)nc * T * kChunkWaves * kWorkInts, 0);
    std::vector<int32_t> cpos((size_t)nnz);
    L.work.assign((size_t)nc, 0);
    int64_t q = 0;
    for (int c = 0; c < nc; ++c) {
        const int64_t q_chunk = q;
        for (int t = 0; t < T; ++t)
            for (int w = 0; w < kChunkWaves; ++w) {
                int32_t *ww = &L.wave_work[((size_t)(c * T + t) * kChunkWaves + w) * kWorkInts];
                ww[0] = static_cast<int32_t>(std::min<int64_t>(q, kMaxNnz));
                int steps = 0;
                for (int j = 0; j < kWaveVoxels; ++j) {
                    const int v = L.chunk_vox[(size_t)c * kChunkVoxels + w * kWaveVoxels + j];
                    if (v >= 0) {
                        const int32_t p0 = tile_ptr[(size_t)v * (T + 1) + t], p1 = tile_ptr[(size_t)v * (T + 1) + t + 1];
                        for (int32_t p = p0; p < p1; ++p) cpos[(size_t)p] = static_cast<int32_t>(q + (p - p0));
                        const int ns = (p1 - p0 + kStepEntries - 1) / kStepEntries;
                        q += kStepEntries * (int64_t)ns;
                        steps += ns;
                    }
                    ww[1 + j] = steps;
                }
            }
        L.work[(size_t)c] = q - q_chunk;
    }
    if (q > kMaxNnz) return LIFE_ERANGE;
    L.n_pad = q;
    // chunk fascicle lists and local indices
    L.cfas_ptr.assign((size_t)nc + 1, 0);
    L.cfas.clear();
    std::vector<int32_t> loc_of((size_t)nf, -1);
    std::vector<int32_t> list;
    L.max_fas = 0;
    for (int c = 0; c < nc; ++c) {
        list.clear();
        ++tag;
        for (int32_t k = L.bounds[c]; k < L.bounds[c + 1]; ++k) {
            const int v = proc_vox ? proc_vox[k] : k;
            if (v < 0) continue;
            for (int32_t p = vox_ptr[v]; p < vox_ptr[v + 1]; ++p)
                if (stamp[(size_t)fas_v[p]] != tag) {
                    stamp[(size_t)fas_v[p]] = tag;
                    list.push_back(fas_v[p]);
                }
        }
        std::sort(list.begin(), list.end());
        L.cfas.insert(L.cfas.end(), list.begin(), list.end());
        L.cfas_ptr[(size_t)c + 1] = static_cast<int32_t>(L.cfas.size());
        L.max_fas = std::max(L.max_fas, (int)list.size());
    }
    if ((int64_t)L.cfas.size() > kMaxNnz) return LIFE_ERANGE;
    // padded copies (pads: value 0, the atom before them, rank 0, local index 0)
    L.atom_c.assign((size_t)L.n_pad, 0);
    L.fas_c.assign((size_t)L.n_pad, 0);
    L.loc_c.assign((size_t)L.n_pad, 0);
    L.phi_c.assign((size_t)L.n_pad, 0.f);
    for (int c = 0; c < nc; ++c) {
        for (int32_t i = L.cfas_ptr[c]; i < L.cfas_ptr[c + 1]; ++i) loc_of[(size_t)L.cfas[i]] = i - L.cfas_ptr[c];
        for (int32_t k = L.bounds[c]; k < L.bounds[c + 1]; ++k) {
            const int v = proc_vox ? proc_vox[k] : k;
            if (v < 0) continue;
            for (int32_t p = vox_ptr[v]; p < vox_ptr[v + 1]; ++p) {
                const size_t e = (size_t)cpos[(size_t)p];
                L.atom_c[e] = atom_v[p];
                L.fas_c[e] = fas_v[p];
                L.loc_c[e] = static_cast<uint16_t>(loc_of[(size_t)fas_v[p]]);
                L.phi_c[e] = phi_v[p];
            }
        }
    }
    for (int c = 0; c < nc; ++c)
        for (int t = 0; t < T; ++t)
            for (int w = 0; w < kChunkWaves; ++w) {
                const int32_t *ww = &L.wave_work[((size_t)(c * T + t) * kChunkWaves + w) * kWorkInts];
                for (int j = 0; j < kWaveVoxels; ++j) {
                    const int v = L.chunk_vox[(size_t)c * kChunkVoxels + w * kWaveVoxels + j];
                    if (v < 0) continue;
                    const int64_t beg = ww[0] + (int64_t)kStepEntries * (j ? ww[j] : 0);
                    const int64_t end = ww[0] + (int64_t)kStepEntries * ww[j + 1];
                    const int64_t n_real = tile_ptr[(size_t)v * (T + 1) + t + 1] - tile_ptr[(size_t)v * (T + 1) + t];
                    for (int64_t e = beg + n_real; e < end; ++e) L.atom_c[(size_t)e] = L.atom_c[(size_t)e - 1];
                }
            }
    // WC pass 1: the WC order bucketed (stably) by (chunk, tile), runs of one fascicle
    const size_t nct = (size_t)nc * T;
    L.wc_ent.assign(nct + 1, 0);
    for (int64_t p = 0; p < nnz; ++p) {
        const int32_t v = voxel_of_dsc[p];
        ++L.wc_ent[(size_t)vox_chunk[(size_t)v] * T + atom_v[p] / TA + 1];
    }
    for (size_t i = 0; i < nct; ++i) L.wc_ent[i + 1] += L.wc_ent[i];
    std::vector<int32_t> next(L.wc_ent.begin(), L.wc_ent.end() - 1), erank((size_t)nnz);
    L.wkey.assign((size_t)nnz, 0);
    L.wphi.assign((size_t)nnz, 0.f);
    for (int64_t j = 0; j < nnz; ++j) {
        const int32_t p = wc_perm[j];
        const int32_t v = voxel_of_dsc[p];
        const int t = atom_v[p] / TA;
        const int32_t e = next[(size_t)vox_chunk[(size_t)v] * T + t]++;
        L.wkey[(size_t)e] = static_cast<uint16_t>(((atom_v[p] - t * TA) << 6) | vox_slot[(size_t)v]);
        L.wphi[(size_t)e] = phi_v[p];
        erank[(size_t)e] = fas_v[p];
    }
    // runs of one fascicle; each bucket cut into kChunkWaves wave ranges of about
    // equal length at run starts
    std::vector<int32_t> run_rank;
    L.wc_wave.assign(nct * kChunkWaves + 1, 0);
    L.wc_wrun.assign(nct * kChunkWaves, 0);
    for (size_t ct = 0; ct < nct; ++ct) {
        const int32_t e0 = L.wc_ent[ct], e1 = L.wc_ent[ct + 1], n = e1 - e0;
        int w = 0;
        for (int32_t e = e0; e < e1; ++e) {
            if (e != e0 && erank[(size_t)e] == erank[(size_t)e - 1]) continue;
            L.wkey[(size_t)e] |= kRunStart;
            // waves w.. whose share starts at or before e begin here
            while (w < kChunkWaves && (int64_t)(e - e0) * kChunkWaves >= (int64_t)w * n) {
                L.wc_wave[ct * kChunkWaves + w] = e;
                L.wc_wrun[ct * kChunkWaves + w] = static_cast<int32_t>(run_rank.size());
                ++w;
            }
            run_rank.push_back(erank[(size_t)e]);
        }
        for (; w < kChunkWaves; ++w) {   // empty wave ranges at the bucket end
            L.wc_wave[ct * kChunkWaves + w] = e1;
            L.wc_wrun[ct * kChunkWaves + w] = static_cast<int32_t>(run_rank.size());
        }
    }
    L.wc_wave[nct * kChunkWaves] = static_cast<int32_t>(nnz);
    L.n_runs = (int64_t)run_rank.size();
    // WC pass 2: each rank's runs in run order
    L.rr_ptr.assign((size_t)nf + 1, 0);
    for (int64_t r = 0; r < L.n_runs; ++r) ++L.rr_ptr[(size_t)run_rank[(size_t)r] + 1];
    for (int r = 0; r < nf; ++r) L.rr_ptr[(size_t)r + 1] += L.rr_ptr[(size_t)r];
    std::vector<int32_t> fill(L.rr_ptr.begin(), L.rr_ptr.end() - 1);
    L.rr.assign((size_t)L.n_runs, 0);
    for (int64_t r = 0; r < L.n_runs; ++r) L.rr[(size_t)fill[(size_t)run_rank[(size_t)r]]++] = static_cast<int32_t>(r);
    return LIFE_OK;
}
std::vector<int32_t> chunk_schedule(const std::vector<int64_t> &work, SchedulePolicy policy)
{
    const int n = static_cast<int>(work.size());
    std::vector<int32_t> map;
    if (policy == kScheduleIndex || n < kXcds) {
        map.resize((size_t)n);
        for (int i = 0; i < n; ++i) map[(size_t)i] = i;
        return map;
    }
    int bound[kXcds + 1];
    if (policy == kScheduleXcdCount) {
        const int per = n / kXcds, rem = n % kXcds;
        bound[0] = 0;
        for (int x = 0; x < kXcds; ++x) bound[x + 1] = bound[x] + per + (x < rem ? 1 : 0);
    } else {
        int64_t total = 0;
        for (int64_t wk : work) total += wk;
        bound[0] = 0;
        bound[kXcds] = n;
        int c = 0;
        int64_t acc = 0;
        for (int x = 1; x < kXcds; ++x) {
            const int64_t target = total * x / kXcds;
            while (c < n && acc + work[(size_t)c] <= target) acc += work[(size_t)c++];
            bound[x] = c;
        }
    }
    int len = 0;
    for (int x = 0; x < kXcds; ++x) len = std::max(len, bound[x + 1] - bound[x]);
    map.assign((size_t)len * kXcds, -1);
    for (int x = 0; x < kXcds; ++x)
        for (int k = 0; k < bound[x + 1] - bound[x]; ++k) map[(size_t)k * kXcds + x] = bound[x] + k;
    return map;
}

}  // namespace life

extern "C" life_status life_plan_host(const life_dims *dims, const int16_t *atom, const int32_t *voxel,
                                      const int32_t *fascicle, const int16_t *voxel_xyz, int32_t *dsc_perm,
                                      int32_t *vox_ptr, int32_t *fas_rank, int32_t *wc_perm, int32_t *fas_ptr)
{
    life_status st = life::validate_dims(dims);
    if (st != LIFE_OK) return st;
    if ((st = life::validate_coords(dims, voxel_xyz)) != LIFE_OK) return st;
    try {
        std::vector<int32_t> pos;
        if (voxel_xyz) {
            pos.resize((size_t)dims->n_voxels);
            life::voxel_order(dims, voxel_xyz, 1, nullptr, pos.data(), nullptr);
        }
        return life::plan_host(dims, atom, voxel, fascicle, voxel_xyz ? pos.data() : nullptr, dims->n_voxels, nullptr,
                               dsc_perm, vox_ptr, fas_rank, wc_perm, fas_ptr);
    } catch (const std::bad_alloc &) {
        return LIFE_ENOMEM;
    }
}

extern "C" life_status life_plan_host_batch(const life_dims *dims, int32_t n_inst, const int32_t *vox_off,
                                            const int32_t *fas_off, const int16_t *atom, const int32_t *voxel,
                                            const int32_t *fascicle, const int16_t *voxel_xyz, int32_t *proc_pos,
                                            int32_t *dsc_perm, int32_t *vox_ptr, int32_t *fas_rank, int32_t *wc_perm,
                                            int32_t *fas_ptr)
{
    life_status st = life::validate_dims(dims);
    if (st != LIFE_OK) return st;
    if ((st = life::validate_coords(dims, voxel_xyz)) != LIFE_OK) return st;
    if ((st = life::validate_indices(dims, atom, voxel, fascicle)) != LIFE_OK) return st;
    if ((st = life::validate_instances(dims, n_inst, vox_off, fas_off, voxel, fascicle)) != LIFE_OK) return st;
    try {
        const int32_t n_pos = life::padded_positions(dims, n_inst, vox_off);
        if (n_pos < 0) return LIFE_ERANGE;
        std::vector<int32_t> pos((size_t)dims->n_voxels);
        life::voxel_order(dims, voxel_xyz, n_inst, vox_off, pos.data(), nullptr);
        std::vector<int32_t> fas_inst((size_t)dims->n_fascicles);
        for (int k = 0; k < n_inst; ++k)
            for (int32_t f = fas_off[k]; f < fas_off[k + 1]; ++f) fas_inst[(size_t)f] = k;
        if (proc_pos && dims->n_voxels) std::memcpy(proc_pos, pos.data(), sizeof(int32_t) * pos.size());
        return life::plan_host(dims, atom, voxel, fascicle, pos.data(), n_pos, fas_inst.data(), dsc_perm, vox_ptr,
                               fas_rank, wc_perm, fas_ptr);
    } catch (const std::bad_alloc &) {
        return LIFE_ENOMEM;
    }
}

extern "C" const char *life_status_str(life_status s)
{
    switch (s) {
    case LIFE_OK: return "LIFE_OK";
    case LIFE_EINVAL: return "LIFE_EINVAL: invalid argument";
    case LIFE_ERANGE: return "LIFE_ERANGE: index or size out of range";
    case LIFE_ENOMEM: return "LIFE_ENOMEM: out of memory";
    case LIFE_EDEVICE: return "LIFE_EDEVICE: HIP runtime error";
    }
    return "LIFE_?: unknown status";
}
