// build.hip -- voxelisation of a labeled point cloud (paper, Section 2.1).
//
// The paper keeps a low-resolution voxel grid for traversal and divides each
// voxel by an integer factor into subvoxels that localise the geometry.  Here
// that becomes a hierarchy of 1..4 levels, each level dividing the previous
// one by an integer ratio:
//
//   level 0          dense int32 map over the coarse grid (node index or -1)
//   levels 1..L-1    occupancy bricks: per occupied parent a bitmask over its
//                    ratio^3 children plus, per 64-bit word, the index of the
//                    first child of that word (child = base + popcount)
//   leaves           (first entry, count) ranges into leaf-ordered surfels
//   surfels          two 16-byte streams per entry, in leaf order:
//                    (x, y, z, point id) and (unit normal, label rank)
//
// A point is listed in EVERY leaf that the axis-aligned box of its disk
// (radius r_s, its own normal) overlaps, padded by a rounding margin, so a
// traversal that tests the leaves it passes finds every disk it crosses.
//
// Pipeline: ingest (normalise normals, validate, AABB, max label) -> sync ->
// label ranks -> per-point leaf counts -> scan -> sync -> emit (key, id) ->
// radix sort -> per-tile node-start counts + their scan -> sync -> level-0
// map, bricks, leaf ranges (one pass over the sorted keys) -> surfel gather.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace pcrl {

constexpr int BUILD_BLOCK = 256;

static unsigned blocks_for(int64_t n, int block = BUILD_BLOCK) {
    int64_t g = (n + block - 1) / block;
    return (unsigned)std::max<int64_t>(1, g);
}

static int bits_for(uint64_t max_value) {
    int b = 1;
    while (b < 64 && (max_value >> b) != 0) ++b;
    return b;
}

// ---------------------------------------------------------------------------
// ingest
// ---------------------------------------------------------------------------

struct IngestOut {
    float lo[3];
    float hi[3];
    uint32_t max_label;
    uint32_t bad;  // bit0 non-finite position, bit1 bad normal
};

__global__ __launch_bounds__(BUILD_BLOCK) void k_ingest(const float* xyz, const float* nrm, const uint32_t* label,
                                                        int64_t n, float4* unit_nrm, IngestOut* partial) {
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    uint32_t ml = 0, bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * BUILD_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BUILD_BLOCK) {
        const float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        if (!isfinite(x) || !isfinite(y) || !isfinite(z)) bad |= 1u;
        lo[0] = fminf(lo[0], x); lo[1] = fminf(lo[1], y); lo[2] = fminf(lo[2], z);
        hi[0] = fmaxf(hi[0], x); hi[1] = fmaxf(hi[1], y); hi[2] = fmaxf(hi[2], z);
        const float a = nrm[3 * i], b = nrm[3 * i + 1], c = nrm[3 * i + 2];
        const float l2 = a * a + b * b + c * c;
        float inv = 0.f;
        if (!(l2 > 0.f) || !isfinite(l2))
            bad |= 2u;
        else
            inv = 1.0f / sqrtf(l2);
        unit_nrm[i] = make_float4(a * inv, b * inv, c * inv, 0.f);
        ml = max(ml, label[i]);
    }
    // block reduction through LDS
    __shared__ float s_lo[3][BUILD_BLOCK / 64], s_hi[3][BUILD_BLOCK / 64];
    __shared__ uint32_t s_ml[BUILD_BLOCK / 64], s_bad[BUILD_BLOCK / 64];
    for (int off = 32; off > 0; off >>= 1) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], off, 64));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off, 64));
        }
        ml = max(ml, __shfl_xor(ml, off, 64));
        bad |= __shfl_xor(bad, off, 64);
    }
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        for (int a = 0; a < 3; ++a) { s_lo[a][w] = lo[a]; s_hi[a][w] = hi[a]; }
        s_ml[w] = ml;
        s_bad[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        IngestOut o;
        for (int a = 0; a < 3; ++a) { o.lo[a] = INFINITY; o.hi[a] = -INFINITY; }
        o.max_label = 0;
        o.bad = 0;
        for (int k = 0; k < BUILD_BLOCK / 64; ++k) {
            for (int a = 0; a < 3; ++a) { o.lo[a] = fminf(o.lo[a], s_lo[a][k]); o.hi[a] = fmaxf(o.hi[a], s_hi[a][k]); }
            o.max_label = max(o.max_label, s_ml[k]);
            o.bad |= s_bad[k];
        }
        partial[blockIdx.x] = o;
    }
}

// One block of BUILD_BLOCK threads folds the per-block partials.
__global__ __launch_bounds__(BUILD_BLOCK) void k_ingest_final(const IngestOut* partial, int nb, IngestOut* out) {
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    uint32_t ml = 0, bad = 0;
    for (int k = threadIdx.x; k < nb; k += BUILD_BLOCK) {
        const IngestOut p = partial[k];
        for (int a = 0; a < 3; ++a) { lo[a] = fminf(lo[a], p.lo[a]); hi[a] = fmaxf(hi[a], p.hi[a]); }
        ml = max(ml, p.max_label);
        bad |= p.bad;
    }
    for (int off = 32; off > 0; off >>= 1) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], off, 64));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off, 64));
        }
        ml = max(ml, __shfl_xor(ml, off, 64));
        bad |= __shfl_xor(bad, off, 64);
    }
    __shared__ IngestOut s[BUILD_BLOCK / 64];
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        for (int a = 0; a < 3; ++a) { s[w].lo[a] = lo[a]; s[w].hi[a] = hi[a]; }
        s[w].max_label = ml;
        s[w].bad = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        IngestOut o = s[0];
        for (int k = 1; k < BUILD_BLOCK / 64; ++k) {
            for (int a = 0; a < 3; ++a) { o.lo[a] = fminf(o.lo[a], s[k].lo[a]); o.hi[a] = fmaxf(o.hi[a], s[k].hi[a]); }
            o.max_label = max(o.max_label, s[k].max_label);
            o.bad |= s[k].bad;
        }
        *out = o;
    }
}

// ---------------------------------------------------------------------------
// dilated keys
// ---------------------------------------------------------------------------

struct KeyParams {
    SceneView v;
    float r_s;
    float pad;
    int32_t id_bits;   // packed 64-bit items: bits of the point index below the key
    uint8_t* occ0;     // k_key_count: level-0 cells that a point's leaf box reaches (set to 1)
    const uint32_t* c0;  // k_key_emit: rank of each such level-0 cell (the key's level-0 part)
};

// Hierarchical key of leaf (x, y, z) with level 0 numbered by `c0` (rank of
// the level-0 cell among the occupied ones) or by its linear index (c0
// null); the quotients use the traversal's magic divisions.  Equal to
// leaf_key_of when c0 is null.
__host__ __device__ __forceinline__ uint64_t leaf_key_fast(const SceneView& v, const uint32_t* c0, int x, int y, int z) {
    int p[3] = {span_div(x, v.mspan[0]), span_div(y, v.mspan[0]), span_div(z, v.mspan[0])};
    const uint32_t cell0 = (uint32_t)p[0] + (uint32_t)v.dim0[0] * ((uint32_t)p[1] + (uint32_t)v.dim0[1] * (uint32_t)p[2]);
    uint64_t k = c0 ? (uint64_t)c0[cell0] : (uint64_t)cell0;
#pragma unroll
    for (int i = 1; i < PCRL_MAX_LEVELS; ++i) {
        if (i >= v.nlev) break;
        const int q[3] = {span_div(x, v.mspan[i]), span_div(y, v.mspan[i]), span_div(z, v.mspan[i])};
        const int r = v.ratio[i - 1];
        const int loc = (q[0] - r * p[0]) + r * ((q[1] - r * p[1]) + r * (q[2] - r * p[2]));
        k = (k << v.lbits[i]) | (uint64_t)loc;
        p[0] = q[0];
        p[1] = q[1];
        p[2] = q[2];
    }
    return k;
}

__device__ __forceinline__ void disk_leaf_box(const KeyParams& kp, const float* xyz, const float4* un, int64_t i,
                                              int lo[3], int hi[3]) {
    const float p[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
    const float4 nn = un[i];
    const float nv[3] = {nn.x, nn.y, nn.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float e = kp.r_s * sqrtf(fmaxf(0.f, 1.f - nv[a] * nv[a])) + kp.pad;
        int l = (int)floorf((p[a] - e - kp.v.org[a]) * kp.v.inv_h);
        int u = (int)floorf((p[a] + e - kp.v.org[a]) * kp.v.inv_h);
        lo[a] = min(max(l, 0), kp.v.dim[a] - 1);
        hi[a] = min(max(u, 0), kp.v.dim[a] - 1);
    }
}

// Whether the disk of point i (radius r_s) may meet leaf (x, y, z), the leaf
// grown by the rounding pad: both the disk's sphere and its plane must reach
// the box.  Both are necessary conditions of an intersection, so no leaf the
// disk touches is dropped; the corner leaves of the disk's bounding box
// (sphere test) and, for tilted disks, off-plane leaves (plane test) are.
__device__ __forceinline__ bool disk_meets_leaf(const KeyParams& kp, const float p[3], const float nv[3], int x, int y,
                                                int z) {
    const float hh = 0.5f * kp.v.h + kp.pad;
    const int c[3] = {x, y, z};
    float d2 = 0.f, pr = 0.f, dn = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float ca = kp.v.org[a] + ((float)c[a] + 0.5f) * kp.v.h;  // leaf centre
        const float q = fabsf(p[a] - ca) - hh;
        if (q > 0.f) d2 += q * q;
        pr += fabsf(nv[a]) * hh;
        dn += nv[a] * (ca - p[a]);
    }
    const float r = kp.r_s + kp.pad;
    return d2 <= r * r && fabsf(dn) <= pr + kp.pad;
}

// Keys of one wave staged in LDS before a coalesced copy out (entries past
// the stage are written directly).
constexpr int EMIT_STAGE = 2048;

template <bool EMIT, typename K>
__device__ __forceinline__ uint32_t disk_leaves(const KeyParams& kp, const float* xyz, const float4* un, int64_t i,
                                                K* keys, uint32_t* ids, uint32_t o, K* stage = nullptr,
                                                uint32_t base = 0) {
    int lo[3], hi[3];
    disk_leaf_box(kp, xyz, un, i, lo, hi);
    const float p[3] = {xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]};
    const float4 nn = un[i];
    const float nv[3] = {nn.x, nn.y, nn.z};
    uint32_t k = 0;
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
                // a disk inside a single leaf keeps it without the test
                const bool one = lo[0] == hi[0] && lo[1] == hi[1] && lo[2] == hi[2];
                if (!one && !disk_meets_leaf(kp, p, nv, x, y, z)) continue;
                if (EMIT) {
                    const uint64_t key = leaf_key_fast(kp.v, kp.c0, x, y, z);
                    if (ids) {
                        keys[o + k] = (K)key;
                        ids[o + k] = (uint32_t)i;
                    } else {
                        // packed: the key above the point index (one 8-byte item to sort)
                        const K item = (K)((key << kp.id_bits) | (uint64_t)i);
                        const uint32_t at = o + k;
                        if (stage && at - base < (uint32_t)EMIT_STAGE) stage[at - base] = item;
                        else keys[at] = item;
                    }
                }
                ++k;
            }
    return k;
}

// Per point, the number of leaves its disk meets; the level-0 cells its leaf
// box reaches are marked in occ0 (a superset of those of its leaves).
__global__ __launch_bounds__(BUILD_BLOCK) void k_key_count(KeyParams kp, const float* xyz, const float4* un, int64_t n,
                                                           uint32_t* cnt) {
    int64_t i = (int64_t)blockIdx.x * BUILD_BLOCK + threadIdx.x;
    if (i >= n) return;
    cnt[i] = disk_leaves<false, uint64_t>(kp, xyz, un, i, nullptr, nullptr, 0);
    if (kp.occ0) {
        int lo[3], hi[3];
        disk_leaf_box(kp, xyz, un, i, lo, hi);
        const SceneView& v = kp.v;
        for (int cz = span_div(lo[2], v.mspan[0]); cz <= span_div(hi[2], v.mspan[0]); ++cz)
            for (int cy = span_div(lo[1], v.mspan[0]); cy <= span_div(hi[1], v.mspan[0]); ++cy)
                for (int cx = span_div(lo[0], v.mspan[0]); cx <= span_div(hi[0], v.mspan[0]); ++cx)
                    kp.occ0[(size_t)cx + (size_t)v.dim0[0] * ((size_t)cy + (size_t)v.dim0[1] * cz)] = 1;
    }
}

// Ranks of the marked level-0 cells (exclusive scan of occ0, widened to 32
// bits first) and the inverse map rank -> cell.
__global__ void k_occ0_widen(const uint8_t* occ0, int64_t n, uint32_t* out) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) out[c] = occ0[c];
}

__global__ void k_occ0_unmap(const uint8_t* occ0, const uint32_t* rank, int64_t n, uint32_t* unmap) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n && occ0[c]) unmap[rank[c]] = (uint32_t)c;
}

// The counts' sum in 64 bits, for inputs whose 32-bit scan might wrap: a
// grid-stride sum per thread, one atomic per wave.
__global__ __launch_bounds__(BUILD_BLOCK) void k_count_total(const uint32_t* cnt, int64_t n, unsigned long long* total) {
    unsigned long long acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * BUILD_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BUILD_BLOCK)
        acc += cnt[i];
    acc = wave_sum_u64(acc);
    if (lane_id() == 0 && acc) atomicAdd(total, acc);
}

// The (key, point) items of every point's leaves at its offset.  Packed items
// (ids null) of a one-wave block are contiguous from its first point's
// offset: they are staged in LDS and copied out with coalesced stores.
template <typename K>
__global__ __launch_bounds__(64) void k_key_emit(KeyParams kp, const float* xyz, const float4* un, int64_t n,
                                                 const uint32_t* off, K* keys, uint32_t* ids) {
    const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const bool in = i < n;
    if (ids) {
        if (in) (void)disk_leaves<true, K>(kp, xyz, un, i, keys, ids, off[i]);
        return;
    }
    __shared__ K stage[EMIT_STAGE];
    const uint32_t o = in ? off[i] : 0u;
    const uint32_t base = __builtin_amdgcn_readfirstlane(o);  // lane 0 holds the block's first point
    const uint32_t cnt = in ? disk_leaves<true, K>(kp, xyz, un, i, keys, nullptr, o, stage, base) : 0u;
    uint32_t end = in ? o + cnt : base;
#pragma unroll
    for (int sh = 32; sh >= 1; sh >>= 1) end = max(end, (uint32_t)__shfl_xor((int)end, sh, 64));
    const uint32_t total = min(end - base, (uint32_t)EMIT_STAGE);
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < total; j += 64) keys[(size_t)base + j] = stage[j];
}

// ---------------------------------------------------------------------------
// hierarchy from sorted keys
// ---------------------------------------------------------------------------

struct LevelShifts {
    int32_t nlev;
    int32_t sh[PCRL_MAX_LEVELS];  // node key of level i = key >> sh[i]
};

struct HierOut {
    const uint32_t* unmap0;   // rank of an occupied level-0 cell -> the cell (null: keys hold the cell)
    int32_t g_sh0;            // bits below the level-0 part of a key (without the packed point index)
    int32_t* map0;
    uint64_t* mask[PCRL_MAX_LEVELS - 1];
    uint32_t* first_child[PCRL_MAX_LEVELS - 1];
    uint2* leaf;
    uint64_t* leaf_key;
};

// Node starts of every level from the sorted keys: an entry opens a node of
// level l when its key differs from the previous entry's above bit sh[l].
// A wave owns a tile of LINK_TILE consecutive entries, read in LINK_ROUNDS
// coalesced rounds of 64 (lane j of round r: entry tile + 64 r + j).
constexpr int LINK_ROUNDS = 16;
constexpr int LINK_TILE = 64 * LINK_ROUNDS;

__device__ __forceinline__ uint32_t link_flags(const uint64_t* keys, int64_t e, const LevelShifts& ls) {
    const uint64_t k = keys[e];
    const uint64_t prev = e > 0 ? keys[e - 1] : 0ull;
    uint32_t f = 0;
#pragma unroll
    for (int l = 0; l < PCRL_MAX_LEVELS; ++l)
        if (l < ls.nlev && (e == 0 || ((k ^ prev) >> ls.sh[l]) != 0)) f |= 1u << l;
    return f;
}

// Per wave tile and level: the nodes that start in the tile ([level][tile]).
__global__ __launch_bounds__(BUILD_BLOCK) void k_link_count(const uint64_t* keys, int64_t m, LevelShifts ls,
                                                            uint32_t* tile_cnt, uint32_t n_tiles) {
    const uint32_t tile = blockIdx.x * (BUILD_BLOCK / 64) + (threadIdx.x >> 6);
    if (tile >= n_tiles) return;
    uint32_t c[PCRL_MAX_LEVELS] = {0u, 0u, 0u, 0u};
    for (int r = 0; r < LINK_ROUNDS; ++r) {
        const int64_t e = (int64_t)tile * LINK_TILE + 64 * r + lane_id();
        const uint32_t f = e < m ? link_flags(keys, e, ls) : 0u;
#pragma unroll
        for (int l = 0; l < PCRL_MAX_LEVELS; ++l) c[l] += (f >> l) & 1u;
    }
#pragma unroll
    for (int l = 0; l < PCRL_MAX_LEVELS; ++l) {
        const uint32_t t = (uint32_t)wave_sum_u64(c[l]);
        if (l < ls.nlev && lane_id() == 0) tile_cnt[(size_t)l * n_tiles + tile] = t;
    }
}

// For every entry that opens a node: register the node with its parent (its
// bit in the parent brick's mask, the parent's first child), the level-0 map
// and the leaf's first entry and key.  tile_off[l][t] is the exclusive scan
// of the tiles' node counts, so the node of level l holding entry e is the
// number of level-l nodes opened up to and including e, minus one.
__global__ __launch_bounds__(BUILD_BLOCK) void k_link(const uint64_t* keys, int64_t m, LevelShifts ls, SceneView v,
                                                      const uint32_t* tile_off, uint32_t n_tiles, HierOut h,
                                                      int id_bits) {
    const uint32_t tile = blockIdx.x * (BUILD_BLOCK / 64) + (threadIdx.x >> 6);
    if (tile >= n_tiles) return;
    const int L = ls.nlev;
    uint32_t carry[PCRL_MAX_LEVELS] = {0u, 0u, 0u, 0u};
    for (int l = 0; l < L; ++l) carry[l] = tile_off[(size_t)l * n_tiles + tile];
    for (int r = 0; r < LINK_ROUNDS; ++r) {
        const int64_t e = (int64_t)tile * LINK_TILE + 64 * r + lane_id();
        const bool in = e < m;
        const uint32_t f = in ? link_flags(keys, e, ls) : 0u;
        const uint64_t k = in ? keys[e] : 0ull;
        // the levels' flags in 8-bit fields of one word (at most 64 per field): one wave scan
        uint32_t fp = 0;
#pragma unroll
        for (int l = 0; l < PCRL_MAX_LEVELS; ++l) fp |= ((f >> l) & 1u) << (8 * l);
        const uint32_t incl = wave_incl_scan(fp);
        const uint32_t sum = __shfl(incl, 63, 64);
        uint32_t node[PCRL_MAX_LEVELS];
#pragma unroll
        for (int l = 0; l < PCRL_MAX_LEVELS; ++l) {
            node[l] = carry[l] + ((incl >> (8 * l)) & 0xFFu) - 1u;
            carry[l] += (sum >> (8 * l)) & 0xFFu;
        }
        if (!in) continue;
#pragma unroll
        for (int l = 0; l < PCRL_MAX_LEVELS; ++l) {
            if (!((f >> l) & 1u)) continue;
            if (l == 0) {
                const uint64_t top = k >> ls.sh[0];
                h.map0[h.unmap0 ? (uint64_t)h.unmap0[top] : top] = (int32_t)node[0];
            }
            if (l == L - 1) {
                const uint64_t top = k >> ls.sh[0];
                const uint64_t cell0 = h.unmap0 ? (uint64_t)h.unmap0[top] : top;
                const uint64_t kk = k >> id_bits;
                h.leaf[node[l]].x = (uint32_t)e;
                // the leaf's key with level 0 as the linear cell index
                h.leaf_key[node[l]] = (cell0 << h.g_sh0) | (kk & ((uint64_t(1) << h.g_sh0) - 1));
            }
            if (l > 0) {
                const uint32_t parent = node[l - 1];
                const uint32_t local = (uint32_t)((k >> ls.sh[l]) & ((uint64_t(1) << v.lbits[l]) - 1));
                atomicOr((unsigned long long*)&h.mask[l - 1][(size_t)parent * v.nw[l - 1] + (local >> 6)],
                         (unsigned long long)(uint64_t(1) << (local & 63)));
                // the first child of a parent is the entry that opens the parent too
                if ((f >> (l - 1)) & 1u) h.first_child[l - 1][parent] = node[l];
            }
        }
    }
}

__global__ void k_brick_base(const uint64_t* mask, const uint32_t* first_child, int64_t n_nodes, int nw,
                             uint32_t* base) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_nodes) return;
    uint32_t run = first_child[p];
    for (int w = 0; w < nw; ++w) {
        base[(size_t)p * nw + w] = run;
        run += (uint32_t)__popcll(mask[(size_t)p * nw + w]);
    }
}

// Box of the occupied children of every brick, in the brick's local child
// coordinates (x + r (y + r z) order of the mask bits): lo x, y, z in bits
// 0-14 and hi x, y, z in bits 15-29, 5 bits each (r <= 32).  Every child
// outside the box is empty, so a ray in such a child crosses the brick's
// empty rest up to the box or the brick's exit in one step.
__global__ void k_brick_aabb(const uint64_t* mask, int64_t n_nodes, int nw, int r, uint32_t* aabb) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_nodes) return;
    int lo0 = 31, lo1 = 31, lo2 = 31, hi0 = 0, hi1 = 0, hi2 = 0;
    for (int w = 0; w < nw; ++w) {
        uint64_t m = mask[(size_t)p * nw + w];
        while (m) {
            const int loc = 64 * w + __ffsll((long long)m) - 1;
            m &= m - 1;
            const int x = loc % r, y = (loc / r) % r, z = loc / (r * r);
            lo0 = min(lo0, x); lo1 = min(lo1, y); lo2 = min(lo2, z);
            hi0 = max(hi0, x); hi1 = max(hi1, y); hi2 = max(hi2, z);
        }
    }
    aabb[p] = (uint32_t)lo0 | ((uint32_t)lo1 << 5) | ((uint32_t)lo2 << 10) | ((uint32_t)hi0 << 15) |
              ((uint32_t)hi1 << 20) | ((uint32_t)hi2 << 25);
}

// Empty-space skip radius of every leaf cell of an occupied parent brick
// (r^3 cells, r <= 16): R = 0 for an occupied leaf; otherwise the largest k
// such that the cube of cells within Chebyshev distance k - 1 is empty and
// inside the brick.  This is the per-voxel march distance of Section 2.2.4
// (the longest per-axis distance to the closest voxel with content), limited
// to the brick.  The cells within Chebyshev distance k of an occupied cell
// are the occupancy dilated k times by the 3 x 3 x 3 cube, and the dilation
// is separable: with the brick held as r^2 rows of r bits (row y + r z, bit
// x), one step ORs each row with its shifts along x, then with its y and z
// neighbour rows.  A cell first reached at step k is at distance k; the
// border limits every radius to at most (r - 1) / 2 + 1, so that many steps
// suffice.  One wave per brick (rows and distances in the wave's LDS).
// RC > 0: the ratio is the compile-time constant RC (index arithmetic by
// constants); RC = 0: the runtime r.
constexpr int BDIST_RMAX = 16;

__device__ __forceinline__ void build_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int RC>
__global__ __launch_bounds__(BUILD_BLOCK) void k_brick_dist(const uint64_t* mask, int nw, int r_rt, int64_t n_bricks,
                                                            uint8_t* dist) {
    __shared__ uint32_t rows_s[BUILD_BLOCK / 64][2][BDIST_RMAX * BDIST_RMAX];
    __shared__ uint8_t d_s[BUILD_BLOCK / 64][BDIST_RMAX * BDIST_RMAX * BDIST_RMAX];
    const int r = RC > 0 ? RC : r_rt;
    const int n2 = r * r, n3 = n2 * r;
    const int w = threadIdx.x >> 6;
    const int lane = (int)lane_id();
    const int64_t P = (int64_t)blockIdx.x * (BUILD_BLOCK / 64) + w;
    if (P >= n_bricks) return;  // the whole wave: no block-wide barrier follows
    uint32_t* cur = rows_s[w][0];
    uint32_t* tmp = rows_s[w][1];
    uint8_t* D = d_s[w];
    const uint32_t full = (1u << r) - 1u;
    // row j holds bits [r j, r j + r) of the brick's mask
    for (int j = lane; j < n2; j += 64) {
        const int b0 = r * j;
        const uint64_t* m = mask + (size_t)P * nw + (b0 >> 6);
        uint64_t bits = m[0] >> (b0 & 63);
        if ((b0 & 63) + r > 64) bits |= m[1] << (64 - (b0 & 63));
        cur[j] = (uint32_t)bits & full;
    }
    build_wave_sync();
    for (int c = lane; c < n3; c += 64) D[c] = ((cur[c / r] >> (c % r)) & 1u) ? 0 : 255;
    const int K = (r - 1) / 2 + 1;
    for (int k = 1; k <= K; ++k) {
        // along x, then y
        for (int j = lane; j < n2; j += 64) {
            const int y = j % r;
            const uint32_t a = cur[j];
            uint32_t t = a | (a << 1) | (a >> 1);
            if (y > 0) {
                const uint32_t b = cur[j - 1];
                t |= b | (b << 1) | (b >> 1);
            }
            if (y < r - 1) {
                const uint32_t b = cur[j + 1];
                t |= b | (b << 1) | (b >> 1);
            }
            tmp[j] = t & full;
        }
        build_wave_sync();
        // along z; the cells reached now are at distance k
        for (int j = lane; j < n2; j += 64) {
            const int z = j / r;
            uint32_t t = tmp[j];
            if (z > 0) t |= tmp[j - r];
            if (z < r - 1) t |= tmp[j + r];
            uint32_t nb = t & ~cur[j];
            while (nb) {
                const int x = __ffs(nb) - 1;
                nb &= nb - 1u;
                D[x + r * j] = (uint8_t)k;
            }
            cur[j] = t;
        }
        build_wave_sync();
    }
    for (int c = lane; c < n3; c += 64) {
        const int x = c % r, y = (c / r) % r, z = c / n2;
        const int db = min(min(min(x, r - 1 - x), min(y, r - 1 - y)), min(z, r - 1 - z));
        dist[P * n3 + c] = (uint8_t)min((int)D[c], db + 1);
    }
}

// Empty-space skip radii of the level-0 grid: for every cell the Chebyshev
// distance (in cells, at most DIST0_CAP + 1) to the nearest occupied cell, so
// the cube of radius d - 1 around an empty cell holds no occupied cell.  The
// same march distance as inside the bricks, one level up.  Separable: one
// pass per axis of out(c) = min over |t| <= DIST0_CAP of max(|t|, in(c + t e)),
// starting from 0 (occupied) / 255 (empty).  A window that misses the
// nearest occupied cell only lowers the result (conservative).
constexpr int DIST0_CAP = 15;

// Largest dense cell table built: the table pays off while it stays resident
// in the 256 MB last-level (MALL) cache; a larger one (3.3 GB for a 20M-point
// street canyon) turns every DDA step into an HBM round trip and doubled that
// scene's trace time.  Beyond it the traversal reads the bricks' masks.
constexpr int64_t CELL_TABLE_MAX_BYTES = (int64_t)256 << 20;

__global__ void k_dist0_pass(const int32_t* map0, const uint8_t* in, uint8_t* out, int dx, int dy, int dz, int axis) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)dx * dy * dz;
    if (c >= n) return;
    const int x = (int)(c % dx), y = (int)((c / dx) % dy), z = (int)(c / ((int64_t)dx * dy));
    const int pos = axis == 0 ? x : (axis == 1 ? y : z);
    const int len = axis == 0 ? dx : (axis == 1 ? dy : dz);
    const int64_t stride = axis == 0 ? 1 : (axis == 1 ? dx : (int64_t)dx * dy);
    int m = 255;
    const int t0 = max(-DIST0_CAP, -pos), t1 = min(DIST0_CAP, len - 1 - pos);
    for (int t = t0; t <= t1; ++t) {
        const int64_t q = c + t * stride;
        const int a = map0 ? (map0[q] >= 0 ? 0 : 255) : (int)in[q];
        m = min(m, max(abs(t), a));
    }
    out[c] = (uint8_t)min(m, DIST0_CAP + 1);
}

// Dense cell table of the leaves' parent bricks: one 8-byte load per DDA
// step gives an occupied leaf's entry range, or, for an empty leaf, its skip
// radii per direction octant.  Radius s of octant (sx, sy, sz) (bit a set:
// the ray's component a is negative) means the box of s x s x s cells that
// starts at the cell and extends along the octant's signs is empty and inside
// the brick; a ray whose direction lies in that octant crosses the box in one
// step.  s is the octant-restricted Chebyshev distance to the nearest
// occupied cell, capped by the brick's far faces and by 15 (4 bits per
// octant, 8 octants in the first word).
// Computed on bit rows (the r <= 16 cells of a brick row along x in one
// 16-bit word), per octant: E_1 = empty cells; E_{s+1}(c) = AND of E_s over the
// 8 cells c + delta, delta in {0, 1}^3 along the octant's signs (a box of s + 1
// is the union of 8 boxes of s), cells outside the brick counting as not
// empty.  The radius of a cell is the number of s <= 15 with E_s(c), kept as a
// 4-bit counter in bit planes.
constexpr int OCT_ITEMS = 8;  // (octant, row) items per thread: 8 * r^2 <= OCT_ITEMS * BUILD_BLOCK for r <= 16

__global__ __launch_bounds__(BUILD_BLOCK) void k_brick_cells(const uint64_t* mask, const uint32_t* base,
                                                            const uint2* leaf, int nw, int r, uint2* cells) {
    extern __shared__ uint16_t rows[];  // [2][8][r^2]: E_s and E_{s+1} per octant and row; then the radii
    __shared__ uint64_t wmask[64];      // the brick's occupancy words (nw <= 64 for r <= 16)
    const int r2 = r * r, n3 = r2 * r;
    const int items = 8 * r2;
    const uint32_t full = (1u << r) - 1u;
    const size_t P = blockIdx.x;
    uint16_t* Ecur = rows;
    uint16_t* Enext = rows + items;
    for (int k = threadIdx.x; k < nw; k += BUILD_BLOCK) wmask[k] = mask[P * nw + k];
    __syncthreads();
    // E_1: empty cells of every row, the same for all octants
    for (int row = threadIdx.x; row < r2; row += BUILD_BLOCK) {
        uint32_t e = 0;
        for (int x = 0; x < r; ++x) {
            const int c = x + r * row;
            if (!((wmask[c >> 6] >> (c & 63)) & 1ull)) e |= 1u << x;
        }
        for (int o = 0; o < 8; ++o) Ecur[o * r2 + row] = (uint16_t)e;
    }
    __syncthreads();
    uint16_t plane[OCT_ITEMS][4];
    for (int k = 0; k < OCT_ITEMS; ++k)
        for (int b = 0; b < 4; ++b) plane[k][b] = 0;
    for (int sz = 1; sz <= 15; ++sz) {
        int any = 0;  // some E_{s+1} is not empty
        for (int k = 0; k < OCT_ITEMS; ++k) {
            const int it = threadIdx.x + k * BUILD_BLOCK;
            if (it >= items) break;
            const int o = it / r2, row = it % r2;
            const uint32_t e = Ecur[it];
            // count this s (4-bit ripple add of the bits of E_s)
            uint32_t carry = e;
            for (int b = 0; b < 4; ++b) {
                const uint32_t pb = plane[k][b];
                plane[k][b] = (uint16_t)(pb ^ carry);
                carry &= pb;
            }
            if (sz == 15) continue;
            const int y = row % r, z = row / r;
            const int sy = (o & 2) ? -1 : 1, szn = (o & 4) ? -1 : 1;
            const bool negx = (o & 1) != 0;
            const uint16_t* Eo = Ecur + (size_t)o * r2;
            auto get = [&](int yy, int zz) -> uint32_t {
                if (yy < 0 || yy >= r || zz < 0 || zz >= r) return 0u;
                const uint32_t v = Eo[yy + r * zz];
                const uint32_t sh = negx ? ((v << 1) & full) : (v >> 1);  // the neighbour along x
                return v & sh;
            };
            const uint16_t en = (uint16_t)(get(y, z) & get(y + sy, z) & get(y, z + szn) & get(y + sy, z + szn));
            Enext[it] = en;
            any |= en;
        }
        // once every E_{s+1} is empty, no later size counts anything
        if (!__syncthreads_or(any)) break;
        uint16_t* t = Ecur;
        Ecur = Enext;
        Enext = t;
    }
    // radii packed per cell (octant o in bits 4o..4o+3), written with the occupied leaves' ranges
    __syncthreads();
    uint32_t* packed = reinterpret_cast<uint32_t*>(rows + 2 * items);  // [n3]
    for (int c = threadIdx.x; c < n3; c += BUILD_BLOCK) packed[c] = 0u;
    __syncthreads();
    for (int k = 0; k < OCT_ITEMS; ++k) {
        const int it = threadIdx.x + k * BUILD_BLOCK;
        if (it >= items) break;
        const int o = it / r2, row = it % r2;
        for (int x = 0; x < r; ++x) {
            const uint32_t n = ((plane[k][0] >> x) & 1u) | (((plane[k][1] >> x) & 1u) << 1) |
                               (((plane[k][2] >> x) & 1u) << 2) | (((plane[k][3] >> x) & 1u) << 3);
            if (n) atomicOr(&packed[x + r * row], n << (4 * o));
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n3; c += BUILD_BLOCK) {
        const size_t i = P * (size_t)n3 + c;
        const uint64_t w = wmask[c >> 6];
        const uint64_t bit = uint64_t(1) << (c & 63);
        if (w & bit)
            cells[i] = leaf[base[P * nw + (c >> 6)] + (uint32_t)__popcll(w & (bit - 1))];
        else
            cells[i] = make_uint2(packed[c], 0u);
    }
}

__global__ void k_leaf_counts(uint2* leaf, int64_t n_leaves, int64_t m) {
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_leaves) return;
    const uint32_t end = (l + 1 < n_leaves) ? leaf[l + 1].x : (uint32_t)m;
    leaf[l].y = end - leaf[l].x;
}

__global__ void k_split_leaf(const uint2* r, int64_t n, uint32_t* b, uint32_t* c) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint2 x = r[i];
    if (b) b[i] = x.x;
    if (c) c[i] = x.y;
}

// With packed items (`packed` non-null) the point index is taken from their
// low id_bits, else from ids (the sort's values).
__global__ void k_gather_surfels(uint32_t* ids, const uint64_t* packed, int id_bits, int64_t m, const float* xyz,
                                 const float4* un, const uint32_t* label, const uint32_t* gid, float4* spos,
                                 float4* snrm) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    uint32_t i;
    if (packed) {
        i = (uint32_t)(packed[e] & ((uint64_t(1) << id_bits) - 1));
    } else {
        i = ids[e];
    }
    const uint32_t g = gid ? gid[i] : i;
    spos[e] = make_float4(xyz[3 * (size_t)i], xyz[3 * (size_t)i + 1], xyz[3 * (size_t)i + 2], __uint_as_float(g));
    const float4 nn = un[i];
    snrm[e] = make_float4(nn.x, nn.y, nn.z, __uint_as_float(label[i]));
}

// Entry -> point table of a scene from its surfel stream.
__global__ void k_entry_points(const float4* spos, int64_t m, uint32_t* out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < m) out[e] = __float_as_uint(spos[e].w);
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------

static int validate_params(const PcrlVoxelParams* p, int32_t ratio[PCRL_MAX_LEVELS]) {
    if (!p) { set_error("build_voxels: params is NULL"); return PCRL_EINVAL; }
    if (p->n_levels < 1 || p->n_levels > PCRL_MAX_LEVELS) {
        set_error("build_voxels: n_levels must be in [1, %d], got %d", PCRL_MAX_LEVELS, p->n_levels);
        return PCRL_EINVAL;
    }
    if (p->flags & ~PCRL_VOXEL_COMPACT) {
        set_error("build_voxels: unknown flags 0x%x", (unsigned)p->flags);
        return PCRL_EINVAL;
    }
    if (!(p->surfel_radius > 0.f) || !std::isfinite(p->surfel_radius)) {
        set_error("build_voxels: surfel_radius must be positive and finite");
        return PCRL_EINVAL;
    }
    for (int i = 0; i < p->n_levels; ++i)
        if (!(p->level_size[i] > 0.f) || !std::isfinite(p->level_size[i])) {
            set_error("build_voxels: level_size[%d] must be positive and finite", i);
            return PCRL_EINVAL;
        }
    for (int i = 0; i + 1 < p->n_levels; ++i) {
        const double q = (double)p->level_size[i] / (double)p->level_size[i + 1];
        const double r = std::round(q);
        if (r < 1.0 || std::fabs(q - r) > 1e-4 * q || r > 64.0) {
            set_error("build_voxels: level_size[%d] = %g is not an integer multiple (1..64) of level_size[%d] = %g", i,
                      p->level_size[i], i + 1, p->level_size[i + 1]);
            return PCRL_EINVAL;
        }
        ratio[i] = (int32_t)r;
    }
    ratio[p->n_levels - 1] = 1;
    return PCRL_OK;
}

// Grid frame of a new scene from its parameters and point AABB.
static int make_frame(const PcrlVoxelParams* params, const int32_t ratio[PCRL_MAX_LEVELS], const IngestOut& io,
                      SceneView& v) {
    const int L = params->n_levels;
    v.nlev = L;
    v.span[L - 1] = 1;
    for (int i = L - 2; i >= 0; --i) v.span[i] = v.span[i + 1] * ratio[i];
    if (v.span[0] > (1 << 18)) {
        set_error("build_voxels: at most 2^18 leaves per coarse cell edge (got %d)", v.span[0]);
        return PCRL_EINVAL;
    }
    for (int i = 0; i < L; ++i) v.mspan[i] = (((uint64_t)1 << 40) + (uint64_t)v.span[i] - 1) / (uint64_t)v.span[i];
    for (int i = 0; i < PCRL_MAX_LEVELS; ++i) v.ratio[i] = ratio[i];
    const float h = params->level_size[L - 1];
    v.h = h;
    v.inv_h = 1.0f / h;
    const float r_s = params->surfel_radius;
    v.r_s = r_s;
    v.rs2 = r_s * r_s;
    float amax = 0.f;
    for (int a = 0; a < 3; ++a) amax = std::max(amax, std::max(std::fabs(io.lo[a]), std::fabs(io.hi[a])));
    v.pad = 1e-3f * h + 4e-6f * amax;
    const double cell0 = (double)h * v.span[0];
    for (int a = 0; a < 3; ++a) {
        const double lo = (double)io.lo[a] - r_s - v.pad - h;
        const double hi = (double)io.hi[a] + r_s + v.pad + h;
        int64_t d0 = (int64_t)std::ceil((hi - lo) / cell0);
        if (d0 < 1) d0 = 1;
        if (d0 * v.span[0] >= (int64_t)1 << 22) {
            set_error("build_voxels: leaf grid too large along axis %d (%lld leaves, max 2^22)", a,
                      (long long)(d0 * v.span[0]));
            return PCRL_EINVAL;
        }
        v.dim0[a] = (int32_t)d0;
        v.dim[a] = (int32_t)(d0 * v.span[0]);
        v.org[a] = (float)lo;
        v.hi[a] = (float)((double)v.org[a] + (double)v.dim[a] * h);
    }
    const uint64_t cells0 = (uint64_t)v.dim0[0] * v.dim0[1] * v.dim0[2];
    v.lbits[0] = bits_for(cells0 - 1);
    int key_bits = v.lbits[0];
    for (int i = 1; i < L; ++i) {
        const uint64_t r3 = (uint64_t)ratio[i - 1] * ratio[i - 1] * ratio[i - 1];
        v.lbits[i] = bits_for(r3 - 1);
        key_bits += v.lbits[i];
        v.nw[i - 1] = (int32_t)((r3 + 63) / 64);
    }
    if (key_bits > 64) {
        set_error("build_voxels: hierarchical key needs %d bits (max 64); use coarser levels", key_bits);
        return PCRL_EINVAL;
    }
    v.key_bits = key_bits;
    const double diag = std::sqrt((double)(io.hi[0] - io.lo[0]) * (io.hi[0] - io.lo[0]) +
                                  (double)(io.hi[1] - io.lo[1]) * (io.hi[1] - io.lo[1]) +
                                  (double)(io.hi[2] - io.lo[2]) * (io.hi[2] - io.lo[2]));
    v.t_eps = params->t_eps > 0.f ? params->t_eps : (float)std::max(1e-5 * diag, 1e-6);
    return PCRL_OK;
}

// What a hierarchy build produces besides its view.
struct HierBuild {
    int64_t n_entries = 0;
    int64_t n_leaves = 0;
    int64_t n_nodes[PCRL_MAX_LEVELS] = {0, 0, 0, 0};
    int64_t bytes = 0;
    uint64_t* leaf_key = nullptr;
    uint32_t* entry_point = nullptr;
    uint2* leaf_range = nullptr;
};

// Voxelise n ingested points into the frame already set in v (level-0 map,
// bricks, leaves, surfel streams).  gid: global point ids (null: 0..n-1).
static int build_hierarchy(const float* xyz, const float4* unit_nrm, const uint32_t* label, const uint32_t* gid,
                           int64_t n, hipStream_t s, bool compact, SceneView& v, DevBufs& B, DevBufs& T,
                           HierBuild& hb) {
    const int L = v.nlev;
    int rc = PCRL_OK;
    LevelShifts ls{};
    ls.nlev = L;
    {
        int acc = 0;
        for (int l = L - 1; l >= 0; --l) {
            ls.sh[l] = acc;
            acc += v.lbits[l];
        }
    }
    const uint64_t cells0 = (uint64_t)v.dim0[0] * v.dim0[1] * v.dim0[2];
    int32_t* map0 = nullptr;
    if ((rc = B.alloc(&map0, (size_t)cells0))) return rc;
    if ((rc = fill_u32((uint32_t*)map0, 0xFFFFFFFFu, (int64_t)cells0, s))) return rc;
    v.map0 = map0;
    for (int l = 0; l < PCRL_MAX_LEVELS; ++l) v.nn[l] = 0;
    hb.bytes = (int64_t)cells0 * 4;
    if (n == 0) return PCRL_OK;

    // dilated key counts and their total
    KeyParams kp{};
    kp.v = v;
    kp.r_s = v.r_s;
    kp.pad = v.pad;
    uint32_t *cnt = nullptr, *tot = nullptr, *rank0 = nullptr;
    uint8_t* occ0 = nullptr;
    if ((rc = T.alloc(&cnt, (size_t)n)) || (rc = T.alloc(&tot, 2)) || (rc = T.alloc(&rank0, (size_t)cells0)) ||
        (rc = T.alloc(&occ0, (size_t)((cells0 + 3) & ~3ull))) ||
        (rc = fill_u32((uint32_t*)occ0, 0u, (int64_t)((cells0 + 3) / 4), s)))
        return rc;
    kp.occ0 = occ0;
    hipLaunchKernelGGL(k_key_count, dim3(blocks_for(n)), dim3(BUILD_BLOCK), 0, s, kp, xyz, unit_nrm, n, cnt);
    // the key's level-0 part: the rank of the cell among the marked ones
    hipLaunchKernelGGL(k_occ0_widen, dim3(blocks_for((int64_t)cells0)), dim3(BUILD_BLOCK), 0, s, occ0,
                       (int64_t)cells0, rank0);
    if ((rc = scan_u32(rank0, rank0, (int64_t)cells0, tot + 1, s))) return rc;
    // a disk meets at most (ceil(2 (r_s + pad) / leaf) + 1)^3 leaves: when n times
    // that could reach 2^32, the counts are also summed in 64 bits
    const double span = std::ceil(2.0 * ((double)v.r_s + (double)v.pad) / (double)v.h) + 1.0;
    const bool may_wrap = (double)n * span * span * span >= 4294967280.0;
    unsigned long long* tot64 = nullptr;
    if (may_wrap) {
        if ((rc = T.alloc(&tot64, 1)) || (rc = fill_u64((uint64_t*)tot64, 0ull, 1, s))) return rc;
        hipLaunchKernelGGL(k_count_total, dim3(std::min<unsigned>(blocks_for(n), 4096u)), dim3(BUILD_BLOCK), 0, s, cnt,
                           n, tot64);
    }
    if ((rc = scan_u32(cnt, cnt, n, tot, s))) return rc;
    unsigned long long host_tot = 0;
    uint32_t host_tot2[2] = {0u, 0u};
    const bool copied = read_back(host_tot2, tot, 8, s) == PCRL_OK &&
                        (!may_wrap || read_back(&host_tot, tot64, 8, s) == PCRL_OK);
    const uint32_t host_tot32 = host_tot2[0], n_marked0 = host_tot2[1];
    if (!copied) {
        set_error("build_voxels: key count failed: %s", hipGetErrorString(hipGetLastError()));
        return PCRL_EHIP;
    }
    if (!may_wrap) host_tot = host_tot32;
    // entries are indexed with 32 bits throughout (ranges, sort values, surfel ids)
    if (host_tot > 0xFFFFFFF0ull) {
        set_error("build_voxels: %llu (leaf, point) entries exceed the 32-bit entry index; use a larger leaf size "
                  "or fewer points", host_tot);
        return PCRL_EINVAL;
    }
    const int64_t m = (int64_t)host_tot;
    hb.n_entries = m;

    // the key's level 0 numbered by rank among the marked cells when that
    // takes fewer bits than the linear cell index (fewer radix passes)
    const int lbits0 = bits_for(n_marked0 > 1 ? n_marked0 - 1 : 1);
    const bool ranked0 = lbits0 < v.lbits[0];
    const int kbits = ranked0 ? v.key_bits - v.lbits[0] + lbits0 : v.key_bits;
    uint32_t* unmap0 = nullptr;
    if (ranked0) {
        if ((rc = T.alloc(&unmap0, n_marked0))) return rc;
        hipLaunchKernelGGL(k_occ0_unmap, dim3(blocks_for((int64_t)cells0)), dim3(BUILD_BLOCK), 0, s, occ0, rank0,
                           (int64_t)cells0, unmap0);
        kp.c0 = rank0;
    }
    kp.occ0 = nullptr;

    // emit and sort (key, local point index): the point index packed below the
    // key in one 64-bit item when both fit (the stable sort on the key bits
    // then moves one 8-byte item per entry), else 64-bit keys and 32-bit ids
    int id_bits = 1;
    while (id_bits < 32 && ((uint64_t)(n > 0 ? n - 1 : 0) >> id_bits)) ++id_bits;
    const bool packed = kbits + id_bits <= 64;
    kp.id_bits = packed ? id_bits : 0;
    const int g_sh0 = ls.sh[0];
    uint64_t* keys = nullptr;
    uint32_t* ids = nullptr;  // entry -> point: packed items carry it; else the sort's values
    if (!packed && (rc = B.alloc(&ids, (size_t)m))) return rc;
    if (packed) {
        if ((rc = T.alloc(&keys, (size_t)m))) return rc;
        hipLaunchKernelGGL(k_key_emit<uint64_t>, dim3(blocks_for(n, 64)), dim3(64), 0, s, kp, xyz, unit_nrm, n, cnt,
                           keys, (uint32_t*)nullptr);
        if ((rc = radix_sort_u64_bits(keys, nullptr, m, id_bits, kbits, s))) return rc;
        for (int l = 0; l < L; ++l) ls.sh[l] += id_bits;
    } else {
        if ((rc = T.alloc(&keys, (size_t)m))) return rc;
        hipLaunchKernelGGL(k_key_emit<uint64_t>, dim3(blocks_for(n, 64)), dim3(64), 0, s, kp, xyz, unit_nrm, n, cnt,
                           keys, ids);
        if ((rc = radix_sort_u64(keys, ids, m, kbits, s))) return rc;
    }
    hb.entry_point = ids;

    // per-level node boundaries: node starts counted per tile, the tiles' counts scanned
    const int64_t n_tiles64 = (m + LINK_TILE - 1) / LINK_TILE;
    const uint32_t n_tiles = (uint32_t)n_tiles64;
    uint32_t *tiles = nullptr, *ltot = nullptr;
    if ((rc = T.alloc(&tiles, (size_t)L * n_tiles)) || (rc = T.alloc(&ltot, PCRL_MAX_LEVELS))) return rc;
    const unsigned link_blocks = (unsigned)((n_tiles64 + BUILD_BLOCK / 64 - 1) / (BUILD_BLOCK / 64));
    hipLaunchKernelGGL(k_link_count, dim3(link_blocks), dim3(BUILD_BLOCK), 0, s, keys, m, ls, tiles, n_tiles);
    for (int l = 0; l < L; ++l)
        if ((rc = scan_u32(tiles + (size_t)l * n_tiles, tiles + (size_t)l * n_tiles, n_tiles, ltot + l, s))) return rc;
    uint32_t host_nodes[PCRL_MAX_LEVELS] = {0, 0, 0, 0};
    if (read_back(host_nodes, ltot, 4 * L, s) != PCRL_OK) {
        set_error("build_voxels: level scan failed: %s", hipGetErrorString(hipGetLastError()));
        return PCRL_EHIP;
    }
    for (int l = 0; l < L; ++l) {
        hb.n_nodes[l] = host_nodes[l];
        v.nn[l] = host_nodes[l];
    }
    const int64_t n_leaves = host_nodes[L - 1];
    hb.n_leaves = n_leaves;

    HierOut ho{};
    ho.unmap0 = unmap0;
    ho.g_sh0 = g_sh0;
    ho.map0 = map0;
    for (int l = 0; l + 1 < L; ++l) {
        const size_t words = (size_t)host_nodes[l] * v.nw[l];
        uint64_t* mk = nullptr;
        uint32_t* bs = nullptr;
        uint32_t* fc = nullptr;
        if ((rc = B.alloc(&mk, words)) || (rc = B.alloc(&bs, words)) || (rc = T.alloc(&fc, host_nodes[l]))) return rc;
        if ((rc = fill_u64(mk, 0ull, (int64_t)words, s))) return rc;
        ho.mask[l] = mk;
        ho.first_child[l] = fc;
        v.mask[l] = mk;
        v.base[l] = bs;
    }
    uint2* leaf = nullptr;
    uint64_t* lkey = nullptr;
    if ((rc = B.alloc(&leaf, (size_t)n_leaves)) || (rc = B.alloc(&lkey, (size_t)n_leaves))) return rc;
    ho.leaf = leaf;
    ho.leaf_key = lkey;
    hipLaunchKernelGGL(k_link, dim3(link_blocks), dim3(BUILD_BLOCK), 0, s, keys, m, ls, v, tiles, n_tiles, ho,
                       packed ? id_bits : 0);
    for (int l = 0; l + 1 < L; ++l)
        hipLaunchKernelGGL(k_brick_base, dim3(blocks_for(host_nodes[l])), dim3(BUILD_BLOCK), 0, s, ho.mask[l],
                           ho.first_child[l], (int64_t)host_nodes[l], v.nw[l], (uint32_t*)v.base[l]);
    for (int l = 0; l + 1 < L; ++l) {
        v.baabb[l] = nullptr;
        if (v.ratio[l] > 32 || host_nodes[l] == 0) continue;
        uint32_t* ab = nullptr;
        if ((rc = B.alloc(&ab, (size_t)host_nodes[l]))) return rc;
        hipLaunchKernelGGL(k_brick_aabb, dim3(blocks_for(host_nodes[l])), dim3(BUILD_BLOCK), 0, s, ho.mask[l],
                           (int64_t)host_nodes[l], v.nw[l], v.ratio[l], ab);
        v.baabb[l] = ab;
        hb.bytes += (int64_t)host_nodes[l] * 4;
    }
    hipLaunchKernelGGL(k_leaf_counts, dim3(blocks_for(n_leaves)), dim3(BUILD_BLOCK), 0, s, leaf, n_leaves, m);
    v.leaf = leaf;
    hb.leaf_range = leaf;
    hb.leaf_key = lkey;
    // Leaf level of the traversal: a dense cell table of the leaves' parent
    // bricks (entry ranges and octant skip radii; needs the leaf ranges, so
    // after k_leaf_counts), or, when it would be too large, per-cell isotropic
    // skip radii beside the bricks' masks.
    v.ldist = nullptr;
    v.cells = nullptr;
    if (L >= 2 && host_nodes[L - 2] > 0) {
        const int r = v.ratio[L - 2];
        const int64_t r3 = (int64_t)r * r * r;
        const int64_t n_cells = (int64_t)host_nodes[L - 2] * r3;
        if (!compact && r <= 16 && n_cells * 8 <= CELL_TABLE_MAX_BYTES) {
            uint2* cells = nullptr;
            if ((rc = B.alloc(&cells, (size_t)n_cells))) return rc;
            const size_t lds = (size_t)2 * 8 * r * r * 2 + (size_t)r3 * 4;
            hipLaunchKernelGGL(k_brick_cells, dim3((unsigned)host_nodes[L - 2]), dim3(BUILD_BLOCK), lds, s,
                               ho.mask[L - 2], (const uint32_t*)v.base[L - 2], (const uint2*)leaf, v.nw[L - 2], r,
                               cells);
            v.cells = cells;
            hb.bytes += n_cells * 8;
        } else if (r >= 3 && r <= 16) {
            uint8_t* ld = nullptr;
            if ((rc = B.alloc(&ld, (size_t)n_cells))) return rc;
            const int64_t nb = host_nodes[L - 2];
            const dim3 g(blocks_for(nb, BUILD_BLOCK / 64));
            if (r == 10)
                hipLaunchKernelGGL(k_brick_dist<10>, g, dim3(BUILD_BLOCK), 0, s, ho.mask[L - 2], v.nw[L - 2], r, nb, ld);
            else if (r == 8)
                hipLaunchKernelGGL(k_brick_dist<8>, g, dim3(BUILD_BLOCK), 0, s, ho.mask[L - 2], v.nw[L - 2], r, nb, ld);
            else
                hipLaunchKernelGGL(k_brick_dist<0>, g, dim3(BUILD_BLOCK), 0, s, ho.mask[L - 2], v.nw[L - 2], r, nb, ld);
            v.ldist = ld;
            hb.bytes += n_cells;
        }
    }

    // empty-space skip radii of the level-0 grid
    {
        uint8_t *d0 = nullptr, *tmp = nullptr;
        if ((rc = B.alloc(&d0, (size_t)cells0)) || (rc = T.alloc(&tmp, (size_t)cells0))) return rc;
        const unsigned g0 = (unsigned)blocks_for((int64_t)cells0);
        hipLaunchKernelGGL(k_dist0_pass, dim3(g0), dim3(BUILD_BLOCK), 0, s, (const int32_t*)map0,
                           (const uint8_t*)nullptr, d0, v.dim0[0], v.dim0[1], v.dim0[2], 0);
        hipLaunchKernelGGL(k_dist0_pass, dim3(g0), dim3(BUILD_BLOCK), 0, s, (const int32_t*)nullptr,
                           (const uint8_t*)d0, tmp, v.dim0[0], v.dim0[1], v.dim0[2], 1);
        hipLaunchKernelGGL(k_dist0_pass, dim3(g0), dim3(BUILD_BLOCK), 0, s, (const int32_t*)nullptr,
                           (const uint8_t*)tmp, d0, v.dim0[0], v.dim0[1], v.dim0[2], 2);
        v.dist0 = d0;
        hb.bytes += (int64_t)cells0;
    }

    // surfel streams in leaf order
    float4 *spos = nullptr, *snrm = nullptr;
    if ((rc = B.alloc(&spos, (size_t)m)) || (rc = B.alloc(&snrm, (size_t)m))) return rc;
    hipLaunchKernelGGL(k_gather_surfels, dim3(blocks_for(m)), dim3(BUILD_BLOCK), 0, s, ids,
                       packed ? (const uint64_t*)keys : (const uint64_t*)nullptr, packed ? id_bits : 0, m, xyz,
                       unit_nrm, label, gid, spos, snrm);
    v.spos = spos;
    v.snrm = snrm;
    if (hipGetLastError() != hipSuccess) {
        set_error("build_voxels: kernel launch failed");
        return PCRL_EHIP;
    }
    hb.bytes += m * ((ids ? 4 : 0) + 32) + n_leaves * 16;
    for (int l = 0; l + 1 < L; ++l) hb.bytes += (int64_t)host_nodes[l] * v.nw[l] * 12;
    return PCRL_OK;
}

// Validate and normalise n points (one synchronisation).  unit_nrm is
// allocated in T.
static int ingest(const float* xyz, const float* nrm, const uint32_t* label, int64_t n, hipStream_t s, DevBufs& T,
                  float4** unit_nrm, IngestOut& io, const char* fn) {
    for (int a = 0; a < 3; ++a) { io.lo[a] = 0.f; io.hi[a] = 0.f; }
    io.max_label = 0;
    io.bad = 0;
    *unit_nrm = nullptr;
    if (n == 0) return PCRL_OK;
    int rc;
    if ((rc = T.alloc(unit_nrm, (size_t)n))) return rc;
    const unsigned nb = std::min<unsigned>(blocks_for(n), (unsigned)device_cus() * 4);
    IngestOut *partial = nullptr, *res = nullptr;
    if ((rc = T.alloc(&partial, nb)) || (rc = T.alloc(&res, 1))) return rc;
    hipLaunchKernelGGL(k_ingest, dim3(nb), dim3(BUILD_BLOCK), 0, s, xyz, nrm, label, n, *unit_nrm, partial);
    hipLaunchKernelGGL(k_ingest_final, dim3(1), dim3(BUILD_BLOCK), 0, s, partial, (int)nb, res);
    if (hipGetLastError() != hipSuccess || read_back(&io, res, sizeof io, s) != PCRL_OK) {
        set_error("%s: ingest failed: %s", fn, hipGetErrorString(hipGetLastError()));
        return PCRL_EHIP;
    }
    if (io.bad & 1u) { set_error("%s: non-finite point coordinate", fn); return PCRL_EINVAL; }
    if (io.bad & 2u) { set_error("%s: zero or non-finite normal", fn); return PCRL_EINVAL; }
    return PCRL_OK;
}

static int build_impl(const float* xyz, const float* nrm, const uint32_t* label, int64_t n,
                      const PcrlVoxelParams* params, hipStream_t s, PcrlScene* S) {
    int32_t ratio[PCRL_MAX_LEVELS] = {1, 1, 1, 1};
    PCRL_TRY(validate_params(params, ratio));
    if (n < 0 || (n > 0 && (!xyz || !nrm || !label))) {
        set_error("build_voxels: invalid point arrays (n = %lld)", (long long)n);
        return PCRL_EINVAL;
    }
    if (n > (int64_t)0x7FFFFFFF) {
        set_error("build_voxels: at most 2^31-1 points are supported");
        return PCRL_EINVAL;
    }
    (void)hipGetDevice(&S->device);
    S->bufs.stream = s;
    DevBufs T;
    T.stream = s;
    auto fail = [&](int code) { T.release(); return code; };
    float4* unit_nrm = nullptr;
    IngestOut io{};
    int rc;
    if ((rc = ingest(xyz, nrm, label, n, s, T, &unit_nrm, io, "build_voxels"))) return fail(rc);
    SceneView& v = S->view;
    if ((rc = make_frame(params, ratio, io, v))) return fail(rc);
    HierBuild hb;
    S->compact = (params->flags & PCRL_VOXEL_COMPACT) != 0;
    if ((rc = build_hierarchy(xyz, unit_nrm, label, nullptr, n, s, S->compact, v, S->bufs, T, hb))) return fail(rc);
    S->max_label = io.max_label;
    S->leaf_key = hb.leaf_key;
    S->entry_point = hb.entry_point;
    S->leaf_range = hb.leaf_range;
    PcrlSceneInfo& info = S->info;
    info.n_points = n;
    info.n_entries = hb.n_entries;
    info.n_leaves = hb.n_leaves;
    for (int l = 0; l < PCRL_MAX_LEVELS; ++l) info.n_nodes[l] = hb.n_nodes[l];
    info.max_label = (int32_t)io.max_label;
    info.n_levels = params->n_levels;
    for (int a = 0; a < 3; ++a) {
        info.dims[a] = v.dim[a];
        info.dims0[a] = v.dim0[a];
        info.origin[a] = v.org[a];
        info.aabb[a] = io.lo[a];
        info.aabb[3 + a] = io.hi[a];
    }
    info.leaf_size = v.h;
    info.surfel_radius = v.r_s;
    info.t_eps = v.t_eps;
    info.key_bits = v.key_bits;
    info.device_bytes = hb.bytes;
    info.n_dynamic = 0;
    info.epoch = 0;
    T.release();
    return PCRL_OK;
}

// Overlay of dynamic points on the frame of `base`.
static int overlay_impl(PcrlScene* S, const uint32_t* gid, const float* xyz, const float* nrm, const uint32_t* label,
                        int64_t n, hipStream_t s) {
    auto ov = std::make_shared<Overlay>();
    ov->bufs.stream = s;
    DevBufs T;
    T.stream = s;
    auto fail = [&](int code) { T.release(); return code; };
    float4* unit_nrm = nullptr;
    IngestOut io{};
    int rc;
    if ((rc = ingest(xyz, nrm, label, n, s, T, &unit_nrm, io, "update_points"))) return fail(rc);
    const SceneView& bv = S->view;
    // every dynamic disk, dilated as in disk_leaf_box, must lie inside the base grid (no leaf clamped)
    for (int a = 0; a < 3; ++a) {
        const float m = bv.r_s + 2.f * bv.pad;
        if (n > 0 && (io.lo[a] - m <= bv.org[a] || io.hi[a] + m >= bv.hi[a])) {
            set_error("update_points: dynamic points leave the scene grid along axis %d ([%g, %g] vs grid [%g, %g])", a,
                      io.lo[a], io.hi[a], bv.org[a], bv.hi[a]);
            return fail(PCRL_EINVAL);
        }
    }
    SceneView v = bv;  // same frame: origin, levels, padding, t_eps
    v.map0 = nullptr;
    for (int l = 0; l + 1 < PCRL_MAX_LEVELS; ++l) {
        v.mask[l] = nullptr;
        v.base[l] = nullptr;
        v.baabb[l] = nullptr;
    }
    v.leaf = nullptr;
    v.ldist = nullptr;
    v.dist0 = nullptr;
    v.cells = nullptr;
    v.spos = v.snrm = nullptr;
    HierBuild hb;
    if ((rc = build_hierarchy(xyz, unit_nrm, label, gid, n, s, S->compact, v, ov->bufs, T, hb))) return fail(rc);
    ov->view = v;
    ov->n_points = n;
    ov->n_entries = hb.n_entries;
    ov->max_label = io.max_label;
    ov->bytes = hb.bytes;
    T.release();
    ov->epoch = S->info.epoch + 1;
    S->info.epoch = ov->epoch;
    S->info.n_dynamic = n;
    S->overlay = n > 0 ? ov : nullptr;
    return PCRL_OK;
}

}  // namespace pcrl

using namespace pcrl;

extern "C" int build_voxels(const float* xyz, const float* normal, const uint32_t* label, int64_t n_points,
                            const PcrlVoxelParams* params, pcrl_stream_t stream, PcrlScene** out) {
    clear_error();
    if (!out) {
        set_error("build_voxels: out is NULL");
        return PCRL_EINVAL;
    }
    *out = nullptr;
    PcrlScene* S = new (std::nothrow) PcrlScene();
    if (!S) {
        set_error("build_voxels: host allocation failed");
        return PCRL_ENOMEM;
    }
    int rc = build_impl(xyz, normal, label, n_points, params, (hipStream_t)stream, S);
    if (rc != PCRL_OK) {
        S->bufs.release();
        delete S;
        return rc;
    }
    *out = S;
    return PCRL_OK;
}

extern "C" int update_points(PcrlScene* scene, const uint32_t* ids, const float* xyz, const float* normal,
                             const uint32_t* label, int64_t n, pcrl_stream_t stream) {
    clear_error();
    if (!scene || n < 0 || (n > 0 && (!ids || !xyz || !normal || !label)) || n > (int64_t)0x7FFFFFFF) {
        set_error("update_points: invalid arguments");
        return PCRL_EINVAL;
    }
    return overlay_impl(scene, ids, xyz, normal, label, n, (hipStream_t)stream);
}

extern "C" int scene_info(const PcrlScene* scene, PcrlSceneInfo* out) {
    clear_error();
    if (!scene || !out) {
        set_error("scene_info: NULL argument");
        return PCRL_EINVAL;
    }
    *out = scene->info;
    if (scene->overlay) out->device_bytes += scene->overlay->bytes;
    return PCRL_OK;
}

extern "C" int scene_leaf_table(const PcrlScene* scene, uint64_t* leaf_key, uint32_t* leaf_begin,
                                uint32_t* leaf_count, uint32_t* entry_point, pcrl_stream_t stream) {
    clear_error();
    if (!scene) {
        set_error("scene_leaf_table: scene is NULL");
        return PCRL_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int64_t nl = scene->info.n_leaves;
    const int64_t m = scene->info.n_entries;
    if (leaf_key && nl)
        PCRL_TRY_HIP(hipMemcpyAsync(leaf_key, scene->leaf_key, (size_t)nl * 8, hipMemcpyDeviceToDevice, s));
    if ((leaf_begin || leaf_count) && nl) {
        hipLaunchKernelGGL(k_split_leaf, dim3(blocks_for(nl)), dim3(BUILD_BLOCK), 0, s, scene->leaf_range, nl,
                           leaf_begin, leaf_count);
        PCRL_TRY_HIP(hipGetLastError());
    }
    if (entry_point && m) {
        if (scene->entry_point) {
            PCRL_TRY_HIP(hipMemcpyAsync(entry_point, scene->entry_point, (size_t)m * 4, hipMemcpyDeviceToDevice, s));
        } else {
            // the point id rides in the surfel stream (x, y, z, id)
            hipLaunchKernelGGL(k_entry_points, dim3(blocks_for(m)), dim3(BUILD_BLOCK), 0, s, scene->view.spos, m,
                               entry_point);
            PCRL_TRY_HIP(hipGetLastError());
        }
    }
    PCRL_TRY_HIP(hipStreamSynchronize(s));
    return PCRL_OK;
}

extern "C" int release_scene(PcrlScene* scene) {
    clear_error();
    if (!scene) return PCRL_OK;
    // launches on any stream may still read the scene (their release does not
    // wait for them), and the build stream may no longer exist: finish all
    // device work, then free on the null stream
    (void)hipDeviceSynchronize();
    scene->overlay.reset();
    scene->bufs.stream = nullptr;
    scene->bufs.release();
    delete scene;
    return PCRL_OK;
}
