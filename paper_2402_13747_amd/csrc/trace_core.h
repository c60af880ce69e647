// trace_core.h -- the per-ray bounce body shared by the single-launch and the
// batched kernels (paper, Section 2.2): hierarchical DDA, surfel intersection,
// RX reception, specular reflection and survivor compaction.  Both kernels
// run exactly this code, so a query gives bitwise the same result alone or
// in a batch.
#pragma once

#include "internal.h"

namespace pcrl {

constexpr int TRACE_BLOCK = 256;
constexpr uint32_t NO_HIT = 0xFFFFFFFFu;

// Statistics of the PCRL_LAUNCH_STATS kernel variant.  ST_BYTES is the exact
// algorithmic traffic of the trace kernels: 4 B per level-0 map read, 8 B per
// brick mask word (+4 B base when the bit is set), 8 B per leaf range, 32 B
// per surfel tested, 36 B of ray state read per segment after the first,
// 36 B of ray state + 16 B of history per reflection, 16 B per record.
enum StatSlot {
    ST_SEGMENTS = 0, ST_DDA, ST_LEAVES, ST_NODES, ST_TESTS, ST_HITS, ST_BYTES, ST_EMPTY_LEAF, ST_UNIFORM,
    ST_WAVE_DDA, ST_WAVE_TESTS, ST_COUNT
};
typedef unsigned long long stat_t;
static_assert(ST_COUNT <= PCRL_NSTATS, "device statistics buffer too small");

struct TraceArgs {
    SceneView v;
    SceneView ov;           // overlay of dynamic points (valid when has_ov)
    int32_t has_ov;
    const float* tx;
    const float* rx;
    const float* dirs;      // [n_rays][3] launch directions (the caller's, or the materialised Fibonacci lattice)
    const uint32_t* perm;   // null, or bounce-0 order of the directions
    const uint32_t* order;  // null, or for bounces >= 1: slot i reads the previous bounce's output order[i]
    uint16_t* okeys;        // with order: coherence bucket of each survivor written by a bounce
    uint32_t* opos;         // with order: the survivor's position among its bucket's survivors
    uint32_t* ocnt;         // with order: [K][65536] survivors per bucket, per bounce
    float3 klo, kscale;     // bucket grid: origin and cells per metre (16 per axis over the grid)
    int32_t n_rx;
    int32_t K;
    uint32_t n_rays;
    uint32_t n_total;
    float sig_c;            // sigma * alpha / sqrt(3)
    float4* buf_o[2];       // ray state (o, L); bounce b writes [b & 1], reads [(b & 1) ^ 1]
    float4* buf_d[2];       // (d, last hit id bits)
    uint32_t* buf_g[2];     // global ray id, NO_HIT for an empty slot
    uint32_t* counters;     // [b] live rays entering bounce b, [K+2] records
    float4* hist;
    uint4* rec;
    uint32_t rec_cap;
    int32_t* hit_id;
    float* hit_t;
    unsigned long long* stats;
};

// Ping-pong ray buffers of bounce b, chosen by selects: a runtime index into
// the argument struct's arrays would force the whole struct into scratch.
__device__ __forceinline__ float4* ray_o(const TraceArgs& a, int k) { return (k & 1) ? a.buf_o[1] : a.buf_o[0]; }
__device__ __forceinline__ float4* ray_d(const TraceArgs& a, int k) { return (k & 1) ? a.buf_d[1] : a.buf_d[0]; }
__device__ __forceinline__ uint32_t* ray_g(const TraceArgs& a, int k) { return (k & 1) ? a.buf_g[1] : a.buf_g[0]; }

struct Hit {
    uint32_t id;
    uint32_t lab;
    float t;
    float nx, ny, nz;
};

// Level-indexed constants for a per-lane level index.  The values are
// selected arithmetically after loading all NL of them: a select between
// loads of argument fields would become a pointer select into the argument
// struct and keep the struct in scratch memory.
template <int NL>
__device__ __forceinline__ int span_at(const SceneView& v, int lvl) {
    int s = 0;
#pragma unroll
    for (int i = 0; i < NL; ++i) s += v.span[i] * (int)(lvl == i);
    return s;
}

template <int NL>
__device__ __forceinline__ uint64_t mspan_at(const SceneView& v, int lvl) {
    uint64_t m = 0;
#pragma unroll
    for (int i = 0; i < NL; ++i) m += v.mspan[i] * (uint64_t)(lvl == i);
    return m;
}

// Box word that no child lies outside of (lo 0, hi 31 on every axis): the
// value used where a brick has no box.
constexpr uint32_t NO_BOX = (31u << 15) | (31u << 20) | (31u << 25);

// Descend from level 0 to level TO (< nlev) for leaf cell c.  Returns the
// level at which the path is empty, or TO + 1 when the level-TO node exists
// (its index in `node`).  Quotients c / span[i] use the precomputed magics.
// BOX: `box` receives the occupied-children box of the brick that holds the
// empty cell (empty at level i >= 1: the level-(i-1) brick), or of the
// level-TO node's own brick when the path exists (TO < nlev - 1); NO_BOX
// where there is none.  The box of a brick is loaded with its mask word.
template <bool STATS, int TO, bool BOX = false>
__device__ __forceinline__ int descend(const SceneView& v, const int c[3], uint32_t& node, int& skip0,
                                       stat_t* cnt, uint32_t* box = nullptr) {
    int p[3] = {span_div(c[0], v.mspan[0]), span_div(c[1], v.mspan[0]), span_div(c[2], v.mspan[0])};
    const size_t i0 = (size_t)p[0] + (size_t)v.dim0[0] * ((size_t)p[1] + (size_t)v.dim0[1] * p[2]);
    // the level-0 node and the cell's skip radius are loaded together
    const int32_t n0 = v.map0[i0];
    const int d0 = v.dist0 ? (int)v.dist0[i0] : 1;
    if (STATS) {
        ++cnt[ST_NODES];
        cnt[ST_BYTES] += (n0 < 0 && v.dist0) ? 5 : 4;
    }
    if (BOX) *box = NO_BOX;
    if (n0 < 0 || (uint32_t)n0 >= v.nn[0]) {
        skip0 = d0;
        return 0;
    }
    uint32_t n = (uint32_t)n0;
#pragma unroll
    for (int i = 1; i <= TO; ++i) {
        const int q[3] = {span_div(c[0], v.mspan[i]), span_div(c[1], v.mspan[i]), span_div(c[2], v.mspan[i])};
        const int r = v.ratio[i - 1];
        const int loc = (q[0] - r * p[0]) + r * ((q[1] - r * p[1]) + r * (q[2] - r * p[2]));
        const size_t wi = (size_t)n * v.nw[i - 1] + (loc >> 6);
        const uint64_t w = v.mask[i - 1][wi];
        const uint32_t bx = (BOX && v.baabb[i - 1]) ? v.baabb[i - 1][n] : NO_BOX;
        const uint64_t bit = uint64_t(1) << (loc & 63);
        if (STATS) {
            ++cnt[ST_NODES];
            cnt[ST_BYTES] += ((w & bit) ? 12 : 8) + ((BOX && v.baabb[i - 1]) ? 4 : 0);
        }
        if (!(w & bit)) {
            if (BOX) *box = bx;
            return i;
        }
        n = v.base[i - 1][wi] + (uint32_t)__popcll(w & (bit - 1));
        if (n >= v.nn[i]) return i;
        p[0] = q[0];
        p[1] = q[1];
        p[2] = q[2];
    }
    node = n;
    if constexpr (BOX) {
        if (v.baabb[TO]) {
            *box = v.baabb[TO][n];
            if (STATS) cnt[ST_BYTES] += 4;
        }
    }
    return TO + 1;
}

// Per-wave LDS of the cooperative leaf test: the rays of the wave's lanes and,
// per lane, the pending leaf, its running nearest hit and the hit's normal.
struct alignas(16) LeafTestLds {
    float4 hn[64];                 // normal + label bits of a new nearest hit
    unsigned long long best[64];   // (t bits << 32) | point id: lexicographic min = nearest, ties by id
    float ox[64], oy[64], oz[64], dx[64], dy[64], dz[64];
    uint32_t last[64];             // point the ray left (excluded)
    uint32_t begin[64];            // first entry of the lane's pending leaf
    uint32_t excl[64];             // exclusive prefix of the pending entry counts over lanes
    uint32_t win[64];              // a test of this pass found a new nearest hit for the lane
    int32_t mark[64];              // lane whose entries start at this position of the current chunk
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Inclusive wave64 scans on the VALU through DPP row shifts and row
// broadcasts (no LDS round trips).  Every lane of the wave must be active.
// Lanes shifted in from outside a row read 0, the identity of both scans
// (max is used on non-negative values only).
__device__ __forceinline__ uint32_t wave_scan_add_dpp(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
    return x;
}

__device__ __forceinline__ int wave_scan_max_dpp(int x) {
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false));
    return x;
}

// Test the pending leaves of all lanes of the wave together: the wave's
// (lane, entry) pairs are dealt out 64 at a time, so every lane tests a
// surfel in every pass whatever the leaves' sizes, and consecutive lanes read
// consecutive entries of a leaf.  Each pair is tested against its owner
// lane's ray and the owner's nearest hit is the minimum of (t, id) over its
// previous hit and all accepted pairs: the same result as testing the
// leaf's entries one after another in the owner's lane.  Called by every
// lane of the wave; `has` marks lanes with a pending leaf (entries r).
template <bool STATS>
__device__ __forceinline__ void leaf_tests(const SceneView& v, LeafTestLds& W, bool has, uint2 r, Hit& hit,
                                           stat_t cnt[ST_COUNT]) {
    const uint32_t lane = lane_id();
    const uint32_t n = has ? r.y : 0u;
    const uint32_t incl = wave_scan_add_dpp(n);
    const uint32_t total = __builtin_amdgcn_readfirstlane(__shfl(incl, 63, 64));
    const uint32_t excl = incl - n;
    W.begin[lane] = r.x;
    W.excl[lane] = excl;
    W.best[lane] = ((unsigned long long)__float_as_uint(hit.t) << 32) | hit.id;
    W.win[lane] = 0u;
    for (uint32_t base = 0; base < total; base += 64) {
        if (STATS && lane == 0) ++cnt[ST_WAVE_TESTS];
        W.mark[lane] = -1;
        wave_sync();
        if (n && excl < base + 64 && incl > base) W.mark[excl > base ? excl - base : 0] = (int)lane;
        wave_sync();
        const int own = wave_scan_max_dpp(W.mark[lane] + 1) - 1;  // marks + 1 >= 0
        const uint32_t pi = base + lane;
        bool ok = false;
        unsigned long long cand = 0;
        float4 N = make_float4(0.f, 0.f, 0.f, 0.f);
        if (pi < total && own >= 0) {  // own >= 0 always: the pair at `base` has an owner
            const uint32_t k = W.begin[own] + (pi - W.excl[own]);
            const float4 P4 = v.spos[k];
            N = v.snrm[k];
            const float o0 = W.ox[own], o1 = W.oy[own], o2 = W.oz[own];
            const float d0 = W.dx[own], d1 = W.dy[own], d2 = W.dz[own];
            const uint32_t id = __float_as_uint(P4.w);
            const float wx = P4.x - o0, wy = P4.y - o1, wz = P4.z - o2;
            const float den = d0 * N.x + d1 * N.y + d2 * N.z;
            const float num = wx * N.x + wy * N.y + wz * N.z;
            const float t = num * __builtin_amdgcn_rcpf(den);
            const float qx = t * d0 - wx, qy = t * d1 - wy, qz = t * d2 - wz;
            const float dist2 = qx * qx + qy * qy + qz * qz;
            ok = fabsf(den) > 1e-7f && t > v.t_eps && id != W.last[own] && dist2 <= v.rs2;
            if (ok) {
                cand = ((unsigned long long)__float_as_uint(t) << 32) | id;
                atomicMin(&W.best[own], cand);
            }
        }
        wave_sync();
        // the pair that holds the minimum publishes the hit's normal and label
        // (pairs with equal (t, id) are the same point: same normal)
        if (ok && W.best[own] == cand) {
            W.hn[own] = N;
            W.win[own] = 1u;
        }
        wave_sync();
    }
    if (has && W.win[lane]) {
        const unsigned long long b = W.best[lane];
        const float4 hn = W.hn[lane];
        hit.t = __uint_as_float((uint32_t)(b >> 32));
        hit.id = (uint32_t)b;
        hit.nx = hn.x;
        hit.ny = hn.y;
        hit.nz = hn.z;
        hit.lab = __float_as_uint(hn.w);
    }
    wave_sync();
}

// DDA state of one lane's segment.
struct Seg {
    float inv[3];   // 1 / d (0 on axes the ray does not move along)
    int c[3];       // current leaf cell
    int cq[3];      // parent cell of the cached descent
    int cres;       // cached descent result
    int cskip0;     // cached skip radius of an empty level-0 cell (cres == 0)
    uint32_t cnode; // cached parent node
    uint32_t cbox;  // cached box word: of the parent node's brick (cres > P), or of the brick holding
                    // the empty cell (0 < cres <= P)
    int it;         // DDA steps taken
    int oct_shift;  // 4 x the ray's direction octant (bit a: component a negative)
};

__device__ __forceinline__ int dir_step(float x) { return x > 0.f ? 1 : (x < 0.f ? -1 : 0); }

// Start a segment from o along d: clip to the grid and find the first cell.
// Returns false when the ray misses the grid.
__device__ __forceinline__ bool seg_begin(const SceneView& v, const float o[3], const float d[3], Seg& S) {
    float t0 = 0.f, t1 = INFINITY;
    // slab test; both faces are read on every path (a choice between two
    // argument fields would be turned into a pointer select into the argument
    // struct, which then stays in scratch memory)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo_a = v.org[a], hi_a = v.hi[a];
        if (d[a] != 0.f) {
            S.inv[a] = 1.0f / d[a];
            const float ta = (lo_a - o[a]) * S.inv[a], tb = (hi_a - o[a]) * S.inv[a];
            t0 = fmaxf(t0, fminf(ta, tb));
            t1 = fminf(t1, fmaxf(ta, tb));
        } else {
            S.inv[a] = 0.f;
            if (o[a] < lo_a || o[a] > hi_a) t1 = -1.f;
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int ci = (int)floorf((o[a] + t0 * d[a] - v.org[a]) * v.inv_h);
        S.c[a] = min(max(ci, 0), v.dim[a] - 1);
        S.cq[a] = -1;
    }
    S.cres = 0;
    S.cskip0 = 1;
    S.cbox = NO_BOX;
    S.oct_shift = 4 * ((d[0] < 0.f ? 1 : 0) | (d[1] < 0.f ? 2 : 0) | (d[2] < 0.f ? 4 : 0));
    S.cnode = 0;
    S.it = 0;
    return t0 <= t1;
}

__device__ __forceinline__ void stage_ray(LeafTestLds& W, const float o[3], const float d[3], uint32_t last) {
    const uint32_t lane = lane_id();
    W.ox[lane] = o[0];
    W.oy[lane] = o[1];
    W.oz[lane] = o[2];
    W.dx[lane] = d[0];
    W.dy[lane] = d[1];
    W.dz[lane] = d[2];
    W.last[lane] = last;
}

__device__ __forceinline__ void hit_reset(Hit& hit) {
    hit.id = NO_HIT;
    hit.t = INFINITY;
    hit.lab = 0;
    hit.nx = hit.ny = hit.nz = 0.f;
}

// Whether local child coordinates (x, y, z) of a brick lie outside its box word.
__device__ __forceinline__ bool box_outside(uint32_t box, int x, int y, int z) {
    return x < (int)(box & 31u) || y < (int)((box >> 5) & 31u) || z < (int)((box >> 10) & 31u) ||
           x > (int)((box >> 15) & 31u) || y > (int)((box >> 20) & 31u) || z > (int)((box >> 25) & 31u);
}

// What the DDA found at the current cell: an occupied leaf (lvl == NL, its
// node and entry range) or an empty cell of level lvl with the empty region
// around it that the ray may skip.
struct DdaCell {
    uint32_t node;
    uint2 range;    // entries of an occupied leaf
    int skip;       // > 1: an empty cube of 2 skip - 1 units centred on the unit holding c
    int oct;        // > 1: an empty box of oct leaves from c along the ray's octant; -1: an empty cell
                    // of level lvl whose brick's occupied-children box is `node` (a box word)
    int unit;       // edge of a skip unit in leaves (1, or a level-0 cell)
    int lvl;        // level of the empty cell containing c, or NL for an occupied leaf
};

__device__ __forceinline__ void dda_cell_reset(DdaCell& k) {
    k.node = 0;
    k.range = make_uint2(0u, 0u);
    k.skip = 1;
    k.oct = 1;
    k.unit = 1;
    k.lvl = 0;
}

// Look the lane's current cell S.c up top-down through a hierarchy of NL
// levels (NL == v.nlev).  Per lane; no cross-lane operations.
template <bool STATS, int NL, bool BX = true>
__device__ __forceinline__ void dda_locate(const SceneView& v, Seg& S, DdaCell& k, stat_t* cnt) {
    constexpr int L = NL;
    constexpr int P = L - 2;  // level of the leaves' parents (-1: single-level grid)
    const int* c = S.c;
    if constexpr (P < 0) {
        const size_t i0 = (size_t)c[0] + (size_t)v.dim0[0] * ((size_t)c[1] + (size_t)v.dim0[1] * c[2]);
        const int32_t n0 = v.map0[i0];
        const int d0 = v.dist0 ? (int)v.dist0[i0] : 1;
        if (STATS) {
            ++cnt[ST_NODES];
            cnt[ST_BYTES] += (n0 < 0 && v.dist0) ? 5 : 4;
        }
        k.lvl = (n0 < 0 || (uint32_t)n0 >= v.nn[0]) ? 0 : L;
        k.node = (uint32_t)n0;
        if (k.lvl == 0) k.skip = max(1, d0);
        if (k.lvl == L) {
            k.range = v.leaf[k.node];
            if (STATS) cnt[ST_BYTES] += 8;
        }
    } else {
        // the descent from level 0 runs only when the parent cell changes
        const int q[3] = {span_div(c[0], v.mspan[P]), span_div(c[1], v.mspan[P]), span_div(c[2], v.mspan[P])};
        if (q[0] != S.cq[0] || q[1] != S.cq[1] || q[2] != S.cq[2]) {
            S.cq[0] = q[0];
            S.cq[1] = q[1];
            S.cq[2] = q[2];
            S.cres = descend<STATS, P, BX>(v, c, S.cnode, S.cskip0, cnt, &S.cbox);
        }
        if (S.cres <= P) {
            k.lvl = S.cres;
            if (k.lvl == 0) {
                // empty level-0 cell: the cube of radius cskip0 - 1 level-0 cells around it is empty
                k.skip = max(1, S.cskip0);
                k.unit = v.span[0];
            } else if (BX && S.cbox != NO_BOX) {
                // empty cell of a brick: the rest of the brick outside its box may be empty too
                k.oct = -1;
                k.node = S.cbox;
            }
        } else if (BX && S.cbox != NO_BOX && !v.cells &&
                   box_outside(S.cbox, c[0] - v.ratio[P] * q[0], c[1] - v.ratio[P] * q[1],
                               c[2] - v.ratio[P] * q[2])) {
            // a leaf outside its parent brick's occupied box: empty, no lookup
            k.lvl = L - 1;
            k.oct = -1;
            k.node = S.cbox;
        } else if (v.cells) {
            // one load: the leaf's entry range, or its skip radius
            const int r = v.ratio[P];
            const int loc = (c[0] - r * q[0]) + r * ((c[1] - r * q[1]) + r * (c[2] - r * q[2]));
            const uint2 cl = v.cells[(size_t)S.cnode * (size_t)(r * r * r) + loc];
            if (STATS) {
                ++cnt[ST_NODES];
                cnt[ST_BYTES] += 8;
            }
            if (cl.y) {
                k.lvl = L;
                k.range = cl;
                k.node = cl.x;
            } else {
                // empty leaf: the box of oct cells from it along the ray's octant is empty
                k.lvl = L - 1;
                k.oct = (int)((cl.x >> S.oct_shift) & 15u);
            }
        } else {
            const int r = v.ratio[P];
            const int loc = (c[0] - r * q[0]) + r * ((c[1] - r * q[1]) + r * (c[2] - r * q[2]));
            const size_t wi = (size_t)S.cnode * v.nw[P] + (loc >> 6);
            // the mask word, the word's child base and the leaf's skip radius are
            // loaded together (one memory round trip); only one of the last two is used
            const uint64_t w = v.mask[P][wi];
            const uint32_t wbase = v.base[P][wi];
            const int ld = v.ldist ? (int)v.ldist[(size_t)S.cnode * (size_t)(r * r * r) + loc] : 1;
            const uint64_t bit = uint64_t(1) << (loc & 63);
            if (STATS) {
                ++cnt[ST_NODES];
                cnt[ST_BYTES] += (w & bit) ? 12 : (v.ldist ? 9 : 8);
            }
            k.lvl = L - 1;
            if (w & bit) {
                k.node = wbase + (uint32_t)__popcll(w & (bit - 1));
                if (k.node < v.nn[L - 1]) {
                    k.lvl = L;
                    k.range = v.leaf[k.node];
                    if (STATS) cnt[ST_BYTES] += 8;
                }
            } else {
                // empty leaf: the whole cube of radius skip - 1 around it is empty
                k.skip = max(1, ld);
            }
        }
    }
}

// Move the lane past the cell (or empty region) `k` describes: S.c becomes
// the next cell along the ray, and `te` the distance at which the ray enters
// it.  Clears `walking` when the next cell starts beyond t_stop or the ray
// leaves the grid.  Per lane; no cross-lane operations.
template <int NL, bool BX = true>
__device__ __forceinline__ void dda_advance(const SceneView& v, bool& walking, const float o[3], const float d[3],
                                            Seg& S, const DdaCell& k, bool at_leaf, float t_stop, float& te) {
    int* c = S.c;
    const int Sz = at_leaf ? 1 : span_at<NL>(v, k.lvl);
    // An empty cell of a brick with an occupied-children box: when the cell is
    // outside the box along some axes, each such axis a bounds an empty slab
    // of the brick (the brick cut at the box's face on a); the ray crosses the
    // slab that it leaves last in one step.
    // The slab along a ends at the box's near face when the ray moves towards
    // the box, else at the brick's face; the ray leaves the slab at
    // min(that face, T) with T its exit from the whole brick.
    int slab = -1, bs = 0;
    bool below = false;
    if (BX && NL > 1 && k.oct < 0) {
        const int us = span_at<NL>(v, k.lvl);
        bs = span_at<NL>(v, k.lvl - 1);
        const uint64_t um = mspan_at<NL>(v, k.lvl), bm = mspan_at<NL>(v, k.lvl - 1);
        const uint32_t box = k.node;
        float T = INFINITY;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int blo = span_div(c[a], bm) * bs;
            if (d[a] != 0.f) T = fminf(T, ((float)(d[a] > 0.f ? blo + bs : blo) * v.h + v.org[a] - o[a]) * S.inv[a]);
        }
        float best = -INFINITY;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int blo = span_div(c[a], bm) * bs;
            const int lc = span_div(c[a] - blo, um);
            const int alo = (int)((box >> (5 * a)) & 31u), ahi = (int)((box >> (15 + 5 * a)) & 31u);
            float t_a = T;
            if (d[a] > 0.f && lc < alo) t_a = fminf(T, ((float)(blo + alo * us) * v.h + v.org[a] - o[a]) * S.inv[a]);
            if (d[a] < 0.f && lc > ahi)
                t_a = fminf(T, ((float)(blo + (ahi + 1) * us) * v.h + v.org[a] - o[a]) * S.inv[a]);
            if ((lc < alo || lc > ahi) && t_a > best) {
                best = t_a;
                slab = a;
                below = lc < alo;
            }
        }
    }
    // exit of the current cell (size Sz leaves)
    int lo[3], hi[3];
    te = INFINITY;
    int axis = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (BX && slab >= 0) {
            // the brick's range, cut at the box's face along the slab axis
            lo[a] = span_div(c[a], mspan_at<NL>(v, k.lvl - 1)) * bs;
            hi[a] = lo[a] + bs;
            if (a == slab) {
                const int us = span_at<NL>(v, k.lvl);
                const int alo = (int)((k.node >> (5 * a)) & 31u), ahi = (int)((k.node >> (15 + 5 * a)) & 31u);
                if (below)
                    hi[a] = lo[a] + alo * us;
                else
                    lo[a] = lo[a] + (ahi + 1) * us;
            }
        } else if (k.oct > 1) {
            // the octant box (inside its brick)
            lo[a] = d[a] < 0.f ? c[a] - (k.oct - 1) : c[a];
            hi[a] = d[a] < 0.f ? c[a] + 1 : c[a] + k.oct;
        } else if (k.skip > 1) {
            // the skip cube, clipped to the grid (beyond it the ray leaves)
            const int uc = (k.unit == 1) ? c[a] : span_div(c[a], v.mspan[0]);
            lo[a] = max((uc - (k.skip - 1)) * k.unit, 0);
            hi[a] = min((uc + k.skip) * k.unit, v.dim[a]);
        } else {
            lo[a] = (Sz == 1) ? c[a] : span_div(c[a], mspan_at<NL>(v, k.lvl)) * Sz;
            hi[a] = lo[a] + Sz;
        }
        float ta = INFINITY;
        if (d[a] > 0.f)
            ta = ((float)hi[a] * v.h + v.org[a] - o[a]) * S.inv[a];
        else if (d[a] < 0.f)
            ta = ((float)lo[a] * v.h + v.org[a] - o[a]) * S.inv[a];
        if (ta < te) {
            te = ta;
            axis = a;
        }
    }
    // next cell along the exit axis (selects, no dynamic indexing of private arrays)
    int nc = 0, dim_ax = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (a == axis) {
            nc = d[a] > 0.f ? hi[a] : lo[a] - 1;
            dim_ax = v.dim[a];
        }
    const int max_iter = v.dim[0] + v.dim[1] + v.dim[2] + 8;
    // no later cell can hold a nearer hit; or the ray leaves the grid
    if (te > t_stop || nc < 0 || nc >= dim_ax || ++S.it >= max_iter) {
        walking = false;
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a == axis) {
                c[a] = nc;
                continue;
            }
            const int sg = dir_step(d[a]);
            if (sg == 0) continue;
            int j = (int)floorf((o[a] + te * d[a] - v.org[a]) * v.inv_h);
            j = min(max(j, lo[a]), hi[a] - 1);
            j = sg > 0 ? max(j, c[a]) : min(j, c[a]);
            c[a] = j;
        }
    }
}

// One DDA step of every walking lane through a hierarchy of NL levels
// (NL == v.nlev): look the current cell up top-down, test an occupied leaf
// (cooperatively, with the other lanes' leaves), then move to the next cell
// or stop.  Called by every lane of the wave; `walking` is cleared when the
// lane's segment ends.  The lane's ray must be staged in W.
template <bool STATS, int NL, bool BX = true>
__device__ __forceinline__ void dda_step(const SceneView& v, LeafTestLds& W, bool& walking, const float o[3],
                                         const float d[3], Hit& hit, Seg& S, stat_t cnt[ST_COUNT]) {
    constexpr int L = NL;
    DdaCell k;
    dda_cell_reset(k);
    if (walking) dda_locate<STATS, NL, BX>(v, S, k, cnt);
    const bool at_leaf = walking && k.lvl == L;
    if (STATS) {
        const uint64_t m_walk = __ballot(walking);
        if (walking) {
            ++cnt[ST_DDA];
            if (k.lvl == L - 1 && L > 1) ++cnt[ST_EMPTY_LEAF];
        }
        // leaf visits where every lane of the wave still walking is in the same leaf
        const uint64_t m_leaf = __ballot(at_leaf);
        const int first = m_leaf ? __ffsll((long long)m_leaf) - 1 : 0;
        const uint32_t lead = __shfl(k.node, first, 64);
        if (at_leaf && __ballot(at_leaf && k.node == lead) == m_walk) ++cnt[ST_UNIFORM];
        if (lane_id() == 0) ++cnt[ST_WAVE_DDA];
    }
    if (STATS && at_leaf) {
        ++cnt[ST_LEAVES];
        cnt[ST_TESTS] += k.range.y;
        cnt[ST_BYTES] += 32ull * k.range.y;
    }
    if (__ballot(at_leaf && k.range.y != 0u)) leaf_tests<STATS>(v, W, at_leaf, k.range, hit, cnt);
    if (walking) {
        float te;
        dda_advance<NL, BX>(v, walking, o, d, S, k, at_leaf, hit.t + (hit.t * 4e-6f + 1e-3f * v.h), te);
    }
}

// One whole segment of every active lane (lanes with `active` false only
// help with the cooperative leaf tests) through the base hierarchy, or the
// overlay when OVL.  The hierarchy is picked by a compile-time member, never
// by a runtime reference: two such calls merged over a reference would keep
// the whole argument struct in scratch memory.  Called by every lane of the
// wave.
template <bool STATS, int NL, bool OVL, bool BX = true>
__device__ __forceinline__ void trace_segment(const TraceArgs& a, LeafTestLds& W, bool active, const float o[3],
                                              const float d[3], Hit& hit, stat_t cnt[ST_COUNT]) {
    const SceneView& v = OVL ? a.ov : a.v;
    Seg S;
    bool walking = seg_begin(v, o, d, S) && active;
    while (__ballot(walking)) dda_step<STATS, NL, BX>(v, W, walking, o, d, hit, S, cnt);
}

// Load slot i of bounce b: the ray, its global id, polyline length and the
// point it left.  Returns false for an empty slot (left by an in-place
// bounce), which an in-place bounce b < K marks empty in its output too.
template <bool FIRST>
__device__ __forceinline__ bool load_ray(const TraceArgs& a, int b, uint32_t i, bool in_place, float o[3], float d[3],
                                         float& L, uint32_t& last, uint32_t& g) {
    L = 0.f;
    last = NO_HIT;
    if (FIRST) {
        const uint32_t ti = i / a.n_rays;
        const uint32_t jl = i - ti * a.n_rays;
        const uint32_t j = a.perm ? a.perm[jl] : jl;  // direction-coherent order
        g = ti * a.n_rays + j;
        o[0] = a.tx[3 * ti];
        o[1] = a.tx[3 * ti + 1];
        o[2] = a.tx[3 * ti + 2];
        d[0] = a.dirs[3 * (size_t)j];
        d[1] = a.dirs[3 * (size_t)j + 1];
        d[2] = a.dirs[3 * (size_t)j + 2];
        const float inv = 1.0f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        d[0] *= inv;
        d[1] *= inv;
        d[2] *= inv;
        return true;
    }
    const uint32_t src = a.order ? a.order[i] : i;  // coherence order (never with in-place bounces)
    g = ray_g(a, b + 1)[src];
    if (g == NO_HIT) {
        // the last bounce (b == K) has no output buffers (they may be unallocated)
        if (in_place && b < a.K) ray_g(a, b)[i] = NO_HIT;
        return false;
    }
    const float4 o4 = ray_o(a, b + 1)[src];
    const float4 d4 = ray_d(a, b + 1)[src];
    o[0] = o4.x; o[1] = o4.y; o[2] = o4.z; L = o4.w;
    d[0] = d4.x; d[1] = d4.y; d[2] = d4.z; last = __float_as_uint(d4.w);
    return true;
}

// Octahedral map of a unit direction onto [-1, 1]^2.
__device__ __forceinline__ void octahedral(float x, float y, float z, float& u, float& w) {
    const float s = fabsf(x) + fabsf(y) + fabsf(z);
    u = s > 0.f ? x / s : 0.f;
    w = s > 0.f ? y / s : 0.f;
    if (z < 0.f) {
        const float uu = (1.f - fabsf(w)) * (u >= 0.f ? 1.f : -1.f);
        const float ww = (1.f - fabsf(u)) * (w >= 0.f ? 1.f : -1.f);
        u = uu;
        w = ww;
    }
}

__device__ __forceinline__ uint32_t cell_of(float u, int cells) {
    return (uint32_t)fminf(fmaxf((u * 0.5f + 0.5f) * (float)cells, 0.f), (float)(cells - 1));
}

__device__ __forceinline__ uint32_t spread_bits4x3(uint32_t x) {
    x &= 15u;
    x = (x | (x << 4)) & 0x0C3u;
    x = (x | (x << 2)) & 0x249u;
    return x;
}

// Coherence bucket of a ray: Morton code of its origin on a 16^3 grid over the
// scene (12 bits), then the 4 x 4 octahedral cell of its direction (4 bits).
// Rays that start close together in similar directions walk the same cells.
__device__ __forceinline__ uint32_t ray_bucket(const TraceArgs& a, const float o[3], const float d[3]) {
    const uint32_t cx = (uint32_t)fminf(fmaxf((o[0] - a.klo.x) * a.kscale.x, 0.f), 15.f);
    const uint32_t cy = (uint32_t)fminf(fmaxf((o[1] - a.klo.y) * a.kscale.y, 0.f), 15.f);
    const uint32_t cz = (uint32_t)fminf(fmaxf((o[2] - a.klo.z) * a.kscale.z, 0.f), 15.f);
    float u, w;
    octahedral(d[0], d[1], d[2], u, w);
    const uint32_t m = spread_bits4x3(cx) | (spread_bits4x3(cy) << 1) | (spread_bits4x3(cz) << 2);
    return (m << 4) | (cell_of(u, 4) << 2) | cell_of(w, 4);
}

// End of the segments of lanes with `done`: log the hit, test every RX on
// [0, t_hit] (rho grows with the unfolded length), reflect at the hit and
// write the survivor (at its own slot i when `in_place`, else compacted with
// one atomic per wave); an in-place bounce marks a dead slot empty.  Called
// by every lane of the wave (ballots).
template <bool FIRST, bool STATS>
__device__ __forceinline__ void finish_segment(const TraceArgs& a, int b, bool done, bool in_place, uint32_t i,
                                               uint32_t g, float o[3], float d[3], float L, uint32_t last,
                                               const Hit& hit, stat_t cnt[ST_COUNT]) {
    const uint32_t lane = lane_id();
    const uint64_t lt = lanemask_lt();
    if (done) {
        if (STATS) {
            ++cnt[ST_SEGMENTS];
            if (hit.id != NO_HIT) ++cnt[ST_HITS];
            if (!FIRST) cnt[ST_BYTES] += 36;
        }
        if (a.hit_id) {
            const size_t idx = (size_t)g * (a.K + 1) + b;
            a.hit_id[idx] = hit.id == NO_HIT ? -1 : (int32_t)hit.id;
            a.hit_t[idx] = hit.id == NO_HIT ? NAN : hit.t;
        }
    }
    uint32_t* rec_counter = &a.counters[PCRL_CNT_REC(a.K)];
    for (int r = 0; r < a.n_rx; ++r) {
        const float rx0 = a.rx[3 * r], rx1 = a.rx[3 * r + 1], rx2 = a.rx[3 * r + 2];
        const float vx = rx0 - o[0], vy = rx1 - o[1], vz = rx2 - o[2];
        const float s = vx * d[0] + vy * d[1] + vz * d[2];
        bool got = false;
        if (done && s > 0.f && s <= hit.t) {
            const float cx = vx - s * d[0], cy = vy - s * d[1], cz = vz - s * d[2];
            const float rho = a.sig_c * (L + s);
            got = cx * cx + cy * cy + cz * cz <= rho * rho;
        }
        const uint64_t m = __ballot(got);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            uint32_t slot = 0;
            if ((int)lane == leader) slot = atomicAdd(rec_counter, (uint32_t)__popcll(m));
            slot = __shfl(slot, leader, 64) + (uint32_t)__popcll(m & lt);
            if (STATS && got) cnt[ST_BYTES] += 16;
            if (got && slot < a.rec_cap) {
                const float lp = L + sqrtf(vx * vx + vy * vy + vz * vz);
                a.rec[slot] = make_uint4(g, (uint32_t)r | ((uint32_t)b << 16), __float_as_uint(lp),
                                         __float_as_uint(L + s));
            }
        }
    }
    // reflect and keep survivors
    const bool surv = done && hit.id != NO_HIT && b < a.K;
    if (surv) {
        const float qx = o[0] + hit.t * d[0], qy = o[1] + hit.t * d[1], qz = o[2] + hit.t * d[2];
        a.hist[(size_t)b * a.n_total + g] = make_float4(qx, qy, qz, __uint_as_float(hit.lab));
        L += hit.t;
        const float dn = d[0] * hit.nx + d[1] * hit.ny + d[2] * hit.nz;
        const float ex = d[0] - 2.f * dn * hit.nx, ey = d[1] - 2.f * dn * hit.ny, ez = d[2] - 2.f * dn * hit.nz;
        const float inv = 1.0f / sqrtf(ex * ex + ey * ey + ez * ez);
        d[0] = ex * inv; d[1] = ey * inv; d[2] = ez * inv;
        o[0] = qx; o[1] = qy; o[2] = qz;
        last = hit.id;
    }
    if (b >= a.K) return;
    const uint64_t m = __ballot(surv);
    uint32_t slot = i;
    if (m) {
        const int leader = __ffsll((long long)m) - 1;
        uint32_t first = 0;
        if ((int)lane == leader) first = atomicAdd(&a.counters[b + 1], (uint32_t)__popcll(m));
        first = __shfl(first, leader, 64);
        if (!in_place) slot = first + (uint32_t)__popcll(m & lt);
    }
    if (STATS && surv) cnt[ST_BYTES] += 52;
    if (surv) {
        ray_o(a, b)[slot] = make_float4(o[0], o[1], o[2], L);
        ray_d(a, b)[slot] = make_float4(d[0], d[1], d[2], __uint_as_float(last));
        ray_g(a, b)[slot] = g;
    } else if (done && in_place) {
        ray_g(a, b)[i] = NO_HIT;
    }
    if (a.okeys && m) {  // compacted survivors only (never in place)
        const uint32_t key = surv ? ray_bucket(a, o, d) : 0u;
        const uint32_t pos = wave_bucket_add(a.ocnt + (size_t)b * 65536, key, surv);
        if (surv) {
            a.okeys[slot] = (uint16_t)key;
            a.opos[slot] = pos;
        }
    }
}

// One wave's 64 consecutive slots [base, base + 64) of bounce b of one query,
// traced in lockstep (base hierarchy, then the overlay).  Slots at or past
// `range` are idle; a slot whose ray id is NO_HIT (left by an in-place
// bounce) is idle too.  Every lane of the wave must call this (ballots).
template <bool FIRST, bool STATS, int NL, bool OV, bool BX = true>
__device__ __forceinline__ void trace_chunk(const TraceArgs& a, LeafTestLds& W, int b, uint32_t base, uint32_t range,
                                            bool in_place, stat_t cnt[ST_COUNT]) {
    const uint32_t i = base + lane_id();
    float o[3] = {0.f, 0.f, 0.f}, d[3] = {1.f, 0.f, 0.f};
    float L = 0.f;
    uint32_t last = NO_HIT, g = NO_HIT;
    const bool act = i < range && load_ray<FIRST>(a, b, i, in_place, o, d, L, last, g);
    Hit hit;
    hit_reset(hit);
    stage_ray(W, o, d, last);
    trace_segment<STATS, NL, false, BX>(a, W, act, o, d, hit, cnt);
    // dynamic points: the nearest hit over base and overlay is the nearest
    // hit of the union (ties again by point id); the overlay shares the
    // base's frame and levels
    if (OV) trace_segment<STATS, NL, true, BX>(a, W, act, o, d, hit, cnt);
    finish_segment<FIRST, STATS>(a, b, act, in_place, i, g, o, d, L, last, hit, cnt);
}

template <bool STATS>
__device__ __forceinline__ void flush_stats(stat_t cnt[ST_COUNT], unsigned long long* stats) {
    if (!STATS) return;
#pragma unroll
    for (int k = 0; k < ST_COUNT; ++k) {
        const uint64_t sum = wave_sum_u64(cnt[k]);
        if (stats && lane_id() == 0 && sum) atomicAdd(&stats[k], (unsigned long long)sum);
        cnt[k] = 0;
    }
}

// Renumber workgroups so that each of the 8 XCDs (workgroups are dispatched
// round-robin over them: block b -> XCD b % 8) works on one contiguous range
// of slots: neighbouring, coherent rays then share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_block() {
    const uint32_t nb = gridDim.x, bx = blockIdx.x;
    const uint32_t xcd = bx & 7u, per = nb >> 3, extra = nb & 7u;
    return xcd * per + min(xcd, extra) + (bx >> 3);
}

// A launch whose segments end at the implicit surface of Eq. 1 instead of the
// surfels (PCRL_LAUNCH_SDF; sdf.hip): runs every segment of every ray.
int sdf_launch_run(PcrlLaunch* L, const TraceArgs& t);

}  // namespace pcrl
