// cone.hip -- environment-driven coarse path tracing with conical rays
// (paper, Section 2.1 intersectable entities; Section 2.2.2 transmission
// phase; Section 2.2.3 propagation phase; Section 2.2.4 voxel cone tracing).
//
// Intersectable entities (IEs): the points of one label inside one subvoxel
// of a low-resolution voxel grid (voxel edge V, subvoxel V / D_v), each with
// a reception point (mean position) and a normal (normalised mean normal);
// and the pieces of caller-given diffraction edges, one per subvoxel an edge
// crosses (reception point its midpoint, the edge's direction and the
// outward normals of its two faces).
// One query is traced generation by generation:
//   transmission   a visibility ray from every TX towards every IE and RX;
//   generation k   the kept partial paths with k interactions; each casts a
//                  reflected cone (a node at a point IE) or the exterior
//                  sectors of its Keller cone (a node at an edge piece,
//                  Section 2.2.4), whose axes are marched through the voxel
//                  grid: the IEs and RX of the voxels within one voxel of the
//                  march (the paper's neighbour evaluation) that meet the cone
//                  (subvoxel bounding sphere), lie in front of the separation
//                  plane (between the sector's two planes) and are visible
//                  become generation k + 1 or receptions;
//   merge          partial paths reaching the same IE with the same labels in
//                  the same order are one (the smallest SplitMix64 priority
//                  wins), sorted by (TX, labels, IE, priority);
//   collect        receptions grouped by (TX, RX, labels), kappa rows each.
// Visibility and axis rays run through the launcher's hierarchy with its
// wave-cooperative surfel tests.  Every step is a kernel; the host only reads
// back the sizes of the next generation.
#include "trace_core.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

namespace pcrl {

constexpr uint32_t RX_BIT = 0x80000000u;  // candidate target: an RX (low bits its index)
constexpr int CONE_BLOCK = 256;

struct IeGrid {
    float org[3];
    float V;       // voxel edge
    float sv;      // subvoxel edge (FP32 V / dv)
    float inv_sv;  // 1 / sv (FP32)
    int32_t dv;
    int32_t dims[3];
};

}  // namespace pcrl

struct PcrlIes {
    const PcrlScene* scene = nullptr;
    int device = 0;
    pcrl::IeGrid g{};
    pcrl::DevBufs bufs;
    int64_t n_ie = 0, n_vox = 0, n_occ = 0, bytes = 0;
    uint64_t* key = nullptr;
    int32_t* sub = nullptr;      // [n,3]
    uint32_t* label = nullptr;
    uint32_t* count = nullptr;
    float4* pos = nullptr;       // reception point
    float4* nrm = nullptr;       // unit normal
    uint2* vox = nullptr;        // per voxel: (first point IE, count)
    uint8_t* near = nullptr;     // per voxel: an IE (point or edge) within Chebyshev distance 1
    // edge IEs (ie_add_edges): indices [n_pt, n_ie) follow the point IEs
    int64_t n_pt = 0, n_edges = 0;
    uint32_t* type = nullptr;    // per IE: 0 points, 1 an edge piece
    uint32_t* eid = nullptr;     // per IE: its edge (edge pieces), else 0xFFFFFFFF
    float4* ew = nullptr;        // per edge piece: unit edge direction
    float4* en1 = nullptr;       // per edge piece: outward normals of the edge's two faces
    float4* en2 = nullptr;
    uint2* vox_e = nullptr;      // per voxel: (first edge piece, count), null without edges
    // the edges as given (refinement of diffraction points)
    int64_t n_lines = 0;
    float* line_seg = nullptr;   // [n_lines,2,3]
    float* line_nrm = nullptr;   // [n_lines,2,3]
    uint32_t* line_label = nullptr;
};

namespace pcrl {

// One generation of partial paths (nodes) with k interactions.
struct Gen {
    int64_t n = 0;
    float4* apex = nullptr;      // reception point, polyline length in w
    uint32_t* ie = nullptr;
    uint32_t* parent = nullptr;
    uint32_t* tx = nullptr;
    uint32_t* gid = nullptr;     // label-sequence group (dense, in (tx, labels) order)
    uint64_t* prio = nullptr;
    uint32_t* ndiff = nullptr;   // diffractions on the partial path
};

// The conical rays of one generation: one reflected cone per node at a point
// IE, the exterior Keller-cone sectors of a node at an edge piece.
struct Cones {
    uint32_t n = 0;
    uint32_t* node = nullptr;
    float4* axis = nullptr;
    float4* s0 = nullptr;        // reflection: separation plane normal; diffraction: lower sector plane
    float4* s1 = nullptr;        // diffraction: upper sector plane
    uint32_t* kind = nullptr;    // 0 reflection, 1 diffraction sector, 2 diffraction without planes (one sector)
    float* t_end = nullptr;      // end of the axis march
};

struct Rec {                     // one reception
    uint32_t node;               // node index in its generation (the TX for k = 0)
    uint32_t rx;
    uint32_t k;
    float len;
};

}  // namespace pcrl

struct PcrlConeLaunch {
    const PcrlIes* ies = nullptr;
    int32_t n_tx = 0, n_rx = 0, K = 0;
    pcrl::DevBufs bufs;
    std::vector<pcrl::Gen> gens;    // gens[k] for k = 1..K (gens[0] unused)
    float4* tx = nullptr;           // TX positions (w = 0)
    float4* rx = nullptr;
    pcrl::Rec* rec = nullptr;
    int64_t n_rec = 0;
    PcrlConeStats stats{};
};

namespace pcrl {

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the output for state x.
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ float dot3f(float ax, float ay, float az, float bx, float by, float bz) {
    return ax * bx + ay * by + az * bz;
}

// Distance along the unit direction u at which the ray from o enters the box
// [lo, lo + e]^3 (0 when o is inside); +inf when it misses.
__device__ __forceinline__ float box_entry(const float o[3], const float u[3], const float lo[3], float e) {
    float t0 = 0.f, t1 = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (u[a] != 0.f) {
            float ta = (lo[a] - o[a]) / u[a], tb = (lo[a] + e - o[a]) / u[a];
            t0 = fmaxf(t0, fminf(ta, tb));
            t1 = fminf(t1, fmaxf(ta, tb));
        } else if (o[a] < lo[a] || o[a] > lo[a] + e) {
            t1 = -1.f;
        }
    }
    return t0 <= t1 ? t0 : INFINITY;
}

// ---------------------------------------------------------------------------
// IE table (Section 2.1)
// ---------------------------------------------------------------------------

__global__ void k_ie_keys(const float4* pos, const float4* nrm, uint32_t n, IeGrid g, uint64_t* key, uint32_t* id,
                          uint32_t* bad) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 p = pos[i];
    const float pc[3] = {p.x, p.y, p.z};
    int s[3];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = floorf((pc[a] - g.org[a]) * g.inv_sv);
        ok = ok && u >= 0.f && u < (float)(g.dims[a] * g.dv);
        s[a] = ok ? (int)u : 0;
    }
    if (!ok) atomicAdd(bad, 1u);
    const int dv = g.dv;
    const uint64_t vox = (uint64_t)(s[0] / dv) + (uint64_t)g.dims[0] * ((uint64_t)(s[1] / dv) +
                                                                       (uint64_t)g.dims[1] * (uint64_t)(s[2] / dv));
    const uint64_t loc = (uint64_t)(s[0] % dv) + (uint64_t)dv * ((uint64_t)(s[1] % dv) + (uint64_t)dv * (s[2] % dv));
    key[i] = ((vox * (uint64_t)(dv * dv * dv) + loc) << 32) | (uint64_t)__float_as_uint(nrm[i].w);
    id[i] = i;
}

__global__ void k_ie_flags(const uint64_t* key, uint32_t n, uint32_t* flag) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flag[i] = (i == 0 || key[i] != key[i - 1]) ? 1u : 0u;
}

// Per IE (one thread): its range of sorted points, the means in FP64.
__global__ void k_ie_reduce(const uint64_t* key, const uint32_t* id, const uint32_t* scan, uint32_t n,
                            const float4* pos, const float4* nrm, IeGrid g, uint32_t n_ie, uint64_t* ie_key,
                            int32_t* sub, uint32_t* label, uint32_t* count, float4* ie_pos, float4* ie_nrm) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!(i == 0 || key[i] != key[i - 1])) return;
    const uint32_t e = scan[i];
    if (e >= n_ie) return;
    uint32_t j = i;
    double px = 0, py = 0, pz = 0, nx = 0, ny = 0, nz = 0;
    for (; j < n && key[j] == key[i]; ++j) {
        const float4 p = pos[id[j]];
        const float4 q = nrm[id[j]];
        px += p.x; py += p.y; pz += p.z;
        nx += q.x; ny += q.y; nz += q.z;
    }
    const double c = (double)(j - i);
    const double ln = sqrt(nx * nx + ny * ny + nz * nz);
    const uint64_t k = key[i];
    ie_key[e] = k;
    const int dv = g.dv;
    const uint64_t cell = k >> 32;
    const uint64_t vox = cell / (uint64_t)(dv * dv * dv);
    const int loc = (int)(cell % (uint64_t)(dv * dv * dv));
    const int vx = (int)(vox % (uint64_t)g.dims[0]);
    const int vy = (int)((vox / (uint64_t)g.dims[0]) % (uint64_t)g.dims[1]);
    const int vz = (int)(vox / ((uint64_t)g.dims[0] * (uint64_t)g.dims[1]));
    sub[3 * (size_t)e] = vx * dv + loc % dv;
    sub[3 * (size_t)e + 1] = vy * dv + (loc / dv) % dv;
    sub[3 * (size_t)e + 2] = vz * dv + loc / (dv * dv);
    label[e] = (uint32_t)(k & 0xFFFFFFFFull);
    count[e] = j - i;
    ie_pos[e] = make_float4((float)(px / c), (float)(py / c), (float)(pz / c), 0.f);
    ie_nrm[e] = ln > 0 ? make_float4((float)(nx / ln), (float)(ny / ln), (float)(nz / ln), 0.f)
                       : make_float4(0.f, 0.f, 1.f, 0.f);
}

__global__ void k_ie_voxels(const uint64_t* ie_key, uint32_t n_ie, int dv3, uint2* vox) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_ie) return;
    const uint64_t v = (ie_key[e] >> 32) / (uint64_t)dv3;
    const bool first = e == 0 || ((ie_key[e - 1] >> 32) / (uint64_t)dv3) != v;
    if (!first) return;
    uint32_t j = e + 1;
    while (j < n_ie && ((ie_key[j] >> 32) / (uint64_t)dv3) == v) ++j;
    vox[v] = make_uint2(e, j - e);
}

__global__ void k_ie_near(const uint2* vox, const uint2* vox_e, IeGrid g, uint32_t n_vox, uint8_t* near) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_vox) return;
    const int x = (int)(v % (uint32_t)g.dims[0]);
    const int y = (int)((v / (uint32_t)g.dims[0]) % (uint32_t)g.dims[1]);
    const int z = (int)(v / ((uint32_t)g.dims[0] * (uint32_t)g.dims[1]));
    uint8_t any = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int a = x + dx, b = y + dy, c = z + dz;
                if (a < 0 || b < 0 || c < 0 || a >= g.dims[0] || b >= g.dims[1] || c >= g.dims[2]) continue;
                const size_t w = (size_t)a + (size_t)g.dims[0] * ((size_t)b + (size_t)g.dims[1] * c);
                if (vox[w].y || (vox_e && vox_e[w].y)) any = 1;
            }
    near[v] = any;
}

// Cut parameters of edge j at the subvoxel face planes it crosses, in
// increasing order, each value once (a corner crossing of two axes is one
// cut): t_k = ((origin + k sv) - a) / (b - a) along every axis, kept when
// 0 < t < 1.  Returns their number; writes the pieces when `write`.
struct EdgeArgs {
    const float* seg;        // [n,2,3]
    const float* nrm;        // [n,2,3]
    const uint32_t* label;
    uint32_t n;
    IeGrid g;
    const uint32_t* offset;  // pieces before each edge ([n + 1])
    uint32_t* count;         // pieces of each edge
    uint32_t* bad;
    uint64_t* key;           // out per piece (edge-major, t increasing)
    uint32_t* edge;
    int32_t* sub;            // [P,3]
    float4* pos;
};

__device__ uint32_t edge_pieces(const EdgeArgs& A, uint32_t j, bool write) {
#pragma clang fp contract(off)
    const IeGrid& g = A.g;
    const float a[3] = {A.seg[6 * j], A.seg[6 * j + 1], A.seg[6 * j + 2]};
    const float b[3] = {A.seg[6 * j + 3], A.seg[6 * j + 4], A.seg[6 * j + 5]};
    const float d[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    // per axis: the next plane index k and its last value, in increasing t
    int kn[3], ke[3], ks[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        ks[ax] = 0;
        kn[ax] = 0;
        ke[ax] = -1;
        if (d[ax] == 0.f) continue;
        const float u0 = (a[ax] - g.org[ax]) * g.inv_sv, u1 = (b[ax] - g.org[ax]) * g.inv_sv;
        const int lo = (int)floorf(fminf(u0, u1)) + 1, hi = (int)floorf(fmaxf(u0, u1));
        if (d[ax] > 0.f) { kn[ax] = lo; ke[ax] = hi; ks[ax] = 1; }
        else { kn[ax] = hi; ke[ax] = lo; ks[ax] = -1; }
    }
    auto t_of = [&](int ax, int k) { return ((g.org[ax] + (float)k * g.sv) - a[ax]) / d[ax]; };
    auto more = [&](int ax) { return ks[ax] != 0 && (ks[ax] > 0 ? kn[ax] <= ke[ax] : kn[ax] >= ke[ax]); };
    float prev = 0.f;
    uint32_t pieces = 0;
    const uint32_t base = write ? A.offset[j] : 0u;
    for (;;) {
        // the smallest next cut in (prev, 1) over the three axes
        float t = 1.f;
        int which = -1;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            while (more(ax) && !(t_of(ax, kn[ax]) > prev)) kn[ax] += ks[ax];   // at or before the last cut
            if (more(ax)) {
                const float tc = t_of(ax, kn[ax]);
                if (tc < t) {
                    t = tc;
                    which = ax;
                }
            }
        }
        if (which < 0 || !(t < 1.f)) t = 1.f;
        if (write) {
            const float tm = (prev + t) * 0.5f;
            const float m[3] = {a[0] + tm * d[0], a[1] + tm * d[1], a[2] + tm * d[2]};
            int c[3];
            bool ok = true;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const float u = floorf((m[ax] - g.org[ax]) * g.inv_sv);
                ok = ok && u >= 0.f && u < (float)(g.dims[ax] * g.dv);
                c[ax] = ok ? (int)u : 0;
            }
            if (!ok) atomicAdd(A.bad, 1u);
            const int dv = g.dv;
            const uint64_t vox = (uint64_t)(c[0] / dv) +
                                 (uint64_t)g.dims[0] * ((uint64_t)(c[1] / dv) + (uint64_t)g.dims[1] * (uint64_t)(c[2] / dv));
            const uint64_t loc = (uint64_t)(c[0] % dv) + (uint64_t)dv * ((uint64_t)(c[1] % dv) + (uint64_t)dv * (c[2] % dv));
            const uint32_t q = base + pieces;
            A.key[q] = ((vox * (uint64_t)(dv * dv * dv) + loc) << 32) | (uint64_t)A.label[j];
            A.edge[q] = j;
            A.sub[3 * (size_t)q] = c[0];
            A.sub[3 * (size_t)q + 1] = c[1];
            A.sub[3 * (size_t)q + 2] = c[2];
            A.pos[q] = make_float4(m[0], m[1], m[2], 0.f);
        }
        ++pieces;
        if (t >= 1.f) break;
        prev = t;
    }
    return pieces;
}

__global__ void k_edge_count(EdgeArgs A) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= A.n) return;
    const float dx = A.seg[6 * j + 3] - A.seg[6 * j], dy = A.seg[6 * j + 4] - A.seg[6 * j + 1],
                dz = A.seg[6 * j + 5] - A.seg[6 * j + 2];
    if (!(dx * dx + dy * dy + dz * dz > 0.f)) {
        atomicAdd(A.bad, 1u);
        A.count[j] = 0;
        return;
    }
    A.count[j] = edge_pieces(A, j, false);
}

__global__ void k_edge_write(EdgeArgs A) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= A.n || A.count[j] == 0) return;
    edge_pieces(A, j, true);
}

// Edge pieces in sorted order appended to the IE arrays (from index n_pt).
struct EdgeAppend {
    const uint32_t* perm;    // sorted order of the pieces
    uint32_t P, n_pt;
    const uint64_t* key;     // sorted keys
    const uint32_t* edge;
    const int32_t* sub;
    const float4* pos;
    const float* seg;
    const float* nrm;
    uint64_t* ie_key;
    int32_t* ie_sub;
    uint32_t* ie_label;
    uint32_t* ie_count;
    float4* ie_pos;
    float4* ie_nrm;
    uint32_t* ie_type;
    uint32_t* ie_eid;
    float4* ew;
    float4* en1;
    float4* en2;
};

__global__ void k_edge_append(EdgeAppend A) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= A.P) return;
    const uint32_t p = A.perm[q];
    const uint32_t j = A.edge[p];
    const uint32_t e = A.n_pt + q;
    A.ie_key[e] = A.key[q];
    A.ie_sub[3 * (size_t)e] = A.sub[3 * (size_t)p];
    A.ie_sub[3 * (size_t)e + 1] = A.sub[3 * (size_t)p + 1];
    A.ie_sub[3 * (size_t)e + 2] = A.sub[3 * (size_t)p + 2];
    A.ie_label[e] = (uint32_t)(A.key[q] & 0xFFFFFFFFull);
    A.ie_count[e] = 0u;
    A.ie_pos[e] = A.pos[p];
    A.ie_nrm[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    A.ie_type[e] = 1u;
    A.ie_eid[e] = j;
    const float dx = A.seg[6 * j + 3] - A.seg[6 * j], dy = A.seg[6 * j + 4] - A.seg[6 * j + 1],
                dz = A.seg[6 * j + 5] - A.seg[6 * j + 2];
    const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
    A.ew[q] = make_float4(dx * il, dy * il, dz * il, 0.f);
    A.en1[q] = make_float4(A.nrm[6 * j], A.nrm[6 * j + 1], A.nrm[6 * j + 2], 0.f);
    A.en2[q] = make_float4(A.nrm[6 * j + 3], A.nrm[6 * j + 4], A.nrm[6 * j + 5], 0.f);
}

// Per voxel the range of the edge pieces [n_pt, n_ie) it holds.
__global__ void k_edge_voxels(const uint64_t* ie_key, uint32_t n_pt, uint32_t n_ie, int dv3, uint2* vox_e) {
    const uint32_t e = n_pt + blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_ie) return;
    const uint64_t v = (ie_key[e] >> 32) / (uint64_t)dv3;
    const bool first = e == n_pt || ((ie_key[e - 1] >> 32) / (uint64_t)dv3) != v;
    if (!first) return;
    uint32_t j = e + 1;
    while (j < n_ie && ((ie_key[j] >> 32) / (uint64_t)dv3) == v) ++j;
    vox_e[v] = make_uint2(e, j - e);
}

// ---------------------------------------------------------------------------
// visibility and axis rays (Sections 2.2.2 and 2.2.4)
// ---------------------------------------------------------------------------

struct VisArgs {
    TraceArgs t;          // the scene's hierarchy (t.v)
    IeGrid g;
    const float4* origin; // per parent: TX (k = 0) or reception point
    const uint32_t* cand_node;
    const uint32_t* cand_target;
    uint32_t n;
    const float4* ie_pos;
    const int32_t* ie_sub;
    const float4* rx;
    const int32_t* rx_sub;
    uint32_t* visible;    // per candidate: 1 visible, 0 blocked
};

// One candidate per lane: a ray from the parent's point towards the target's
// reception point; blocked when a surfel disk is hit before the ray enters
// the target's subvoxel (the lane's nearest hit starts at that distance, so
// only nearer hits register).
template <int NL, bool BX>
__global__ __launch_bounds__(TRACE_BLOCK) void k_visibility(VisArgs a) {
    __shared__ LeafTestLds lds[TRACE_BLOCK / 64];
    LeafTestLds& W = lds[threadIdx.x >> 6];
    stat_t cnt[ST_COUNT] = {};
    const uint32_t wave = blockIdx.x * (TRACE_BLOCK / 64) + (threadIdx.x >> 6);
    const uint32_t n_waves = gridDim.x * (TRACE_BLOCK / 64);
    for (uint32_t base = wave * 64; base < a.n; base += n_waves * 64) {
        const uint32_t i = base + lane_id();
        const bool act = i < a.n;
        float o[3] = {0.f, 0.f, 0.f}, u[3] = {1.f, 0.f, 0.f};
        Hit hit;
        hit_reset(hit);
        if (act) {
            const float4 O = a.origin[a.cand_node[i]];
            const uint32_t tg = a.cand_target[i];
            float4 P;
            int s0, s1, s2;
            if (tg & RX_BIT) {
                const uint32_t j = tg & ~RX_BIT;
                P = a.rx[j];
                s0 = a.rx_sub[3 * j]; s1 = a.rx_sub[3 * j + 1]; s2 = a.rx_sub[3 * j + 2];
            } else {
                P = a.ie_pos[tg];
                s0 = a.ie_sub[3 * (size_t)tg]; s1 = a.ie_sub[3 * (size_t)tg + 1]; s2 = a.ie_sub[3 * (size_t)tg + 2];
            }
            o[0] = O.x; o[1] = O.y; o[2] = O.z;
            u[0] = P.x - O.x; u[1] = P.y - O.y; u[2] = P.z - O.z;
            const float len = sqrtf(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            if (len > 0.f) {
                const float inv = 1.0f / len;
                u[0] *= inv; u[1] *= inv; u[2] *= inv;
                const float lo[3] = {a.g.org[0] + (float)s0 * a.g.sv, a.g.org[1] + (float)s1 * a.g.sv,
                                     a.g.org[2] + (float)s2 * a.g.sv};
                hit.t = box_entry(o, u, lo, a.g.sv);
            } else {
                u[0] = 1.f; u[1] = 0.f; u[2] = 0.f;
                hit.t = 0.f;
            }
        }
        stage_ray(W, o, u, NO_HIT);
        trace_segment<false, NL, false, BX>(a.t, W, act && hit.t > 0.f, o, u, hit, cnt);
        if (act) a.visible[i] = hit.id == NO_HIT ? 1u : 0u;
    }
}

// ---------------------------------------------------------------------------
// cones of a generation (Sections 2.2.3 and 2.2.4)
// ---------------------------------------------------------------------------

struct ExpandArgs {
    Gen gen;
    const float4* parent_pos;   // previous generation's apex (or the TX)
    const uint32_t* type;
    const float4* ie_nrm;
    const float4* ew;
    const float4* en1;
    const float4* en2;
    uint32_t n_pt;
    float half;                 // cone half-angle
    const uint32_t* offset;     // k_cone_fill: exclusive scan of the counts ([n + 1])
    uint32_t* count;            // k_cone_count: cones per node
    Cones out;
};

// The cones of node i: count them, or write them from `base`.  A point IE
// reflects: d' = d - 2 (d.n) n, separation plane normal n on the reflected
// side.  An edge piece diffracts: Keller's cone of the directions d with
// d.w = d_in.w is cut into N = max(1, ceil(2 pi sin(beta) / (2 half)))
// sectors of azimuth 2 pi / N measured from the face-1 normal; a sector whose
// middle direction leaves the wedge (v.n1 >= 0 or v.n2 >= 0) is a cone, with
// the planes through the edge at its two bounding azimuths.
__device__ uint32_t node_cones(const ExpandArgs& a, uint32_t i, bool write, uint32_t base) {
#pragma clang fp contract(off)
    const float4 A = a.gen.apex[i];
    const float4 Pp = a.parent_pos[a.gen.parent[i]];
    const uint32_t e = a.gen.ie[i];
    float di[3] = {A.x - Pp.x, A.y - Pp.y, A.z - Pp.z};
    const float li = 1.0f / sqrtf(di[0] * di[0] + di[1] * di[1] + di[2] * di[2]);
    di[0] *= li; di[1] *= li; di[2] *= li;
    if (a.type[e] == 0u) {
        if (write) {
            const float4 N = a.ie_nrm[e];
            const float dn = di[0] * N.x + di[1] * N.y + di[2] * N.z;
            float d[3] = {di[0] - 2.f * dn * N.x, di[1] - 2.f * dn * N.y, di[2] - 2.f * dn * N.z};
            const float lo = 1.0f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            d[0] *= lo; d[1] *= lo; d[2] *= lo;
            const float side = d[0] * N.x + d[1] * N.y + d[2] * N.z > 0.f ? 1.f : -1.f;
            a.out.node[base] = i;
            a.out.axis[base] = make_float4(d[0], d[1], d[2], 0.f);
            a.out.s0[base] = make_float4(side * N.x, side * N.y, side * N.z, 0.f);
            a.out.s1[base] = make_float4(0.f, 0.f, 0.f, 0.f);
            a.out.kind[base] = 0u;
        }
        return 1u;
    }
    const uint32_t q = e - a.n_pt;
    const float4 W = a.ew[q], N1 = a.en1[q], N2 = a.en2[q];
    const float cb = di[0] * W.x + di[1] * W.y + di[2] * W.z;
    const float sb = sqrtf(fmaxf(0.f, 1.f - cb * cb));
    const float nw = N1.x * W.x + N1.y * W.y + N1.z * W.z;
    float e1[3] = {N1.x - nw * W.x, N1.y - nw * W.y, N1.z - nw * W.z};
    const float l1 = 1.0f / sqrtf(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    e1[0] *= l1; e1[1] *= l1; e1[2] *= l1;
    const float e2[3] = {W.y * e1[2] - W.z * e1[1], W.z * e1[0] - W.x * e1[2], W.x * e1[1] - W.y * e1[0]};
    const float arg = 3.14159265358979f * sb / a.half;
    const int N = max(1, (int)ceilf(arg));
    const float dphi = 6.28318530717959f / (float)N;
    uint32_t c = 0;
    for (int k = 0; k < N; ++k) {
        const float phi = ((float)k + 0.5f) * dphi;
        const float cp = cosf(phi), sp = sinf(phi);
        const float v[3] = {cp * e1[0] + sp * e2[0], cp * e1[1] + sp * e2[1], cp * e1[2] + sp * e2[2]};
        const float x1 = v[0] * N1.x + v[1] * N1.y + v[2] * N1.z;
        const float x2 = v[0] * N2.x + v[1] * N2.y + v[2] * N2.z;
        if (fmaxf(x1, x2) < 0.f) continue;
        if (write) {
            float d[3] = {cb * W.x + sb * v[0], cb * W.y + sb * v[1], cb * W.z + sb * v[2]};
            const float ld = 1.0f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            d[0] *= ld; d[1] *= ld; d[2] *= ld;
            const float c0 = cosf((float)k * dphi), s0 = sinf((float)k * dphi);
            const float c1 = cosf((float)(k + 1) * dphi), s1 = sinf((float)(k + 1) * dphi);
            a.out.node[base + c] = i;
            a.out.axis[base + c] = make_float4(d[0], d[1], d[2], 0.f);
            a.out.s0[base + c] = make_float4(c0 * e2[0] - s0 * e1[0], c0 * e2[1] - s0 * e1[1],
                                             c0 * e2[2] - s0 * e1[2], 0.f);
            a.out.s1[base + c] = make_float4(c1 * e2[0] - s1 * e1[0], c1 * e2[1] - s1 * e1[1],
                                             c1 * e2[2] - s1 * e1[2], 0.f);
            a.out.kind[base + c] = N > 1 ? 1u : 2u;
        }
        ++c;
    }
    return c;
}

__global__ void k_cone_count(ExpandArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)a.gen.n) return;
    a.count[i] = node_cones(a, i, false, 0u);
}

__global__ void k_cone_fill(ExpandArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)a.gen.n) return;
    node_cones(a, i, true, a.offset[i]);
}

struct AxisArgs {
    TraceArgs t;
    const float4* apex;         // the generation's nodes
    Cones cones;
};

// The first surfel hit (t > t_eps) of every cone's axis: the end of its march.
template <int NL, bool BX>
__global__ __launch_bounds__(TRACE_BLOCK) void k_axis(AxisArgs a) {
    __shared__ LeafTestLds lds[TRACE_BLOCK / 64];
    LeafTestLds& W = lds[threadIdx.x >> 6];
    stat_t cnt[ST_COUNT] = {};
    const uint32_t wave = blockIdx.x * (TRACE_BLOCK / 64) + (threadIdx.x >> 6);
    const uint32_t n_waves = gridDim.x * (TRACE_BLOCK / 64);
    const uint32_t n = a.cones.n;
    for (uint32_t base = wave * 64; base < n; base += n_waves * 64) {
        const uint32_t i = base + lane_id();
        const bool act = i < n;
        float o[3] = {0.f, 0.f, 0.f}, d[3] = {1.f, 0.f, 0.f};
        Hit hit;
        hit_reset(hit);
        if (act) {
            const float4 A = a.apex[a.cones.node[i]];
            const float4 D = a.cones.axis[i];
            o[0] = A.x; o[1] = A.y; o[2] = A.z;
            d[0] = D.x; d[1] = D.y; d[2] = D.z;
        }
        stage_ray(W, o, d, NO_HIT);
        trace_segment<false, NL, false, BX>(a.t, W, act, o, d, hit, cnt);
        if (act) a.cones.t_end[i] = hit.id == NO_HIT ? INFINITY : hit.t;
    }
}

// ---------------------------------------------------------------------------
// cone targets (Section 2.2.4)
// ---------------------------------------------------------------------------

struct ConeArgs {
    IeGrid g;
    Gen gen;
    Cones cones;
    const uint2* vox;
    const uint2* vox_e;   // null without edges
    const uint8_t* near;
    const float4* ie_pos;
    const int32_t* ie_sub;
    const uint32_t* eid;
    const float4* rx;
    const int32_t* rx_sub;
    int32_t n_rx;
    int32_t want_ie;      // 0 at the last generation: RX targets only
    int32_t max_diff;
    float cos_t, sin_t, R;
    float tau;            // a reflected target lies in front of the separation plane by more than tau
    uint32_t cap;
    uint32_t* n_cand;     // counts every candidate, also beyond cap
    uint32_t* cand_node;
    uint32_t* cand_target;
};

// Whether the cone (apex o, unit axis d, half-angle t) meets the sphere
// (c, R): distance from c to the solid cone against R.
__device__ __forceinline__ bool cone_meets(const ConeArgs& a, const float o[3], const float d[3], float cx, float cy,
                                           float cz) {
    const float vx = cx - o[0], vy = cy - o[1], vz = cz - o[2];
    const float ax = vx * d[0] + vy * d[1] + vz * d[2];
    const float wx = vx - ax * d[0], wy = vy - ax * d[1], wz = vz - ax * d[2];
    const float rho = sqrtf(wx * wx + wy * wy + wz * wz);
    const float lateral = rho * a.cos_t - ax * a.sin_t;
    float dist;
    if (lateral <= 0.f) dist = 0.f;
    else if (ax * a.cos_t + rho * a.sin_t < 0.f) dist = sqrtf(vx * vx + vy * vy + vz * vz);
    else dist = lateral;
    return dist <= a.R;
}

// The separation test of a target point p for cone q: in front of the
// reflection's plane, or between the sector's two planes.
__device__ __forceinline__ bool cone_separates(const ConeArgs& a, uint32_t q, const float o[3], float4 P) {
    const uint32_t kind = a.cones.kind[q];
    if (kind == 2u) return true;
    const float4 S0 = a.cones.s0[q];
    const float m0 = (P.x - o[0]) * S0.x + (P.y - o[1]) * S0.y + (P.z - o[2]) * S0.z;
    if (kind == 0u) return m0 - a.tau > 0.f;
    const float4 S1 = a.cones.s1[q];
    const float m1 = (P.x - o[0]) * S1.x + (P.y - o[1]) * S1.y + (P.z - o[2]) * S1.z;
    return m0 >= 0.f && m1 < 0.f;
}

__device__ __forceinline__ void cone_emit(const ConeArgs& a, uint32_t node, uint32_t target) {
    const uint32_t slot = atomicAdd(a.n_cand, 1u);
    if (slot < a.cap) {
        a.cand_node[slot] = node;
        a.cand_target[slot] = target;
    }
}

__device__ __forceinline__ void cone_range(const ConeArgs& a, uint32_t q, uint32_t node, uint32_t own_ie,
                                           uint32_t own_edge, const float o[3], const float d[3], uint2 r) {
    const IeGrid& g = a.g;
    for (uint32_t e = r.x; e < r.x + r.y; ++e) {
        if (e == own_ie || (own_edge != 0xFFFFFFFFu && a.eid[e] == own_edge)) continue;
        const int s0 = a.ie_sub[3 * (size_t)e], s1 = a.ie_sub[3 * (size_t)e + 1], s2 = a.ie_sub[3 * (size_t)e + 2];
        const float cx = g.org[0] + ((float)s0 + 0.5f) * g.sv;
        const float cy = g.org[1] + ((float)s1 + 0.5f) * g.sv;
        const float cz = g.org[2] + ((float)s2 + 0.5f) * g.sv;
        if (!cone_meets(a, o, d, cx, cy, cz)) continue;
        if (!cone_separates(a, q, o, a.ie_pos[e])) continue;
        cone_emit(a, node, e);
    }
}

// The IE targets of voxel w (in the grid) for cone q of node `node`.
__device__ __forceinline__ void cone_voxel(const ConeArgs& a, uint32_t q, uint32_t node, uint32_t own_ie,
                                           uint32_t own_edge, bool edges_ok, const float o[3], const float d[3],
                                           int wx, int wy, int wz) {
    const IeGrid& g = a.g;
    if (wx < 0 || wy < 0 || wz < 0 || wx >= g.dims[0] || wy >= g.dims[1] || wz >= g.dims[2]) return;
    const size_t w = (size_t)wx + (size_t)g.dims[0] * ((size_t)wy + (size_t)g.dims[1] * wz);
    cone_range(a, q, node, own_ie, own_edge, o, d, a.vox[w]);
    if (edges_ok) cone_range(a, q, node, own_ie, own_edge, o, d, a.vox_e[w]);
}

// The RX of voxel w (in the grid) for cone q of node `node`.
__device__ __forceinline__ void cone_voxel_rx(const ConeArgs& a, uint32_t q, uint32_t node, const float o[3],
                                              const float d[3], int wx, int wy, int wz) {
    const IeGrid& g = a.g;
    for (int j = 0; j < a.n_rx; ++j) {
        const int s0 = a.rx_sub[3 * j], s1 = a.rx_sub[3 * j + 1], s2 = a.rx_sub[3 * j + 2];
        if (s0 / g.dv != wx || s1 / g.dv != wy || s2 / g.dv != wz) continue;
        const float cx = g.org[0] + ((float)s0 + 0.5f) * g.sv;
        const float cy = g.org[1] + ((float)s1 + 0.5f) * g.sv;
        const float cz = g.org[2] + ((float)s2 + 0.5f) * g.sv;
        if (!cone_meets(a, o, d, cx, cy, cz)) continue;
        if (!cone_separates(a, q, o, a.rx[j])) continue;
        cone_emit(a, node, RX_BIT | (uint32_t)j);
    }
}

// One cone per thread: march the axis voxel by voxel (Amanatides and Woo;
// every boundary distance computed from the origin, no accumulation) up to
// the voxel holding t_end; at every voxel the neighbours it adds to the
// union of 3x3x3 blocks along the march are evaluated (all 27 at the first
// voxel, then the 9 of the block's leading face along the step's axis).
// IE targets only where the block holds some (the march distance); the RX
// always.  Edge pieces only below the diffraction limit, never of the node's
// own edge.
__global__ __launch_bounds__(CONE_BLOCK) void k_cones(ConeArgs a) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= a.cones.n) return;
    const IeGrid& g = a.g;
    const uint32_t node = a.cones.node[q];
    const float4 A = a.gen.apex[node];
    const float4 D = a.cones.axis[q];
    const float o[3] = {A.x, A.y, A.z}, d[3] = {D.x, D.y, D.z};
    const uint32_t own = a.gen.ie[node];
    const uint32_t own_edge = a.eid[own];
    const bool edges_ok = a.vox_e && (int32_t)a.gen.ndiff[node] < a.max_diff;
    const float t_end = a.cones.t_end[q];
    int c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = min(max((int)floorf((o[k] - g.org[k]) / g.V), 0), g.dims[k] - 1);
    int step_axis = -1;
    for (int it = 0; it < g.dims[0] + g.dims[1] + g.dims[2] + 3; ++it) {
        const size_t cv = (size_t)c[0] + (size_t)g.dims[0] * ((size_t)c[1] + (size_t)g.dims[1] * c[2]);
        const bool ies_near = a.want_ie && a.near[cv];
        if (ies_near || a.n_rx > 0) {
            if (step_axis < 0) {
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            if (ies_near)
                                cone_voxel(a, q, node, own, own_edge, edges_ok, o, d, c[0] + dx, c[1] + dy, c[2] + dz);
                            cone_voxel_rx(a, q, node, o, d, c[0] + dx, c[1] + dy, c[2] + dz);
                        }
            } else {
                // the block's leading face along the step: the voxels the previous blocks did not hold
                const int sg = d[step_axis] > 0.f ? 1 : -1;
                const int a1 = step_axis == 0 ? 1 : 0, a2 = step_axis == 2 ? 1 : 2;
                for (int p = -1; p <= 1; ++p)
                    for (int r = -1; r <= 1; ++r) {
                        int w[3] = {c[0], c[1], c[2]};
                        w[step_axis] += sg;
                        w[a1] += p;
                        w[a2] += r;
                        if (ies_near) cone_voxel(a, q, node, own, own_edge, edges_ok, o, d, w[0], w[1], w[2]);
                        cone_voxel_rx(a, q, node, o, d, w[0], w[1], w[2]);
                    }
            }
        }
        // next voxel: the nearest boundary along the ray
        float tn = INFINITY;
        int ax = -1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (d[k] == 0.f) continue;
            const float b = g.org[k] + (float)(d[k] > 0.f ? c[k] + 1 : c[k]) * g.V;
            const float t = (b - o[k]) / d[k];
            if (t < tn) {
                tn = t;
                ax = k;
            }
        }
        if (ax < 0 || !(tn <= t_end)) break;
        c[ax] += d[ax] > 0.f ? 1 : -1;
        if (c[ax] < 0 || c[ax] >= g.dims[ax]) break;
        step_axis = ax;
    }
}

// ---------------------------------------------------------------------------
// generations: children, merge of similar partial paths, receptions
// ---------------------------------------------------------------------------

struct SplitArgs {
    uint32_t n;
    const uint32_t* cand_node;
    const uint32_t* cand_target;
    const uint32_t* visible;
    uint32_t* child_count;   // [1]
    uint32_t* child_node;
    uint32_t* child_ie;
    uint32_t* rec_count;     // [1]
    Rec* rec;
    uint32_t rec_cap;
    uint32_t k;              // interactions of the parents
    const float4* parent_pos;
    const float4* rx;
};

__global__ void k_split(SplitArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool v = i < a.n && a.visible[i];
    const uint32_t tg = v ? a.cand_target[i] : 0u;
    const bool is_rx = v && (tg & RX_BIT);
    const bool is_ie = v && !(tg & RX_BIT);
    const uint32_t cs = wave_append(a.child_count, is_ie ? 1u : 0u);
    const uint32_t rs = wave_append(a.rec_count, is_rx ? 1u : 0u);
    if (is_ie) {
        a.child_node[cs] = a.cand_node[i];
        a.child_ie[cs] = tg;
    }
    if (is_rx && rs < a.rec_cap) {
        const uint32_t node = a.cand_node[i];
        const float4 P = a.parent_pos[node];
        const float4 R = a.rx[tg & ~RX_BIT];
        const float dx = R.x - P.x, dy = R.y - P.y, dz = R.z - P.z;
        Rec r;
        r.node = node;
        r.rx = tg & ~RX_BIT;
        r.k = a.k;
        r.len = P.w + sqrtf(dx * dx + dy * dy + dz * dz);
        a.rec[rs] = r;
    }
}

struct ChildArgs {
    uint32_t n;
    const uint32_t* node;        // parent index
    const uint32_t* ie;
    const uint32_t* parent_gid;  // the TX index for k = 0
    const uint64_t* parent_prio;
    const uint32_t* ie_label;
    uint64_t* key;               // out: parent gid << 32 | label
    uint64_t* prio;              // out
};

__global__ void k_child_keys(ChildArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const uint32_t p = a.node[i], e = a.ie[i];
    a.key[i] = ((uint64_t)a.parent_gid[p] << 32) | a.ie_label[e];
    a.prio[i] = splitmix64(a.parent_prio[p] + (uint64_t)e + 1ull);
}

template <typename T>
__global__ void k_gather_by(const T* src, const uint32_t* perm, uint32_t n, T* dst) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

// In sorted order (key, IE, priority, parent): flags of the first child of
// every (key, IE) group (kept) and of every key group (new label group).
__global__ void k_merge_flags(const uint64_t* key, const uint32_t* ie, const uint32_t* perm, uint32_t n,
                              uint32_t* keep, uint32_t* newgroup) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = perm[i];
    bool first_key = i == 0, first_ie = i == 0;
    if (i > 0) {
        const uint32_t b = perm[i - 1];
        first_key = key[b] != key[c];
        first_ie = first_key || ie[b] != ie[c];
    }
    keep[i] = first_ie ? 1u : 0u;
    newgroup[i] = (first_key && first_ie) ? 1u : 0u;
}

struct NodeArgs {
    uint32_t n;
    const uint32_t* perm;
    const uint32_t* keep;        // exclusive scan of the keep flags ([n + 1])
    const uint32_t* group;       // exclusive scan of the new-group flags
    const uint32_t* newgroup;
    const uint32_t* node;
    const uint32_t* ie;
    const uint64_t* prio;
    const float4* parent_pos;
    const uint32_t* parent_tx;   // null for k = 0 (the parent is the TX)
    const uint32_t* parent_ndiff;// null for k = 0
    const float4* ie_pos;
    const uint32_t* ie_type;
    Gen out;
};

__global__ void k_make_nodes(NodeArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    if (a.keep[i + 1] == a.keep[i]) return;
    const uint32_t s = a.keep[i];
    const uint32_t c = a.perm[i];
    const uint32_t p = a.node[c], e = a.ie[c];
    const float4 P = a.parent_pos[p];
    const float4 Q = a.ie_pos[e];
    const float dx = Q.x - P.x, dy = Q.y - P.y, dz = Q.z - P.z;
    a.out.apex[s] = make_float4(Q.x, Q.y, Q.z, P.w + sqrtf(dx * dx + dy * dy + dz * dz));
    a.out.ie[s] = e;
    a.out.parent[s] = p;
    a.out.tx[s] = a.parent_tx ? a.parent_tx[p] : p;
    a.out.gid[s] = a.group[i] + a.newgroup[i] - 1u;
    a.out.prio[s] = a.prio[c];
    a.out.ndiff[s] = (a.parent_ndiff ? a.parent_ndiff[p] : 0u) + a.ie_type[e];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static unsigned blocks(int64_t n, int b = 256) { return (unsigned)std::max<int64_t>(1, (n + b - 1) / b); }

static int read_u32(uint32_t* dev, uint32_t* host, hipStream_t s) { return read_back(host, dev, 4, s); }

static int grid_of(const PcrlIeGrid* p, IeGrid& g) {
    if (!p || p->dv < 1 || p->dv > 8 || !(p->voxel > 0.f) || !std::isfinite(p->voxel)) return PCRL_EINVAL;
    int64_t nv = 1;
    for (int a = 0; a < 3; ++a) {
        if (p->dims[a] < 1 || !std::isfinite(p->origin[a])) return PCRL_EINVAL;
        nv *= p->dims[a];
    }
    if (nv * p->dv * p->dv * p->dv >= ((int64_t)1 << 31)) return PCRL_EINVAL;
    for (int a = 0; a < 3; ++a) {
        g.org[a] = p->origin[a];
        g.dims[a] = p->dims[a];
    }
    g.V = p->voxel;
    g.dv = p->dv;
    g.sv = p->voxel / (float)p->dv;
    g.inv_sv = 1.0f / g.sv;
    return PCRL_OK;
}

static int64_t n_voxels(const IeGrid& g) { return (int64_t)g.dims[0] * g.dims[1] * g.dims[2]; }

static int ie_build_impl(PcrlScene* S, const PcrlIeGrid* params, hipStream_t s, PcrlIes** out) {
    std::unique_ptr<PcrlIes> I(new PcrlIes());
    I->scene = S;
    I->device = S->device;
    if (grid_of(params, I->g)) {
        set_error("ie_build: need dv in 1..8, voxel > 0, dims >= 1 and dims product * dv^3 < 2^31");
        return PCRL_EINVAL;
    }
    if (S->overlay && S->overlay->n_entries > 0) {
        set_error("ie_build: the scene has dynamic points (update_points); IEs are built from the static points");
        return PCRL_EINVAL;
    }
    const int64_t np = S->info.n_points;
    if (np >= ((int64_t)1 << 31)) {
        set_error("ie_build: at most 2^31 - 1 points");
        return PCRL_EINVAL;
    }
    I->bufs.stream = s;
    DevBufs T;
    T.stream = s;
    auto fail = [&](int rc) { T.release(); I->bufs.release(); return rc; };
    const IeGrid g = I->g;
    I->n_vox = n_voxels(g);
    int rc;
    if ((rc = I->bufs.alloc(&I->vox, (size_t)I->n_vox)) || (rc = I->bufs.alloc(&I->near, (size_t)I->n_vox)))
        return fail(rc);
    if ((rc = fill_u32((uint32_t*)I->vox, 0u, 2 * I->n_vox, s))) return fail(rc);
    const uint32_t n = (uint32_t)np;
    if (n > 0) {
        if ((rc = scene_own_index(S, s))) return fail(rc);
        uint64_t* key = nullptr;
        uint32_t *id = nullptr, *flag = nullptr, *bad = nullptr;
        if ((rc = T.alloc(&key, n)) || (rc = T.alloc(&id, n)) || (rc = T.alloc(&flag, (size_t)n + 1)) ||
            (rc = T.alloc(&bad, 1)))
            return fail(rc);
        if ((rc = fill_u32(bad, 0u, 1, s))) return fail(rc);
        hipLaunchKernelGGL(k_ie_keys, dim3(blocks(n)), dim3(256), 0, s, S->own_pos, S->own_nrm, n, g, key, id, bad);
        uint32_t h_bad = 0;
        if ((rc = read_u32(bad, &h_bad, s))) return fail(rc);
        if (h_bad) {
            set_error("ie_build: %u points lie outside the IE grid", h_bad);
            return fail(PCRL_EINVAL);
        }
        int bits = 1;
        const uint64_t max_cell = (uint64_t)I->n_vox * (uint64_t)(g.dv * g.dv * g.dv);
        while (bits < 32 && (max_cell >> bits)) ++bits;
        if ((rc = radix_sort_u64(key, id, n, 32 + bits, s))) return fail(rc);
        hipLaunchKernelGGL(k_ie_flags, dim3(blocks(n)), dim3(256), 0, s, key, n, flag);
        if ((rc = scan_u32(flag, flag, n, flag + n, s))) return fail(rc);
        uint32_t n_ie = 0;
        if ((rc = read_u32(flag + n, &n_ie, s))) return fail(rc);
        I->n_ie = n_ie;
        if ((rc = I->bufs.alloc(&I->key, n_ie)) || (rc = I->bufs.alloc(&I->sub, (size_t)n_ie * 3)) ||
            (rc = I->bufs.alloc(&I->label, n_ie)) || (rc = I->bufs.alloc(&I->count, n_ie)) ||
            (rc = I->bufs.alloc(&I->pos, n_ie)) || (rc = I->bufs.alloc(&I->nrm, n_ie)))
            return fail(rc);
        hipLaunchKernelGGL(k_ie_reduce, dim3(blocks(n)), dim3(256), 0, s, key, id, flag, n, S->own_pos, S->own_nrm, g,
                           n_ie, I->key, I->sub, I->label, I->count, I->pos, I->nrm);
        if ((rc = I->bufs.alloc(&I->type, n_ie)) || (rc = I->bufs.alloc(&I->eid, n_ie)) ||
            (rc = fill_u32(I->type, 0u, n_ie, s)) || (rc = fill_u32(I->eid, 0xFFFFFFFFu, n_ie, s)))
            return fail(rc);
        hipLaunchKernelGGL(k_ie_voxels, dim3(blocks(n_ie)), dim3(256), 0, s, I->key, n_ie, g.dv * g.dv * g.dv,
                           I->vox);
    }
    hipLaunchKernelGGL(k_ie_near, dim3(blocks(I->n_vox)), dim3(256), 0, s, I->vox, (const uint2*)nullptr, g,
                       (uint32_t)I->n_vox, I->near);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        set_error("ie_build: kernels failed: %s", hipGetErrorString(hipGetLastError()));
        return fail(PCRL_EHIP);
    }
    T.release();
    // occupied voxels (host count from the table)
    std::vector<uint2> hv((size_t)I->n_vox);
    if (hipMemcpy(hv.data(), I->vox, hv.size() * sizeof(uint2), hipMemcpyDeviceToHost) != hipSuccess) {
        set_error("ie_build: reading the voxel table failed");
        return fail(PCRL_EHIP);
    }
    for (const uint2& r : hv) I->n_occ += r.y ? 1 : 0;
    I->n_pt = I->n_ie;
    I->bytes = I->n_ie * (8 + 12 + 4 + 4 + 32 + 8) + I->n_vox * 9;
    *out = I.release();
    return PCRL_OK;
}

static int ie_add_edges_impl(PcrlIes* I, const float* seg, const float* nrm, const uint32_t* label, int64_t n_edges,
                             hipStream_t s) {
    if (I->n_edges) {
        set_error("ie_add_edges: the table already has edges");
        return PCRL_EINVAL;
    }
    if (n_edges == 0) return PCRL_OK;
    const IeGrid g = I->g;
    DevBufs T;
    T.stream = s;
    auto fail = [&](int rc) { T.release(); return rc; };
    const uint32_t n = (uint32_t)n_edges;
    uint32_t *cnt = nullptr, *bad = nullptr;
    int rc;
    if ((rc = T.alloc(&cnt, (size_t)n + 1)) || (rc = T.alloc(&bad, 1)) || (rc = fill_u32(bad, 0u, 1, s)))
        return fail(rc);
    EdgeArgs A{seg, nrm, label, n, g, cnt, cnt, bad, nullptr, nullptr, nullptr, nullptr};
    hipLaunchKernelGGL(k_edge_count, dim3(blocks(n)), dim3(256), 0, s, A);
    if ((rc = scan_u32(cnt, cnt, n, cnt + n, s))) return fail(rc);
    uint32_t P = 0, h_bad = 0;
    if ((rc = read_u32(cnt + n, &P, s)) || (rc = read_u32(bad, &h_bad, s))) return fail(rc);
    if (h_bad) {
        set_error("ie_add_edges: %u edges have zero length", h_bad);
        return fail(PCRL_EINVAL);
    }
    // counts again (the scan replaced them) for the write pass
    uint32_t* cnt2 = nullptr;
    uint64_t* key = nullptr;
    uint32_t *edge = nullptr, *perm = nullptr;
    int32_t* sub = nullptr;
    float4* pos = nullptr;
    if ((rc = T.alloc(&cnt2, n)) || (rc = T.alloc(&key, P)) || (rc = T.alloc(&edge, P)) || (rc = T.alloc(&perm, P)) ||
        (rc = T.alloc(&sub, (size_t)P * 3)) || (rc = T.alloc(&pos, P)))
        return fail(rc);
    EdgeArgs C{seg, nrm, label, n, g, cnt, cnt2, bad, key, edge, sub, pos};
    hipLaunchKernelGGL(k_edge_count, dim3(blocks(n)), dim3(256), 0, s, C);
    hipLaunchKernelGGL(k_edge_write, dim3(blocks(n)), dim3(256), 0, s, C);
    if ((rc = read_u32(bad, &h_bad, s))) return fail(rc);
    if (h_bad) {
        set_error("ie_add_edges: %u edge pieces lie outside the IE grid", h_bad);
        return fail(PCRL_EINVAL);
    }
    // stable sort of the (edge, t)-ordered pieces by key: (key, edge) order
    if ((rc = iota_u32(perm, P, s))) return fail(rc);
    int bits = 1;
    const uint64_t max_cell = (uint64_t)I->n_vox * (uint64_t)(g.dv * g.dv * g.dv);
    while (bits < 32 && (max_cell >> bits)) ++bits;
    if ((rc = radix_sort_u64(key, perm, P, 32 + bits, s))) return fail(rc);
    // the combined arrays
    const uint32_t n_pt = (uint32_t)I->n_pt, N = n_pt + P;
    uint64_t* nkey = nullptr;
    int32_t* nsub = nullptr;
    uint32_t *nlabel = nullptr, *ncount = nullptr, *ntype = nullptr, *neid = nullptr;
    float4 *npos = nullptr, *nnrm = nullptr, *ew = nullptr, *en1 = nullptr, *en2 = nullptr;
    uint2* vox_e = nullptr;
    float *lseg = nullptr, *lnrm = nullptr;
    uint32_t* llab = nullptr;
    DevBufs& B = I->bufs;
    if ((rc = B.alloc(&nkey, N)) || (rc = B.alloc(&nsub, (size_t)N * 3)) || (rc = B.alloc(&nlabel, N)) ||
        (rc = B.alloc(&ncount, N)) || (rc = B.alloc(&ntype, N)) || (rc = B.alloc(&neid, N)) ||
        (rc = B.alloc(&npos, N)) || (rc = B.alloc(&nnrm, N)) || (rc = B.alloc(&ew, P)) || (rc = B.alloc(&en1, P)) ||
        (rc = B.alloc(&en2, P)) || (rc = B.alloc(&vox_e, (size_t)I->n_vox)) || (rc = B.alloc(&lseg, (size_t)n * 6)) ||
        (rc = B.alloc(&lnrm, (size_t)n * 6)) || (rc = B.alloc(&llab, n)))
        return fail(rc);
    hipError_t e = hipMemcpyAsync(lseg, seg, (size_t)n * 24, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(lnrm, nrm, (size_t)n * 24, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(llab, label, (size_t)n * 4, hipMemcpyDeviceToDevice, s);
    if (n_pt && e == hipSuccess) {
        e = hipMemcpyAsync(nkey, I->key, (size_t)n_pt * 8, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(nsub, I->sub, (size_t)n_pt * 12, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(nlabel, I->label, (size_t)n_pt * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(ncount, I->count, (size_t)n_pt * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(ntype, I->type, (size_t)n_pt * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(neid, I->eid, (size_t)n_pt * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(npos, I->pos, (size_t)n_pt * 16, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(nnrm, I->nrm, (size_t)n_pt * 16, hipMemcpyDeviceToDevice, s);
    }
    if (e != hipSuccess) {
        set_error("ie_add_edges: copy failed: %s", hipGetErrorString(e));
        return fail(PCRL_EHIP);
    }
    EdgeAppend ap{perm, P, n_pt, key, edge, sub, pos, seg, nrm, nkey, nsub, nlabel, ncount, npos, nnrm, ntype, neid,
                  ew, en1, en2};
    hipLaunchKernelGGL(k_edge_append, dim3(blocks(P)), dim3(256), 0, s, ap);
    if ((rc = fill_u32((uint32_t*)vox_e, 0u, 2 * I->n_vox, s))) return fail(rc);
    hipLaunchKernelGGL(k_edge_voxels, dim3(blocks(P)), dim3(256), 0, s, nkey, n_pt, N, g.dv * g.dv * g.dv, vox_e);
    hipLaunchKernelGGL(k_ie_near, dim3(blocks(I->n_vox)), dim3(256), 0, s, I->vox, (const uint2*)vox_e, g,
                       (uint32_t)I->n_vox, I->near);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        set_error("ie_add_edges: kernels failed: %s", hipGetErrorString(hipGetLastError()));
        return fail(PCRL_EHIP);
    }
    I->key = nkey;
    I->sub = nsub;
    I->label = nlabel;
    I->count = ncount;
    I->type = ntype;
    I->eid = neid;
    I->pos = npos;
    I->nrm = nnrm;
    I->ew = ew;
    I->en1 = en1;
    I->en2 = en2;
    I->vox_e = vox_e;
    I->n_ie = N;
    I->n_edges = P;
    I->n_lines = n;
    I->line_seg = lseg;
    I->line_nrm = lnrm;
    I->line_label = llab;
    I->bytes += (int64_t)P * (8 + 12 + 4 + 4 + 32 + 8 + 48) + I->n_vox * 8 + (int64_t)n * 52;
    T.release();
    return PCRL_OK;
}

template <int NL, bool BX>
static void launch_vis(const VisArgs& a, hipStream_t s) {
    const unsigned grid = (unsigned)std::min<int64_t>(blocks(a.n, TRACE_BLOCK), (int64_t)device_cus() * 16);
    hipLaunchKernelGGL((k_visibility<NL, BX>), dim3(grid), dim3(TRACE_BLOCK), 0, s, a);
}

template <int NL, bool BX>
static void launch_axis(const AxisArgs& a, hipStream_t s) {
    const unsigned grid = (unsigned)std::min<int64_t>(blocks(a.cones.n, TRACE_BLOCK), (int64_t)device_cus() * 16);
    hipLaunchKernelGGL((k_axis<NL, BX>), dim3(grid), dim3(TRACE_BLOCK), 0, s, a);
}

template <int NL>
static void dispatch_vis(const VisArgs& a, hipStream_t s) {
    if (NL > 1 && !a.t.v.cells) launch_vis<NL, true>(a, s);
    else launch_vis<NL, false>(a, s);
}

template <int NL>
static void dispatch_axis(const AxisArgs& a, hipStream_t s) {
    if (NL > 1 && !a.t.v.cells) launch_axis<NL, true>(a, s);
    else launch_axis<NL, false>(a, s);
}

static void run_vis(const VisArgs& a, hipStream_t s) {
    if (a.n == 0) return;
    switch (a.t.v.nlev) {
    case 1: dispatch_vis<1>(a, s); break;
    case 2: dispatch_vis<2>(a, s); break;
    case 3: dispatch_vis<3>(a, s); break;
    default: dispatch_vis<4>(a, s); break;
    }
}

static void run_axis(const AxisArgs& a, hipStream_t s) {
    if (a.cones.n == 0) return;
    switch (a.t.v.nlev) {
    case 1: dispatch_axis<1>(a, s); break;
    case 2: dispatch_axis<2>(a, s); break;
    case 3: dispatch_axis<3>(a, s); break;
    default: dispatch_axis<4>(a, s); break;
    }
}

__global__ void k_pairs(uint32_t n_tx, uint32_t n_t, uint32_t n_ie, uint32_t* node, uint32_t* target) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)n_tx * n_t) return;
    const uint32_t t = (uint32_t)(i % n_t);
    node[i] = (uint32_t)(i / n_t);
    target[i] = t < n_ie ? t : (RX_BIT | (t - n_ie));
}

__global__ void k_pack_antennas(const float* p, int32_t n, IeGrid g, float4* out, int32_t* sub, uint32_t* bad) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float c[3] = {p[3 * i], p[3 * i + 1], p[3 * i + 2]};
    out[i] = make_float4(c[0], c[1], c[2], 0.f);
    if (!sub) return;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float u = floorf((c[a] - g.org[a]) * g.inv_sv);
        if (!(u >= 0.f && u < (float)(g.dims[a] * g.dv))) {
            atomicAdd(bad, 1u);
            sub[3 * i + a] = 0;
        } else {
            sub[3 * i + a] = (int)u;
        }
    }
}

__global__ void k_root_prio(uint32_t n_tx, uint64_t* prio, uint32_t* gid) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_tx) return;
    prio[i] = splitmix64(i);
    gid[i] = i;
}

// Children of the visible IE candidates -> merged, sorted generation.
static int make_generation(PcrlConeLaunch* L, uint32_t n_child, const uint32_t* child_node, const uint32_t* child_ie,
                           const uint32_t* parent_gid, const uint64_t* parent_prio, const float4* parent_pos,
                           const uint32_t* parent_tx, const uint32_t* parent_ndiff, Gen& out, hipStream_t s) {
    const PcrlIes* I = L->ies;
    DevBufs T;
    T.stream = s;
    auto fail = [&](int rc) { T.release(); return rc; };
    out.n = 0;
    if (n_child == 0) return PCRL_OK;
    const uint32_t n = n_child;
    uint64_t *key = nullptr, *prio = nullptr, *tmp64 = nullptr;
    uint32_t *perm = nullptr, *tmp32 = nullptr, *keep = nullptr, *grp = nullptr, *newg = nullptr;
    int rc;
    if ((rc = T.alloc(&key, n)) || (rc = T.alloc(&prio, n)) || (rc = T.alloc(&tmp64, n)) || (rc = T.alloc(&perm, n)) ||
        (rc = T.alloc(&tmp32, n)) || (rc = T.alloc(&keep, (size_t)n + 1)) || (rc = T.alloc(&grp, (size_t)n + 1)) ||
        (rc = T.alloc(&newg, n)))
        return fail(rc);
    ChildArgs ca{n, child_node, child_ie, parent_gid, parent_prio, I->label, key, prio};
    hipLaunchKernelGGL(k_child_keys, dim3(blocks(n)), dim3(256), 0, s, ca);
    if ((rc = iota_u32(perm, n, s))) return fail(rc);
    // LSD by parent, priority, IE, key: sorted by (key, IE, priority, parent)
    hipLaunchKernelGGL(k_gather_by<uint32_t>, dim3(blocks(n)), dim3(256), 0, s, child_node, perm, n, tmp32);
    if ((rc = radix_sort_u32(tmp32, perm, n, 32, s))) return fail(rc);
    hipLaunchKernelGGL(k_gather_by<uint64_t>, dim3(blocks(n)), dim3(256), 0, s, prio, perm, n, tmp64);
    if ((rc = radix_sort_u64(tmp64, perm, n, 64, s))) return fail(rc);
    hipLaunchKernelGGL(k_gather_by<uint32_t>, dim3(blocks(n)), dim3(256), 0, s, child_ie, perm, n, tmp32);
    if ((rc = radix_sort_u32(tmp32, perm, n, 32, s))) return fail(rc);
    hipLaunchKernelGGL(k_gather_by<uint64_t>, dim3(blocks(n)), dim3(256), 0, s, key, perm, n, tmp64);
    if ((rc = radix_sort_u64(tmp64, perm, n, 64, s))) return fail(rc);
    hipLaunchKernelGGL(k_merge_flags, dim3(blocks(n)), dim3(256), 0, s, key, child_ie, perm, n, keep, newg);
    if ((rc = scan_u32(keep, keep, n, keep + n, s))) return fail(rc);
    if ((rc = scan_u32(newg, grp, n, grp + n, s))) return fail(rc);
    uint32_t n_keep = 0;
    if ((rc = read_u32(keep + n, &n_keep, s))) return fail(rc);
    DevBufs& B = L->bufs;
    if ((rc = B.alloc(&out.apex, n_keep)) || (rc = B.alloc(&out.ie, n_keep)) || (rc = B.alloc(&out.parent, n_keep)) ||
        (rc = B.alloc(&out.tx, n_keep)) || (rc = B.alloc(&out.gid, n_keep)) || (rc = B.alloc(&out.prio, n_keep)) ||
        (rc = B.alloc(&out.ndiff, n_keep)))
        return fail(rc);
    out.n = n_keep;
    NodeArgs na{n, perm, keep, grp, newg, child_node, child_ie, prio, parent_pos, parent_tx, parent_ndiff, I->pos,
                I->type, out};
    hipLaunchKernelGGL(k_make_nodes, dim3(blocks(n)), dim3(256), 0, s, na);
    if (hipGetLastError() != hipSuccess) {
        set_error("cone_launch: merge kernels failed");
        return fail(PCRL_EHIP);
    }
    T.release();
    return PCRL_OK;
}

static double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static int cone_launch_impl(const PcrlIes* I, const float* tx, int32_t n_tx, const float* rx, int32_t n_rx,
                            const PcrlConeParams* P, hipStream_t s, PcrlConeLaunch** out) {
    const PcrlScene* S = I->scene;
    std::unique_ptr<PcrlConeLaunch> L(new PcrlConeLaunch());
    L->ies = I;
    L->n_tx = n_tx;
    L->n_rx = n_rx;
    L->K = P->max_interactions;
    L->bufs.stream = s;
    const int K = L->K;
    const float half = P->half_angle > 0.f ? P->half_angle : (float)(2.5 * M_PI / 180.0);
    DevBufs T;
    T.stream = s;
    auto fail = [&](int rc) { T.release(); L->bufs.release(); return rc; };
    int rc;
    int32_t* rx_sub = nullptr;
    uint32_t *bad = nullptr, *counters = nullptr;
    uint64_t* root_prio = nullptr;
    uint32_t* root_gid = nullptr;
    if ((rc = L->bufs.alloc(&L->tx, n_tx)) || (rc = L->bufs.alloc(&L->rx, std::max(n_rx, 1))) ||
        (rc = T.alloc(&rx_sub, (size_t)std::max(n_rx, 1) * 3)) || (rc = T.alloc(&bad, 1)) ||
        (rc = T.alloc(&counters, 4)) || (rc = T.alloc(&root_prio, n_tx)) || (rc = T.alloc(&root_gid, n_tx)))
        return fail(rc);
    if ((rc = fill_u32(bad, 0u, 1, s))) return fail(rc);
    hipLaunchKernelGGL(k_pack_antennas, dim3(blocks(n_tx)), dim3(256), 0, s, tx, n_tx, I->g, L->tx, (int32_t*)nullptr,
                       bad);
    if (n_rx > 0)
        hipLaunchKernelGGL(k_pack_antennas, dim3(blocks(n_rx)), dim3(256), 0, s, rx, n_rx, I->g, L->rx, rx_sub, bad);
    hipLaunchKernelGGL(k_root_prio, dim3(blocks(n_tx)), dim3(256), 0, s, (uint32_t)n_tx, root_prio, root_gid);
    uint32_t h_bad = 0;
    if ((rc = read_u32(bad, &h_bad, s))) return fail(rc);
    if (h_bad) {
        set_error("cone_launch: an RX lies outside the IE grid");
        return fail(PCRL_EINVAL);
    }
    TraceArgs ta{};
    ta.v = S->view;
    VisArgs va{};
    va.t = ta;
    va.g = I->g;
    va.ie_pos = I->pos;
    va.ie_sub = I->sub;
    va.rx = L->rx;
    va.rx_sub = rx_sub;
    L->gens.assign((size_t)K + 2, Gen{});
    std::vector<Rec> recs;
    auto add_records = [&](uint32_t n_rec, Rec* dev) -> int {
        const size_t at = recs.size();
        recs.resize(at + n_rec);
        if (n_rec && hipMemcpy(recs.data() + at, dev, (size_t)n_rec * sizeof(Rec), hipMemcpyDeviceToHost) != hipSuccess)
            return PCRL_EHIP;
        return PCRL_OK;
    };
    const double t0 = now_ms();
    // ---- transmission phase: every TX towards every IE and RX
    // edge pieces are targets only when diffraction is allowed
    const int32_t max_diff = P->max_diffractions;
    const uint64_t n_tie = max_diff > 0 ? (uint64_t)I->n_ie : (uint64_t)I->n_pt;
    const uint64_t n_t = n_tie + (uint64_t)n_rx;
    const uint64_t n_pairs = (uint64_t)n_tx * n_t;
    if (n_pairs >= ((uint64_t)1 << 31)) {
        set_error("cone_launch: %llu transmission rays exceed 2^31", (unsigned long long)n_pairs);
        return fail(PCRL_EINVAL);
    }
    uint32_t n_child = 0;
    uint32_t *child_node = nullptr, *child_ie = nullptr;
    {
        const uint32_t n = (uint32_t)n_pairs;
        uint32_t *node = nullptr, *target = nullptr, *vis = nullptr;
        Rec* rec = nullptr;
        if ((rc = T.alloc(&node, std::max(n, 1u))) || (rc = T.alloc(&target, std::max(n, 1u))) ||
            (rc = T.alloc(&vis, std::max(n, 1u))) || (rc = T.alloc(&child_node, std::max(n, 1u))) ||
            (rc = T.alloc(&child_ie, std::max(n, 1u))) || (rc = T.alloc(&rec, std::max<uint32_t>(n_tx * n_rx, 1u))))
            return fail(rc);
        if (n) hipLaunchKernelGGL(k_pairs, dim3(blocks(n)), dim3(256), 0, s, (uint32_t)n_tx, (uint32_t)n_t,
                                  (uint32_t)n_tie, node, target);
        va.origin = L->tx;
        va.cand_node = node;
        va.cand_target = target;
        va.n = n;
        va.visible = vis;
        run_vis(va, s);
        if ((rc = fill_u32(counters, 0u, 4, s))) return fail(rc);
        SplitArgs sa{n, node, target, vis, counters, child_node, child_ie, counters + 1, rec,
                     (uint32_t)std::max(n_tx * n_rx, 1), 0u, L->tx, L->rx};
        if (n) hipLaunchKernelGGL(k_split, dim3(blocks(n)), dim3(256), 0, s, sa);
        uint32_t h[2] = {0, 0};
        if (hipGetLastError() != hipSuccess || read_back(h, counters, 8, s)) {
            set_error("cone_launch: transmission kernels failed: %s", hipGetErrorString(hipGetLastError()));
            return fail(PCRL_EHIP);
        }
        n_child = h[0];
        if ((rc = add_records(h[1], rec))) return fail(rc);
        L->stats.candidates[0] = n;
        L->stats.visible[0] = (int64_t)h[0] + h[1];
    }
    L->stats.ms_transmission = now_ms() - t0;
    const double t1 = now_ms();
    // ---- propagation: generations 1..K
    const uint32_t* p_gid = root_gid;
    const uint64_t* p_prio = root_prio;
    const float4* p_pos = L->tx;
    const uint32_t* p_tx = nullptr;
    const uint32_t* p_ndiff = nullptr;
    const float cos_t = cosf(half), sin_t = sinf(half);
    const float R = I->g.sv * sqrtf(3.0f) * 0.5f;
    for (int k = 1; k <= K; ++k) {
        Gen& G = L->gens[k];
        if ((rc = make_generation(L.get(), n_child, child_node, child_ie, p_gid, p_prio, p_pos, p_tx, p_ndiff, G,
                                  s)))
            return fail(rc);
        L->stats.nodes[k] = G.n;
        if (G.n == 0) break;
        // the generation's cones: count per node, scan, fill
        Cones cs;
        uint32_t* ccount = nullptr;
        if ((rc = T.alloc(&ccount, (size_t)G.n + 1))) return fail(rc);
        ExpandArgs ea{G, p_pos, I->type, I->nrm, I->ew, I->en1, I->en2, (uint32_t)I->n_pt, half, ccount, ccount, cs};
        hipLaunchKernelGGL(k_cone_count, dim3(blocks(G.n)), dim3(256), 0, s, ea);
        if ((rc = scan_u32(ccount, ccount, G.n, ccount + G.n, s))) return fail(rc);
        if ((rc = read_u32(ccount + G.n, &cs.n, s))) return fail(rc);
        if (cs.n == 0) break;
        if ((rc = T.alloc(&cs.node, cs.n)) || (rc = T.alloc(&cs.axis, cs.n)) || (rc = T.alloc(&cs.s0, cs.n)) ||
            (rc = T.alloc(&cs.s1, cs.n)) || (rc = T.alloc(&cs.kind, cs.n)) || (rc = T.alloc(&cs.t_end, cs.n)))
            return fail(rc);
        ea.out = cs;
        hipLaunchKernelGGL(k_cone_fill, dim3(blocks(G.n)), dim3(256), 0, s, ea);
        L->stats.cones[k] = cs.n;
        AxisArgs aa{ta, G.apex, cs};
        run_axis(aa, s);
        // candidates: a first guess, then exactly what the kernel counted
        uint32_t cap = (uint32_t)std::min<int64_t>((int64_t)cs.n * 64 + 1024, (int64_t)1 << 30);
        uint32_t *cnode = nullptr, *ctarget = nullptr;
        uint32_t n_cand = 0;
        for (int attempt = 0; attempt < 2; ++attempt) {
            if ((rc = T.alloc(&cnode, cap)) || (rc = T.alloc(&ctarget, cap))) return fail(rc);
            if ((rc = fill_u32(counters, 0u, 4, s))) return fail(rc);
            ConeArgs c{};
            c.g = I->g;
            c.gen = G;
            c.cones = cs;
            c.vox = I->vox;
            c.vox_e = I->vox_e;
            c.eid = I->eid;
            c.max_diff = max_diff;
            c.near = I->near;
            c.ie_pos = I->pos;
            c.ie_sub = I->sub;
            c.rx = L->rx;
            c.rx_sub = rx_sub;
            c.n_rx = n_rx;
            c.want_ie = k < K ? 1 : 0;
            c.cos_t = cos_t;
            c.sin_t = sin_t;
            c.tau = 1e-3f * I->g.sv;
            c.R = R;
            c.cap = cap;
            c.n_cand = counters;
            c.cand_node = cnode;
            c.cand_target = ctarget;
            hipLaunchKernelGGL(k_cones, dim3(blocks(cs.n, CONE_BLOCK)), dim3(CONE_BLOCK), 0, s, c);
            if (hipGetLastError() != hipSuccess || read_u32(counters, &n_cand, s)) {
                set_error("cone_launch: cone kernel failed: %s", hipGetErrorString(hipGetLastError()));
                return fail(PCRL_EHIP);
            }
            if (n_cand <= cap) break;
            if (n_cand >= ((uint32_t)1 << 30)) {
                set_error("cone_launch: %u cone targets in generation %d exceed 2^30", n_cand, k);
                return fail(PCRL_EINVAL);
            }
            cap = n_cand;
        }
        L->stats.candidates[k] = n_cand;
        uint32_t* vis = nullptr;
        Rec* rec = nullptr;
        uint32_t* nchild_node = nullptr;
        uint32_t* nchild_ie = nullptr;
        if ((rc = T.alloc(&vis, std::max(n_cand, 1u))) || (rc = T.alloc(&rec, std::max(n_cand, 1u))) ||
            (rc = T.alloc(&nchild_node, std::max(n_cand, 1u))) || (rc = T.alloc(&nchild_ie, std::max(n_cand, 1u))))
            return fail(rc);
        va.origin = G.apex;
        va.cand_node = cnode;
        va.cand_target = ctarget;
        va.n = n_cand;
        va.visible = vis;
        run_vis(va, s);
        if ((rc = fill_u32(counters, 0u, 4, s))) return fail(rc);
        SplitArgs sa{n_cand, cnode, ctarget, vis, counters, nchild_node, nchild_ie, counters + 1, rec,
                     std::max(n_cand, 1u), (uint32_t)k, G.apex, L->rx};
        if (n_cand) hipLaunchKernelGGL(k_split, dim3(blocks(n_cand)), dim3(256), 0, s, sa);
        uint32_t h[2] = {0, 0};
        if (hipGetLastError() != hipSuccess || read_back(h, counters, 8, s)) {
            set_error("cone_launch: generation %d kernels failed: %s", k, hipGetErrorString(hipGetLastError()));
            return fail(PCRL_EHIP);
        }
        if ((rc = add_records(h[1], rec))) return fail(rc);
        L->stats.visible[k] = (int64_t)h[0] + h[1];
        n_child = k < K ? h[0] : 0u;
        child_node = nchild_node;
        child_ie = nchild_ie;
        p_gid = G.gid;
        p_prio = G.prio;
        p_pos = G.apex;
        p_tx = G.tx;
        p_ndiff = G.ndiff;
    }
    L->stats.ms_propagation = now_ms() - t1;
    L->n_rec = (int64_t)recs.size();
    L->stats.records = L->n_rec;
    if ((rc = L->bufs.alloc(&L->rec, std::max<size_t>(recs.size(), 1)))) return fail(rc);
    if (!recs.empty() && hipMemcpy(L->rec, recs.data(), recs.size() * sizeof(Rec), hipMemcpyHostToDevice) != hipSuccess) {
        set_error("cone_launch: storing the receptions failed");
        return fail(PCRL_EHIP);
    }
    if (hipStreamSynchronize(s) != hipSuccess) {
        set_error("cone_launch: kernels failed: %s", hipGetErrorString(hipGetLastError()));
        return fail(PCRL_EHIP);
    }
    T.release();
    *out = L.release();
    return PCRL_OK;
}

// ---------------------------------------------------------------------------
// collect: coarse paths (Section 2.2.3)
// ---------------------------------------------------------------------------

struct CollectView {
    Gen gens[PCRL_MAX_REFLECTIONS + 1];
    const float4* tx;
    const uint32_t* ie_label;
    const float4* ie_pos;
};

// Sort key of a reception: (tx, rx, k, label group of its node).
__global__ void k_rec_keys(const Rec* rec, uint32_t n, CollectView cv, uint64_t* key, uint64_t* prio,
                           uint32_t* nodeord) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Rec r = rec[i];
    uint32_t tx = r.node, gid = 0;
    uint64_t pr = splitmix64(r.node);
    if (r.k > 0) {
        const Gen& G = cv.gens[r.k];
        tx = G.tx[r.node];
        gid = G.gid[r.node];
        pr = G.prio[r.node];
    }
    key[i] = ((uint64_t)tx << 56) | ((uint64_t)r.rx << 40) | ((uint64_t)r.k << 36) | (uint64_t)gid;
    prio[i] = pr;
    nodeord[i] = r.node;
}

__global__ void k_rec_groups(const uint64_t* key, const uint32_t* perm, uint32_t n, uint32_t* first) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    first[i] = (i == 0 || key[perm[i]] != key[perm[i - 1]]) ? 1u : 0u;
}

struct RowArgs {
    const Rec* rec;
    const uint64_t* key;
    const uint32_t* perm;
    const uint32_t* first;   // group start flags (sorted order)
    uint32_t n;
    int32_t kappa;
    int32_t K;
    CollectView cv;
    uint32_t* n_rows;        // [2]: rows, keys
    int64_t cap;
    PcrlPaths out;
};

// Rows in sorted order: row slot = exclusive scan of kept counts.
__global__ void k_rec_keepflags(const uint32_t* first, uint32_t n, int32_t kappa, uint32_t* keep) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // rank inside the group: distance to the group start
    uint32_t g = i;
    while (!first[g]) --g;
    keep[i] = (kappa <= 0 || i - g < (uint32_t)kappa) ? 1u : 0u;
}

__global__ void k_rec_write(RowArgs a, const uint32_t* slot) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    if (slot[i + 1] == slot[i]) return;
    const uint32_t row = slot[i];
    if ((int64_t)row >= a.cap) return;
    uint32_t g = i;
    while (!a.first[g]) --g;
    uint32_t j = i + 1;
    while (j < a.n && !a.first[j]) ++j;
    const Rec r = a.rec[a.perm[i]];
    const int K = a.K;
    uint32_t tx = r.node;
    if (r.k > 0) tx = a.cv.gens[r.k].tx[r.node];
    if (a.out.tx) a.out.tx[row] = (int32_t)tx;
    if (a.out.rx) a.out.rx[row] = (int32_t)r.rx;
    if (a.out.n_refl) a.out.n_refl[row] = (int32_t)r.k;
    if (a.out.count) a.out.count[row] = (int64_t)(j - g);
    if (a.out.rank) a.out.rank[row] = (int32_t)(i - g);
    if (a.out.ray) a.out.ray[row] = ((int64_t)r.k << 40) | (int64_t)r.node;
    if (a.out.len_poly) a.out.len_poly[row] = r.len;
    if (a.out.len_unf) a.out.len_unf[row] = r.len;
    for (int q = 0; q < K; ++q) {
        if (a.out.key) a.out.key[(size_t)row * K + q] = -1;
        if (a.out.points)
            for (int c = 0; c < 3; ++c) a.out.points[((size_t)row * K + q) * 3 + c] = NAN;
    }
    uint32_t node = r.node;
    for (int q = (int)r.k; q >= 1; --q) {
        const Gen& G = a.cv.gens[q];
        const uint32_t e = G.ie[node];
        if (a.out.key) a.out.key[(size_t)row * K + (q - 1)] = (int64_t)a.cv.ie_label[e];
        if (a.out.points) {
            const float4 P = a.cv.ie_pos[e];
            a.out.points[((size_t)row * K + (q - 1)) * 3] = P.x;
            a.out.points[((size_t)row * K + (q - 1)) * 3 + 1] = P.y;
            a.out.points[((size_t)row * K + (q - 1)) * 3 + 2] = P.z;
        }
        node = G.parent[node];
    }
}

static int cone_collect_impl(PcrlConeLaunch* L, int32_t kappa, PcrlPaths* out, hipStream_t s) {
    out->n_rows = 0;
    out->n_keys = 0;
    const uint32_t n = (uint32_t)L->n_rec;
    if (n == 0) return PCRL_OK;
    DevBufs T;
    T.stream = s;
    auto fail = [&](int rc) { T.release(); return rc; };
    uint64_t *key = nullptr, *prio = nullptr, *tmp64 = nullptr;
    uint32_t *perm = nullptr, *ord = nullptr, *tmp32 = nullptr, *first = nullptr, *slot = nullptr, *cnt = nullptr;
    int rc;
    if ((rc = T.alloc(&key, n)) || (rc = T.alloc(&prio, n)) || (rc = T.alloc(&tmp64, n)) || (rc = T.alloc(&perm, n)) ||
        (rc = T.alloc(&ord, n)) || (rc = T.alloc(&tmp32, n)) || (rc = T.alloc(&first, n)) ||
        (rc = T.alloc(&slot, (size_t)n + 1)) || (rc = T.alloc(&cnt, 2)))
        return fail(rc);
    CollectView cv{};
    for (int k = 1; k <= L->K && k <= PCRL_MAX_REFLECTIONS; ++k) cv.gens[k] = L->gens[k];
    cv.tx = L->tx;
    cv.ie_label = L->ies->label;
    cv.ie_pos = L->ies->pos;
    hipLaunchKernelGGL(k_rec_keys, dim3(blocks(n)), dim3(256), 0, s, L->rec, n, cv, key, prio, ord);
    if ((rc = iota_u32(perm, n, s))) return fail(rc);
    // LSD: node index, priority, key -> sorted by (key, priority, node)
    hipLaunchKernelGGL(k_gather_by<uint32_t>, dim3(blocks(n)), dim3(256), 0, s, ord, perm, n, tmp32);
    if ((rc = radix_sort_u32(tmp32, perm, n, 32, s))) return fail(rc);
    hipLaunchKernelGGL(k_gather_by<uint64_t>, dim3(blocks(n)), dim3(256), 0, s, prio, perm, n, tmp64);
    if ((rc = radix_sort_u64(tmp64, perm, n, 64, s))) return fail(rc);
    hipLaunchKernelGGL(k_gather_by<uint64_t>, dim3(blocks(n)), dim3(256), 0, s, key, perm, n, tmp64);
    if ((rc = radix_sort_u64(tmp64, perm, n, 64, s))) return fail(rc);
    hipLaunchKernelGGL(k_rec_groups, dim3(blocks(n)), dim3(256), 0, s, key, perm, n, first);
    hipLaunchKernelGGL(k_rec_keepflags, dim3(blocks(n)), dim3(256), 0, s, first, n, kappa, slot);
    if ((rc = scan_u32(slot, slot, n, slot + n, s))) return fail(rc);
    if ((rc = scan_u32(first, tmp32, n, cnt + 1, s))) return fail(rc);
    uint32_t rows = 0, keys = 0;
    if ((rc = read_u32(slot + n, &rows, s)) || (rc = read_u32(cnt + 1, &keys, s))) return fail(rc);
    out->n_keys = keys;
    if ((int64_t)rows > out->capacity) {
        out->n_rows = rows;
        set_error("cone_collect: %u rows do not fit in capacity %lld", rows, (long long)out->capacity);
        return fail(PCRL_EOVERFLOW);
    }
    RowArgs ra{L->rec, key, perm, first, n, kappa, L->K, cv, cnt, out->capacity, *out};
    hipLaunchKernelGGL(k_rec_write, dim3(blocks(n)), dim3(256), 0, s, ra, slot);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        set_error("cone_collect: kernels failed: %s", hipGetErrorString(hipGetLastError()));
        return fail(PCRL_EHIP);
    }
    out->n_rows = rows;
    T.release();
    return PCRL_OK;
}

}  // namespace pcrl

using namespace pcrl;

extern "C" int ie_build(PcrlScene* scene, const PcrlIeGrid* grid, pcrl_stream_t stream, PcrlIes** out) {
    clear_error();
    if (!scene || !grid || !out) {
        set_error("ie_build: scene, grid and out must be given");
        return PCRL_EINVAL;
    }
    return ie_build_impl(scene, grid, (hipStream_t)stream, out);
}

extern "C" int ie_add_edges(PcrlIes* ies, const float* seg, const float* normals, const uint32_t* label,
                            int64_t n_edges, pcrl_stream_t stream) {
    clear_error();
    if (!ies || n_edges < 0 || n_edges >= ((int64_t)1 << 31) || (n_edges > 0 && (!seg || !normals || !label))) {
        set_error("ie_add_edges: need an IE table, 0 <= n_edges < 2^31 and the three arrays");
        return PCRL_EINVAL;
    }
    return ie_add_edges_impl(ies, seg, normals, label, n_edges, (hipStream_t)stream);
}

extern "C" int ie_info(const PcrlIes* ies, PcrlIeInfo* out) {
    clear_error();
    if (!ies || !out) {
        set_error("ie_info: NULL argument");
        return PCRL_EINVAL;
    }
    out->n_ies = ies->n_ie;
    out->n_edge_ies = ies->n_edges;
    out->n_voxels = ies->n_vox;
    out->n_occupied = ies->n_occ;
    out->device_bytes = ies->bytes;
    return PCRL_OK;
}

extern "C" int ie_table(const PcrlIes* ies, uint64_t* key, int32_t* sub, uint32_t* label, uint32_t* count, float* pos,
                        float* nrm, pcrl_stream_t stream) {
    clear_error();
    if (!ies) {
        set_error("ie_table: NULL IE table");
        return PCRL_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)ies->n_ie;
    if (n == 0) return PCRL_OK;
    hipError_t e = hipSuccess;
    if (key && e == hipSuccess) e = hipMemcpyAsync(key, ies->key, n * 8, hipMemcpyDeviceToDevice, s);
    if (sub && e == hipSuccess) e = hipMemcpyAsync(sub, ies->sub, n * 12, hipMemcpyDeviceToDevice, s);
    if (label && e == hipSuccess) e = hipMemcpyAsync(label, ies->label, n * 4, hipMemcpyDeviceToDevice, s);
    if (count && e == hipSuccess) e = hipMemcpyAsync(count, ies->count, n * 4, hipMemcpyDeviceToDevice, s);
    if (pos && e == hipSuccess) e = hipMemcpy2DAsync(pos, 12, ies->pos, 16, 12, n, hipMemcpyDeviceToDevice, s);
    if (nrm && e == hipSuccess) e = hipMemcpy2DAsync(nrm, 12, ies->nrm, 16, 12, n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) {
        set_error("ie_table: copy failed: %s", hipGetErrorString(e));
        return PCRL_EHIP;
    }
    return PCRL_OK;
}

extern "C" int release_ies(PcrlIes* ies) {
    clear_error();
    if (!ies) return PCRL_OK;
    ies->bufs.release();
    delete ies;
    return PCRL_OK;
}

extern "C" int cone_launch(const PcrlIes* ies, const float* tx, int32_t n_tx, const float* rx, int32_t n_rx,
                           const PcrlConeParams* params, pcrl_stream_t stream, PcrlConeLaunch** out) {
    clear_error();
    if (!ies || !params || !out || !tx || n_tx < 1 || n_tx > 255 || n_rx < 0 || n_rx > 65535 || (n_rx > 0 && !rx) ||
        params->max_interactions < 0 || params->max_interactions > PCRL_MAX_REFLECTIONS ||
        !(params->half_angle <= (float)(M_PI / 4)) || params->flags != 0 || params->max_diffractions < 0) {
        set_error("cone_launch: need IEs, 1 <= n_tx <= 255 TX, 0 <= n_rx <= 65535 RX, 0 <= max_interactions <= %d, "
                  "half_angle <= pi/4 and flags 0", PCRL_MAX_REFLECTIONS);
        return PCRL_EINVAL;
    }
    if (ies->scene->overlay && ies->scene->overlay->n_entries > 0) {
        set_error("cone_launch: the scene has dynamic points (update_points)");
        return PCRL_EINVAL;
    }
    return cone_launch_impl(ies, tx, n_tx, rx, n_rx, params, (hipStream_t)stream, out);
}

extern "C" int cone_stats(const PcrlConeLaunch* launch, PcrlConeStats* out) {
    clear_error();
    if (!launch || !out) {
        set_error("cone_stats: NULL argument");
        return PCRL_EINVAL;
    }
    *out = launch->stats;
    return PCRL_OK;
}

extern "C" int cone_nodes(const PcrlConeLaunch* L, int32_t k, int32_t* ie, int32_t* parent, int32_t* tx,
                          uint64_t* prio, float* length, pcrl_stream_t stream) {
    clear_error();
    if (!L || k < 1 || k > L->K) {
        set_error("cone_nodes: need 1 <= k <= max_interactions");
        return PCRL_EINVAL;
    }
    const Gen& G = L->gens[k];
    const size_t n = (size_t)G.n;
    if (n == 0) return PCRL_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (ie && e == hipSuccess) e = hipMemcpyAsync(ie, G.ie, n * 4, hipMemcpyDeviceToDevice, s);
    if (parent && e == hipSuccess) e = hipMemcpyAsync(parent, G.parent, n * 4, hipMemcpyDeviceToDevice, s);
    if (tx && e == hipSuccess) e = hipMemcpyAsync(tx, G.tx, n * 4, hipMemcpyDeviceToDevice, s);
    if (prio && e == hipSuccess) e = hipMemcpyAsync(prio, G.prio, n * 8, hipMemcpyDeviceToDevice, s);
    if (length && e == hipSuccess)
        e = hipMemcpy2DAsync(length, 4, (const char*)G.apex + 12, 16, 4, n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) {
        set_error("cone_nodes: copy failed: %s", hipGetErrorString(e));
        return PCRL_EHIP;
    }
    return PCRL_OK;
}

extern "C" int cone_collect(PcrlConeLaunch* launch, int32_t kappa, PcrlPaths* out, pcrl_stream_t stream) {
    clear_error();
    if (!launch || !out || kappa < 1 || out->capacity < 0) {
        set_error("cone_collect: need a launch, kappa >= 1 and capacity >= 0");
        return PCRL_EINVAL;
    }
    return cone_collect_impl(launch, kappa, out, (hipStream_t)stream);
}

// Per row of a cone_collect result: the edge of every interaction (-1 for a
// reflection), walking the row's chain from its last node up the generations.
struct RowEdgeArgs {
    const int64_t* ray;
    uint32_t n;
    int32_t K;
    const uint32_t* ie[PCRL_MAX_REFLECTIONS + 1];
    const uint32_t* parent[PCRL_MAX_REFLECTIONS + 1];
    const uint32_t* type;
    const uint32_t* eid;
    int32_t* edge_of;           // [n][K]
};

__global__ void k_row_edges(RowEdgeArgs a) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int64_t r = a.ray[i];
    const int k = (int)(r >> 40);
    uint32_t node = (uint32_t)(r & ((1ll << 40) - 1));
    for (int j = a.K - 1; j >= k; --j) a.edge_of[(size_t)i * a.K + j] = -1;
    for (int j = k; j >= 1; --j) {
        const uint32_t e = a.ie[j][node];
        a.edge_of[(size_t)i * a.K + j - 1] = a.type[e] ? (int32_t)a.eid[e] : -1;
        node = a.parent[j][node];
    }
}

extern "C" int refine_cone_paths(const PcrlConeLaunch* L, const PcrlPaths* paths, const PcrlRefineParams* params,
                                 PcrlRefined* out, pcrl_stream_t stream) {
    clear_error();
    if (!L || !paths || !out || paths->n_rows < 0) {
        set_error("refine_cone_paths: need a launch, paths and outputs");
        return PCRL_EINVAL;
    }
    if (params && (params->edge_of || params->edge_seg || params->edge_normals || params->edge_label ||
                   params->n_edges)) {
        set_error("refine_cone_paths: the launch supplies the edges; leave params->edge_* unset");
        return PCRL_EINVAL;
    }
    const int64_t n = paths->n_rows;
    out->n_kept = 0;
    if (n == 0) return PCRL_OK;
    if (L->n_rx < 1 || !paths->ray || !paths->n_refl) {
        set_error("refine_cone_paths: rows need their ray and n_refl (a cone_collect result of this launch)");
        return PCRL_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const PcrlIes* I = L->ies;
    const int K = L->K;
    // the rows must be this launch's: k = n_refl and a node of generation k
    std::vector<int64_t> h_ray(n);
    std::vector<int32_t> h_n(n);
    PCRL_TRY_HIP(hipMemcpyAsync(h_ray.data(), paths->ray, n * 8, hipMemcpyDeviceToHost, s));
    PCRL_TRY_HIP(hipMemcpyAsync(h_n.data(), paths->n_refl, n * 4, hipMemcpyDeviceToHost, s));
    PCRL_TRY_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i) {
        const int k = (int)(h_ray[i] >> 40);
        const int64_t node = h_ray[i] & ((1ll << 40) - 1);
        const bool ok = h_ray[i] >= 0 && k == h_n[i] && k <= K &&
                        (k == 0 ? node < L->n_tx : (k < (int)L->gens.size() && node < L->gens[k].n));
        if (!ok) {
            set_error("refine_cone_paths: row %lld (ray %lld, n_refl %d) is not a reception of this launch",
                      (long long)i, (long long)h_ray[i], h_n[i]);
            return PCRL_EINVAL;
        }
    }
    DevBufs T;
    T.stream = s;
    auto fail = [&](int rc) { T.release(); return rc; };
    float *tx3 = nullptr, *rx3 = nullptr;
    int32_t* edge_of = nullptr;
    int rc;
    if ((rc = T.alloc(&tx3, (size_t)L->n_tx * 3)) || (rc = T.alloc(&rx3, (size_t)L->n_rx * 3))) return fail(rc);
    hipError_t e = hipMemcpy2DAsync(tx3, 12, L->tx, 16, 12, L->n_tx, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpy2DAsync(rx3, 12, L->rx, 16, 12, L->n_rx, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) {
        set_error("refine_cone_paths: copy failed: %s", hipGetErrorString(e));
        return fail(PCRL_EHIP);
    }
    PcrlRefineParams P{};
    if (params) P = *params;
    if (I->n_lines > 0 && K > 0) {
        if ((rc = T.alloc(&edge_of, (size_t)n * K))) return fail(rc);
        RowEdgeArgs a{};
        a.ray = paths->ray;
        a.n = (uint32_t)n;
        a.K = K;
        for (int j = 1; j < (int)L->gens.size() && j <= PCRL_MAX_REFLECTIONS; ++j) {
            a.ie[j] = L->gens[j].ie;
            a.parent[j] = L->gens[j].parent;
        }
        a.type = I->type;
        a.eid = I->eid;
        a.edge_of = edge_of;
        hipLaunchKernelGGL(k_row_edges, dim3(blocks(n)), dim3(256), 0, s, a);
        if (hipGetLastError() != hipSuccess) {
            set_error("refine_cone_paths: kernel launch failed");
            return fail(PCRL_EHIP);
        }
        P.edge_of = edge_of;
        P.n_edges = (int32_t)I->n_lines;
        P.edge_seg = I->line_seg;
        P.edge_normals = I->line_nrm;
        P.edge_label = I->line_label;
    }
    rc = refine_paths(I->scene, tx3, L->n_tx, rx3, L->n_rx, paths, K, &P, out, stream);
    if (hipStreamSynchronize(s) != hipSuccess && !rc) {
        set_error("refine_cone_paths: HIP error: %s", hipGetErrorString(hipGetLastError()));
        rc = PCRL_EHIP;
    }
    T.release();
    return rc;
}

extern "C" int release_cone(PcrlConeLaunch* launch) {
    clear_error();
    if (!launch) return PCRL_OK;
    launch->bufs.release();
    delete launch;
    return PCRL_OK;
}
