// sdf.hip -- ray intersection with the implicit surface of Eq. 1 (paper,
// Section 2.2.1 "Intersections"): the signed distance
//   f(x) = (x - p(x)) . n(x),
// p and n the weighted averages of the positions and normals of the points
// within h of x (weights (1 - |x - q|^2 / h^2)^4; n normalised), is marched
// along the ray: for every occupied leaf the ray crosses, a line segment one
// leaf diagonal long is centred on the projection onto the ray of the centre
// of the box around the leaf's own points (points whose centre lies in the
// leaf); from its near end the march moves by |f(s_i)| and stops at a sample
// with |f| <= eps, or between two samples of opposite sign (at the zero of
// the linear interpolation), or at the segment's far end, or after max_steps
// evaluations.  Where no point lies within h, f is undefined: the march moves
// by h / 2 and compares no sign across that sample.  The ray's intersection is
// the nearest over the leaves; its normal is n at the final sample.
//
// Lane = ray.  The leaves come from the launcher's hierarchical DDA
// (trace_core.h), walked per lane; the walk stops once the next cell starts
// more than 1.5 leaf diagonals beyond the nearest intersection found (no
// later leaf's segment starts before that).  The neighbours of x are the
// entries of the 27 leaves around x's leaf (h is at most 0.98 leaf edges)
// whose centre lies in that leaf, so each point is counted once.
#include "trace_core.h"

#include <cmath>

namespace pcrl {

constexpr int SDF_BLOCK = 64;  // one wave per block: the lanes finish unevenly, small blocks refill the CUs sooner
constexpr int64_t SDF_ORDER_MIN = 65536;  // rays from which a call sorts them into a coherent order

struct SdfArgs {
    SceneView v;
    SceneView ov;          // v with leaf and cell ranges into the own entries (neighbour lookups)
    const float* o;        // [n][3]
    const float* d;        // [n][3]
    const float* tr;       // [n][2] (t_lo, t_hi), or null for (0, inf)
    const uint32_t* order; // null, or lane -> ray (a coherent order of the rays)
    const uint32_t* oscan; // [n_entries + 1] own entries before each entry of the hierarchy
    const float4* opos;    // own entries (each point once, in the leaf of its centre), leaf order
    const float4* onrm;
    uint32_t n;
    int32_t max_steps;
    float h2;              // h^2
    float hl2;             // (h / leaf edge + 1e-3)^2: leaves farther than this from x hold no neighbour
    float half_h;          // step over an undefined sample
    float eps;
    float half_diam;       // half the segment length (half a leaf diagonal)
    float reach;           // 1.5 leaf diagonals and a rounding margin
    int32_t empty;         // the scene holds no point
    float* t;              // [n]
    float* pt;             // [n][3]
    float* nrm;            // [n][3]
    int32_t* cell;         // [n][3] or null
    unsigned long long* stats;  // null, or [2]: evaluations of f, entries read
};

__device__ __forceinline__ bool in_leaf(const SceneView& v, const float4& P, const int cell[3]) {
    return (int)floorf((P.x - v.org[0]) * v.inv_h) == cell[0] && (int)floorf((P.y - v.org[1]) * v.inv_h) == cell[1] &&
           (int)floorf((P.z - v.org[2]) * v.inv_h) == cell[2];
}

// Accumulate the weighted sums of f(x) over the own entries [e0, e1) that
// lie within h of x.  Four entries' positions are loaded before any is used
// (more loads in flight per lane).
__device__ __forceinline__ void sdf_accumulate(const SdfArgs& a, const float x[3], uint32_t e0, uint32_t e1,
                                               float& sw, float sp[3], float sn[3]) {
    const float h2 = a.h2;
    uint32_t e = e0;
    for (; e < e1; e += 4) {
        float4 P[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) P[k] = a.opos[min(e + k, e1 - 1)];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float ex = P[k].x - x[0], ey = P[k].y - x[1], ez = P[k].z - x[2];
            const float d2 = ex * ex + ey * ey + ez * ez;
            if (e + k >= e1 || !(d2 < h2)) continue;
            const float4 N = a.onrm[e + k];
            float w = 1.0f - d2 / h2;
            w *= w;
            w *= w;
            sw += w;
            sp[0] += w * ex;
            sp[1] += w * ey;
            sp[2] += w * ez;
            sn[0] += w * N.x;
            sn[1] += w * N.y;
            sn[2] += w * N.z;
        }
    }
}

// f(x) of Eq. 1 and the unit normal n(x); false where f is undefined.  The
// offset p(x) - x is accumulated relative to x.  The 27 leaves are looked up
// with the DDA's own cell lookup (the cell table where the scene has one),
// whose descent is cached per parent cell: neighbouring leaves mostly share
// their parent.
template <int NL>
__device__ __forceinline__ bool sdf_eval(const SdfArgs& a, const float x[3], float& f, float n[3], uint32_t& reads) {
    const SceneView& v = a.v;
    int lc[3];
    float fr[3];  // position of x inside its leaf, in leaf edges
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float u = (x[k] - v.org[k]) * v.inv_h;
        lc[k] = (int)floorf(u);
        fr[k] = u - (float)lc[k];
    }
    float sw = 0.f, sp[3] = {0.f, 0.f, 0.f}, sn[3] = {0.f, 0.f, 0.f};
    Seg N;
    N.cq[0] = N.cq[1] = N.cq[2] = -1;
    N.cres = 0;
    N.cskip0 = 1;
    N.cbox = NO_BOX;
    N.cnode = 0;
    N.oct_shift = 0;
    // one rolled loop over the 27 leaves (unrolled, the lookups would multiply the registers)
#pragma unroll 1
    for (int q = 0; q < 27; ++q) {
        const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = q / 9 - 1;
        // distance (in leaf edges) from x to the neighbour leaf: skip leaves beyond h
        const float gx = dx < 0 ? fr[0] : (dx > 0 ? 1.f - fr[0] : 0.f);
        const float gy = dy < 0 ? fr[1] : (dy > 0 ? 1.f - fr[1] : 0.f);
        const float gz = dz < 0 ? fr[2] : (dz > 0 ? 1.f - fr[2] : 0.f);
        if (gx * gx + gy * gy + gz * gz >= a.hl2) continue;
        N.c[0] = lc[0] + dx;
        N.c[1] = lc[1] + dy;
        N.c[2] = lc[2] + dz;
        if (N.c[0] < 0 || N.c[1] < 0 || N.c[2] < 0 || N.c[0] >= v.dim[0] || N.c[1] >= v.dim[1] ||
            N.c[2] >= v.dim[2])
            continue;
        DdaCell k;
        dda_cell_reset(k);
        dda_locate<false, NL>(a.ov, N, k, nullptr);
        if (k.lvl != NL || k.range.y == 0u) continue;
        reads += k.range.y;
        sdf_accumulate(a, x, k.range.x, k.range.x + k.range.y, sw, sp, sn);
    }
    const float ln = sqrtf(sn[0] * sn[0] + sn[1] * sn[1] + sn[2] * sn[2]);
    if (!(sw > 0.f) || !(ln > 0.f)) return false;
    const float inv = 1.0f / ln;
    n[0] = sn[0] * inv;
    n[1] = sn[1] * inv;
    n[2] = sn[2] * inv;
    f = -(sp[0] * n[0] + sp[1] * n[1] + sp[2] * n[2]) / sw;
    return true;
}

// Centre of the box around the own entries [e0, e1) of a leaf; false when
// there is none.
__device__ __forceinline__ bool own_box_centre(const SdfArgs& a, uint32_t e0, uint32_t e1, float c[3]) {
    float lo0 = INFINITY, lo1 = INFINITY, lo2 = INFINITY, hi0 = -INFINITY, hi1 = -INFINITY, hi2 = -INFINITY;
    for (uint32_t e = e0; e < e1; ++e) {
        const float4 P = a.opos[e];
        lo0 = fminf(lo0, P.x);
        lo1 = fminf(lo1, P.y);
        lo2 = fminf(lo2, P.z);
        hi0 = fmaxf(hi0, P.x);
        hi1 = fmaxf(hi1, P.y);
        hi2 = fmaxf(hi2, P.z);
    }
    if (!(e0 < e1)) return false;
    c[0] = 0.5f * (lo0 + hi0);
    c[1] = 0.5f * (lo1 + hi1);
    c[2] = 0.5f * (lo2 + hi2);
    return true;
}

// 1 for each entry of the hierarchy listed in the leaf that holds its point's
// centre (the cell taken in FP32 as everywhere else), else 0.
template <int NL>
__global__ void k_own_flags(SceneView v, uint32_t m, uint32_t* flag) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const float4 P = v.spos[e];
    Seg N;
    N.c[0] = (int)floorf((P.x - v.org[0]) * v.inv_h);
    N.c[1] = (int)floorf((P.y - v.org[1]) * v.inv_h);
    N.c[2] = (int)floorf((P.z - v.org[2]) * v.inv_h);
    uint32_t own = 0u;
    if (N.c[0] >= 0 && N.c[1] >= 0 && N.c[2] >= 0 && N.c[0] < v.dim[0] && N.c[1] < v.dim[1] && N.c[2] < v.dim[2]) {
        N.cq[0] = N.cq[1] = N.cq[2] = -1;
        N.cres = 0;
        N.cskip0 = 1;
    N.cbox = NO_BOX;
        N.cnode = 0;
        N.oct_shift = 0;
        DdaCell k;
        dda_cell_reset(k);
        dda_locate<false, NL>(v, N, k, nullptr);
        own = (k.lvl == NL && k.range.x <= e && e - k.range.x < k.range.y) ? 1u : 0u;
    }
    flag[e] = own;
}

// Copy the own entries to their compacted slots.
__global__ void k_own_scatter(const float4* spos, const float4* snrm, const uint32_t* scan, uint32_t m,
                              uint32_t cap, float4* opos, float4* onrm) {
    const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    const uint32_t j = scan[e];
    if (scan[e + 1] == j || j >= cap) return;
    opos[j] = spos[e];
    onrm[j] = snrm[e];
}

// 8 bits spread to the even bits of 16.
__device__ __forceinline__ uint32_t spread_bits8(uint32_t x) {
    x &= 0xFFu;
    x = (x | (x << 4)) & 0x0F0Fu;
    x = (x | (x << 2)) & 0x3333u;
    x = (x | (x << 1)) & 0x5555u;
    return x;
}

// Coherence key of a ray: Morton code of its origin on a 16^3 grid over the
// scene (12 bits) above the Morton code of its direction's cell on a 256 x 256
// octahedral grid (16 bits).  Sorting by it puts rays that start close
// together in close directions into the same waves, which then march the same
// leaves (shared cache lines, similar step counts).  The octahedral map only
// needs the direction's signs and ratios, so d need not be normalised.
__device__ __forceinline__ uint64_t coherence_key(const float o[3], const float d[3], float3 lo, float3 scale) {
    float u = 0.f, w = 0.f;
    octahedral(d[0], d[1], d[2], u, w);
    const uint32_t dk = spread_bits8(cell_of(u, 256)) | (spread_bits8(cell_of(w, 256)) << 1);
    const uint32_t cx = (uint32_t)fminf(fmaxf((o[0] - lo.x) * scale.x, 0.f), 15.f);
    const uint32_t cy = (uint32_t)fminf(fmaxf((o[1] - lo.y) * scale.y, 0.f), 15.f);
    const uint32_t cz = (uint32_t)fminf(fmaxf((o[2] - lo.z) * scale.z, 0.f), 15.f);
    const uint32_t m = spread_bits4x3(cx) | (spread_bits4x3(cy) << 1) | (spread_bits4x3(cz) << 2);
    return ((uint64_t)m << 16) | dk;
}

__global__ void k_sdf_keys(const float* o, const float* d, uint32_t n, float3 lo, float3 scale, uint64_t* keys,
                           uint32_t* idx) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const size_t j3 = 3 * (size_t)j;
    const float oj[3] = {o[j3], o[j3 + 1], o[j3 + 2]};
    const float dj[3] = {d[j3], d[j3 + 1], d[j3 + 2]};
    keys[j] = coherence_key(oj, dj, lo, scale);
    idx[j] = j;
}

template <int NL>
__device__ __forceinline__ void sdf_first_hit(const SdfArgs& a, const float o[3], const float d[3], float t_lo,
                                              float t_hi, float& best, float bn[3], int bc[3], uint32_t& evals,
                                              uint32_t& reads) {
    const SceneView& v = a.v;
    best = INFINITY;
    bn[0] = bn[1] = bn[2] = 0.f;
    bc[0] = bc[1] = bc[2] = -1;
    Seg S;
    bool walking = !a.empty && t_lo <= t_hi && seg_begin(v, o, d, S);
    float t_in = 0.f;  // where the ray enters the current cell
    if (walking) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            float tf = -INFINITY;
            if (d[ax] > 0.f) tf = ((float)S.c[ax] * v.h + v.org[ax] - o[ax]) * S.inv[ax];
            else if (d[ax] < 0.f) tf = ((float)(S.c[ax] + 1) * v.h + v.org[ax] - o[ax]) * S.inv[ax];
            t_in = fmaxf(t_in, tf);
        }
    }
    // Every leaf whose segment starts at or before t_lo marches from t_lo: the
    // same samples, cut at different far ends.  One shared march serves them
    // all: a leaf whose far end it has already passed, or after it found an
    // intersection or stopped (step limit, nothing nearer possible), adds
    // nothing; a leaf reaching further resumes it.  Exact: the nearest over
    // these leaves is unchanged.
    float c_t = t_lo, c_fp = 0.f, c_tp = 0.f, c_tb = -INFINITY;
    bool c_prev = false, c_done = false;
    int c_s = 0;
    while (walking) {
        DdaCell k;
        dda_cell_reset(k);
        dda_locate<false, NL>(v, S, k, nullptr);
        const bool at_leaf = k.lvl == NL;
        float c[3];
        uint32_t o0 = 0u, o1 = 0u;
        if (at_leaf && t_in <= t_hi) {
            o0 = a.oscan[k.range.x];
            o1 = a.oscan[k.range.x + k.range.y];
        }
        if (at_leaf && t_in <= t_hi && own_box_centre(a, o0, o1, c)) {
            reads += o1 - o0;
            const float tc = (c[0] - o[0]) * d[0] + (c[1] - o[1]) * d[1] + (c[2] - o[2]) * d[2];
            const bool shared = tc - a.half_diam <= t_lo;
            float t = fmaxf(tc - a.half_diam, t_lo);
            const float tb = fminf(tc + a.half_diam, t_hi);
            float fp = 0.f, tp = 0.f;
            bool prev = false;
            int s = 0;
            bool stop = false;  // the march ended by an intersection, the step limit or `best`
            if (shared) {
                if (c_done || tb <= c_tb) s = a.max_steps;  // nothing new from this leaf
                t = c_t;
                fp = c_fp;
                tp = c_tp;
                prev = c_prev;
                if (s < a.max_steps) s = c_s;
            }
            for (; s < a.max_steps && t <= tb; ++s) {
                // every later result of this leaf lies at or beyond t
                if (t >= best && !(prev && tp < best)) {
                    stop = true;
                    break;
                }
                const float x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
                float f, n[3];
                ++evals;
                if (!sdf_eval<NL>(a, x, f, n, reads)) {
                    prev = false;
                    t += a.half_h;
                    continue;
                }
                float th = t;
                bool found = fabsf(f) <= a.eps;
                if (!found && prev && ((f < 0.f) != (fp < 0.f))) {
                    th = tp + (t - tp) * fp / (fp - f);
                    found = true;
                }
                if (found) {
                    if (th < best) {
                        best = th;
                        bn[0] = n[0];
                        bn[1] = n[1];
                        bn[2] = n[2];
                        bc[0] = S.c[0];
                        bc[1] = S.c[1];
                        bc[2] = S.c[2];
                    }
                    stop = true;
                    break;
                }
                prev = true;
                fp = f;
                tp = t;
                t += fabsf(f);
            }
            if (shared && !c_done && tb > c_tb) {
                c_t = t;
                c_fp = fp;
                c_tp = tp;
                c_prev = prev;
                c_s = s;
                c_tb = tb;
                c_done = stop || s >= a.max_steps;
            }
        }
        float te;
        dda_advance<NL>(v, walking, o, d, S, k, at_leaf, fminf(best + a.reach, t_hi), te);
        t_in = te;
    }
}

template <int NL>
__global__ __launch_bounds__(SDF_BLOCK) void k_sdf(SdfArgs a) {
    const uint32_t lane_ray = blockIdx.x * SDF_BLOCK + threadIdx.x;
    if (lane_ray >= a.n) return;
    const uint32_t i = a.order ? a.order[lane_ray] : lane_ray;
    const size_t i3 = 3 * (size_t)i, i2 = 2 * (size_t)i;  // n may exceed 2^32 / 3
    const float o[3] = {a.o[i3], a.o[i3 + 1], a.o[i3 + 2]};
    float d[3] = {a.d[i3], a.d[i3 + 1], a.d[i3 + 2]};
    const float t_lo = a.tr ? a.tr[i2] : 0.f;
    const float t_hi = a.tr ? a.tr[i2 + 1] : INFINITY;
    const float len = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const bool ok = len > 0.f && isfinite(len) && isfinite(o[0]) && isfinite(o[1]) && isfinite(o[2]);
    float best = INFINITY, bn[3] = {0.f, 0.f, 0.f};
    int bc[3] = {-1, -1, -1};
    uint32_t evals = 0, reads = 0;
    if (ok) {
        const float il = 1.0f / len;
        d[0] *= il;
        d[1] *= il;
        d[2] *= il;
        sdf_first_hit<NL>(a, o, d, t_lo, t_hi, best, bn, bc, evals, reads);
    }
    a.t[i] = best;
    const bool hit = bc[0] >= 0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        a.pt[i3 + ax] = hit ? o[ax] + best * d[ax] : NAN;
        a.nrm[i3 + ax] = bn[ax];
        if (a.cell) a.cell[i3 + ax] = bc[ax];
    }
    if (a.stats) {
        atomicAdd(&a.stats[0], (unsigned long long)evals);
        atomicAdd(&a.stats[1], (unsigned long long)reads);
    }
}

// Id and label of the point nearest to x among those within h (smallest
// distance, then smallest id); false if none.
template <int NL>
__device__ __forceinline__ bool nearest_own(const SdfArgs& a, const float x[3], uint32_t& id, uint32_t& label) {
    const SceneView& v = a.v;
    int lc[3];
    float fr[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float u = (x[k] - v.org[k]) * v.inv_h;
        lc[k] = (int)floorf(u);
        fr[k] = u - (float)lc[k];
    }
    float bd = a.h2;
    bool found = false;
    Seg N;
    N.cq[0] = N.cq[1] = N.cq[2] = -1;
    N.cres = 0;
    N.cskip0 = 1;
    N.cbox = NO_BOX;
    N.cnode = 0;
    N.oct_shift = 0;
#pragma unroll 1
    for (int q = 0; q < 27; ++q) {
        const int dx = q % 3 - 1, dy = (q / 3) % 3 - 1, dz = q / 9 - 1;
        const float gx = dx < 0 ? fr[0] : (dx > 0 ? 1.f - fr[0] : 0.f);
        const float gy = dy < 0 ? fr[1] : (dy > 0 ? 1.f - fr[1] : 0.f);
        const float gz = dz < 0 ? fr[2] : (dz > 0 ? 1.f - fr[2] : 0.f);
        if (gx * gx + gy * gy + gz * gz >= a.hl2) continue;
        N.c[0] = lc[0] + dx;
        N.c[1] = lc[1] + dy;
        N.c[2] = lc[2] + dz;
        if (N.c[0] < 0 || N.c[1] < 0 || N.c[2] < 0 || N.c[0] >= v.dim[0] || N.c[1] >= v.dim[1] ||
            N.c[2] >= v.dim[2])
            continue;
        DdaCell k;
        dda_cell_reset(k);
        dda_locate<false, NL>(a.ov, N, k, nullptr);
        if (k.lvl != NL || k.range.y == 0u) continue;
        const uint32_t e1 = k.range.x + k.range.y;
        for (uint32_t e = k.range.x; e < e1; ++e) {
            const float4 P = a.opos[e];
            const float ex = P.x - x[0], ey = P.y - x[1], ez = P.z - x[2];
            const float d2 = ex * ex + ey * ey + ez * ez;
            const uint32_t pid = __float_as_uint(P.w);
            if (d2 < bd || (d2 == bd && found && pid < id)) {
                bd = d2;
                id = pid;
                label = __float_as_uint(a.onrm[e].w);
                found = true;
            }
        }
    }
    return found;
}

// A launch whose intersections are those of the implicit surface (launch_rays
// with PCRL_LAUNCH_SDF): one lane per ray runs all its segments.
struct SdfLaunchArgs {
    SdfArgs s;
    const float* tx;
    const float* rx;
    const float* dirs;
    const uint32_t* order;  // null, or lane -> global ray id
    int32_t n_rx;
    int32_t K;
    uint32_t n_rays;
    uint32_t n_total;
    float sig_c;            // rho(u) = sig_c * u
    float4* hist;
    uint4* rec;
    uint32_t rec_cap;
    uint32_t* counters;
    int32_t* hit_id;
    float* hit_t;
};

// Add x (the same on every lane) to *p for each lane active here, with one
// atomic per wave.
__device__ __forceinline__ void wave_add(uint32_t* p, uint32_t x) {
    const uint64_t m = __ballot(1);
    const int leader = __ffsll((long long)m) - 1;
    if ((int)lane_id() == leader) atomicAdd(p, (uint32_t)__popcll(m) * x);
}

// Every segment of a ray, as the launcher's bounce kernels do with surfels:
// the segment from o along d ends at the implicit surface's first
// intersection (from t_lo: 0 from the TX, after a reflection 4 eps / |d.n|
// so that the march starts outside the |f| <= eps band it left); the RX
// spheres are tested on [0, t]; at the intersection the ray reflects about
// n(x) and records the label of the nearest point.
template <int NL>
__global__ __launch_bounds__(SDF_BLOCK) void k_sdf_launch(SdfLaunchArgs A) {
    const uint32_t lane_ray = blockIdx.x * SDF_BLOCK + threadIdx.x;
    if (lane_ray >= A.n_total) return;
    const uint32_t g = A.order ? A.order[lane_ray] : lane_ray;
    const SdfArgs& a = A.s;
    const uint32_t ti = g / A.n_rays, j = g - ti * A.n_rays;
    float o[3] = {A.tx[3 * ti], A.tx[3 * ti + 1], A.tx[3 * ti + 2]};
    float d[3] = {A.dirs[3 * (size_t)j], A.dirs[3 * (size_t)j + 1], A.dirs[3 * (size_t)j + 2]};
    {
        const float il = 1.0f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        d[0] *= il;
        d[1] *= il;
        d[2] *= il;
    }
    float L = 0.f, t_lo = 0.f;
    uint32_t* rec_counter = &A.counters[PCRL_CNT_REC(A.K)];
    for (int b = 0; b <= A.K; ++b) {
        wave_add(&A.counters[b], 1u);
        float t, n[3];
        int bc[3];
        uint32_t ev = 0, rd = 0;
        sdf_first_hit<NL>(a, o, d, t_lo, INFINITY, t, n, bc, ev, rd);
        bool hit = bc[0] >= 0;
        float q[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
        uint32_t pid = 0, lab = 0;
        if (hit) hit = nearest_own<NL>(a, q, pid, lab);
        if (!hit) t = INFINITY;
        if (A.hit_id) {
            const size_t idx = (size_t)g * (A.K + 1) + b;
            A.hit_id[idx] = hit ? (int32_t)pid : -1;
            A.hit_t[idx] = hit ? t : NAN;
        }
        for (int r = 0; r < A.n_rx; ++r) {
            const float vx = A.rx[3 * r] - o[0], vy = A.rx[3 * r + 1] - o[1], vz = A.rx[3 * r + 2] - o[2];
            const float sp = vx * d[0] + vy * d[1] + vz * d[2];
            if (!(sp > 0.f && sp <= t)) continue;
            const float cx = vx - sp * d[0], cy = vy - sp * d[1], cz = vz - sp * d[2];
            const float rho = A.sig_c * (L + sp);
            if (!(cx * cx + cy * cy + cz * cz <= rho * rho)) continue;
            const uint32_t slot = atomicAdd(rec_counter, 1u);
            if (slot < A.rec_cap) {
                const float lp = L + sqrtf(vx * vx + vy * vy + vz * vz);
                A.rec[slot] = make_uint4(g, (uint32_t)r | ((uint32_t)b << 16), __float_as_uint(lp),
                                         __float_as_uint(L + sp));
            }
        }
        if (!hit || b >= A.K) break;
        A.hist[(size_t)b * A.n_total + g] = make_float4(q[0], q[1], q[2], __uint_as_float(lab));
        L += t;
        const float dn = d[0] * n[0] + d[1] * n[1] + d[2] * n[2];
        const float ex = d[0] - 2.f * dn * n[0], ey = d[1] - 2.f * dn * n[1], ez = d[2] - 2.f * dn * n[2];
        const float inv = 1.0f / sqrtf(ex * ex + ey * ey + ez * ez);
        d[0] = ex * inv;
        d[1] = ey * inv;
        d[2] = ez * inv;
        o[0] = q[0];
        o[1] = q[1];
        o[2] = q[2];
        t_lo = 4.f * a.eps / fmaxf(fabsf(dn), 0.05f);
    }
}

// Coherence key of global ray g of a launch (its TX and launch direction).
__global__ void k_sdf_launch_keys(const float* tx, const float* dirs, uint32_t n_rays, uint32_t n_total, float3 lo,
                                  float3 scale, uint64_t* keys, uint32_t* idx) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_total) return;
    const uint32_t ti = g / n_rays, j = g - ti * n_rays;
    const float o[3] = {tx[3 * ti], tx[3 * ti + 1], tx[3 * ti + 2]};
    const float d[3] = {dirs[3 * (size_t)j], dirs[3 * (size_t)j + 1], dirs[3 * (size_t)j + 2]};
    keys[g] = coherence_key(o, d, lo, scale);
    idx[g] = g;
}

template <int NL>
static void launch_sdf_nl(const SdfArgs& a, hipStream_t s) {
    const unsigned grid = (a.n + SDF_BLOCK - 1) / SDF_BLOCK;
    hipLaunchKernelGGL((k_sdf<NL>), dim3(grid), dim3(SDF_BLOCK), 0, s, a);
}

// Entry ranges (first, count) of a leaf table or a dense cell table turned
// into ranges of own entries; an entry with count 0 (an empty cell's skip
// radius) is kept as it is.
__global__ void k_own_ranges(const uint2* in, uint32_t n, const uint32_t* scan, uint2* out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint2 r = in[i];
    out[i] = r.y ? make_uint2(scan[r.x], scan[r.x + r.y] - scan[r.x]) : r;
}

// The integer block of the own-point index: the scan [n_entries + 1], then
// (8-byte aligned) the own range of every leaf and, where the scene has a
// dense cell table, that table with own ranges.
struct OwnLayout {
    size_t leaf_off, n_leaves, cells_off, n_cells, bytes;
};

static OwnLayout own_layout(const PcrlScene* S) {
    const SceneView& v = S->view;
    OwnLayout L{};
    L.leaf_off = ((size_t)(S->info.n_entries + 1) * sizeof(uint32_t) + 7) / 8 * 8;
    L.n_leaves = v.nn[v.nlev - 1];
    L.cells_off = L.leaf_off + L.n_leaves * sizeof(uint2);
    if (v.cells && v.nlev >= 2) {
        const size_t r = (size_t)v.ratio[v.nlev - 2];
        L.n_cells = (size_t)v.nn[v.nlev - 2] * r * r * r;
    }
    L.bytes = L.cells_off + L.n_cells * sizeof(uint2);
    return L;
}

// The scene's view with its leaf and cell ranges pointing into the own entries.
static SceneView own_view(const PcrlScene* S) {
    const OwnLayout L = own_layout(S);
    SceneView ov = S->view;
    char* base = (char*)S->own_scan;
    ov.leaf = (const uint2*)(base + L.leaf_off);
    if (L.n_cells) ov.cells = (const uint2*)(base + L.cells_off);
    return ov;
}

template <int NL>
static void launch_own_flags(const SceneView& v, uint32_t m, uint32_t* flag, hipStream_t s) {
    hipLaunchKernelGGL((k_own_flags<NL>), dim3((unsigned)(((uint64_t)m + 255) / 256)), dim3(256), 0, s, v, m, flag);
}

// The scene's own-point index, built on the first call (under the scene's
// lock) and kept with the scene.  The build waits for its stream, so calls on
// any stream find the index complete.
static int own_index(PcrlScene* S, hipStream_t s) {
    std::lock_guard<std::mutex> lock(S->own_mu);
    if (S->own_scan) return PCRL_OK;
    const int64_t m = S->info.n_entries, np = S->info.n_points;
    const OwnLayout lay = own_layout(S);
    uint32_t* scan = nullptr;
    float4 *pos = nullptr, *nrm = nullptr;
    int rc = dalloc((void**)&scan, lay.bytes, s);
    if (!rc) rc = dalloc((void**)&pos, (size_t)(np > 0 ? np : 1) * sizeof(float4), s);
    if (!rc) rc = dalloc((void**)&nrm, (size_t)(np > 0 ? np : 1) * sizeof(float4), s);
    if (!rc) {
        switch (S->view.nlev) {
        case 1: launch_own_flags<1>(S->view, (uint32_t)m, scan, s); break;
        case 2: launch_own_flags<2>(S->view, (uint32_t)m, scan, s); break;
        case 3: launch_own_flags<3>(S->view, (uint32_t)m, scan, s); break;
        default: launch_own_flags<4>(S->view, (uint32_t)m, scan, s); break;
        }
        rc = hipGetLastError() == hipSuccess ? scan_u32(scan, scan, m, scan + m, s) : PCRL_EHIP;
    }
    if (!rc) {
        hipLaunchKernelGGL(k_own_scatter, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, S->view.spos,
                           S->view.snrm, scan, (uint32_t)m, (uint32_t)np, pos, nrm);
        char* base = (char*)scan;
        hipLaunchKernelGGL(k_own_ranges, dim3((unsigned)((lay.n_leaves + 255) / 256)), dim3(256), 0, s,
                           S->view.leaf, (uint32_t)lay.n_leaves, scan, (uint2*)(base + lay.leaf_off));
        if (lay.n_cells)
            hipLaunchKernelGGL(k_own_ranges, dim3((unsigned)((lay.n_cells + 255) / 256)), dim3(256), 0, s,
                               S->view.cells, (uint32_t)lay.n_cells, scan, (uint2*)(base + lay.cells_off));
        rc = hipGetLastError() == hipSuccess && hipStreamSynchronize(s) == hipSuccess ? PCRL_OK : PCRL_EHIP;
    }
    if (rc) {
        dfree(scan, s);
        dfree(pos, s);
        dfree(nrm, s);
        if (rc == PCRL_EHIP) set_error("sdf_intersect: building the own-point index failed");
        return rc;
    }
    S->bufs.ptrs.push_back(scan);
    S->bufs.ptrs.push_back(pos);
    S->bufs.ptrs.push_back(nrm);
    S->own_scan = scan;
    S->own_pos = pos;
    S->own_nrm = nrm;
    return PCRL_OK;
}

int scene_own_index(PcrlScene* S, hipStream_t s) { return own_index(S, s); }

// Defaults of the implicit surface for a scene (h, eps, max_steps as
// sdf_intersect's when its parameters are not given).
static void sdf_defaults(const PcrlScene* scene, SdfArgs& a) {
    const float leaf = scene->view.h;
    const float h = 0.95f * leaf;
    a.v = scene->view;
    a.max_steps = 64;
    a.h2 = h * h;
    a.hl2 = (h / leaf + 1e-3f) * (h / leaf + 1e-3f);
    a.half_h = 0.5f * h;
    a.eps = 1e-3f * leaf;
    const float diag = sqrtf(3.0f) * leaf;
    a.half_diam = 0.5f * diag;
    a.reach = 1.5f * diag * (1.0f + 1e-5f) + 1e-3f * leaf;
    a.empty = scene->info.n_points == 0;
}

template <int NL>
static void launch_sdf_launch_nl(const SdfLaunchArgs& A, hipStream_t s) {
    const unsigned grid = (A.n_total + SDF_BLOCK - 1) / SDF_BLOCK;
    hipLaunchKernelGGL((k_sdf_launch<NL>), dim3(grid), dim3(SDF_BLOCK), 0, s, A);
}

int sdf_launch_run(PcrlLaunch* L, const TraceArgs& t) {
    const PcrlScene* scene = L->scene;
    hipStream_t s = L->stream;
    if (L->stats || t.has_ov) {
        set_error("launch_rays: PCRL_LAUNCH_SDF takes no PCRL_LAUNCH_STATS and no scene with dynamic points");
        return PCRL_EINVAL;
    }
    SdfLaunchArgs A{};
    sdf_defaults(scene, A.s);
    if (!A.s.empty) {
        PCRL_TRY(own_index(const_cast<PcrlScene*>(scene), s));
        A.s.oscan = scene->own_scan;
        A.s.opos = scene->own_pos;
        A.s.onrm = scene->own_nrm;
        A.s.ov = own_view(scene);
    }
    A.tx = t.tx;
    A.rx = t.rx;
    A.dirs = t.dirs;
    A.n_rx = t.n_rx;
    A.K = t.K;
    A.n_rays = t.n_rays;
    A.n_total = t.n_total;
    A.sig_c = t.sig_c;
    A.hist = t.hist;
    A.rec = t.rec;
    A.rec_cap = t.rec_cap;
    A.counters = t.counters;
    A.hit_id = t.hit_id;
    A.hit_t = t.hit_t;
    if ((L->flags & PCRL_LAUNCH_COHERENT) && !A.s.empty) {
        uint64_t* keys = nullptr;
        uint32_t* idx = nullptr;
        int rc = L->bufs.alloc(&keys, (size_t)A.n_total);
        if (!rc) rc = L->bufs.alloc(&idx, (size_t)A.n_total);
        if (rc) return rc;
        const SceneView& v = scene->view;
        const float3 lo = make_float3(v.org[0], v.org[1], v.org[2]);
        const float3 sc = make_float3(16.f / (v.hi[0] - v.org[0]), 16.f / (v.hi[1] - v.org[1]),
                                      16.f / (v.hi[2] - v.org[2]));
        hipLaunchKernelGGL(k_sdf_launch_keys, dim3((A.n_total + 255) / 256), dim3(256), 0, s, A.tx, A.dirs, A.n_rays,
                           A.n_total, lo, sc, keys, idx);
        PCRL_TRY_HIP(hipGetLastError());
        PCRL_TRY(radix_sort_u64_bits(keys, idx, (int64_t)A.n_total, 0, 28, s));
        A.order = idx;
    }
    const bool timing = !L->events.empty();
    if (timing) PCRL_TRY_HIP(hipEventRecord(L->events[0], s));
    switch (scene->view.nlev) {
    case 1: launch_sdf_launch_nl<1>(A, s); break;
    case 2: launch_sdf_launch_nl<2>(A, s); break;
    case 3: launch_sdf_launch_nl<3>(A, s); break;
    default: launch_sdf_launch_nl<4>(A, s); break;
    }
    PCRL_TRY_HIP(hipGetLastError());
    if (timing) {
        // one kernel runs every segment: its time is reported as bounce 0's
        for (size_t e = 1; e < L->events.size(); ++e) PCRL_TRY_HIP(hipEventRecord(L->events[e], s));
    }
    return PCRL_OK;
}

}  // namespace pcrl

using namespace pcrl;

extern "C" int sdf_intersect(const PcrlScene* scene, const float* o, const float* d, const float* t_range,
                             int64_t n_rays, const PcrlSdfParams* params, float* t, float* point, float* normal,
                             int32_t* leaf_cell, pcrl_stream_t stream) {
    clear_error();
    if (!scene || n_rays < 0 || n_rays >= ((int64_t)1 << 31)) {
        set_error("sdf_intersect: invalid scene or ray count (0 <= n_rays < 2^31)");
        return PCRL_EINVAL;
    }
    if (n_rays > 0 && (!o || !d || !t || !point || !normal)) {
        set_error("sdf_intersect: a ray or output array is NULL");
        return PCRL_EINVAL;
    }
    if (scene->overlay && scene->overlay->n_entries > 0) {
        set_error("sdf_intersect: the scene has dynamic points (update_points); the implicit surface is defined "
                  "over the static points only");
        return PCRL_EINVAL;
    }
    PcrlSdfParams P{};
    if (params) P = *params;
    const float leaf = scene->view.h;
    const float h = P.h > 0.f ? P.h : 0.95f * leaf;
    const float eps = P.eps > 0.f ? P.eps : 1e-3f * leaf;
    const int32_t max_steps = P.max_steps > 0 ? P.max_steps : 64;
    if (!(h <= 0.98f * leaf) || !std::isfinite(eps) || max_steps > (1 << 20) || P.flags != 0) {
        set_error("sdf_intersect: need 0 < h <= 0.98 leaf edges (h %g, leaf %g), a finite eps, max_steps <= 2^20 "
                  "and flags 0", (double)h, (double)leaf);
        return PCRL_EINVAL;
    }
    if (n_rays == 0) return PCRL_OK;
    SdfArgs a{};
    a.v = scene->view;
    a.o = o;
    a.d = d;
    a.tr = t_range;
    a.n = (uint32_t)n_rays;
    a.max_steps = max_steps;
    a.h2 = h * h;
    a.hl2 = (h / leaf + 1e-3f) * (h / leaf + 1e-3f);
    a.half_h = 0.5f * h;
    a.eps = eps;
    const float diag = sqrtf(3.0f) * leaf;
    a.half_diam = 0.5f * diag;
    a.reach = 1.5f * diag * (1.0f + 1e-5f) + 1e-3f * leaf;
    a.empty = scene->info.n_points == 0;
    a.t = t;
    a.pt = point;
    a.nrm = normal;
    a.cell = leaf_cell;
    a.stats = (unsigned long long*)P.stats;
    hipStream_t s = (hipStream_t)stream;
    if (!a.empty) {
        // the index is a cache of the scene's data: building it does not change the scene
        const int rc = own_index(const_cast<PcrlScene*>(scene), s);
        if (rc) return rc;
        a.oscan = scene->own_scan;
        a.opos = scene->own_pos;
        a.onrm = scene->own_nrm;
        a.ov = own_view(scene);
    }
    DevBufs T;
    T.stream = s;
    // large batches run in a coherent order (the outputs keep the callers')
    if (n_rays >= SDF_ORDER_MIN && !a.empty) {
        uint64_t* keys = nullptr;
        uint32_t* idx = nullptr;
        int rc = T.alloc(&keys, (size_t)n_rays);
        if (!rc) rc = T.alloc(&idx, (size_t)n_rays);
        if (rc) {
            T.release();
            return rc;
        }
        const SceneView& v = scene->view;
        const float3 lo = make_float3(v.org[0], v.org[1], v.org[2]);
        const float3 sc = make_float3(16.f / (v.hi[0] - v.org[0]), 16.f / (v.hi[1] - v.org[1]),
                                      16.f / (v.hi[2] - v.org[2]));
        hipLaunchKernelGGL(k_sdf_keys, dim3((unsigned)((n_rays + 255) / 256)), dim3(256), 0, s, o, d,
                           (uint32_t)n_rays, lo, sc, keys, idx);
        rc = hipGetLastError() == hipSuccess ? radix_sort_u64_bits(keys, idx, n_rays, 0, 28, s) : PCRL_EHIP;
        if (rc) {
            T.release();
            set_error("sdf_intersect: ordering the rays failed");
            return rc;
        }
        a.order = idx;
    }
    switch (scene->view.nlev) {
    case 1: launch_sdf_nl<1>(a, s); break;
    case 2: launch_sdf_nl<2>(a, s); break;
    case 3: launch_sdf_nl<3>(a, s); break;
    default: launch_sdf_nl<4>(a, s); break;
    }
    const bool ok = hipGetLastError() == hipSuccess;
    T.release();  // stream-ordered: the buffers stay valid for the kernel
    if (!ok) {
        set_error("sdf_intersect: kernel launch failed");
        return PCRL_EHIP;
    }
    return PCRL_OK;
}
