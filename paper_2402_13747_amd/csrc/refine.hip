// refine.hip -- path refinement (paper, Section 2.3, Eq. 2) and the dedup of
// refined paths (Section 2.3, last paragraph).
//
// A coarse path TX -> q_1 .. q_N -> RX becomes an exact path by gradient
// descent on its length f = sum_k |I_k - I_{k+1}| (Eq. 2).  Every
// interaction point moves in the tangent plane of the surface at its current
// position c_k; the step r_k u_k + s_k v_k of the paper is the tangent-plane
// projection of the step, so no basis (u_k, v_k) is formed.  Per iteration:
//   - the derivative of the local length f_k, G_k = (I_k - I_{k-1})/|.| +
//     (I_k - I_{k+1})/|.|, projected onto the tangent plane: g_k;
//   - converged when |(g_1 .. g_N)| < delta; given up after rho steps;
//   - all points step at once, R_k = c_k - a_k g_k with
//     a_k = eta / (1/|c_k - I_{k-1}| + 1/|c_k - I_{k+1}|) (the paper gives no
//     step size: this one divides by the largest tangent curvature of f_k);
//   - for k = 1..N a ray from the new I_{k-1} towards R_k finds the new c_k
//     and its normal (the hit surfel's) through the voxel hierarchy, exactly
//     as a launched ray; a ray that hits nothing ends the path (invalid).
// With PCRL_REFINE_SMOOTH the normal at c_k is instead the weighted average
// of the normals of the points near c_k (the smooth normal of Eq. 1).
// A diffraction point D_k = a + t_k w stays on its edge (Section 2.3): t_k
// steps along G_k . w with the same a_k, no ray is traced to it, a ray
// leaving it starts r_s along its direction (the surfels of the edge's own
// faces meet the edge), a segment arriving at it is blocked only by a hit
// more than r_s before it, and a step off the edge's segment ends the path.
// The first c_k come from the same tracing towards the coarse points.  A
// converged path is kept if every interaction has both neighbours on one
// side of its surfel and the last segment reaches the RX unblocked.
//
// Lane = path, with few paths per wave (one, unless the paths outnumber the
// GPU's SIMDs): a wave iterates in lockstep until all its paths are done, and
// all 64 lanes share the leaf tests of its rays (traversal and leaf tests are
// the launcher's own, trace_core.h).  The per-path interaction state lives
// in global arrays [k][path] (a dynamically indexed private array would be
// placed in scratch memory).
//
// Dedup of the valid paths of one (TX, RX, number of reflections) group, in
// order of increasing length: a path whose label sequence already occurred
// is dropped (the shortest per sequence is kept); a path whose every
// interaction point lies inside the first Fresnel zone of the corresponding
// point of an already kept path is dropped as well.
#include "trace_core.h"

#include <algorithm>
#include <cmath>
#include <tuple>
#include <vector>

namespace pcrl {

constexpr int REFINE_BLOCK = 64;     // one wave per block: refinement batches are small
constexpr int SWEEP_KEPT_MAX = 2048; // kept paths of one (TX, RX, reflections) group held in LDS

struct RefineArgs {
    TraceArgs t;                // scene views only (v, ov, has_ov)
    const float* tx;            // [n_tx][3]
    const float* rx;            // [n_rx][3]
    const int32_t* p_tx;        // per path: TX index
    const int32_t* p_rx;        // per path: RX index
    const int32_t* p_n;         // per path: reflections N
    const float* p_pts;         // [n][K][3] coarse interaction points
    uint32_t n;
    uint32_t ppw;               // paths per wave (lanes 0..ppw-1 hold one each; the others help the leaf tests)
    int32_t K;
    int32_t max_iters;
    float grad_tol;
    float step;
    float smooth_h2;            // > 0: surface normals averaged over this squared radius
    float4* cpos;               // [K][n] current point, surfel id (bits)
    float4* cnrm;               // [K][n] its surfel's normal, label (bits)
    float4* tgt;                // [K][n] point the next trace aims at
    int32_t* status;
    int32_t* iters;
    float* grad;
    float* length;
    float* out_pts;             // [n][K][3]
    int32_t* out_id;            // [n][K]
    int64_t* out_key;           // [n][K]
    // diffraction edges (p_edge null: reflections only)
    const int32_t* p_edge;      // [n][K]: edge of interaction k, -1 a reflection
    const float4* e_a;          // per edge: end point a, length |b - a| in w
    const float4* e_w;          // per edge: unit direction, label (bits) in w
    const float4* e_n1;         // per edge: outward normals of its two faces
    const float4* e_n2;
    float clear;                // r_s: the clearance at a diffraction point
};

__device__ __forceinline__ int edge_at(const RefineArgs& a, uint32_t p, int k) {
    return a.p_edge ? a.p_edge[(size_t)p * a.K + k] : -1;
}

__device__ __forceinline__ float dist3(const float a[3], const float b[3]) {
    const float x = a[0] - b[0], y = a[1] - b[1], z = a[2] - b[2];
    return sqrtf(x * x + y * y + z * z);
}

// The largest value of x over the wave (x >= 0).
__device__ __forceinline__ int wave_max(int x) {
    return __builtin_amdgcn_readlane(wave_scan_max_dpp(x), 63);
}

// Trace every lane's ray from o towards `target`, starting `skip` along its
// direction (lanes with `act` false only help with the leaf tests).  Returns
// the hit in `hit` (t from the start os = o + skip d); `len` is the distance
// from o to the target (0: the target is o, no ray).
template <int NL, bool OV>
__device__ __forceinline__ void trace_towards(const RefineArgs& a, LeafTestLds& W, bool act, const float o[3],
                                              const float target[3], uint32_t last, float skip, Hit& hit, float d[3],
                                              float os[3], float& len, stat_t cnt[ST_COUNT]) {
    d[0] = target[0] - o[0];
    d[1] = target[1] - o[1];
    d[2] = target[2] - o[2];
    len = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const bool go = act && len > 0.f;
    if (go) {
        const float inv = 1.0f / len;
        d[0] *= inv;
        d[1] *= inv;
        d[2] *= inv;
    } else {
        d[0] = 1.f;
        d[1] = d[2] = 0.f;
    }
    os[0] = o[0] + skip * d[0];
    os[1] = o[1] + skip * d[1];
    os[2] = o[2] + skip * d[2];
    hit_reset(hit);
    stage_ray(W, os, d, last);
    trace_segment<false, NL, false>(a.t, W, go, os, d, hit, cnt);
    if (OV) trace_segment<false, NL, true>(a.t, W, go, os, d, hit, cnt);
}

// Add the weighted normals of the points of hierarchy v within sqrt(h2) of c
// (the n(x) of Eq. 1; weights (1 - d^2/h2)^4, each normal turned to agree
// with nh).  h2 is below one leaf edge squared, so the points lie in the 27
// leaves around c's; a point is taken from the leaf holding its centre only
// (every leaf its disk meets lists it).
template <int NL>
__device__ __forceinline__ void gather_normals(const SceneView& v, const float c[3], float h2, const float nh[3],
                                               float acc[3]) {
    int lc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) lc[a] = (int)floorf((c[a] - v.org[a]) * v.inv_h);
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int cell[3] = {lc[0] + dx, lc[1] + dy, lc[2] + dz};
                if (cell[0] < 0 || cell[1] < 0 || cell[2] < 0 || cell[0] >= v.dim[0] || cell[1] >= v.dim[1] ||
                    cell[2] >= v.dim[2])
                    continue;
                uint32_t node = 0;
                int skip0 = 0;
                if (descend<false, NL - 1>(v, cell, node, skip0, nullptr) != NL) continue;
                const uint2 r = v.leaf[node];
                for (uint32_t e = r.x; e < r.x + r.y; ++e) {
                    const float4 P = v.spos[e];
                    const float x = P.x - c[0], y = P.y - c[1], z = P.z - c[2];
                    const float d2 = x * x + y * y + z * z;
                    if (!(d2 < h2)) continue;
                    if ((int)floorf((P.x - v.org[0]) * v.inv_h) != cell[0] ||
                        (int)floorf((P.y - v.org[1]) * v.inv_h) != cell[1] ||
                        (int)floorf((P.z - v.org[2]) * v.inv_h) != cell[2])
                        continue;
                    const float4 N = v.snrm[e];
                    float w = 1.0f - d2 / h2;
                    w *= w;
                    w *= w;
                    if (N.x * nh[0] + N.y * nh[1] + N.z * nh[2] < 0.f) w = -w;
                    acc[0] += w * N.x;
                    acc[1] += w * N.y;
                    acc[2] += w * N.z;
                }
            }
}

__device__ __forceinline__ void load3(const float4* p, float x[3]) {
    const float4 v = *p;
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
}

template <int NL, bool OV>
__global__ __launch_bounds__(REFINE_BLOCK) void k_refine(RefineArgs a) {
    __shared__ LeafTestLds W;
    stat_t cnt[ST_COUNT] = {};
    const uint32_t p = blockIdx.x * a.ppw + threadIdx.x;
    const bool in = threadIdx.x < a.ppw && p < a.n;
    const size_t n = a.n;
    int N = 0;
    float T[3] = {0.f, 0.f, 0.f}, R[3] = {0.f, 0.f, 0.f};
    if (in) {
        N = a.p_n[p];
        const int ti = a.p_tx[p], ri = a.p_rx[p];
        T[0] = a.tx[3 * ti];
        T[1] = a.tx[3 * ti + 1];
        T[2] = a.tx[3 * ti + 2];
        R[0] = a.rx[3 * ri];
        R[1] = a.rx[3 * ri + 1];
        R[2] = a.rx[3 * ri + 2];
        for (int k = 0; k < N; ++k) {
            const float* q = a.p_pts + ((size_t)p * a.K + k) * 3;
            // a diffraction point starts at the coarse point's projection onto its edge (t in w)
            float t = 0.f;
            const int e = edge_at(a, p, k);
            if (e >= 0) {
                const float4 A = a.e_a[e], Wd = a.e_w[e];
                t = (q[0] - A.x) * Wd.x + (q[1] - A.y) * Wd.y + (q[2] - A.z) * Wd.z;
            }
            a.tgt[k * n + p] = make_float4(q[0], q[1], q[2], t);
        }
    }
    const int nmax = wave_max(N);
    int status = PCRL_REFINE_VALID;
    int it = 0;
    float gnorm = 0.f;
    bool run = in && N > 0;
    while (__ballot(run)) {
        // the interaction points: diffraction points on their edges, reflection points where the
        // rays towards the targets hit
        float o[3] = {T[0], T[1], T[2]};
        uint32_t last = NO_HIT;
        float skip = 0.f;
        for (int k = 0; k < nmax; ++k) {
            const bool act = run && k < N;
            const int e = act ? edge_at(a, p, k) : -1;
            float tg[3] = {0.f, 0.f, 0.f}, d[3], os[3], len;
            if (act) load3(&a.tgt[k * n + p], tg);
            Hit hit;
            trace_towards<NL, OV>(a, W, act && e < 0, o, tg, last, skip, hit, d, os, len, cnt);
            if (act && e >= 0) {
                const float4 A = a.e_a[e], Wd = a.e_w[e];
                const float t = a.tgt[k * n + p].w;
                o[0] = A.x + t * Wd.x;
                o[1] = A.y + t * Wd.y;
                o[2] = A.z + t * Wd.z;
                last = NO_HIT;
                skip = a.clear;
                a.cpos[k * n + p] = make_float4(o[0], o[1], o[2], __uint_as_float(NO_HIT));
                a.cnrm[k * n + p] = make_float4(0.f, 0.f, 0.f, Wd.w);
            } else if (act) {
                if (!(len > 0.f)) {
                    status = PCRL_REFINE_DEGENERATE;
                    run = false;
                } else if (hit.id == NO_HIT) {
                    status = PCRL_REFINE_MISS;
                    run = false;
                } else {
                    o[0] = os[0] + hit.t * d[0];
                    o[1] = os[1] + hit.t * d[1];
                    o[2] = os[2] + hit.t * d[2];
                    last = hit.id;
                    skip = 0.f;
                    float nr[3] = {hit.nx, hit.ny, hit.nz};
                    if (a.smooth_h2 > 0.f) {
                        float acc[3] = {0.f, 0.f, 0.f};
                        gather_normals<NL>(a.t.v, o, a.smooth_h2, nr, acc);
                        if (OV) gather_normals<NL>(a.t.ov, o, a.smooth_h2, nr, acc);
                        const float l = sqrtf(acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2]);
                        if (l > 0.f) {
                            nr[0] = acc[0] / l;
                            nr[1] = acc[1] / l;
                            nr[2] = acc[2] / l;
                        }
                    }
                    a.cpos[k * n + p] = make_float4(o[0], o[1], o[2], __uint_as_float(hit.id));
                    a.cnrm[k * n + p] = make_float4(nr[0], nr[1], nr[2], __uint_as_float(hit.lab));
                }
            }
        }
        if (!run) continue;
        // gradient of the path length (tangent planes of reflections, edge directions of
        // diffractions) and the next targets
        float prev[3] = {T[0], T[1], T[2]}, cur[3], next[3];
        load3(&a.cpos[p], cur);
        float gg = 0.f;
        bool off = false;
        for (int k = 0; k < N; ++k) {
            if (k + 1 < N) load3(&a.cpos[(k + 1) * n + p], next);
            else {
                next[0] = R[0];
                next[1] = R[1];
                next[2] = R[2];
            }
            const float lp = dist3(cur, prev), ln = dist3(cur, next);
            if (!(lp > 0.f) || !(ln > 0.f)) {
                status = PCRL_REFINE_DEGENERATE;
                run = false;
                break;
            }
            float G[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) G[j] = (cur[j] - prev[j]) / lp + (cur[j] - next[j]) / ln;
            const float ak = a.step / (1.0f / lp + 1.0f / ln);
            const int e = edge_at(a, p, k);
            if (e >= 0) {
                const float4 A = a.e_a[e], Wd = a.e_w[e];
                const float gw = G[0] * Wd.x + G[1] * Wd.y + G[2] * Wd.z;
                gg += gw * gw;
                const float4 tq = a.tgt[k * n + p];
                const float t = tq.w - ak * gw;
                off = off || !(t >= 0.f && t <= A.w);
                a.tgt[k * n + p] = make_float4(tq.x, tq.y, tq.z, t);
            } else {
                float nrm[3];
                load3(&a.cnrm[k * n + p], nrm);
                const float gn = G[0] * nrm[0] + G[1] * nrm[1] + G[2] * nrm[2];
                float g[3];
#pragma unroll
                for (int j = 0; j < 3; ++j) g[j] = G[j] - gn * nrm[j];
                gg += g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
                a.tgt[k * n + p] = make_float4(cur[0] - ak * g[0], cur[1] - ak * g[1], cur[2] - ak * g[2], 0.f);
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                prev[j] = cur[j];
                cur[j] = next[j];
            }
        }
        if (!run) continue;
        gnorm = sqrtf(gg);
        if (gnorm < a.grad_tol) {
            run = false;  // converged
        } else if (it == a.max_iters) {
            status = PCRL_REFINE_NOT_CONVERGED;
            run = false;
        } else if (off) {
            status = PCRL_REFINE_OFF_EDGE;
            run = false;
        } else {
            ++it;
        }
    }
    // a reflection keeps both neighbours on one side of its surfel; a diffraction has both
    // outside its edge's wedge
    if (in && status == PCRL_REFINE_VALID && N > 0) {
        float prev[3] = {T[0], T[1], T[2]}, cur[3], next[3], nrm[3];
        load3(&a.cpos[p], cur);
        for (int k = 0; k < N; ++k) {
            if (k + 1 < N) load3(&a.cpos[(k + 1) * n + p], next);
            else {
                next[0] = R[0];
                next[1] = R[1];
                next[2] = R[2];
            }
            const int e = edge_at(a, p, k);
            bool ok;
            if (e >= 0) {
                const float4 N1 = a.e_n1[e], N2 = a.e_n2[e];
                const float p1 = (prev[0] - cur[0]) * N1.x + (prev[1] - cur[1]) * N1.y + (prev[2] - cur[2]) * N1.z;
                const float p2 = (prev[0] - cur[0]) * N2.x + (prev[1] - cur[1]) * N2.y + (prev[2] - cur[2]) * N2.z;
                const float q1 = (next[0] - cur[0]) * N1.x + (next[1] - cur[1]) * N1.y + (next[2] - cur[2]) * N1.z;
                const float q2 = (next[0] - cur[0]) * N2.x + (next[1] - cur[1]) * N2.y + (next[2] - cur[2]) * N2.z;
                ok = (p1 > 0.f || p2 > 0.f) && (q1 > 0.f || q2 > 0.f);
            } else {
                load3(&a.cnrm[k * n + p], nrm);
                float sp = 0.f, sn = 0.f;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    sp += (prev[j] - cur[j]) * nrm[j];
                    sn += (next[j] - cur[j]) * nrm[j];
                }
                ok = sp * sn > 0.f;
            }
            if (!ok) {
                status = PCRL_REFINE_WRONG_SIDE;
                break;
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                prev[j] = cur[j];
                cur[j] = next[j];
            }
        }
    }
    // segments arriving at a diffraction point: blocked by a hit more than r_s before it
    if (a.p_edge) {
        for (int k = 0; k < nmax; ++k) {
            const bool act = in && status == PCRL_REFINE_VALID && k < N && edge_at(a, p, k) >= 0;
            float o[3] = {T[0], T[1], T[2]}, tg[3] = {0.f, 0.f, 0.f};
            uint32_t last = NO_HIT;
            float skip = 0.f;
            if (act) {
                load3(&a.cpos[k * n + p], tg);
                if (k > 0) {
                    const float4 c = a.cpos[(k - 1) * n + p];
                    o[0] = c.x;
                    o[1] = c.y;
                    o[2] = c.z;
                    if (edge_at(a, p, k - 1) >= 0) skip = a.clear;
                    else last = __float_as_uint(c.w);
                }
            }
            float d[3], os[3], len;
            Hit hit;
            trace_towards<NL, OV>(a, W, act, o, tg, last, skip, hit, d, os, len, cnt);
            if (act) {
                if (!(len > 0.f)) status = PCRL_REFINE_DEGENERATE;
                else if (hit.id != NO_HIT && skip + hit.t < len - a.clear) status = PCRL_REFINE_OCCLUDED;
            }
        }
    }
    // the last segment must reach the RX unblocked
    {
        const bool act = in && status == PCRL_REFINE_VALID;
        float o[3] = {T[0], T[1], T[2]};
        uint32_t last = NO_HIT;
        float skip = 0.f;
        if (act && N > 0) {
            const float4 c = a.cpos[(N - 1) * n + p];
            o[0] = c.x;
            o[1] = c.y;
            o[2] = c.z;
            if (edge_at(a, p, N - 1) >= 0) skip = a.clear;
            else last = __float_as_uint(c.w);
        }
        float d[3], os[3], len;
        Hit hit;
        trace_towards<NL, OV>(a, W, act, o, R, last, skip, hit, d, os, len, cnt);
        if (act) {
            if (!(len > 0.f)) status = PCRL_REFINE_DEGENERATE;
            else if (hit.id != NO_HIT && skip + hit.t < len) status = PCRL_REFINE_OCCLUDED;
        }
    }
    if (!in) return;
    const bool finite = status != PCRL_REFINE_MISS && status != PCRL_REFINE_DEGENERATE;
    float f = 0.f;
    if (finite) {
        float prev[3] = {T[0], T[1], T[2]}, cur[3];
        for (int k = 0; k < N; ++k) {
            const float4 c = a.cpos[k * n + p];
            const float4 m = a.cnrm[k * n + p];
            cur[0] = c.x;
            cur[1] = c.y;
            cur[2] = c.z;
            f += dist3(cur, prev);
            prev[0] = cur[0];
            prev[1] = cur[1];
            prev[2] = cur[2];
            float* q = a.out_pts + ((size_t)p * a.K + k) * 3;
            q[0] = c.x;
            q[1] = c.y;
            q[2] = c.z;
            const int e = edge_at(a, p, k);
            a.out_id[(size_t)p * a.K + k] = e >= 0 ? -2 - e : (int32_t)__float_as_uint(c.w);
            a.out_key[(size_t)p * a.K + k] = (int64_t)__float_as_uint(m.w);
        }
        f += dist3(R, prev);
    }
    for (int k = finite ? N : 0; k < a.K; ++k) {
        float* q = a.out_pts + ((size_t)p * a.K + k) * 3;
        q[0] = q[1] = q[2] = NAN;
        a.out_id[(size_t)p * a.K + k] = -1;
        a.out_key[(size_t)p * a.K + k] = -1;
    }
    a.status[p] = status;
    a.iters[p] = it;
    a.grad[p] = finite ? gnorm : NAN;
    a.length[p] = finite ? f : NAN;
}

// Per edge of refine_paths' edge table: start point and length, unit
// direction and label, the two face normals.  Zero-length edges are counted
// in *bad.
__global__ void k_refine_edges(const float* seg, const float* nrm, const uint32_t* label, uint32_t n, float4* ea,
                               float4* ew, float4* en1, float4* en2, uint32_t* bad) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* s = seg + 6 * (size_t)i;
    const float* m = nrm + 6 * (size_t)i;
    const float d[3] = {s[3] - s[0], s[4] - s[1], s[5] - s[2]};
    const float L = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(L > 0.f)) atomicAdd(bad, 1u);
    const float inv = L > 0.f ? 1.0f / L : 0.f;
    ea[i] = make_float4(s[0], s[1], s[2], L);
    ew[i] = make_float4(d[0] * inv, d[1] * inv, d[2] * inv, __uint_as_float(label[i]));
    en1[i] = make_float4(m[0], m[1], m[2], 0.f);
    en2[i] = make_float4(m[3], m[4], m[5], 0.f);
}

// Sort key of a refined path: its group (the first row of its (TX, RX,
// reflections) run: rows come sorted by coarse key, which starts with these)
// in the high word, its length in the low word (invalid paths last).
__device__ __forceinline__ uint64_t group_of(const int32_t* p_tx, const int32_t* p_rx, const int32_t* p_n, uint32_t i) {
    return ((uint64_t)(uint32_t)p_tx[i] << 24) | ((uint64_t)(uint32_t)p_rx[i] << 8) | (uint64_t)(uint32_t)p_n[i];
}

__global__ void k_refine_keys(const int32_t* p_tx, const int32_t* p_rx, const int32_t* p_n, const int32_t* status,
                              const float* length, uint32_t n, uint64_t* keys, uint32_t* idx) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t g = group_of(p_tx, p_rx, p_n, i);
    uint32_t lo = 0, hi = i;  // first row of the run holding i
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (group_of(p_tx, p_rx, p_n, mid) < g) lo = mid + 1;
        else hi = mid;
    }
    const uint32_t lb = status[i] == PCRL_REFINE_VALID ? __float_as_uint(length[i]) : 0xFFFFFFFFu;
    keys[i] = ((uint64_t)lo << 32) | lb;
    idx[i] = i;
}

// One wave per group (the block whose sorted position starts a group; the
// others return at once).  Candidates in order of length; lanes compare a
// candidate with 64 earlier paths at a time.
__global__ __launch_bounds__(64) void k_refine_sweep(const uint64_t* skey, const uint32_t* sidx, uint32_t n, int32_t K,
                                                     const int32_t* p_tx, const int32_t* p_n, const float* tx,
                                                     const int32_t* status, const float* length, const float* pts,
                                                     const int64_t* key, float lambda, int32_t* kept,
                                                     uint32_t* counters) {
    __shared__ uint32_t klist[SWEEP_KEPT_MAX];
    const uint32_t j0 = blockIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t grp = (uint32_t)(skey[j0] >> 32);
    if (j0 > 0 && (uint32_t)(skey[j0 - 1] >> 32) == grp) return;
    uint32_t j1 = j0 + 1;
    while (j1 < n && (uint32_t)(skey[j1] >> 32) == grp) ++j1;
    uint32_t nk = 0;
    for (uint32_t q = j0; q < j1; ++q) {
        const uint32_t c = sidx[q];
        if (status[c] != PCRL_REFINE_VALID) break;  // invalid paths sort last
        const int N = p_n[c];
        bool dup = false;
        // an earlier (shorter) valid path with the same label sequence
        for (uint32_t e0 = j0; e0 < q && !dup; e0 += 64) {
            const uint32_t e = e0 + lane;
            bool same = false;
            if (e < q) {
                const uint32_t r = sidx[e];
                same = true;
                for (int k = 0; k < N; ++k) same = same && key[(size_t)r * K + k] == key[(size_t)c * K + k];
            }
            dup = __ballot(same) != 0;
        }
        // every point inside the first Fresnel zone of a kept path's point
        if (lambda > 0.f) {
            for (uint32_t e0 = 0; e0 < nk && !dup; e0 += 64) {
                const uint32_t e = e0 + lane;
                bool close = false;
                if (e < nk && e < (uint32_t)SWEEP_KEPT_MAX) {
                    const uint32_t r = klist[e];
                    const float L = length[r];
                    const int ti = p_tx[r];
                    float prev[3] = {tx[3 * ti], tx[3 * ti + 1], tx[3 * ti + 2]};
                    float d1 = 0.f;
                    close = true;
                    for (int k = 0; k < N && close; ++k) {
                        const float* pr = pts + ((size_t)r * K + k) * 3;
                        const float* pc = pts + ((size_t)c * K + k) * 3;
                        const float cur[3] = {pr[0], pr[1], pr[2]};
                        d1 += dist3(cur, prev);
                        const float rf2 = lambda * d1 * (L - d1) / L;
                        const float x = pc[0] - pr[0], y = pc[1] - pr[1], z = pc[2] - pr[2];
                        close = x * x + y * y + z * z <= rf2;
                        prev[0] = cur[0];
                        prev[1] = cur[1];
                        prev[2] = cur[2];
                    }
                }
                dup = __ballot(close) != 0;
            }
        }
        if (!dup) {
            if (lane == 0) {
                if (nk < (uint32_t)SWEEP_KEPT_MAX) klist[nk] = c;
                kept[c] = 1;
            }
            ++nk;
            wave_sync();  // the new entry of klist is visible to every lane
        }
    }
    if (lane == 0) {
        atomicAdd(&counters[0], nk);
        if (nk > (uint32_t)SWEEP_KEPT_MAX) atomicMax(&counters[1], nk);
    }
}

template <int NL>
static void launch_refine_nl(const RefineArgs& a, hipStream_t s) {
    const unsigned grid = (a.n + a.ppw - 1) / a.ppw;
    if (a.t.has_ov) hipLaunchKernelGGL((k_refine<NL, true>), dim3(grid), dim3(REFINE_BLOCK), 0, s, a);
    else hipLaunchKernelGGL((k_refine<NL, false>), dim3(grid), dim3(REFINE_BLOCK), 0, s, a);
}

}  // namespace pcrl

using namespace pcrl;

extern "C" int refine_paths(const PcrlScene* scene, const float* tx, int32_t n_tx, const float* rx, int32_t n_rx,
                            const PcrlPaths* paths, int32_t k_stride, const PcrlRefineParams* params,
                            PcrlRefined* out, pcrl_stream_t stream) {
    clear_error();
    if (!scene || !tx || n_tx < 1 || !rx || n_rx < 1 || !paths || !out || k_stride < 0 ||
        k_stride > PCRL_MAX_REFLECTIONS || paths->n_rows < 0) {
        set_error("refine_paths: invalid scene, antennas, paths or output");
        return PCRL_EINVAL;
    }
    const int64_t n = paths->n_rows;
    if (n >= ((int64_t)1 << 31)) {
        set_error("refine_paths: at most 2^31 - 1 paths");
        return PCRL_EINVAL;
    }
    out->n_kept = 0;
    if (n == 0) return PCRL_OK;
    if (!paths->tx || !paths->rx || !paths->n_refl || (k_stride > 0 && !paths->points) || !out->status ||
        !out->iters || !out->grad || !out->length || !out->kept || (k_stride > 0 && (!out->points ||
        !out->point_id || !out->key))) {
        set_error("refine_paths: a path or output array is NULL");
        return PCRL_EINVAL;
    }
    PcrlRefineParams P{};
    if (params) P = *params;
    const int32_t max_iters = P.max_iters > 0 ? P.max_iters : 2000;
    const float grad_tol = P.grad_tol > 0.f ? P.grad_tol : 1e-4f;
    const float step = P.step > 0.f ? P.step : 0.75f;
    const double carrier = P.carrier_hz == 0.f ? 60e9 : (double)P.carrier_hz;
    if (!(step <= 1.0f) || (P.flags & ~PCRL_REFINE_SMOOTH) || !std::isfinite(carrier)) {
        set_error("refine_paths: need 0 < step <= 1, known flags and a finite carrier");
        return PCRL_EINVAL;
    }
    float smooth_h = 0.f;
    if (P.flags & PCRL_REFINE_SMOOTH) {
        const float leaf = scene->view.h, rs = scene->view.r_s;
        smooth_h = P.smooth_radius > 0.f ? P.smooth_radius : 0.95f * leaf;
        if (!(smooth_h > rs) || !(smooth_h <= 0.98f * leaf)) {
            set_error("refine_paths: the smoothing radius %g must exceed the surfel radius %g and stay within 0.98 "
                      "leaf edges (%g)", (double)smooth_h, (double)rs, (double)leaf);
            return PCRL_EINVAL;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    // the path table is small: validate its indices on the host
    std::vector<int32_t> h_tx(n), h_rx(n), h_n(n);
    PCRL_TRY_HIP(hipMemcpyAsync(h_tx.data(), paths->tx, n * 4, hipMemcpyDeviceToHost, s));
    PCRL_TRY_HIP(hipMemcpyAsync(h_rx.data(), paths->rx, n * 4, hipMemcpyDeviceToHost, s));
    PCRL_TRY_HIP(hipMemcpyAsync(h_n.data(), paths->n_refl, n * 4, hipMemcpyDeviceToHost, s));
    PCRL_TRY_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i) {
        if (h_tx[i] < 0 || h_tx[i] >= n_tx || h_rx[i] < 0 || h_rx[i] >= n_rx || h_n[i] < 0 || h_n[i] > k_stride ||
            h_rx[i] >= (1 << 16)) {
            set_error("refine_paths: row %lld has tx %d, rx %d, n_refl %d (n_tx %d, n_rx %d, K %d)", (long long)i,
                      h_tx[i], h_rx[i], h_n[i], n_tx, n_rx, k_stride);
            return PCRL_EINVAL;
        }
        if (i > 0) {
            const auto g0 = std::make_tuple(h_tx[i - 1], h_rx[i - 1], h_n[i - 1]);
            const auto g1 = std::make_tuple(h_tx[i], h_rx[i], h_n[i]);
            if (g1 < g0) {
                set_error("refine_paths: rows must be sorted by (tx, rx, n_refl) as collect_paths returns them");
                return PCRL_EINVAL;
            }
        }
    }
    // diffraction edges: indices checked on the host (the table is small)
    const bool has_edges = P.edge_of != nullptr && k_stride > 0;
    if (has_edges) {
        if (P.n_edges < 1 || !P.edge_seg || !P.edge_normals || !P.edge_label) {
            set_error("refine_paths: edge_of needs n_edges >= 1 edges with segments, normals and labels");
            return PCRL_EINVAL;
        }
        std::vector<int32_t> h_e((size_t)n * k_stride);
        PCRL_TRY_HIP(hipMemcpyAsync(h_e.data(), P.edge_of, h_e.size() * 4, hipMemcpyDeviceToHost, s));
        PCRL_TRY_HIP(hipStreamSynchronize(s));
        for (size_t i = 0; i < h_e.size(); ++i)
            if (h_e[i] < -1 || h_e[i] >= P.n_edges) {
                set_error("refine_paths: row %lld interaction %d has edge %d (n_edges %d)",
                          (long long)(i / k_stride), (int)(i % k_stride), h_e[i], P.n_edges);
                return PCRL_EINVAL;
            }
    }
    DevBufs T;
    T.stream = s;
    RefineArgs a{};
    a.t.v = scene->view;
    if (scene->overlay && scene->overlay->n_entries > 0) {
        a.t.ov = scene->overlay->view;
        a.t.has_ov = 1;
    }
    a.tx = tx;
    a.rx = rx;
    a.p_tx = paths->tx;
    a.p_rx = paths->rx;
    a.p_n = paths->n_refl;
    a.p_pts = paths->points;
    a.n = (uint32_t)n;
    // paths per wave: a path's iterations run in lockstep with the wave's other paths, so
    // few paths per wave (down to one) as long as the waves still fill the GPU (one per SIMD)
    {
        const int64_t waves = (int64_t)device_cus() * 4;
        a.ppw = (uint32_t)std::min<int64_t>(REFINE_BLOCK, std::max<int64_t>(1, (n + waves - 1) / waves));
    }
    a.K = k_stride;
    a.max_iters = max_iters;
    a.grad_tol = grad_tol;
    a.step = step;
    a.smooth_h2 = smooth_h * smooth_h;
    a.status = out->status;
    a.iters = out->iters;
    a.grad = out->grad;
    a.length = out->length;
    a.out_pts = out->points;
    a.out_id = out->point_id;
    a.out_key = out->key;
    uint64_t* keys = nullptr;
    uint32_t *idx = nullptr, *counters = nullptr;
    int rc = PCRL_OK;
    if (k_stride > 0) {
        const size_t m = (size_t)k_stride * n;
        if (!(rc = T.alloc(&a.cpos, m)) && !(rc = T.alloc(&a.cnrm, m))) rc = T.alloc(&a.tgt, m);
    }
    if (!rc && !(rc = T.alloc(&keys, n)) && !(rc = T.alloc(&idx, n))) rc = T.alloc(&counters, 2);
    if (!rc) rc = fill_u32(counters, 0u, 2, s);
    if (!rc) rc = fill_u32((uint32_t*)out->kept, 0u, n, s);
    if (!rc && has_edges) {
        const uint32_t ne = (uint32_t)P.n_edges;
        float4 *ea = nullptr, *ew = nullptr, *en1 = nullptr, *en2 = nullptr;
        if (!(rc = T.alloc(&ea, ne)) && !(rc = T.alloc(&ew, ne)) && !(rc = T.alloc(&en1, ne)) &&
            !(rc = T.alloc(&en2, ne))) {
            hipLaunchKernelGGL(k_refine_edges, dim3((ne + 255) / 256), dim3(256), 0, s, P.edge_seg, P.edge_normals,
                               P.edge_label, ne, ea, ew, en1, en2, counters);
            uint32_t bad = 0;
            if (hipMemcpyAsync(&bad, counters, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                set_error("refine_paths: edge table failed: %s", hipGetErrorString(hipGetLastError()));
                rc = PCRL_EHIP;
            } else if (bad) {
                set_error("refine_paths: %u edges have zero length", bad);
                rc = PCRL_EINVAL;
            } else {
                rc = fill_u32(counters, 0u, 2, s);
            }
        }
        a.p_edge = P.edge_of;
        a.e_a = ea;
        a.e_w = ew;
        a.e_n1 = en1;
        a.e_n2 = en2;
    }
    a.clear = scene->view.r_s;
    if (rc) {
        T.release();
        return rc;
    }
    switch (scene->view.nlev) {
    case 1: launch_refine_nl<1>(a, s); break;
    case 2: launch_refine_nl<2>(a, s); break;
    case 3: launch_refine_nl<3>(a, s); break;
    default: launch_refine_nl<4>(a, s); break;
    }
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_refine_keys, dim3(g), dim3(256), 0, s, paths->tx, paths->rx, paths->n_refl, out->status,
                       out->length, (uint32_t)n, keys, idx);
    if (hipGetLastError() != hipSuccess) {
        T.release();
        set_error("refine_paths: kernel launch failed");
        return PCRL_EHIP;
    }
    int bits = 32;
    while (bits < 64 && ((uint64_t)n >> (bits - 32))) ++bits;
    rc = radix_sort_u64(keys, idx, n, bits, s);
    if (!rc) {
        const float lambda = carrier > 0.0 ? (float)(299792458.0 / carrier) : 0.f;
        hipLaunchKernelGGL(k_refine_sweep, dim3((unsigned)n), dim3(64), 0, s, keys, idx, (uint32_t)n, k_stride,
                           paths->tx, paths->n_refl, tx, out->status, out->length, out->points, out->key, lambda,
                           out->kept, counters);
        if (hipGetLastError() != hipSuccess) rc = PCRL_EHIP;
    }
    uint32_t h_cnt[2] = {0u, 0u};
    if (!rc && hipMemcpyAsync(h_cnt, counters, sizeof(h_cnt), hipMemcpyDeviceToHost, s) != hipSuccess) rc = PCRL_EHIP;
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = PCRL_EHIP;
    T.release();
    if (rc == PCRL_EHIP) set_error("refine_paths: HIP error: %s", hipGetErrorString(hipGetLastError()));
    if (rc) return rc;
    out->n_kept = h_cnt[0];
    if (h_cnt[1]) {
        set_error("refine_paths: a (tx, rx, n_refl) group keeps %u paths, more than %d", h_cnt[1], SWEEP_KEPT_MAX);
        return PCRL_EOVERFLOW;
    }
    return PCRL_OK;
}
