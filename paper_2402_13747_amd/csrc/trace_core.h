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
    ST_SEGMENTS = 0, ST_DDA, ST_LEAVES, ST_NODES, ST_TESTS, ST_HITS, ST_BYTES, ST_EMPTY_LEAF, ST_UNIFORM, ST_COUNT
};
typedef unsigned long long stat_t;
static_assert(ST_COUNT <= PCRL_NSTATS, "device statistics buffer too small");

struct TraceArgs {
    SceneView v;
    SceneView ov;           // overlay of dynamic points (valid when has_ov)
    int32_t has_ov;
    const float* tx;
    const float* rx;
    const float* dirs;      // null: Fibonacci lattice
    const uint32_t* perm;   // null, or bounce-0 order of the directions
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

struct Hit {
    uint32_t id;
    uint32_t lab;
    float t;
    float nx, ny, nz;
};

// Fibonacci-lattice direction j of n (FP64, rounded to FP32).
__device__ __forceinline__ void fib_dir(uint32_t j, uint32_t n, float& x, float& y, float& z) {
#pragma clang fp contract(off)
    const double g = (3.0 - sqrt(5.0)) / 2.0;
    const double two_pi = 6.283185307179586476925286766559;
    const double zz = 1.0 - (double)(2ull * j + 1ull) / (double)n;
    const double r = sqrt(fmax(0.0, 1.0 - zz * zz));
    const double jg = (double)j * g;
    const double f = jg - floor(jg);
    const double phi = two_pi * f;
    double s, c;
    sincos(phi, &s, &c);
    x = (float)(r * c);
    y = (float)(r * s);
    z = (float)zz;
}

// Descend from level 0 to level `to` (< nlev) for leaf cell c.  Returns the
// level at which the path is empty, or to + 1 when the level-`to` node exists
// (its index in `node`).  Quotients c / span[i] use the precomputed magics.
template <bool STATS>
__device__ __forceinline__ int descend(const SceneView& v, const int c[3], int to, uint32_t& node, stat_t* cnt) {
    int p[3] = {span_div(c[0], v.mspan[0]), span_div(c[1], v.mspan[0]), span_div(c[2], v.mspan[0])};
    const int32_t n0 = v.map0[p[0] + v.dim0[0] * (p[1] + v.dim0[1] * p[2])];
    if (STATS) {
        ++cnt[ST_NODES];
        cnt[ST_BYTES] += 4;
    }
    if (n0 < 0 || (uint32_t)n0 >= v.nn[0]) return 0;
    uint32_t n = (uint32_t)n0;
    for (int i = 1; i <= to; ++i) {
        const int q[3] = {span_div(c[0], v.mspan[i]), span_div(c[1], v.mspan[i]), span_div(c[2], v.mspan[i])};
        const int r = v.ratio[i - 1];
        const int loc = (q[0] - r * p[0]) + r * ((q[1] - r * p[1]) + r * (q[2] - r * p[2]));
        const size_t wi = (size_t)n * v.nw[i - 1] + (loc >> 6);
        const uint64_t w = v.mask[i - 1][wi];
        const uint64_t bit = uint64_t(1) << (loc & 63);
        if (STATS) {
            ++cnt[ST_NODES];
            cnt[ST_BYTES] += (w & bit) ? 12 : 8;
        }
        if (!(w & bit)) return i;
        n = v.base[i - 1][wi] + (uint32_t)__popcll(w & (bit - 1));
        if (n >= v.nn[i]) return i;
        p[0] = q[0];
        p[1] = q[1];
        p[2] = q[2];
    }
    node = n;
    return to + 1;
}

template <bool STATS>
__device__ void trace_segment(const SceneView& v, const float o[3], const float d[3], uint32_t last, Hit& hit,
                              stat_t cnt[ST_COUNT], bool keep = false) {
    if (!keep) {  // keep: continue from a hit found in another hierarchy (overlay)
        hit.id = NO_HIT;
        hit.t = INFINITY;
        hit.lab = 0;
        hit.nx = hit.ny = hit.nz = 0.f;
    }
    float inv[3];
    int step[3];
    float t0 = 0.f, t1 = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (d[a] > 0.f) {
            step[a] = 1;
            inv[a] = 1.0f / d[a];
            t0 = fmaxf(t0, (v.org[a] - o[a]) * inv[a]);
            t1 = fminf(t1, (v.hi[a] - o[a]) * inv[a]);
        } else if (d[a] < 0.f) {
            step[a] = -1;
            inv[a] = 1.0f / d[a];
            t0 = fmaxf(t0, (v.hi[a] - o[a]) * inv[a]);
            t1 = fminf(t1, (v.org[a] - o[a]) * inv[a]);
        } else {
            step[a] = 0;
            inv[a] = 0.f;
            if (o[a] < v.org[a] || o[a] > v.hi[a]) t1 = -1.f;
        }
    }
    if (!(t0 <= t1)) return;
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int ci = (int)floorf((o[a] + t0 * d[a] - v.org[a]) * v.inv_h);
        c[a] = min(max(ci, 0), v.dim[a] - 1);
    }
    const int max_iter = v.dim[0] + v.dim[1] + v.dim[2] + 8;
    const int L = v.nlev;
    const int P = L - 2;  // level of the leaves' parents (-1: single-level grid)
    // Cache of the parent lookup: consecutive leaves mostly share a parent, so
    // the descent from level 0 runs only when the parent cell changes.
    int cq[3] = {-1, -1, -1};
    int cres = 0;
    uint32_t cnode = 0;
    for (int it = 0; it < max_iter; ++it) {
        uint32_t node = 0;
        int skip = 1;  // > 1: an empty cube of 2 skip - 1 leaves centred on c
        int lvl;       // level of the empty cell containing c, or L for an occupied leaf
        if (P < 0) {
            const int32_t n0 = v.map0[c[0] + v.dim0[0] * (c[1] + v.dim0[1] * c[2])];
            if (STATS) {
                ++cnt[ST_NODES];
                cnt[ST_BYTES] += 4;
            }
            lvl = (n0 < 0 || (uint32_t)n0 >= v.nn[0]) ? 0 : L;
            node = (uint32_t)n0;
        } else {
            const int q[3] = {span_div(c[0], v.mspan[P]), span_div(c[1], v.mspan[P]), span_div(c[2], v.mspan[P])};
            if (q[0] != cq[0] || q[1] != cq[1] || q[2] != cq[2]) {
                cq[0] = q[0];
                cq[1] = q[1];
                cq[2] = q[2];
                cres = descend<STATS>(v, c, P, cnode, cnt);
            }
            if (cres <= P) {
                lvl = cres;
            } else {
                const int r = v.ratio[P];
                const int loc = (c[0] - r * q[0]) + r * ((c[1] - r * q[1]) + r * (c[2] - r * q[2]));
                const size_t wi = (size_t)cnode * v.nw[P] + (loc >> 6);
                const uint64_t w = v.mask[P][wi];
                const uint64_t bit = uint64_t(1) << (loc & 63);
                if (STATS) {
                    ++cnt[ST_NODES];
                    cnt[ST_BYTES] += (w & bit) ? 12 : 8;
                }
                lvl = L - 1;
                if (w & bit) {
                    node = v.base[P][wi] + (uint32_t)__popcll(w & (bit - 1));
                    if (node < v.nn[L - 1]) lvl = L;
                } else if (v.ldist) {
                    // empty leaf: the whole cube of radius skip - 1 around it is empty
                    skip = max(1, (int)v.ldist[(size_t)cnode * (size_t)(r * r * r) + loc]);
                    if (STATS) cnt[ST_BYTES] += 1;
                }
            }
        }
        if (STATS) {
            ++cnt[ST_DDA];
            if (lvl == L - 1 && L > 1) ++cnt[ST_EMPTY_LEAF];
            // leaf visits where every lane of the wave still walking is in the same leaf
            const uint64_t m_leaf = __ballot(lvl == L);
            const int first = m_leaf ? __ffsll((long long)m_leaf) - 1 : 0;
            const uint32_t lead = __shfl(node, first, 64);
            const uint64_t m_walk = __ballot(true);
            if (lvl == L && __ballot(lvl == L && node == lead) == m_walk) ++cnt[ST_UNIFORM];
        }
        int S = 1;
        if (lvl == L) {
            const uint2 r = v.leaf[node];
            if (STATS) {
                ++cnt[ST_LEAVES];
                cnt[ST_TESTS] += r.y;
                cnt[ST_BYTES] += 8 + 32ull * r.y;
            }
            for (uint32_t k = r.x; k < r.x + r.y; ++k) {
                const float4 P4 = v.spos[k];
                const float4 N = v.snrm[k];
                const uint32_t id = __float_as_uint(P4.w);
                const float wx = P4.x - o[0], wy = P4.y - o[1], wz = P4.z - o[2];
                const float den = d[0] * N.x + d[1] * N.y + d[2] * N.z;
                const float num = wx * N.x + wy * N.y + wz * N.z;
                const float t = num * __builtin_amdgcn_rcpf(den);
                const float qx = t * d[0] - wx, qy = t * d[1] - wy, qz = t * d[2] - wz;
                const float dist2 = qx * qx + qy * qy + qz * qz;
                const bool ok = fabsf(den) > 1e-7f && t > v.t_eps && id != last && dist2 <= v.rs2 &&
                                (t < hit.t || (t == hit.t && id < hit.id));
                if (ok) {
                    hit.id = id;
                    hit.t = t;
                    hit.nx = N.x;
                    hit.ny = N.y;
                    hit.nz = N.z;
                    hit.lab = __float_as_uint(N.w);
                }
            }
        } else {
            S = v.span[lvl];
        }
        // exit of the current cell (size S leaves)
        int lo[3], hi[3];
        float te = INFINITY;
        int axis = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (skip > 1) {
                lo[a] = c[a] - (skip - 1);
                hi[a] = c[a] + skip;
            } else {
                lo[a] = (S == 1) ? c[a] : span_div(c[a], v.mspan[lvl]) * S;
                hi[a] = lo[a] + S;
            }
            float ta = INFINITY;
            if (step[a] > 0)
                ta = ((float)hi[a] * v.h + v.org[a] - o[a]) * inv[a];
            else if (step[a] < 0)
                ta = ((float)lo[a] * v.h + v.org[a] - o[a]) * inv[a];
            if (ta < te) {
                te = ta;
                axis = a;
            }
        }
        // no later cell can hold a nearer hit
        if (te > hit.t + (hit.t * 4e-6f + 1e-3f * v.h)) break;
        const int nc = step[axis] > 0 ? hi[axis] : lo[axis] - 1;
        if (nc < 0 || nc >= v.dim[axis]) break;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a == axis || step[a] == 0) continue;
            int j = (int)floorf((o[a] + te * d[a] - v.org[a]) * v.inv_h);
            j = min(max(j, lo[a]), hi[a] - 1);
            j = step[a] > 0 ? max(j, c[a]) : min(j, c[a]);
            c[a] = j;
        }
        c[axis] = nc;
    }
}


// One wave's 64 consecutive slots [base, base + 64) of bounce b of one query.
// Slots at or past `range` are idle; a slot whose ray id is NO_HIT (left by
// an in-place bounce) is idle too.  Survivors go to the other ping-pong
// buffer, compacted with one atomic per wave, or at their own slot when
// `in_place` (dead slots then get NO_HIT).  Every lane of the wave must call
// this (ballots).
template <bool FIRST, bool STATS>
__device__ __forceinline__ void trace_chunk(const TraceArgs& a, int b, uint32_t base, uint32_t range, bool in_place,
                                            stat_t cnt[ST_COUNT]) {
    const uint32_t lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const float4* in_o = a.buf_o[(b & 1) ^ 1];
    const float4* in_d = a.buf_d[(b & 1) ^ 1];
    const uint32_t* in_g = a.buf_g[(b & 1) ^ 1];
    float4* out_o = a.buf_o[b & 1];
    float4* out_d = a.buf_d[b & 1];
    uint32_t* out_g = a.buf_g[b & 1];
    uint32_t* rec_counter = &a.counters[PCRL_CNT_REC(a.K)];
    const uint32_t i = base + lane;
    const bool in_range = i < range;
    bool act = in_range;
    float o[3] = {0.f, 0.f, 0.f}, d[3] = {1.f, 0.f, 0.f};
    float L = 0.f;
    uint32_t last = NO_HIT, g = NO_HIT;
    if (act) {
        if (FIRST) {
            const uint32_t ti = i / a.n_rays;
            const uint32_t jl = i - ti * a.n_rays;
            const uint32_t j = a.perm ? a.perm[jl] : jl;  // direction-coherent order
            g = ti * a.n_rays + j;
            o[0] = a.tx[3 * ti];
            o[1] = a.tx[3 * ti + 1];
            o[2] = a.tx[3 * ti + 2];
            if (a.dirs) {
                d[0] = a.dirs[3 * (size_t)j];
                d[1] = a.dirs[3 * (size_t)j + 1];
                d[2] = a.dirs[3 * (size_t)j + 2];
            } else {
                fib_dir(j, a.n_rays, d[0], d[1], d[2]);
            }
            const float inv = 1.0f / sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            d[0] *= inv;
            d[1] *= inv;
            d[2] *= inv;
        } else {
            g = in_g[i];
            if (g == NO_HIT) {
                act = false;
            } else {
                const float4 o4 = in_o[i];
                const float4 d4 = in_d[i];
                o[0] = o4.x; o[1] = o4.y; o[2] = o4.z; L = o4.w;
                d[0] = d4.x; d[1] = d4.y; d[2] = d4.z; last = __float_as_uint(d4.w);
            }
        }
    }
    Hit hit;
    hit.id = NO_HIT;
    hit.t = INFINITY;
    if (act) {
        trace_segment<STATS>(a.v, o, d, last, hit, cnt);
        // dynamic points: the nearest hit over base and overlay is the nearest
        // hit of the union (ties again by point id)
        if (a.has_ov) trace_segment<STATS>(a.ov, o, d, last, hit, cnt, true);
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
    // reception on [0, t_hit]
    for (int r = 0; r < a.n_rx; ++r) {
        const float rx0 = a.rx[3 * r], rx1 = a.rx[3 * r + 1], rx2 = a.rx[3 * r + 2];
        const float vx = rx0 - o[0], vy = rx1 - o[1], vz = rx2 - o[2];
        const float s = vx * d[0] + vy * d[1] + vz * d[2];
        bool got = false;
        if (act && s > 0.f && s <= hit.t) {
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
    const bool surv = act && hit.id != NO_HIT && b < a.K;
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
        out_o[slot] = make_float4(o[0], o[1], o[2], L);
        out_d[slot] = make_float4(d[0], d[1], d[2], __uint_as_float(last));
        out_g[slot] = g;
    } else if (in_place && in_range) {
        out_g[i] = NO_HIT;
    }
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

}  // namespace pcrl
