// trace.hip -- uniform ray launching over the voxel hierarchy (paper, Section 2.2).
//
// One kernel launch per bounce b = 0..K.  Lane = ray.  Per segment a lane
//   1. walks the hierarchy by DDA in finest-leaf integer coordinates: at every
//      step it looks the current leaf up top-down (level-0 map, then one brick
//      word per level); an empty cell at level i is skipped whole (its exit
//      along the ray is computed at level i's size), an occupied leaf has
//      all its surfels tested;
//   2. keeps the nearest surfel hit (ties: smaller point id) and stops once
//      the next cell starts beyond it;
//   3. tests every RX sphere on [0, t_hit] (rho grows with unfolded length);
//   4. reflects at the hit (d' = d - 2 (d.n) n) and appends the surviving ray
//      to the next bounce's buffer with one atomic per wave (ballot + popcount
//      rank).
// Reception records are appended the same way.  The bounce kernels read the
// active ray count from device memory, so the whole bounce loop is enqueued
// without host synchronisation.
#include "internal.h"

#include <cmath>
#include <cstring>

namespace pcrl {

constexpr int TRACE_BLOCK = 256;
constexpr uint32_t NO_HIT = 0xFFFFFFFFu;

// Statistics of the PCRL_LAUNCH_STATS kernel variant.  ST_BYTES is the exact
// algorithmic traffic of the trace kernels: 4 B per level-0 map read, 8 B per
// brick mask word (+4 B base when the bit is set), 8 B per leaf range, 32 B
// per surfel tested, 36 B of ray state read per segment after the first,
// 36 B of ray state + 16 B of history per reflection, 16 B per record.
enum StatSlot { ST_SEGMENTS = 0, ST_DDA, ST_LEAVES, ST_NODES, ST_TESTS, ST_HITS, ST_BYTES, ST_COUNT };
typedef unsigned long long stat_t;

struct TraceArgs {
    SceneView v;
    const float* tx;
    const float* rx;
    const float* dirs;      // null: Fibonacci lattice
    const uint32_t* perm;   // null, or bounce-0 order of the directions
    int32_t n_rx;
    int32_t K;
    int32_t b;
    uint32_t n_rays;
    uint32_t n_total;
    float sig_c;            // sigma * alpha / sqrt(3)
    const float4* in_o;     // (o, L)
    const float4* in_d;     // (d, last id bits)
    const uint32_t* in_g;
    float4* out_o;
    float4* out_d;
    uint32_t* out_g;
    uint32_t* counters;     // [b] active rays of bounce b, [K+2] records
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
                              stat_t cnt[ST_COUNT]) {
    hit.id = NO_HIT;
    hit.t = INFINITY;
    hit.lab = 0;
    hit.nx = hit.ny = hit.nz = 0.f;
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
        int lvl;  // level of the empty cell containing c, or L for an occupied leaf
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
                }
            }
        }
        if (STATS) ++cnt[ST_DDA];
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
            lo[a] = (S == 1) ? c[a] : span_div(c[a], v.mspan[lvl]) * S;
            hi[a] = lo[a] + S;
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

template <bool FIRST, bool STATS>
__global__ __launch_bounds__(TRACE_BLOCK) void k_trace(TraceArgs a) {
    const uint32_t n_act = FIRST ? a.n_total : a.counters[a.b];
    // Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD
    // b % 8).  Renumber them so that each XCD works on one contiguous range of
    // rays: neighbouring (coherent) rays then share that XCD's L2.
    const uint32_t nb = gridDim.x, bx = blockIdx.x;
    const uint32_t xcd = bx & 7u, per = nb >> 3, extra = nb & 7u;
    const uint32_t lblock = xcd * per + min(xcd, extra) + (bx >> 3);
    const uint32_t wave = lblock * (TRACE_BLOCK / 64) + (threadIdx.x >> 6);
    const uint32_t n_waves = gridDim.x * (TRACE_BLOCK / 64);
    const uint32_t lane = lane_id();
    const uint64_t lt = lanemask_lt();
    stat_t cnt[ST_COUNT] = {0, 0, 0, 0, 0, 0, 0};
    uint32_t* rec_counter = &a.counters[PCRL_CNT_REC(a.K)];
    for (uint32_t base = wave * 64; base < n_act; base += n_waves * 64) {
        const uint32_t i = base + lane;
        const bool act = i < n_act;
        float o[3] = {0.f, 0.f, 0.f}, d[3] = {1.f, 0.f, 0.f};
        float L = 0.f;
        uint32_t last = NO_HIT, g = 0;
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
                const float4 o4 = a.in_o[i];
                const float4 d4 = a.in_d[i];
                o[0] = o4.x; o[1] = o4.y; o[2] = o4.z; L = o4.w;
                d[0] = d4.x; d[1] = d4.y; d[2] = d4.z; last = __float_as_uint(d4.w);
                g = a.in_g[i];
            }
        }
        Hit hit;
        hit.id = NO_HIT;
        hit.t = INFINITY;
        if (act) {
            trace_segment<STATS>(a.v, o, d, last, hit, cnt);
            if (STATS) {
                ++cnt[ST_SEGMENTS];
                if (hit.id != NO_HIT) ++cnt[ST_HITS];
                if (!FIRST) cnt[ST_BYTES] += 36;
            }
            if (a.hit_id) {
                const size_t idx = (size_t)g * (a.K + 1) + a.b;
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
                    a.rec[slot] = make_uint4(g, (uint32_t)r | ((uint32_t)a.b << 16), __float_as_uint(lp),
                                             __float_as_uint(L + s));
                }
            }
        }
        // reflect and compact survivors
        const bool surv = act && hit.id != NO_HIT && a.b < a.K;
        if (surv) {
            const float qx = o[0] + hit.t * d[0], qy = o[1] + hit.t * d[1], qz = o[2] + hit.t * d[2];
            a.hist[(size_t)a.b * a.n_total + g] = make_float4(qx, qy, qz, __uint_as_float(hit.lab));
            L += hit.t;
            const float dn = d[0] * hit.nx + d[1] * hit.ny + d[2] * hit.nz;
            float ex = d[0] - 2.f * dn * hit.nx, ey = d[1] - 2.f * dn * hit.ny, ez = d[2] - 2.f * dn * hit.nz;
            const float inv = 1.0f / sqrtf(ex * ex + ey * ey + ez * ez);
            d[0] = ex * inv; d[1] = ey * inv; d[2] = ez * inv;
            o[0] = qx; o[1] = qy; o[2] = qz;
            last = hit.id;
        }
        const uint64_t m = __ballot(surv);
        if (m) {
            const int leader = __ffsll((long long)m) - 1;
            uint32_t slot = 0;
            if ((int)lane == leader) slot = atomicAdd(&a.counters[a.b + 1], (uint32_t)__popcll(m));
            slot = __shfl(slot, leader, 64) + (uint32_t)__popcll(m & lt);
            if (STATS && surv) cnt[ST_BYTES] += 52;
            if (surv) {
                a.out_o[slot] = make_float4(o[0], o[1], o[2], L);
                a.out_d[slot] = make_float4(d[0], d[1], d[2], __uint_as_float(last));
                a.out_g[slot] = g;
            }
        }
    }
    if (STATS) {
#pragma unroll
        for (int k = 0; k < ST_COUNT; ++k) {
            const uint64_t sum = wave_sum_u64(cnt[k]);
            if (lane == 0 && sum) atomicAdd(&a.stats[k], (unsigned long long)sum);
        }
    }
}

__global__ void k_fib(uint32_t n, float* out) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float x, y, z;
    fib_dir(j, n, x, y, z);
    out[3 * (size_t)j] = x;
    out[3 * (size_t)j + 1] = y;
    out[3 * (size_t)j + 2] = z;
}

__device__ __forceinline__ uint32_t spread_bits16(uint32_t x) {
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

// Sort key of a launch direction: Morton code of its octahedral map, so rays
// that are close on the sphere are close in the bounce-0 order.
__global__ void k_dir_keys(const float* dirs, uint32_t n, uint32_t* keys, uint32_t* idx) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float x, y, z;
    if (dirs) {
        x = dirs[3 * (size_t)j];
        y = dirs[3 * (size_t)j + 1];
        z = dirs[3 * (size_t)j + 2];
    } else {
        fib_dir(j, n, x, y, z);
    }
    const float s = fabsf(x) + fabsf(y) + fabsf(z);
    float u = s > 0.f ? x / s : 0.f, w = s > 0.f ? y / s : 0.f;
    if (z < 0.f) {
        const float uu = (1.f - fabsf(w)) * (u >= 0.f ? 1.f : -1.f);
        const float ww = (1.f - fabsf(u)) * (w >= 0.f ? 1.f : -1.f);
        u = uu;
        w = ww;
    }
    const uint32_t qu = (uint32_t)fminf(fmaxf((u * 0.5f + 0.5f) * 65535.f, 0.f), 65535.f);
    const uint32_t qw = (uint32_t)fminf(fmaxf((w * 0.5f + 0.5f) * 65535.f, 0.f), 65535.f);
    keys[j] = spread_bits16(qu) | (spread_bits16(qw) << 1);
    idx[j] = j;
}

__global__ void k_fill_logs(int32_t* id, float* t, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    id[i] = -2;
    if (t) t[i] = NAN;
}

__global__ void k_unpack_records(const uint4* rec, const uint32_t* count, uint32_t cap, int64_t* ray, int32_t* rx,
                                 int32_t* nb, float* lp, float* lu) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t n = min(*count, cap);
    if (i >= n) return;
    const uint4 r = rec[i];
    if (ray) ray[i] = r.x;
    if (rx) rx[i] = (int32_t)(r.y & 0xFFFFu);
    if (nb) nb[i] = (int32_t)(r.y >> 16);
    if (lp) lp[i] = __uint_as_float(r.z);
    if (lu) lu[i] = __uint_as_float(r.w);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

template <bool FIRST, bool STATS>
static void launch_trace(const TraceArgs& a, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((k_trace<FIRST, STATS>), dim3(grid), dim3(TRACE_BLOCK), 0, s, a);
}

int launch_enqueue(PcrlLaunch* L, const float* tx, const float* rx, const float* dirs, int32_t* hit_id, float* hit_t) {
    const PcrlScene* S = L->scene;
    hipStream_t s = L->stream;
    const int K = L->K;
    const uint32_t n_total = (uint32_t)L->n_total;
    DevBufs& B = L->bufs;
    float4 *oa = nullptr, *da = nullptr, *ob = nullptr, *db = nullptr;
    uint32_t *ga = nullptr, *gb = nullptr;
    if (K > 0) {
        PCRL_TRY(B.alloc(&oa, n_total));
        PCRL_TRY(B.alloc(&da, n_total));
        PCRL_TRY(B.alloc(&ga, n_total));
        if (K > 1) {
            PCRL_TRY(B.alloc(&ob, n_total));
            PCRL_TRY(B.alloc(&db, n_total));
            PCRL_TRY(B.alloc(&gb, n_total));
        }
    }
    PCRL_TRY(fill_u32(L->counters, 0u, PCRL_NCOUNTERS(K), s));
    if (L->stats) PCRL_TRY(fill_u64((uint64_t*)L->stats, 0ull, 8, s));
    if (hit_id) {
        const size_t n = (size_t)n_total * (K + 1);
        hipLaunchKernelGGL(k_fill_logs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, hit_id, hit_t, n);
    }
    uint32_t* perm = nullptr;
    if (L->flags & PCRL_LAUNCH_COHERENT) {
        const uint32_t nr = (uint32_t)L->n_rays;
        uint32_t* keys = nullptr;
        PCRL_TRY(B.alloc(&keys, nr));
        PCRL_TRY(B.alloc(&perm, nr));
        hipLaunchKernelGGL(k_dir_keys, dim3((nr + 255) / 256), dim3(256), 0, s, dirs, nr, keys, perm);
        PCRL_TRY_HIP(hipGetLastError());
        PCRL_TRY(radix_sort_u32(keys, perm, nr, 32, s));
    }
    TraceArgs a{};
    a.v = S->view;
    a.tx = tx;
    a.rx = rx;
    a.dirs = dirs;
    a.perm = perm;
    a.n_rx = L->n_rx;
    a.K = K;
    a.n_rays = (uint32_t)L->n_rays;
    a.n_total = n_total;
    a.sig_c = (float)((double)L->sigma * (double)L->alpha / std::sqrt(3.0));
    a.counters = L->counters;
    a.hist = L->hist;
    a.rec = L->rec;
    a.rec_cap = (uint32_t)L->rec_cap;
    a.hit_id = hit_id;
    a.hit_t = hit_t;
    a.stats = L->stats;
    const bool stats = L->stats != nullptr;
    const bool timing = !L->events.empty();
    const unsigned full = (unsigned)((n_total + TRACE_BLOCK - 1) / TRACE_BLOCK);
    const unsigned capped = std::min<unsigned>(full, (unsigned)device_cus() * 16);
    for (int b = 0; b <= K; ++b) {
        a.b = b;
        // ping-pong: bounce b reads the survivors of b-1 and writes survivors of b
        float4* wo = (b % 2 == 0) ? oa : ob;
        float4* wd = (b % 2 == 0) ? da : db;
        uint32_t* wg = (b % 2 == 0) ? ga : gb;
        a.in_o = (b % 2 == 0) ? ob : oa;
        a.in_d = (b % 2 == 0) ? db : da;
        a.in_g = (b % 2 == 0) ? gb : ga;
        a.out_o = wo;
        a.out_d = wd;
        a.out_g = wg;
        if (timing) PCRL_TRY_HIP(hipEventRecord(L->events[2 * b], s));
        if (b == 0) {
            if (stats) launch_trace<true, true>(a, full, s);
            else launch_trace<true, false>(a, full, s);
        } else {
            if (stats) launch_trace<false, true>(a, capped, s);
            else launch_trace<false, false>(a, capped, s);
        }
        PCRL_TRY_HIP(hipGetLastError());
        if (timing) PCRL_TRY_HIP(hipEventRecord(L->events[2 * b + 1], s));
    }
    return PCRL_OK;
}

}  // namespace pcrl

using namespace pcrl;

extern "C" int launch_rays(const PcrlScene* scene, const float* tx, int32_t n_tx, const float* rx, int32_t n_rx,
                           const PcrlLaunchParams* p, pcrl_stream_t stream, PcrlLaunch** out) {
    clear_error();
    if (!out) {
        set_error("launch_rays: out is NULL");
        return PCRL_EINVAL;
    }
    *out = nullptr;
    if (!scene || !p || !tx || n_tx < 1 || n_rx < 0 || (n_rx > 0 && !rx)) {
        set_error("launch_rays: invalid scene, params or antenna arrays");
        return PCRL_EINVAL;
    }
    if (p->n_rays < 1 || p->max_reflections < 0 || p->max_reflections > PCRL_MAX_REFLECTIONS || n_rx > 65535) {
        set_error("launch_rays: need n_rays >= 1, 0 <= max_reflections <= %d, n_rx <= 65535", PCRL_MAX_REFLECTIONS);
        return PCRL_EINVAL;
    }
    const int64_t n_total = (int64_t)n_tx * p->n_rays;
    if (n_total >= ((int64_t)1 << 31)) {
        set_error("launch_rays: n_tx * n_rays must stay below 2^31");
        return PCRL_EINVAL;
    }
    if ((p->hit_log_id == nullptr) != (p->hit_log_t == nullptr)) {
        set_error("launch_rays: hit_log_id and hit_log_t must be given together");
        return PCRL_EINVAL;
    }
    PcrlLaunch* L = new (std::nothrow) PcrlLaunch();
    if (!L) {
        set_error("launch_rays: host allocation failed");
        return PCRL_ENOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    L->scene = scene;
    L->stream = s;
    L->bufs.stream = s;
    L->n_rays = p->n_rays;
    L->n_total = n_total;
    L->n_tx = n_tx;
    L->n_rx = n_rx;
    L->K = p->max_reflections;
    L->flags = p->flags;
    L->sigma = p->rx_radius_scale > 0.f ? p->rx_radius_scale : 1.25f;
    L->alpha = p->ray_spacing > 0.f ? p->ray_spacing
                                    : (float)std::sqrt(8.0 * M_PI / (std::sqrt(3.0) * (double)p->n_rays));
    if (p->record_capacity > 0) {
        L->rec_cap = p->record_capacity;
    } else {
        const int64_t est = n_total * (L->K + 1) * std::min<int64_t>(n_rx, 8) / 16 + 65536;
        L->rec_cap = n_rx == 0 ? 1 : est;
    }
    if (L->rec_cap > (int64_t)0xFFFFFFF0ll) L->rec_cap = (int64_t)0xFFFFFFF0ll;
    int rc = PCRL_OK;
    const int K = L->K;
    if (K > 0) rc = L->bufs.alloc(&L->hist, (size_t)K * n_total);
    if (!rc) rc = L->bufs.alloc(&L->rec, (size_t)L->rec_cap);
    if (!rc) rc = L->bufs.alloc(&L->counters, PCRL_NCOUNTERS(K));
    if (!rc && (p->flags & PCRL_LAUNCH_STATS)) rc = L->bufs.alloc(&L->stats, 8);
    if (!rc && (p->flags & PCRL_LAUNCH_TIMING)) {
        L->events.resize(2 * (K + 1));
        for (auto& e : L->events) {
            if (hipEventCreate(&e) != hipSuccess) {
                set_error("launch_rays: hipEventCreate failed");
                rc = PCRL_EHIP;
                e = nullptr;
            }
        }
    }
    if (!rc) rc = launch_enqueue(L, tx, rx, p->directions, p->hit_log_id, p->hit_log_t);
    if (rc) {
        for (auto e : L->events)
            if (e) (void)hipEventDestroy(e);
        L->bufs.release();
        delete L;
        return rc;
    }
    *out = L;
    return PCRL_OK;
}

extern "C" int launch_directions(int64_t n_rays, float* out, pcrl_stream_t stream) {
    clear_error();
    if (n_rays < 1 || n_rays >= ((int64_t)1 << 31) || !out) {
        set_error("launch_directions: need 1 <= n_rays < 2^31 and an output array");
        return PCRL_EINVAL;
    }
    hipLaunchKernelGGL(k_fib, dim3((unsigned)((n_rays + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       (uint32_t)n_rays, out);
    PCRL_TRY_HIP(hipGetLastError());
    return PCRL_OK;
}

extern "C" int launch_stats(PcrlLaunch* L, PcrlLaunchStats* out) {
    clear_error();
    if (!L || !out) {
        set_error("launch_stats: NULL argument");
        return PCRL_EINVAL;
    }
    std::memset(out, 0, sizeof *out);
    const int K = L->K;
    uint32_t cnt[PCRL_NCOUNTERS(PCRL_MAX_REFLECTIONS)];
    unsigned long long st[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    PCRL_TRY_HIP(hipMemcpyAsync(cnt, L->counters, sizeof(uint32_t) * PCRL_NCOUNTERS(K), hipMemcpyDeviceToHost, L->stream));
    if (L->stats) PCRL_TRY_HIP(hipMemcpyAsync(st, L->stats, sizeof st, hipMemcpyDeviceToHost, L->stream));
    PCRL_TRY_HIP(hipStreamSynchronize(L->stream));
    out->rays = L->n_total;
    out->active[0] = L->n_total;
    int64_t seg = L->n_total;
    for (int b = 1; b <= K; ++b) {
        out->active[b] = cnt[b];
        seg += cnt[b];
    }
    out->segments = seg;
    out->records = cnt[PCRL_CNT_REC(K)];
    out->record_capacity = L->rec_cap;
    out->dda_steps = (int64_t)st[ST_DDA];
    out->leaves_visited = (int64_t)st[ST_LEAVES];
    out->node_lookups = (int64_t)st[ST_NODES];
    out->surfel_tests = (int64_t)st[ST_TESTS];
    out->hits = (int64_t)st[ST_HITS];
    out->algo_bytes = (int64_t)st[ST_BYTES];
    if (!L->events.empty()) {
        float total = 0.f;
        for (int b = 0; b <= K; ++b) {
            float ms = 0.f;
            PCRL_TRY_HIP(hipEventElapsedTime(&ms, L->events[2 * b], L->events[2 * b + 1]));
            out->kernel_ms[b] = ms;
        }
        PCRL_TRY_HIP(hipEventElapsedTime(&total, L->events[0], L->events[2 * K + 1]));
        out->total_ms = total;
    }
    return PCRL_OK;
}

extern "C" int launch_records(PcrlLaunch* L, int64_t cap, int64_t* ray, int32_t* rx, int32_t* n_refl,
                              float* len_poly, float* len_unf, int64_t* n_out) {
    clear_error();
    if (!L || !n_out || cap < 0) {
        set_error("launch_records: invalid arguments");
        return PCRL_EINVAL;
    }
    uint32_t n = 0;
    PCRL_TRY_HIP(hipMemcpyAsync(&n, L->counters + PCRL_CNT_REC(L->K), 4, hipMemcpyDeviceToHost, L->stream));
    PCRL_TRY_HIP(hipStreamSynchronize(L->stream));
    *n_out = n;
    if ((int64_t)n > L->rec_cap) {
        set_error("launch_records: the launch produced %u records but holds %lld; relaunch with record_capacity >= %u", n,
                  (long long)L->rec_cap, n);
        return PCRL_EOVERFLOW;
    }
    if ((int64_t)n > cap) {
        set_error("launch_records: %u records do not fit in %lld", n, (long long)cap);
        return PCRL_EOVERFLOW;
    }
    if (n) {
        hipLaunchKernelGGL(k_unpack_records, dim3((n + 255) / 256), dim3(256), 0, L->stream, L->rec,
                           L->counters + PCRL_CNT_REC(L->K), (uint32_t)L->rec_cap, ray, rx, n_refl, len_poly, len_unf);
        PCRL_TRY_HIP(hipGetLastError());
        PCRL_TRY_HIP(hipStreamSynchronize(L->stream));
    }
    return PCRL_OK;
}

extern "C" int release_launch(PcrlLaunch* L) {
    clear_error();
    if (!L) return PCRL_OK;
    for (auto e : L->events)
        if (e) (void)hipEventDestroy(e);
    L->bufs.release();
    delete L;
    return PCRL_OK;
}
