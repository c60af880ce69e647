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
#include "trace_core.h"

#include <cmath>
#include <cstring>

namespace pcrl {

// Specialised on the number of voxel levels NL and on the presence of an
// overlay OV, so every level index in the traversal is a compile-time constant.
// Each wave traces 64 consecutive slots in lockstep (neighbouring slots hold
// coherent rays: their lookups share cache lines), grid-stride over the
// active slots; with an overlay, the base hierarchy and then the overlay.
// BX: the traversal uses the bricks' occupied-children boxes (scenes without
// a dense cell table; the table's octant radii already skip empty leaves, and
// the box code's registers would cost those scenes a wave per SIMD).
template <bool FIRST, bool STATS, int NL, bool OV, bool BX>
__global__ __launch_bounds__(TRACE_BLOCK) void k_trace(TraceArgs a, int b) {
    const uint32_t n_act = FIRST ? a.n_total : a.counters[b];
    const uint32_t wave = xcd_block() * (TRACE_BLOCK / 64) + (threadIdx.x >> 6);
    const uint32_t n_waves = gridDim.x * (TRACE_BLOCK / 64);
    __shared__ LeafTestLds lds[TRACE_BLOCK / 64];
    stat_t cnt[ST_COUNT] = {};
    for (uint32_t base = wave * 64; base < n_act; base += n_waves * 64)
        trace_chunk<FIRST, STATS, NL, OV, BX>(a, lds[threadIdx.x >> 6], b, base, n_act, false, cnt);
    flush_stats<STATS>(cnt, a.stats ? a.stats + (size_t)b * PCRL_NSTATS : nullptr);
}

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

// Bucket of a launch direction: Morton code of its cell in a 256 x 256 grid
// over the octahedral map, so rays that are close on the sphere are close in
// the bounce-0 order.
__global__ void k_dir_keys(const float* dirs, uint32_t n, uint16_t* keys) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float u, w;
    octahedral(dirs[3 * (size_t)j], dirs[3 * (size_t)j + 1], dirs[3 * (size_t)j + 2], u, w);
    keys[j] = (uint16_t)(spread_bits16(cell_of(u, 256)) | (spread_bits16(cell_of(w, 256)) << 1));
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

template <bool FIRST, bool STATS, int NL, bool BX>
static void launch_trace_bx(const TraceArgs& a, int b, unsigned grid, hipStream_t s) {
    if (a.has_ov) hipLaunchKernelGGL((k_trace<FIRST, STATS, NL, true, BX>), dim3(grid), dim3(TRACE_BLOCK), 0, s, a, b);
    else hipLaunchKernelGGL((k_trace<FIRST, STATS, NL, false, BX>), dim3(grid), dim3(TRACE_BLOCK), 0, s, a, b);
}

template <bool FIRST, bool STATS, int NL>
static void launch_trace_nl(const TraceArgs& a, int b, unsigned grid, hipStream_t s) {
    if constexpr (NL == 1) {
        launch_trace_bx<FIRST, STATS, NL, false>(a, b, grid, s);   // no bricks
    } else {
        if (a.v.cells) launch_trace_bx<FIRST, STATS, NL, false>(a, b, grid, s);
        else launch_trace_bx<FIRST, STATS, NL, true>(a, b, grid, s);
    }
}

template <bool FIRST, bool STATS>
static void launch_trace(const TraceArgs& a, int b, unsigned grid, hipStream_t s) {
    static_assert(PCRL_MAX_LEVELS == 4, "one kernel specialisation per level count");
    switch (a.v.nlev) {
    case 1: launch_trace_nl<FIRST, STATS, 1>(a, b, grid, s); break;
    case 2: launch_trace_nl<FIRST, STATS, 2>(a, b, grid, s); break;
    case 3: launch_trace_nl<FIRST, STATS, 3>(a, b, grid, s); break;
    default: launch_trace_nl<FIRST, STATS, 4>(a, b, grid, s); break;
    }
}

void destroy_launch(PcrlLaunch* L) {
    if (!L) return;
    // the overlay may be freed (stream-ordered on its build stream) when this
    // reference drops: the launch's own work must be finished first
    if (L->overlay) (void)hipStreamSynchronize(L->stream);
    if (L->owns_events)
        for (auto e : L->events)
            if (e) (void)hipEventDestroy(e);
    L->bufs.release();
    L->shared.reset();
    delete L;
}

// Validate one query, create its launch object, allocate its buffers,
// initialise counters / logs / the coherent ray order, and fill its per-query
// kernel arguments.  Enqueues only initialisation work on `s`.
int launch_prepare(const PcrlScene* scene, const float* tx, int32_t n_tx, const float* rx, int32_t n_rx,
                   const PcrlLaunchParams* p, hipStream_t s, bool timing_events, PcrlLaunch** out, TraceArgs* args) {
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
    const int K = L->K;
    DevBufs& B = L->bufs;
    float4 *oa = nullptr, *da = nullptr, *ob = nullptr, *db = nullptr;
    uint32_t *ga = nullptr, *gb = nullptr, *perm = nullptr;
    int rc = PCRL_OK;
    if (K > 0) rc = B.alloc(&L->hist, (size_t)K * n_total);
    if (!rc) rc = B.alloc(&L->rec, (size_t)L->rec_cap);
    if (!rc) rc = B.alloc(&L->counters, PCRL_NCOUNTERS(K));
    if (!rc && (p->flags & PCRL_LAUNCH_STATS)) rc = B.alloc(&L->stats, (size_t)PCRL_NSTATS * (K + 1));
    if (!rc && K > 0) {
        if (!(rc = B.alloc(&oa, (size_t)n_total)) && !(rc = B.alloc(&da, (size_t)n_total)))
            rc = B.alloc(&ga, (size_t)n_total);
        if (!rc && K > 1 && !(rc = B.alloc(&ob, (size_t)n_total)) && !(rc = B.alloc(&db, (size_t)n_total)))
            rc = B.alloc(&gb, (size_t)n_total);
    }
    if (!rc) rc = fill_u32(L->counters, 0u, PCRL_NCOUNTERS(K), s);
    if (!rc && L->stats) rc = fill_u64((uint64_t*)L->stats, 0ull, (int64_t)PCRL_NSTATS * (K + 1), s);
    if (!rc && p->hit_log_id) {
        const size_t n = (size_t)n_total * (K + 1);
        hipLaunchKernelGGL(k_fill_logs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p->hit_log_id,
                           p->hit_log_t, n);
        if (hipGetLastError() != hipSuccess) rc = PCRL_EHIP;
    }
    // the Fibonacci lattice is materialised once per launch (the trace kernels only read directions)
    const float* dirs = p->directions;
    if (!rc && !dirs) {
        const uint32_t nr = (uint32_t)L->n_rays;
        float* fd = nullptr;
        if (!(rc = B.alloc(&fd, (size_t)3 * nr))) {
            hipLaunchKernelGGL(k_fib, dim3((nr + 255) / 256), dim3(256), 0, s, nr, fd);
            if (hipGetLastError() != hipSuccess) rc = PCRL_EHIP;
        }
        dirs = fd;
    }
    if (!rc && (p->flags & PCRL_LAUNCH_COHERENT)) {
        const uint32_t nr = (uint32_t)L->n_rays;
        uint16_t* keys = nullptr;
        if (!(rc = B.alloc(&keys, nr)) && !(rc = B.alloc(&perm, nr))) {
            hipLaunchKernelGGL(k_dir_keys, dim3((nr + 255) / 256), dim3(256), 0, s, dirs, nr, keys);
            rc = hipGetLastError() == hipSuccess ? bucket_order_u16(keys, nr, nullptr, perm, s) : PCRL_EHIP;
        }
    }
    if (!rc && timing_events && (p->flags & PCRL_LAUNCH_TIMING)) {
        L->events.resize(2 * (K + 1));
        L->owns_events = true;
        for (auto& e : L->events) {
            if (hipEventCreate(&e) != hipSuccess) {
                set_error("launch_rays: hipEventCreate failed");
                rc = PCRL_EHIP;
                e = nullptr;
            }
        }
    }
    if (rc) {
        if (rc == PCRL_EHIP) set_error("launch_rays: HIP error during preparation: %s", hipGetErrorString(hipGetLastError()));
        destroy_launch(L);
        return rc;
    }
    TraceArgs& a = *args;
    a = TraceArgs{};
    a.v = scene->view;
    L->overlay = scene->overlay;  // pin this epoch's dynamic points
    L->max_label = scene->max_label;
    if (L->overlay && L->overlay->n_entries > 0) {
        a.ov = L->overlay->view;
        a.has_ov = 1;
        L->max_label = std::max(L->max_label, L->overlay->max_label);
    }
    a.tx = tx;
    a.rx = rx;
    a.dirs = dirs;
    a.perm = perm;
    a.n_rx = n_rx;
    a.K = K;
    a.n_rays = (uint32_t)L->n_rays;
    a.n_total = (uint32_t)n_total;
    a.sig_c = (float)((double)L->sigma * (double)L->alpha / std::sqrt(3.0));
    a.buf_o[0] = oa;
    a.buf_d[0] = da;
    a.buf_g[0] = ga;
    a.buf_o[1] = ob;
    a.buf_d[1] = db;
    a.buf_g[1] = gb;
    a.counters = L->counters;
    a.hist = L->hist;
    a.rec = L->rec;
    a.rec_cap = (uint32_t)L->rec_cap;
    a.hit_id = p->hit_log_id;
    a.hit_t = p->hit_log_t;
    a.stats = L->stats;
    *out = L;
    return PCRL_OK;
}

// Launches at least this large re-sort the survivors of every bounce for coherence.
constexpr int64_t RESORT_MIN_RAYS = 1 << 16;

// The bounce loop of one query: K + 1 kernel launches (plus, with `order`,
// a key kernel and a radix sort of the survivors between bounces), no host
// synchronisation.
static int launch_run(PcrlLaunch* L, const TraceArgs& a) {
    hipStream_t s = L->stream;
    const int K = L->K;
    const uint32_t n_total = (uint32_t)L->n_total;
    const bool stats = L->stats != nullptr;
    const bool timing = !L->events.empty();
    const unsigned full = (unsigned)((n_total + TRACE_BLOCK - 1) / TRACE_BLOCK);
    const unsigned capped = std::min<unsigned>(full, (unsigned)device_cus() * 16);
    for (int b = 0; b <= K; ++b) {
        if (timing) PCRL_TRY_HIP(hipEventRecord(L->events[2 * b], s));
        if (b == 0) {
            if (stats) launch_trace<true, true>(a, b, full, s);
            else launch_trace<true, false>(a, b, full, s);
        } else {
            if (stats) launch_trace<false, true>(a, b, capped, s);
            else launch_trace<false, false>(a, b, capped, s);
        }
        PCRL_TRY_HIP(hipGetLastError());
        if (timing) PCRL_TRY_HIP(hipEventRecord(L->events[2 * b + 1], s));
        if (a.order && b < K) {
            // the bounce kernel wrote each survivor's bucket and counted the buckets
            PCRL_TRY(bucket_place_u16(a.okeys, a.opos, n_total, a.counters + b + 1, a.ocnt + (size_t)b * 65536,
                                      const_cast<uint32_t*>(a.order), s));
        }
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
    PcrlLaunch* L = nullptr;
    TraceArgs a;
    PCRL_TRY(launch_prepare(scene, tx, n_tx, rx, n_rx, p, (hipStream_t)stream, true, &L, &a));
    // coherence order of the later bounces (results do not depend on it)
    int rc = PCRL_OK;
    if (L->K > 0 && (p->flags & PCRL_LAUNCH_COHERENT) && !(p->flags & PCRL_LAUNCH_SDF) &&
        L->n_total >= RESORT_MIN_RAYS) {
        uint32_t* order = nullptr;
        rc = L->bufs.alloc(&order, (size_t)L->n_total);
        if (!rc) rc = L->bufs.alloc(&a.okeys, (size_t)L->n_total);
        if (!rc) rc = L->bufs.alloc(&a.opos, (size_t)L->n_total);
        if (!rc) rc = L->bufs.alloc(&a.ocnt, (size_t)L->K * 65536);
        if (!rc) rc = fill_u32(a.ocnt, 0u, (int64_t)L->K * 65536, L->stream);
        const SceneView& v = a.v;
        a.klo = make_float3(v.org[0], v.org[1], v.org[2]);
        a.kscale = make_float3(16.f / (v.hi[0] - v.org[0]), 16.f / (v.hi[1] - v.org[1]), 16.f / (v.hi[2] - v.org[2]));
        a.order = order;
    }
    if (!rc) rc = (p->flags & PCRL_LAUNCH_SDF) ? sdf_launch_run(L, a) : launch_run(L, a);
    if (rc) {
        destroy_launch(L);
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
    unsigned long long stb[PCRL_MAX_REFLECTIONS + 1][PCRL_NSTATS] = {};  // per bounce
    unsigned long long st[PCRL_NSTATS] = {};
    PCRL_TRY_HIP(hipMemcpyAsync(cnt, L->counters, sizeof(uint32_t) * PCRL_NCOUNTERS(K), hipMemcpyDeviceToHost, L->stream));
    if (L->stats)
        PCRL_TRY_HIP(hipMemcpyAsync(stb, L->stats, sizeof(unsigned long long) * PCRL_NSTATS * (K + 1),
                                    hipMemcpyDeviceToHost, L->stream));
    PCRL_TRY_HIP(hipStreamSynchronize(L->stream));
    for (int b = 0; b <= K; ++b) {
        for (int k = 0; k < PCRL_NSTATS; ++k) st[k] += stb[b][k];
        out->algo_bytes_bounce[b] = (int64_t)stb[b][ST_BYTES];
        out->dda_steps_bounce[b] = (int64_t)stb[b][ST_DDA];
        out->surfel_tests_bounce[b] = (int64_t)stb[b][ST_TESTS];
        out->wave_dda_bounce[b] = (int64_t)stb[b][ST_WAVE_DDA];
    }
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
    out->empty_leaf_steps = (int64_t)st[ST_EMPTY_LEAF];
    out->uniform_leaf_visits = (int64_t)st[ST_UNIFORM];
    out->wave_dda_iters = (int64_t)st[ST_WAVE_DDA];
    out->wave_test_iters = (int64_t)st[ST_WAVE_TESTS];
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
    destroy_launch(L);
    return PCRL_OK;
}
