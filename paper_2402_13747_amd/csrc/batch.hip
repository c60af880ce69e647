// batch.hip -- many (scene, TX/RX query) launches traced together.
//
// The paper traces each TX separately (Section 2.2); a serving system sees many
// independent queries on scenes of very different sizes.  Launching each
// query on its own leaves the GPU mostly idle in small queries and in the
// tails of every bounce.  Here all queries of a batch share one persistent
// kernel per bounce:
//
//   k_batch_tiles   (1 block)  per query: slots to scan this bounce (range),
//                   and whether survivors are written in place or compacted;
//                   prefix of tiles over queries; resets the work queue.
//   k_trace_batch   (persistent waves) each wave pops a tile (query, first
//                   slot) from the queue and runs the same per-ray bounce
//                   body as the single launch (trace_core.h) on it.
//
// Compaction threshold theta: a bounce writes its survivors in place (no
// atomics, ray order kept) when the predicted density of live rays in the
// scanned range, (live / range) * (live / live of the previous bounce), is at
// least theta; otherwise it compacts them.  theta > 1 always compacts.
//
// Everything the kernels read lives in one device control block, so the whole
// bounce loop can be captured once in a hipGraph and replayed for any batch
// with the same maximum K (the host only rewrites the control block).
#include "trace_core.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

namespace pcrl {

struct BatchCtl {
    const TraceArgs* qs;   // [n_q]
    uint32_t n_q;
    uint32_t tile;         // slots per work item (multiple of 64)
    float theta;
    uint32_t n_tiles;      // tiles of the current bounce
    uint32_t next_tile;    // work-queue head
    uint32_t pad;
    uint32_t* tile_off;    // [n_q + 1]
    uint32_t* range;       // [n_q] slots scanned by the current bounce
    uint32_t* in_place;    // [n_q] current bounce writes survivors in place
    uint32_t* prev_live;   // [n_q] live rays entering the previous bounce
};

constexpr int TILE_BLOCK = 256;

__global__ __launch_bounds__(TILE_BLOCK) void k_batch_tiles(BatchCtl* c, int b) {
    __shared__ uint32_t carry;
    __shared__ uint32_t wsum[TILE_BLOCK / 64];
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const uint32_t n_q = c->n_q;
    const uint32_t tile = c->tile;
    for (uint32_t q0 = 0; q0 < n_q; q0 += TILE_BLOCK) {
        const uint32_t q = q0 + threadIdx.x;
        uint32_t ntiles = 0;
        if (q < n_q) {
            const TraceArgs& a = c->qs[q];
            uint32_t range = 0, live = 0;
            if (b <= a.K) {
                if (b == 0) {
                    range = a.n_total;
                    live = a.n_total;
                } else {
                    live = a.counters[b];
                    range = c->in_place[q] ? c->range[q] : live;
                }
            }
            const uint32_t prev = c->prev_live[q];
            const float dens = range ? (float)live / (float)range : 0.f;
            const float surv = (b == 0 || prev == 0) ? 1.f : (float)live / (float)prev;
            c->in_place[q] = (dens * surv >= c->theta) ? 1u : 0u;
            c->range[q] = range;
            c->prev_live[q] = live;
            ntiles = (range + tile - 1) / tile;
        }
        // block-wide exclusive scan of ntiles
        const uint32_t incl = wave_incl_scan(ntiles);
        const int w = threadIdx.x >> 6;
        if (lane_id() == 63) wsum[w] = incl;
        __syncthreads();
        uint32_t off = carry, tot = 0;
        for (int k = 0; k < TILE_BLOCK / 64; ++k) {
            off += (k < w) ? wsum[k] : 0u;
            tot += wsum[k];
        }
        if (q < n_q) c->tile_off[q] = off + incl - ntiles;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        c->tile_off[n_q] = carry;
        c->n_tiles = carry;
        c->next_tile = 0;
    }
}

// One persistent kernel per group of queries with the same number of voxel
// levels NL and overlay presence OV (the specialisations of the bounce body).
template <bool FIRST, bool STATS, int NL, bool OV>
__global__ __launch_bounds__(TRACE_BLOCK) void k_trace_batch(BatchCtl* c, int b) {
    __shared__ LeafTestLds lds[TRACE_BLOCK / 64];
    stat_t cnt[ST_COUNT] = {};
    const uint32_t n_tiles = c->n_tiles;
    const uint32_t n_q = c->n_q;
    const uint32_t tile = c->tile;
    for (;;) {
        uint32_t t = 0;
        if (lane_id() == 0) t = atomicAdd(&c->next_tile, 1u);
        t = __builtin_amdgcn_readfirstlane(__shfl(t, 0, 64));
        if (t >= n_tiles) break;
        // query owning tile t: the largest q with tile_off[q] <= t
        uint32_t lo = 0, hi = n_q;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (c->tile_off[mid] <= t) lo = mid;
            else hi = mid;
        }
        const uint32_t q = __builtin_amdgcn_readfirstlane(lo);
        const TraceArgs& a = c->qs[q];
        const uint32_t range = c->range[q];
        const bool ip = c->in_place[q] != 0u;
        const uint32_t start = (t - c->tile_off[q]) * tile;
        const uint32_t end = min(start + tile, range);
        for (uint32_t base = start; base < end; base += 64)
            trace_chunk<FIRST, STATS, NL, OV>(a, lds[threadIdx.x >> 6], b, base, range, ip, cnt);
        if (STATS) flush_stats<STATS>(cnt, a.stats ? a.stats + (size_t)b * PCRL_NSTATS : nullptr);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// Batch-level device state kept alive by every query's launch object.
struct BatchShared {
    DevBufs bufs;
    std::vector<hipEvent_t> events;
    ~BatchShared() {
        for (auto e : events)
            if (e) (void)hipEventDestroy(e);
        bufs.release();
    }
};

// Queries of one kernel specialisation, contiguous in the query table.
struct BatchGroup {
    int nl;
    bool ov;
};

template <bool FIRST, bool STATS, int NL>
static void launch_group_nl(bool ov, BatchCtl* ctl, int b, unsigned grid, hipStream_t s) {
    if (ov) hipLaunchKernelGGL((k_trace_batch<FIRST, STATS, NL, true>), dim3(grid), dim3(TRACE_BLOCK), 0, s, ctl, b);
    else hipLaunchKernelGGL((k_trace_batch<FIRST, STATS, NL, false>), dim3(grid), dim3(TRACE_BLOCK), 0, s, ctl, b);
}

template <bool FIRST, bool STATS>
static void launch_group(const BatchGroup& g, BatchCtl* ctl, int b, unsigned grid, hipStream_t s) {
    static_assert(PCRL_MAX_LEVELS == 4, "one kernel specialisation per level count");
    switch (g.nl) {
    case 1: launch_group_nl<FIRST, STATS, 1>(g.ov, ctl, b, grid, s); break;
    case 2: launch_group_nl<FIRST, STATS, 2>(g.ov, ctl, b, grid, s); break;
    case 3: launch_group_nl<FIRST, STATS, 3>(g.ov, ctl, b, grid, s); break;
    default: launch_group_nl<FIRST, STATS, 4>(g.ov, ctl, b, grid, s); break;
    }
}

// A captured bounce loop: replayable for any batch with the same maximum K,
// groups, stream and launch shape; kernels read everything from the groups'
// control blocks.
struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    std::vector<BatchCtl*> ctl;
};

static std::mutex g_graph_mu;
static std::map<std::string, GraphEntry> g_graphs;

template <bool STATS>
static void enqueue_bounces(BatchCtl* const* ctl, const std::vector<BatchGroup>& groups, int kmax, unsigned grid,
                            hipStream_t s, const std::vector<hipEvent_t>* ev) {
    for (int b = 0; b <= kmax; ++b) {
        if (ev) (void)hipEventRecord((*ev)[2 * b], s);
        for (size_t g = 0; g < groups.size(); ++g) {
            hipLaunchKernelGGL(k_batch_tiles, dim3(1), dim3(TILE_BLOCK), 0, s, ctl[g], b);
            if (b == 0) launch_group<true, STATS>(groups[g], ctl[g], b, grid, s);
            else launch_group<false, STATS>(groups[g], ctl[g], b, grid, s);
        }
        if (ev) (void)hipEventRecord((*ev)[2 * b + 1], s);
    }
}

static int run_graph(const std::vector<BatchCtl>& host_ctl, const std::vector<BatchGroup>& groups, int kmax,
                     unsigned grid, bool stats, hipStream_t s) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::string key;
    {
        char head[96];
        snprintf(head, sizeof head, "%d/%p/%d/%u/%d", dev, (void*)s, kmax, grid, stats ? 1 : 0);
        key = head;
        for (const auto& g : groups) key += "/" + std::to_string(g.nl) + (g.ov ? "o" : "b");
    }
    std::lock_guard<std::mutex> lock(g_graph_mu);
    GraphEntry& e = g_graphs[key];
    if (!e.exec) {
        // the control blocks outlive the process's batches (one set per graph)
        e.ctl.assign(groups.size(), nullptr);
        for (auto& c : e.ctl)
            if (hipMalloc((void**)&c, sizeof(BatchCtl)) != hipSuccess) {
                for (auto& x : e.ctl)
                    if (x) (void)hipFree(x);
                g_graphs.erase(key);
                set_error("launch_batch: control block allocation failed");
                return PCRL_ENOMEM;
            }
        // capture on a private stream (the caller's may be the legacy null
        // stream, which cannot be captured); the graph is launched on `s`
        hipStream_t cap = nullptr;
        PCRL_TRY_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (ce == hipSuccess) {
            if (stats) enqueue_bounces<true>(e.ctl.data(), groups, kmax, grid, cap, nullptr);
            else enqueue_bounces<false>(e.ctl.data(), groups, kmax, grid, cap, nullptr);
            ce = hipStreamEndCapture(cap, &g);
        }
        (void)hipStreamDestroy(cap);
        if (ce != hipSuccess) {
            set_error("launch_batch: graph capture failed: %s", hipGetErrorString(ce));
            return PCRL_EHIP;
        }
        const hipError_t ie = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            e.exec = nullptr;
            set_error("launch_batch: hipGraphInstantiate failed: %s", hipGetErrorString(ie));
            return PCRL_EHIP;
        }
    }
    for (size_t g = 0; g < groups.size(); ++g)
        PCRL_TRY_HIP(hipMemcpyAsync(e.ctl[g], &host_ctl[g], sizeof(BatchCtl), hipMemcpyHostToDevice, s));
    PCRL_TRY_HIP(hipGraphLaunch(e.exec, s));
    return PCRL_OK;
}

static int batch_impl(const PcrlQuery* q, int32_t n_q, const PcrlBatchParams* bp, hipStream_t s, PcrlLaunch** out) {
    for (int i = 0; i < n_q; ++i) out[i] = nullptr;
    auto shared = std::make_shared<BatchShared>();
    shared->bufs.stream = s;
    std::vector<TraceArgs> args((size_t)n_q);
    int kmax = 0;
    bool stats = false;
    bool timing = false;
    int rc = PCRL_OK;
    for (int i = 0; i < n_q && !rc; ++i) {
        rc = launch_prepare(q[i].scene, q[i].tx, q[i].n_tx, q[i].rx, q[i].n_rx, &q[i].params, s, false, &out[i],
                            &args[(size_t)i]);
        if (!rc) {
            kmax = std::max(kmax, q[i].params.max_reflections);
            stats |= (q[i].params.flags & PCRL_LAUNCH_STATS) != 0;
            timing |= (q[i].params.flags & PCRL_LAUNCH_TIMING) != 0;
            out[i]->shared = shared;
        } else {
            char msg[1100];
            snprintf(msg, sizeof msg, "launch_batch: query %d: %s", i, get_error());
            set_error("%s", msg);
        }
    }
    // query table ordered by kernel specialisation (levels, overlay); one group per run
    std::vector<BatchGroup> groups;
    std::vector<uint32_t> g_first, g_count;
    if (!rc) {
        std::vector<int> order((size_t)n_q);
        for (int i = 0; i < n_q; ++i) order[(size_t)i] = i;
        auto cls = [&](int i) { return args[(size_t)i].v.nlev * 2 + (args[(size_t)i].has_ov ? 1 : 0); };
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cls(x) < cls(y); });
        std::vector<TraceArgs> sorted((size_t)n_q);
        for (int k = 0; k < n_q; ++k) {
            const TraceArgs& a = args[(size_t)order[(size_t)k]];
            sorted[(size_t)k] = a;
            if (k == 0 || cls(order[(size_t)k]) != cls(order[(size_t)k - 1])) {
                groups.push_back(BatchGroup{a.v.nlev, a.has_ov != 0});
                g_first.push_back((uint32_t)k);
                g_count.push_back(0);
            }
            ++g_count.back();
        }
        args.swap(sorted);
    }
    const size_t n_g = groups.size();
    TraceArgs* qs = nullptr;
    uint32_t *tile_off = nullptr, *range = nullptr, *inpl = nullptr, *prev = nullptr;
    BatchCtl* ctl = nullptr;
    if (!rc) rc = shared->bufs.alloc(&qs, (size_t)n_q);
    if (!rc) rc = shared->bufs.alloc(&tile_off, (size_t)n_q + n_g);
    if (!rc) rc = shared->bufs.alloc(&range, (size_t)n_q);
    if (!rc) rc = shared->bufs.alloc(&inpl, (size_t)n_q);
    if (!rc) rc = shared->bufs.alloc(&prev, (size_t)n_q);
    if (!rc) rc = shared->bufs.alloc(&ctl, n_g);
    if (!rc) rc = fill_u32(inpl, 0u, n_q, s);
    if (!rc) rc = fill_u32(prev, 0u, n_q, s);
    if (!rc && hipMemcpyAsync(qs, args.data(), sizeof(TraceArgs) * (size_t)n_q, hipMemcpyHostToDevice, s) != hipSuccess) {
        set_error("launch_batch: query table upload failed");
        rc = PCRL_EHIP;
    }
    std::vector<BatchCtl> hc(n_g);
    for (size_t g = 0; g < n_g; ++g) {
        const uint32_t f = g_first[g];
        BatchCtl& c = hc[g];
        c.qs = qs + f;
        c.n_q = g_count[g];
        c.tile = (uint32_t)std::max(64, (bp->tile_rays / 64) * 64);
        c.theta = bp->compact_threshold;
        c.tile_off = tile_off + f + g;  // n_q + 1 entries per group
        c.range = range + f;
        c.in_place = inpl + f;
        c.prev_live = prev + f;
    }
    const int wpc = bp->waves_per_cu > 0 ? bp->waves_per_cu : 16;
    const unsigned grid = (unsigned)std::max(1, device_cus() * wpc / (TRACE_BLOCK / 64));
    if (!rc && timing) {
        shared->events.resize(2 * (kmax + 1));
        for (auto& e : shared->events)
            if (hipEventCreate(&e) != hipSuccess) rc = PCRL_EHIP;
        for (int i = 0; i < n_q && !rc; ++i) out[i]->events = shared->events;
    }
    if (!rc) {
        if (bp->use_graph && !timing) {
            rc = run_graph(hc, groups, kmax, grid, stats, s);
        } else {
            if (hipMemcpyAsync(ctl, hc.data(), sizeof(BatchCtl) * n_g, hipMemcpyHostToDevice, s) != hipSuccess) {
                set_error("launch_batch: control block upload failed");
                rc = PCRL_EHIP;
            } else {
                std::vector<BatchCtl*> dctl(n_g);
                for (size_t g = 0; g < n_g; ++g) dctl[g] = ctl + g;
                const std::vector<hipEvent_t>* ev = timing ? &shared->events : nullptr;
                if (stats) enqueue_bounces<true>(dctl.data(), groups, kmax, grid, s, ev);
                else enqueue_bounces<false>(dctl.data(), groups, kmax, grid, s, ev);
                if (hipGetLastError() != hipSuccess) {
                    set_error("launch_batch: kernel launch failed");
                    rc = PCRL_EHIP;
                }
            }
        }
    }
    if (rc) {
        for (int i = 0; i < n_q; ++i) {
            destroy_launch(out[i]);
            out[i] = nullptr;
        }
        return rc;
    }
    return PCRL_OK;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------

static std::mutex g_tune_mu;
static std::map<std::string, PcrlBatchParams> g_tuned;

// Scene class of a batch: number of voxel levels, log2 of the mean entries per
// scene and of the mean rays per query (the quantities that set the best tile
// size, occupancy and compaction policy).
static std::string batch_class(const PcrlQuery* q, int32_t n_q) {
    double pts = 0, rays = 0;
    int lev = 0;
    for (int i = 0; i < n_q; ++i) {
        pts += (double)q[i].scene->info.n_entries;
        rays += (double)q[i].params.n_rays * q[i].n_tx;
        lev = std::max(lev, q[i].scene->info.n_levels);
    }
    char key[96];
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    const char* name = hipGetDeviceProperties(&prop, dev) == hipSuccess ? prop.gcnArchName : "gpu";
    snprintf(key, sizeof key, "%s/L%d/e%d/r%d", name, lev, (int)std::lround(std::log2(std::max(1.0, pts / n_q))),
             (int)std::lround(std::log2(std::max(1.0, rays / n_q))));
    return key;
}

static int timed_batch(const PcrlQuery* q, int32_t n_q, const PcrlBatchParams& p, hipStream_t s, float* ms) {
    std::vector<PcrlLaunch*> L((size_t)n_q, nullptr);
    hipEvent_t e0, e1;
    PCRL_TRY_HIP(hipEventCreate(&e0));
    PCRL_TRY_HIP(hipEventCreate(&e1));
    PCRL_TRY_HIP(hipEventRecord(e0, s));
    int rc = batch_impl(q, n_q, &p, s, L.data());
    if (!rc) {
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(ms, e0, e1);
    }
    for (auto* x : L) destroy_launch(x);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

static int autotune_impl(const PcrlQuery* q, int32_t n_q, hipStream_t s, PcrlBatchParams* best) {
    // coordinate descent: occupancy, then tile size, then compaction threshold
    PcrlBatchParams p{};
    p.tile_rays = 1024;
    p.compact_threshold = 0.6f;
    p.waves_per_cu = 16;
    p.use_graph = 0;
    float best_ms = 1e30f, ms = 0.f;
    PCRL_TRY(timed_batch(q, n_q, p, s, &ms));  // warm-up
    const int waves[] = {8, 16, 32};
    const int tiles[] = {256, 1024, 4096};
    const float thetas[] = {0.0f, 0.6f, 2.0f};
    PcrlBatchParams cur = p;
    for (int w : waves) {
        PcrlBatchParams t = cur;
        t.waves_per_cu = w;
        PCRL_TRY(timed_batch(q, n_q, t, s, &ms));
        if (ms < best_ms) { best_ms = ms; p = t; }
    }
    cur = p;
    for (int ti : tiles) {
        PcrlBatchParams t = cur;
        t.tile_rays = ti;
        PCRL_TRY(timed_batch(q, n_q, t, s, &ms));
        if (ms < best_ms) { best_ms = ms; p = t; }
    }
    cur = p;
    for (float th : thetas) {
        PcrlBatchParams t = cur;
        t.compact_threshold = th;
        PCRL_TRY(timed_batch(q, n_q, t, s, &ms));
        if (ms < best_ms) { best_ms = ms; p = t; }
    }
    *best = p;
    return PCRL_OK;
}

}  // namespace pcrl

using namespace pcrl;

static int validate_batch(const PcrlQuery* q, int32_t n_q, PcrlLaunch** out, const char* fn) {
    if (!q || n_q < 1 || !out) {
        set_error("%s: need queries, n_q >= 1 and an output array", fn);
        return PCRL_EINVAL;
    }
    for (int i = 0; i < n_q; ++i) {
        if (!q[i].scene) {
            set_error("%s: query %d has no scene", fn, i);
            return PCRL_EINVAL;
        }
        if (q[i].params.flags & PCRL_LAUNCH_SDF) {
            set_error("%s: query %d asks for PCRL_LAUNCH_SDF, which only launch_rays runs", fn, i);
            return PCRL_EINVAL;
        }
    }
    return PCRL_OK;
}

extern "C" int batch_autotune(const PcrlQuery* queries, int32_t n_q, pcrl_stream_t stream, PcrlBatchParams* out) {
    clear_error();
    PcrlLaunch* dummy[1];
    PCRL_TRY(validate_batch(queries, n_q, dummy, "batch_autotune"));
    if (!out) {
        set_error("batch_autotune: out is NULL");
        return PCRL_EINVAL;
    }
    PcrlBatchParams best{};
    PCRL_TRY(autotune_impl(queries, n_q, (hipStream_t)stream, &best));
    best.use_graph = out->use_graph;
    best.autotune = 0;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[batch_class(queries, n_q)] = best;
    }
    *out = best;
    return PCRL_OK;
}

extern "C" int launch_batch(const PcrlQuery* queries, int32_t n_q, const PcrlBatchParams* params, pcrl_stream_t stream,
                            PcrlLaunch** out) {
    clear_error();
    PCRL_TRY(validate_batch(queries, n_q, out, "launch_batch"));
    PcrlBatchParams p{};
    if (params) p = *params;
    if (p.autotune) {
        const std::string key = batch_class(queries, n_q);
        bool found = false;
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            auto it = g_tuned.find(key);
            if (it != g_tuned.end()) {
                const int g = p.use_graph;
                p = it->second;
                p.use_graph = g;
                found = true;
            }
        }
        if (!found) {
            PcrlBatchParams t{};
            t.use_graph = p.use_graph;
            const int n_sample = std::min<int32_t>(n_q, 32);
            PCRL_TRY(batch_autotune(queries, n_sample, stream, &t));
            p = t;
        }
    }
    if (p.tile_rays <= 0) p.tile_rays = 1024;
    if (p.waves_per_cu <= 0) p.waves_per_cu = 16;
    if (!(p.compact_threshold >= 0.f)) p.compact_threshold = 0.6f;
    return batch_impl(queries, n_q, &p, (hipStream_t)stream, out);
}
