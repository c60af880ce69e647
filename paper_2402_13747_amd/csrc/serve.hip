// serve.hip -- a request loop over one device-resident, incrementally
// re-voxelised scene.
//
// TX/RX queries arrive at any time (serve_submit, host arrays).  A worker
// thread owns the GPU side:
//   * admission: a pending query starts once a stream is free, the number of
//     queries in flight is below max_inflight and its memory estimate fits
//     the device budget (queries larger than the whole budget are refused with
//     PCRL_EBUSY at submission);
//   * continuous batching: every admission round takes all admissible pending
//     queries onto a free stream, while earlier rounds are still running on
//     the other streams, so their work overlaps on the GPU; a round of small
//     queries shares one launch_batch, a round of large ones (>= 65536 rays
//     per query on average) launches them one by one (launch_rays);
//   * completion: when a round's event has fired its queries are deduplicated
//     (collect_paths) and copied to host memory; latency = completion time -
//     submission time.
// serve_update replaces the dynamic points (update_points): rounds admitted
// afterwards trace the new epoch, rounds in flight keep the one they started
// with.  Every query is traced by exactly the kernels of launch_rays, so its
// result is the same alone and in the mix.
#include "internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

namespace pcrl {

using clk = std::chrono::steady_clock;

// Mean rays per query from which a round launches its queries one by one.
constexpr int64_t SOLO_MIN_RAYS = 65536;

struct ServeReq {
    int64_t ticket = 0;
    std::vector<float> tx, rx;
    int32_t n_tx = 0, n_rx = 0;
    PcrlLaunchParams p{};
    int64_t bytes = 0;
    clk::time_point t_submit, t_admit, t_done;
    int status = 0;  // 0 pending, 1 running, 2 done, < 0 failed (PCRL status)
    bool cancel = false;  // serve_cancel while running: drop the result when the round retires
    int64_t epoch = 0;
    int32_t K = 0;
    // results, host
    int64_t n_rows = 0, n_keys = 0;
    std::vector<int32_t> tx_id, rx_id, n_refl, rank;
    std::vector<int64_t> key, count, ray;
    std::vector<float> len_poly, len_unf, points;
    std::string error;
};

struct Round {
    int stream = 0;
    std::vector<ServeReq*> reqs;
    std::vector<PcrlLaunch*> launches;
    float* d_tx = nullptr;  // device copies of the antennas of the round
    float* d_rx = nullptr;
    hipEvent_t done = nullptr;
    int64_t bytes = 0;
};

}  // namespace pcrl

struct PcrlServer {
    PcrlScene* scene = nullptr;
    PcrlServeParams prm{};
    int device = 0;
    std::vector<hipStream_t> streams;
    std::vector<bool> stream_busy;
    hipStream_t update_stream = nullptr;
    std::mutex mu;                 // queue, rounds, accounting, results
    std::condition_variable cv;
    std::mutex scene_mu;           // overlay swaps vs admissions
    std::deque<pcrl::ServeReq*> pending;
    std::map<int64_t, pcrl::ServeReq*> reqs;
    std::vector<pcrl::Round> rounds;
    int64_t next_ticket = 1;
    int64_t used_bytes = 0;
    int32_t inflight = 0;
    bool stop = false;
    std::thread worker;
    // statistics
    int64_t completed = 0, rays_done = 0, n_rounds = 0, queries_in_rounds = 0;
    std::vector<double> latencies_ms;
    pcrl::clk::time_point t_first, t_last;
    bool have_first = false;
};

namespace pcrl {

// Device bytes a served query holds while it is in flight, as the library
// allocates them (every block rounded up to its size class): its launch's
// buffers (history, records, counters, statistics, the ray state of even and
// of odd bounces, the Fibonacci directions; with PCRL_LAUNCH_COHERENT the
// bounce-0 order and its sort's counts, positions and starts, and, for a
// launch of 65536 rays or more run on its own, the order of the later
// bounces), plus its share of the round's antenna arrays and of the batch
// kernel's per-query words.  The collection of a finished query is left out:
// rounds collect one query at a time, for a moment, with O(records) bytes.
static int64_t query_device_bytes(int32_t n_tx, int32_t n_rx, const PcrlLaunchParams& p) {
    auto cls = [](int64_t b) { return (int64_t)size_class((size_t)std::max<int64_t>(b, 1)); };
    const int64_t nr = p.n_rays, rays = (int64_t)n_tx * nr, K = p.max_reflections;
    int64_t rec = p.record_capacity > 0 ? p.record_capacity
                                        : (n_rx == 0 ? 1 : rays * (K + 1) * std::min<int64_t>(n_rx, 8) / 16 + 65536);
    rec = std::min<int64_t>(rec, 0xFFFFFFF0ll);
    int64_t b = cls(rec * 16) + cls((K + 3) * 4);  // records, counters
    if (K > 0) b += cls(K * rays * 16);             // history
    if (p.flags & PCRL_LAUNCH_STATS) b += cls((int64_t)PCRL_NSTATS * (K + 1) * 8);
    if (K > 0) b += 2 * cls(rays * 16) + cls(rays * 4);
    if (K > 1) b += 2 * cls(rays * 16) + cls(rays * 4);
    b += cls(nr * 12);
    if (p.flags & PCRL_LAUNCH_COHERENT) {
        b += cls(nr * 2) + cls(nr * 4) + 2 * cls(65536 * 4) + cls(nr * 4);
        if (K > 0 && rays >= 65536) b += cls(rays * 4) + cls(rays * 2) + cls(rays * 4) + cls(K * 65536 * 4);
    }
    return b + (int64_t)n_tx * 12 + (int64_t)std::max<int32_t>(n_rx, 1) * 12 + 64;
}

// The arguments a served query may have (serve_submit's checks).
static bool served_params_ok(int32_t n_tx, int32_t n_rx, const PcrlLaunchParams* p) {
    return n_tx >= 1 && n_rx >= 0 && p && !p->directions && !p->hit_log_id && !p->hit_log_t && p->n_rays >= 1 &&
           p->max_reflections >= 0 && p->max_reflections <= PCRL_MAX_REFLECTIONS && !(p->flags & PCRL_LAUNCH_SDF);
}

static int collect_one(PcrlServer* S, PcrlLaunch* L, ServeReq* r, hipStream_t s) {
    const int K = r->K;
    int64_t cap = 1024;
    for (int attempt = 0; attempt < 3; ++attempt) {
        DevBufs B;
        B.stream = s;
        PcrlPaths P{};
        P.capacity = cap;
        int rc;
        if ((rc = B.alloc(&P.tx, cap)) || (rc = B.alloc(&P.rx, cap)) || (rc = B.alloc(&P.n_refl, cap)) ||
            (rc = B.alloc(&P.key, std::max<int64_t>(cap * K, 1))) || (rc = B.alloc(&P.count, cap)) ||
            (rc = B.alloc(&P.rank, cap)) || (rc = B.alloc(&P.ray, cap)) || (rc = B.alloc(&P.len_poly, cap)) ||
            (rc = B.alloc(&P.len_unf, cap)) || (rc = B.alloc(&P.points, std::max<int64_t>(cap * K * 3, 1)))) {
            B.release();
            return rc;
        }
        rc = collect_paths(L, S->prm.kappa > 0 ? S->prm.kappa : 1, S->prm.key_mode, &P, s);
        if (rc == PCRL_EOVERFLOW && P.n_rows > cap) {
            cap = P.n_rows;
            B.release();
            continue;
        }
        if (rc) {
            B.release();
            return rc;
        }
        const int64_t n = P.n_rows;
        r->n_rows = n;
        r->n_keys = P.n_keys;
        r->tx_id.resize(n); r->rx_id.resize(n); r->n_refl.resize(n); r->rank.resize(n);
        r->key.resize(n * K); r->count.resize(n); r->ray.resize(n);
        r->len_poly.resize(n); r->len_unf.resize(n); r->points.resize(n * K * 3);
        if (n) {
            hipMemcpyAsync(r->tx_id.data(), P.tx, n * 4, hipMemcpyDeviceToHost, s);
            hipMemcpyAsync(r->rx_id.data(), P.rx, n * 4, hipMemcpyDeviceToHost, s);
            hipMemcpyAsync(r->n_refl.data(), P.n_refl, n * 4, hipMemcpyDeviceToHost, s);
            hipMemcpyAsync(r->rank.data(), P.rank, n * 4, hipMemcpyDeviceToHost, s);
            if (K) hipMemcpyAsync(r->key.data(), P.key, n * K * 8, hipMemcpyDeviceToHost, s);
            hipMemcpyAsync(r->count.data(), P.count, n * 8, hipMemcpyDeviceToHost, s);
            hipMemcpyAsync(r->ray.data(), P.ray, n * 8, hipMemcpyDeviceToHost, s);
            hipMemcpyAsync(r->len_poly.data(), P.len_poly, n * 4, hipMemcpyDeviceToHost, s);
            hipMemcpyAsync(r->len_unf.data(), P.len_unf, n * 4, hipMemcpyDeviceToHost, s);
            if (K) hipMemcpyAsync(r->points.data(), P.points, n * K * 12, hipMemcpyDeviceToHost, s);
        }
        const hipError_t e = hipStreamSynchronize(s);
        B.release();
        if (e != hipSuccess) {
            set_error("serve: result copy failed: %s", hipGetErrorString(e));
            return PCRL_EHIP;
        }
        return PCRL_OK;
    }
    set_error("serve: row capacity retries exhausted");
    return PCRL_EOVERFLOW;
}

// Retire every finished round.  Called by the worker without S->mu held.
static void retire(PcrlServer* S) {
    std::vector<Round> done;
    {
        std::lock_guard<std::mutex> lock(S->mu);
        for (size_t i = 0; i < S->rounds.size();) {
            if (hipEventQuery(S->rounds[i].done) == hipSuccess) {
                done.push_back(S->rounds[i]);
                S->rounds.erase(S->rounds.begin() + (long)i);
            } else {
                ++i;
            }
        }
    }
    for (Round& R : done) {
        hipStream_t s = S->streams[(size_t)R.stream];
        for (size_t k = 0; k < R.reqs.size(); ++k) {
            ServeReq* r = R.reqs[k];
            bool cancelled = false;
            {
                std::lock_guard<std::mutex> lock(S->mu);
                cancelled = r->cancel;
            }
            // PCRL_EOVERFLOW here means the query's records exceeded its record
            // capacity; the message names the capacity to resubmit with
            int rc = PCRL_ECANCELED;
            if (!cancelled) rc = collect_one(S, R.launches[k], r, s);
            else set_error("serve: ticket %lld was cancelled", (long long)r->ticket);
            destroy_launch(R.launches[k]);
            const clk::time_point now = clk::now();
            std::lock_guard<std::mutex> lock(S->mu);
            r->t_done = now;
            if (rc == PCRL_OK) {
                r->status = 2;
                S->completed++;
                S->rays_done += (int64_t)r->n_tx * r->p.n_rays;
                S->latencies_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
                if (!S->have_first) {
                    S->t_first = r->t_admit;
                    S->have_first = true;
                }
                S->t_last = now;
            } else {
                r->status = rc;
                r->error = get_error();
            }
        }
        dfree(R.d_tx, s);
        dfree(R.d_rx, s);
        (void)hipEventDestroy(R.done);
        std::lock_guard<std::mutex> lock(S->mu);
        S->used_bytes -= R.bytes;
        S->inflight -= (int32_t)R.reqs.size();
        S->stream_busy[(size_t)R.stream] = false;
        S->cv.notify_all();
    }
}

// Start one round with every admissible pending query.  Returns true if a
// round was started.
static bool admit(PcrlServer* S) {
    Round R;
    {
        std::lock_guard<std::mutex> lock(S->mu);
        if (S->pending.empty()) return false;
        int free_stream = -1;
        for (size_t i = 0; i < S->streams.size(); ++i)
            if (!S->stream_busy[i]) {
                free_stream = (int)i;
                break;
            }
        if (free_stream < 0) return false;
        const int max_batch = S->prm.max_batch > 0 ? S->prm.max_batch : 64;
        while (!S->pending.empty() && (int)R.reqs.size() < max_batch) {
            ServeReq* r = S->pending.front();
            if (S->inflight + (int)R.reqs.size() >= S->prm.max_inflight) break;
            if (S->used_bytes + R.bytes + r->bytes > S->prm.hbm_budget_bytes) break;
            S->pending.pop_front();
            R.reqs.push_back(r);
            R.bytes += r->bytes;
        }
        if (R.reqs.empty()) return false;
        R.stream = free_stream;
        S->stream_busy[(size_t)free_stream] = true;
        S->used_bytes += R.bytes;
        S->inflight += (int32_t)R.reqs.size();
        S->n_rounds++;
        S->queries_in_rounds += (int64_t)R.reqs.size();
    }
    hipStream_t s = S->streams[(size_t)R.stream];
    // antennas of the round in one device buffer each
    int64_t ntx = 0, nrx = 0;
    for (ServeReq* r : R.reqs) {
        ntx += r->n_tx;
        nrx += r->n_rx;
    }
    std::vector<float> htx((size_t)ntx * 3), hrx((size_t)std::max<int64_t>(nrx, 1) * 3);
    std::vector<PcrlQuery> q(R.reqs.size());
    int rc = dalloc((void**)&R.d_tx, (size_t)ntx * 12, s);
    if (!rc) rc = dalloc((void**)&R.d_rx, (size_t)std::max<int64_t>(nrx, 1) * 12, s);
    int64_t otx = 0, orx = 0;
    for (size_t k = 0; k < R.reqs.size(); ++k) {
        ServeReq* r = R.reqs[k];
        std::memcpy(&htx[(size_t)otx * 3], r->tx.data(), r->tx.size() * 4);
        if (r->n_rx) std::memcpy(&hrx[(size_t)orx * 3], r->rx.data(), r->rx.size() * 4);
        q[k].scene = S->scene;
        q[k].tx = R.d_tx + otx * 3;
        q[k].n_tx = r->n_tx;
        q[k].rx = r->n_rx ? R.d_rx + orx * 3 : nullptr;
        q[k].n_rx = r->n_rx;
        q[k].params = r->p;
        otx += r->n_tx;
        orx += r->n_rx;
    }
    if (!rc && (hipMemcpyAsync(R.d_tx, htx.data(), htx.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
                hipMemcpyAsync(R.d_rx, hrx.data(), hrx.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess))
        rc = PCRL_EHIP;
    R.launches.assign(R.reqs.size(), nullptr);
    int64_t epoch = 0;
    if (!rc) {
        std::lock_guard<std::mutex> sl(S->scene_mu);
        epoch = S->scene->info.epoch;
        // Rounds of large queries launch each query on its own (the launch's
        // coherence order of later bounces pays off from 65536 rays on); rounds
        // of small ones share one persistent batch kernel per bounce.
        int64_t rays = 0;
        for (const PcrlQuery& x : q) rays += x.params.n_rays * x.n_tx;
        if (rays >= SOLO_MIN_RAYS * (int64_t)q.size()) {
            for (size_t k = 0; k < q.size() && !rc; ++k)
                rc = launch_rays(q[k].scene, q[k].tx, q[k].n_tx, q[k].rx, q[k].n_rx, &q[k].params, s,
                                 &R.launches[k]);
        } else {
            rc = launch_batch(q.data(), (int32_t)q.size(), &S->prm.batch, s, R.launches.data());
        }
    }
    if (!rc && hipEventCreateWithFlags(&R.done, hipEventDisableTiming) != hipSuccess) rc = PCRL_EHIP;
    if (!rc && hipEventRecord(R.done, s) != hipSuccess) rc = PCRL_EHIP;
    const clk::time_point now = clk::now();
    std::lock_guard<std::mutex> lock(S->mu);
    for (ServeReq* r : R.reqs) {
        r->t_admit = now;
        r->epoch = epoch;
        r->status = rc ? rc : 1;
        if (rc) r->error = get_error();
    }
    if (rc) {
        for (auto* L : R.launches) destroy_launch(L);
        (void)hipStreamSynchronize(s);
        dfree(R.d_tx, s);
        dfree(R.d_rx, s);
        if (R.done) (void)hipEventDestroy(R.done);
        S->used_bytes -= R.bytes;
        S->inflight -= (int32_t)R.reqs.size();
        S->stream_busy[(size_t)R.stream] = false;
        S->cv.notify_all();
        return true;
    }
    S->rounds.push_back(R);
    return true;
}

static void worker_main(PcrlServer* S) {
    (void)hipSetDevice(S->device);
    for (;;) {
        {
            std::lock_guard<std::mutex> lock(S->mu);
            if (S->stop && S->pending.empty() && S->rounds.empty()) break;
        }
        retire(S);
        bool started = admit(S);
        if (!started) {
            std::unique_lock<std::mutex> lock(S->mu);
            if (S->stop && S->pending.empty() && S->rounds.empty()) break;
            // wake on a new submission, or poll the running rounds' events
            S->cv.wait_for(lock, std::chrono::microseconds(S->rounds.empty() ? 2000 : 100));
        }
    }
}

}  // namespace pcrl

using namespace pcrl;

extern "C" int serve_create(PcrlScene* scene, const PcrlServeParams* params, PcrlServer** out) {
    clear_error();
    if (!scene || !params || !out) {
        set_error("serve_create: NULL argument");
        return PCRL_EINVAL;
    }
    *out = nullptr;
    PcrlServer* S = new (std::nothrow) PcrlServer();
    if (!S) {
        set_error("serve_create: host allocation failed");
        return PCRL_ENOMEM;
    }
    S->scene = scene;
    S->prm = *params;
    if (S->prm.n_streams <= 0) S->prm.n_streams = 4;
    if (S->prm.max_inflight <= 0) S->prm.max_inflight = 256;
    if (S->prm.hbm_budget_bytes <= 0) S->prm.hbm_budget_bytes = (int64_t)64 << 30;
    if (S->prm.kappa <= 0) S->prm.kappa = 1;
    (void)hipGetDevice(&S->device);
    for (int i = 0; i < S->prm.n_streams; ++i) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : S->streams) (void)hipStreamDestroy(x);
            delete S;
            set_error("serve_create: stream creation failed");
            return PCRL_EHIP;
        }
        S->streams.push_back(s);
        S->stream_busy.push_back(false);
    }
    if (hipStreamCreateWithFlags(&S->update_stream, hipStreamNonBlocking) != hipSuccess) {
        for (auto x : S->streams) (void)hipStreamDestroy(x);
        delete S;
        set_error("serve_create: stream creation failed");
        return PCRL_EHIP;
    }
    S->worker = std::thread(worker_main, S);
    *out = S;
    return PCRL_OK;
}

extern "C" int serve_query_bytes(int32_t n_tx, int32_t n_rx, const PcrlLaunchParams* p, int64_t* bytes) {
    clear_error();
    if (!bytes || !served_params_ok(n_tx, n_rx, p)) {
        set_error("serve_query_bytes: invalid arguments (n_tx >= 1, n_rx >= 0, the params of a served query)");
        return PCRL_EINVAL;
    }
    *bytes = query_device_bytes(n_tx, n_rx, *p);
    return PCRL_OK;
}

extern "C" int serve_submit(PcrlServer* S, const float* tx, int32_t n_tx, const float* rx, int32_t n_rx,
                            const PcrlLaunchParams* p, int64_t* ticket) {
    clear_error();
    if (!S || !tx || n_tx < 1 || n_rx < 0 || (n_rx > 0 && !rx) || !p || !ticket) {
        set_error("serve_submit: invalid arguments");
        return PCRL_EINVAL;
    }
    if (!served_params_ok(n_tx, n_rx, p)) {
        set_error("serve_submit: served queries use Fibonacci directions, surfels (no PCRL_LAUNCH_SDF), no hit logs, 0 <= K <= 8");
        return PCRL_EINVAL;
    }
    ServeReq* r = new (std::nothrow) ServeReq();
    if (!r) {
        set_error("serve_submit: host allocation failed");
        return PCRL_ENOMEM;
    }
    r->tx.assign(tx, tx + 3 * (size_t)n_tx);
    r->rx.assign(rx ? rx : tx, rx ? rx + 3 * (size_t)n_rx : tx);
    r->n_tx = n_tx;
    r->n_rx = n_rx;
    r->p = *p;
    r->p.flags &= ~PCRL_LAUNCH_TIMING;
    r->K = p->max_reflections;
    r->bytes = query_device_bytes(n_tx, n_rx, r->p);
    r->t_submit = clk::now();
    std::lock_guard<std::mutex> lock(S->mu);
    if (r->bytes > S->prm.hbm_budget_bytes) {
        const long long need = (long long)r->bytes;
        delete r;
        set_error("serve_submit: the query needs ~%lld bytes, more than the whole budget %lld", need,
                  (long long)S->prm.hbm_budget_bytes);
        return PCRL_EBUSY;
    }
    if (S->stop) {
        delete r;
        set_error("serve_submit: server is shutting down");
        return PCRL_EBUSY;
    }
    r->ticket = S->next_ticket++;
    S->reqs[r->ticket] = r;
    S->pending.push_back(r);
    *ticket = r->ticket;
    S->cv.notify_all();
    return PCRL_OK;
}

extern "C" int serve_update(PcrlServer* S, const uint32_t* ids, const float* xyz, const float* normal,
                            const uint32_t* label, int64_t n) {
    clear_error();
    if (!S) {
        set_error("serve_update: server is NULL");
        return PCRL_EINVAL;
    }
    std::lock_guard<std::mutex> sl(S->scene_mu);
    return update_points(S->scene, ids, xyz, normal, label, n, S->update_stream);
}

extern "C" int serve_poll(PcrlServer* S, int64_t ticket, double timeout_s, PcrlServeResult* out) {
    clear_error();
    if (!S || !out) {
        set_error("serve_poll: NULL argument");
        return PCRL_EINVAL;
    }
    std::unique_lock<std::mutex> lock(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("serve_poll: unknown ticket %lld", (long long)ticket);
        return PCRL_EINVAL;
    }
    ServeReq* r = it->second;
    if (timeout_s > 0)
        S->cv.wait_for(lock, std::chrono::duration<double>(timeout_s), [&] { return r->status == 2 || r->status < 0; });
    out->status = r->status;
    out->epoch = r->epoch;
    out->n_rows = r->n_rows;
    out->n_keys = r->n_keys;
    auto ms = [](clk::time_point a, clk::time_point b) { return std::chrono::duration<double, std::milli>(b - a).count(); };
    out->queue_ms = r->status >= 1 || r->status < 0 ? ms(r->t_submit, r->t_admit) : -1.0;
    out->latency_ms = r->status == 2 ? ms(r->t_submit, r->t_done) : -1.0;
    if (r->status < 0) {
        set_error("%s", r->error.c_str());
        return r->status;
    }
    return PCRL_OK;
}

extern "C" int serve_result(PcrlServer* S, int64_t ticket, PcrlPaths* out) {
    clear_error();
    if (!S || !out) {
        set_error("serve_result: NULL argument");
        return PCRL_EINVAL;
    }
    std::lock_guard<std::mutex> lock(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end() || it->second->status != 2) {
        set_error("serve_result: ticket %lld has no result (unknown or not finished)", (long long)ticket);
        return PCRL_EINVAL;
    }
    ServeReq* r = it->second;
    out->n_rows = r->n_rows;
    out->n_keys = r->n_keys;
    if (r->n_rows > out->capacity) {
        set_error("serve_result: %lld rows do not fit in %lld", (long long)r->n_rows, (long long)out->capacity);
        return PCRL_EOVERFLOW;
    }
    const size_t n = (size_t)r->n_rows, K = (size_t)r->K;
    if (out->tx) std::memcpy(out->tx, r->tx_id.data(), n * 4);
    if (out->rx) std::memcpy(out->rx, r->rx_id.data(), n * 4);
    if (out->n_refl) std::memcpy(out->n_refl, r->n_refl.data(), n * 4);
    if (out->key && K) std::memcpy(out->key, r->key.data(), n * K * 8);
    if (out->count) std::memcpy(out->count, r->count.data(), n * 8);
    if (out->rank) std::memcpy(out->rank, r->rank.data(), n * 4);
    if (out->ray) std::memcpy(out->ray, r->ray.data(), n * 8);
    if (out->len_poly) std::memcpy(out->len_poly, r->len_poly.data(), n * 4);
    if (out->len_unf) std::memcpy(out->len_unf, r->len_unf.data(), n * 4);
    if (out->points && K) std::memcpy(out->points, r->points.data(), n * K * 12);
    return PCRL_OK;
}

extern "C" int serve_cancel(PcrlServer* S, int64_t ticket) {
    clear_error();
    if (!S) {
        set_error("serve_cancel: NULL server");
        return PCRL_EINVAL;
    }
    std::lock_guard<std::mutex> lock(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) {
        set_error("serve_cancel: unknown ticket %lld", (long long)ticket);
        return PCRL_EINVAL;
    }
    ServeReq* r = it->second;
    if (r->status == 0) {
        // not admitted yet: leave the queue now
        for (auto q = S->pending.begin(); q != S->pending.end(); ++q)
            if (*q == r) {
                S->pending.erase(q);
                break;
            }
        r->status = PCRL_ECANCELED;
        r->error = "serve: ticket was cancelled before admission";
        r->t_admit = r->t_done = clk::now();
        S->cv.notify_all();
    } else if (r->status == 1) {
        r->cancel = true;  // its kernels finish; the result is not collected
    }
    return PCRL_OK;
}

extern "C" int serve_release(PcrlServer* S, int64_t ticket) {
    clear_error();
    if (!S) {
        set_error("serve_release: NULL server");
        return PCRL_EINVAL;
    }
    std::lock_guard<std::mutex> lock(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return PCRL_OK;
    if (it->second->status == 0 || it->second->status == 1) {
        set_error("serve_release: ticket %lld is still pending or running", (long long)ticket);
        return PCRL_EBUSY;
    }
    delete it->second;
    S->reqs.erase(it);
    return PCRL_OK;
}

extern "C" int serve_stats(PcrlServer* S, PcrlServeStats* out) {
    clear_error();
    if (!S || !out) {
        set_error("serve_stats: NULL argument");
        return PCRL_EINVAL;
    }
    std::lock_guard<std::mutex> lock(S->mu);
    std::memset(out, 0, sizeof *out);
    out->completed = S->completed;
    out->pending = (int64_t)S->pending.size();
    out->inflight = S->inflight;
    out->rounds = S->n_rounds;
    out->mean_batch = S->n_rounds ? (double)S->queries_in_rounds / (double)S->n_rounds : 0.0;
    out->rays = S->rays_done;
    std::vector<double> l = S->latencies_ms;
    if (!l.empty()) {
        std::sort(l.begin(), l.end());
        auto pct = [&](double q) { return l[(size_t)std::min<double>(l.size() - 1, std::floor(q * (l.size() - 1) + 0.5))]; };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->max_ms = l.back();
        double sum = 0;
        for (double x : l) sum += x;
        out->mean_ms = sum / (double)l.size();
    }
    if (S->have_first) {
        const double sec = std::chrono::duration<double>(S->t_last - S->t_first).count();
        out->rays_per_s = sec > 0 ? (double)S->rays_done / sec : 0.0;
    }
    out->used_bytes = S->used_bytes;
    return PCRL_OK;
}

extern "C" int serve_destroy(PcrlServer* S) {
    clear_error();
    if (!S) return PCRL_OK;
    {
        std::lock_guard<std::mutex> lock(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    for (auto& kv : S->reqs) delete kv.second;
    for (auto s : S->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    (void)hipStreamSynchronize(S->update_stream);
    (void)hipStreamDestroy(S->update_stream);
    delete S;
    return PCRL_OK;
}
