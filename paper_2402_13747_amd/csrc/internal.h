// internal.h -- shared declarations of the gfx950 coarse-path ray launcher.
//
// Device helpers (wave64 ballots and scans), the scene view that every
// kernel receives by value, the opaque PcrlScene / PcrlLaunch objects and
// the host-side primitives (allocation, scan, radix sort) shared by the
// translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "pcrl.h"

namespace pcrl {

// ---------------------------------------------------------------------------
// error state
// ---------------------------------------------------------------------------

void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();
const char* get_error();

#define PCRL_TRY_HIP(call)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            ::pcrl::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__,   \
                              __LINE__);                                                          \
            return e_ == hipErrorOutOfMemory ? PCRL_ENOMEM : PCRL_EHIP;                           \
        }                                                                                         \
    } while (0)

#define PCRL_TRY(call)              \
    do {                            \
        int s_ = (call);            \
        if (s_ != PCRL_OK) return s_; \
    } while (0)

// ---------------------------------------------------------------------------
// device memory: stream-ordered pool allocations
// ---------------------------------------------------------------------------

int dalloc(void** p, size_t bytes, hipStream_t s);
void dfree(void* p, hipStream_t s);

// While an ArenaScope lives on a thread, dalloc on that thread carves blocks
// out of the given device range (256-byte aligned, last in first out: a block
// is reclaimed once it and every block above it are freed) and never calls
// the runtime or a caller's allocator; dalloc fails with PCRL_ENOMEM when the
// range is exhausted.  read_back then copies without pinned staging memory.
// Blocks are handed out again in stream order, so every user of one arena
// must run on the stream of the scope's call.
struct Arena {
    static constexpr int kMaxBlocks = 64;
    char* base = nullptr;
    size_t cap = 0, top = 0, peak = 0;
    int n = 0;                        // live blocks, in allocation order
    size_t off[kMaxBlocks], end[kMaxBlocks];
    bool freed[kMaxBlocks];
};
struct ArenaScope {
    ArenaScope(void* base, size_t bytes);
    ~ArenaScope();
    size_t peak() const { return arena.peak; }   // most bytes in use at once
    ArenaScope(const ArenaScope&) = delete;
    ArenaScope& operator=(const ArenaScope&) = delete;
    Arena arena;
    Arena* prev;
};

// Owns a list of device allocations released together (stream ordered).
struct DevBufs {
    std::vector<void*> ptrs;
    hipStream_t stream = nullptr;
    template <typename T>
    int alloc(T** p, size_t count) {
        void* q = nullptr;
        int rc = dalloc(&q, count * sizeof(T), stream);
        if (rc != PCRL_OK) return rc;
        ptrs.push_back(q);
        *p = static_cast<T*>(q);
        return PCRL_OK;
    }
    void release() {
        for (void* q : ptrs) dfree(q, stream);
        ptrs.clear();
    }
};

// ---------------------------------------------------------------------------
// primitives (prims.hip)
// ---------------------------------------------------------------------------

// Exclusive prefix sum of n uint32 values (in may equal out).  If total is
// non-null the sum of all n values is written to *total (device).
int scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `bits` key bits.
// keys/vals are sorted in place (a temporary double buffer is used).
// vals may be null (keys only).
int radix_sort_u64(uint64_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s);
int radix_sort_u32(uint32_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s);
// The same on key bits [lo_bit, lo_bit + bits) only (lower bits ride along).
int radix_sort_u64_bits(uint64_t* keys, uint32_t* vals, int64_t n, int lo_bit, int bits, hipStream_t s);

// order[0 .. n) = the indices j < n of `keys` grouped by key (ascending
// buckets, any order inside a bucket: one counting pass with atomics), where
// n = min(*n_dev, n_max) when n_dev (device) is given, else n_max.
int bucket_order_u16(const uint16_t* keys, int64_t n_max, const uint32_t* n_dev, uint32_t* order, hipStream_t s);
// The second half of bucket_order_u16 when the 65536 bucket counts `cnt` and
// every item's position inside its bucket `pos` were produced elsewhere (with
// wave_bucket_add): scan the counts (into a temporary), then scatter.
int bucket_place_u16(const uint16_t* keys, const uint32_t* pos, int64_t n_max, const uint32_t* n_dev,
                     const uint32_t* cnt, uint32_t* order, hipStream_t s);

// Copy `bytes` from device memory to host memory and wait for the stream
// (used for the few sizes the host needs before it can continue).
int read_back(void* host, const void* dev, size_t bytes, hipStream_t s);

// Fill helpers.
int fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
int fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s);
int iota_u32(uint32_t* p, int64_t n, hipStream_t s);

// Bytes the device allocator reserves for a request of `bytes`: 512 B, then
// two size classes per power of two (1.5 * 2^e and 2^(e+1) for requests
// above 2^e; under 50 % slack).
size_t size_class(size_t bytes);

// Number of CUs of the current device (cached).
int device_cus();

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (uint64_t(1) << lane_id()) - 1;
}

// Inclusive wave64 scan.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off, 64);
        if ((int)lane_id() >= off) x += y;
    }
    return x;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Append `want` items per lane to a global list with one atomic per wave.
// Returns this lane's first slot (only meaningful where want != 0).
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, uint32_t want) {
    uint32_t incl = wave_incl_scan(want);
    uint32_t total = __shfl(incl, 63, 64);
    uint32_t base = 0;
    if (total) {
        if (lane_id() == 63) base = atomicAdd(counter, total);
        base = __shfl(base, 63, 64);
    }
    return base + incl - want;
}

// Add this lane's item to the count of its bucket with one atomic per
// distinct key of the wave (keys of neighbouring items often repeat); returns
// the item's position among the bucket's items added so far.  Every lane of
// the wave must call this.
__device__ __forceinline__ uint32_t wave_bucket_add(uint32_t* cnt, uint32_t key, bool valid) {
    const uint32_t lane = lane_id();
    const uint64_t lt = lanemask_lt();
    uint64_t todo = __ballot(valid);
    uint32_t pos = 0;
    while (todo) {
        const int l = __ffsll((long long)todo) - 1;
        const uint32_t k = __shfl(key, l, 64);
        const uint64_t m = __ballot(valid && key == k) & todo;
        uint32_t base = 0;
        if ((int)lane == l) base = atomicAdd(&cnt[k], (uint32_t)__popcll(m));
        base = __shfl(base, l, 64);
        if ((m >> lane) & 1ull) pos = base + (uint32_t)__popcll(m & lt);
        todo &= ~m;
    }
    return pos;
}

__device__ __forceinline__ float as_float(uint32_t u) { return __uint_as_float(u); }
__device__ __forceinline__ uint32_t as_uint(float f) { return __float_as_uint(f); }

// ---------------------------------------------------------------------------
// scene view: everything a traversal kernel needs, passed by value
// ---------------------------------------------------------------------------

struct SceneView {
    float org[3];          // grid origin
    float hi[3];           // grid far corner (org + dims * h)
    float h;               // leaf edge
    float inv_h;
    float rs2;             // r_s^2
    float t_eps;
    float r_s;
    float pad;             // rounding margin added to every disk's leaf box
    int32_t key_bits;      // bits of the hierarchical leaf key
    int32_t dim[3];        // leaf grid dims
    int32_t dim0[3];       // level-0 grid dims
    int32_t nlev;
    int32_t span[PCRL_MAX_LEVELS];   // leaves per cell edge at level i (span[nlev-1] = 1)
    int32_t ratio[PCRL_MAX_LEVELS];  // span[i] / span[i+1]
    int32_t lbits[PCRL_MAX_LEVELS];  // key bits of level i (level 0: linear coarse index)
    int32_t nw[PCRL_MAX_LEVELS];     // 64-bit mask words of a level-i brick (i < nlev-1)
    uint32_t nn[PCRL_MAX_LEVELS];    // occupied nodes per level (bounds of every index)
    uint64_t mspan[PCRL_MAX_LEVELS]; // ceil(2^40 / span[i]): x / span[i] == (x * mspan[i]) >> 40 for x < 2^22
    const int32_t* map0;             // [dim0 x*y*z] level-0 node or -1
    const uint64_t* mask[PCRL_MAX_LEVELS - 1];  // child occupancy bricks of level i
    const uint32_t* base[PCRL_MAX_LEVELS - 1];  // child index of the first set bit of each word
    const uint32_t* baabb[PCRL_MAX_LEVELS - 1]; // null, or per node of level i the box of its occupied
                                                // children (local coordinates, 5 bits each: lo x, y, z,
                                                // then hi x, y, z; ratio <= 32)
    const uint2* leaf;               // per leaf: (first entry, entry count)
    const uint8_t* ldist;            // null, or per leaf cell of each parent brick its empty-space skip radius
    const uint8_t* dist0;            // null, or per level-0 cell its empty-space skip radius (level-0 cells)
    const uint2* cells;              // null, or per leaf cell of every parent brick: (first entry, count) of
                                     // an occupied leaf, or (skip radius, 0) of an empty one
    const float4* spos;              // per entry: x, y, z, point id (bits)
    const float4* snrm;              // per entry: unit normal, label (bits)
};

// x / span for 0 <= x < 2^22 and span <= 2^18 with a precomputed ceil(2^40 / span):
// x * m / 2^40 = x / span + x * e / 2^40 with 0 <= e < 1, and x * e / 2^40 < 1 / span,
// so the floor is exact.
__host__ __device__ __forceinline__ int span_div(int x, uint64_t m) {
    return (int)(((uint64_t)(uint32_t)x * m) >> 40);
}

__host__ __device__ inline uint64_t leaf_key_of(const SceneView& v, int ix, int iy, int iz) {
    const int s0 = v.span[0];
    uint64_t k = (uint64_t)((ix / s0) + v.dim0[0] * ((iy / s0) + v.dim0[1] * (iz / s0)));
    for (int i = 1; i < v.nlev; ++i) {
        const int s = v.span[i];
        const int r = v.ratio[i - 1];
        const int lx = (ix / s) % r, ly = (iy / s) % r, lz = (iz / s) % r;
        k = (k << v.lbits[i]) | (uint64_t)(lx + r * (ly + r * lz));
    }
    return k;
}

}  // namespace pcrl

// ---------------------------------------------------------------------------
// opaque objects
// ---------------------------------------------------------------------------

namespace pcrl {
// Dynamic points of one epoch, voxelised on the base scene's frame.  Held by
// the scene until the next update and by every launch that traced it.
struct Overlay {
    SceneView view{};
    DevBufs bufs;
    int64_t n_points = 0;
    int64_t n_entries = 0;
    int64_t bytes = 0;
    uint32_t max_label = 0;
    int64_t epoch = 0;
    // The stream the overlay was built on may be gone by now (a server's
    // update stream), so free on the null stream.  Nothing uses the overlay
    // any more: every launch that held it synchronised before letting go.
    ~Overlay() {
        bufs.stream = nullptr;
        bufs.release();
    }
};
}  // namespace pcrl

struct PcrlScene {
    int device = 0;
    pcrl::SceneView view{};           // static base hierarchy
    pcrl::DevBufs bufs;
    PcrlSceneInfo info{};
    uint64_t* leaf_key = nullptr;     // per leaf hierarchical key
    uint32_t* entry_point = nullptr;  // per entry: point id (leaf order); null: read from spos.w
    uint2* leaf_range = nullptr;
    uint32_t max_label = 0;
    bool compact = false;             // PCRL_VOXEL_COMPACT: no dense cell tables (base and overlays)
    std::shared_ptr<pcrl::Overlay> overlay;  // current epoch of dynamic points (may be null)
    // own-point index of the implicit-surface intersection (sdf_intersect), built
    // on first use: every point once, in the leaf holding its centre, in leaf order
    std::mutex own_mu;
    uint32_t* own_scan = nullptr;     // [n_entries + 1] own entries before each entry
    float4* own_pos = nullptr;        // [n_points] positions (w: point id bits)
    float4* own_nrm = nullptr;        // [n_points] unit normals (w: label bits)
};

struct PcrlLaunch {
    const PcrlScene* scene = nullptr;
    hipStream_t stream = nullptr;
    pcrl::DevBufs bufs;
    int64_t n_rays = 0, n_total = 0;
    int32_t n_tx = 0, n_rx = 0, K = 0;
    int32_t flags = 0;
    float sigma = 1.25f, alpha = 0.f;
    int64_t rec_cap = 0;
    std::shared_ptr<pcrl::Overlay> overlay;  // epoch of dynamic points this launch traced
    uint32_t max_label = 0;         // largest label of base and overlay
    float4* hist = nullptr;         // [K][n_total]: interaction point, label (bits)
    uint4* rec = nullptr;           // [rec_cap]: ray, rx | b << 16, len_poly, len_unf
    uint32_t* counters = nullptr;   // [0..K+1] active rays per bounce, [K+2] records
    unsigned long long* stats = nullptr;  // [K+1][PCRL_NSTATS] device counters (PCRL_LAUNCH_STATS)
    std::vector<hipEvent_t> events; // 2 per bounce (PCRL_LAUNCH_TIMING)
    bool owns_events = false;       // false: events belong to a batch (shared)
    std::shared_ptr<void> shared;   // batch-level state kept alive by every query of a batch
};

// counters layout
#define PCRL_CNT_REC(K) ((K) + 2)
#define PCRL_NCOUNTERS(K) ((K) + 3)
#define PCRL_NSTATS 16  // device statistics slots of a launch (PCRL_LAUNCH_STATS)

// internal entry points of the launch translation unit (used by batching)
namespace pcrl {
struct TraceArgs;
int launch_prepare(const PcrlScene* scene, const float* tx, int32_t n_tx, const float* rx, int32_t n_rx,
                   const PcrlLaunchParams* p, hipStream_t s, bool timing_events, PcrlLaunch** out, TraceArgs* args);
void destroy_launch(PcrlLaunch* L);
// Every static point once, in the leaf that holds its centre (built on first
// use and kept with the scene; sdf.hip): scene->own_pos / own_nrm.
int scene_own_index(PcrlScene* S, hipStream_t s);
}
