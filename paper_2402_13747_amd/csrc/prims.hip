// prims.hip -- allocation, error state, prefix scan and LSD radix sort for gfx950.
//
// The radix sort is the voxel build's dominant step (sorting (leaf key,
// point id) pairs) and also orders reception records for deduplication.
// Design: one wave64 per block; each block owns a tile of ITEMS x 64 keys.
//   pass = hist (LDS histogram per tile, digit-major output)
//        -> exclusive scan over [digit][tile]
//        -> scatter (stable in-tile rank from 8 ballots per key, running
//           per-digit offsets in LDS).
// Stability across tiles follows from the digit-major scan order; within a
// tile keys are ranked in input order, so the whole sort is stable.
#include "internal.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace pcrl {

// ---------------------------------------------------------------------------
// error state
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

const char* get_error() { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// allocation: a caching device allocator
// ---------------------------------------------------------------------------
//
// Freeing through the runtime's stream-ordered pool costs tens of
// microseconds of host time per call, and one build + launch + collect frees
// about eighty buffers.  Freed blocks are kept instead, per device and size
// class, and handed out again:
//   * to an allocation on the stream that freed the block at once (stream
//     order keeps the old and the new user apart);
//   * to an allocation on another stream once an event recorded at the free
//     has completed.
// Size classes are 512 B, then two per power of two: a request above 2^e
// and at most 2^(e+1) bytes gets 1.5 * 2^e or 2^(e+1) (under 50 % slack).  Cached blocks are returned to the runtime when an allocation
// fails, then the allocation is retried once.

size_t size_class(size_t bytes) {
    if (bytes <= 512) return 512;
    int e = 63 - __builtin_clzll((unsigned long long)(bytes - 1));  // 2^e < bytes <= 2^(e+1)
    const size_t q = (size_t)1 << (e - 1);                           // quarter of 2^(e+1)
    return (bytes + q - 1) / q * q;
}

namespace {

struct FreeBlock {
    void* p;
    hipStream_t stream;
    hipEvent_t ev;
};

struct Pool {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<FreeBlock>> free_;  // (device, class) -> blocks
    std::unordered_map<void*, std::pair<int, size_t>> live;         // block -> (device, class)
    std::map<int, std::vector<hipEvent_t>> events;                   // spare events per device
};

Pool& pool() {
    static Pool* p = new Pool();  // never destroyed: blocks live until the process ends
    return *p;
}

// Return every cached block whose last use has completed to the runtime.
void trim_locked(Pool& P) {
    for (auto& kv : P.free_) {
        auto& v = kv.second;
        for (size_t i = 0; i < v.size();) {
            if (hipEventQuery(v[i].ev) == hipSuccess) {
                (void)hipFree(v[i].p);
                P.events[kv.first.first].push_back(v[i].ev);
                v[i] = v.back();
                v.pop_back();
            } else {
                ++i;
            }
        }
    }
}

}  // namespace

// A caller's allocator (set_allocator) replaces the pool for new blocks;
// every block remembers the allocator that made it, so switching is safe
// while blocks are alive.  The callbacks run with no lock of the library
// held (they may re-enter it, e.g. a framework's collector releasing a
// scene).
namespace {
struct UserAlloc {
    std::mutex mu;
    PcrlAllocator a{};
    bool on = false;
    std::unordered_map<void*, PcrlAllocator> live;
};
UserAlloc& user_alloc() {
    static UserAlloc* u = new UserAlloc();
    return *u;
}
}  // namespace

namespace {
thread_local Arena* t_arena = nullptr;

int arena_alloc(Arena& A, void** p, size_t bytes) {
    const size_t off = (A.top + 255) & ~(size_t)255;
    const size_t want = bytes == 0 ? 1 : bytes;
    if (A.n == Arena::kMaxBlocks) {
        set_error("scratch memory: more than %d blocks in use at once", Arena::kMaxBlocks);
        return PCRL_ENOMEM;
    }
    if (off > A.cap || want > A.cap - off) {
        set_error("scratch memory exhausted: %zu more bytes needed at offset %zu of %zu", want, off, A.cap);
        return PCRL_ENOMEM;
    }
    A.off[A.n] = off;
    A.end[A.n] = off + want;
    A.freed[A.n] = false;
    ++A.n;
    A.top = off + want;
    A.peak = std::max(A.peak, A.top);
    *p = A.base + off;
    return PCRL_OK;
}

bool arena_free(Arena& A, void* p) {
    char* c = static_cast<char*>(p);
    if (c < A.base || c >= A.base + A.cap) return false;
    const size_t off = (size_t)(c - A.base);
    for (int i = A.n; i-- > 0;) {
        if (A.off[i] == off && !A.freed[i]) {
            A.freed[i] = true;
            break;
        }
    }
    while (A.n > 0 && A.freed[A.n - 1]) --A.n;
    A.top = A.n ? A.end[A.n - 1] : 0;
    return true;
}
}  // namespace

ArenaScope::ArenaScope(void* base, size_t bytes) : prev(t_arena) {
    arena.base = static_cast<char*>(base);
    arena.cap = bytes;
    t_arena = &arena;
}

ArenaScope::~ArenaScope() { t_arena = prev; }

int dalloc(void** p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    if (t_arena) return arena_alloc(*t_arena, p, bytes);
    int dev = 0;
    (void)hipGetDevice(&dev);
    const size_t cls = size_class(bytes == 0 ? 1 : bytes);
    UserAlloc& U = user_alloc();
    PcrlAllocator ua{};
    bool use_user = false;
    {
        std::lock_guard<std::mutex> lock(U.mu);
        use_user = U.on;
        ua = U.a;
    }
    if (use_user) {
        void* q = ua.alloc(cls, (pcrl_stream_t)s, ua.ctx);
        if (!q) {
            set_error("device allocation of %zu bytes failed in the caller's allocator", bytes);
            return PCRL_ENOMEM;
        }
        std::lock_guard<std::mutex> lock(U.mu);
        U.live[q] = ua;
        *p = q;
        return PCRL_OK;
    }
    Pool& P = pool();
    std::lock_guard<std::mutex> lock(P.mu);
    auto it = P.free_.find({dev, cls});
    if (it != P.free_.end()) {
        auto& v = it->second;
        for (size_t i = v.size(); i-- > 0;) {
            if (v[i].stream == s || hipEventQuery(v[i].ev) == hipSuccess) {
                *p = v[i].p;
                P.events[dev].push_back(v[i].ev);
                v[i] = v.back();
                v.pop_back();
                P.live[*p] = {dev, cls};
                return PCRL_OK;
            }
        }
    }
    hipError_t e = hipMalloc(p, cls);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        trim_locked(P);
        e = hipMalloc(p, cls);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        *p = nullptr;
        return e == hipErrorOutOfMemory ? PCRL_ENOMEM : PCRL_EHIP;
    }
    P.live[*p] = {dev, cls};
    return PCRL_OK;
}

void dfree(void* p, hipStream_t s) {
    if (!p) return;
    if (t_arena && arena_free(*t_arena, p)) return;
    {
        UserAlloc& U = user_alloc();
        PcrlAllocator ua{};
        bool found = false;
        {
            std::lock_guard<std::mutex> lock(U.mu);
            auto u = U.live.find(p);
            if (u != U.live.end()) {
                ua = u->second;
                U.live.erase(u);
                found = true;
            }
        }
        if (found) {
            ua.free(p, (pcrl_stream_t)s, ua.ctx);
            return;
        }
    }
    Pool& P = pool();
    std::lock_guard<std::mutex> lock(P.mu);
    auto it = P.live.find(p);
    if (it == P.live.end()) return;  // not ours
    const int dev = it->second.first;
    const size_t cls = it->second.second;
    P.live.erase(it);
    hipEvent_t ev = nullptr;
    auto& spare = P.events[dev];
    if (!spare.empty()) {
        ev = spare.back();
        spare.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);  // no event: make the block safe for any stream now
        (void)hipFree(p);
        return;
    }
    if (hipEventRecord(ev, s) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        (void)hipEventRecord(ev, nullptr);
    }
    P.free_[{dev, cls}].push_back(FreeBlock{p, s, ev});
}

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_iota(uint32_t* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = (uint32_t)i;
}

static unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    int64_t cap = (int64_t)device_cus() * 16;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

int fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return PCRL_OK;
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    PCRL_TRY_HIP(hipGetLastError());
    return PCRL_OK;
}

int fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return PCRL_OK;
    hipLaunchKernelGGL(k_fill<uint64_t>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    PCRL_TRY_HIP(hipGetLastError());
    return PCRL_OK;
}

int iota_u32(uint32_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return PCRL_OK;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
    PCRL_TRY_HIP(hipGetLastError());
    return PCRL_OK;
}

// ---------------------------------------------------------------------------
// exclusive scan (reduce -> scan of tile sums -> apply)
// ---------------------------------------------------------------------------

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;  // 4096 values per block

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* total) {
    __shared__ uint32_t wsum[SCAN_BLOCK / 64];
    const int w = threadIdx.x >> 6;
    uint32_t incl = wave_incl_scan(x);
    if (lane_id() == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_BLOCK / 64; ++k) {
        uint32_t v = wsum[k];
        off += (k < w) ? v : 0u;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return off + incl - x;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const uint32_t* in, int64_t n, uint32_t* sums) {
    const int64_t tile = (int64_t)blockIdx.x * SCAN_TILE;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = tile + (int64_t)k * SCAN_BLOCK + threadIdx.x;
        if (i < n) acc += in[i];
    }
    uint32_t tot;
    (void)block_excl_scan(acc, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Each thread owns SCAN_ITEMS consecutive values of the tile, moved as
// 16-byte vectors when VEC (both arrays 16-byte aligned) and the thread's
// values lie inside the array.
template <bool VEC>
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const uint32_t* in, uint32_t* out, int64_t n,
                                                           const uint32_t* offs, uint32_t* total) {
    const int64_t tile = (int64_t)blockIdx.x * SCAN_TILE;
    const int64_t first = tile + (int64_t)threadIdx.x * SCAN_ITEMS;
    const bool whole = VEC && first + SCAN_ITEMS <= n;
    uint32_t v[SCAN_ITEMS];
    uint32_t acc = 0;
    if (whole) {
        const uint4* q = reinterpret_cast<const uint4*>(in + first);
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS / 4; ++k) {
            const uint4 u = q[k];
            v[4 * k] = u.x;
            v[4 * k + 1] = u.y;
            v[4 * k + 2] = u.z;
            v[4 * k + 3] = u.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            int64_t i = first + k;
            v[k] = (i < n) ? in[i] : 0u;
        }
    }
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) acc += v[k];
    uint32_t tot;
    uint32_t run = block_excl_scan(acc, &tot) + (offs ? offs[blockIdx.x] : 0u);
    uint32_t r[SCAN_ITEMS];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        r[k] = run;
        run += v[k];
    }
    if (whole) {
        uint4* q = reinterpret_cast<uint4*>(out + first);
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS / 4; ++k) q[k] = make_uint4(r[4 * k], r[4 * k + 1], r[4 * k + 2], r[4 * k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            int64_t i = first + k;
            if (i < n) out[i] = r[k];
        }
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BLOCK - 1) *total = run;
}

static void launch_scan_apply(unsigned grid, const uint32_t* in, uint32_t* out, int64_t n, const uint32_t* offs,
                              uint32_t* total, hipStream_t s) {
    const bool vec = (((uintptr_t)in | (uintptr_t)out) & 15u) == 0;
    if (vec) hipLaunchKernelGGL(k_scan_apply<true>, dim3(grid), dim3(SCAN_BLOCK), 0, s, in, out, n, offs, total);
    else hipLaunchKernelGGL(k_scan_apply<false>, dim3(grid), dim3(SCAN_BLOCK), 0, s, in, out, n, offs, total);
}

int scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, hipStream_t s) {
    if (n <= 0) {
        if (total) PCRL_TRY(fill_u32(total, 0u, 1, s));
        return PCRL_OK;
    }
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        launch_scan_apply(1, in, out, n, nullptr, total, s);
        PCRL_TRY_HIP(hipGetLastError());
        return PCRL_OK;
    }
    uint32_t* sums = nullptr;
    PCRL_TRY(dalloc((void**)&sums, (size_t)nb * sizeof(uint32_t), s));
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, sums);
    int rc = hipGetLastError() == hipSuccess ? PCRL_OK : PCRL_EHIP;
    if (rc == PCRL_OK) rc = scan_u32(sums, sums, nb, nullptr, s);
    if (rc == PCRL_OK) {
        launch_scan_apply((unsigned)nb, in, out, n, sums, total, s);
        if (hipGetLastError() != hipSuccess) rc = PCRL_EHIP;
    }
    dfree(sums, s);
    if (rc == PCRL_EHIP) set_error("scan kernel launch failed");
    return rc;
}

// ---------------------------------------------------------------------------
// LSD radix sort, 8-bit digits
// ---------------------------------------------------------------------------

// Digits of DB bits (4..8): a sort of `bits` key bits takes ceil(bits / 8)
// passes, with the digit width spread evenly over them (fewer digits mean
// longer runs per digit in a tile: better-coalesced scatter writes).
constexpr int SORT_WAVE = 64;
constexpr int SORT_ITEMS = 32;
constexpr int SORT_TILE = SORT_WAVE * SORT_ITEMS;  // 2048 keys per one-wave block

template <typename K, int DB>
__global__ __launch_bounds__(SORT_WAVE) void k_radix_hist(const K* keys, int64_t n, int shift, uint32_t* hist,
                                                          uint32_t n_tiles) {
    constexpr int R = 1 << DB;
    __shared__ uint32_t h[R];
    for (int d = threadIdx.x; d < R; d += SORT_WAVE) h[d] = 0;
    const int64_t tile = (int64_t)blockIdx.x * SORT_TILE;
    // all of the lane's loads first (one memory round trip per tile)
    K kr[SORT_ITEMS];
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k) {
        const int64_t i = tile + (int64_t)k * SORT_WAVE + threadIdx.x;
        kr[k] = i < n ? keys[i] : K(0);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k) {
        const int64_t i = tile + (int64_t)k * SORT_WAVE + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(kr[k] >> shift) & (R - 1)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < R; d += SORT_WAVE) hist[(size_t)d * n_tiles + blockIdx.x] = h[d];
}

// One tile of one pass: the keys are ranked stably by digit into LDS (digit
// by digit, input order within a digit), then copied out in that order, so
// that consecutive lanes write consecutive addresses of one digit's run.
// offs is the exclusive scan of the histogram in [digit][tile] order: cell
// (d, t) starts at offs[d n_tiles + t] and ends where the next cell starts
// (the last cell at n).  V: values move with the keys.
template <typename K, int DB, bool V>
__global__ __launch_bounds__(SORT_WAVE) void k_radix_scatter(const K* keys_in, const uint32_t* vals_in, K* keys_out,
                                                             uint32_t* vals_out, int64_t n, int shift,
                                                             const uint32_t* offs, uint32_t n_tiles) {
    constexpr int R = 1 << DB;
    constexpr int PER = (R + SORT_WAVE - 1) / SORT_WAVE;
    __shared__ uint32_t gstart[R], lstart[R], lrun[R];
    __shared__ K skey[SORT_TILE];
    __shared__ uint32_t sval[V ? SORT_TILE : 1];
    const uint32_t lane = lane_id();
    const int64_t tile = (int64_t)blockIdx.x * SORT_TILE;
    const uint32_t tn = (uint32_t)min((int64_t)SORT_TILE, n - tile);
    // all of the lane's loads first (one memory round trip per tile)
    K kr[SORT_ITEMS];
    uint32_t vr[V ? SORT_ITEMS : 1];
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k) {
        const int64_t i = tile + (int64_t)k * SORT_WAVE + lane;
        kr[k] = i < n ? keys_in[i] : K(0);
        if (V) vr[k] = i < n ? vals_in[i] : 0u;
    }
    const size_t cells = (size_t)R * n_tiles;
    for (int d = lane; d < R; d += SORT_WAVE) {
        const size_t c = (size_t)d * n_tiles + blockIdx.x;
        const uint32_t a = offs[c];
        gstart[d] = a;
        lrun[d] = (c + 1 < cells ? offs[c + 1] : (uint32_t)n) - a;  // the tile's count of digit d
    }
    __syncthreads();
    {
        // tile-local start of every digit: exclusive scan of the counts (PER consecutive digits per lane)
        uint32_t cnt[PER], sum = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int d = (int)lane * PER + j;
            cnt[j] = d < R ? lrun[d] : 0u;
            sum += cnt[j];
        }
        uint32_t run = wave_incl_scan(sum) - sum;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int d = (int)lane * PER + j;
            if (d < R) {
                lstart[d] = run;
                lrun[d] = 0u;
            }
            run += cnt[j];
        }
    }
    __syncthreads();
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int k = 0; k < SORT_ITEMS; ++k) {
        const uint32_t i = (uint32_t)k * SORT_WAVE + lane;
        const bool valid = i < tn;
        const uint32_t digit = (uint32_t)(kr[k] >> shift) & (R - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < DB; ++b) {
            const bool bit = (digit >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lt);
        uint32_t pos = 0;
        if (valid) pos = lstart[digit] + lrun[digit] + rank;
        __syncthreads();
        // the highest lane of each digit group advances the digit's running count
        if (valid && (peers >> lane) == 1ull) lrun[digit] += rank + 1;
        if (valid) {
            skey[pos] = kr[k];
            if (V) sval[pos] = vr[k];
        }
        __syncthreads();
    }
    for (uint32_t j = lane; j < tn; j += SORT_WAVE) {
        const K key = skey[j];
        const uint32_t d = (uint32_t)(key >> shift) & (R - 1);
        const uint32_t g = gstart[d] + (j - lstart[d]);
        keys_out[g] = key;
        if (V) vals_out[g] = sval[j];
    }
}

template <typename K, int DB>
static int radix_pass(const K* ka, const uint32_t* va, K* kb, uint32_t* vb, int64_t n, int shift, uint32_t* hist,
                      uint32_t n_tiles, hipStream_t s) {
    hipLaunchKernelGGL((k_radix_hist<K, DB>), dim3(n_tiles), dim3(SORT_WAVE), 0, s, ka, n, shift, hist, n_tiles);
    if (hipGetLastError() != hipSuccess) return PCRL_EHIP;
    PCRL_TRY(scan_u32(hist, hist, ((int64_t)1 << DB) * n_tiles, nullptr, s));
    if (va)
        hipLaunchKernelGGL((k_radix_scatter<K, DB, true>), dim3(n_tiles), dim3(SORT_WAVE), 0, s, ka, va, kb, vb, n, shift,
                           hist, n_tiles);
    else
        hipLaunchKernelGGL((k_radix_scatter<K, DB, false>), dim3(n_tiles), dim3(SORT_WAVE), 0, s, ka, va, kb, vb, n,
                           shift, hist, n_tiles);
    return hipGetLastError() == hipSuccess ? PCRL_OK : PCRL_EHIP;
}

template <typename K>
static int radix_sort_impl(K* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s, int lo_bit = 0) {
    if (n <= 1 || bits <= 0) return PCRL_OK;
    if (n > (int64_t)0xFFFFFFF0ll) {
        set_error("radix sort of %lld items exceeds the 32-bit index range", (long long)n);
        return PCRL_EINVAL;
    }
    const int64_t n_tiles64 = (n + SORT_TILE - 1) / SORT_TILE;
    const uint32_t n_tiles = (uint32_t)n_tiles64;
    const int passes = (bits + 7) / 8;
    const int db = std::max(4, (bits + passes - 1) / passes);  // 4..8
    K* k2 = nullptr;
    uint32_t* v2 = nullptr;
    uint32_t* hist = nullptr;
    int rc = dalloc((void**)&k2, (size_t)n * sizeof(K), s);
    if (rc == PCRL_OK && vals) rc = dalloc((void**)&v2, (size_t)n * sizeof(uint32_t), s);
    if (rc == PCRL_OK) rc = dalloc((void**)&hist, ((size_t)1 << db) * n_tiles * sizeof(uint32_t), s);
    K* ka = keys;
    K* kb = k2;
    uint32_t* va = vals;
    uint32_t* vb = v2;
    for (int p = 0; p < passes && rc == PCRL_OK; ++p) {
        const int shift = lo_bit + p * db;
        switch (db) {
        case 4: rc = radix_pass<K, 4>(ka, va, kb, vb, n, shift, hist, n_tiles, s); break;
        case 5: rc = radix_pass<K, 5>(ka, va, kb, vb, n, shift, hist, n_tiles, s); break;
        case 6: rc = radix_pass<K, 6>(ka, va, kb, vb, n, shift, hist, n_tiles, s); break;
        case 7: rc = radix_pass<K, 7>(ka, va, kb, vb, n, shift, hist, n_tiles, s); break;
        default: rc = radix_pass<K, 8>(ka, va, kb, vb, n, shift, hist, n_tiles, s); break;
        }
        K* tk = ka; ka = kb; kb = tk;
        uint32_t* tv = va; va = vb; vb = tv;
    }
    if (rc == PCRL_OK && ka != keys) {
        if (hipMemcpyAsync(keys, ka, (size_t)n * sizeof(K), hipMemcpyDeviceToDevice, s) != hipSuccess) rc = PCRL_EHIP;
        if (rc == PCRL_OK && vals &&
            hipMemcpyAsync(vals, va, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s) != hipSuccess)
            rc = PCRL_EHIP;
    }
    if (rc == PCRL_EHIP) set_error("radix sort kernel failed: %s", hipGetErrorString(hipGetLastError()));
    dfree(k2, s);
    dfree(v2, s);
    dfree(hist, s);
    return rc;
}

// ---------------------------------------------------------------------------
// bucket order: items grouped by a 16-bit key, any order inside a bucket
// ---------------------------------------------------------------------------

// Counting pass: one atomic per item (neighbouring keys rarely repeat here);
// pos[j] = the item's position among its bucket's items.
__global__ __launch_bounds__(256) void k_bucket_count(const uint16_t* keys, uint32_t n_max, const uint32_t* n_dev,
                                                      uint32_t* cnt, uint32_t* pos) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n = n_dev ? min(*n_dev, n_max) : n_max;
    if (j < n) pos[j] = atomicAdd(&cnt[keys[j]], 1u);
}

// Exclusive scan of the 65536 bucket counts into start[]: 64 workgroups of
// 1024 buckets, each adding the counts of the buckets before its own range
// (read coalesced from cnt, which nothing writes meanwhile).
constexpr int BUCKET_SCAN_BLOCK = 1024;
__global__ __launch_bounds__(BUCKET_SCAN_BLOCK) void k_bucket_scan(const uint32_t* cnt, uint32_t* start) {
    __shared__ uint32_t wsum[BUCKET_SCAN_BLOCK / 64];
    __shared__ uint32_t wprev[BUCKET_SCAN_BLOCK / 64];
    const uint32_t b = blockIdx.x, t = threadIdx.x, w = t >> 6;
    // the buckets before this range as 16-byte vectors (cnt is 16-byte aligned):
    // at most 16 per thread, eight loads in flight at a time
    const uint4* c4 = reinterpret_cast<const uint4*>(cnt);
    uint32_t prev = 0;
#pragma unroll 8
    for (uint32_t i = t; i < (uint32_t)(BUCKET_SCAN_BLOCK / 4) * b; i += BUCKET_SCAN_BLOCK) {
        const uint4 u = c4[i];
        prev += u.x + u.y + u.z + u.w;
    }
    const uint32_t x = cnt[(size_t)BUCKET_SCAN_BLOCK * b + t];
    const uint32_t incl = wave_incl_scan(x);
    const uint32_t pincl = wave_incl_scan(prev);
    if (lane_id() == 63) {
        wsum[w] = incl;
        wprev[w] = pincl;
    }
    __syncthreads();
    uint32_t off = 0, base = 0;
#pragma unroll
    for (int k = 0; k < BUCKET_SCAN_BLOCK / 64; ++k) {
        off += ((uint32_t)k < w) ? wsum[k] : 0u;
        base += wprev[k];
    }
    start[(size_t)BUCKET_SCAN_BLOCK * b + t] = base + off + incl - x;
}

__global__ __launch_bounds__(256) void k_bucket_scatter(const uint16_t* keys, const uint32_t* pos, uint32_t n_max,
                                                        const uint32_t* n_dev, const uint32_t* start,
                                                        uint32_t* order) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n = n_dev ? min(*n_dev, n_max) : n_max;
    if (j < n) order[start[keys[j]] + pos[j]] = j;
}

int bucket_place_u16(const uint16_t* keys, const uint32_t* pos, int64_t n_max, const uint32_t* n_dev,
                     const uint32_t* cnt, uint32_t* order, hipStream_t s) {
    if (n_max <= 0) return PCRL_OK;
    if ((uintptr_t)cnt & 15u) {
        set_error("bucket counts must be 16-byte aligned");
        return PCRL_EINVAL;
    }
    uint32_t* start = nullptr;
    PCRL_TRY(dalloc((void**)&start, (size_t)65536 * sizeof(uint32_t), s));
    hipLaunchKernelGGL(k_bucket_scan, dim3(65536 / BUCKET_SCAN_BLOCK), dim3(BUCKET_SCAN_BLOCK), 0, s, cnt, start);
    hipLaunchKernelGGL(k_bucket_scatter, dim3((unsigned)((n_max + 255) / 256)), dim3(256), 0, s, keys, pos,
                       (uint32_t)n_max, n_dev, (const uint32_t*)start, order);
    const hipError_t e = hipGetLastError();
    dfree(start, s);
    if (e != hipSuccess) {
        set_error("bucket placement kernel failed: %s", hipGetErrorString(e));
        return PCRL_EHIP;
    }
    return PCRL_OK;
}

int bucket_order_u16(const uint16_t* keys, int64_t n_max, const uint32_t* n_dev, uint32_t* order, hipStream_t s) {
    if (n_max <= 0) return PCRL_OK;
    if (n_max > (int64_t)0xFFFFFFF0ll) {
        set_error("bucket order of %lld items exceeds the 32-bit index range", (long long)n_max);
        return PCRL_EINVAL;
    }
    uint32_t *cnt = nullptr, *pos = nullptr;
    PCRL_TRY(dalloc((void**)&cnt, (size_t)65536 * sizeof(uint32_t), s));
    int rc = dalloc((void**)&pos, (size_t)n_max * sizeof(uint32_t), s);
    if (!rc) rc = fill_u32(cnt, 0u, 65536, s);
    if (!rc) {
        hipLaunchKernelGGL(k_bucket_count, dim3((unsigned)((n_max + 255) / 256)), dim3(256), 0, s, keys,
                           (uint32_t)n_max, n_dev, cnt, pos);
        rc = hipGetLastError() == hipSuccess ? PCRL_OK : PCRL_EHIP;
    }
    if (!rc) rc = bucket_place_u16(keys, pos, n_max, n_dev, cnt, order, s);
    if (rc == PCRL_EHIP) set_error("bucket order kernel failed: %s", hipGetErrorString(hipGetLastError()));
    dfree(pos, s);
    dfree(cnt, s);
    return rc;
}

int radix_sort_u64(uint64_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s) {
    return radix_sort_impl<uint64_t>(keys, vals, n, bits > 64 ? 64 : bits, s);
}

int radix_sort_u64_bits(uint64_t* keys, uint32_t* vals, int64_t n, int lo_bit, int bits, hipStream_t s) {
    if (lo_bit < 0 || bits < 0 || lo_bit + bits > 64) {
        set_error("radix sort of bits [%d, %d) of 64-bit keys", lo_bit, lo_bit + bits);
        return PCRL_EINVAL;
    }
    return radix_sort_impl<uint64_t>(keys, vals, n, bits, s, lo_bit);
}

int radix_sort_u32(uint32_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s) {
    return radix_sort_impl<uint32_t>(keys, vals, n, bits > 32 ? 32 : bits, s);
}

}  // namespace pcrl

extern "C" const char* last_error(void) { return pcrl::get_error(); }

extern "C" const char* pcrl_version(void) { return "pcrl 0.1.0 (gfx950)"; }

namespace pcrl {

// Small device-to-host reads (sizes the host needs before it can go on)
// through a per-thread pinned buffer: the copy goes straight to host memory
// without a pageable staging step.
int read_back(void* host, const void* dev, size_t bytes, hipStream_t s) {
    static thread_local void* pinned = nullptr;
    static thread_local size_t cap = 0;
    if (t_arena) {  // no allocation of any kind: a pageable copy
        if (hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return PCRL_EHIP;
        return PCRL_OK;
    }
    if (bytes > cap) {
        if (pinned) (void)hipHostFree(pinned);
        pinned = nullptr;
        cap = 0;
        const size_t want = std::max<size_t>(bytes, 4096);
        if (hipHostMalloc(&pinned, want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            pinned = nullptr;
        } else {
            cap = want;
        }
    }
    if (!pinned) {  // no pinned memory: plain pageable copy
        if (hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return PCRL_EHIP;
        return PCRL_OK;
    }
    if (hipMemcpyAsync(pinned, dev, bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return PCRL_EHIP;
    std::memcpy(host, pinned, bytes);
    return PCRL_OK;
}

}  // namespace pcrl

extern "C" int set_allocator(const PcrlAllocator* a) {
    pcrl::clear_error();
    if (a && (!a->alloc || !a->free)) {
        pcrl::set_error("set_allocator: alloc and free must both be given");
        return PCRL_EINVAL;
    }
    pcrl::UserAlloc& u = pcrl::user_alloc();
    std::lock_guard<std::mutex> lock(u.mu);
    u.on = a != nullptr;
    u.a = a ? *a : PcrlAllocator{};
    return PCRL_OK;
}
