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

#include <cstdio>
#include <mutex>

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
// allocation
// ---------------------------------------------------------------------------

static int g_pool_ready = -1;  // -1 unknown, 0 no async pool, 1 pool configured
static std::once_flag g_pool_once;

int dalloc(void** p, size_t bytes, hipStream_t s) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    std::call_once(g_pool_once, [] {
        int dev = 0;
        int supported = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&supported, hipDeviceAttributeMemoryPoolsSupported, dev) == hipSuccess &&
            supported) {
            hipMemPool_t pool;
            if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
                uint64_t thr = UINT64_MAX;
                hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
                g_pool_ready = 1;
            } else {
                g_pool_ready = 0;
            }
        } else {
            g_pool_ready = 0;
        }
    });
    hipError_t e = g_pool_ready ? hipMallocAsync(p, bytes, s) : hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
        *p = nullptr;
        return e == hipErrorOutOfMemory ? PCRL_ENOMEM : PCRL_EHIP;
    }
    return PCRL_OK;
}

void dfree(void* p, hipStream_t s) {
    if (!p) return;
    if (g_pool_ready == 1)
        (void)hipFreeAsync(p, s);
    else
        (void)hipFree(p);
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

// Each thread owns SCAN_ITEMS consecutive values of the tile.
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(const uint32_t* in, uint32_t* out, int64_t n,
                                                           const uint32_t* offs, uint32_t* total) {
    const int64_t tile = (int64_t)blockIdx.x * SCAN_TILE;
    const int64_t first = tile + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = first + k;
        v[k] = (i < n) ? in[i] : 0u;
        acc += v[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(acc, &tot) + (offs ? offs[blockIdx.x] : 0u);
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int64_t i = first + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BLOCK - 1) *total = run;
}

int scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, hipStream_t s) {
    if (n <= 0) {
        if (total) PCRL_TRY(fill_u32(total, 0u, 1, s));
        return PCRL_OK;
    }
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(SCAN_BLOCK), 0, s, in, out, n, (const uint32_t*)nullptr,
                           total);
        PCRL_TRY_HIP(hipGetLastError());
        return PCRL_OK;
    }
    uint32_t* sums = nullptr;
    PCRL_TRY(dalloc((void**)&sums, (size_t)nb * sizeof(uint32_t), s));
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, n, sums);
    int rc = hipGetLastError() == hipSuccess ? PCRL_OK : PCRL_EHIP;
    if (rc == PCRL_OK) rc = scan_u32(sums, sums, nb, nullptr, s);
    if (rc == PCRL_OK) {
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, in, out, n, sums, total);
        if (hipGetLastError() != hipSuccess) rc = PCRL_EHIP;
    }
    dfree(sums, s);
    if (rc == PCRL_EHIP) set_error("scan kernel launch failed");
    return rc;
}

// ---------------------------------------------------------------------------
// LSD radix sort, 8-bit digits
// ---------------------------------------------------------------------------

constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int SORT_WAVE = 64;
constexpr int SORT_ITEMS = 32;
constexpr int SORT_TILE = SORT_WAVE * SORT_ITEMS;  // 2048 keys per one-wave block

template <typename K>
__global__ __launch_bounds__(SORT_WAVE) void k_radix_hist(const K* keys, int64_t n, int shift, uint32_t* hist,
                                                          uint32_t n_tiles) {
    __shared__ uint32_t h[RADIX];
    for (int d = threadIdx.x; d < RADIX; d += SORT_WAVE) h[d] = 0;
    __syncthreads();
    const int64_t tile = (int64_t)blockIdx.x * SORT_TILE;
    for (int k = 0; k < SORT_ITEMS; ++k) {
        int64_t i = tile + (int64_t)k * SORT_WAVE + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & (RADIX - 1)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < RADIX; d += SORT_WAVE) hist[(size_t)d * n_tiles + blockIdx.x] = h[d];
}

template <typename K>
__global__ __launch_bounds__(SORT_WAVE) void k_radix_scatter(const K* keys_in, const uint32_t* vals_in, K* keys_out,
                                                             uint32_t* vals_out, int64_t n, int shift,
                                                             const uint32_t* offs, uint32_t n_tiles) {
    __shared__ uint32_t run[RADIX];
    for (int d = threadIdx.x; d < RADIX; d += SORT_WAVE) run[d] = offs[(size_t)d * n_tiles + blockIdx.x];
    __syncthreads();
    const int64_t tile = (int64_t)blockIdx.x * SORT_TILE;
    const uint64_t lt = lanemask_lt();
    for (int k = 0; k < SORT_ITEMS; ++k) {
        const int64_t i = tile + (int64_t)k * SORT_WAVE + threadIdx.x;
        const bool valid = i < n;
        K key = valid ? keys_in[i] : K(0);
        uint32_t val = (valid && vals_in) ? vals_in[i] : 0u;
        const uint32_t digit = (uint32_t)(key >> shift) & (RADIX - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RADIX_BITS; ++b) {
            const bool bit = (digit >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lt);
        uint32_t pos = 0;
        if (valid) pos = run[digit] + rank;
        __syncthreads();
        // the highest lane of each digit group advances the running offset
        if (valid && (peers >> lane_id()) == 1ull) run[digit] += rank + 1;
        __syncthreads();
        if (valid) {
            keys_out[pos] = key;
            if (vals_out) vals_out[pos] = val;
        }
    }
}

template <typename K>
static int radix_sort_impl(K* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s) {
    if (n <= 1 || bits <= 0) return PCRL_OK;
    if (n > (int64_t)0xFFFFFFF0ll) {
        set_error("radix sort of %lld items exceeds the 32-bit index range", (long long)n);
        return PCRL_EINVAL;
    }
    const int64_t n_tiles64 = (n + SORT_TILE - 1) / SORT_TILE;
    const uint32_t n_tiles = (uint32_t)n_tiles64;
    const int passes = (bits + RADIX_BITS - 1) / RADIX_BITS;
    K* k2 = nullptr;
    uint32_t* v2 = nullptr;
    uint32_t* hist = nullptr;
    int rc = dalloc((void**)&k2, (size_t)n * sizeof(K), s);
    if (rc == PCRL_OK && vals) rc = dalloc((void**)&v2, (size_t)n * sizeof(uint32_t), s);
    if (rc == PCRL_OK) rc = dalloc((void**)&hist, (size_t)RADIX * n_tiles * sizeof(uint32_t), s);
    K* ka = keys;
    K* kb = k2;
    uint32_t* va = vals;
    uint32_t* vb = v2;
    for (int p = 0; p < passes && rc == PCRL_OK; ++p) {
        const int shift = p * RADIX_BITS;
        hipLaunchKernelGGL(k_radix_hist<K>, dim3(n_tiles), dim3(SORT_WAVE), 0, s, ka, n, shift, hist, n_tiles);
        if (hipGetLastError() != hipSuccess) {
            rc = PCRL_EHIP;
            break;
        }
        rc = scan_u32(hist, hist, (int64_t)RADIX * n_tiles, nullptr, s);
        if (rc != PCRL_OK) break;
        hipLaunchKernelGGL(k_radix_scatter<K>, dim3(n_tiles), dim3(SORT_WAVE), 0, s, ka, va, kb, vb, n, shift, hist,
                           n_tiles);
        if (hipGetLastError() != hipSuccess) {
            rc = PCRL_EHIP;
            break;
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

int radix_sort_u64(uint64_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s) {
    return radix_sort_impl<uint64_t>(keys, vals, n, bits > 64 ? 64 : bits, s);
}

int radix_sort_u32(uint32_t* keys, uint32_t* vals, int64_t n, int bits, hipStream_t s) {
    return radix_sort_impl<uint32_t>(keys, vals, n, bits > 32 ? 32 : bits, s);
}

}  // namespace pcrl

extern "C" const char* last_error(void) { return pcrl::get_error(); }

extern "C" const char* pcrl_version(void) { return "pcrl 0.1.0 (gfx950)"; }
