// collect.hip -- coarse paths from reception records (paper, Section 2.2.3).
//
// A coarse path is a reception keyed by (TX, RX, number of reflections, the
// labels of its interactions in order); Section 2.2.3 caps the number of kept
// paths with the same labels in the same order at kappa.  Here:
//   1. every record gets a packed multi-word key (tx | rx | b | lab_0..lab_K-1,
//      most significant first; a label is its rank + 1, 0 past b), or leaf
//      indices of the interaction points instead of labels;
//   2. records are sorted by (key, len_poly, ray) with LSD radix passes over
//      a permutation (ray bits, then len_poly bits, then key words);
//   3. key boundaries -> per-key count and in-key rank; rows with rank <
//      kappa are compacted into the caller's arrays.
// The output order is fully determined by the records, so it is bitwise
// reproducible even though records are appended in a racy order.
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace pcrl {

constexpr int MAXW = 6;

struct KeySpec {
    int32_t W;         // 64-bit words per key
    int32_t K;
    int32_t bt, br, bb, bl;
    int32_t mode;      // PCRL_KEY_LABELS / PCRL_KEY_LEAVES
    uint32_t n_rays;
    uint32_t n_total;
    float org[3];
    float inv_h;
    int32_t dim[3];
};

__device__ __forceinline__ void put_bits(uint64_t* w, int pos, int width, uint64_t val) {
    const int wi = pos >> 6, sh = pos & 63;
    w[wi] |= val << sh;
    if (sh + width > 64) w[wi + 1] |= val >> (64 - sh);
}

__global__ void k_path_keys(const uint4* rec, uint32_t n, const float4* hist, KeySpec ks, uint64_t* words,
                            uint32_t* lp_bits, uint32_t* ray) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 r = rec[i];
    const uint32_t g = r.x;
    const uint32_t rx = r.y & 0xFFFFu;
    const uint32_t b = r.y >> 16;
    const uint32_t tx = g / ks.n_rays;
    uint64_t w[MAXW] = {0, 0, 0, 0, 0, 0};
    for (int k = 0; k < ks.K; ++k) {
        uint64_t val = 0;
        if ((uint32_t)k < b) {
            const float4 h = hist[(size_t)k * ks.n_total + g];
            if (ks.mode == PCRL_KEY_LABELS) {
                val = (uint64_t)__float_as_uint(h.w) + 1;
            } else {
                const float p[3] = {h.x, h.y, h.z};
                int64_t c[3];
                for (int a = 0; a < 3; ++a) {
                    int ci = (int)floorf((p[a] - ks.org[a]) * ks.inv_h);
                    c[a] = min(max(ci, 0), ks.dim[a] - 1);
                }
                val = (uint64_t)(c[0] + (int64_t)ks.dim[0] * (c[1] + (int64_t)ks.dim[1] * c[2])) + 1;
            }
        }
        put_bits(w, (ks.K - 1 - k) * ks.bl, ks.bl, val);
    }
    int pos = ks.K * ks.bl;
    put_bits(w, pos, ks.bb, b);
    pos += ks.bb;
    put_bits(w, pos, ks.br, rx);
    pos += ks.br;
    put_bits(w, pos, ks.bt, tx);
    for (int q = 0; q < ks.W; ++q) words[(size_t)q * n + i] = w[q];
    lp_bits[i] = r.z;  // len_poly >= 0: IEEE bits order like the values
    ray[i] = g;
}

__global__ void k_gather_u64(const uint64_t* src, const uint32_t* perm, uint32_t n, uint64_t* dst) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

__global__ void k_gather_u32(const uint32_t* src, const uint32_t* perm, uint32_t n, uint32_t* dst) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

__global__ void k_key_flags(const uint64_t* words, int W, const uint32_t* perm, uint32_t n, uint32_t* flag) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t f = 1;
    if (i > 0) {
        f = 0;
        const uint32_t a = perm[i], b = perm[i - 1];
        for (int q = 0; q < W; ++q) f |= words[(size_t)q * n + a] != words[(size_t)q * n + b] ? 1u : 0u;
    }
    flag[i] = f;
}

// key index of sorted position i (flags recomputed from keys)
__global__ void k_key_starts(const uint64_t* words, int W, const uint32_t* perm, uint32_t n, const uint32_t* kscan,
                             uint32_t* start) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool f = (i == 0);
    if (!f) {
        const uint32_t a = perm[i], b = perm[i - 1];
        for (int q = 0; q < W; ++q) f |= words[(size_t)q * n + a] != words[(size_t)q * n + b];
    }
    if (f) start[kscan[i]] = i;
}

__global__ void k_keep_flags(const uint64_t* words, int W, const uint32_t* perm, uint32_t n, const uint32_t* kscan,
                             const uint32_t* start, int32_t kappa, uint32_t* keep) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool f = (i == 0);
    if (!f) {
        const uint32_t a = perm[i], b = perm[i - 1];
        for (int q = 0; q < W; ++q) f |= words[(size_t)q * n + a] != words[(size_t)q * n + b];
    }
    const uint32_t key = kscan[i] + (f ? 1u : 0u) - 1u;
    keep[i] = (i - start[key]) < (uint32_t)kappa ? 1u : 0u;
}

struct OutArrays {
    int32_t* tx;
    int32_t* rx;
    int32_t* n_refl;
    int64_t* key;
    int64_t* count;
    int32_t* rank;
    int64_t* ray;
    float* len_poly;
    float* len_unf;
    float* points;
};

__global__ void k_write_rows(const uint4* rec, const float4* hist, const uint64_t* words, int W, const uint32_t* perm,
                             uint32_t n, const uint32_t* kscan, const uint32_t* start, const uint32_t* n_keys,
                             const uint32_t* keep_scan, int32_t kappa, KeySpec ks,
                             OutArrays o) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool f = (i == 0);
    if (!f) {
        const uint32_t a = perm[i], b = perm[i - 1];
        for (int q = 0; q < W; ++q) f |= words[(size_t)q * n + a] != words[(size_t)q * n + b];
    }
    const uint32_t key = kscan[i] + (f ? 1u : 0u) - 1u;
    const uint32_t rank = i - start[key];
    if (rank >= (uint32_t)kappa) return;
    const uint32_t end = (key + 1 < *n_keys) ? start[key + 1] : n;
    const uint32_t row = keep_scan[i];
    const uint4 r = rec[perm[i]];
    const uint32_t g = r.x;
    const uint32_t b = r.y >> 16;
    if (o.tx) o.tx[row] = (int32_t)(g / ks.n_rays);
    if (o.rx) o.rx[row] = (int32_t)(r.y & 0xFFFFu);
    if (o.n_refl) o.n_refl[row] = (int32_t)b;
    if (o.count) o.count[row] = (int64_t)(end - start[key]);
    if (o.rank) o.rank[row] = (int32_t)rank;
    if (o.ray) o.ray[row] = (int64_t)g;
    if (o.len_poly) o.len_poly[row] = __uint_as_float(r.z);
    if (o.len_unf) o.len_unf[row] = __uint_as_float(r.w);
    for (int k = 0; k < ks.K; ++k) {
        float4 h = make_float4(NAN, NAN, NAN, 0.f);
        if ((uint32_t)k < b) h = hist[(size_t)k * ks.n_total + g];
        if (o.key) {
            int64_t kv = -1;
            if ((uint32_t)k < b) {
                if (ks.mode == PCRL_KEY_LABELS) {
                    kv = (int64_t)__float_as_uint(h.w);
                } else {
                    int64_t c[3];
                    const float p[3] = {h.x, h.y, h.z};
                    for (int a = 0; a < 3; ++a) {
                        int ci = (int)floorf((p[a] - ks.org[a]) * ks.inv_h);
                        c[a] = min(max(ci, 0), ks.dim[a] - 1);
                    }
                    kv = c[0] + (int64_t)ks.dim[0] * (c[1] + (int64_t)ks.dim[1] * c[2]);
                }
            }
            o.key[(size_t)row * ks.K + k] = kv;
        }
        if (o.points) {
            o.points[((size_t)row * ks.K + k) * 3 + 0] = h.x;
            o.points[((size_t)row * ks.K + k) * 3 + 1] = h.y;
            o.points[((size_t)row * ks.K + k) * 3 + 2] = h.z;
        }
    }
}

// ---------------------------------------------------------------------------
// small record sets: the whole collection in one workgroup
// ---------------------------------------------------------------------------
//
// A launch usually yields few reception records (hundreds to a few
// thousand).  Then keys, the (key, len_poly, ray) sort (bitonic, in LDS),
// key boundaries, counts, ranks and the row compaction run in one kernel of
// one workgroup: one launch instead of some fifty small ones.

constexpr int SMALL_N = 2048;      // records (power of two)
constexpr int SMALL_BLOCK = 1024;  // threads; each owns positions 2t and 2t + 1
constexpr int SMALL_W = 2;         // key words

__device__ __forceinline__ uint32_t block_incl_scan_small(uint32_t x, uint32_t* wsum, uint32_t* total) {
    const int w = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan(x);
    if (lane_id() == 63) wsum[w] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < SMALL_BLOCK / 64; ++k) {
        const uint32_t v = wsum[k];
        off += (k < w) ? v : 0u;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return off + incl;
}

__global__ __launch_bounds__(SMALL_BLOCK) void k_collect_small(const uint4* rec, uint32_t n, const float4* hist,
                                                               KeySpec ks, int32_t kappa, int64_t capacity,
                                                               OutArrays o, uint32_t* tots) {
    __shared__ uint64_t sw[SMALL_W][SMALL_N];
    __shared__ uint32_t slp[SMALL_N];
    __shared__ uint32_t sray[SMALL_N];
    __shared__ uint16_t sidx[SMALL_N];
    __shared__ uint16_t sstart[SMALL_N];
    __shared__ uint32_t wsum[SMALL_BLOCK / 64];
    const uint32_t t = threadIdx.x;
    uint32_t n2 = 1;
    while (n2 < n) n2 <<= 1;
    // 1. keys (as k_path_keys)
    for (uint32_t i = t; i < n2; i += SMALL_BLOCK) {
        sidx[i] = (uint16_t)i;
        if (i >= n) continue;
        const uint4 r = rec[i];
        const uint32_t g = r.x;
        const uint32_t b = r.y >> 16;
        uint64_t w[MAXW] = {0, 0, 0, 0, 0, 0};
        for (int k = 0; k < ks.K; ++k) {
            uint64_t val = 0;
            if ((uint32_t)k < b) {
                const float4 h = hist[(size_t)k * ks.n_total + g];
                if (ks.mode == PCRL_KEY_LABELS) {
                    val = (uint64_t)__float_as_uint(h.w) + 1;
                } else {
                    const float pp[3] = {h.x, h.y, h.z};
                    int64_t c[3];
                    for (int a = 0; a < 3; ++a) {
                        int ci = (int)floorf((pp[a] - ks.org[a]) * ks.inv_h);
                        c[a] = min(max(ci, 0), ks.dim[a] - 1);
                    }
                    val = (uint64_t)(c[0] + (int64_t)ks.dim[0] * (c[1] + (int64_t)ks.dim[1] * c[2])) + 1;
                }
            }
            put_bits(w, (ks.K - 1 - k) * ks.bl, ks.bl, val);
        }
        int pos = ks.K * ks.bl;
        put_bits(w, pos, ks.bb, b);
        pos += ks.bb;
        put_bits(w, pos, ks.br, r.y & 0xFFFFu);
        pos += ks.br;
        put_bits(w, pos, ks.bt, g / ks.n_rays);
        sw[0][i] = w[0];
        sw[1][i] = w[1];
        slp[i] = r.z;
        sray[i] = g;
    }
    __syncthreads();
    // 2. bitonic sort of the record indices by (key words, len_poly bits, ray); padding last
    auto less = [&](uint32_t a, uint32_t b) -> bool {
        if (a >= n) return false;
        if (b >= n) return true;
        for (int q = ks.W - 1; q >= 0; --q)
            if (sw[q][a] != sw[q][b]) return sw[q][a] < sw[q][b];
        if (slp[a] != slp[b]) return slp[a] < slp[b];
        return sray[a] < sray[b];
    };
    for (uint32_t k = 2; k <= n2; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = t; i < n2; i += SMALL_BLOCK) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint32_t a = sidx[i], b = sidx[l];
                    const bool up = (i & k) == 0;
                    if (up ? less(b, a) : less(a, b)) {
                        sidx[i] = (uint16_t)b;
                        sidx[l] = (uint16_t)a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // 3. key boundaries, key index, first position of each key
    auto same_key = [&](uint32_t p) -> bool {  // sorted position p (> 0) has the key of p - 1
        const uint32_t a = sidx[p], b = sidx[p - 1];
        for (int q = 0; q < ks.W; ++q)
            if (sw[q][a] != sw[q][b]) return false;
        return true;
    };
    const uint32_t p0 = 2 * t, p1 = 2 * t + 1;
    const bool f0 = p0 < n && (p0 == 0 || !same_key(p0));
    const bool f1 = p1 < n && !same_key(p1);
    uint32_t n_keys = 0;
    const uint32_t kin = block_incl_scan_small((f0 ? 1u : 0u) + (f1 ? 1u : 0u), wsum, &n_keys);
    const uint32_t key1 = kin - 1;                     // key index of p1
    const uint32_t key0 = kin - (f1 ? 1u : 0u) - 1;    // key index of p0
    if (f0) sstart[key0] = (uint16_t)p0;
    if (f1) sstart[key1] = (uint16_t)p1;
    __syncthreads();
    // 4. ranks inside keys, kept rows
    const bool k0 = p0 < n && p0 - sstart[key0] < (uint32_t)kappa;
    const bool k1 = p1 < n && p1 - sstart[key1] < (uint32_t)kappa;
    uint32_t n_rows = 0;
    const uint32_t rin = block_incl_scan_small((k0 ? 1u : 0u) + (k1 ? 1u : 0u), wsum, &n_rows);
    if (t == 0) {
        tots[0] = n_keys;
        tots[1] = n_rows;
    }
    if ((int64_t)n_rows > capacity) return;  // the host reports the overflow
    // 5. rows (rows before this thread's: rin minus its own kept rows)
    const uint32_t rbase = rin - (k0 ? 1u : 0u) - (k1 ? 1u : 0u);
    for (int e = 0; e < 2; ++e) {
        const uint32_t p = e ? p1 : p0;
        const bool keep = e ? k1 : k0;
        if (!keep) continue;
        const uint32_t key = e ? key1 : key0;
        const uint32_t row = e ? rbase + (k0 ? 1u : 0u) : rbase;
        const uint32_t first = sstart[key];
        const uint32_t end = (key + 1 < n_keys) ? sstart[key + 1] : n;
        const uint4 r = rec[sidx[p]];
        const uint32_t g = r.x;
        const uint32_t b = r.y >> 16;
        if (o.tx) o.tx[row] = (int32_t)(g / ks.n_rays);
        if (o.rx) o.rx[row] = (int32_t)(r.y & 0xFFFFu);
        if (o.n_refl) o.n_refl[row] = (int32_t)b;
        if (o.count) o.count[row] = (int64_t)(end - first);
        if (o.rank) o.rank[row] = (int32_t)(p - first);
        if (o.ray) o.ray[row] = (int64_t)g;
        if (o.len_poly) o.len_poly[row] = __uint_as_float(r.z);
        if (o.len_unf) o.len_unf[row] = __uint_as_float(r.w);
        for (int k = 0; k < ks.K; ++k) {
            float4 h = make_float4(NAN, NAN, NAN, 0.f);
            if ((uint32_t)k < b) h = hist[(size_t)k * ks.n_total + g];
            if (o.key) {
                int64_t kv = -1;
                if ((uint32_t)k < b) {
                    if (ks.mode == PCRL_KEY_LABELS) {
                        kv = (int64_t)__float_as_uint(h.w);
                    } else {
                        int64_t c[3];
                        const float pp[3] = {h.x, h.y, h.z};
                        for (int a = 0; a < 3; ++a) {
                            int ci = (int)floorf((pp[a] - ks.org[a]) * ks.inv_h);
                            c[a] = min(max(ci, 0), ks.dim[a] - 1);
                        }
                        kv = c[0] + (int64_t)ks.dim[0] * (c[1] + (int64_t)ks.dim[1] * c[2]);
                    }
                }
                o.key[(size_t)row * ks.K + k] = kv;
            }
            if (o.points) {
                o.points[((size_t)row * ks.K + k) * 3 + 0] = h.x;
                o.points[((size_t)row * ks.K + k) * 3 + 1] = h.y;
                o.points[((size_t)row * ks.K + k) * 3 + 2] = h.z;
            }
        }
    }
}

static int bits_for(uint64_t max_value) {
    int b = 1;
    while (b < 64 && (max_value >> b) != 0) ++b;
    return b;
}

static unsigned nblk(uint32_t n) { return std::max(1u, (n + 255u) / 256u); }

// Scratch bytes collect_impl needs for n records with W-word keys: the
// per-record arrays (W key words, a 64-bit and seven 32-bit arrays), the
// radix sort's double buffer and tile histograms, the scan's block sums,
// and 256-byte alignment of every block.
static size_t collect_scratch_bytes(uint64_t n, int W) {
    const uint64_t tiles = (n + 2047) / 2048;
    return (size_t)(n * (8ull * W + 8 + 28) + n * 12 + tiles * 256 * 4 + (n / 512 + 64) * 4 + 64 * 256);
}

// scratch_limit > 0: the call may use at most that many bytes of temporaries
// (checked before any is taken).
static int collect_impl(PcrlLaunch* L, int32_t kappa, int32_t key_mode, PcrlPaths* out, hipStream_t s,
                        size_t scratch_limit = 0) {
    const PcrlScene* S = L->scene;
    const int K = L->K;
    uint32_t n_rec = 0;
    if (L->stream != s) PCRL_TRY_HIP(hipStreamSynchronize(L->stream));
    if (read_back(&n_rec, L->counters + PCRL_CNT_REC(K), 4, s) != PCRL_OK) {
        set_error("collect_paths: reading the record count failed: %s", hipGetErrorString(hipGetLastError()));
        return PCRL_EHIP;
    }
    out->n_rows = 0;
    out->n_keys = 0;
    if ((int64_t)n_rec > L->rec_cap) {
        out->n_rows = -1;
        set_error("collect_paths: the launch produced %u reception records but its capacity is %lld; "
                  "relaunch with record_capacity >= %u",
                  n_rec, (long long)L->rec_cap, n_rec);
        return PCRL_EOVERFLOW;
    }
    if (n_rec == 0) return PCRL_OK;
    const uint32_t n = n_rec;

    KeySpec ks{};
    ks.K = K;
    ks.mode = key_mode;
    ks.n_rays = (uint32_t)L->n_rays;
    ks.n_total = (uint32_t)L->n_total;
    ks.bt = bits_for((uint64_t)(L->n_tx - 1));
    ks.br = bits_for((uint64_t)std::max(L->n_rx - 1, 0));
    ks.bb = bits_for((uint64_t)K);
    if (key_mode == PCRL_KEY_LABELS) {
        ks.bl = bits_for((uint64_t)L->max_label + 1);  // label + 1, 0 past the path's end
    } else {
        const uint64_t cells = (uint64_t)S->view.dim[0] * S->view.dim[1] * S->view.dim[2];
        ks.bl = bits_for(cells);
        if (ks.bl > 62) {
            set_error("collect_paths: leaf grid too large for leaf-index keys");
            return PCRL_EINVAL;
        }
    }
    for (int a = 0; a < 3; ++a) {
        ks.org[a] = S->view.org[a];
        ks.dim[a] = S->view.dim[a];
    }
    ks.inv_h = S->view.inv_h;
    const int total_bits = ks.bt + ks.br + ks.bb + K * ks.bl;
    ks.W = (total_bits + 63) / 64;
    if (ks.W > MAXW) {
        set_error("collect_paths: coarse-path key needs %d bits (max %d)", total_bits, 64 * MAXW);
        return PCRL_EINVAL;
    }

    if (scratch_limit && collect_scratch_bytes(n, ks.W) > scratch_limit) {
        set_error("collect_paths_noalloc: %u records with %d-word keys need %zu bytes of scratch, more than the "
                  "%zu bytes of the fixed array; use collect_paths",
                  n, ks.W, collect_scratch_bytes(n, ks.W), scratch_limit);
        return PCRL_EINVAL;
    }
    DevBufs T;
    T.stream = s;
    auto fail = [&](int code) { T.release(); return code; };
    OutArrays oa{out->tx, out->rx, out->n_refl, out->key, out->count, out->rank, out->ray, out->len_poly, out->len_unf,
                 out->points};
    if (n <= (uint32_t)SMALL_N && ks.W <= SMALL_W) {
        uint32_t* tots = nullptr;
        int rc = T.alloc(&tots, 2);
        if (rc) return fail(rc);
        hipLaunchKernelGGL(k_collect_small, dim3(1), dim3(SMALL_BLOCK), 0, s, L->rec, n, L->hist, ks, kappa,
                           out->capacity, oa, tots);
        uint32_t host[2] = {0, 0};
        if (hipGetLastError() != hipSuccess || read_back(host, tots, 8, s) != PCRL_OK) {
            set_error("collect_paths: kernel failed: %s", hipGetErrorString(hipGetLastError()));
            return fail(PCRL_EHIP);
        }
        out->n_keys = host[0];
        out->n_rows = host[1];
        T.release();
        if ((int64_t)host[1] > out->capacity) {
            set_error("collect_paths: %u rows do not fit in capacity %lld", host[1], (long long)out->capacity);
            return PCRL_EOVERFLOW;
        }
        return PCRL_OK;
    }
    uint64_t *words = nullptr, *tmp64 = nullptr;
    uint32_t *lp = nullptr, *ray = nullptr, *perm = nullptr, *tmp32 = nullptr, *kscan = nullptr, *start = nullptr,
             *keep = nullptr, *tots = nullptr;
    int rc;
    if ((rc = T.alloc(&words, (size_t)ks.W * n)) || (rc = T.alloc(&tmp64, n)) || (rc = T.alloc(&lp, n)) ||
        (rc = T.alloc(&ray, n)) || (rc = T.alloc(&perm, n)) || (rc = T.alloc(&tmp32, n)) ||
        (rc = T.alloc(&kscan, n)) || (rc = T.alloc(&start, n)) || (rc = T.alloc(&keep, n)) || (rc = T.alloc(&tots, 2)))
        return fail(rc);
    hipLaunchKernelGGL(k_path_keys, dim3(nblk(n)), dim3(256), 0, s, L->rec, n, L->hist, ks, words, lp, ray);
    if ((rc = iota_u32(perm, n, s))) return fail(rc);
    // LSD: ray id, then len_poly, then key words from least significant
    hipLaunchKernelGGL(k_gather_u32, dim3(nblk(n)), dim3(256), 0, s, ray, perm, n, tmp32);
    if ((rc = radix_sort_u32(tmp32, perm, n, bits_for((uint64_t)L->n_total), s))) return fail(rc);
    hipLaunchKernelGGL(k_gather_u32, dim3(nblk(n)), dim3(256), 0, s, lp, perm, n, tmp32);
    if ((rc = radix_sort_u32(tmp32, perm, n, 32, s))) return fail(rc);
    for (int q = 0; q < ks.W; ++q) {
        const int wb = (q == ks.W - 1) ? total_bits - 64 * q : 64;
        hipLaunchKernelGGL(k_gather_u64, dim3(nblk(n)), dim3(256), 0, s, words + (size_t)q * n, perm, n, tmp64);
        if ((rc = radix_sort_u64(tmp64, perm, n, wb, s))) return fail(rc);
    }
    // key boundaries
    hipLaunchKernelGGL(k_key_flags, dim3(nblk(n)), dim3(256), 0, s, words, ks.W, perm, n, kscan);
    if ((rc = scan_u32(kscan, kscan, n, tots, s))) return fail(rc);
    hipLaunchKernelGGL(k_key_starts, dim3(nblk(n)), dim3(256), 0, s, words, ks.W, perm, n, kscan, start);
    hipLaunchKernelGGL(k_keep_flags, dim3(nblk(n)), dim3(256), 0, s, words, ks.W, perm, n, kscan, start, kappa, keep);
    if ((rc = scan_u32(keep, keep, n, tots + 1, s))) return fail(rc);
    uint32_t host[2] = {0, 0};
    if (read_back(host, tots, 8, s) != PCRL_OK) {
        set_error("collect_paths: kernels failed: %s", hipGetErrorString(hipGetLastError()));
        return fail(PCRL_EHIP);
    }
    out->n_keys = host[0];
    out->n_rows = host[1];
    if ((int64_t)host[1] > out->capacity) {
        set_error("collect_paths: %u rows do not fit in capacity %lld", host[1], (long long)out->capacity);
        return fail(PCRL_EOVERFLOW);
    }
    hipLaunchKernelGGL(k_write_rows, dim3(nblk(n)), dim3(256), 0, s, L->rec, L->hist, words, ks.W, perm, n, kscan,
                       start, tots, keep, kappa, ks, oa);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        set_error("collect_paths: output kernel failed: %s", hipGetErrorString(hipGetLastError()));
        return fail(PCRL_EHIP);
    }
    T.release();
    return PCRL_OK;
}

// ---------------------------------------------------------------------------
// collect_paths without allocation: temporaries in a fixed device array
// ---------------------------------------------------------------------------

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

// Every no-allocation call on a device shares that device's copy of this
// array (held until the process ends); host code reaches it only through
// the address hipGetSymbolAddress returns for the device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];

static int scratch_of_current_device(void** out) {
    int dev = 0;
    PCRL_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        set_error("collect_paths_noalloc: device ordinal %d beyond %d", dev, NOALLOC_MAX_DEVICES);
        return PCRL_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            set_error("collect_paths_noalloc: address of the scratch array on device %d: %s", dev,
                      hipGetErrorString(e));
            return PCRL_EHIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PCRL_OK;
}

}  // namespace pcrl

using namespace pcrl;

extern "C" int collect_paths_noalloc(PcrlLaunch* launch, int32_t kappa, int32_t key_mode, PcrlPaths* out,
                                     pcrl_stream_t stream) {
    clear_error();
    if (!launch || !out || kappa < 1 || (key_mode != PCRL_KEY_LABELS && key_mode != PCRL_KEY_LEAVES) ||
        out->capacity < 0) {
        set_error("collect_paths_noalloc: invalid arguments (kappa >= 1, key_mode 0 or 1, capacity >= 0)");
        return PCRL_EINVAL;
    }
    void* base = nullptr;
    int rc = scratch_of_current_device(&base);
    if (rc) return rc;
    ArenaScope arena(base, NOALLOC_SCRATCH_BYTES);
    return collect_impl(launch, kappa, key_mode, out, (hipStream_t)stream, NOALLOC_SCRATCH_BYTES);
}

extern "C" int collect_paths(PcrlLaunch* launch, int32_t kappa, int32_t key_mode, PcrlPaths* out,
                             pcrl_stream_t stream) {
    clear_error();
    if (!launch || !out || kappa < 1 || (key_mode != PCRL_KEY_LABELS && key_mode != PCRL_KEY_LEAVES) ||
        out->capacity < 0) {
        set_error("collect_paths: invalid arguments (kappa >= 1, key_mode 0 or 1, capacity >= 0)");
        return PCRL_EINVAL;
    }
    return collect_impl(launch, kappa, key_mode, out, (hipStream_t)stream);
}
