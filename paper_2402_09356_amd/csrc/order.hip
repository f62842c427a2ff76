// Location orderings of paper Section 3 on the GPU: 16-bit encoding,
// Morton / Hilbert / SplitMix64 keys, a stable LSD radix sort with an index
// payload, and the KD-tree ordering as level-synchronous segmented sorts.
#include "common.h"

#include <cmath>
#include <mutex>
#include <vector>

namespace tlr {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 4;                        // elements per thread per block
constexpr int kSortTile = kSortThreads * kSortItems; // 1024 elements per block
constexpr int kRadixBits = 8;
constexpr int kBuckets = 1 << kRadixBits;

// ---------------------------------------------------------------- encoding --

// rint(x * 65535) with round-half-even, clamped; x already checked to be in
// [0, 1].  rint() rounds ties to even under the default rounding mode.
__device__ inline uint32_t encode16(double x) {
    double q = rint(x * 65535.0);
    q = fmin(fmax(q, 0.0), 65535.0);
    return (uint32_t)q;
}

// Morton key: x bit b -> key bit 2b, y bit b -> key bit 2b+1 (Section 3.1.1).
__device__ inline uint32_t spread_bits16(uint32_t v) {
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

__device__ inline uint32_t morton_key(uint32_t qx, uint32_t qy) {
    return spread_bits16(qx) | (spread_bits16(qy) << 1);
}

// Hilbert key of the order-16 curve (Section 3.1.2, Skilling 2004), oriented
// so that the order-1 pattern is (0,0) (0,1) (1,1) (1,0).  This follows
// Skilling's "transpose" formulation: the coordinates are transformed in
// place, from the most significant bit down, into the Gray-coded transpose
// of the curve index, which is then Gray-decoded and bit-interleaved.
__device__ inline uint32_t hilbert_key(uint32_t x, uint32_t y) {
    // axes -> transpose (Skilling's AxestoTranspose for 2 dimensions, 16 bits)
    uint32_t X[2] = {x, y};
    const uint32_t M = 1u << 15;
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        uint32_t P = Q - 1;
        for (int i = 0; i < 2; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;  // invert low bits of the first axis
            } else {
                uint32_t t = (X[0] ^ X[i]) & P;  // exchange low bits
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    // Gray encode
    X[1] ^= X[0];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[1] & Q) t ^= Q - 1;
    X[0] ^= t;
    X[1] ^= t;
    // interleave the transpose: bit b of axis 0 is the more significant of the pair
    return (spread_bits16(X[0]) << 1) | spread_bits16(X[1]);
}

// SplitMix64 (Steele, Lea, Flood 2014): output number i+1 of the stream that
// starts at state `seed` (counter form: state_k = seed + k * gamma).
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_check_domain(const double *__restrict__ locs, int64_t n, int *__restrict__ bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = locs[2 * i], y = locs[2 * i + 1];
    bool ok = (x >= 0.0) && (x <= 1.0) && (y >= 0.0) && (y <= 1.0);  // false for NaN
    if (!ok) atomicOr(bad, 1);
}

// kind: 2 morton, 3 hilbert (32-bit keys)
__global__ void k_curve_keys(const double *__restrict__ locs, int64_t n, int kind,
                             uint32_t *__restrict__ keys, int32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t qx = encode16(locs[2 * i]);
    uint32_t qy = encode16(locs[2 * i + 1]);
    keys[i] = (kind == TLR_ORDER_MORTON) ? morton_key(qx, qy) : hilbert_key(qx, qy);
    vals[i] = (int32_t)i;
}

__global__ void k_random_keys(int64_t n, uint64_t seed, uint64_t *__restrict__ keys,
                              int32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = splitmix64_at(seed, (uint64_t)i + 1);
    vals[i] = (int32_t)i;
}

__global__ void k_iota(int64_t n, int32_t *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)i;
}

// --------------------------------------------------------------- radix sort --

template <typename K>
__device__ inline uint32_t digit_of(K key, int shift) {
    return (uint32_t)((key >> shift) & (K)(kBuckets - 1));
}

// Per-block digit histogram, stored digit-major: hist[d * nblocks + b].
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const K *__restrict__ keys, int64_t n,
                                                             int shift, uint32_t *__restrict__ hist,
                                                             int nblocks) {
    __shared__ uint32_t cnt[kBuckets];
    const int tid = threadIdx.x;
    cnt[tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        int64_t i = base + r * kSortThreads + tid;
        if (i < n) atomicAdd(&cnt[digit_of(keys[i], shift)], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * nblocks + blockIdx.x] = cnt[tid];
}

// Exclusive scan of `count` uint32 values in place (single work-group).
__global__ __launch_bounds__(1024) void k_scan_exclusive(uint32_t *__restrict__ data, int64_t count) {
    __shared__ uint32_t part[1024];
    const int tid = threadIdx.x;
    const int64_t chunk = (count + 1023) / 1024;
    const int64_t lo = tid * chunk;
    const int64_t hi = (lo + chunk < count) ? lo + chunk : count;
    uint32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += data[i];
    part[tid] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the partial sums
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = (tid >= off) ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint32_t run = (tid > 0) ? part[tid - 1] : 0u;
    for (int64_t i = lo; i < hi; ++i) {
        uint32_t v = data[i];
        data[i] = run;
        run += v;
    }
}

// Stable scatter: elements of a block keep their relative order within each
// digit.  Elements are taken in rounds of 256 (round-major, then thread), the
// same order as the input positions.
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const K *__restrict__ keys_in, const int32_t *__restrict__ vals_in, K *__restrict__ keys_out,
    int32_t *__restrict__ vals_out, int64_t n, int shift, const uint32_t *__restrict__ offsets,
    int nblocks) {
    __shared__ uint32_t run[kBuckets];                         // running count per digit
    __shared__ uint32_t wave_cnt[kSortThreads / 64][kBuckets];  // this round, per wave
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    run[tid] = offsets[(int64_t)tid * nblocks + blockIdx.x];
    for (int w = 0; w < kSortThreads / 64; ++w) wave_cnt[w][tid] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = base + r * kSortThreads + tid;
        const bool valid = i < n;
        K key = valid ? keys_in[i] : (K)0;
        int32_t val = valid ? vals_in[i] : 0;
        uint32_t d = valid ? digit_of(key, shift) : 0u;
        // lanes of this wave holding the same digit
        uint64_t same = __ballot(valid);
        for (int b = 0; b < kRadixBits; ++b) {
            uint64_t ones = __ballot(valid && ((d >> b) & 1u));
            same &= ((d >> b) & 1u) ? ones : ~ones;
        }
        const uint32_t rank_in_wave = __popcll(same & lt_mask);
        const uint32_t count_in_wave = __popcll(same);
        if (valid && rank_in_wave == 0) wave_cnt[wave][d] = count_in_wave;
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank_in_wave;
            for (int w = 0; w < wave; ++w) pos += wave_cnt[w][d];
            keys_out[pos] = key;
            vals_out[pos] = val;
        }
        __syncthreads();
        // advance the running counts, then clear this round's counts
        uint32_t add = 0;
        for (int w = 0; w < kSortThreads / 64; ++w) {
            add += wave_cnt[w][tid];
            wave_cnt[w][tid] = 0;
        }
        run[tid] += add;
        __syncthreads();
    }
}

// Sorts (keys, vals) stably by the low `bits` bits of the keys.  Ping-pongs
// between the given buffers; returns via *result_in_alt whether the sorted data
// ended in the alternate buffers.
template <typename K>
tlr_status radix_sort(K *keys, int32_t *vals, K *keys_alt, int32_t *vals_alt, uint32_t *hist,
                      int64_t n, int bits, bool *result_in_alt, hipStream_t s) {
    const int nblocks = (int)cdiv(n, kSortTile);
    bool alt = false;
    for (int shift = 0; shift < bits; shift += kRadixBits) {
        K *kin = alt ? keys_alt : keys;
        int32_t *vin = alt ? vals_alt : vals;
        K *kout = alt ? keys : keys_alt;
        int32_t *vout = alt ? vals : vals_alt;
        hipLaunchKernelGGL(k_radix_hist<K>, dim3(nblocks), dim3(kSortThreads), 0, s, kin, n, shift,
                           hist, nblocks);
        hipLaunchKernelGGL(k_scan_exclusive, dim3(1), dim3(1024), 0, s, hist,
                           (int64_t)nblocks * kBuckets);
        hipLaunchKernelGGL(k_radix_scatter<K>, dim3(nblocks), dim3(kSortThreads), 0, s, kin, vin,
                           kout, vout, n, shift, hist, nblocks);
        alt = !alt;
    }
    TLR_HIP(hipGetLastError());
    *result_in_alt = alt;
    return TLR_OK;
}

// ------------------------------------------------------------------ KD-tree --

__global__ void k_coord_keys(const double *__restrict__ locs, int64_t n, int dim,
                             uint64_t *__restrict__ keys, int32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = locs[2 * i + dim] + 0.0;  // -0.0 -> +0.0 so bit order = value order
    keys[i] = (uint64_t)__double_as_longlong(v);
    vals[i] = (int32_t)i;
}

__global__ void k_scatter_rank(const int32_t *__restrict__ sorted_vals, int64_t n,
                               int32_t *__restrict__ rank) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) rank[sorted_vals[p]] = (int32_t)p;
}

// Start of the segment holding position p after `level` halvings of [0, n):
// a segment of size m splits into ceil(m/2) and floor(m/2).
__device__ inline int64_t seg_start(int64_t p, int64_t n, int level, int64_t *size_out) {
    int64_t start = 0, size = n;
    for (int l = 0; l < level && size > 1; ++l) {
        int64_t left = (size + 1) / 2;
        if (p < start + left) {
            size = left;
        } else {
            start += left;
            size -= left;
        }
    }
    *size_out = size;
    return start;
}

__global__ void k_seg_init(int64_t n, unsigned long long *__restrict__ mn,
                           unsigned long long *__restrict__ mx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    mn[2 * i] = ~0ull;
    mn[2 * i + 1] = ~0ull;
    mx[2 * i] = 0ull;
    mx[2 * i + 1] = 0ull;
}

// Per-segment min/max of x and y (coordinates are >= 0, so their bit
// patterns order like the values).
__global__ void k_seg_bbox(const double *__restrict__ locs, const int32_t *__restrict__ pts,
                           int64_t n, int level, unsigned long long *__restrict__ mn,
                           unsigned long long *__restrict__ mx) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int64_t size;
    int64_t s = seg_start(p, n, level, &size);
    if (size <= 1) return;
    int32_t id = pts[p];
    for (int d = 0; d < 2; ++d) {
        unsigned long long b = (unsigned long long)__double_as_longlong(locs[2 * (int64_t)id + d] + 0.0);
        atomicMin(&mn[2 * s + d], b);
        atomicMax(&mx[2 * s + d], b);
    }
}

// Key = segment start (high bits) | rank of the point along the segment's
// split coordinate (low 32 bits).  The split coordinate is y only when the y
// range is strictly larger (ranges computed in float64 as max - min).
__global__ void k_seg_keys(const int32_t *__restrict__ pts, int64_t n, int level,
                           const unsigned long long *__restrict__ mn,
                           const unsigned long long *__restrict__ mx,
                           const int32_t *__restrict__ rank_x, const int32_t *__restrict__ rank_y,
                           int rank_bits, uint64_t *__restrict__ keys, int32_t *__restrict__ vals) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    int64_t size;
    int64_t s = seg_start(p, n, level, &size);
    int32_t id = pts[p];
    uint32_t r = 0;
    if (size > 1) {
        double rx = __longlong_as_double((long long)mx[2 * s]) - __longlong_as_double((long long)mn[2 * s]);
        double ry = __longlong_as_double((long long)mx[2 * s + 1]) - __longlong_as_double((long long)mn[2 * s + 1]);
        r = (uint32_t)((ry > rx) ? rank_y[id] : rank_x[id]);
    } else {
        r = (uint32_t)p;  // single-point segment: nothing to order
    }
    keys[p] = ((uint64_t)s << rank_bits) | (uint64_t)r;
    vals[p] = id;
}

int bits_for(int64_t n) {
    int b = 1;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

}  // namespace

namespace {
constexpr size_t au256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace bytes of one ordering of n points (kd: the KD-tree's extra arrays).
constexpr size_t ws_bytes_for(int64_t n, bool kd) {
    return n <= 0 ? 256
                  : 256                                                                       // flag
                        + au256(sizeof(uint32_t) * (size_t)((n + kSortTile - 1) / kSortTile) * kBuckets)  // hist
                        + 2 * au256(sizeof(uint64_t) * (size_t)n)                             // keys, keys_alt
                        + 2 * au256(sizeof(int32_t) * (size_t)n)                              // vals, vals_alt
                        + (kd ? 2 * au256(sizeof(int32_t) * (size_t)n)                        // rank_x, rank_y
                                    + 2 * au256(sizeof(unsigned long long) * 2 * (size_t)n)   // seg min/max
                              : 0);
}
}  // namespace

size_t reorder_ws_bytes(int64_t n, tlr_ordering kind) { return ws_bytes_for(n, kind == TLR_ORDER_KDTREE); }

tlr_status reorder(const double *d_locs, int64_t n, tlr_ordering kind, uint64_t seed, uint32_t flags,
                   int32_t *d_perm, void *d_ws, size_t ws_bytes, hipStream_t s) {
    (void)flags;
    if (n < 0 || (n > 0 && (!d_locs || !d_perm))) return TLR_E_INVAL;
    if (n > (int64_t)0x7fffffff) return TLR_E_UNSUPPORTED;
    if ((int)kind < 0 || (int)kind > 4) return TLR_E_INVAL;
    if (n == 0) return TLR_OK;
    if (!d_ws || ws_bytes < reorder_ws_bytes(n, kind)) return TLR_E_NOMEM;

    char *w = static_cast<char *>(d_ws);
    int *d_bad = reinterpret_cast<int *>(w);
    w += 256;
    const int64_t nblocks = cdiv(n, kSortTile);
    uint32_t *hist = reinterpret_cast<uint32_t *>(w);
    w += align_up(sizeof(uint32_t) * nblocks * kBuckets, 256);
    uint64_t *keys = reinterpret_cast<uint64_t *>(w);
    w += align_up(sizeof(uint64_t) * n, 256);
    uint64_t *keys_alt = reinterpret_cast<uint64_t *>(w);
    w += align_up(sizeof(uint64_t) * n, 256);
    int32_t *vals = reinterpret_cast<int32_t *>(w);
    w += align_up(sizeof(int32_t) * n, 256);
    int32_t *vals_alt = reinterpret_cast<int32_t *>(w);
    w += align_up(sizeof(int32_t) * n, 256);

    const dim3 blk(256), grd((unsigned)cdiv(n, 256));
    // domain check (synchronous): every coordinate in [0,1], no NaN
    TLR_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_check_domain, grd, blk, 0, s, d_locs, n, d_bad);
    int bad = 0;
    TLR_HIP(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    TLR_HIP(hipStreamSynchronize(s));
    if (bad) return TLR_E_DOMAIN;

    if (kind == TLR_ORDER_NONE) {
        hipLaunchKernelGGL(k_iota, grd, blk, 0, s, n, d_perm);
        TLR_HIP(hipGetLastError());
        return TLR_OK;
    }
    bool alt = false;
    if (kind == TLR_ORDER_MORTON || kind == TLR_ORDER_HILBERT) {
        uint32_t *k32 = reinterpret_cast<uint32_t *>(keys);
        uint32_t *k32_alt = reinterpret_cast<uint32_t *>(keys_alt);
        hipLaunchKernelGGL(k_curve_keys, grd, blk, 0, s, d_locs, n, (int)kind, k32, vals);
        TLR_TRY(radix_sort<uint32_t>(k32, vals, k32_alt, vals_alt, hist, n, 32, &alt, s));
    } else if (kind == TLR_ORDER_RANDOM) {
        hipLaunchKernelGGL(k_random_keys, grd, blk, 0, s, n, seed, keys, vals);
        TLR_TRY(radix_sort<uint64_t>(keys, vals, keys_alt, vals_alt, hist, n, 64, &alt, s));
    } else {  // KD-tree
        int32_t *rank_x = reinterpret_cast<int32_t *>(w);
        w += align_up(sizeof(int32_t) * n, 256);
        int32_t *rank_y = reinterpret_cast<int32_t *>(w);
        w += align_up(sizeof(int32_t) * n, 256);
        unsigned long long *mn = reinterpret_cast<unsigned long long *>(w);
        w += align_up(sizeof(unsigned long long) * 2 * n, 256);
        unsigned long long *mx = reinterpret_cast<unsigned long long *>(w);
        // global ranks along x and along y, ties by original index
        for (int d = 0; d < 2; ++d) {
            hipLaunchKernelGGL(k_coord_keys, grd, blk, 0, s, d_locs, n, d, keys, vals);
            TLR_TRY(radix_sort<uint64_t>(keys, vals, keys_alt, vals_alt, hist, n, 64, &alt, s));
            hipLaunchKernelGGL(k_scatter_rank, grd, blk, 0, s, alt ? vals_alt : vals, n,
                               d == 0 ? rank_x : rank_y);
        }
        // current arrangement: original order
        hipLaunchKernelGGL(k_iota, grd, blk, 0, s, n, vals_alt);
        int32_t *pts = vals_alt;
        const int levels = bits_for(n);
        const int rank_bits = bits_for(n + 1);
        const int key_bits = 2 * rank_bits;
        for (int level = 0; level < levels; ++level) {
            hipLaunchKernelGGL(k_seg_init, grd, blk, 0, s, n, mn, mx);
            hipLaunchKernelGGL(k_seg_bbox, grd, blk, 0, s, d_locs, pts, n, level, mn, mx);
            int32_t *other = (pts == vals_alt) ? vals : vals_alt;
            hipLaunchKernelGGL(k_seg_keys, grd, blk, 0, s, pts, n, level, mn, mx, rank_x, rank_y,
                               rank_bits, keys, other);
            // sort (keys, other) in place using (keys_alt, pts) as the alternate buffers
            bool a2 = false;
            TLR_TRY(radix_sort<uint64_t>(keys, other, keys_alt, pts, hist, n, key_bits, &a2, s));
            pts = a2 ? pts : other;
        }
        TLR_HIP(hipMemcpyAsync(d_perm, pts, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        TLR_HIP(hipGetLastError());
        return TLR_OK;
    }
    TLR_HIP(hipMemcpyAsync(d_perm, alt ? vals_alt : vals, sizeof(int32_t) * n,
                           hipMemcpyDeviceToDevice, s));
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

namespace {
__global__ void k_apply_perm(const int32_t *__restrict__ perm, int64_t n, const double *__restrict__ locs,
                             const double *__restrict__ z, double *__restrict__ locs_out,
                             double *__restrict__ z_out, int dequant) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int64_t src = perm[k];
    double x = locs[2 * src], y = locs[2 * src + 1];
    if (dequant) {
        x = (double)encode16(x) / 65535.0;
        y = (double)encode16(y) / 65535.0;
    }
    locs_out[2 * k] = x;
    locs_out[2 * k + 1] = y;
    if (z && z_out) z_out[k] = z[src];
}
}  // namespace

tlr_status apply_perm(const int32_t *d_perm, int64_t n, const double *d_locs, const double *d_z,
                      double *d_locs_out, double *d_z_out, int dequant, hipStream_t s) {
    if (n < 0) return TLR_E_INVAL;
    if (n == 0) return TLR_OK;
    if (!d_perm || !d_locs || !d_locs_out) return TLR_E_INVAL;
    if ((d_z == nullptr) != (d_z_out == nullptr)) return TLR_E_INVAL;
    if (d_locs == d_locs_out || (d_z && d_z == d_z_out)) return TLR_E_INVAL;  // no in-place gather
    hipLaunchKernelGGL(k_apply_perm, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, d_perm, n, d_locs,
                       d_z, d_locs_out, d_z_out, dequant);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

// ------------------------------------------ allocation-free ordering --
//
// The same ordering with its workspace in a file-scope device array, for
// callers that cannot allocate.  Each device holds its own copy of the array
// from the library's load to the end of the process; the host reaches it only
// through the address hipGetSymbolAddress returns on that device, taken on the
// first call there and kept per device.

constexpr int64_t kNoAllocMaxN = int64_t(1) << 17;
constexpr size_t kNoAllocBytes = ws_bytes_for(kNoAllocMaxN, true);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};
}  // namespace

int64_t reorder_noalloc_max_n() { return kNoAllocMaxN; }

tlr_status reorder_noalloc(const double *d_locs, int64_t n, tlr_ordering kind, uint64_t seed, uint32_t flags,
                           int32_t *d_perm, hipStream_t s) {
    if (n < 0 || (n > 0 && (!d_locs || !d_perm))) return TLR_E_INVAL;
    if ((int)kind < 0 || (int)kind > 4) return TLR_E_INVAL;
    if (n > kNoAllocMaxN) return TLR_E_NOMEM;
    if (n == 0) return TLR_OK;
    int dev = 0;
    TLR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return TLR_E_UNSUPPORTED;
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> g(g_scratch_mu);
        if (!g_scratch[dev]) {
            void *ptr = nullptr;
            TLR_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr) return TLR_E_HIP;
            g_scratch[dev] = ptr;
        }
        ws = g_scratch[dev];
    }
    return reorder(d_locs, n, kind, seed, flags, d_perm, ws, kNoAllocBytes, s);
}

}  // namespace tlr
