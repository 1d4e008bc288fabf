// Device-wide stable radix sort of (key, u32 value) pairs and exclusive sums,
// written for gfx950 (wave64): the event stream orders its records by these
// (sections "Sorting Events using the Water-Level Algorithm" and "Reporting
// Coalescence Events Independently").
//
// Sort: least-significant-digit passes of 8 bits.  A pass is three launches
// over tiles of 4096 items (256 threads x 16 rows of 256):
//   1. k_radix_hist: each tile counts its digits in LDS and writes the 256
//      counts digit-major (hist[digit * tiles + tile]);
//   2. an exclusive sum over that array turns the counts into each tile's first
//      output position per digit (digit-major order keeps the pass stable);
//   3. k_radix_scatter: each tile walks its rows in order; within a row a wave
//      finds the lanes that share its digit with eight ballots (one per digit
//      bit), ranks itself among them, adds the counts of the earlier waves of
//      the row and the tile's running position for that digit, and writes the
//      pair there.
// Passes alternate between the caller's output buffers and a scratch copy so
// that the last pass writes the output; the input is never written.
//
// Exclusive sum: per tile of 4096 items a sum (k_scan_tile_sums), the sums
// scanned the same way one level up (recursively), then each tile scanned in
// LDS from its offset (k_scan_tile).  A tile is scanned in place safely: it is
// read whole into LDS before it is written.
#include "stream_sort.h"

#include <algorithm>

namespace nh_sort {
namespace {

constexpr uint32_t kThreads = 256;             // 4 waves
constexpr uint32_t kRows = 16;
constexpr uint32_t kTile = kThreads * kRows;   // items per tile
constexpr uint32_t kBuckets = 256;             // 8-bit digits
constexpr uint32_t kWaves = kThreads / 64;

inline uint32_t tiles_of(uint32_t n) { return (n + kTile - 1) / kTile; }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename K>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const K *__restrict__ keys, uint32_t n, uint32_t shift,
                                                         uint32_t *__restrict__ hist, uint32_t tiles) {
    __shared__ uint32_t h[kBuckets];
    const uint32_t t = threadIdx.x;
    h[t] = 0u;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
#pragma unroll 4
    for (uint32_t r = 0; r < kRows; ++r) {
        const uint64_t i = base + (uint64_t)r * kThreads + t;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & (kBuckets - 1u)], 1u);
    }
    __syncthreads();
    hist[(uint64_t)t * tiles + blockIdx.x] = h[t];
}

template <typename K>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const K *__restrict__ k_in, const uint32_t *__restrict__ v_in,
                                                            K *__restrict__ k_out, uint32_t *__restrict__ v_out,
                                                            uint32_t n, uint32_t shift,
                                                            const uint32_t *__restrict__ offs, uint32_t tiles) {
    __shared__ uint32_t run[kBuckets];          // the tile's next output position per digit
    __shared__ uint32_t cnt[kWaves][kBuckets];  // per wave: pairs of each digit in the current row
    const uint32_t t = threadIdx.x, wave = t / 64u, lane = t % 64u;
    run[t] = offs[(uint64_t)t * tiles + blockIdx.x];
#pragma unroll
    for (uint32_t w = 0; w < kWaves; ++w) cnt[w][t] = 0u;
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    for (uint32_t r = 0; r < kRows; ++r) {
        const uint64_t i = base + (uint64_t)r * kThreads + t;
        const bool valid = i < n;
        const K key = valid ? k_in[i] : (K)0;
        const uint32_t val = valid ? v_in[i] : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & (kBuckets - 1u);
        // lanes of this wave holding the same digit (ballot per digit bit)
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (uint32_t b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & below);
        if (valid && rank == 0u) cnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        uint32_t pos = run[d] + rank;
        for (uint32_t w = 0; w < wave; ++w) pos += cnt[w][d];
        __syncthreads();
        uint32_t total = 0;
#pragma unroll
        for (uint32_t w = 0; w < kWaves; ++w) {
            total += cnt[w][t];
            cnt[w][t] = 0u;
        }
        run[t] += total;
        __syncthreads();
        if (valid) {
            k_out[pos] = key;
            v_out[pos] = val;
        }
    }
}

// Sum of a wave's values over lanes <= this lane.
template <typename T>
__device__ __forceinline__ T wave_inclusive(T x) {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_tile_sums(const T *__restrict__ in, uint32_t n, T *__restrict__ sums) {
    __shared__ T part[kWaves];
    const uint32_t t = threadIdx.x;
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    T s = 0;
    for (uint32_t r = 0; r < kRows; ++r) {
        const uint64_t i = base + (uint64_t)r * kThreads + t;
        if (i < n) s += in[i];
    }
    s = wave_inclusive(s);
    if (t % 64u == 63u) part[t / 64u] = s;
    __syncthreads();
    if (t == 0) {
        T total = 0;
        for (uint32_t w = 0; w < kWaves; ++w) total += part[w];
        sums[blockIdx.x] = total;
    }
}

// Exclusive sum of one tile plus the tile's offset (offsets == nullptr: 0).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_tile(const T *in, T *out, uint32_t n, const T *offsets) {
    __shared__ T items[kTile];
    __shared__ T part[kWaves];
    const uint32_t t = threadIdx.x;
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    for (uint32_t r = 0; r < kRows; ++r) { // coalesced load of the whole tile
        const uint64_t i = base + (uint64_t)r * kThreads + t;
        items[r * kThreads + t] = i < n ? in[i] : (T)0;
    }
    __syncthreads();
    // thread t owns items [16 t, 16 t + 16)
    T own = 0;
#pragma unroll
    for (uint32_t k = 0; k < kRows; ++k) own += items[t * kRows + k];
    const T incl = wave_inclusive(own);
    if (t % 64u == 63u) part[t / 64u] = incl;
    __syncthreads();
    T run = (offsets ? offsets[blockIdx.x] : (T)0) + incl - own;
    for (uint32_t w = 0; w < t / 64u; ++w) run += part[w];
#pragma unroll
    for (uint32_t k = 0; k < kRows; ++k) {
        const T x = items[t * kRows + k];
        items[t * kRows + k] = run;
        run += x;
    }
    __syncthreads();
    for (uint32_t r = 0; r < kRows; ++r) {
        const uint64_t i = base + (uint64_t)r * kThreads + t;
        if (i < n) out[i] = items[r * kThreads + t];
    }
}

// Scratch of an exclusive sum over n items: the tile sums of every level and their scans.
template <typename T>
size_t scan_bytes(uint32_t n) {
    size_t b = 0;
    while (n > kTile) {
        const uint32_t nt = tiles_of(n);
        b += 2 * align256(sizeof(T) * nt);
        n = nt;
    }
    return b;
}

template <typename T>
hipError_t scan(const T *in, T *out, uint32_t n, char *tmp, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const uint32_t nt = tiles_of(n);
    if (nt == 1) {
        k_scan_tile<T><<<1, kThreads, 0, stream>>>(in, out, n, nullptr);
        return hipGetLastError();
    }
    T *sums = (T *)tmp;
    T *offs = (T *)(tmp + align256(sizeof(T) * nt));
    char *rest = tmp + 2 * align256(sizeof(T) * nt);
    k_scan_tile_sums<T><<<nt, kThreads, 0, stream>>>(in, n, sums);
    if (hipError_t e = hipGetLastError()) return e;
    if (hipError_t e = scan<T>(sums, offs, nt, rest, stream)) return e;
    k_scan_tile<T><<<nt, kThreads, 0, stream>>>(in, out, n, offs);
    return hipGetLastError();
}

template <typename T>
hipError_t exclusive_sum(void *tmp, size_t &tmp_bytes, const T *in, T *out, uint32_t n, hipStream_t stream) {
    const size_t need = std::max<size_t>(scan_bytes<T>(n), 256);
    if (!tmp) {
        tmp_bytes = need;
        return hipSuccess;
    }
    if (tmp_bytes < need) return hipErrorInvalidValue;
    return scan<T>(in, out, n, (char *)tmp, stream);
}

template <typename K>
hipError_t sort_pairs(void *tmp, size_t &tmp_bytes, const K *k_in, K *k_out, const uint32_t *v_in, uint32_t *v_out,
                      uint32_t n, int end_bit, hipStream_t stream) {
    const uint32_t tiles = tiles_of(std::max<uint32_t>(n, 1));
    const size_t b_keys = align256(sizeof(K) * (size_t)std::max<uint32_t>(n, 1));
    const size_t b_vals = align256(sizeof(uint32_t) * (size_t)std::max<uint32_t>(n, 1));
    const uint32_t n_hist = kBuckets * tiles;
    const size_t b_hist = align256(sizeof(uint32_t) * (size_t)n_hist);
    const size_t need = b_keys + b_vals + b_hist + scan_bytes<uint32_t>(n_hist);
    if (!tmp) {
        tmp_bytes = need;
        return hipSuccess;
    }
    if (tmp_bytes < need) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    char *p = (char *)tmp;
    K *k_alt = (K *)p;
    uint32_t *v_alt = (uint32_t *)(p + b_keys);
    uint32_t *hist = (uint32_t *)(p + b_keys + b_vals);
    char *scan_tmp = p + b_keys + b_vals + b_hist;
    const uint32_t bits = (uint32_t)std::max(1, std::min<int>(end_bit, 8 * (int)sizeof(K)));
    const uint32_t passes = (bits + 7u) / 8u;
    const K *ks = k_in;
    const uint32_t *vs = v_in;
    for (uint32_t q = 0; q < passes; ++q) {
        // the last pass writes the caller's output; earlier ones alternate back from it
        const bool to_out = ((passes - 1u - q) % 2u) == 0u;
        K *kd = to_out ? k_out : k_alt;
        uint32_t *vd = to_out ? v_out : v_alt;
        const uint32_t shift = 8u * q;
        k_radix_hist<K><<<tiles, kThreads, 0, stream>>>(ks, n, shift, hist, tiles);
        if (hipError_t e = hipGetLastError()) return e;
        if (hipError_t e = scan<uint32_t>(hist, hist, n_hist, scan_tmp, stream)) return e;
        k_radix_scatter<K><<<tiles, kThreads, 0, stream>>>(ks, vs, kd, vd, n, shift, hist, tiles);
        if (hipError_t e = hipGetLastError()) return e;
        ks = kd;
        vs = vd;
    }
    return hipSuccess;
}

} // namespace

hipError_t sort_pairs_u64(void *tmp, size_t &tmp_bytes, const uint64_t *k_in, uint64_t *k_out, const uint32_t *v_in,
                          uint32_t *v_out, uint32_t n, int end_bit, hipStream_t stream) {
    return sort_pairs<uint64_t>(tmp, tmp_bytes, k_in, k_out, v_in, v_out, n, end_bit, stream);
}

hipError_t sort_pairs_u32(void *tmp, size_t &tmp_bytes, const uint32_t *k_in, uint32_t *k_out, const uint32_t *v_in,
                          uint32_t *v_out, uint32_t n, int end_bit, hipStream_t stream) {
    return sort_pairs<uint32_t>(tmp, tmp_bytes, k_in, k_out, v_in, v_out, n, end_bit, stream);
}

hipError_t exclusive_sum_u64(void *tmp, size_t &tmp_bytes, const uint64_t *in, uint64_t *out, uint32_t n,
                             hipStream_t stream) {
    return exclusive_sum<uint64_t>(tmp, tmp_bytes, in, out, n, stream);
}

hipError_t exclusive_sum_u32(void *tmp, size_t &tmp_bytes, const uint32_t *in, uint32_t *out, uint32_t n,
                             hipStream_t stream) {
    return exclusive_sum<uint32_t>(tmp, tmp_bytes, in, out, n, stream);
}

} // namespace nh_sort
