// Stable least-significant-digit radix sort and device-wide prefix sums.
//
// Layout: a fixed grid of kWorkers blocks; worker b owns one contiguous slice
// of the input (whole tiles of kTile keys), so every pass is
//   hist    : per-worker digit counts            -> hist[digit][worker]
//   scan    : exclusive scan of each digit's row -> hist (in place), dtotal
//   scatter : stable rank inside the worker's slice, write to
//             digit base + hist[digit][worker] + rank
// The element count may live in device memory (count_ptr), so a sort whose
// length is only known on the device needs no host round trip.
#pragma once

#include "common.h"

namespace plmss {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;  // == kBlock: one thread per digit
constexpr int kWorkers = 1024;
constexpr int kItems = 16;               // keys per thread per tile
constexpr int kTile = kBlock * kItems;
static_assert(kRadix == kBlock, "one thread per digit");

__device__ __forceinline__ uint32_t load_count(const uint32_t* count_ptr, uint32_t n) {
    return count_ptr ? *count_ptr : n;
}

// Slice [lo, hi) of worker b out of nworkers, in whole tiles.
__device__ __forceinline__ void worker_range(uint32_t count, uint32_t b, uint32_t nworkers,
                                             uint32_t tile, uint32_t* lo, uint32_t* hi) {
    const uint32_t tiles = (count + tile - 1) / tile;
    const uint32_t per = (tiles + nworkers - 1) / nworkers;
    const uint64_t l = uint64_t(b) * per * tile, h = l + uint64_t(per) * tile;
    *lo = l < count ? uint32_t(l) : count;
    *hi = h < count ? uint32_t(h) : count;
}

// ---- key sources ---------------------------------------------------------------

// Keys of a float field (order-preserving transform), values = vertex ids.
template <typename T, typename K>
struct FieldSrc {
    using key_t = K;
    const T* f;
    __device__ __forceinline__ K key(uint32_t i) const { return sos_key(f[i]); }
    __device__ __forceinline__ uint32_t val(uint32_t i) const { return i; }
    __device__ __forceinline__ bool nan(uint32_t i) const { return is_nan(f[i]); }
};

template <typename K>
struct ArraySrc {
    using key_t = K;
    const K* keys;
    const uint32_t* vals;
    __device__ __forceinline__ K key(uint32_t i) const { return keys[i]; }
    __device__ __forceinline__ uint32_t val(uint32_t i) const { return vals[i]; }
    __device__ __forceinline__ bool nan(uint32_t) const { return false; }
};

// ---- destinations ----------------------------------------------------------------

template <typename K>
struct ArrayDst {
    K* keys;
    uint32_t* vals;
    __device__ __forceinline__ void put(uint32_t pos, K k, uint32_t v) const {
        keys[pos] = k;
        vals[pos] = v;
    }
};

// Final pass of the order field: the value is the vertex id, the position its
// rank.
template <typename K>
struct RankDst {
    int32_t* order;
    __device__ __forceinline__ void put(uint32_t pos, K, uint32_t v) const {
        order[v] = int32_t(pos);
    }
};

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift) {
    return uint32_t(k >> shift) & (kRadix - 1);
}

// Lanes of the wave whose digit equals this lane's (only lanes with valid set).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

// ---- kernels -----------------------------------------------------------------------

template <class Src, bool CHECK_NAN>
__global__ __launch_bounds__(kBlock) void k_radix_hist(Src src, const uint32_t* count_ptr,
                                                       uint32_t n, int shift, uint32_t* hist,
                                                       int32_t* info) {
    __shared__ uint32_t h[kWavesPerBlock][kRadix];
    __shared__ int nan_seen;
    const int t = threadIdx.x, w = wave_id();
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) h[i][t] = 0;
    if (t == 0) nan_seen = 0;
    __syncthreads();
    uint32_t lo, hi;
    worker_range(load_count(count_ptr, n), blockIdx.x, gridDim.x, kTile, &lo, &hi);
    bool bad = false;
    for (uint32_t i = lo + t; i < hi; i += kBlock) {
        atomicAdd(&h[w][digit_of(src.key(i), shift)], 1u);
        if (CHECK_NAN) bad |= src.nan(i);
    }
    if (CHECK_NAN && bad) nan_seen = 1;
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) s += h[i][t];
    hist[size_t(t) * gridDim.x + blockIdx.x] = s;
    if (CHECK_NAN && t == 0 && nan_seen && info) info[0] = -4;  // PLMSS_E_NAN
}

// One block per digit: exclusive scan of hist[d][0..workers) in place; dtotal[d]
// receives the row sum.
__global__ __launch_bounds__(kBlock) void k_radix_digit_scan(uint32_t* hist, uint32_t* dtotal,
                                                             int workers) {
    __shared__ uint32_t tmp[kWavesPerBlock];
    uint32_t* row = hist + size_t(blockIdx.x) * workers;
    const int per = (workers + kBlock - 1) / kBlock;
    const int beg = threadIdx.x * per;
    uint32_t s = 0;
    for (int i = 0; i < per; ++i)
        if (beg + i < workers) s += row[beg + i];
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, tmp, &tot);
    for (int i = 0; i < per; ++i) {
        if (beg + i < workers) {
            const uint32_t c = row[beg + i];
            row[beg + i] = run;
            run += c;
        }
    }
    if (threadIdx.x == 0) dtotal[blockIdx.x] = tot;
}

template <class Src, class Dst>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(Src src, Dst dst,
                                                          const uint32_t* count_ptr, uint32_t n,
                                                          int shift, const uint32_t* hist,
                                                          const uint32_t* dtotal) {
    using K = typename Src::key_t;
    __shared__ uint32_t run[kRadix];
    __shared__ uint32_t wcnt[kWavesPerBlock][kRadix];
    __shared__ uint32_t tmp[kWavesPerBlock];
    const int t = threadIdx.x, w = wave_id(), lane = lane_id();
    uint32_t tot;
    const uint32_t base = block_exclusive_scan(dtotal[t], tmp, &tot);
    run[t] = base + hist[size_t(t) * gridDim.x + blockIdx.x];
    uint32_t lo, hi;
    worker_range(load_count(count_ptr, n), blockIdx.x, gridDim.x, kTile, &lo, &hi);
    const uint64_t lt = lanemask_lt();
    for (uint32_t tile = lo; tile < hi; tile += kTile) {
#pragma unroll
        for (int i = 0; i < kWavesPerBlock; ++i) wcnt[i][t] = 0;
        __syncthreads();
        K key[kItems];
        uint32_t val[kItems], dig[kItems], local[kItems];
        const uint32_t wbase = tile + uint32_t(w) * kWave * kItems + lane;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t idx = wbase + uint32_t(i) * kWave;
            const bool valid = idx < hi;
            key[i] = valid ? src.key(idx) : K(0);
            val[i] = valid ? src.val(idx) : 0u;
            dig[i] = valid ? digit_of(key[i], shift) : 0u;
            const uint64_t peers = match_digit(dig[i], valid);
            uint32_t prior = 0;
            if (valid) prior = wcnt[w][dig[i]];
            local[i] = prior + uint32_t(__popcll(peers & lt));
            // the highest peer lane publishes the new count for this digit
            if (valid && (peers >> lane) == 1ull) wcnt[w][dig[i]] = prior + uint32_t(__popcll(peers));
        }
        __syncthreads();
        {
            uint32_t acc = run[t];
#pragma unroll
            for (int i = 0; i < kWavesPerBlock; ++i) {
                const uint32_t c = wcnt[i][t];
                wcnt[i][t] = acc;
                acc += c;
            }
            run[t] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t idx = wbase + uint32_t(i) * kWave;
            if (idx < hi) dst.put(wcnt[w][dig[i]] + local[i], key[i], val[i]);
        }
        __syncthreads();
    }
}

// ---- device-wide exclusive prefix sums over uint32 ---------------------------------

// partial[b] = sum of in[lo..hi) over worker b's slice.
__global__ __launch_bounds__(kBlock) void k_sum_reduce(const uint32_t* in,
                                                       const uint32_t* count_ptr, uint32_t n,
                                                       uint32_t* partial) {
    __shared__ uint32_t tmp[kWavesPerBlock];
    uint32_t lo, hi;
    worker_range(load_count(count_ptr, n), blockIdx.x, gridDim.x, kBlock, &lo, &hi);
    uint32_t s = 0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kBlock) s += in[i];
    uint32_t tot;
    block_exclusive_scan(s, tmp, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One block: exclusive scan of partial[0..m) in place; *total = the sum.
__global__ __launch_bounds__(kBlock) void k_scan_partials(uint32_t* partial, int m,
                                                          uint32_t* total) {
    __shared__ uint32_t tmp[kWavesPerBlock];
    const int per = (m + kBlock - 1) / kBlock;
    const int beg = threadIdx.x * per;
    uint32_t s = 0;
    for (int i = 0; i < per; ++i)
        if (beg + i < m) s += partial[beg + i];
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, tmp, &tot);
    for (int i = 0; i < per; ++i) {
        if (beg + i < m) {
            const uint32_t c = partial[beg + i];
            partial[beg + i] = run;
            run += c;
        }
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

}  // namespace plmss
