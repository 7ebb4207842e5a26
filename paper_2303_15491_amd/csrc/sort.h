// Stable least-significant-digit radix sort and device-wide prefix sums.
//
// Every pass is a histogram and a scatter over the same grid of "workers"
// (blocks, numbered XCD by XCD), with a digit scan between them; worker b
// owns one contiguous slice of whole kTile-key tiles:
//   hist    : per-worker digit counts            -> hist[digit][worker]
//   scan    : exclusive scan of each digit's row -> hist (in place), dtotal
//             (long rows are split over up to 16 blocks each)
//   scatter : stable rank inside each tile, staged through LDS so that each
//             digit's run leaves the block as one contiguous write, at
//             digit base + hist[digit][worker] + rank
// With a host-known length the grid can have one worker per tile.  The length
// may instead live in device memory (count_ptr) with a fixed grid, so a sort
// whose size only the device knows needs no host round trip.
#pragma once

#include "common.h"

namespace plmss {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;  // == kBlock: one thread per digit
constexpr int kItems = 16;               // keys per thread per tile
constexpr int kTile = kBlock * kItems;
constexpr int kWorkers = 512;            // default grid of device-sized sorts and scans
constexpr int kMaxWorkers = 4096;        // largest such grid (sizes the workspace)
static_assert(kRadix == kBlock, "one thread per digit");

__device__ __forceinline__ uint32_t load_count(const uint32_t* count_ptr, uint32_t n) {
    return count_ptr ? *count_ptr : n;
}

// Radix workers are numbered with xcd_block: neighbouring workers write
// neighbouring parts of every digit's output range, and with each XCD
// holding one contiguous run of workers the cache lines two neighbours share
// stay in one XCD's L2, where their partial writes merge.
__device__ __forceinline__ uint32_t xcd_worker() { return xcd_block(blockIdx.x, gridDim.x); }

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

// Loads of a pass's input, which the pass reads exactly once.  Over a whole
// field (NT) they are non-temporal: streamed past the caches, they do not
// push out the partial lines that the pass's scattered writes are still
// filling (middle passes of a 512^3 order field 0.55 -> 0.46 ms, its
// histograms 0.24 -> 0.19 ms).  A source small enough to stay in the
// memory-side cache from one pass to the next (the listed pairs of the MS
// ids) keeps ordinary loads, which were faster there.
template <bool NT, typename T>
__device__ __forceinline__ T pass_load(const T* p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

// Keys of a float field (order-preserving transform), values = vertex ids.
template <typename T, typename K>
struct FieldSrc {
    using key_t = K;
    const T* f;
    __device__ __forceinline__ K key(uint32_t i) const { return sos_key(pass_load<true>(f + i)); }
    __device__ __forceinline__ uint32_t val(uint32_t i) const { return i; }
    // NaN test on the transformed key, so the value is loaded once
    __device__ __forceinline__ static bool nan_key(K k) { return key_is_nan(k); }
};

template <typename K, bool NT = true>
struct ArraySrc {
    using key_t = K;
    const K* keys;
    const uint32_t* vals;
    __device__ __forceinline__ K key(uint32_t i) const { return pass_load<NT>(keys + i); }
    __device__ __forceinline__ uint32_t val(uint32_t i) const { return pass_load<NT>(vals + i); }
    __device__ __forceinline__ static bool nan_key(key_t) { return false; }
};

// Keys whose value is their own index (a list in its original order): the
// value is generated, not read.
template <typename K, bool NT = true>
struct IndexValSrc {
    using key_t = K;
    const K* keys;
    __device__ __forceinline__ K key(uint32_t i) const { return pass_load<NT>(keys + i); }
    __device__ __forceinline__ uint32_t val(uint32_t i) const { return i; }
    __device__ __forceinline__ static bool nan_key(key_t) { return false; }
};

// 32-bit keys and their ids packed in one word, key in the high half: one
// load and one store per item, and one output stream per digit.
struct PackedSrc {
    using key_t = uint32_t;
    const uint64_t* kv;
    __device__ __forceinline__ uint32_t key(uint32_t i) const { return uint32_t(pass_load<true>(kv + i) >> 32); }
    __device__ __forceinline__ uint32_t val(uint32_t i) const { return uint32_t(pass_load<true>(kv + i)); }
    __device__ __forceinline__ static bool nan_key(key_t) { return false; }
};

struct PackedDst {
    uint64_t* kv;
    __device__ __forceinline__ void put(uint32_t pos, uint32_t k, uint32_t v) const {
        kv[pos] = (uint64_t(k) << 32) | v;
    }
};

// One item of a source: key and value from a single read of its storage.
template <typename T, typename K>
__device__ __forceinline__ void load_item(const FieldSrc<T, K>& s, uint32_t i, K& k, uint32_t& v) {
    k = s.key(i);
    v = i;
}
template <typename K, bool NT>
__device__ __forceinline__ void load_item(const ArraySrc<K, NT>& s, uint32_t i, K& k, uint32_t& v) {
    k = s.key(i);
    v = s.val(i);
}
template <typename K, bool NT>
__device__ __forceinline__ void load_item(const IndexValSrc<K, NT>& s, uint32_t i, K& k, uint32_t& v) {
    k = s.key(i);
    v = i;
}
__device__ __forceinline__ void load_item(const PackedSrc& s, uint32_t i, uint32_t& k, uint32_t& v) {
    const uint64_t x = pass_load<true>(s.kv + i);
    k = uint32_t(x >> 32);
    v = uint32_t(x);
}

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

// 64-bit keys whose low half is sorted: the high half packed with the id in
// one word (key in the high word), for passes over PackedSrc.
struct HighPackedDst {
    uint64_t* kv;
    __device__ __forceinline__ void put(uint32_t pos, uint64_t k, uint32_t v) const {
        kv[pos] = (k & 0xffffffff00000000ull) | v;
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

// Last pass of the order field when the inversion runs separately: only the
// vertex ids, in sorted order.
template <typename K>
struct IdDst {
    uint32_t* ids;
    __device__ __forceinline__ void put(uint32_t pos, K, uint32_t v) const { ids[pos] = v; }
};

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift) {
    return uint32_t(k >> shift) & (kRadix - 1);
}

// Lanes of the wave whose digit equals this lane's (only lanes with valid set).
// Per bit: s = all ones where this lane's bit is set, m = the wave's ballot of
// that bit; a lane keeps the lanes where m agrees with s, ~(m ^ s).
// Two forms.  The plain one leaves the compiler free to schedule (it ballots
// a shifted copy of the digit and folds the eight terms with three-input ORs).
// The SHORT one issues a sixth fewer VALU instructions: the ballot tests s
// itself (hidden from the compiler, which would otherwise test a second
// shifted copy) and each bit takes one three-input bit operation per 32-bit
// half (truth table 0x84: the middle operand AND (first XNOR last), the same
// whichever end of the table index the first operand sits at), but each step
// then waits on the one before.  SHORT is faster in the passes bound by
// instruction issue (the first pass, which also transforms the field values,
// and the last, which also groups by id range: 0.396 -> 0.380 and 0.531 ->
// 0.512 ms at 512^3), slower in the middle passes (0.46 -> 0.49 ms each).
template <bool SHORT>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    const uint64_t v = __ballot(valid);
    uint32_t lo = uint32_t(v), hi = uint32_t(v >> 32);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        uint32_t s = uint32_t(int32_t(d << (31 - b)) >> 31);
        if constexpr (SHORT) {
            asm("" : "+v"(s));
            const uint64_t m = __ballot(s != 0u);
            lo = __builtin_amdgcn_bitop3_b32(uint32_t(m), lo, s, 0x84);
            hi = __builtin_amdgcn_bitop3_b32(uint32_t(m >> 32), hi, s, 0x84);
        } else {
            const uint64_t m = __ballot(s != 0u);
            lo &= ~(uint32_t(m) ^ s);
            hi &= ~(uint32_t(m >> 32) ^ s);
        }
    }
    return (uint64_t(hi) << 32) | lo;
}

// Sources of field values (the first pass of an order sort).
template <class S>
struct is_field_src : std::false_type {};
template <typename T, typename K>
struct is_field_src<FieldSrc<T, K>> : std::true_type {};

// Highest lane of a non-empty lane set.
__device__ __forceinline__ int top_lane(uint64_t m) { return 63 - __clzll(static_cast<long long>(m)); }

// ---- kernels -----------------------------------------------------------------------

// IDS: also counts the values (vertex ids) per id range, id >> id_shift, into
// ihist (same layout), for the last pass of the order field.
template <class Src, bool CHECK_NAN, bool IDS = false>
__global__ __launch_bounds__(kBlock) void k_radix_hist(Src src, const uint32_t* count_ptr,
                                                       uint32_t n, int shift, uint32_t* hist,
                                                       int32_t* info, int id_shift = 0,
                                                       uint32_t* ihist = nullptr) {
    using K = typename Src::key_t;
    __shared__ uint32_t h[kWavesPerBlock][kRadix];
    __shared__ uint32_t hi_ids[IDS ? kWavesPerBlock : 1][kRadix];
    __shared__ int nan_seen;
    const int t = threadIdx.x, w = wave_id();
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) h[i][t] = 0;
    if (IDS) {
#pragma unroll
        for (int i = 0; i < kWavesPerBlock; ++i) hi_ids[IDS ? i : 0][t] = 0;
    }
    if (t == 0) nan_seen = 0;
    __syncthreads();
    uint32_t lo, hi;
    const uint32_t wk = xcd_worker();
    worker_range(load_count(count_ptr, n), wk, gridDim.x, kTile, &lo, &hi);
    bool bad = false;
    for (uint32_t tile = lo; tile < hi; tile += kTile) {
        if constexpr (std::is_same<Src, PackedSrc>::value) {
            // counting order is free: each lane reads two consecutive packed
            // items per 16-byte load (key in the high word).  A pair starting
            // at or past the slice end reads the slice's last even pair
            // instead and counts nothing.
            constexpr int kPairs = kItems / 2;
            const uint32_t last = (hi - 1u) & ~1u;
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
            u32x4 x[kPairs];
#pragma unroll
            for (int j = 0; j < kPairs; ++j) {
                const uint32_t first = tile + uint32_t(j * kBlock + t) * 2u;
                x[j] = pass_load<true>(reinterpret_cast<const u32x4*>(src.kv + min(first, last)));
            }
            // keep each load 16 bytes wide when the ids are not counted (the
            // compiler would otherwise narrow it to the two key words)
#pragma unroll
            for (int j = 0; j < kPairs; ++j) asm volatile("" : "+v"(x[j]));
#pragma unroll
            for (int j = 0; j < kPairs; ++j) {
                const uint32_t first = tile + uint32_t(j * kBlock + t) * 2u;
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    if (first + uint32_t(k) < hi) {
                        const uint32_t kk = k ? x[j].w : x[j].y, vv = k ? x[j].z : x[j].x;
                        atomicAdd(&h[w][digit_of(kk, shift)], 1u);
                        if (IDS) atomicAdd(&hi_ids[IDS ? w : 0][vv >> id_shift], 1u);
                    }
                }
            }
            continue;
        }
        K key[kItems];
        uint32_t val[kItems];
        // every load reads a valid element (the index is clamped to the
        // slice), so all of them are issued before the first is waited for;
        // items past the slice are masked afterwards
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t idx = min(tile + uint32_t(i) * kBlock + t, hi - 1u);
            if (IDS)
                load_item(src, idx, key[i], val[i]);
            else
                key[i] = src.key(idx);
        }
#pragma unroll
        for (int i = 0; i < kItems; ++i)
            if (CHECK_NAN && tile + uint32_t(i) * kBlock + t < hi) bad |= Src::nan_key(key[i]);
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t idx = tile + uint32_t(i) * kBlock + t;
            if (idx < hi) {
                atomicAdd(&h[w][digit_of(key[i], shift)], 1u);
                if (IDS) atomicAdd(&hi_ids[IDS ? w : 0][val[i] >> id_shift], 1u);
            }
        }
    }
    if (CHECK_NAN && bad) nan_seen = 1;
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) s += h[i][t];
    hist[size_t(t) * gridDim.x + wk] = s;
    if (IDS) {
        uint32_t c = 0;
#pragma unroll
        for (int i = 0; i < kWavesPerBlock; ++i) c += hi_ids[IDS ? i : 0][t];
        ihist[size_t(t) * gridDim.x + wk] = c;
    }
    if (CHECK_NAN && t == 0 && nan_seen && info) info[0] = -4;  // PLMSS_E_NAN
}

// Exclusive scan of each digit's row hist[d][0..workers) in place; dtotal[d]
// receives the row sum.  A long row is split into nseg segments of seglen
// entries, one block each (block b: digit b / nseg, segment b % nseg):
// k_digit_seg_sum adds up every segment into segsum[b], then
// k_radix_digit_scan scans each segment starting from the sum of the
// segments before it.  With nseg = 1 the second kernel alone scans the row.
constexpr int kSegment = 2048;     // preferred segment length
constexpr int kMaxSegments = 16;   // kRadix x 16 segment sums fit u32[kMaxWorkers]

__global__ __launch_bounds__(kBlock) void k_digit_seg_sum(const uint32_t* hist, int workers, int nseg, int seglen,
                                                          uint32_t* segsum) {
    __shared__ uint32_t tmp[kWavesPerBlock];
    const int d = blockIdx.x / nseg, sg = blockIdx.x % nseg;
    const uint32_t* row = hist + size_t(d) * workers;
    const int lo = sg * seglen, hi = min(lo + seglen, workers);
    uint32_t sum = 0;
    for (int base = lo; base < hi; base += kBlock * 4) {
        uint32_t c[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = row[min(base + i * kBlock + int(threadIdx.x), hi - 1)];
#pragma unroll
        for (int i = 0; i < 4; ++i) sum += base + i * kBlock + int(threadIdx.x) < hi ? c[i] : 0u;
    }
    uint32_t tot;
    block_exclusive_scan(sum, tmp, &tot);
    if (threadIdx.x == 0) segsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_radix_digit_scan(uint32_t* hist, uint32_t* dtotal, int workers,
                                                             int nseg, int seglen, const uint32_t* segsum) {
    __shared__ uint32_t tmp[kWavesPerBlock];
    const int d = blockIdx.x / nseg, sg = blockIdx.x % nseg;
    uint32_t* row = hist + size_t(d) * workers;
    const int lo = sg * seglen, hi = min(lo + seglen, workers);
    uint32_t run = 0, total = 0;
    for (int k = 0; k < nseg && nseg > 1; ++k) {
        const uint32_t v = segsum[d * nseg + k];
        run += k < sg ? v : 0u;
        total += v;
    }
    for (int base = lo; base < hi; base += kBlock * 4) {
        // four consecutive entries per thread per round, loads issued together
        const int beg = base + threadIdx.x * 4;
        uint32_t c[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = row[min(beg + i, hi - 1)];
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = beg + i < hi ? c[i] : 0u;
        uint32_t tot;
        uint32_t e = run + block_exclusive_scan(c[0] + c[1] + c[2] + c[3], tmp, &tot);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (beg + i < hi) row[beg + i] = e;
            e += c[i];
        }
        run += tot;
    }
    if (threadIdx.x == 0 && sg == 0) dtotal[d] = nseg > 1 ? total : run;
}

// The per-wave digit counters (and then offsets) hold at most a wave's 1024
// keys of a tile, and a digit's start and count in the tile at most 4096: two
// 16-bit halves share one word (waves 2i and 2i + 1; start low, count high),
// which with 64-bit keys brings the block to 52 KB of LDS, three per CU.
template <typename K>
struct ScatterSmem {
    K keys[kTile];
    uint32_t vals[kTile];
    uint32_t wcnt[kWavesPerBlock / 2][kRadix];
    uint32_t run[kRadix];
    uint32_t tspan[kRadix];
    uint32_t tmp[kWavesPerBlock];
};
static_assert(kItems * kWave < (1 << 16) && kTile < (1 << 16), "16-bit halves");

// 32-bit keys: four blocks per CU, 64-bit keys three (the LDS allows that
// many; the register budget of the unrolled tile is held to it)
template <class Src, class Dst>
__global__ __launch_bounds__(kBlock, sizeof(typename Src::key_t) == 4 ? 4 : 3) void k_radix_scatter(Src src, Dst dst,
                                                          const uint32_t* count_ptr, uint32_t n,
                                                          int shift, const uint32_t* hist,
                                                          const uint32_t* dtotal) {
    using K = typename Src::key_t;
    __shared__ ScatterSmem<K> sm;
    const int t = threadIdx.x, w = wave_id(), lane = lane_id();
    uint32_t tot;
    const uint32_t base = block_exclusive_scan(dtotal[t], sm.tmp, &tot);
    const uint32_t wk = xcd_worker();
    sm.run[t] = base + hist[size_t(t) * gridDim.x + wk];
    uint32_t lo, hi;
    worker_range(load_count(count_ptr, n), wk, gridDim.x, kTile, &lo, &hi);
    const uint64_t lt = lanemask_lt();
    // wave w owns keys [w*64*kItems, (w+1)*64*kItems) of a tile, row i of the
    // wave holds 64 consecutive keys: (w, i, lane) is the input order.  Loads
    // use indices clamped into the slice, so all of a tile's loads issue
    // before the first wait; a tile's loads are issued while the tile before
    // it is still being written out.
    K key[kItems];
    uint32_t val[kItems];
    auto load_tile = [&](uint32_t tl) {
        const uint32_t base = tl + uint32_t(w) * kWave * kItems + lane;
#pragma unroll
        for (int i = 0; i < kItems; ++i) load_item(src, min(base + uint32_t(i) * kWave, hi - 1u), key[i], val[i]);
    };
    auto step = [&](uint32_t tile) {
        const uint32_t tsize = min(uint32_t(kTile), hi - tile);
#pragma unroll
        for (int i = 0; i < kWavesPerBlock / 2; ++i) sm.wcnt[i][t] = 0;
        const uint32_t wbase = tile + uint32_t(w) * kWave * kItems + lane;
        const uint32_t half = 16u * uint32_t(w & 1);  // this wave's half of its counter words
        __syncthreads();
        // rank inside the wave: the highest lane of each digit group adds the
        // group's size to the wave's counter and gets the count before it;
        // the adds of all rows are issued back to back (LDS keeps a wave's
        // operations in order), then each group reads its leader's result
        // local[i]: the rank among the row's peers, with the group's leader
        // lane in bits 8-13 until the leader's count is read back
        uint32_t local[kItems], prior[kItems];
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t idx = wbase + uint32_t(i) * kWave;
            const bool valid = idx < hi;
            const uint32_t d = digit_of(key[i], shift);
            const uint64_t peers = match_digit<is_field_src<Src>::value>(d, valid);
            const int leader = peers ? top_lane(peers) : lane;
            local[i] = uint32_t(__popcll(peers & lt)) | (uint32_t(leader) << 8);
            prior[i] = 0;
            if (valid && leader == lane)
                prior[i] = (atomicAdd(&sm.wcnt[w >> 1][d], uint32_t(__popcll(peers)) << half) >> half) & 0xffffu;
        }
#pragma unroll
        for (int i = 0; i < kItems; ++i)
            local[i] = (local[i] & 0xffu) + uint32_t(__shfl(int(prior[i]), int(local[i] >> 8)));
        __syncthreads();
        {
            uint32_t c[kWavesPerBlock], sum = 0;
#pragma unroll
            for (int i = 0; i < kWavesPerBlock; ++i) {
                c[i] = (sm.wcnt[i >> 1][t] >> (16 * (i & 1))) & 0xffffu;
                sum += c[i];
            }
            uint32_t ttot;
            uint32_t acc = block_exclusive_scan(sum, sm.tmp, &ttot);
            sm.tspan[t] = acc | (sum << 16);
#pragma unroll
            for (int i = 0; i < kWavesPerBlock; i += 2) {
                sm.wcnt[i >> 1][t] = acc | ((acc + c[i]) << 16);
                acc += c[i] + c[i + 1];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t idx = wbase + uint32_t(i) * kWave;
            if (idx < hi) {
                const uint32_t p =
                    ((sm.wcnt[w >> 1][digit_of(key[i], shift)] >> half) & 0xffffu) + local[i];
                sm.keys[p] = key[i];
                sm.vals[p] = val[i];
            }
        }
        // the items are in LDS: their registers take the next tile
        if (tile + kTile < hi) load_tile(tile + kTile);
        __syncthreads();
        // every thread stores kItems items: past the tile's end it repeats
        // the tile's last item (same address, same value), so the number of
        // stores after the next tile's loads is fixed and waiting for those
        // loads does not wait for the stores
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t j = min(uint32_t(i) * kBlock + t, tsize - 1u);
            const K k = sm.keys[j];
            const uint32_t d = digit_of(k, shift);
            dst.put(sm.run[d] + (j - (sm.tspan[d] & 0xffffu)), k, sm.vals[j]);
        }
        __syncthreads();
        sm.run[t] += sm.tspan[t] >> 16;
    };
    // the first tile is peeled off, so that every pass through the loop
    // starts with the same memory operations in flight
    if (lo < hi) {
        load_tile(lo);
        step(lo);
    }
    for (uint32_t tile = lo + kTile; tile < hi; tile += kTile) step(tile);
}

// Last pass of the order field without a scattered write over the whole
// order array: each key's sorted position comes from the same stable rank by
// the top digit as in k_radix_scatter, and the pair (id, position) is then
// written to one of at most 256 id ranges (id >> id_shift), from which
// k_chunk_partition and k_invert_chunks write order[] one chunk at a time.  ihist/itotal: the per-worker id-range
// counts and their totals (k_radix_hist with IDS, then the digit scan).
template <class Src>
__global__ __launch_bounds__(kBlock, 3) void k_rank_partition(Src src, const uint32_t* count_ptr, uint32_t n, int shift,
                                                           const uint32_t* hist, const uint32_t* dtotal,
                                                           const uint32_t* ihist, const uint32_t* itotal,
                                                           int id_shift, uint64_t* out) {
    using K = typename Src::key_t;
    __shared__ uint32_t wcnt[kWavesPerBlock][kRadix];
    __shared__ uint32_t run[kRadix], tstart[kRadix], tcount[kRadix];
    __shared__ uint32_t irun[kRadix], istart[kRadix], icount[kRadix], ifill[kRadix];
    __shared__ uint64_t stage[kTile];
    __shared__ uint32_t tmp[kWavesPerBlock];
    const int t = threadIdx.x, w = wave_id(), lane = lane_id();
    uint32_t tot;
    const uint32_t wk = xcd_worker();
    run[t] = block_exclusive_scan(dtotal[t], tmp, &tot) + hist[size_t(t) * gridDim.x + wk];
    irun[t] = block_exclusive_scan(itotal[t], tmp, &tot) + ihist[size_t(t) * gridDim.x + wk];
    uint32_t lo, hi;
    worker_range(load_count(count_ptr, n), wk, gridDim.x, kTile, &lo, &hi);
    const uint64_t lt = lanemask_lt();
    // tiles are loaded as in k_radix_scatter: clamped indices, and the next
    // tile's loads issued before the current tile is written out
    K key[kItems];
    uint32_t val[kItems];
    auto load_tile = [&](uint32_t tl) {
        const uint32_t base = tl + uint32_t(w) * kWave * kItems + lane;
#pragma unroll
        for (int i = 0; i < kItems; ++i) load_item(src, min(base + uint32_t(i) * kWave, hi - 1u), key[i], val[i]);
    };
    auto step = [&](uint32_t tile) {
        const uint32_t tsize = min(uint32_t(kTile), hi - tile);
#pragma unroll
        for (int i = 0; i < kWavesPerBlock; ++i) wcnt[i][t] = 0;
        icount[t] = 0;
        ifill[t] = 0;
        const uint32_t wbase = tile + uint32_t(w) * kWave * kItems + lane;
        __syncthreads();
        uint32_t local[kItems], prior[kItems];
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t idx = wbase + uint32_t(i) * kWave;
            const bool valid = idx < hi;
            const uint32_t d = digit_of(key[i], shift);
            const uint64_t peers = match_digit<true>(d, valid);
            const int leader = peers ? top_lane(peers) : lane;
            local[i] = uint32_t(__popcll(peers & lt)) | (uint32_t(leader) << 8);
            prior[i] = 0;
            if (valid && leader == lane) prior[i] = atomicAdd(&wcnt[w][d], uint32_t(__popcll(peers)));
            if (valid) atomicAdd(&icount[val[i] >> id_shift], 1u);
        }
#pragma unroll
        for (int i = 0; i < kItems; ++i)
            local[i] = (local[i] & 0xffu) + uint32_t(__shfl(int(prior[i]), int(local[i] >> 8)));
        __syncthreads();
        {
            uint32_t c[kWavesPerBlock], sum = 0;
#pragma unroll
            for (int i = 0; i < kWavesPerBlock; ++i) {
                c[i] = wcnt[i][t];
                sum += c[i];
            }
            uint32_t ttot;
            uint32_t acc = block_exclusive_scan(sum, tmp, &ttot);
            tstart[t] = acc;
            tcount[t] = sum;
#pragma unroll
            for (int i = 0; i < kWavesPerBlock; ++i) {
                wcnt[i][t] = acc;
                acc += c[i];
            }
            istart[t] = block_exclusive_scan(icount[t], tmp, &ttot);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t idx = wbase + uint32_t(i) * kWave;
            if (idx < hi) {
                const uint32_t d = digit_of(key[i], shift);
                const uint32_t pos = run[d] + (wcnt[w][d] + local[i] - tstart[d]);
                const uint32_t r = val[i] >> id_shift;
                const uint32_t slot = istart[r] + atomicAdd(&ifill[r], 1u);
                stage[slot] = (uint64_t(val[i]) << 32) | pos;
            }
        }
        if (tile + kTile < hi) load_tile(tile + kTile);
        __syncthreads();
        // stores as in k_radix_scatter: kItems per thread, the last item
        // repeated past the tile's end
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t j = min(uint32_t(i) * kBlock + t, tsize - 1u);
            const uint64_t x = stage[j];
            const uint32_t r = uint32_t(x >> 32) >> id_shift;
            out[irun[r] + (j - istart[r])] = x;
        }
        __syncthreads();
        run[t] += tcount[t];
        irun[t] += icount[t];
    };
    if (lo < hi) {
        load_tile(lo);
        step(lo);
    }
    for (uint32_t tile = lo + kTile; tile < hi; tile += kTile) step(tile);
}

// The inversion order[id] = position by id chunks of kChunk ids, each
// inverted inside one block's LDS so that order[] is written in whole
// coalesced rows.  The pairs reach their chunk in two regroupings with long
// write runs: k_rank_partition groups them by range (id >> range_shift: at
// most 256 ranges of 1 to 256 chunks), k_chunk_partition by chunk inside the
// ranges.  A chunk c holds exactly min(kChunk, n - c*kChunk) pairs (the ids
// are a permutation), so its pairs go to [c*kChunk, c*kChunk + that count).
constexpr int kChunkBits = 15;
constexpr uint32_t kChunk = 1u << kChunkBits;  // 128 KB of order per block
constexpr int kMaxRel = 512;                   // chunks a tile can touch: two ranges of <= 256
constexpr int kInvertBlock = 1024;

__device__ __forceinline__ uint32_t chunk_count(uint32_t c, uint32_t n) {
    const uint32_t base = c << kChunkBits;
    return min(kChunk, n - base);
}

// chunk_fill: u32 per chunk, zero on entry.  Grid: one block per kTile pairs
// (of the length count_ptr points to, when given, or n; blocks past it exit).
// Every pair has a place by construction (the ids are a permutation, ranges
// other than the last hold at least kTile ids); a pair that found none all
// the same sets *bad, which the inversion reports instead of a silently
// wrong order field.
__global__ __launch_bounds__(kBlock) void k_chunk_partition(const uint64_t* parts, const uint32_t* count_ptr,
                                                            uint32_t n_host, int range_shift,
                                                            uint32_t* chunk_fill, uint64_t* out, uint32_t* bad) {
    __shared__ uint32_t cnt[kMaxRel], start[kMaxRel], base[kMaxRel], fill[kMaxRel];
    __shared__ uint64_t stage[kTile];
    __shared__ uint32_t tmp[kWavesPerBlock];
    __shared__ uint32_t s_first;
    const int t = threadIdx.x;
    const uint32_t n = load_count(count_ptr, n_host);
    // tiles numbered XCD by XCD, so that tiles reserving neighbouring runs
    // of a chunk mostly share an L2
    const uint32_t lo = xcd_worker() * uint32_t(kTile);
    if (lo >= n) return;  // the whole block: no barrier has been passed yet
    const uint32_t hi = min(n, lo + uint32_t(kTile));
    for (int i = t; i < kMaxRel; i += kBlock) {
        cnt[i] = 0;
        fill[i] = 0;
    }
    // first chunk of the range the tile starts in (pairs are grouped by range)
    if (t == 0) s_first = ((uint32_t(parts[lo] >> 32) >> range_shift) << (range_shift - kChunkBits));
    __syncthreads();
    const uint32_t first = s_first;
    uint64_t x[kItems];
    uint32_t rel[kItems];
#pragma unroll
    for (int i = 0; i < kItems; ++i) x[i] = parts[min(lo + uint32_t(i) * kBlock + t, hi - 1u)];
    bool lost = false;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const uint32_t j = lo + uint32_t(i) * kBlock + t;
        rel[i] = j < hi ? (uint32_t(x[i] >> 32) >> kChunkBits) - first : uint32_t(kMaxRel);
        if (rel[i] < uint32_t(kMaxRel))
            atomicAdd(&cnt[rel[i]], 1u);
        else if (j < hi)
            lost = true;
    }
    __syncthreads();
    constexpr int kPer = kMaxRel / kBlock;
    uint32_t c[kPer], sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        c[k] = cnt[t * kPer + k];
        sum += c[k];
    }
    uint32_t tot;
    uint32_t e = block_exclusive_scan(sum, tmp, &tot);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        start[t * kPer + k] = e;
        base[t * kPer + k] = c[k] ? atomicAdd(&chunk_fill[first + uint32_t(t * kPer + k)], c[k]) : 0u;
        e += c[k];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kItems; ++i)
        if (rel[i] < uint32_t(kMaxRel)) stage[start[rel[i]] + atomicAdd(&fill[rel[i]], 1u)] = x[i];
    __syncthreads();
    const uint32_t tsize = hi > lo ? hi - lo : 0u;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const uint32_t j = uint32_t(i) * kBlock + t;
        if (j < tsize) {
            const uint64_t y = stage[j];
            const uint32_t ch = uint32_t(y >> 32) >> kChunkBits;
            const uint32_t r = ch - first;
            const uint32_t slot = base[r] + (j - start[r]);
            if (slot < chunk_count(ch, n))
                out[(size_t(ch) << kChunkBits) + slot] = y;
            else
                lost = true;
        }
    }
    if (lost) atomicOr(bad, 1u);
}

// One block per chunk: order[c*kChunk + i] for the chunk's pairs, through LDS.
// A pair lost by the regrouping (*bad) is reported in info[0] (nullable) as
// PLMSS_E_INTERNAL.
__global__ __launch_bounds__(kInvertBlock) void k_invert_chunks(const uint64_t* parts, uint32_t n, int32_t* order,
                                                                const uint32_t* bad, int32_t* info) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && info && *bad) info[0] = -8;  // PLMSS_E_INTERNAL
    __shared__ uint32_t buf[kChunk];
    const uint32_t base = blockIdx.x << kChunkBits;
    const uint32_t cnt = chunk_count(blockIdx.x, n);
    constexpr int kBatch = 8;
    for (uint32_t j0 = 0; j0 < cnt; j0 += uint32_t(kInvertBlock * kBatch)) {
        uint64_t x[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const uint32_t j = j0 + uint32_t(k * kInvertBlock) + threadIdx.x;
            x[k] = j < cnt ? parts[base + j] : ~0ull;
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const uint32_t r = uint32_t(x[k] >> 32) - base;
            if (x[k] != ~0ull && r < cnt) buf[r] = uint32_t(x[k]);
        }
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < cnt; j += kInvertBlock) order[base + j] = int32_t(buf[j]);
}

__global__ void k_zero_u32(uint32_t* p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// order[ids[i]] = i for the ids in [lo, hi): the inversion of the sorted ids,
// restricted to one window of the id range so that the scattered writes of
// one launch stay within a region the memory-side cache can hold.
__global__ __launch_bounds__(kBlock) void k_invert(const uint32_t* ids, uint32_t n, uint32_t lo,
                                                   uint32_t hi, int32_t* order) {
    const uint32_t base = blockIdx.x * uint32_t(kTile) + threadIdx.x;
    uint32_t v[kItems];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const uint32_t j = base + uint32_t(i) * kBlock;
        v[i] = j < n ? ids[j] : 0xffffffffu;
    }
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        const uint32_t j = base + uint32_t(i) * kBlock;
        if (v[i] - lo < hi - lo) order[v[i]] = int32_t(j);
    }
}

// ---- device-wide exclusive prefix sums over uint32 ---------------------------------

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
