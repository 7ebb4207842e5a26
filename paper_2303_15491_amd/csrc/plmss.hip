// libplmss: C ABI of the gfx950 Morse-Smale segmentation (see include/plmss.h).
#include "plmss.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <mutex>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "marching.h"
#include "order_batch.h"
#include "segment.h"
#include "sort.h"

using namespace plmss;

namespace {

constexpr int64_t kMaxN = 2147483647;  // int32 labels

// ---- launch-shape knobs (results never depend on them) ------------------------------
struct KnobRange {
    int64_t lo, hi, def;
    bool zero_ok, pow2;
};
constexpr KnobRange kKnobs[PLMSS_TUNE_KNOBS] = {
    {64, 1 << 16, 0, true, false},             // ORDER_WORKERS: 0 = one block per tile
    {1, 64, 1, true, false},                   // ORDER_INVERT: 0 fused, 1 id ranges, 2.. windows
    {64, kMaxWorkers, kWorkers, false, false},  // SORT_WORKERS
    {64, 16384, 2048, false, false},           // PERSIST_BLOCKS
    {8, 32, 16, false, true},                  // SCAN_DEPTH: 8, 16 or 32 planes
    {1, 1, 1, true, false},                    // ORDER_PACKED: 32-bit keys packed with ids
    {1, 8, kResolveRounds, false, false},      // SCAN_ROUNDS: in-tile jumping sweeps
    {1, 1, 0, true, false},                    // ORDER_CONCURRENT: order field on a second stream
    {1, 1, 1, true, false},                    // PACKED_CODES: rank and code in one word when they fit
    {0, 2, 2, false, false},                   // PAIR_STREAM: 0 cached, 1 streamed, 2 streamed for batches
};
std::atomic<int64_t> g_knob[PLMSS_TUNE_KNOBS] = {kKnobs[0].def, kKnobs[1].def, kKnobs[2].def,
                                                 kKnobs[3].def, kKnobs[4].def, kKnobs[5].def,
                                                 kKnobs[6].def, kKnobs[7].def, kKnobs[8].def, kKnobs[9].def};

int64_t knob(int k) { return g_knob[k].load(std::memory_order_relaxed); }
unsigned sort_workers() { return unsigned(knob(PLMSS_TUNE_SORT_WORKERS)); }
unsigned persist_blocks() { return unsigned(knob(PLMSS_TUNE_PERSIST_BLOCKS)); }
int scan_depth() { return int(knob(PLMSS_TUNE_SCAN_DEPTH)); }
int scan_rounds() { return int(knob(PLMSS_TUNE_SCAN_ROUNDS)); }

constexpr size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int bit_width(uint64_t x) {
    int b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

// Bits of one vertex id in a pair key: ids are < n.
int id_bits(uint64_t n) { return std::max(1, bit_width(n - 1)); }

int check_dims(const plmss_dims& d, uint64_t* n_out) {
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) return PLMSS_E_DIMS;
    if (d.nx > kMaxN || d.ny > kMaxN || d.nz > kMaxN) return PLMSS_E_TOO_LARGE;
    const uint64_t nxy = uint64_t(d.nx) * uint64_t(d.ny);
    if (nxy > uint64_t(kMaxN)) return PLMSS_E_TOO_LARGE;
    const uint64_t n = nxy * uint64_t(d.nz);
    if (n > uint64_t(kMaxN)) return PLMSS_E_TOO_LARGE;
    *n_out = n;
    return PLMSS_OK;
}

// ---- shape classes ------------------------------------------------------------------
// 3-D fields (nz > 1) use 64x8xZC scan tiles (ZC = the scan depth, 8, 16 or
// 32 planes) and 32x8x8 chase tiles; planar fields (nz == 1) 64x16 and 64x32;
// lines (ny == nz == 1) 64x16 and 2048x1.
constexpr int kClasses = 3;
int class_of(const plmss_dims& d) { return d.nz > 1 ? 0 : (d.ny > 1 ? 1 : 2); }

uint32_t s_tiles_of(const plmss_dims& d, int zc) {
    return class_of(d) == 0 ? steepest_tiles(d.nx, d.ny, d.nz, 8, zc) : steepest_tiles(d.nx, d.ny, d.nz, 16, 1);
}

uint32_t j_tiles_of(const plmss_dims& d) {
    switch (class_of(d)) {
        case 0: return chase_tiles<JTile3>(d.nx, d.ny, d.nz);
        case 1: return chase_tiles<JTile2>(d.nx, d.ny, d.nz);
        default: return chase_tiles<JTile1>(d.nx, d.ny, d.nz);
    }
}

// ---- workspace ----------------------------------------------------------------------

struct Work {
    uint8_t* keys[2];    // u64[npad] each: sort keys (ping-pong).  keys[0] also
                         // holds the tile-compressed pointers U, D (u32[npad]
                         // each) and keys[1] the listed MS pairs (at most one
                         // per vertex)
    uint32_t* vals[2];   // u32[npad] each: sort values
    uint32_t* rank_of;   // u32[npad]: MS id of each listed pair (dense index)
    uint32_t* hist;      // u32[kRadix * max(kMaxWorkers, ntiles)]
    uint32_t* dtotal;    // u32[kRadix]
    uint32_t* partial;   // u32[kMaxWorkers]
    uint32_t* counters;  // u32[64]: [0] = #pairs listed, [1] = K, [32..63] batch totals
    uint32_t* sortaux;   // u32[kSortAux]: order sort, id-range totals and chunk fill counters
    uint32_t* fbase;     // u32[nfields]: first MS id of each field
    FieldDesc* tables;   // batch tables: all fields, then one slot range per class
    uint64_t npad;
};

struct Sizes {
    size_t keys, vals, rank, hist, dtotal, partial, counters, sortaux, fbase, tables, total;
    uint64_t npad;
};

// Order-sort bookkeeping: totals of the id ranges, then one fill counter per
// id chunk (at most 2^31 / kChunk), then the regrouping's lost-pair flag.
constexpr size_t kSortAux = kRadix + (size_t(1) << (31 - kChunkBits)) + 1;

constexpr uint64_t n_tiles(uint64_t n) { return (n + kTile - 1) / kTile; }

// nv vertices; table_stride > 0 reserves batch tables of that many entries per
// range (all fields + 3 classes).
constexpr Sizes work_sizes(uint64_t nv, uint64_t nfields, uint64_t table_stride) {
    Sizes s{};
    s.npad = align_up(std::max<uint64_t>(nv, 1), kBlock);
    s.keys = align_up(8 * s.npad, 256);
    s.vals = align_up(4 * s.npad, 256);
    s.rank = align_up(4 * s.npad, 256);
    s.hist = align_up(size_t(4) * kRadix * std::max<uint64_t>(kMaxWorkers, n_tiles(nv)), 256);
    s.dtotal = align_up(4 * kRadix, 256);
    s.partial = align_up(4 * kMaxWorkers, 256);
    s.counters = 256;
    s.sortaux = align_up(4 * kSortAux, 256);
    s.fbase = align_up(4 * std::max<uint64_t>(nfields, 1), 256);
    s.tables = table_stride ? align_up(sizeof(FieldDesc) * 4 * table_stride, 256) : 0;
    s.total = 2 * s.keys + 2 * s.vals + s.rank + s.hist + s.dtotal + s.partial +
              s.counters + s.sortaux + s.fbase + s.tables;
    return s;
}

Work carve(void* ws, const Sizes& s) {
    Work w;
    uint8_t* p = static_cast<uint8_t*>(ws);
    auto take = [&](size_t bytes) {
        uint8_t* q = p;
        p += bytes;
        return q;
    };
    w.keys[0] = take(s.keys);
    w.keys[1] = take(s.keys);
    w.vals[0] = reinterpret_cast<uint32_t*>(take(s.vals));
    w.vals[1] = reinterpret_cast<uint32_t*>(take(s.vals));
    w.rank_of = reinterpret_cast<uint32_t*>(take(s.rank));
    w.hist = reinterpret_cast<uint32_t*>(take(s.hist));
    w.dtotal = reinterpret_cast<uint32_t*>(take(s.dtotal));
    w.partial = reinterpret_cast<uint32_t*>(take(s.partial));
    w.counters = reinterpret_cast<uint32_t*>(take(s.counters));
    w.sortaux = reinterpret_cast<uint32_t*>(take(s.sortaux));
    w.fbase = reinterpret_cast<uint32_t*>(take(s.fbase));
    w.tables = s.tables ? reinterpret_cast<FieldDesc*>(take(s.tables)) : nullptr;
    w.npad = s.npad;
    return w;
}

bool ws_ok(const void* ws, size_t have, size_t need) {
    return ws != nullptr && have >= need && (reinterpret_cast<uintptr_t>(ws) % 256) == 0;
}

int launch_status() { return hipGetLastError() == hipSuccess ? PLMSS_OK : PLMSS_E_HIP; }

unsigned grid_for(uint64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

// ---- marching index sizes -------------------------------------------------------------------
// Rows of cells: the (y, z) rows of cubes of a 3-D grid, the y rows of squares
// of a 2-D one (nz == 1), none for lines and for grids one vertex thick.
int64_t march_rows(const plmss_dims& d) {
    if (d.nx > 1 && d.ny > 1 && d.nz > 1) return (d.ny - 1) * (d.nz - 1);
    if (d.nz == 1 && d.nx > 1 && d.ny > 1) return d.ny - 1;
    return 0;
}

// One u64 per count block (its sum, then its first offset).
uint64_t march_blocks(uint64_t rows) {
    const uint64_t rpb = uint64_t(march_rows_per_wave(rows)) * kWavesPerBlock;
    return (rows + rpb - 1) / rpb;
}

size_t march_ws_bytes(uint64_t rows) { return align_up(8 * std::max<uint64_t>(1, march_blocks(rows)), 256); }

// ---- optional launch tracing -------------------------------------------------------------
// While a trace is active on the calling host thread, every kernel launch is
// bracketed by two hipEvents recorded on the launch stream.

struct Trace {
    hipEvent_t* ev = nullptr;  // 2 per launch
    int32_t* kind = nullptr;
    int32_t cap = 0;
    int32_t n = 0;
};

thread_local Trace* g_trace = nullptr;

template <typename F>
void launch(int kind, hipStream_t s, F&& f) {
    Trace* t = g_trace;
    const bool rec = t && t->n < t->cap;
    if (rec) (void)hipEventRecord(t->ev[2 * t->n], s);
    f();
    if (rec) {
        (void)hipEventRecord(t->ev[2 * t->n + 1], s);
        t->kind[t->n++] = kind;
    }
}

// ---- radix sort driver -------------------------------------------------------------------

// Trace kinds of one radix pass: histogram and scatter.
struct PassKinds {
    int hist, scatter;  // the digit scans are PLMSS_KERNEL_RADIX_SCAN
};
constexpr PassKinds kPairKinds{PLMSS_KERNEL_RADIX_HIST, PLMSS_KERNEL_RADIX_SCATTER};
constexpr PassKinds kOrderKinds{PLMSS_KERNEL_ORDER_HIST, PLMSS_KERNEL_ORDER_SCATTER};
static_assert(kRadix * kMaxSegments <= kMaxWorkers, "segment sums fit the partial buffer");

// Exclusive scan of the kRadix rows of `workers` entries in hist (row sums in
// dtotal), segmented over several blocks per row when rows are long; the
// segment sums go to w.partial.
void digit_scan(uint32_t* hist, uint32_t* dtotal, unsigned workers, const Work& w, hipStream_t s) {
    const int nseg = int(std::min<unsigned>(kMaxSegments, (workers + kSegment - 1) / kSegment));
    const int seglen = int((workers + unsigned(nseg) - 1) / unsigned(nseg));
    if (nseg > 1)
        launch(PLMSS_KERNEL_RADIX_SCAN, s, [&] {
            k_digit_seg_sum<<<kRadix * nseg, kBlock, 0, s>>>(hist, int(workers), nseg, seglen, w.partial);
        });
    launch(PLMSS_KERNEL_RADIX_SCAN, s, [&] {
        k_radix_digit_scan<<<kRadix * nseg, kBlock, 0, s>>>(hist, dtotal, int(workers), nseg, seglen, w.partial);
    });
}

// One pass over `workers` blocks; cnt (device) or n (host) is the length.
template <class Src, class Dst>
void radix_pass(Src src, Dst dst, const uint32_t* cnt, uint32_t n, unsigned workers, int shift,
                bool check_nan, const Work& w, int32_t* info, hipStream_t s, PassKinds kinds = kPairKinds,
                int scatter_kind = -1) {
    if (check_nan)
        launch(kinds.hist, s, [&] {
            k_radix_hist<Src, true><<<workers, kBlock, 0, s>>>(src, cnt, n, shift, w.hist, info);
        });
    else
        launch(kinds.hist, s, [&] {
            k_radix_hist<Src, false><<<workers, kBlock, 0, s>>>(src, cnt, n, shift, w.hist, info);
        });
    digit_scan(w.hist, w.dtotal, workers, w, s);
    launch(scatter_kind >= 0 ? scatter_kind : kinds.scatter, s, [&] {
        k_radix_scatter<Src, Dst><<<workers, kBlock, 0, s>>>(src, dst, cnt, n, shift, w.hist, w.dtotal);
    });
}

// Ping-pong storage of the order sort's (key, id) items: 32-bit keys packed
// with their ids in one word, or keys and ids in two arrays.  The packed form
// halves the write streams of a scatter, the split form halves what a
// histogram of keys alone reads; so the packed storage turns split for a last
// pass whose histogram reads only keys (the pass before it writes keys and
// ids into the two halves of one buffer).
struct PackedItems {
    uint64_t* kv[2];
    uint32_t* ids_buf;
    uint64_t npad;
    PackedSrc src(int c) const { return {kv[c]}; }
    PackedDst dst(int c) const { return {kv[c]}; }
    ArrayDst<uint32_t> split_dst(int c) const {
        uint32_t* k = reinterpret_cast<uint32_t*>(kv[c]);
        return {k, k + npad};
    }
    ArraySrc<uint32_t> last_src(int c) const {
        const uint32_t* k = reinterpret_cast<const uint32_t*>(kv[c]);
        return {k, k + npad};
    }
    uint64_t* spare(int c) const { return kv[c ^ 1]; }
    uint64_t* own(int c) const { return kv[c]; }
    uint32_t* ids(int) const { return ids_buf; }
};

template <typename K>
struct SplitItems {
    K* keys[2];
    uint32_t* vals[2];
    ArraySrc<K> src(int c) const { return {keys[c], vals[c]}; }
    ArrayDst<K> dst(int c) const { return {keys[c], vals[c]}; }
    ArrayDst<K> split_dst(int c) const { return dst(c); }
    ArraySrc<K> last_src(int c) const { return src(c); }
    uint64_t* spare(int c) const { return reinterpret_cast<uint64_t*>(keys[c ^ 1]); }
    uint64_t* own(int c) const { return reinterpret_cast<uint64_t*>(keys[c]); }
    uint32_t* ids(int c) const { return vals[c ^ 1]; }
};

// Last pass of the order field and the inversion by id chunks: the last
// pass writes (id, position) pairs grouped by id range to parts,
// k_chunk_partition regroups them by chunk into parts2, and the chunks are
// inverted in LDS: into `order` (one field), or through the descriptors of
// `batch` into each field's order array (batch != nullptr).  cnt: the length
// on the device (capacity launches; the grids are sized for n), or nullptr.
template <class Src>
void invert_by_chunks(Src src, const uint32_t* cnt, uint32_t n, unsigned workers, int last, uint64_t* parts,
                      uint64_t* parts2, int32_t* order, const Fields* batch, const Work& w, int32_t* info,
                      hipStream_t s) {
    // id ranges of 1 to 256 chunks, at most 64 of them below 2^29 vertices
    // (longer write runs) and 256 above; ihist (256 x workers <= npad
    // entries) in rank_of, which the order sort does not otherwise use
    const int id_shift = std::min(kChunkBits + 8, std::max(kChunkBits, bit_width(uint64_t(n) - 1) - 6));
    const unsigned tiles = unsigned(n_tiles(n));
    uint32_t* ihist = w.rank_of;
    uint32_t* itotal = w.sortaux;
    uint32_t* chunk_fill = w.sortaux + kRadix;
    const uint32_t chunks = uint32_t((uint64_t(n) + kChunk - 1) / kChunk);
    launch(PLMSS_KERNEL_ORDER_HIST, s, [&] {
        k_radix_hist<Src, false, true><<<workers, kBlock, 0, s>>>(src, cnt, n, last, w.hist, info, id_shift,
                                                                  ihist);
    });
    digit_scan(w.hist, w.dtotal, workers, w, s);
    digit_scan(ihist, itotal, workers, w, s);
    launch(PLMSS_KERNEL_ORDER_LAST, s, [&] {
        k_rank_partition<Src><<<workers, kBlock, 0, s>>>(src, cnt, n, last, w.hist, w.dtotal, ihist, itotal,
                                                         id_shift, parts);
    });
    uint32_t* bad = chunk_fill + chunks;  // set if the regrouping lost a pair
    launch(PLMSS_KERNEL_MISC, s, [&] {
        k_zero_u32<<<std::min(256u, (chunks + 1 + kBlock - 1) / kBlock), kBlock, 0, s>>>(chunk_fill, chunks + 1);
    });
    launch(PLMSS_KERNEL_ORDER_REGROUP, s, [&] {
        k_chunk_partition<<<tiles, kBlock, 0, s>>>(parts, cnt, n, id_shift, chunk_fill, parts2, bad);
    });
    if (batch)
        launch(PLMSS_KERNEL_ORDER_INVERT, s,
               [&] { k_invert_chunks_batch<<<chunks, kInvertBlock, 0, s>>>(parts2, cnt, n, *batch, bad); });
    else
        launch(PLMSS_KERNEL_ORDER_INVERT, s,
               [&] { k_invert_chunks<<<chunks, kInvertBlock, 0, s>>>(parts2, n, order, bad, info); });
}

// The passes of an order sort after its first: middle passes at shifts
// first_shift, first_shift + 8, ... below `last` over the items in buffer
// cur, then the last pass at shift `last` and order[id] = position, written
// in one of three ways (PLMSS_TUNE_ORDER_INVERT): fused into the last pass
// (scattered writes over the whole order array); by id chunk (the last pass
// writes (id, position) grouped by id range, k_chunk_partition regroups them
// by chunk of kChunk ids, k_invert_chunks inverts each chunk in LDS); or as
// sorted ids inverted by `windows` launches over parts of the id range.  K is
// the key type of the items.
template <typename K, class Items>
void order_tail(const Items& it, int cur, int first_shift, int last, uint32_t n, unsigned workers,
                int32_t* order, const Work& w, int32_t* info, hipStream_t s) {
    const unsigned tiles = unsigned(n_tiles(n));
    const int64_t inv = knob(PLMSS_TUNE_ORDER_INVERT);
    for (int shift = first_shift; shift < last; shift += kRadixBits) {
        // the by-chunk inversion's histogram reads the ids with the keys, so
        // the items stay as they are to the end; the other inversions'
        // histograms read only keys, which the pass before the last splits off
        if (shift + kRadixBits == last && inv != 1)
            radix_pass(it.src(cur), it.split_dst(cur ^ 1), nullptr, n, workers, shift, false, w, info, s,
                       kOrderKinds);
        else
            radix_pass(it.src(cur), it.dst(cur ^ 1), nullptr, n, workers, shift, false, w, info, s, kOrderKinds);
        cur ^= 1;
    }
    if (inv == 1) {
        // the pairs go to it.spare(cur); it.own(cur) is free once the last
        // pass has read it
        invert_by_chunks(it.src(cur), nullptr, n, workers, last, it.spare(cur), it.own(cur), order, nullptr, w,
                         info, s);
        return;
    }
    const auto src = it.last_src(cur);
    if (inv == 0) {
        radix_pass(src, RankDst<K>{order}, nullptr, n, workers, last, false, w, info, s, kOrderKinds,
                   PLMSS_KERNEL_ORDER_INVERT);
        return;
    }
    uint32_t* ids = it.ids(cur);
    radix_pass(src, IdDst<K>{ids}, nullptr, n, workers, last, false, w, info, s, kOrderKinds,
               PLMSS_KERNEL_ORDER_LAST);
    const uint32_t span = uint32_t((uint64_t(n) + uint64_t(inv) - 1) / uint64_t(inv));
    for (uint64_t lo = 0; lo < n; lo += span) {
        const uint32_t hi = uint32_t(std::min<uint64_t>(n, lo + span));
        launch(PLMSS_KERNEL_ORDER_INVERT, s,
               [&] { k_invert<<<tiles, kBlock, 0, s>>>(ids, n, uint32_t(lo), hi, order); });
    }
}

unsigned order_workers(uint32_t n) {
    const unsigned tiles = unsigned(n_tiles(n));
    const int64_t kw = knob(PLMSS_TUNE_ORDER_WORKERS);
    return kw == 0 ? tiles : unsigned(std::min<int64_t>(kw, tiles));
}

// Order field of a float field: an LSD radix sort of (key, id) with keys from
// the values (8-bit digits), then the inversion (order_tail).
template <typename T, typename K, class Items>
void sort_order_items(const T* f, uint32_t n, int32_t* order, const Work& w, int32_t* info, hipStream_t s,
                      const Items& it) {
    constexpr int passes = int(sizeof(K)) * 8 / kRadixBits;
    const unsigned workers = order_workers(n);
    radix_pass(FieldSrc<T, K>{f}, it.dst(0), nullptr, n, workers, 0, true, w, info, s, kOrderKinds,
               PLMSS_KERNEL_ORDER_FIRST);
    order_tail<K>(it, 0, kRadixBits, kRadixBits * (passes - 1), n, workers, order, w, info, s);
}

// 64-bit keys with packed items: the first four passes move (key, id) as a
// key array and an id array; the fourth writes each key's high half packed
// with its id in one word, and the last four passes sort those words like
// 32-bit keys (8 bytes an item instead of 12).
template <typename T>
void sort_order_wide_packed(const T* f, uint32_t n, int32_t* order, const Work& w, int32_t* info,
                            hipStream_t s) {
    const unsigned workers = order_workers(n);
    const SplitItems<uint64_t> sp{{reinterpret_cast<uint64_t*>(w.keys[0]), reinterpret_cast<uint64_t*>(w.keys[1])},
                                  {w.vals[0], w.vals[1]}};
    radix_pass(FieldSrc<T, uint64_t>{f}, sp.dst(0), nullptr, n, workers, 0, true, w, info, s, kOrderKinds,
               PLMSS_KERNEL_ORDER_FIRST);
    radix_pass(sp.src(0), sp.dst(1), nullptr, n, workers, kRadixBits, false, w, info, s, kOrderKinds);
    radix_pass(sp.src(1), sp.dst(0), nullptr, n, workers, 2 * kRadixBits, false, w, info, s, kOrderKinds);
    // keys[0]/vals[0] -> packed (high half, id) words in keys[1]
    radix_pass(sp.src(0), HighPackedDst{reinterpret_cast<uint64_t*>(w.keys[1])}, nullptr, n, workers,
               3 * kRadixBits, false, w, info, s, kOrderKinds);
    const PackedItems pk{{reinterpret_cast<uint64_t*>(w.keys[1]), reinterpret_cast<uint64_t*>(w.keys[0])},
                         w.vals[1], w.npad};
    order_tail<uint32_t>(pk, 0, 0, 3 * kRadixBits, n, workers, order, w, info, s);
}

template <typename T, typename K>
void sort_order(const T* f, uint32_t n, int32_t* order, const Work& w, int32_t* info, hipStream_t s) {
    if (knob(PLMSS_TUNE_ORDER_PACKED) != 0) {
        if constexpr (sizeof(K) == 4) {
            const PackedItems it{{reinterpret_cast<uint64_t*>(w.keys[0]), reinterpret_cast<uint64_t*>(w.keys[1])},
                                 w.vals[1], w.npad};
            sort_order_items<T, K>(f, n, order, w, info, s, it);
        } else {
            sort_order_wide_packed<T>(f, n, order, w, info, s);
        }
        return;
    }
    const SplitItems<K> it{{reinterpret_cast<K*>(w.keys[0]), reinterpret_cast<K*>(w.keys[1])},
                           {w.vals[0], w.vals[1]}};
    sort_order_items<T, K>(f, n, order, w, info, s, it);
}

void order_any(const void* field, int32_t dtype, uint32_t n, int32_t* order, const Work& w,
               int32_t* info, hipStream_t s) {
    if (dtype == PLMSS_F32)
        sort_order<float, uint32_t>(static_cast<const float*>(field), n, order, w, info, s);
    else
        sort_order<double, uint64_t>(static_cast<const double*>(field), n, order, w, info, s);
}

// Order fields of every field of a batch (order_batch.h): one sort of all the
// batch's vertices by (field index, key, id).  n: the vertices the grids are
// sized for (a capacity when cnt points to the batch's own total on the
// device); max_fields bounds the field indices.
template <typename T>
void order_batch_sort(const Fields& all, const uint32_t* cnt, uint32_t n, uint32_t max_fields, const Work& w,
                      hipStream_t s) {
    const unsigned tiles = unsigned(n_tiles(n));
    const unsigned workers = order_workers(n);
    uint64_t* kv0 = reinterpret_cast<uint64_t*>(w.keys[0]);
    uint64_t* kv1 = reinterpret_cast<uint64_t*>(w.keys[1]);
    const PackedItems pk{{kv0, kv1}, w.vals[1], w.npad};
    int cur = 0;
    int shift0 = 0;  // the key passes still to run on packed items start here
    if constexpr (sizeof(T) == 8) {
        // 64-bit keys: the low four digits as a key array and an id array
        // (the first pass generating the ids), the fourth pass packing each
        // key's high half with its id
        launch(PLMSS_KERNEL_ORDER_FIRST, s,
               [&] { k_batch_keys<T, uint64_t><<<tiles, kBlock, 0, s>>>(all, cnt, n, kv0); });
        const SplitItems<uint64_t> sp{{kv0, kv1}, {w.vals[0], w.vals[1]}};
        radix_pass(IndexValSrc<uint64_t>{kv0}, sp.dst(1), cnt, n, workers, 0, false, w, nullptr, s, kOrderKinds);
        radix_pass(sp.src(1), sp.dst(0), cnt, n, workers, kRadixBits, false, w, nullptr, s, kOrderKinds);
        radix_pass(sp.src(0), sp.dst(1), cnt, n, workers, 2 * kRadixBits, false, w, nullptr, s, kOrderKinds);
        radix_pass(sp.src(1), HighPackedDst{kv0}, cnt, n, workers, 3 * kRadixBits, false, w, nullptr, s,
                   kOrderKinds);
    } else {
        // 32-bit keys in a 4-byte array; the first pass generates the ids
        // and leaves (key, id) packed in one word
        launch(PLMSS_KERNEL_ORDER_FIRST, s,
               [&] { k_batch_keys<T, uint32_t><<<tiles, kBlock, 0, s>>>(all, cnt, n, w.vals[0]); });
        radix_pass(IndexValSrc<uint32_t>{w.vals[0]}, pk.dst(1), cnt, n, workers, 0, false, w, nullptr, s,
                   kOrderKinds);
        cur = 1;
        shift0 = kRadixBits;
    }
    for (int shift = shift0; shift < 32; shift += kRadixBits) {
        // the last key pass stores each item's field index in place of its key
        if (shift + kRadixBits < 32)
            radix_pass(pk.src(cur), pk.dst(cur ^ 1), cnt, n, workers, shift, false, w, nullptr, s, kOrderKinds);
        else
            radix_pass(pk.src(cur), PackedFieldDst{pk.kv[cur ^ 1], all}, cnt, n, workers, shift, false, w, nullptr,
                       s, kOrderKinds);
        cur ^= 1;
    }
    // the field index, most significant, one digit per pass
    const int fpasses = (std::max(1, bit_width(uint64_t(max_fields) - 1)) + kRadixBits - 1) / kRadixBits;
    for (int p = 0; p + 1 < fpasses; ++p) {
        radix_pass(pk.src(cur), pk.dst(cur ^ 1), cnt, n, workers, kRadixBits * p, false, w, nullptr, s,
                   kOrderKinds);
        cur ^= 1;
    }
    invert_by_chunks(pk.src(cur), cnt, n, workers, kRadixBits * (fpasses - 1), pk.spare(cur), pk.own(cur), nullptr,
                     &all, w, nullptr, s);
}

// Sorts the listed (asc, desc) pair keys (keys[1], record indices in vals[0];
// the count in counters[0], known only on the device).
struct PairList {
    const uint64_t* keys;
    const uint32_t* vals;
};

template <bool NT>
PairList sort_pairs_t(int bits, const Work& w, hipStream_t s) {
    const int passes = (bits + kRadixBits - 1) / kRadixBits;
    uint64_t* keys[2] = {reinterpret_cast<uint64_t*>(w.keys[1]), reinterpret_cast<uint64_t*>(w.keys[0])};
    uint32_t* vals[2] = {w.vals[0], w.vals[1]};
    // the listed records' values are their own indices: the first pass
    // generates them instead of reading them
    radix_pass(IndexValSrc<uint64_t, NT>{keys[0]}, ArrayDst<uint64_t>{keys[1], vals[1]}, w.counters, 0,
               sort_workers(), 0, false, w, nullptr, s);
    int cur = 1;
    for (int p = 1; p < passes; ++p) {
        radix_pass(ArraySrc<uint64_t, NT>{keys[cur], vals[cur]}, ArrayDst<uint64_t>{keys[cur ^ 1], vals[cur ^ 1]},
                   w.counters, 0, sort_workers(), kRadixBits * p, false, w, nullptr, s);
        cur ^= 1;
    }
    return {keys[cur], vals[cur]};
}

// The pair list's loads (pass_load): streamed when the list outgrows the
// memory-side cache, as a batch's does (the noisy 64-field batch lists 22 M
// pairs, 0.5 GB with their ping-pong copies: scatters 1.41 -> 1.07 ms), and
// cached otherwise (a 512^3 field lists 8 M: streamed loads cost its
// scatters 5%).  The length is known only on the device, so the choice
// follows the launch (PLMSS_TUNE_PAIR_STREAM).
PairList sort_pairs(int bits, bool batch, const Work& w, hipStream_t s) {
    const int64_t mode = knob(PLMSS_TUNE_PAIR_STREAM);
    if (mode == 1 || (mode == 2 && batch)) return sort_pairs_t<true>(bits, w, s);
    return sort_pairs_t<false>(bits, w, s);
}

// ---- one launch over a set of fields -------------------------------------------------------

// The fields of one call, grouped by shape class.  `all` lists every field in
// launch order (vertex numbering); cls[c] the fields of class c.
struct LaunchSet {
    Fields all;
    Fields cls[kClasses];
    bool used[kClasses];
    unsigned grid_s[kClasses], grid_j[kClasses];
    bool capacity;                // grids sized for a capacity, totals on the device
    bool batch_order;             // build the order fields of a batch's jobs
    uint32_t nv;                  // vertices of the launch (its capacity when `capacity`)
    const uint32_t* nv_dev;       // the launch's own total on the device (capacity launches)
    uint32_t max_fields;          // fields of the launch (its capacity when `capacity`)
    int bn;
    int32_t dtype;
    int zc;                       // scan depth of the 3-D scan tiles
};

// zc: the scan depth the tile counts of F were computed with.
template <bool RESOLVE, class Src>
void launch_steepest_cls(int c, int zc, const Fields& F, unsigned grid, uint32_t* up, uint32_t* dn,
                         hipStream_t s) {
    if (grid == 0) return;
    const int rounds = scan_rounds();
    // packed codes: 512-thread blocks fit their registers at six waves per
    // SIMD; the other sources keep 256-thread blocks
    constexpr int NT = Src::kPackedCodes ? kSteepBlock : kBlock;
    launch(PLMSS_KERNEL_STEEPEST, s, [&] {
        if (c != 0)
            k_steepest<Src, 16, 1, RESOLVE, NT><<<grid, NT, 0, s>>>(F, up, dn, rounds);
        else if (zc == 8)
            k_steepest<Src, 8, 8, RESOLVE, NT><<<grid, NT, 0, s>>>(F, up, dn, rounds);
        else if (zc == 32)
            k_steepest<Src, 8, 32, RESOLVE, NT><<<grid, NT, 0, s>>>(F, up, dn, rounds);
        else
            k_steepest<Src, 8, 16, RESOLVE, NT><<<grid, NT, 0, s>>>(F, up, dn, rounds);
    });
}

template <bool RESOLVE>
void launch_steepest_any(int c, int zc, const Fields& F, unsigned grid, int32_t dtype, bool order,
                         uint32_t* up, uint32_t* dn, hipStream_t s) {
    // ranks of a field below 2^28 vertices leave four bits for the code
    const bool packed = order && knob(PLMSS_TUNE_PACKED_CODES) != 0 &&
                        uint64_t(F.one.nx) * uint64_t(F.one.ny) * uint64_t(F.one.nz) < (1ull << 28);
    if (packed)
        launch_steepest_cls<RESOLVE, RankOrderPacked>(c, zc, F, grid, up, dn, s);
    else if (order)
        launch_steepest_cls<RESOLVE, RankOrder>(c, zc, F, grid, up, dn, s);
    else if (dtype == PLMSS_F32)
        launch_steepest_cls<RESOLVE, FieldOrder<float, uint32_t>>(c, zc, F, grid, up, dn, s);
    else
        launch_steepest_cls<RESOLVE, FieldOrder<double, uint64_t>>(c, zc, F, grid, up, dn, s);
}

// A launch over one field whose label rows are whole cache lines (the
// kernels' STREAM forms, segment.h kWholeLines).  Only 3-D fields have the
// streaming forms compiled; batches and plans keep the plain ones, since
// their fields' rows rarely fill whole lines.
bool whole_lines(const Fields& F) { return F.table == nullptr && (F.one.flags & kWholeLines); }

template <bool CHASE>
void launch_chase_cls(int c, const Fields& F, unsigned grid, uint32_t* U, uint32_t* D, int bn, const Work& w,
                      hipStream_t s) {
    if (grid == 0) return;
    uint64_t* rec = reinterpret_cast<uint64_t*>(w.keys[1]);
    // ids below 2^30: 32-bit byte offsets address every array of the chase
    const bool o32 = bn <= 30;
    launch(PLMSS_KERNEL_JUMP, s, [&] {
        if (CHASE && c == 0 && o32 && whole_lines(F))
            k_chase<JTile3, CHASE, true, CHASE><<<grid, kChaseBlock, 0, s>>>(F, U, D, bn, rec, w.counters + 0);
        else if (c == 0 && o32)
            k_chase<JTile3, CHASE, true><<<grid, kChaseBlock, 0, s>>>(F, U, D, bn, rec, w.counters + 0);
        else if (c == 0)
            k_chase<JTile3, CHASE, false><<<grid, kChaseBlock, 0, s>>>(F, U, D, bn, rec, w.counters + 0);
        else if (c == 1 && o32)
            k_chase<JTile2, CHASE, true><<<grid, kChaseBlock, 0, s>>>(F, U, D, bn, rec, w.counters + 0);
        else if (c == 1)
            k_chase<JTile2, CHASE, false><<<grid, kChaseBlock, 0, s>>>(F, U, D, bn, rec, w.counters + 0);
        else if (o32)
            k_chase<JTile1, CHASE, true><<<grid, kChaseBlock, 0, s>>>(F, U, D, bn, rec, w.counters + 0);
        else
            k_chase<JTile1, CHASE, false><<<grid, kChaseBlock, 0, s>>>(F, U, D, bn, rec, w.counters + 0);
    });
}

void launch_ms_final_cls(int c, const Fields& F, unsigned grid, const Work& w, hipStream_t s) {
    if (grid == 0) return;
    launch(PLMSS_KERNEL_MS_FINAL, s, [&] {
        if (c == 0 && whole_lines(F))
            k_ms_final<JTile3, true><<<grid, kBlock, 0, s>>>(F, w.rank_of, w.fbase);
        else if (c == 0)
            k_ms_final<JTile3><<<grid, kBlock, 0, s>>>(F, w.rank_of, w.fbase);
        else if (c == 1)
            k_ms_final<JTile2><<<grid, kBlock, 0, s>>>(F, w.rank_of, w.fbase);
        else
            k_ms_final<JTile1><<<grid, kBlock, 0, s>>>(F, w.rank_of, w.fbase);
    });
}

// MS ids from the pairs the chase listed: sort, rank, per-field bases,
// relabel.
void ms_from_pairs(const LaunchSet& L, const Work& w, hipStream_t s) {
    const PairList sorted = sort_pairs(2 * L.bn, L.all.table != nullptr, w, s);
    const uint64_t* sk = sorted.keys;
    const unsigned nw = sort_workers();
    launch(PLMSS_KERNEL_RANK, s, [&] { k_rank_reduce<<<nw, kBlock, 0, s>>>(sk, w.counters + 0, w.partial); });
    launch(PLMSS_KERNEL_PREFIX, s, [&] { k_scan_partials<<<1, kBlock, 0, s>>>(w.partial, int(nw), w.counters + 1); });
    launch(PLMSS_KERNEL_RANK, s, [&] {
        k_rank_apply<<<nw, kBlock, 0, s>>>(sk, sorted.vals, w.counters + 0, w.partial, w.rank_of);
    });
    launch(PLMSS_KERNEL_RANK, s, [&] {
        k_field_base<<<1, kBlock, 0, s>>>(L.all, sk, sorted.vals, w.counters + 0, w.counters + 1, w.rank_of,
                                          L.bn, w.fbase);
    });
    for (int c = 0; c < kClasses; ++c)
        if (L.used[c]) launch_ms_final_cls(c, L.cls[c], L.grid_j[c], w, s);
}

void init_set(const LaunchSet& L, const Work& w, hipStream_t s) {
    launch(PLMSS_KERNEL_MISC, s, [&] { k_init<<<1, 64, 0, s>>>(nullptr, w.counters, 8); });
    launch(PLMSS_KERNEL_MISC, s, [&] { k_init_fields<<<L.capacity ? 64u : 1u, kBlock, 0, s>>>(L.all); });
}

// Steepest neighbours, chase, MS ids for every field of L; the vertex order
// comes from a materialised order field when `order` is given, else from the
// field values.
void labels_set(const LaunchSet& L, const int32_t* order, const Work& w, hipStream_t s) {
    uint32_t* U = reinterpret_cast<uint32_t*>(w.keys[0]);
    uint32_t* D = U + w.npad;
    for (int c = 0; c < kClasses; ++c)
        if (L.used[c]) {
            Fields F = L.cls[c];
            if (order) F.one.src = order;
            launch_steepest_any<true>(c, L.zc, F, L.grid_s[c], L.dtype, order != nullptr, U, D, s);
        }
    for (int c = 0; c < kClasses; ++c)
        if (L.used[c]) launch_chase_cls<true>(c, L.cls[c], L.grid_j[c], U, D, L.bn, w, s);
    ms_from_pairs(L, w, s);
}

// The segmentation of every field of L (an order field only for a single
// field: `order` != nullptr), all on stream s.
void run_set(const LaunchSet& L, const void* field, int32_t* order, uint32_t n_single, const Work& w,
             hipStream_t s) {
    init_set(L, w, s);
    if (order)
        order_any(field, L.dtype, n_single, order, w, L.all.one.info, s);
    else if (L.batch_order && L.dtype == PLMSS_F32)
        order_batch_sort<float>(L.all, L.nv_dev, L.nv, L.max_fields, w, s);
    else if (L.batch_order)
        order_batch_sort<double>(L.all, L.nv_dev, L.nv, L.max_fields, w, s);
    labels_set(L, order, w, s);
}

// A library-owned non-blocking stream per device (created on first use, kept
// for the life of the process), default priority.
hipStream_t aux_stream() {
    constexpr int kMaxDevices = 64;
    static std::mutex mutex;
    static hipStream_t streams[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mutex);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess) {
        streams[dev] = nullptr;
        return nullptr;
    }
    return streams[dev];
}

// Host staging of the descriptor tables a batch call uploads: page-locked
// buffers the library keeps for the life of the process.  A buffer is handed
// out again only once the copy that last read it has completed (an event
// recorded after the copy), so a call returns without waiting for the device.
struct StageBuf {
    void* host = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    int device = -1;
};

// One host-to-device copy of a staged upload.
struct Upload {
    const void* src;
    size_t bytes;
    void* dst;
};

// Copies `parts` through one staging buffer on stream s.
int staged_upload(const Upload* parts, int nparts, hipStream_t s) {
    constexpr size_t kMaxBufs = 64;
    static std::mutex mutex;
    static std::vector<StageBuf> bufs;
    size_t need = 0;
    for (int i = 0; i < nparts; ++i) need += align_up(parts[i].bytes, 256);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PLMSS_E_HIP;
    std::lock_guard<std::mutex> lock(mutex);
    StageBuf* b = nullptr;
    for (StageBuf& c : bufs)
        if (c.device == dev && c.bytes >= need && hipEventQuery(c.done) == hipSuccess) {
            b = &c;
            break;
        }
    if (!b && bufs.size() >= kMaxBufs) {
        // every buffer is still being read: wait for the first large enough one
        for (StageBuf& c : bufs)
            if (c.device == dev && c.bytes >= need) {
                if (hipEventSynchronize(c.done) != hipSuccess) return PLMSS_E_HIP;
                b = &c;
                break;
            }
        if (!b) return PLMSS_E_HIP;
    }
    if (!b) {
        StageBuf c;
        c.bytes = std::max<size_t>(align_up(need, 4096), 64 * 1024);
        c.device = dev;
        if (hipHostMalloc(&c.host, c.bytes) != hipSuccess) return PLMSS_E_HIP;
        if (hipEventCreateWithFlags(&c.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipHostFree(c.host);
            return PLMSS_E_HIP;
        }
        bufs.push_back(c);
        b = &bufs.back();
    }
    uint8_t* h = static_cast<uint8_t*>(b->host);
    for (int i = 0; i < nparts; ++i) {
        std::memcpy(h, parts[i].src, parts[i].bytes);
        if (hipMemcpyAsync(parts[i].dst, h, parts[i].bytes, hipMemcpyHostToDevice, s) != hipSuccess)
            return PLMSS_E_HIP;
        h += align_up(parts[i].bytes, 256);
    }
    return hipEventRecord(b->done, s) == hipSuccess ? PLMSS_OK : PLMSS_E_HIP;
}

// One field with its order field: the order field is sorted on the auxiliary
// stream (its own half of the workspace, wo) while the labels, which compare
// the field values in place and so do not need it, run on s; s then waits for
// the order field.  Same results as run_set.
int run_single_concurrent(const LaunchSet& L, const plmss_job& job, uint32_t n, const Work& w, const Work& wo,
                          hipStream_t s) {
    hipStream_t aux = aux_stream();
    if (!aux) return PLMSS_E_HIP;
    hipEvent_t fork = nullptr, join = nullptr;
    if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) return PLMSS_E_HIP;
    if (hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) {
        (void)hipEventDestroy(fork);
        return PLMSS_E_HIP;
    }
    init_set(L, w, s);  // clears info before either stream may report into it
    int rc = PLMSS_OK;
    if (hipEventRecord(fork, s) != hipSuccess || hipStreamWaitEvent(aux, fork, 0) != hipSuccess) rc = PLMSS_E_HIP;
    if (rc == PLMSS_OK) {
        order_any(job.field, L.dtype, n, job.order, wo, L.all.one.info, aux);
        if (hipEventRecord(join, aux) != hipSuccess) rc = PLMSS_E_HIP;
    }
    labels_set(L, nullptr, w, s);
    if (rc == PLMSS_OK && hipStreamWaitEvent(s, join, 0) != hipSuccess) rc = PLMSS_E_HIP;
    (void)hipEventDestroy(fork);  // released once the recorded work completes
    (void)hipEventDestroy(join);
    return rc;
}

FieldDesc desc_of(const plmss_job& j, uint32_t vbase, uint32_t sbase, uint32_t jbase, uint32_t index = 0) {
    FieldDesc d;
    d.index = index;
    d.src = j.field;
    d.asc = j.asc;
    d.desc = j.desc;
    d.ms = j.ms;
    d.info = j.info;
    d.order = j.order;
    d.nx = int32_t(j.dims.nx);
    d.ny = int32_t(j.dims.ny);
    d.nz = int32_t(j.dims.nz);
    d.vbase = vbase;
    d.sbase = sbase;
    d.jbase = jbase;
    // whole 128-byte lines per row of the label arrays (segment.h, kWholeLines)
    const auto line = [](const void* p) { return p == nullptr || reinterpret_cast<uintptr_t>(p) % 128 == 0; };
    d.flags = (j.dims.nx % 32 == 0 && line(j.asc) && line(j.desc) && line(j.ms)) ? kWholeLines : 0u;
    return d;
}

Fields fields_one(const FieldDesc& d, uint32_t s_tiles, uint32_t j_tiles) {
    Fields F{};
    F.table = nullptr;
    F.n = 1;
    F.s_tiles = s_tiles;
    F.j_tiles = j_tiles;
    F.region0 = 0;
    F.dev_tiles = nullptr;
    F.one = d;
    return F;
}

// A single field: everything passed by value, one block per tile.
LaunchSet single_set(const plmss_job& job, uint64_t n, int zc) {
    LaunchSet L{};
    L.zc = zc;
    const int c = class_of(job.dims);
    const uint32_t st = s_tiles_of(job.dims, zc), jt = j_tiles_of(job.dims);
    const FieldDesc d = desc_of(job, 0, 0, 0);
    L.all = fields_one(d, st, jt);
    for (int k = 0; k < kClasses; ++k) L.used[k] = false;
    L.used[c] = true;
    L.cls[c] = fields_one(d, st, jt);
    L.grid_s[c] = st;
    L.grid_j[c] = jt;
    L.capacity = false;
    L.batch_order = false;
    L.nv = uint32_t(n);
    L.nv_dev = nullptr;
    L.max_fields = 1;
    L.bn = id_bits(n);
    L.dtype = job.dtype;
    return L;
}

// Host-side layout of a batch: descriptors of all fields and of each class
// (class-local tile bases), totals.
struct BatchLayout {
    std::vector<FieldDesc> all, cls[kClasses];
    uint32_t s_tiles[kClasses] = {0, 0, 0}, j_tiles[kClasses] = {0, 0, 0}, region0[kClasses] = {0, 0, 0};
    uint64_t nv = 0, regions = 0;
    int zc = 16;
    bool with_order = false;  // some job asks for its order field
};

int batch_layout(int32_t n_jobs, const plmss_job* jobs, int zc, BatchLayout* B) {
    B->zc = zc;
    if (n_jobs < 1 || !jobs) return PLMSS_E_ARG;
    const int32_t dtype = jobs[0].dtype;
    std::vector<uint64_t> nvert(n_jobs);
    for (int32_t i = 0; i < n_jobs; ++i) {
        const plmss_job& j = jobs[i];
        if (!j.field || !j.asc || !j.desc || !j.ms) return PLMSS_E_ARG;
        B->with_order |= j.order != nullptr;
        if (j.dtype != PLMSS_F32 && j.dtype != PLMSS_F64) return PLMSS_E_ARG;
        if (j.dtype != dtype) return PLMSS_E_ARG;
        int rc = check_dims(j.dims, &nvert[i]);
        if (rc) return rc;
        B->nv += nvert[i];
        if (B->nv > uint64_t(kMaxN)) return PLMSS_E_TOO_LARGE;
    }
    uint32_t vb = 0;
    for (int32_t i = 0; i < n_jobs; ++i) {
        const int c = class_of(jobs[i].dims);
        const FieldDesc d = desc_of(jobs[i], vb, B->s_tiles[c], B->j_tiles[c], uint32_t(i));
        B->all.push_back(d);
        B->cls[c].push_back(d);
        vb += uint32_t(nvert[i]);
        B->s_tiles[c] += s_tiles_of(jobs[i].dims, zc);
        B->j_tiles[c] += j_tiles_of(jobs[i].dims);
    }
    // chase tiles: class 0 first, then class 1, then class 2
    B->region0[1] = B->j_tiles[0];
    B->region0[2] = B->j_tiles[0] + B->j_tiles[1];
    B->regions = uint64_t(B->j_tiles[0]) + B->j_tiles[1] + B->j_tiles[2];
    return PLMSS_OK;
}

// Table image: range 0 = all fields, range 1 + c = class c, `stride` entries each.
std::vector<FieldDesc> table_image(const BatchLayout& B, size_t stride) {
    std::vector<FieldDesc> img(4 * stride);
    std::copy(B.all.begin(), B.all.end(), img.begin());
    for (int c = 0; c < kClasses; ++c) std::copy(B.cls[c].begin(), B.cls[c].end(), img.begin() + (1 + c) * stride);
    return img;
}

// A batch with host-known totals over the device tables.
LaunchSet batch_set(const BatchLayout& B, const FieldDesc* tables, size_t stride, int32_t dtype, int bn) {
    LaunchSet L{};
    L.all = Fields{};
    L.all.table = tables;
    L.all.n = uint32_t(B.all.size());
    for (int c = 0; c < kClasses; ++c) {
        Fields F{};
        F.table = tables + (1 + c) * stride;
        F.n = uint32_t(B.cls[c].size());
        F.s_tiles = B.s_tiles[c];
        F.j_tiles = B.j_tiles[c];
        F.region0 = B.region0[c];
        F.dev_tiles = nullptr;
        L.cls[c] = F;
        L.used[c] = F.n > 0;
        L.grid_s[c] = B.s_tiles[c];
        L.grid_j[c] = B.j_tiles[c];
    }
    L.capacity = false;
    L.batch_order = B.with_order;
    L.nv = uint32_t(B.nv);
    L.nv_dev = nullptr;
    L.max_fields = uint32_t(B.all.size());
    L.bn = bn;
    L.dtype = dtype;
    L.zc = B.zc;
    return L;
}

// Device totals block of a capacity launch (u32, in counters[32..63]):
//   [4c .. 4c+3]  class c: scan tiles, chase tiles, fields, first region
//   [12 .. 15]    all fields: 0, vertices, fields, 0
constexpr int kTot = 32;

LaunchSet capacity_set(const Work& w, size_t stride, unsigned grid_s, unsigned grid_j, int32_t dtype, int bn,
                       int zc, bool with_order, uint32_t max_vertices) {
    const uint32_t* tot = w.counters + kTot;
    LaunchSet L{};
    L.all = Fields{};
    L.all.table = w.tables;
    L.all.n = uint32_t(stride);
    L.all.dev_tiles = tot + 12;
    for (int c = 0; c < kClasses; ++c) {
        Fields F{};
        F.table = w.tables + (1 + c) * stride;
        F.n = uint32_t(stride);
        F.dev_tiles = tot + 4 * c;
        L.cls[c] = F;
        L.used[c] = true;  // a class without fields runs empty grids
        L.grid_s[c] = grid_s;
        L.grid_j[c] = grid_j;
    }
    L.capacity = true;
    L.batch_order = with_order;
    L.nv = max_vertices;
    L.nv_dev = tot + 13;
    L.max_fields = uint32_t(stride);
    L.bn = bn;
    L.dtype = dtype;
    L.zc = zc;
    return L;
}

}  // namespace

// ---- library-owned scratch for callers that cannot allocate ---------------------------------
// One fixed array per GPU, sized for the workspace of a single field of up to
// kStaticMaxVertices vertices, held until the process ends.  Host code never
// takes the array's name as an address: it asks the runtime for the array's
// address on the current device once (static_scratch) and uses that.
constexpr uint64_t kStaticMaxVertices = PLMSS_STATIC_MAX_VERTICES;
constexpr size_t kStaticScratchBytes = work_sizes(kStaticMaxVertices, 1, 0).total;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

namespace {

// The scratch array's device address on the current device; looked up once
// per device, with that device current.  nullptr if the runtime fails.
void* static_scratch() {
    constexpr int kMaxDevices = 64;
    static std::mutex mutex;
    static void* ptrs[kMaxDevices] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mutex);
    if (!ptrs[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        ptrs[dev] = p;
    }
    return ptrs[dev];
}

}  // namespace

// ---- capacity plans (batched launches that a hipGraph can replay) -----------------------

struct plmss_plan {
    int64_t max_vertices = 0;
    int32_t max_fields = 0;
    int64_t max_scan_tiles = 0;
    int64_t max_chase_tiles = 0;
    int32_t dtype = 0;
    bool with_order = false;  // the plan builds the order fields its jobs ask for
    int bn = 1;
    int zc = 16;  // scan depth, fixed at creation: tables and launches agree
    Sizes sizes{};
    hipGraphExec_t exec = nullptr;
    void* graph_ws = nullptr;            // workspace the graph was captured with
    hipStream_t capture_stream = nullptr;  // private: capture never runs work
};

struct plmss_trace {
    Trace t;
};

extern "C" {

const char* plmss_status_string(int code) {
    switch (code) {
        case PLMSS_OK: return "ok";
        case PLMSS_E_ARG: return "invalid argument (NULL pointer or bad enum value)";
        case PLMSS_E_DIMS: return "invalid grid dimensions (each must be >= 1)";
        case PLMSS_E_TOO_LARGE: return "too large (more than 2^31-1 vertices, or beyond a plan's capacity)";
        case PLMSS_E_NAN: return "the field contains NaN";
        case PLMSS_E_WORKSPACE: return "workspace missing, misaligned or too small";
        case PLMSS_E_HIP: return "HIP runtime or launch error";
        case PLMSS_E_NOCONV: return "path compression did not converge (pointers do not form a forest)";
        case PLMSS_E_INTERNAL: return "internal error: the order field's inversion lost a pair";
        default: return "unknown status";
    }
}

const char* plmss_build_info(void) { return "libplmss 0.2 gfx950 wave64"; }

size_t plmss_workspace_bytes(plmss_dims dims, int32_t dtype, int32_t with_order) {
    uint64_t n;
    if (check_dims(dims, &n) != PLMSS_OK) return 0;
    (void)dtype;
    // with the order field: a second half for the order sort, which may run
    // concurrently with the labels
    return work_sizes(n, 1, 0).total * (with_order ? 2 : 1);
}

int plmss_segment(const plmss_job* job, void* workspace, size_t workspace_bytes, void* stream) {
    if (!job || !job->field || !job->asc || !job->desc || !job->ms) return PLMSS_E_ARG;
    if (job->dtype != PLMSS_F32 && job->dtype != PLMSS_F64) return PLMSS_E_ARG;
    uint64_t n;
    int rc = check_dims(job->dims, &n);
    if (rc) return rc;
    const Sizes sz = work_sizes(n, 1, 0);
    if (!ws_ok(workspace, workspace_bytes, sz.total * (job->order ? 2 : 1))) return PLMSS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Work w = carve(workspace, sz);
    const LaunchSet L = single_set(*job, n, scan_depth());
    if (job->order && knob(PLMSS_TUNE_ORDER_CONCURRENT) != 0) {
        const Work wo = carve(static_cast<uint8_t*>(workspace) + sz.total, sz);
        const int rc = run_single_concurrent(L, *job, uint32_t(n), w, wo, s);
        return rc != PLMSS_OK ? rc : launch_status();
    }
    run_set(L, job->field, job->order, uint32_t(n), w, s);
    return launch_status();
}

size_t plmss_static_scratch_bytes(void) { return kStaticScratchBytes; }

int plmss_segment_static(const plmss_job* job, void* stream) {
    if (!job || !job->field || !job->asc || !job->desc || !job->ms) return PLMSS_E_ARG;
    if (job->dtype != PLMSS_F32 && job->dtype != PLMSS_F64) return PLMSS_E_ARG;
    uint64_t n;
    int rc = check_dims(job->dims, &n);
    if (rc) return rc;
    if (n > kStaticMaxVertices) return PLMSS_E_TOO_LARGE;
    const Sizes sz = work_sizes(n, 1, 0);
    if (sz.total > kStaticScratchBytes) return PLMSS_E_TOO_LARGE;
    void* ws = static_scratch();
    if (!ws) return PLMSS_E_HIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // one half only: the order field, if asked for, is built on this stream
    // before the labels (never on the concurrent stream, which needs a second half)
    run_set(single_set(*job, n, scan_depth()), job->field, job->order, uint32_t(n), carve(ws, sz), s);
    return launch_status();
}

size_t plmss_order_workspace_bytes(plmss_dims dims, int32_t dtype) {
    return plmss_workspace_bytes(dims, dtype, 1);
}

int plmss_order_field(const void* field, plmss_dims dims, int32_t dtype, int32_t* order,
                      int32_t* info, void* workspace, size_t workspace_bytes, void* stream) {
    if (!field || !order || (dtype != PLMSS_F32 && dtype != PLMSS_F64)) return PLMSS_E_ARG;
    uint64_t n;
    int rc = check_dims(dims, &n);
    if (rc) return rc;
    const Sizes sz = work_sizes(n, 1, 0);
    if (!ws_ok(workspace, workspace_bytes, sz.total)) return PLMSS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Work w = carve(workspace, sz);
    if (info) launch(PLMSS_KERNEL_MISC, s, [&] { k_init<<<1, 64, 0, s>>>(info, nullptr, 0); });
    order_any(field, dtype, uint32_t(n), order, w, info, s);
    return launch_status();
}

int plmss_steepest(const void* field, const int32_t* order, plmss_dims dims, int32_t dtype,
                   int32_t* up, int32_t* dn, int32_t* info, void* stream) {
    if (!up || !dn || (!field && !order)) return PLMSS_E_ARG;
    if (!order && dtype != PLMSS_F32 && dtype != PLMSS_F64) return PLMSS_E_ARG;
    uint64_t n;
    int rc = check_dims(dims, &n);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (info) launch(PLMSS_KERNEL_MISC, s, [&] { k_init<<<1, 64, 0, s>>>(info, nullptr, 0); });
    plmss_job j{};
    j.field = order ? static_cast<const void*>(order) : field;
    j.dims = dims;
    j.info = info;
    const int zc = scan_depth();
    const Fields F = fields_one(desc_of(j, 0, 0, 0), s_tiles_of(dims, zc), j_tiles_of(dims));
    launch_steepest_any<false>(class_of(dims), zc, F, s_tiles_of(dims, zc), order ? PLMSS_F32 : dtype,
                               order != nullptr, reinterpret_cast<uint32_t*>(up),
                               reinterpret_cast<uint32_t*>(dn), s);
    return launch_status();
}

int plmss_compress(int32_t* desc, int32_t* asc, int64_t n, void* stream) {
    if (!desc || !asc) return PLMSS_E_ARG;
    if (n < 1) return PLMSS_E_DIMS;
    if (n > kMaxN) return PLMSS_E_TOO_LARGE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    launch(PLMSS_KERNEL_JUMP, s, [&] { k_jump<<<grid_for(uint64_t(n)), kBlock, 0, s>>>(desc, asc, uint32_t(n)); });
    return launch_status();
}

size_t plmss_ms_workspace_bytes(int64_t n) {
    if (n < 1 || n > kMaxN) return 0;
    return work_sizes(uint64_t(n), 1, 0).total;
}

int plmss_ms_ids(const int32_t* asc, const int32_t* desc, int64_t n, int32_t* ms, int32_t* info,
                 void* workspace, size_t workspace_bytes, void* stream) {
    if (!asc || !desc || !ms) return PLMSS_E_ARG;
    if (n < 1) return PLMSS_E_DIMS;
    if (n > kMaxN) return PLMSS_E_TOO_LARGE;
    const plmss_dims d{n, 1, 1};
    const Sizes sz = work_sizes(uint64_t(n), 1, 0);
    if (!ws_ok(workspace, workspace_bytes, sz.total)) return PLMSS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Work w = carve(workspace, sz);
    plmss_job j{};
    j.field = asc;  // not read: only the labels are
    j.dims = d;
    j.asc = const_cast<int32_t*>(asc);
    j.desc = const_cast<int32_t*>(desc);
    j.ms = ms;
    j.info = info;
    const LaunchSet L = single_set(j, uint64_t(n), scan_depth());
    launch(PLMSS_KERNEL_MISC, s, [&] { k_init<<<1, 64, 0, s>>>(info, w.counters, 8); });
    launch_chase_cls<false>(class_of(d), L.cls[class_of(d)], L.grid_j[class_of(d)], nullptr, nullptr, L.bn, w, s);
    ms_from_pairs(L, w, s);
    return launch_status();
}

int64_t plmss_marching_rows(plmss_dims dims) {
    uint64_t n;
    if (check_dims(dims, &n) != PLMSS_OK) return -1;
    return march_rows(dims);
}

size_t plmss_marching_workspace_bytes(plmss_dims dims) {
    uint64_t n;
    if (check_dims(dims, &n) != PLMSS_OK) return 0;
    return march_ws_bytes(uint64_t(march_rows(dims)));
}

int plmss_marching_index(const int32_t* labels, plmss_dims dims, int32_t mode, uint8_t* codes,
                         uint64_t* row_offsets, void* workspace, size_t workspace_bytes, void* stream) {
    if (!labels || !row_offsets || (mode != PLMSS_MARCH_SEPARATORS && mode != PLMSS_MARCH_BOUNDARIES))
        return PLMSS_E_ARG;
    if (codes && (reinterpret_cast<uintptr_t>(codes) & 1u)) return PLMSS_E_ARG;
    uint64_t n;
    const int rc = check_dims(dims, &n);
    if (rc != PLMSS_OK) return rc;
    const uint64_t rows = uint64_t(march_rows(dims));
    if (!ws_ok(workspace, workspace_bytes, march_ws_bytes(rows))) return PLMSS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint64_t* block_sums = static_cast<uint64_t*>(workspace);
    const int rpw = march_rows_per_wave(rows);
    const unsigned blocks = unsigned(march_blocks(rows));
    const int nx = int(dims.nx), ny = int(dims.ny);
    if (rows > 0)
        launch(PLMSS_KERNEL_MARCH, s, [&] {
            const int shape = (dims.nz > 1 ? 4 : 0) | (mode ? 2 : 0) | (codes ? 1 : 0);
            auto go = [&](auto kernel) {
                kernel<<<blocks, kBlock, 0, s>>>(labels, nx, ny, uint32_t(rows), codes, row_offsets, block_sums, rpw);
            };
            switch (shape) {
                case 0: go(k_march_count<false, 0, false>); break;
                case 1: go(k_march_count<false, 0, true>); break;
                case 2: go(k_march_count<false, 1, false>); break;
                case 3: go(k_march_count<false, 1, true>); break;
                case 4: go(k_march_count<true, 0, false>); break;
                case 5: go(k_march_count<true, 0, true>); break;
                case 6: go(k_march_count<true, 1, false>); break;
                default: go(k_march_count<true, 1, true>); break;
            }
        });
    launch(PLMSS_KERNEL_PREFIX, s, [&] {
        k_march_scan_blocks<<<1, kBlock, 0, s>>>(block_sums, blocks, row_offsets + rows);
    });
    if (rows > 0)
        launch(PLMSS_KERNEL_PREFIX, s, [&] {
            k_march_offsets<<<blocks, kBlock, 0, s>>>(row_offsets, uint32_t(rows), block_sums, rpw * kWavesPerBlock);
        });
    return launch_status();
}

int plmss_marching_geometry(const int32_t* labels, plmss_dims dims, int32_t mode, const uint64_t* row_offsets,
                            uint64_t capacity, float* xyz, int32_t* sides, void* stream) {
    if (!labels || !row_offsets || (mode != PLMSS_MARCH_SEPARATORS && mode != PLMSS_MARCH_BOUNDARIES))
        return PLMSS_E_ARG;
    if ((xyz && (reinterpret_cast<uintptr_t>(xyz) & 3u)) || (sides && (reinterpret_cast<uintptr_t>(sides) & 7u)))
        return PLMSS_E_ARG;
    uint64_t n;
    const int rc = check_dims(dims, &n);
    if (rc != PLMSS_OK) return rc;
    const uint64_t rows = uint64_t(march_rows(dims));
    if (rows == 0 || (!xyz && !sides)) return PLMSS_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const unsigned blocks = unsigned((rows + kGeoWaves - 1) / kGeoWaves);
    const int nx = int(dims.nx), ny = int(dims.ny);
    launch(PLMSS_KERNEL_MARCH_GEOMETRY, s, [&] {
        auto go = [&](auto kernel) {
            kernel<<<blocks, kBlock, 0, s>>>(labels, nx, ny, uint32_t(rows), row_offsets, capacity, xyz, sides);
        };
        switch ((dims.nz > 1 ? 2 : 0) | (mode ? 1 : 0)) {
            case 0: go(k_march_geometry<false, 0>); break;
            case 1: go(k_march_geometry<false, 1>); break;
            case 2: go(k_march_geometry<true, 0>); break;
            default: go(k_march_geometry<true, 1>); break;
        }
    });
    return launch_status();
}

size_t plmss_batch_workspace_bytes(int32_t n_jobs, const plmss_job* jobs) {
    BatchLayout B;
    if (batch_layout(n_jobs, jobs, scan_depth(), &B) != PLMSS_OK) return 0;
    return work_sizes(B.nv, uint64_t(n_jobs), uint64_t(n_jobs)).total;
}

int plmss_segment_batch(int32_t n_jobs, const plmss_job* jobs, void* workspace,
                        size_t workspace_bytes, void* stream) {
    BatchLayout B;
    int rc = batch_layout(n_jobs, jobs, scan_depth(), &B);
    if (rc) return rc;
    const Sizes sz = work_sizes(B.nv, uint64_t(n_jobs), uint64_t(n_jobs));
    if (!ws_ok(workspace, workspace_bytes, sz.total)) return PLMSS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Work w = carve(workspace, sz);
    const std::vector<FieldDesc> img = table_image(B, size_t(n_jobs));
    const Upload part{img.data(), sizeof(FieldDesc) * img.size(), w.tables};
    rc = staged_upload(&part, 1, s);
    if (rc != PLMSS_OK) return rc;
    const LaunchSet L = batch_set(B, w.tables, size_t(n_jobs), jobs[0].dtype, id_bits(B.nv));
    run_set(L, nullptr, nullptr, 0, w, s);
    return launch_status();
}

int32_t plmss_batch_needs(int32_t n_jobs, const plmss_job* jobs, int64_t* needs) {
    if (!needs) return PLMSS_E_ARG;
    BatchLayout B;
    int rc = batch_layout(n_jobs, jobs, scan_depth(), &B);
    if (rc) return rc;
    needs[0] = int64_t(B.nv);
    needs[1] = n_jobs;
    needs[2] = int64_t(B.s_tiles[0]) + B.s_tiles[1] + B.s_tiles[2];
    needs[3] = int64_t(B.regions);
    return PLMSS_OK;
}

plmss_plan* plmss_plan_create(int64_t max_vertices, int32_t max_fields, int64_t max_scan_tiles,
                              int64_t max_chase_tiles, int32_t dtype, int32_t with_order) {
    if (max_vertices < 1 || max_vertices > kMaxN || max_fields < 1 || max_scan_tiles < 1 ||
        max_chase_tiles < 1 || (dtype != PLMSS_F32 && dtype != PLMSS_F64) || (with_order != 0 && with_order != 1))
        return nullptr;
    plmss_plan* p = new (std::nothrow) plmss_plan;
    if (!p) return nullptr;
    p->max_vertices = max_vertices;
    p->max_fields = max_fields;
    p->max_scan_tiles = max_scan_tiles;
    p->max_chase_tiles = max_chase_tiles;
    p->dtype = dtype;
    p->with_order = with_order != 0;
    p->bn = id_bits(uint64_t(max_vertices));
    p->zc = scan_depth();
    p->sizes = work_sizes(uint64_t(max_vertices), uint64_t(max_fields),
                          uint64_t(max_fields));
    return p;
}

void plmss_plan_destroy(plmss_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    delete p;
}

size_t plmss_plan_workspace_bytes(const plmss_plan* p) { return p ? p->sizes.total : 0; }

int plmss_plan_set(plmss_plan* p, int32_t n_jobs, const plmss_job* jobs, void* workspace,
                   size_t workspace_bytes, void* stream) {
    if (!p) return PLMSS_E_ARG;
    BatchLayout B;
    int rc = batch_layout(n_jobs, jobs, p->zc, &B);
    if (rc) return rc;
    if (jobs[0].dtype != p->dtype) return PLMSS_E_ARG;
    if (B.with_order && !p->with_order) return PLMSS_E_ARG;
    if (n_jobs > p->max_fields || B.nv > uint64_t(p->max_vertices) ||
        B.regions > uint64_t(p->max_chase_tiles) ||
        uint64_t(B.s_tiles[0]) + B.s_tiles[1] + B.s_tiles[2] > uint64_t(p->max_scan_tiles))
        return PLMSS_E_TOO_LARGE;
    if (!ws_ok(workspace, workspace_bytes, p->sizes.total)) return PLMSS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Work w = carve(workspace, p->sizes);
    const std::vector<FieldDesc> img = table_image(B, size_t(p->max_fields));
    uint32_t tot[32] = {};
    for (int c = 0; c < kClasses; ++c) {
        tot[4 * c + 0] = B.s_tiles[c];
        tot[4 * c + 1] = B.j_tiles[c];
        tot[4 * c + 2] = uint32_t(B.cls[c].size());
        tot[4 * c + 3] = B.region0[c];
    }
    tot[13] = uint32_t(B.nv);
    tot[14] = uint32_t(n_jobs);
    const Upload parts[2] = {{img.data(), sizeof(FieldDesc) * img.size(), w.tables},
                             {tot, sizeof(tot), w.counters + kTot}};
    return staged_upload(parts, 2, s);
}

int plmss_plan_launch(plmss_plan* p, void* workspace, size_t workspace_bytes, void* stream) {
    if (!p) return PLMSS_E_ARG;
    if (!ws_ok(workspace, workspace_bytes, p->sizes.total)) return PLMSS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Work w = carve(workspace, p->sizes);
    const unsigned gs = unsigned(std::min<int64_t>(persist_blocks(), p->max_scan_tiles));
    const unsigned gj = unsigned(std::min<int64_t>(persist_blocks(), p->max_chase_tiles));
    const LaunchSet L = capacity_set(w, size_t(p->max_fields), gs, gj, p->dtype, p->bn, p->zc, p->with_order,
                                     uint32_t(p->max_vertices));
    run_set(L, nullptr, nullptr, 0, w, s);
    return launch_status();
}

int plmss_plan_launch_graph(plmss_plan* p, void* workspace, size_t workspace_bytes, void* stream) {
    if (!p) return PLMSS_E_ARG;
    if (!ws_ok(workspace, workspace_bytes, p->sizes.total)) return PLMSS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!p->exec || p->graph_ws != workspace) {
        if (p->exec) {
            (void)hipGraphExecDestroy(p->exec);
            p->exec = nullptr;
        }
        // capture on a private stream (the caller's may be the null stream,
        // which cannot be captured); the graph then runs on the caller's
        if (!p->capture_stream &&
            hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) != hipSuccess) {
            p->capture_stream = nullptr;
            return PLMSS_E_HIP;
        }
        Trace* saved = g_trace;  // events are not recorded into a graph
        g_trace = nullptr;
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
            g_trace = saved;
            return PLMSS_E_HIP;
        }
        const int rc = plmss_plan_launch(p, workspace, workspace_bytes, p->capture_stream);
        const hipError_t e = hipStreamEndCapture(p->capture_stream, &graph);
        g_trace = saved;
        if (rc != PLMSS_OK || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return PLMSS_E_HIP;
        }
        const hipError_t ie = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            p->exec = nullptr;
            return PLMSS_E_HIP;
        }
        p->graph_ws = workspace;
    }
    return hipGraphLaunch(p->exec, s) == hipSuccess ? PLMSS_OK : PLMSS_E_HIP;
}

// ---- tracing ----------------------------------------------------------------------------

plmss_trace* plmss_trace_create(int32_t max_launches) {
    if (max_launches < 1) return nullptr;
    plmss_trace* tr = new (std::nothrow) plmss_trace;
    if (!tr) return nullptr;
    tr->t.ev = new (std::nothrow) hipEvent_t[2 * size_t(max_launches)];
    tr->t.kind = new (std::nothrow) int32_t[max_launches];
    if (!tr->t.ev || !tr->t.kind) {
        delete[] tr->t.ev;
        delete[] tr->t.kind;
        delete tr;
        return nullptr;
    }
    for (int32_t i = 0; i < 2 * max_launches; ++i) {
        if (hipEventCreate(&tr->t.ev[i]) != hipSuccess) {
            for (int32_t j = 0; j < i; ++j) (void)hipEventDestroy(tr->t.ev[j]);
            delete[] tr->t.ev;
            delete[] tr->t.kind;
            delete tr;
            return nullptr;
        }
    }
    tr->t.cap = max_launches;
    return tr;
}

void plmss_trace_destroy(plmss_trace* tr) {
    if (!tr) return;
    if (g_trace == &tr->t) g_trace = nullptr;
    for (int32_t i = 0; i < 2 * tr->t.cap; ++i) (void)hipEventDestroy(tr->t.ev[i]);
    delete[] tr->t.ev;
    delete[] tr->t.kind;
    delete tr;
}

int plmss_trace_begin(plmss_trace* tr) {
    if (!tr) return PLMSS_E_ARG;
    tr->t.n = 0;
    g_trace = &tr->t;
    return PLMSS_OK;
}

int plmss_trace_end(plmss_trace* tr) {
    if (!tr) return PLMSS_E_ARG;
    if (g_trace == &tr->t) g_trace = nullptr;
    return PLMSS_OK;
}

int32_t plmss_trace_read(plmss_trace* tr, int32_t* kinds, float* ms, int32_t max) {
    if (!tr || max < 0 || (max > 0 && (!kinds || !ms))) return PLMSS_E_ARG;
    const int32_t m = std::min(max, tr->t.n);
    for (int32_t i = 0; i < m; ++i) {
        if (hipEventSynchronize(tr->t.ev[2 * i + 1]) != hipSuccess) return PLMSS_E_HIP;
        float e = 0.f;
        if (hipEventElapsedTime(&e, tr->t.ev[2 * i], tr->t.ev[2 * i + 1]) != hipSuccess) return PLMSS_E_HIP;
        kinds[i] = tr->t.kind[i];
        ms[i] = e;
    }
    return m;
}

const char* plmss_kernel_name(int32_t kind) {
    static const char* names[PLMSS_KERNEL_KINDS] = {
        "misc", "radix_hist", "radix_digit_scan", "radix_scatter", "steepest", "jump", "prefix_sum",
        "pair_compact", "pair_rank", "ms_final", "order_hist", "order_scatter", "order_invert",
        "order_first", "order_last", "order_regroup", "march_count", "march_geometry"};
    return (kind >= 0 && kind < PLMSS_KERNEL_KINDS) ? names[kind] : "unknown";
}

// ---- launch-shape knobs -------------------------------------------------------------------

int32_t plmss_tune_set(int32_t knob_id, int64_t value) {
    if (knob_id < 0 || knob_id >= PLMSS_TUNE_KNOBS) return PLMSS_E_ARG;
    const KnobRange& r = kKnobs[knob_id];
    if (!(value == 0 && r.zero_ok) && (value < r.lo || value > r.hi)) return PLMSS_E_ARG;
    if (r.pow2 && (value & (value - 1)) != 0) return PLMSS_E_ARG;
    g_knob[knob_id].store(value, std::memory_order_relaxed);
    return PLMSS_OK;
}

int64_t plmss_tune_get(int32_t knob_id) {
    if (knob_id < 0 || knob_id >= PLMSS_TUNE_KNOBS) return -1;
    return knob(knob_id);
}

}  // extern "C"
