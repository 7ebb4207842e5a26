// libplmss: C ABI of the gfx950 Morse-Smale segmentation (see include/plmss.h).
#include "plmss.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>

#include "common.h"
#include "segment.h"
#include "sort.h"

using namespace plmss;

namespace {

constexpr int64_t kMaxN = 2147483647;  // int32 labels

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

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

// Workspace of one field of n vertices (also the shape of a batch's
// workspace, with n = the batch's total).
struct Work {
    uint8_t* keys[2];        // u64[npad] each: sort keys (ping-pong).  keys[0] also holds
                             // the tile-compressed pointers U, D (u32[npad] each) and
                             // keys[1] the per-block pair lists
    uint32_t* vals[2];       // u32[npad] each: sort values
    uint32_t* rank_of;       // u32[npad]: MS id of each listed pair (dense index)
    uint32_t* reg_cnt;       // u32[nregions]: pairs listed per chase tile
    uint32_t* reg_off;       // u32[nregions]: their exclusive prefix
    uint32_t* hist;          // u32[kRadix * max(kWorkers, ntiles)]
    uint32_t* dtotal;        // u32[kRadix]
    uint32_t* partial;       // u32[kWorkers]
    uint32_t* counters;      // u32[64]: [0] = #pairs listed, [1] = K
    uint8_t* extra;          // batch tables
    uint64_t npad;
};

struct Sizes {
    size_t keys, vals, rank, regions, hist, dtotal, partial, counters, extra, total;
    uint64_t npad;
};

uint64_t n_tiles(uint64_t n) { return (n + kTile - 1) / kTile; }

// Tile grid of the chase kernel for a field of dims d: 3-D, 2-D or 1-D tiles.
struct ChasePlan {
    int kind;            // 3, 2 or 1
    uint64_t regions;    // number of tiles
};

ChasePlan chase_plan(const plmss_dims& d) {
    const GridDims g{int32_t(d.nx), int32_t(d.ny), int32_t(d.nz)};
    if (d.nz > 1) return {3, chase_blocks<JTile3>(g)};
    if (d.ny > 1) return {2, chase_blocks<JTile2>(g)};
    return {1, chase_blocks<JTile1>(g)};
}

Sizes work_sizes(uint64_t n, uint64_t regions, size_t extra) {
    Sizes s;
    s.npad = align_up(n, kBlock);
    const uint64_t rec = std::max<uint64_t>(s.npad, regions * kJV);
    s.keys = align_up(8 * rec, 256);
    s.vals = align_up(4 * s.npad, 256);
    s.rank = align_up(4 * s.npad, 256);
    s.regions = align_up(4 * std::max<uint64_t>(regions, 1), 256);
    s.hist = align_up(size_t(4) * kRadix * std::max<uint64_t>(kWorkers, n_tiles(n)), 256);
    s.dtotal = align_up(4 * kRadix, 256);
    s.partial = align_up(4 * kWorkers, 256);
    s.counters = 256;
    s.extra = align_up(extra, 256);
    s.total = 2 * s.keys + 2 * s.vals + s.rank + 2 * s.regions + s.hist + s.dtotal + s.partial +
              s.counters + s.extra;
    return s;
}

Sizes work_sizes(const plmss_dims& d, uint64_t n) { return work_sizes(n, chase_plan(d).regions, 0); }

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
    w.reg_cnt = reinterpret_cast<uint32_t*>(take(s.regions));
    w.reg_off = reinterpret_cast<uint32_t*>(take(s.regions));
    w.hist = reinterpret_cast<uint32_t*>(take(s.hist));
    w.dtotal = reinterpret_cast<uint32_t*>(take(s.dtotal));
    w.partial = reinterpret_cast<uint32_t*>(take(s.partial));
    w.counters = reinterpret_cast<uint32_t*>(take(s.counters));
    w.extra = take(s.extra);
    w.npad = s.npad;
    return w;
}

int launch_status() { return hipGetLastError() == hipSuccess ? PLMSS_OK : PLMSS_E_HIP; }

unsigned grid_for(uint64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

// ---- optional launch tracing -------------------------------------------------------------
// While a trace is active on the calling host thread, every kernel launch is
// bracketed by two hipEvents recorded on the launch stream.

struct Trace {
    hipEvent_t* ev = nullptr;   // 2 per launch
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

// One pass over `workers` blocks; cnt (device) or n (host) is the length.
template <class Src, class Dst>
void radix_pass(Src src, Dst dst, const uint32_t* cnt, uint32_t n, unsigned workers, int shift,
                bool check_nan, const Work& w, int32_t* info, hipStream_t s) {
    if (check_nan)
        launch(PLMSS_KERNEL_RADIX_HIST, s, [&] {
            k_radix_hist<Src, true><<<workers, kBlock, 0, s>>>(src, cnt, n, shift, w.hist, info);
        });
    else
        launch(PLMSS_KERNEL_RADIX_HIST, s, [&] {
            k_radix_hist<Src, false><<<workers, kBlock, 0, s>>>(src, cnt, n, shift, w.hist, info);
        });
    launch(PLMSS_KERNEL_RADIX_SCAN, s, [&] {
        k_radix_digit_scan<<<kRadix, kBlock, 0, s>>>(w.hist, w.dtotal, int(workers));
    });
    launch(PLMSS_KERNEL_RADIX_SCATTER, s, [&] {
        k_radix_scatter<Src, Dst><<<workers, kBlock, 0, s>>>(src, dst, cnt, n, shift, w.hist, w.dtotal);
    });
}

// Order field of a float field: keys from the values, values = ids; the last
// pass writes order[id] = position.  One worker per tile.
template <typename T, typename K>
void sort_order(const T* f, uint32_t n, int32_t* order, const Work& w, int32_t* info,
                hipStream_t s) {
    constexpr int passes = int(sizeof(K)) * 8 / kRadixBits;
    const unsigned workers = unsigned(n_tiles(n));
    K* keys[2] = {reinterpret_cast<K*>(w.keys[0]), reinterpret_cast<K*>(w.keys[1])};
    FieldSrc<T, K> first{f};
    radix_pass(first, ArrayDst<K>{keys[0], w.vals[0]}, nullptr, n, workers, 0, true, w, info, s);
    int cur = 0;
    for (int p = 1; p < passes - 1; ++p) {
        radix_pass(ArraySrc<K>{keys[cur], w.vals[cur]}, ArrayDst<K>{keys[cur ^ 1], w.vals[cur ^ 1]},
                   nullptr, n, workers, kRadixBits * p, false, w, info, s);
        cur ^= 1;
    }
    radix_pass(ArraySrc<K>{keys[cur], w.vals[cur]}, RankDst<K>{order}, nullptr, n, workers,
               kRadixBits * (passes - 1), false, w, info, s);
}

// Sorts the listed (asc, desc) pair keys in keys[0]/vals[0] (count in
// counters[0], known only on the device); returns the buffer index holding the
// result.
int sort_pairs(int bits, const Work& w, hipStream_t s) {
    const int passes = (bits + kRadixBits - 1) / kRadixBits;
    uint64_t* keys[2] = {reinterpret_cast<uint64_t*>(w.keys[0]),
                         reinterpret_cast<uint64_t*>(w.keys[1])};
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        radix_pass(ArraySrc<uint64_t>{keys[cur], w.vals[cur]},
                   ArrayDst<uint64_t>{keys[cur ^ 1], w.vals[cur ^ 1]}, w.counters, 0, kWorkers,
                   kRadixBits * p, false, w, nullptr, s);
        cur ^= 1;
    }
    return cur;
}

// Exclusive prefix of in[0..m) into out (host-known m).
void prefix_sum(const uint32_t* in, uint32_t m, uint32_t* out, uint32_t* total, const Work& w,
                hipStream_t s) {
    launch(PLMSS_KERNEL_PREFIX, s, [&] { k_sum_reduce<<<kWorkers, kBlock, 0, s>>>(in, nullptr, m, w.partial); });
    launch(PLMSS_KERNEL_PREFIX, s, [&] { k_scan_partials<<<1, kBlock, 0, s>>>(w.partial, kWorkers, total); });
    launch(PLMSS_KERNEL_PREFIX, s, [&] { k_scan_apply<<<kWorkers, kBlock, 0, s>>>(in, nullptr, m, w.partial, out); });
}

// MS ids from the pairs listed per chase tile (rec = keys[1], counts in
// reg_cnt, slots in ms): compact, sort, rank, relabel.
void ms_from_pairs(int32_t* ms, uint32_t n, uint32_t nregions, int bn, int32_t* info, const Work& w,
                   hipStream_t s) {
    uint64_t* rec = reinterpret_cast<uint64_t*>(w.keys[1]);
    prefix_sum(w.reg_cnt, nregions, w.reg_off, w.counters + 0, w, s);
    launch(PLMSS_KERNEL_COMPACT, s, [&] {
        k_compact_pairs<<<nregions, kBlock, 0, s>>>(w.reg_cnt, w.reg_off, rec,
                                                     reinterpret_cast<uint64_t*>(w.keys[0]), w.vals[0]);
    });
    const int r = sort_pairs(2 * bn, w, s);
    const uint64_t* sk = reinterpret_cast<const uint64_t*>(w.keys[r]);
    launch(PLMSS_KERNEL_RANK, s, [&] { k_rank_reduce<<<kWorkers, kBlock, 0, s>>>(sk, w.counters + 0, w.partial); });
    launch(PLMSS_KERNEL_PREFIX, s, [&] { k_scan_partials<<<1, kBlock, 0, s>>>(w.partial, kWorkers, w.counters + 1); });
    launch(PLMSS_KERNEL_RANK, s, [&] {
        k_rank_apply<<<kWorkers, kBlock, 0, s>>>(sk, w.vals[r], w.counters + 0, w.partial, w.rank_of);
    });
    if (info) launch(PLMSS_KERNEL_MISC, s, [&] { k_store_k<<<1, 64, 0, s>>>(info, w.counters + 1); });
    launch(PLMSS_KERNEL_MS_FINAL, s, [&] {
        k_ms_final<<<unsigned((uint64_t(n) + 4 * kBlock - 1) / (4 * kBlock)), kBlock, 0, s>>>(
            ms, n, w.reg_off, w.rank_of);
    });
}

// Labels and pair lists over chase tiles of the plan's shape.
template <bool CHASE>
void launch_chase(const ChasePlan& cp, const plmss_dims& d, uint32_t* U, uint32_t* D, int32_t* desc,
                  int32_t* asc, int bn, int32_t* ms, int32_t* info, const Work& w, hipStream_t s) {
    const GridDims g{int32_t(d.nx), int32_t(d.ny), int32_t(d.nz)};
    uint64_t* rec = reinterpret_cast<uint64_t*>(w.keys[1]);
    const unsigned blocks = unsigned(cp.regions);
    launch(PLMSS_KERNEL_JUMP, s, [&] {
        if (cp.kind == 3)
            k_chase<JTile3, CHASE><<<blocks, kBlock, 0, s>>>(U, D, g, desc, asc, bn, rec, w.reg_cnt, ms, info);
        else if (cp.kind == 2)
            k_chase<JTile2, CHASE><<<blocks, kBlock, 0, s>>>(U, D, g, desc, asc, bn, rec, w.reg_cnt, ms, info);
        else
            k_chase<JTile1, CHASE><<<blocks, kBlock, 0, s>>>(U, D, g, desc, asc, bn, rec, w.reg_cnt, ms, info);
    });
}

// Tile shape of the neighbour scan: kTX x TY columns over ZC planes (3-D), or
// kTX x 16 rectangles (2-D and 1-D fields).
template <bool RESOLVE, class Src>
void launch_steepest(Src src, const plmss_dims& d, uint32_t* up, uint32_t* dn, int32_t* info,
                     hipStream_t s) {
    const GridDims g{int32_t(d.nx), int32_t(d.ny), int32_t(d.nz)};
    launch(PLMSS_KERNEL_STEEPEST, s, [&] {
        if (d.nz > 1)
            k_steepest<Src, 8, 16, RESOLVE><<<steepest_blocks(g, 8, 16), kBlock, 0, s>>>(src, g, up, dn, info);
        else
            k_steepest<Src, 16, 1, RESOLVE><<<steepest_blocks(g, 16, 1), kBlock, 0, s>>>(src, g, up, dn, info);
    });
}

template <bool RESOLVE>
void steepest_any(const void* field, const int32_t* order, const plmss_dims& d, int32_t dtype,
                  uint32_t* up, uint32_t* dn, int32_t* info, hipStream_t s) {
    if (order)
        launch_steepest<RESOLVE>(RankOrder{order}, d, up, dn, info, s);
    else if (dtype == PLMSS_F32)
        launch_steepest<RESOLVE>(FieldOrder<float, uint32_t>{static_cast<const float*>(field)}, d, up,
                                 dn, info, s);
    else
        launch_steepest<RESOLVE>(FieldOrder<double, uint64_t>{static_cast<const double*>(field)}, d,
                                 up, dn, info, s);
}

void order_any(const void* field, int32_t dtype, uint32_t n, int32_t* order, const Work& w,
               int32_t* info, hipStream_t s) {
    if (dtype == PLMSS_F32)
        sort_order<float, uint32_t>(static_cast<const float*>(field), n, order, w, info, s);
    else
        sort_order<double, uint64_t>(static_cast<const double*>(field), n, order, w, info, s);
}

bool ws_ok(const void* ws, size_t have, size_t need) {
    return ws != nullptr && have >= need && (reinterpret_cast<uintptr_t>(ws) % 256) == 0;
}

}  // namespace

extern "C" {

const char* plmss_status_string(int code) {
    switch (code) {
        case PLMSS_OK: return "ok";
        case PLMSS_E_ARG: return "invalid argument (NULL pointer or bad enum value)";
        case PLMSS_E_DIMS: return "invalid grid dimensions (each must be >= 1)";
        case PLMSS_E_TOO_LARGE: return "grid too large (more than 2^31-1 vertices)";
        case PLMSS_E_NAN: return "the field contains NaN";
        case PLMSS_E_WORKSPACE: return "workspace missing, misaligned or too small";
        case PLMSS_E_HIP: return "HIP runtime or launch error";
        case PLMSS_E_NOCONV: return "path compression did not converge (pointers do not form a forest)";
        default: return "unknown status";
    }
}

const char* plmss_build_info(void) { return "libplmss 0.1 gfx950 wave64"; }

size_t plmss_workspace_bytes(plmss_dims dims, int32_t dtype, int32_t with_order) {
    uint64_t n;
    if (check_dims(dims, &n) != PLMSS_OK) return 0;
    (void)dtype;
    (void)with_order;
    return work_sizes(dims, n).total;
}

int plmss_segment(const plmss_job* job, void* workspace, size_t workspace_bytes, void* stream) {
    if (!job || !job->field || !job->asc || !job->desc || !job->ms) return PLMSS_E_ARG;
    if (job->dtype != PLMSS_F32 && job->dtype != PLMSS_F64) return PLMSS_E_ARG;
    uint64_t n;
    int rc = check_dims(job->dims, &n);
    if (rc) return rc;
    const ChasePlan cp = chase_plan(job->dims);
    if (cp.regions * kJV > 0xffffffffull) return PLMSS_E_TOO_LARGE;
    const Sizes sz = work_sizes(n, cp.regions, 0);
    if (!ws_ok(workspace, workspace_bytes, sz.total)) return PLMSS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Work w = carve(workspace, sz);
    const uint32_t n32 = uint32_t(n);
    const int bn = id_bits(n);
    uint32_t* U = reinterpret_cast<uint32_t*>(w.keys[0]);
    uint32_t* D = U + w.npad;
    launch(PLMSS_KERNEL_MISC, s, [&] { k_init<<<1, 64, 0, s>>>(job->info, w.counters, 64); });
    if (job->order) order_any(job->field, job->dtype, n32, job->order, w, job->info, s);
    steepest_any<true>(job->field, job->order, job->dims, job->dtype, U, D, job->info, s);
    launch_chase<true>(cp, job->dims, U, D, job->desc, job->asc, bn, job->ms, job->info, w, s);
    ms_from_pairs(job->ms, n32, uint32_t(cp.regions), bn, job->info, w, s);
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
    const Sizes sz = work_sizes(dims, n);
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
    steepest_any<false>(field, order, dims, dtype, reinterpret_cast<uint32_t*>(up),
                        reinterpret_cast<uint32_t*>(dn), info, s);
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
    return work_sizes(plmss_dims{n, 1, 1}, uint64_t(n)).total;
}

int plmss_ms_ids(const int32_t* asc, const int32_t* desc, int64_t n, int32_t* ms, int32_t* info,
                 void* workspace, size_t workspace_bytes, void* stream) {
    if (!asc || !desc || !ms) return PLMSS_E_ARG;
    if (n < 1) return PLMSS_E_DIMS;
    if (n > kMaxN) return PLMSS_E_TOO_LARGE;
    const plmss_dims d{n, 1, 1};
    const ChasePlan cp = chase_plan(d);
    const Sizes sz = work_sizes(uint64_t(n), cp.regions, 0);
    if (!ws_ok(workspace, workspace_bytes, sz.total)) return PLMSS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Work w = carve(workspace, sz);
    const uint32_t n32 = uint32_t(n);
    const int bn = id_bits(uint64_t(n));
    launch(PLMSS_KERNEL_MISC, s, [&] { k_init<<<1, 64, 0, s>>>(info, w.counters, 64); });
    // the labels are only read
    launch_chase<false>(cp, d, nullptr, nullptr, const_cast<int32_t*>(desc), const_cast<int32_t*>(asc), bn,
                        ms, info, w, s);
    ms_from_pairs(ms, n32, uint32_t(cp.regions), bn, info, w, s);
    return launch_status();
}

size_t plmss_batch_workspace_bytes(int32_t n_jobs, const plmss_job* jobs) {
    (void)n_jobs;
    (void)jobs;
    return 0;
}

int plmss_segment_batch(int32_t n_jobs, const plmss_job* jobs, void* workspace,
                        size_t workspace_bytes, void* stream) {
    (void)n_jobs;
    (void)jobs;
    (void)workspace;
    (void)workspace_bytes;
    (void)stream;
    return PLMSS_E_ARG;
}

struct plmss_trace {
    Trace t;
};

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
        "misc", "radix_hist", "radix_digit_scan", "radix_scatter", "steepest",
        "jump", "prefix_sum", "pair_compact", "pair_rank", "ms_final"};
    return (kind >= 0 && kind < PLMSS_KERNEL_KINDS) ? names[kind] : "unknown";
}

}  // extern "C"
