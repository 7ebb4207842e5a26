// libplmss: C ABI of the gfx950 Morse-Smale segmentation (see include/plmss.h).
#include "plmss.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>

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
    uint8_t* keys[2];      // u64[npad] each: sort keys (ping-pong); keys[1] also holds the
                           // gapped pair list written by the compression kernel
    uint32_t* vals[2];     // u32[npad] each: sort values
    uint32_t* rank_of_slot;  // u32[npad]
    uint32_t* wave_cnt;    // u32[nwaves]
    uint32_t* hist;        // u32[kRadix * kWorkers]
    uint32_t* dtotal;      // u32[kRadix]
    uint32_t* partial;     // u32[kWorkers]
    uint32_t* counters;    // u32[64]: [0] = #pairs listed, [1] = K
    uint8_t* extra;        // batch tables
};

struct Sizes {
    size_t keys, vals, rank, wave_cnt, hist, dtotal, partial, counters, extra, total;
};

Sizes work_sizes(uint64_t n, size_t extra) {
    Sizes s;
    const uint64_t npad = align_up(n, kBlock);
    const uint64_t nwaves = (n + kWave - 1) / kWave;
    s.keys = align_up(8 * npad, 256);
    s.vals = align_up(4 * npad, 256);
    s.rank = align_up(4 * npad, 256);
    s.wave_cnt = align_up(4 * nwaves, 256);
    s.hist = align_up(size_t(4) * kRadix * kWorkers, 256);
    s.dtotal = align_up(4 * kRadix, 256);
    s.partial = align_up(4 * kWorkers, 256);
    s.counters = 256;
    s.extra = align_up(extra, 256);
    s.total = 2 * s.keys + 2 * s.vals + s.rank + s.wave_cnt + s.hist + s.dtotal + s.partial +
              s.counters + s.extra;
    return s;
}

Work carve(void* ws, const Sizes& s) {
    Work w;
    uint8_t* p = static_cast<uint8_t*>(ws);
    w.keys[0] = p;
    p += s.keys;
    w.keys[1] = p;
    p += s.keys;
    w.vals[0] = reinterpret_cast<uint32_t*>(p);
    p += s.vals;
    w.vals[1] = reinterpret_cast<uint32_t*>(p);
    p += s.vals;
    w.rank_of_slot = reinterpret_cast<uint32_t*>(p);
    p += s.rank;
    w.wave_cnt = reinterpret_cast<uint32_t*>(p);
    p += s.wave_cnt;
    w.hist = reinterpret_cast<uint32_t*>(p);
    p += s.hist;
    w.dtotal = reinterpret_cast<uint32_t*>(p);
    p += s.dtotal;
    w.partial = reinterpret_cast<uint32_t*>(p);
    p += s.partial;
    w.counters = reinterpret_cast<uint32_t*>(p);
    p += s.counters;
    w.extra = p;
    return w;
}

int launch_status() { return hipGetLastError() == hipSuccess ? PLMSS_OK : PLMSS_E_HIP; }

unsigned grid_for(uint64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

// ---- radix sort driver -------------------------------------------------------------------

template <class Src, class Dst>
void radix_pass(Src src, Dst dst, const uint32_t* cnt, uint32_t n, int shift, bool check_nan,
                const Work& w, int32_t* info, hipStream_t s) {
    if (check_nan)
        k_radix_hist<Src, true><<<kWorkers, kBlock, 0, s>>>(src, cnt, n, shift, w.hist, info);
    else
        k_radix_hist<Src, false><<<kWorkers, kBlock, 0, s>>>(src, cnt, n, shift, w.hist, info);
    k_radix_digit_scan<<<kRadix, kBlock, 0, s>>>(w.hist, w.dtotal, kWorkers);
    k_radix_scatter<Src, Dst><<<kWorkers, kBlock, 0, s>>>(src, dst, cnt, n, shift, w.hist, w.dtotal);
}

// Order field of a float field: keys from the values, values = ids; the last
// pass writes order[id] = position.
template <typename T, typename K>
void sort_order(const T* f, uint32_t n, int32_t* order, const Work& w, int32_t* info,
                hipStream_t s) {
    constexpr int passes = int(sizeof(K)) * 8 / kRadixBits;
    K* keys[2] = {reinterpret_cast<K*>(w.keys[0]), reinterpret_cast<K*>(w.keys[1])};
    FieldSrc<T, K> first{f};
    radix_pass(first, ArrayDst<K>{keys[0], w.vals[0]}, nullptr, n, 0, true, w, info, s);
    int cur = 0;
    for (int p = 1; p < passes - 1; ++p) {
        radix_pass(ArraySrc<K>{keys[cur], w.vals[cur]}, ArrayDst<K>{keys[cur ^ 1], w.vals[cur ^ 1]},
                   nullptr, n, kRadixBits * p, false, w, info, s);
        cur ^= 1;
    }
    radix_pass(ArraySrc<K>{keys[cur], w.vals[cur]}, RankDst<K>{order}, nullptr, n,
               kRadixBits * (passes - 1), false, w, info, s);
}

// Sorts the listed (asc, desc) pair keys in keys[0]/vals[0] (count in
// counters[0]); returns the buffer index holding the result.
int sort_pairs(int bits, uint32_t nmax, const Work& w, hipStream_t s) {
    const int passes = (bits + kRadixBits - 1) / kRadixBits;
    uint64_t* keys[2] = {reinterpret_cast<uint64_t*>(w.keys[0]),
                         reinterpret_cast<uint64_t*>(w.keys[1])};
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        radix_pass(ArraySrc<uint64_t>{keys[cur], w.vals[cur]},
                   ArrayDst<uint64_t>{keys[cur ^ 1], w.vals[cur ^ 1]}, w.counters, nmax,
                   kRadixBits * p, false, w, nullptr, s);
        cur ^= 1;
    }
    return cur;
}

// MS ids from the pairs the compression kernel listed: compact, sort, rank,
// relabel.  ms[] holds gapped slots on entry.
void ms_from_pairs(int32_t* ms, uint32_t n, int bn, int32_t* info, const Work& w, hipStream_t s) {
    const uint32_t nwaves = uint32_t((uint64_t(n) + kWave - 1) / kWave);
    uint64_t* rec = reinterpret_cast<uint64_t*>(w.keys[1]);
    k_sum_reduce<<<kWorkers, kBlock, 0, s>>>(w.wave_cnt, nullptr, nwaves, w.partial);
    k_scan_partials<<<1, kBlock, 0, s>>>(w.partial, kWorkers, w.counters + 0);
    k_compact_pairs<<<kWorkers, kBlock, 0, s>>>(w.wave_cnt, nwaves, w.partial, rec,
                                                reinterpret_cast<uint64_t*>(w.keys[0]), w.vals[0]);
    const int r = sort_pairs(2 * bn, n, w, s);
    const uint64_t* sk = reinterpret_cast<const uint64_t*>(w.keys[r]);
    k_rank_reduce<<<kWorkers, kBlock, 0, s>>>(sk, w.counters + 0, w.partial);
    k_scan_partials<<<1, kBlock, 0, s>>>(w.partial, kWorkers, w.counters + 1);
    k_rank_apply<<<kWorkers, kBlock, 0, s>>>(sk, w.vals[r], w.counters + 0, w.partial,
                                             w.rank_of_slot);
    if (info) k_store_k<<<1, 64, 0, s>>>(info, w.counters + 1);
    k_ms_final<<<grid_for(n), kBlock, 0, s>>>(ms, n, w.rank_of_slot);
}

template <class Src>
void launch_steepest(Src src, const plmss_dims& d, int32_t* up, int32_t* dn, int32_t* info,
                     hipStream_t s) {
    const GridDims g{int32_t(d.nx), int32_t(d.ny), int32_t(d.nz)};
    k_steepest<Src><<<steepest_blocks(g), kBlock, 0, s>>>(src, g, up, dn, info);
}

void steepest_any(const void* field, const int32_t* order, const plmss_dims& d, int32_t dtype,
                  int32_t* up, int32_t* dn, int32_t* info, hipStream_t s) {
    if (order)
        launch_steepest(RankOrder{order}, d, up, dn, info, s);
    else if (dtype == PLMSS_F32)
        launch_steepest(FieldOrder<float, uint32_t>{static_cast<const float*>(field)}, d, up, dn,
                        info, s);
    else
        launch_steepest(FieldOrder<double, uint64_t>{static_cast<const double*>(field)}, d, up, dn,
                        info, s);
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
        default: return "unknown status";
    }
}

const char* plmss_build_info(void) { return "libplmss 0.1 gfx950 wave64"; }

size_t plmss_workspace_bytes(plmss_dims dims, int32_t dtype, int32_t with_order) {
    uint64_t n;
    if (check_dims(dims, &n) != PLMSS_OK) return 0;
    (void)dtype;
    (void)with_order;
    return work_sizes(n, 0).total;
}

int plmss_segment(const plmss_job* job, void* workspace, size_t workspace_bytes, void* stream) {
    if (!job || !job->field || !job->asc || !job->desc || !job->ms) return PLMSS_E_ARG;
    if (job->dtype != PLMSS_F32 && job->dtype != PLMSS_F64) return PLMSS_E_ARG;
    uint64_t n;
    int rc = check_dims(job->dims, &n);
    if (rc) return rc;
    const Sizes sz = work_sizes(n, 0);
    if (!ws_ok(workspace, workspace_bytes, sz.total)) return PLMSS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Work w = carve(workspace, sz);
    const uint32_t n32 = uint32_t(n);
    const int bn = id_bits(n);
    k_init<<<1, 64, 0, s>>>(job->info, w.counters, 64);
    if (job->order) order_any(job->field, job->dtype, n32, job->order, w, job->info, s);
    steepest_any(job->field, job->order, job->dims, job->dtype, job->desc, job->asc, job->info, s);
    k_jump<true, true><<<grid_for(n), kBlock, 0, s>>>(job->desc, job->asc, n32, bn,
                                                      reinterpret_cast<uint64_t*>(w.keys[1]),
                                                      w.wave_cnt, job->ms);
    ms_from_pairs(job->ms, n32, bn, job->info, w, s);
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
    const Sizes sz = work_sizes(n, 0);
    if (!ws_ok(workspace, workspace_bytes, sz.total)) return PLMSS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Work w = carve(workspace, sz);
    if (info) k_init<<<1, 64, 0, s>>>(info, nullptr, 0);
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
    if (info) k_init<<<1, 64, 0, s>>>(info, nullptr, 0);
    steepest_any(field, order, dims, dtype, up, dn, info, s);
    return launch_status();
}

int plmss_compress(int32_t* desc, int32_t* asc, int64_t n, void* stream) {
    if (!desc || !asc) return PLMSS_E_ARG;
    if (n < 1) return PLMSS_E_DIMS;
    if (n > kMaxN) return PLMSS_E_TOO_LARGE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    k_jump<true, false><<<grid_for(uint64_t(n)), kBlock, 0, s>>>(desc, asc, uint32_t(n), 1, nullptr,
                                                                 nullptr, nullptr);
    return launch_status();
}

size_t plmss_ms_workspace_bytes(int64_t n) {
    if (n < 1 || n > kMaxN) return 0;
    return work_sizes(uint64_t(n), 0).total;
}

int plmss_ms_ids(const int32_t* asc, const int32_t* desc, int64_t n, int32_t* ms, int32_t* info,
                 void* workspace, size_t workspace_bytes, void* stream) {
    if (!asc || !desc || !ms) return PLMSS_E_ARG;
    if (n < 1) return PLMSS_E_DIMS;
    if (n > kMaxN) return PLMSS_E_TOO_LARGE;
    const Sizes sz = work_sizes(uint64_t(n), 0);
    if (!ws_ok(workspace, workspace_bytes, sz.total)) return PLMSS_E_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Work w = carve(workspace, sz);
    const uint32_t n32 = uint32_t(n);
    const int bn = id_bits(uint64_t(n));
    k_init<<<1, 64, 0, s>>>(info, w.counters, 64);
    // the labels are only read when JUMP is false
    k_jump<false, true><<<grid_for(uint64_t(n)), kBlock, 0, s>>>(
        const_cast<int32_t*>(desc), const_cast<int32_t*>(asc), n32, bn,
        reinterpret_cast<uint64_t*>(w.keys[1]), w.wave_cnt, ms);
    ms_from_pairs(ms, n32, bn, info, w, s);
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

}  // extern "C"
