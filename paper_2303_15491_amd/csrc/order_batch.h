// Order fields of a batch (paper, Sec. "Preprocessing", for every field of a
// batch at once).  All fields' vertices are sorted together by the key (field
// index, value, vertex id): the launch numbers field j's vertices
// vbase_j .. vbase_j + N_j - 1 in job order, so after the sort field j
// occupies exactly those positions, and a vertex's order within its field is
// its position minus vbase_j.  Ties of value fall to the id, as for one field,
// because launch-wide ids follow field-local ids within a field.
//
// The passes: a gather writes each vertex's key at its launch-wide id; the
// first LSD pass reads those keys with the ids generated from their
// positions (IndexValSrc), and it and the usual LSD passes after it sort the
// (key, id) items by key, the last of them storing each item's field index
// (found from its id) in place of the key; then passes over the digits of
// the field index make the field the most significant part; the last of
// them feeds the inversion by id chunks, whose final kernel writes each
// chunk's entries through the descriptors into the fields' own order arrays.
#pragma once

#include "segment.h"
#include "sort.h"

namespace plmss {

// Index of the field holding launch-wide vertex g (fields are in vbase order).
__device__ __forceinline__ uint32_t field_index_of_vertex(const Fields& F, uint32_t g) {
    if (!F.table) return 0;
    uint32_t lo = 0, hi = fields_count(F);
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (gmem(F.table)[mid].vbase <= g)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// The keys of a batch in launch-wide order: keys[g] = key of field j's value
// at g - vbase_j (the id g is implied by the position).  A NaN sets its
// field's info[0].  Grid: one block per kTile vertices of the length
// count_ptr points to (or n); blocks past it exit.
template <typename T, typename K>
__global__ __launch_bounds__(kBlock) void k_batch_keys(Fields F, const uint32_t* count_ptr, uint32_t n_host,
                                                       K* keys) {
    const uint32_t n = load_count(count_ptr, n_host);
    const uint32_t lo = blockIdx.x * uint32_t(kTile);
    if (lo >= n) return;
    const uint32_t hi = min(n, lo + uint32_t(kTile));
    const uint32_t nf = fields_count(F);
    const uint32_t first = lo + threadIdx.x;
    if (first >= hi) return;
    uint32_t f = field_index_of_vertex(F, first);
    uint32_t next = f + 1 < nf ? gmem(F.table)[f + 1].vbase : ~0u;
    const T* src = static_cast<const T*>(gmem(F.table)[f].src);
    uint32_t vbase = gmem(F.table)[f].vbase;
    for (uint32_t g = first; g < hi; g += kBlock) {
        if (g >= next) {
            do {
                ++f;
                next = f + 1 < nf ? gmem(F.table)[f + 1].vbase : ~0u;
            } while (g >= next);
            src = static_cast<const T*>(gmem(F.table)[f].src);
            vbase = gmem(F.table)[f].vbase;
        }
        const T v = gmem(src)[g - vbase];
        if (is_nan(v)) {
            int32_t* info = gmem(F.table)[f].info;
            if (info) gmem(info)[0] = -4;  // PLMSS_E_NAN
        }
        keys[g] = sos_key(v);
    }
}

// The last key pass of a batch's order sort: each item leaves as (index of
// the field holding its id, id), the field index in place of the key (which
// the remaining passes, over the field index, no longer need).
struct PackedFieldDst {
    uint64_t* kv;
    Fields F;
    __device__ __forceinline__ void put(uint32_t pos, uint32_t, uint32_t v) const {
        kv[pos] = (uint64_t(field_index_of_vertex(F, v)) << 32) | v;
    }
};

// The inversion of one id chunk of a batch: as k_invert_chunks, but entry
// (launch-wide id g, position p) becomes order_j[g - vbase_j] = p - vbase_j in
// the order array of the field j holding g (fields without one are skipped).
// Grid: one block per chunk of the length count_ptr points to (or n).
// A pair lost by the regrouping (*bad) is reported in every field's info[0]
// as PLMSS_E_INTERNAL.
__global__ __launch_bounds__(kInvertBlock) void k_invert_chunks_batch(const uint64_t* parts,
                                                                      const uint32_t* count_ptr, uint32_t n_host,
                                                                      Fields F, const uint32_t* bad) {
    __shared__ uint32_t buf[kChunk];
    if (blockIdx.x == 0 && *bad)
        for (uint32_t f = threadIdx.x; f < fields_count(F); f += kInvertBlock) {
            int32_t* info = gmem(F.table)[f].info;
            if (info) gmem(info)[0] = -8;  // PLMSS_E_INTERNAL
        }
    const uint32_t n = load_count(count_ptr, n_host);
    const uint32_t base = blockIdx.x << kChunkBits;
    if (base >= n) return;
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
    const uint32_t nf = fields_count(F);
    const uint32_t first = base + threadIdx.x;
    if (threadIdx.x >= cnt) return;
    uint32_t f = field_index_of_vertex(F, first);
    uint32_t next = f + 1 < nf ? gmem(F.table)[f + 1].vbase : ~0u;
    int32_t* order = gmem(F.table)[f].order;
    uint32_t vbase = gmem(F.table)[f].vbase;
    for (uint32_t j = threadIdx.x; j < cnt; j += kInvertBlock) {
        const uint32_t g = base + j;
        if (g >= next) {
            do {
                ++f;
                next = f + 1 < nf ? gmem(F.table)[f + 1].vbase : ~0u;
            } while (g >= next);
            order = gmem(F.table)[f].order;
            vbase = gmem(F.table)[f].vbase;
        }
        if (order) gmem(order)[g - vbase] = int32_t(buf[j] - vbase);
    }
}

}  // namespace plmss
