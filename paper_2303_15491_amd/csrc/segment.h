// Segmentation kernels: steepest neighbours, path compression with MS-pair
// emission, MS-pair compaction and ranking.
#pragma once

#include "common.h"
#include "sort.h"

namespace plmss {

// ---- vertex-order sources for the neighbour scan ---------------------------------

// The order of a float field under the paper's tie rule, compared through
// order-preserving integer keys (vertex ids break ties, see k_steepest).
template <typename T, typename K>
struct FieldOrder {
    using key_t = K;
    static constexpr bool kCheckNan = true;
    const T* f;
    __device__ __forceinline__ K load(size_t i, bool& nan) const {
        const T a = f[i];
        nan |= is_nan(a);
        return sos_key(a);
    }
};

// A materialised order field (distinct ranks).
struct RankOrder {
    using key_t = uint32_t;
    static constexpr bool kCheckNan = false;
    const int32_t* order;
    __device__ __forceinline__ uint32_t load(size_t i, bool&) const { return uint32_t(order[i]); }
};

// ---- steepest neighbours ------------------------------------------------------------
//
// A block owns a kTX x kTY column of the grid over kZC consecutive planes and
// marches through them, keeping planes z-1, z, z+1 (with a one-vertex halo) in
// LDS.  Every vertex compares its 14 neighbours.  The neighbourhood listed in
// increasing vertex-id order is
//   (-1,-1,-1) (0,-1,-1) (-1,0,-1) (0,0,-1) (-1,-1,0) (0,-1,0) (-1,0,0)
//   [self] (1,0,0) (0,1,0) (1,1,0) (0,0,1) (1,0,1) (0,1,1) (1,1,1)
// (true whenever the offsets are inside the grid), so scanning it in that
// order with ">=" for the maximum and "<" for the minimum breaks equal keys by
// vertex id exactly as the vertex order does.

constexpr int kTX = 64, kTY = 8, kZC = 16;
constexpr int kPX = kTX + 2, kPY = kTY + 2;
constexpr int kRowsPerWave = kTY / kWavesPerBlock;

struct GridDims {
    int32_t nx, ny, nz;
};

template <class Src, bool CHECK>
__device__ __forceinline__ void steepest_vertex(const typename Src::key_t (*pl)[kPY][kPX], int pm,
                                                int pc, int pn, int lx, int ly, bool xm, bool xp,
                                                bool ym, bool yp, bool zm, bool zp,
                                                const int32_t* offs, int32_t& off_up,
                                                int32_t& off_dn) {
    using K = typename Src::key_t;
    K bu = K(0), bd = ~K(0);
    int32_t ou = 0, od = 0;
    auto cand = [&](K k, bool ok, int32_t o) {
        const bool gu = (!CHECK || ok) && (k >= bu);
        const bool gd = (!CHECK || ok) && (k < bd);
        bu = gu ? k : bu;
        ou = gu ? o : ou;
        bd = gd ? k : bd;
        od = gd ? o : od;
    };
    const int cx = lx + 1, cy = ly + 1;
    cand(pl[pm][cy - 1][cx - 1], xm && ym && zm, offs[0]);
    cand(pl[pm][cy - 1][cx], ym && zm, offs[1]);
    cand(pl[pm][cy][cx - 1], xm && zm, offs[2]);
    cand(pl[pm][cy][cx], zm, offs[3]);
    cand(pl[pc][cy - 1][cx - 1], xm && ym, offs[4]);
    cand(pl[pc][cy - 1][cx], ym, offs[5]);
    cand(pl[pc][cy][cx - 1], xm, offs[6]);
    cand(pl[pc][cy][cx], true, 0);
    cand(pl[pc][cy][cx + 1], xp, offs[7]);
    cand(pl[pc][cy + 1][cx], yp, offs[8]);
    cand(pl[pc][cy + 1][cx + 1], xp && yp, offs[9]);
    cand(pl[pn][cy][cx], zp, offs[10]);
    cand(pl[pn][cy][cx + 1], xp && zp, offs[11]);
    cand(pl[pn][cy + 1][cx], yp && zp, offs[12]);
    cand(pl[pn][cy + 1][cx + 1], xp && yp && zp, offs[13]);
    off_up = ou;
    off_dn = od;
}

// up/dn: the steepest ascending / descending neighbour (v itself at a
// maximum / minimum).  cnt[0] += #minima, cnt[1] += #maxima; info[0] = NaN flag.
template <class Src>
__global__ __launch_bounds__(kBlock) void k_steepest(Src src, GridDims g, int32_t* up,
                                                     int32_t* dn, int32_t* info) {
    using K = typename Src::key_t;
    __shared__ K pl[3][kPY][kPX];
    __shared__ uint32_t cnt_min, cnt_max;
    __shared__ int nan_seen;
    const int t = threadIdx.x, w = wave_id(), lane = lane_id();
    const int tx = (g.nx + kTX - 1) / kTX, ty = (g.ny + kTY - 1) / kTY;
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const int bx = int(b % uint32_t(tx));
    const int by = int((b / uint32_t(tx)) % uint32_t(ty));
    const int bz = int(b / (uint32_t(tx) * uint32_t(ty)));
    const int x0 = bx * kTX, y0 = by * kTY, z0 = bz * kZC;
    const int z1 = min(g.nz, z0 + kZC);
    const size_t sx = size_t(g.nx), sxy = size_t(g.nx) * size_t(g.ny);
    // linear offsets of the 14 neighbours in increasing order (self excluded);
    // unsigned arithmetic so that offsets leaving a degenerate grid wrap
    // harmlessly (they are never used)
    const uint32_t S = uint32_t(sxy), X = uint32_t(g.nx);
    const int32_t offs[14] = {int32_t(0u - (S + X + 1)), int32_t(0u - (S + X)), int32_t(0u - (S + 1)),
                              int32_t(0u - S),           int32_t(0u - (X + 1)), int32_t(0u - X),
                              -1,                        1,                     int32_t(X),
                              int32_t(X + 1),            int32_t(S),            int32_t(S + 1),
                              int32_t(S + X),            int32_t(S + X + 1)};
    if (t == 0) {
        cnt_min = 0;
        cnt_max = 0;
        nan_seen = 0;
    }
    bool nan = false;
    auto load_plane = [&](int slot, int z) {
        for (int i = t; i < kPY * kPX; i += kBlock) {
            const int r = i / kPX, c = i - r * kPX;
            const int gx = x0 - 1 + c, gy = y0 - 1 + r;
            K k = K(0);
            if (gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny)
                k = src.load(size_t(z) * sxy + size_t(gy) * sx + size_t(gx), nan);
            pl[slot][r][c] = k;
        }
    };
    int pm = 0, pc = 1, pn = 2;
    if (z0 > 0) load_plane(pm, z0 - 1);
    load_plane(pc, z0);
    const int x = x0 + lane;
    const bool xm = x > 0, xp = x < g.nx - 1;
    uint32_t my_min = 0, my_max = 0;
    for (int z = z0; z < z1; ++z) {
        if (z + 1 < g.nz) load_plane(pn, z + 1);
        __syncthreads();
        const bool zm = z > 0, zp = z < g.nz - 1;
        const bool interior = x0 > 0 && x0 + kTX < g.nx && y0 > 0 && y0 + kTY < g.ny && zm && zp;
#pragma unroll
        for (int r = 0; r < kRowsPerWave; ++r) {
            const int ly = w * kRowsPerWave + r, y = y0 + ly;
            const bool inside = x < g.nx && y < g.ny;
            const bool ym = y > 0, yp = y < g.ny - 1;
            int32_t ou, od;
            if (interior)
                steepest_vertex<Src, false>(pl, pm, pc, pn, lane, ly, xm, xp, ym, yp, zm, zp, offs,
                                            ou, od);
            else
                steepest_vertex<Src, true>(pl, pm, pc, pn, lane, ly, xm, xp, ym, yp, zm, zp, offs,
                                           ou, od);
            if (inside) {
                const size_t v = size_t(z) * sxy + size_t(y) * sx + size_t(x);
                up[v] = int32_t(v) + ou;
                dn[v] = int32_t(v) + od;
                my_max += (ou == 0);
                my_min += (od == 0);
            }
        }
        __syncthreads();
        const int tmp = pm;
        pm = pc;
        pc = pn;
        pn = tmp;
    }
    if (my_min) atomicAdd(&cnt_min, my_min);
    if (my_max) atomicAdd(&cnt_max, my_max);
    if (Src::kCheckNan && nan) nan_seen = 1;
    __syncthreads();
    if (t == 0 && info) {
        if (cnt_min) atomicAdd(reinterpret_cast<uint32_t*>(info + 1), cnt_min);
        if (cnt_max) atomicAdd(reinterpret_cast<uint32_t*>(info + 2), cnt_max);
        if (nan_seen) info[0] = -4;  // PLMSS_E_NAN
    }
}

inline int steepest_blocks(const GridDims& g) {
    const int tx = (g.nx + kTX - 1) / kTX, ty = (g.ny + kTY - 1) / kTY, tz = (g.nz + kZC - 1) / kZC;
    return tx * ty * tz;
}

// ---- path compression -----------------------------------------------------------------
//
// One lane per vertex chases both of its pointers, p <- p[p], until p[p] == p.
// The arrays are updated in place as lanes go, so a lane reading a pointer that
// another lane has already compressed jumps further.  Every value a lane can
// read for p[x] is an ancestor of x on the same chain (roots never change and a
// non-root is never set to itself), so each step advances and the fixed point
// is the chain's root whatever the interleaving.
//
// EMIT: afterwards every wave of 64 consecutive vertices lists its distinct
// (asc, desc) pairs as keys (asc << bn) | desc in rec[64*wave + j], stores the
// count in wave_cnt[wave] and writes the gapped slot 64*wave + j of each
// vertex's pair into ms[v] (replaced by the MS id later).

template <bool JUMP, bool EMIT>
__global__ __launch_bounds__(kBlock) void k_jump(int32_t* desc, int32_t* asc, uint32_t n, int bn,
                                                 uint64_t* rec, uint32_t* wave_cnt, int32_t* ms) {
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t v = b * kBlock + threadIdx.x;
    const bool valid = v < n;
    int32_t pu = valid ? desc[v] : 0, pd = valid ? asc[v] : 0;
    if (JUMP) {
        bool du = !valid || pu == int32_t(v), dd = !valid || pd == int32_t(v);
        while (!(du && dd)) {
            if (!du) {
                const int32_t q = desc[pu];
                if (q == pu) {
                    du = true;
                } else {
                    pu = q;
                    desc[v] = q;
                }
            }
            if (!dd) {
                const int32_t q = asc[pd];
                if (q == pd) {
                    dd = true;
                } else {
                    pd = q;
                    asc[v] = q;
                }
            }
        }
    }
    if (EMIT) {
        const int lane = lane_id();
        const uint32_t wave = v / kWave;
        const uint64_t key = (uint64_t(uint32_t(pd)) << bn) | uint64_t(uint32_t(pu));
        uint64_t rem = __ballot(valid);
        uint32_t j = 0, mine = 0;
        while (rem) {
            const int leader = __ffsll(static_cast<unsigned long long>(rem)) - 1;
            const uint64_t lk = __shfl(key, leader, kWave);
            const bool m = valid && key == lk;
            const uint64_t mm = __ballot(m);
            if (m) mine = j;
            if (lane == leader) rec[size_t(wave) * kWave + j] = lk;
            rem &= ~mm;
            ++j;
        }
        if (valid) ms[v] = int32_t(wave * kWave + mine);
        if (lane == 0 && wave * kWave < n) wave_cnt[wave] = j;
    }
}

// Exclusive scan of wave_cnt (worker slices of kBlock waves, offsets from
// partial[]) fused with copying each wave's pairs into a dense array:
// keys[off + j] = rec[64*wave + j], vals[off + j] = 64*wave + j.
__global__ __launch_bounds__(kBlock) void k_compact_pairs(const uint32_t* wave_cnt, uint32_t nwaves,
                                                          const uint32_t* partial,
                                                          const uint64_t* rec, uint64_t* keys,
                                                          uint32_t* vals) {
    __shared__ uint32_t tmp[kWavesPerBlock];
    uint32_t lo, hi;
    worker_range(nwaves, blockIdx.x, gridDim.x, kBlock, &lo, &hi);
    uint32_t run = partial[blockIdx.x];
    for (uint32_t base = lo; base < hi; base += kBlock) {
        const uint32_t wv = base + threadIdx.x;
        const uint32_t c = wv < hi ? wave_cnt[wv] : 0u;
        uint32_t tot;
        const uint32_t off = run + block_exclusive_scan(c, tmp, &tot);
        for (uint32_t j = 0; j < c; ++j) {
            keys[off + j] = rec[size_t(wv) * kWave + j];
            vals[off + j] = wv * kWave + j;
        }
        run += tot;
    }
}

// Ranking the sorted pairs: flag[i] = (i == 0 || key[i] != key[i-1]);
// rank[i] = (number of flags in 0..i) - 1.
__device__ __forceinline__ uint32_t pair_flag(const uint64_t* keys, uint32_t i) {
    return (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ __launch_bounds__(kBlock) void k_rank_reduce(const uint64_t* keys,
                                                        const uint32_t* count_ptr,
                                                        uint32_t* partial) {
    __shared__ uint32_t tmp[kWavesPerBlock];
    uint32_t lo, hi;
    worker_range(*count_ptr, blockIdx.x, gridDim.x, kBlock, &lo, &hi);
    uint32_t s = 0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += kBlock) s += pair_flag(keys, i);
    uint32_t tot;
    block_exclusive_scan(s, tmp, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// rank_of_slot[vals[i]] = rank[i]; info[3] = K (taken from *k_total).
__global__ __launch_bounds__(kBlock) void k_rank_apply(const uint64_t* keys, const uint32_t* vals,
                                                       const uint32_t* count_ptr,
                                                       const uint32_t* partial,
                                                       uint32_t* rank_of_slot) {
    __shared__ uint32_t tmp[kWavesPerBlock];
    uint32_t lo, hi;
    worker_range(*count_ptr, blockIdx.x, gridDim.x, kBlock, &lo, &hi);
    uint32_t run = partial[blockIdx.x];
    for (uint32_t base = lo; base < hi; base += kBlock) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t f = i < hi ? pair_flag(keys, i) : 0u;
        uint32_t tot;
        const uint32_t excl = block_exclusive_scan(f, tmp, &tot);
        if (i < hi) rank_of_slot[vals[i]] = run + excl + f - 1;
        run += tot;
    }
}

__global__ __launch_bounds__(kBlock) void k_ms_final(int32_t* ms, uint32_t n,
                                                     const uint32_t* rank_of_slot) {
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t v = b * kBlock + threadIdx.x;
    if (v < n) ms[v] = int32_t(rank_of_slot[uint32_t(ms[v])]);
}

// info[0..3] = 0; counters[0..m) = 0.
__global__ void k_init(int32_t* info, uint32_t* counters, int m) {
    const int t = threadIdx.x;
    if (info && t < 4) info[t] = 0;
    if (counters && t < m) counters[t] = 0;
}

__global__ void k_store_k(int32_t* info, const uint32_t* k_total) {
    if (threadIdx.x == 0 && info) info[3] = int32_t(*k_total);
}

}  // namespace plmss
