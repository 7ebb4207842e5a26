// Segmentation kernels: steepest neighbours with tile-local path compression,
// cross-tile chase, MS-pair listing, compaction and ranking.
#pragma once

#include "common.h"
#include "sort.h"

namespace plmss {

// ---- vertex-order sources for the neighbour scan ---------------------------------

// The order of a float field under the paper's tie rule, compared through
// order-preserving integer keys (vertex ids break ties, see below).
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

struct GridDims {
    int32_t nx, ny, nz;
};

// ---- neighbour codes --------------------------------------------------------------
//
// The 14 neighbours (and the vertex itself) are coded 0..14 as
//   code = 7 + s*(bx + 2*by + 4*bz),  offset = s*(bx, by, bz),  s = +-1,
// with code 7 the vertex itself.  In increasing code order the neighbours are
//   (-1,-1,-1) (0,-1,-1) (-1,0,-1) (0,0,-1) (-1,-1,0) (0,-1,0) (-1,0,0) [self]
//   (1,0,0) (0,1,0) (1,1,0) (0,0,1) (1,0,1) (0,1,1) (1,1,1),
// which is also increasing vertex-id order whenever the offsets lie inside the
// grid.  Scanning them in that order with ">=" for the maximum and "<" for the
// minimum therefore breaks equal keys by vertex id exactly as the vertex order
// of the paper (value, then id) does.
constexpr int kSelf = 7;

__device__ __forceinline__ int32_t code_offset(int code, int32_t nx, int32_t s) {
    const int d = code - kSelf, m = d < 0 ? -d : d;
    const int32_t o = (m & 1) + ((m >> 1) & 1) * nx + ((m >> 2) & 1) * s;
    return d < 0 ? -o : o;
}

constexpr int kTX = 64;  // tile width = one wave

template <class Src, int PY, bool CHECK>
__device__ __forceinline__ void steepest_codes(const typename Src::key_t (*pl)[PY][kTX + 2], int pm,
                                               int pc, int pn, int lx, int ly, bool xm, bool xp,
                                               bool ym, bool yp, bool zm, bool zp, int& cu,
                                               int& cd) {
    using K = typename Src::key_t;
    K bu = K(0), bd = ~K(0);
    int ou = kSelf, od = kSelf;
    auto cand = [&](K k, bool ok, int c) {
        const bool gu = (!CHECK || ok) && (k >= bu);
        const bool gd = (!CHECK || ok) && (k < bd);
        bu = gu ? k : bu;
        ou = gu ? c : ou;
        bd = gd ? k : bd;
        od = gd ? c : od;
    };
    const int x = lx + 1, y = ly + 1;
    cand(pl[pm][y - 1][x - 1], xm && ym && zm, 0);
    cand(pl[pm][y - 1][x], ym && zm, 1);
    cand(pl[pm][y][x - 1], xm && zm, 2);
    cand(pl[pm][y][x], zm, 3);
    cand(pl[pc][y - 1][x - 1], xm && ym, 4);
    cand(pl[pc][y - 1][x], ym, 5);
    cand(pl[pc][y][x - 1], xm, 6);
    cand(pl[pc][y][x], true, 7);
    cand(pl[pc][y][x + 1], xp, 8);
    cand(pl[pc][y + 1][x], yp, 9);
    cand(pl[pc][y + 1][x + 1], xp && yp, 10);
    cand(pl[pn][y][x], zp, 11);
    cand(pl[pn][y][x + 1], xp && zp, 12);
    cand(pl[pn][y + 1][x], yp && zp, 13);
    cand(pl[pn][y + 1][x + 1], xp && yp && zp, 14);
    cu = ou;
    cd = od;
}

constexpr uint32_t kMark = 0x80000000u;     // "this label is an extremum" in a resolved pointer
constexpr uint32_t kMaxHops = 1u << 24;     // iteration cap of the pointer-chasing loops
constexpr uint32_t kExit = 0x8000u;      // local pointer: the target lies outside the tile

// Steepest neighbours of every vertex.
//
// A block owns a kTX x TY column of the grid over ZC consecutive planes and
// marches through them, keeping planes z-1, z, z+1 (with a one-vertex halo) in
// LDS, so the field is read from HBM about once.
//
// RESOLVE == false: up[v] / dn[v] = the steepest ascending / descending
//   neighbour (v itself at a maximum / minimum).
// RESOLVE == true: the paper's path compression is run inside the tile first.
//   Every vertex keeps, in LDS, a pointer to its steepest neighbour if that
//   lies in the tile (or an exit mark with the direction if it does not); the
//   pointers are compressed in place, p <- p[p], until each points at a root
//   of the tile: a true extremum or an exit vertex.  The result written is
//     up[v] = kMark | maximum           if v's ascending chain ends in the tile,
//     up[v] = first vertex outside      otherwise (a pointer still to follow);
//   likewise dn[v].
// info[1] += #minima, info[2] += #maxima; info[0] = PLMSS_E_NAN on a NaN.
template <class Src, int TY, int ZC, bool RESOLVE>
__global__ __launch_bounds__(kBlock) void k_steepest(Src src, GridDims g, uint32_t* up,
                                                     uint32_t* dn, int32_t* info) {
    using K = typename Src::key_t;
    constexpr int PX = kTX + 2, PY = TY + 2, RPW = TY / kWavesPerBlock;
    constexpr int TV = RESOLVE ? kTX * TY * ZC : 1;
    static_assert(TY % kWavesPerBlock == 0, "rows per wave");
    static_assert(kTX * TY * ZC < int(kExit), "local indices need 15 bits");
    __shared__ K pl[3][PY][PX];
    __shared__ uint32_t lp[TV];  // local pointers: up in the low half, dn in the high half
    __shared__ uint32_t cnt_min, cnt_max;
    __shared__ int nan_seen;
    const int t = threadIdx.x, w = wave_id(), lane = lane_id();
    const int tx = (g.nx + kTX - 1) / kTX, ty = (g.ny + TY - 1) / TY;
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const int bx = int(b % uint32_t(tx));
    const int by = int((b / uint32_t(tx)) % uint32_t(ty));
    const int bz = int(b / (uint32_t(tx) * uint32_t(ty)));
    const int x0 = bx * kTX, y0 = by * TY, z0 = bz * ZC;
    const int z1 = min(g.nz, z0 + ZC);
    const size_t sx = size_t(g.nx), sxy = size_t(g.nx) * size_t(g.ny);
    const int32_t S = int32_t(sxy);
    if (t == 0) {
        cnt_min = 0;
        cnt_max = 0;
        nan_seen = 0;
    }
    bool nan = false;
    auto load_plane = [&](int slot, int z) {
        for (int i = t; i < PY * PX; i += kBlock) {
            const int r = i / PX, c = i - r * PX;
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
        const bool interior = x0 > 0 && x0 + kTX < g.nx && y0 > 0 && y0 + TY < g.ny && zm && zp;
        const int lz = z - z0;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int ly = w * RPW + r, y = y0 + ly;
            const bool inside = x < g.nx && y < g.ny;
            const bool ym = y > 0, yp = y < g.ny - 1;
            int cu, cd;
            if (interior)
                steepest_codes<Src, PY, false>(pl, pm, pc, pn, lane, ly, xm, xp, ym, yp, zm, zp, cu, cd);
            else
                steepest_codes<Src, PY, true>(pl, pm, pc, pn, lane, ly, xm, xp, ym, yp, zm, zp, cu, cd);
            if (inside) {
                my_max += (cu == kSelf);
                my_min += (cd == kSelf);
            }
            if (!RESOLVE) {
                if (inside) {
                    const size_t v = size_t(z) * sxy + size_t(y) * sx + size_t(x);
                    up[v] = uint32_t(int32_t(v) + code_offset(cu, g.nx, S));
                    dn[v] = uint32_t(int32_t(v) + code_offset(cd, g.nx, S));
                }
            } else {
                const int li = (lz * TY + ly) * kTX + lane;
                auto local = [&](int c) -> uint32_t {
                    if (!inside) return uint32_t(li);  // padding: a harmless root
                    const int d = c - kSelf, m = d < 0 ? -d : d, s = d < 0 ? -1 : 1;
                    const int ax = lane + s * (m & 1), ay = ly + s * ((m >> 1) & 1),
                              az = lz + s * ((m >> 2) & 1);
                    if (ax < 0 || ax >= kTX || ay < 0 || ay >= TY || az < 0 || az >= ZC)
                        return kExit | uint32_t(c);
                    return uint32_t((az * TY + ay) * kTX + ax);
                };
                lp[li] = local(cu) | (local(cd) << 16);
            }
        }
        __syncthreads();
        const int tmp = pm;
        pm = pc;
        pc = pn;
        pn = tmp;
    }
    if (RESOLVE) {
        // tile-local rows of the last chunk may be missing (z1 - z0 < ZC)
        for (int lz = z1 - z0; lz < ZC; ++lz)
            for (int r = 0; r < RPW; ++r) {
                const int li = (lz * TY + w * RPW + r) * kTX + lane;
                lp[li] = uint32_t(li) | (uint32_t(li) << 16);
            }
        __syncthreads();
        // in-place pointer jumping over the tile; a pointer whose target is
        // an exit vertex (kExit mark) or a root stays put
        for (int round = 0; round < 16; ++round) {
            bool changed = false;
            for (int i = t; i < TV; i += kBlock) {
                const uint32_t e = lp[i];
                uint32_t pu = e & 0xffffu, pd = e >> 16;
                bool ch = false;
                if (!(pu & kExit)) {
                    const uint32_t q = lp[pu] & 0xffffu;
                    if (!(q & kExit) && q != pu) {
                        pu = q;
                        ch = true;
                    }
                }
                if (!(pd & kExit)) {
                    const uint32_t q = lp[pd] >> 16;
                    if (!(q & kExit) && q != pd) {
                        pd = q;
                        ch = true;
                    }
                }
                if (ch) lp[i] = pu | (pd << 16);
                changed |= ch;
            }
            if (!__syncthreads_or(changed)) break;
        }
        // write-out: the root of the tile chain, resolved or to be followed
        const size_t tile0 = size_t(z0) * sxy + size_t(y0) * sx + size_t(x0);
        auto gid = [&](uint32_t li) -> int32_t {
            const int ax = int(li % kTX), ay = int((li / kTX) % TY), az = int(li / (kTX * TY));
            return int32_t(tile0 + size_t(az) * sxy + size_t(ay) * sx + size_t(ax));
        };
        for (int lz = 0; lz < z1 - z0; ++lz) {
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const int ly = w * RPW + r, y = y0 + ly;
                if (x >= g.nx || y >= g.ny) continue;
                const uint32_t li = uint32_t((lz * TY + ly) * kTX + lane);
                const uint32_t e = lp[li];
                auto resolve = [&](uint32_t p, int half) -> uint32_t {
                    if (p & kExit)  // v itself is an exit vertex
                        return uint32_t(gid(li) + code_offset(int(p & 0xffu), g.nx, S));
                    const uint32_t q = (lp[p] >> half) & 0xffffu;
                    if (q == p) return kMark | uint32_t(gid(p));  // an extremum
                    if (q & kExit) return uint32_t(gid(p) + code_offset(int(q & 0xffu), g.nx, S));
                    return uint32_t(gid(p));  // not fully compressed: follow later
                };
                const size_t v = size_t(z0 + lz) * sxy + size_t(y) * sx + size_t(x);
                up[v] = resolve(e & 0xffffu, 0);
                dn[v] = resolve(e >> 16, 16);
            }
        }
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

inline int steepest_blocks(const GridDims& g, int ty, int zc) {
    const int tx = (g.nx + kTX - 1) / kTX, tyn = (g.ny + ty - 1) / ty, tz = (g.nz + zc - 1) / zc;
    return tx * tyn * tz;
}

// ---- chase, labels and MS pair listing ----------------------------------------------
//
// One block per JX x JY x JZ tile (kJV = 2048 vertices, 8 per thread).  For
// every vertex it finishes the tile-compressed pointers: an unresolved pointer
// is followed from tile to tile (each hop lands on the next tile's compressed
// pointer, and is written back so that later readers jump further) until a
// marked extremum.  It writes desc/asc, then lists the tile's distinct
// (asc, desc) pairs through an LDS hash set: keys (asc << bn) | desc go to
// rec[kJV*tile + j], j < reg_cnt[tile], and each vertex's slot kJV*tile + j to
// ms[v] (replaced by the MS id later).  MS regions are a few vertices across,
// so a 3-D tile lists far fewer pairs than a row of the same size would.
constexpr int kJV = 2048;            // vertices per tile
constexpr int kJPer = kJV / kBlock;  // per thread
constexpr int kHash = 2 * kJV;       // hash slots: never more than half full
constexpr uint64_t kEmpty = ~0ull;   // pair keys are < 2^62

template <int JX, int JY, int JZ>
struct JTile {
    static_assert(JX * JY * JZ == kJV, "tile size");
    static constexpr int X = JX, Y = JY, Z = JZ;
};
using JTile3 = JTile<32, 8, 8>;
using JTile2 = JTile<64, 32, 1>;
using JTile1 = JTile<2048, 1, 1>;

template <class T>
inline unsigned chase_blocks(const GridDims& g) {
    return unsigned(((g.nx + T::X - 1) / T::X) * ((g.ny + T::Y - 1) / T::Y) * ((g.nz + T::Z - 1) / T::Z));
}

__device__ __forceinline__ uint32_t pair_hash(uint64_t k) {
    const uint32_t lo = uint32_t(k), hi = uint32_t(k >> 32);
    return (lo * 0x9E3779B1u) ^ (hi * 0x85EBCA77u) ^ (lo >> 15);
}

// CHASE: labels from the tile-compressed pointers U/D (written back as they
// are followed).  Otherwise the labels are read from desc/asc as given.
template <class T, bool CHASE>
__global__ __launch_bounds__(kBlock) void k_chase(uint32_t* U, uint32_t* D, GridDims g,
                                                  int32_t* desc, int32_t* asc, int bn,
                                                  uint64_t* rec, uint32_t* reg_cnt, int32_t* ms,
                                                  int32_t* info) {
    __shared__ uint64_t table[kHash];
    __shared__ uint16_t dense[kHash];
    __shared__ uint32_t tmp[kWavesPerBlock];
    const int t = threadIdx.x;
    const int tx = (g.nx + T::X - 1) / T::X, ty = (g.ny + T::Y - 1) / T::Y;
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const int x0 = int(b % uint32_t(tx)) * T::X;
    const int y0 = int((b / uint32_t(tx)) % uint32_t(ty)) * T::Y;
    const int z0 = int(b / (uint32_t(tx) * uint32_t(ty))) * T::Z;
    const size_t sx = size_t(g.nx), sxy = size_t(g.nx) * size_t(g.ny);
#pragma unroll
    for (int i = 0; i < kHash / kBlock; ++i) table[t + i * kBlock] = kEmpty;
    uint32_t vid[kJPer], pu[kJPer], pd[kJPer];
    bool ok[kJPer];
#pragma unroll
    for (int i = 0; i < kJPer; ++i) {
        const int li = t + i * kBlock;
        const int x = x0 + li % T::X, y = y0 + (li / T::X) % T::Y, z = z0 + li / (T::X * T::Y);
        ok[i] = x < g.nx && y < g.ny && z < g.nz;
        vid[i] = ok[i] ? uint32_t(size_t(z) * sxy + size_t(y) * sx + size_t(x)) : 0u;
        if (CHASE) {
            pu[i] = ok[i] ? U[vid[i]] : kMark;
            pd[i] = ok[i] ? D[vid[i]] : kMark;
        } else {
            pu[i] = ok[i] ? uint32_t(desc[vid[i]]) : 0u;
            pd[i] = ok[i] ? uint32_t(asc[vid[i]]) : 0u;
        }
    }
    if (CHASE) {
        // a pointer leads strictly up (down) its chain, so the hops end; the
        // cap only guards against a malformed input
        // the eight vertices of a thread advance together, so their gathers
        // are in flight at the same time
        bool pending = true;
        uint32_t hops = 0;
        while (pending && hops < kMaxHops) {
            pending = false;
#pragma unroll
            for (int i = 0; i < kJPer; ++i) {
                if (!(pu[i] & kMark)) {
                    pu[i] = U[pu[i]];
                    U[vid[i]] = pu[i];
                    pending = true;
                }
                if (!(pd[i] & kMark)) {
                    pd[i] = D[pd[i]];
                    D[vid[i]] = pd[i];
                    pending = true;
                }
            }
            ++hops;
        }
        const bool capped = pending;
#pragma unroll
        for (int i = 0; i < kJPer; ++i) {
            pu[i] &= ~kMark;
            pd[i] &= ~kMark;
            if (ok[i]) {
                desc[vid[i]] = int32_t(pu[i]);
                asc[vid[i]] = int32_t(pd[i]);
            }
        }
        if (capped && info) info[0] = -7;  // PLMSS_E_NOCONV
    }
    __syncthreads();
    // insert every vertex's pair; slot[i] = its hash slot
    uint32_t slot[kJPer];
#pragma unroll
    for (int i = 0; i < kJPer; ++i) {
        slot[i] = 0;
        if (!ok[i]) continue;
        const uint64_t key = (uint64_t(pd[i]) << bn) | uint64_t(pu[i]);
        uint32_t h = pair_hash(key) & (kHash - 1);
        for (;;) {
            uint64_t cur = table[h];
            if (cur == kEmpty) {
                cur = atomicCAS(reinterpret_cast<unsigned long long*>(&table[h]),
                                static_cast<unsigned long long>(kEmpty),
                                static_cast<unsigned long long>(key));
                if (cur == kEmpty) cur = key;
            }
            if (cur == key) break;
            h = (h + 1) & (kHash - 1);
        }
        slot[i] = h;
    }
    __syncthreads();
    // number the occupied slots in slot order; list their keys
    constexpr int kSlotsPer = kHash / kBlock;
    uint32_t occ = 0;
#pragma unroll
    for (int i = 0; i < kSlotsPer; ++i) occ += table[t * kSlotsPer + i] != kEmpty;
    uint32_t total;
    uint32_t j = block_exclusive_scan(occ, tmp, &total);
    const size_t region = size_t(b) * kJV;
#pragma unroll
    for (int i = 0; i < kSlotsPer; ++i) {
        const int sl = t * kSlotsPer + i;
        const uint64_t k = table[sl];
        if (k != kEmpty) {
            dense[sl] = uint16_t(j);
            rec[region + j] = k;
            ++j;
        }
    }
    if (t == 0) reg_cnt[b] = total;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kJPer; ++i)
        if (ok[i]) ms[vid[i]] = int32_t(uint32_t(region) + dense[slot[i]]);
}

// ---- path compression on global pointers (the step on its own) ---------------------
//
// One lane per vertex chases both of its pointers, p <- p[p], until p[p] == p,
// updating the arrays in place as it goes, so a lane that reads a pointer
// another lane has already compressed jumps further.  Every value a lane can
// read for p[x] is an ancestor of x on the same chain (roots never change and a
// non-root is never set to itself), so each step advances and the fixed point
// is the chain's root whatever the interleaving.
__global__ __launch_bounds__(kBlock) void k_jump(int32_t* desc, int32_t* asc, uint32_t n) {
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t v = b * kBlock + threadIdx.x;
    if (v >= n) return;
    int32_t pu = desc[v], pd = asc[v];
    bool du = pu == int32_t(v), dd = pd == int32_t(v);
    for (uint32_t it = 0; !(du && dd) && it < kMaxHops; ++it) {
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

// ---- pair compaction and ranking ------------------------------------------------------

// One block per tile region: copy its listed pairs to the dense arrays at
// off[region] (exclusive prefix of reg_cnt): keys[o + j] = pair, vals[o + j] =
// o + j (the dense index travels with the key through the sort).
__global__ __launch_bounds__(kBlock) void k_compact_pairs(const uint32_t* reg_cnt,
                                                          const uint32_t* off, const uint64_t* rec,
                                                          uint64_t* keys, uint32_t* vals) {
    const uint32_t r = blockIdx.x;
    const uint32_t c = reg_cnt[r], o = off[r];
    for (uint32_t j = threadIdx.x; j < c; j += kBlock) {
        keys[o + j] = rec[size_t(r) * kJV + j];
        vals[o + j] = o + j;
    }
}

// flag[i] = (i == 0 || key[i] != key[i-1]); rank[i] = (flags in 0..i) - 1.
__device__ __forceinline__ uint32_t pair_flag(const uint64_t* keys, uint32_t i) {
    return (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ __launch_bounds__(kBlock) void k_rank_reduce(const uint64_t* keys,
                                                        const uint32_t* count_ptr,
                                                        uint32_t* partial) {
    __shared__ uint32_t tmp[kWavesPerBlock];
    uint32_t lo, hi;
    worker_range(*count_ptr, blockIdx.x, gridDim.x, kTile, &lo, &hi);
    uint32_t s = 0;
    for (uint32_t tile = lo; tile < hi; tile += kTile) {
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t idx = tile + uint32_t(i) * kBlock + threadIdx.x;
            if (idx < hi) s += pair_flag(keys, idx);
        }
    }
    uint32_t tot;
    block_exclusive_scan(s, tmp, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// rank_of_slot[vals[i]] = rank[i].
__global__ __launch_bounds__(kBlock) void k_rank_apply(const uint64_t* keys, const uint32_t* vals,
                                                       const uint32_t* count_ptr,
                                                       const uint32_t* partial,
                                                       uint32_t* rank_of_slot) {
    __shared__ uint32_t tmp[kWavesPerBlock];
    uint32_t lo, hi;
    worker_range(*count_ptr, blockIdx.x, gridDim.x, kTile, &lo, &hi);
    uint32_t run = partial[blockIdx.x];
    for (uint32_t tile = lo; tile < hi; tile += kTile) {
        const uint32_t beg = tile + threadIdx.x * kItems;
        uint32_t f[kItems], s = 0;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            f[i] = beg + i < hi ? pair_flag(keys, beg + i) : 0u;
            s += f[i];
        }
        uint32_t tot;
        uint32_t r = run + block_exclusive_scan(s, tmp, &tot);
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            r += f[i];
            if (beg + i < hi) rank_of_slot[vals[beg + i]] = r - 1;
        }
        run += tot;
    }
}

// ms[v] = rank of its listed pair: rank_of[off[slot / kJV] + slot % kJV] with
// slot = ms[v] on entry.  Four vertices per thread.
__global__ __launch_bounds__(kBlock) void k_ms_final(int32_t* ms, uint32_t n, const uint32_t* off,
                                                     const uint32_t* rank_of) {
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t base = b * (kBlock * 4) + threadIdx.x;
    uint32_t s[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t v = base + uint32_t(i) * kBlock;
        s[i] = v < n ? uint32_t(ms[v]) : 0u;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t v = base + uint32_t(i) * kBlock;
        if (v < n) ms[v] = int32_t(rank_of[off[s[i] / kJV] + s[i] % kJV]);
    }
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
