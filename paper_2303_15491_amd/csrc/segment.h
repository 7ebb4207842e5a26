// Segmentation kernels: steepest neighbours with tile-local path compression,
// cross-tile chase, MS-pair listing, compaction and ranking.
#pragma once

#include <type_traits>

#include "common.h"
#include "sort.h"

namespace plmss {

// ---- vertex-order sources for the neighbour scan ---------------------------------

// The order of a float field under the paper's tie rule, compared through
// order-preserving integer keys (vertex ids break ties, see below).
// fetch() issues the load; key() turns the loaded value into the key, so
// that loads can stay in flight while other work runs.
template <typename T, typename K>
struct FieldOrder {
    using key_t = K;
    using raw_t = T;
    static constexpr bool kCheckNan = true;
    static constexpr bool kPackedCodes = false;
    const T* f;
    static __device__ __forceinline__ FieldOrder from(const void* p) { return {static_cast<const T*>(p)}; }
    __device__ __forceinline__ T fetch(size_t i) const { return gmem(f)[i]; }
    static __device__ __forceinline__ K key(T a, bool& nan) {
        nan |= is_nan(a);
        return sos_key(a);
    }
};

// A materialised order field (distinct ranks), as rank + 1 so that key 0 stays
// below every vertex (it marks grid positions outside the field).
struct RankOrder {
    using key_t = uint32_t;
    using raw_t = int32_t;
    static constexpr bool kCheckNan = false;
    static constexpr bool kPackedCodes = false;
    const int32_t* order;
    static __device__ __forceinline__ RankOrder from(const void* p) { return {static_cast<const int32_t*>(p)}; }
    __device__ __forceinline__ int32_t fetch(size_t i) const { return gmem(order)[i]; }
    static __device__ __forceinline__ uint32_t key(int32_t a, bool&) { return uint32_t(a) + 1u; }
};

// The same order field when every rank is below 2^28 - 1 (fields of fewer
// than 2^28 vertices): a key and a neighbour code then share one 32-bit word,
// (key << 4) | code, and the steepest candidate is a plain unsigned max (min)
// of such words.  No tie rule is needed: ranks are distinct, and the only
// candidate seen twice, the vertex itself, carries the same code both times.
struct RankOrderPacked : RankOrder {
    static constexpr bool kPackedCodes = true;
    static __device__ __forceinline__ RankOrderPacked from(const void* p) {
        return {{static_cast<const int32_t*>(p)}};
    }
};

struct GridDims {
    int32_t nx, ny, nz;
};

// One field of a launch.  Vertex v of the field is vertex vbase + v of the
// launch's concatenated numbering (pointers U/D, MS pair keys); its labels are
// written field-local.
struct FieldDesc {
    const void* src;   // values (FieldOrder) or order field (RankOrder)
    int32_t* asc;
    int32_t* desc;
    int32_t* ms;
    int32_t* info;     // {status, #minima, #maxima, K} or nullptr
    int32_t* order;    // order field out (batches), or nullptr
    int32_t nx, ny, nz;
    uint32_t vbase;    // first launch-wide vertex id
    uint32_t sbase;    // first steepest tile (within its shape class)
    uint32_t jbase;    // first chase tile (within its shape class)
    uint32_t index;    // position among all fields of the launch
    uint32_t flags;    // kWholeLines or 0
};

// The field's label arrays (asc, desc, ms) start on a 128-byte line and its
// rows are whole lines (nx a multiple of 32 vertices): then every row of a
// chase tile covers whole lines, and a launch over such a field alone takes
// the kernels' STREAM forms, whose label stores (chase) and record loads (MS
// write-back) bypass the caches (non-temporal: labels are written once,
// record indices read once).  Otherwise neighbouring tiles share lines, and
// non-temporal accesses would move each shared line as two partial
// transfers instead of letting the cache merge them.  (A compile-time
// choice: a run-time branch between the two forms of the same access is
// merged by the compiler into the plain one.)
constexpr uint32_t kWholeLines = 1u;

// The fields of a launch: a device table (batches) or a single descriptor
// passed by value.  Tile totals are host values, or device values for launches
// sized for a capacity (graph replays over varying batches).
struct Fields {
    const FieldDesc* table;
    uint32_t n;
    uint32_t s_tiles, j_tiles;
    uint32_t region0;           // chase tile t of this launch is pair-list region region0 + t
    const uint32_t* dev_tiles;  // nullptr, or {s_tiles, j_tiles, n, region0} on the device
    FieldDesc one;
};

// A descriptor read from a device table (member by member: the table lives
// in global memory, and a struct copy cannot bind across address spaces).
__device__ __forceinline__ FieldDesc load_desc(const FieldDesc* table, uint32_t f) {
    const auto* g = gmem(table) + f;
    FieldDesc d;
    d.src = g->src;
    d.asc = g->asc;
    d.desc = g->desc;
    d.ms = g->ms;
    d.info = g->info;
    d.order = g->order;
    d.nx = g->nx;
    d.ny = g->ny;
    d.nz = g->nz;
    d.vbase = g->vbase;
    d.sbase = g->sbase;
    d.jbase = g->jbase;
    d.index = g->index;
    d.flags = g->flags;
    return d;
}

// Descriptor of field f of the launch.
__device__ __forceinline__ FieldDesc field_desc(const Fields& F, uint32_t f) {
    return F.table ? load_desc(F.table, f) : F.one;
}

__device__ __forceinline__ uint32_t fields_region0(const Fields& F) {
    return F.dev_tiles ? gmem(F.dev_tiles)[3] : F.region0;
}

__device__ __forceinline__ uint32_t fields_count(const Fields& F) {
    return F.dev_tiles ? gmem(F.dev_tiles)[2] : (F.table ? F.n : 1u);
}

// Field owning launch-wide tile `tile` (by sbase when STEEP, else jbase).
template <bool STEEP>
__device__ __forceinline__ FieldDesc field_of_tile(const Fields& F, uint32_t tile, uint32_t* index) {
    if (!F.table) {
        *index = 0;
        return F.one;
    }
    uint32_t lo = 0, hi = fields_count(F);
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        const uint32_t b = STEEP ? gmem(F.table)[mid].sbase : gmem(F.table)[mid].jbase;
        if (b <= tile)
            lo = mid;
        else
            hi = mid;
    }
    *index = lo;
    return load_desc(F.table, lo);
}

// The field of each tile of a block's run of consecutive tiles: one binary
// search for the run's first tile, then a step to the next field each time a
// tile reaches that field's first tile (the descriptor is reloaded only
// then), instead of a search through the table in global memory per tile.
template <bool STEEP>
struct FieldCursor {
    const FieldDesc* table;
    uint32_t idx = 0, count = 0, next = 0;
    bool started = false;
    FieldDesc fd;
    __device__ explicit FieldCursor(const Fields& F) : table(F.table) {
        if (!table) fd = F.one;
    }
    __device__ __forceinline__ uint32_t base(uint32_t i) const {
        return STEEP ? gmem(table)[i].sbase : gmem(table)[i].jbase;
    }
    // Tiles must come in increasing order.
    __device__ __forceinline__ FieldDesc at(const Fields& F, uint32_t tile) {
        if (!table) return fd;
        if (!started) {
            fd = field_of_tile<STEEP>(F, tile, &idx);
            count = fields_count(F);
            next = idx + 1 < count ? base(idx + 1) : ~0u;
            started = true;
        } else if (tile >= next) {
            do {
                ++idx;
                next = idx + 1 < count ? base(idx + 1) : ~0u;
            } while (tile >= next);
            fd = load_desc(table, idx);
        }
        return fd;
    }
};

// This block's tiles: a contiguous run, so that each XCD works on a compact
// part of the grid.
__device__ __forceinline__ void block_tiles(uint32_t total, uint32_t* first, uint32_t* last) {
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t per = (total + gridDim.x - 1) / gridDim.x;
    *first = min(total, b * per);
    *last = min(total, *first + per);
}

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
constexpr uint32_t kExit = 0x8000u;         // local pointer: the target lies outside the tile
constexpr int kResolveRounds = 3;           // in-tile jumping sweeps (default)

// In-tile move of neighbour code c in a kTX x ty x zc tile: bits 0-15 the
// change of the local index (two's complement), bits 16-21 the tile sides the
// move crosses when taken from a vertex on that side (x-, x+, y-, y+, z-, z+).
__host__ __device__ constexpr uint32_t local_move(int c, int ty) {
    const int d = c - 7, m = d < 0 ? -d : d;
    const int dx = m & 1, dy = (m >> 1) & 1, dz = (m >> 2) & 1;
    const int delta = dx + dy * kTX + dz * kTX * ty;
    const uint32_t side = d < 0 ? uint32_t(dx | (dy << 2) | (dz << 4)) : uint32_t((dx << 1) | (dy << 3) | (dz << 5));
    return (side << 16) | (uint32_t(d < 0 ? -delta : delta) & 0xffffu);
}

// Steepest neighbours of every vertex.
//
// A block owns a kTX x TY column of the grid over ZC consecutive planes and
// marches through them, so the field is read from HBM about once.  Positions
// outside the grid hold key 0, below every vertex.
//
// Search (32-bit keys): the candidate set of v -- its 14 neighbours and v --
// is the union of four 2x2 squares: at (x-1, y-1) in planes z-1 and z, and at
// (x, y) in planes z and z+1, listed here in increasing vertex-id order
// (within a square: (0,0) (1,0) (0,1) (1,1)).  Each square's maximum and
// minimum is found once per plane and shared by the four vertices that use
// it; a vertex combines four squares.  ">=" for the maximum and "<" for the
// minimum, in id order, break equal keys by vertex id as the paper's order
// does.  64-bit keys (float64 fields) use the plain 15-candidate scan.
//
// RESOLVE == false: up[v] / dn[v] = the steepest ascending / descending
//   neighbour (v itself at a maximum / minimum).
// RESOLVE == true: the paper's path compression is run inside the tile first.
//   Every vertex keeps, in LDS, a pointer to its steepest neighbour if that
//   lies in the tile, or an exit mark with the direction if it does not; the
//   pointers are then compressed in place, p <- p[p], round by round, until
//   each points at the end of its tile chain.  The result written is
//     up[v] = kMark | maximum           if v's ascending chain ends in the tile,
//     up[v] = first vertex outside      otherwise (a pointer still to follow);
//   likewise dn[v].
// info[1] += #minima, info[2] += #maxima; info[0] = PLMSS_E_NAN on a NaN.
template <typename K, int TY>
struct SquarePlanes {
    K mx[3][TY + 1][kTX + 1];  // square maxima
    K mn[3][TY + 1][kTX + 1];  // square minima of (key - 1): key 0 becomes the largest
    uint8_t tag[3][TY + 1][kTX + 1];  // winner positions: max in bits 0-1, min in bits 2-3
};

// NT threads per block (eight waves: one row of the tile per wave and plane
// in 3-D, so that each thread holds half the state of a 256-thread block and
// twice the waves fit beside the LDS the tile needs).
template <class Src, int TY, int ZC, bool RESOLVE, int NT>
__global__ __launch_bounds__(NT, NT >= 512 && ZC <= 16 ? 6 : 1) void k_steepest(Fields F, uint32_t* up, uint32_t* dn, int rounds) {
    using K = typename Src::key_t;
    constexpr bool kSquares = sizeof(K) == 4;
    constexpr bool kPacked = kSquares && Src::kPackedCodes;
    constexpr int PX = kTX + 2, PY = TY + 2, RPW = TY / (NT / kWave);
    constexpr int TV = RESOLVE ? kTX * TY * ZC : 1;
    constexpr int kLoads = (PY * PX + NT - 1) / NT;
    constexpr int kSq = (TY + 1) * (kTX + 1);
    constexpr int kSqLoops = (kSq + NT - 1) / NT;
    static_assert(TY % (NT / kWave) == 0, "rows per wave");
    static_assert((TY & (TY - 1)) == 0, "power-of-two rows");
    static_assert(kTX * TY * ZC < int(kExit), "local indices need 15 bits");
    // raw key planes: the ring of three for the plain scan, one staging plane
    // for the square search
    __shared__ K pl[kSquares ? 1 : 3][PY][PX];
    __shared__ SquarePlanes<K, kSquares ? TY : 0> sq;
    __shared__ uint32_t lp[TV];  // local pointers: up in the low half, dn in the high half
    __shared__ int32_t off_tab[16];  // vertex-id offset of each neighbour code
    __shared__ uint32_t loc_tab[16];  // in-tile move of each neighbour code
    __shared__ uint32_t row_off[RESOLVE ? ZC * TY : 1];  // vertex-id offset of each tile row from the tile's first
    __shared__ uint32_t cnt_min, cnt_max;
    __shared__ int nan_seen;
    const int t = threadIdx.x, w = wave_id(), lane = lane_id();
    if (t < 16) loc_tab[t] = t < 15 ? local_move(t, TY) : 0u;
    // the x sides of this thread's column (the y and z sides are uniform)
    const uint32_t xside = (lane == 0 ? 1u : 0u) | (lane == kTX - 1 ? 2u : 0u);
    uint32_t tfirst, tlast;
    block_tiles(F.dev_tiles ? gmem(F.dev_tiles)[0] : F.s_tiles, &tfirst, &tlast);
    FieldCursor<true> cursor(F);
    for (uint32_t tile = tfirst; tile < tlast; ++tile) {
    const FieldDesc fd = cursor.at(F, tile);
    const Src src = Src::from(fd.src);
    const GridDims g{fd.nx, fd.ny, fd.nz};
    int32_t* const info = fd.info;
    const uint32_t vbase = fd.vbase;
    const uint32_t b = tile - fd.sbase;
    const int tx = (g.nx + kTX - 1) / kTX, ty = (g.ny + TY - 1) / TY;
    const int bx = int(b % uint32_t(tx));
    const int by = int((b / uint32_t(tx)) % uint32_t(ty));
    const int bz = int(b / (uint32_t(tx) * uint32_t(ty)));
    const int x0 = bx * kTX, y0 = by * TY, z0 = bz * ZC;
    const int z1 = min(g.nz, z0 + ZC);
    const size_t sx = size_t(g.nx), sxy = size_t(g.nx) * size_t(g.ny);
    const int32_t S = int32_t(sxy);
    __syncthreads();  // the previous tile's readers of LDS are done
    if (t == 0) {
        cnt_min = 0;
        cnt_max = 0;
        nan_seen = 0;
    }
    if (t < 16) off_tab[t] = t < 15 ? code_offset(t, g.nx, S) : 0;
    // this thread's share of a plane load: LDS slot and in-plane offset, the
    // same for every plane
    // Slots outside the grid read the plane's first vertex and store a zero
    // key instead, so a plane's loads need no branch and issue together.
    int ld_slot[kLoads];
    bool ld_in[kLoads];
    uint32_t ld_off[kLoads];
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
        const int i = t + k * NT;
        const int r = i / PX, c = i - r * PX;
        const int gx = x0 - 1 + c, gy = y0 - 1 + r;
        ld_in[k] = i < PY * PX && gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny;
        ld_slot[k] = i < PY * PX ? i : -1;
        ld_off[k] = ld_in[k] ? uint32_t(gy) * uint32_t(sx) + uint32_t(gx) : 0u;
    }
    bool nan = false;
    // plane loads go through registers as raw values, so that the next
    // plane's loads are in flight while the current plane is computed; the
    // key transform waits until the plane is stored
    using R = typename Src::raw_t;
    R pre[kLoads];
    auto fetch_plane = [&](int z) {
        const size_t zb = size_t(z) * sxy;
#pragma unroll
        for (int k = 0; k < kLoads; ++k) pre[k] = src.fetch(zb + size_t(ld_off[k]));
    };
    auto store_plane = [&](int slot) {
        K* dst = &pl[kSquares ? 0 : slot][0][0];
#pragma unroll
        for (int k = 0; k < kLoads; ++k)
            if (ld_slot[k] >= 0) dst[ld_slot[k]] = ld_in[k] ? Src::key(pre[k], nan) : K(0);
    };
    auto load_plane = [&](int slot, int z) {
        fetch_plane(z);
        store_plane(slot);
    };
    // square results of one plane (z valid) or of a missing plane
    auto squares = [&](int slot, bool exists) {
        if constexpr (kSquares) {
#pragma unroll
            for (int k = 0; k < kSqLoops; ++k) {
                const int i = t + k * NT;
                if (i >= kSq) break;
                const int r = i / (kTX + 1), c = i - r * (kTX + 1);
                K hi = K(0), lo = ~K(0);
                uint32_t th = 0, tl = 0;
                if (exists) {
                    const K a[4] = {pl[0][r][c], pl[0][r][c + 1], pl[0][r + 1][c], pl[0][r + 1][c + 1]};
                    if constexpr (kPacked) {
                        // (key << 4) | position; the minimum of (key - 1): a
                        // position outside the grid (key 0) becomes the largest
                        hi = max(max((a[0] << 4) | 0u, (a[1] << 4) | 1u), max((a[2] << 4) | 2u, (a[3] << 4) | 3u));
                        lo = min(min(((a[0] - 1u) << 4) | 0u, ((a[1] - 1u) << 4) | 1u),
                                 min(((a[2] - 1u) << 4) | 2u, ((a[3] - 1u) << 4) | 3u));
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const bool gh = a[q] >= hi;
                            hi = gh ? a[q] : hi;
                            th = gh ? uint32_t(q) : th;
                            const K am = a[q] - K(1);
                            const bool gl = am < lo;
                            lo = gl ? am : lo;
                            tl = gl ? uint32_t(q) : tl;
                        }
                    }
                } else if constexpr (kPacked) {
                    lo = ~K(15);  // low bits clear: adding a code base cannot wrap
                }
                sq.mx[slot][r][c] = hi;
                sq.mn[slot][r][c] = lo;
                if constexpr (!kPacked) sq.tag[slot][r][c] = uint8_t(th | (tl << 2));
            }
        }
    };
    int pm = 0, pc = 1, pn = 2;
    if (z0 > 0) {
        load_plane(pm, z0 - 1);
        if (kSquares) {
            __syncthreads();
            squares(pm, true);
        }
    } else if (kSquares) {
        squares(pm, false);
    }
    if (kSquares) __syncthreads();
    load_plane(pc, z0);
    if (kSquares) {
        __syncthreads();
        squares(pc, true);
    }
    if (z0 + 1 < g.nz) fetch_plane(z0 + 1);
    const int x = x0 + lane;
    const bool xm = x > 0, xp = x < g.nx - 1;
    uint32_t my_min = 0, my_max = 0;
    for (int z = z0; z < z1; ++z) {
        // The plain scan's ring slot pn was read as pm by the previous plane:
        // wait for its readers.  The square search needs no barrier here
        // after its first plane: the staging plane was last read before the
        // previous plane's last barrier, and the square slot it rewrites
        // below (pn, the previous plane's pm) is written only after the
        // next barrier, which every wave reaches after that plane's
        // best-of-squares.  Its first plane waits for the prologue's square
        // search to release the staging plane.
        if (!kSquares || z == z0) __syncthreads();
        if (z + 1 < g.nz) store_plane(pn);  // plane z + 1, fetched one step ahead
        if (kSquares) {
            __syncthreads();
            squares(pn, z + 1 < g.nz);
        }
        __syncthreads();
        if (z + 2 < g.nz && z + 1 < z1) fetch_plane(z + 2);
        const bool zm = z > 0, zp = z < g.nz - 1;
        const bool interior = x0 > 0 && x0 + kTX < g.nx && y0 > 0 && y0 + TY < g.ny && zm && zp;
        const int lz = z - z0;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int ly = w * RPW + r, y = y0 + ly;
            const bool inside = x < g.nx && y < g.ny;
            int cu, cd;
            if constexpr (kSquares) {
                // squares k = 0..3 in id order; code = base_k + winner position
                const int sl[4] = {pm, pc, pc, pn};
                const int rr[4] = {ly, ly, ly + 1, ly + 1};
                const int cc[4] = {lane, lane, lane + 1, lane + 1};
                const int base[4] = {0, 4, 7, 11};
                K bu = K(0), bd = ~K(0);
                cu = kSelf;
                cd = kSelf;
                if constexpr (kPacked) {
                    // the code is the square's base plus the winner's
                    // position, kept in the low four bits (at most 14)
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        bu = max(bu, sq.mx[sl[k]][rr[k]][cc[k]] + K(base[k]));
                        bd = min(bd, sq.mn[sl[k]][rr[k]][cc[k]] + K(base[k]));
                    }
                    cu = int(bu & 15u);
                    cd = int(bd & 15u);
                } else {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const K h = sq.mx[sl[k]][rr[k]][cc[k]];
                        const K l = sq.mn[sl[k]][rr[k]][cc[k]];
                        const uint32_t tg = sq.tag[sl[k]][rr[k]][cc[k]];
                        const bool gu = h >= bu, gd = l < bd;
                        bu = gu ? h : bu;
                        cu = gu ? base[k] + int(tg & 3u) : cu;
                        bd = gd ? l : bd;
                        cd = gd ? base[k] + int(tg >> 2) : cd;
                    }
                }
            } else {
                const bool ym = y > 0, yp = y < g.ny - 1;
                if (interior)
                    steepest_codes<Src, PY, false>(pl, pm, pc, pn, lane, ly, xm, xp, ym, yp, zm, zp, cu, cd);
                else
                    steepest_codes<Src, PY, true>(pl, pm, pc, pn, lane, ly, xm, xp, ym, yp, zm, zp, cu, cd);
            }
            if (inside) {
                my_max += (cu == kSelf);
                my_min += (cd == kSelf);
            }
            if (!RESOLVE) {
                if (inside) {
                    const uint32_t v = vbase + uint32_t(z) * uint32_t(S) + uint32_t(y) * uint32_t(g.nx) + uint32_t(x);
                    up[v] = uint32_t(int32_t(v) + code_offset(cu, g.nx, S));
                    dn[v] = uint32_t(int32_t(v) + code_offset(cd, g.nx, S));
                }
            } else {
                const int li = (lz * TY + ly) * kTX + lane;
                // the tile sides this vertex lies on; a move across one of
                // them leaves the tile and is kept as an exit mark with its code
                const uint32_t side = xside | (ly == 0 ? 4u : 0u) | (ly == TY - 1 ? 8u : 0u) |
                                      (lz == 0 ? 16u : 0u) | (lz == ZC - 1 ? 32u : 0u);
                auto local = [&](int c) -> uint32_t {
                    const uint32_t mv = loc_tab[c];
                    return ((mv >> 16) & side) ? (kExit | uint32_t(c))
                                               : uint32_t(li + int32_t(int16_t(uint16_t(mv & 0xffffu))));
                };
                // padding (outside the grid) is a harmless root
                lp[li] = inside ? (local(cu) | (local(cd) << 16)) : (uint32_t(li) | (uint32_t(li) << 16));
            }
        }
        const int tmp = pm;
        pm = pc;
        pc = pn;
        pn = tmp;
    }
    if (RESOLVE) {
        // the write-out turns local indices into vertex ids through this
        // table (row = plane * TY + row in plane) instead of two 32-bit
        // multiplies per pointer
        for (int i = t; i < ZC * TY; i += NT)
            row_off[RESOLVE ? i : 0] = uint32_t(i / TY) * uint32_t(S) + uint32_t(i % TY) * uint32_t(g.nx);
        __syncthreads();
        // entries of this thread: (lz, row) pairs over the tile's planes; entry
        // e has local index li0 + (e / RPW) * TY * kTX + (e % RPW) * kTX
        constexpr int kMine = ZC * RPW;
        const int nz_t = z1 - z0;
        const int li0 = (w * RPW) * kTX + lane;
        // in-place rounds of p <- p[p] on both halves of an entry at once.  A
        // half stays when it or its target is an exit mark, or when its target
        // is a root (points to itself); otherwise it takes the target's
        // pointer.  Planes past the field's last plane hold nothing of this
        // tile and are skipped; every pointer written above stays in the
        // planes that were written.
        // Entries are taken kGroup at a time: the group's own pointers are
        // read, then their targets, then the changed entries are written, so
        // that the LDS reads of a group are in flight together instead of each
        // waiting for the write before it.  Inside a group a target may be
        // read before its own update; any pointer on the path is a valid
        // value, so this only changes how much each sweep compresses.
        constexpr int kGroup = kMine < 4 ? kMine : 4;
        static_assert(kMine % kGroup == 0, "whole groups");
        auto group = [&](int g0, bool rev, bool& ch) {
            if (g0 / RPW >= nz_t) return;
            int li[kGroup];
            bool act[kGroup];
            uint32_t own[kGroup], q[kGroup];
#pragma unroll
            for (int k = 0; k < kGroup; ++k) {
                const int e = rev ? g0 + (kGroup - 1 - k) : g0 + k;
                act[k] = e / RPW < nz_t;
                li[k] = li0 + (e / RPW) * (TY * kTX) + (e % RPW) * kTX;
                own[k] = lp[li[k]];
            }
#pragma unroll
            for (int k = 0; k < kGroup; ++k) {
                // an entry in a plane past the field reads itself (in bounds)
                // and is not written
                own[k] = act[k] ? own[k] : (uint32_t(li[k]) | (uint32_t(li[k]) << 16));
                const uint32_t qu = lp[own[k] & (kExit - 1)], qd = lp[(own[k] >> 16) & (kExit - 1)];
                q[k] = (qu & 0xffffu) | (qd & 0xffff0000u);
            }
#pragma unroll
            for (int k = 0; k < kGroup; ++k) {
                // a half keeps its pointer when it or its target's pointer is
                // an exit mark, else it takes the target's pointer (for a root
                // target that is its own value again).  The exit bits (15 and
                // 31) become the half masks by one 24-bit multiply.
                const uint32_t cross = own[k] | q[k];
                const uint32_t keep = ((cross >> 15) & 0x10001u) * 0xffffu;
                const uint32_t nw = (own[k] & keep) | (q[k] & ~keep);
                if (act[k] && nw != own[k]) {
                    lp[li[k]] = nw;  // each entry has one owner
                    ch = true;
                }
            }
        };
        // sweeps alternate direction, so chains of either orientation compress
        // in one sweep when their entries happen to lie in sweep order.  A few
        // sweeps finish almost every tile chain; what is left is written as an
        // unfinished pointer, which the chase kernel follows.
        for (int round = 0; round < rounds; ++round) {
            bool ch = false;
            if (round & 1) {
#pragma unroll
                for (int g = kMine - kGroup; g >= 0; g -= kGroup) group(g, true, ch);
            } else {
#pragma unroll
                for (int g = 0; g < kMine; g += kGroup) group(g, false, ch);
            }
            if (!__syncthreads_or(ch)) break;
        }
        // write-out: the end of the tile chain, resolved or to be followed.
        // Vertex ids fit in 32 bits.
        const uint32_t tile0 =
            vbase + uint32_t(z0) * uint32_t(S) + uint32_t(y0) * uint32_t(g.nx) + uint32_t(x0);
        auto gid = [&](uint32_t li) -> uint32_t {
            return tile0 + row_off[RESOLVE ? li / kTX : 0] + (li & (kTX - 1));
        };
        // p: the vertex's pointer; q: the pointer of p's vertex; v: the vertex
        auto resolve = [&](uint32_t v, uint32_t p, uint32_t q) -> uint32_t {
            const bool own_exit = p & kExit;
            const uint32_t base = own_exit ? v : gid(p);
            const uint32_t code = (own_exit ? p : q) & 0xffu;
            const uint32_t ext = base + uint32_t(off_tab[code & 15u]);
            if (own_exit || (q & kExit)) return ext;  // leaves the tile
            return q == p ? (kMark | base) : base;     // an extremum, or still to follow
        };
        for (int lz = 0; lz < nz_t; ++lz) {
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const int ly = w * RPW + r, y = y0 + ly;
                if (x >= g.nx || y >= g.ny) continue;
                const uint32_t li = uint32_t((lz * TY + ly) * kTX + lane);
                const uint32_t v = tile0 + row_off[RESOLVE ? lz * TY + ly : 0] + uint32_t(lane);
                const uint32_t own = lp[li];
                const uint32_t pu = own & 0xffffu, pd = own >> 16;
                const uint32_t qu = lp[pu & (kExit - 1)] & 0xffffu, qd = lp[pd & (kExit - 1)] >> 16;
                // whole rows of a tile, written once: streamed past the
                // caches (non-temporal), which the field's loads then keep
                __builtin_nontemporal_store(resolve(v, pu, qu), up + v);
                __builtin_nontemporal_store(resolve(v, pd, qd), dn + v);
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
    }  // tiles
}

constexpr int kSteepBlock = 512;  // threads per neighbour-scan block

inline uint32_t steepest_tiles(int64_t nx, int64_t ny, int64_t nz, int ty, int zc) {
    return uint32_t(((nx + kTX - 1) / kTX) * ((ny + ty - 1) / ty) * ((nz + zc - 1) / zc));
}

// ---- chase, labels and MS pair listing ----------------------------------------------
//
// One block per JX x JY x JZ tile (kJV = 2048 vertices, 4 per thread of 512).  For
// every vertex it finishes the tile-compressed pointers: an unresolved pointer
// is followed from tile to tile (each hop lands on the next tile's compressed
// pointer, and is written back so that later readers jump further) until a
// marked extremum.  It writes desc/asc, then lists the tile's distinct
// (asc, desc) pairs through an LDS hash set: the tile takes a run of
// consecutive record indices from a launch-wide counter (one atomic add per
// tile), writes each pair key (asc << bn) | desc to rec_keys at its record
// index (the pair sort generates the indices as the keys' values), and stores
// each vertex's record index in ms[v] (replaced by the MS id later).  MS regions are a few vertices across, so a 3-D tile
// lists far fewer pairs than a row of the same size would.
constexpr int kJV = 2048;            // vertices per tile
constexpr int kJPer = kJV / kBlock;  // per thread (256-thread blocks)
// The chase runs 512-thread blocks, four vertices per thread: its pointer
// hops are dependent gathers, and the smaller per-thread state lets twice as
// many waves hide their latency.
constexpr int kChaseBlock = 512;
constexpr int kChaseWaves = kChaseBlock / kWave;
constexpr int kChasePer = kJV / kChaseBlock;
constexpr int kHash = kJV;           // hash slots: a tile has at most kJV distinct pairs
constexpr uint64_t kEmpty = ~0ull;   // pair keys are < 2^62

template <int JX, int JY, int JZ>
struct JTile {
    static_assert(JX * JY * JZ == kJV, "tile size");
    static constexpr int X = JX, Y = JY, Z = JZ;
    // a thread's vertices are kChaseBlock entries apart in the tile: the
    // step between them in x, y, z (the same for every thread)
    static constexpr int SX = kChaseBlock % JX;
    static constexpr int SY = (kChaseBlock / JX) % JY;
    static constexpr int SZ = kChaseBlock / (JX * JY);
    static_assert(SX * 1 + SY * JX + SZ * JX * JY == kChaseBlock && (SX == 0 || JX % kChaseBlock == 0) &&
                      (SY == 0 || (JY % SY == 0 && JX * SY == kChaseBlock)),
                  "a thread's vertices differ in one coordinate");
};
using JTile3 = JTile<32, 8, 8>;
using JTile2 = JTile<64, 32, 1>;
using JTile1 = JTile<2048, 1, 1>;

template <class T>
inline uint32_t chase_tiles(int64_t nx, int64_t ny, int64_t nz) {
    return uint32_t(((nx + T::X - 1) / T::X) * ((ny + T::Y - 1) / T::Y) * ((nz + T::Z - 1) / T::Z));
}

__device__ __forceinline__ uint32_t pair_hash(uint64_t k) {
    const uint32_t lo = uint32_t(k), hi = uint32_t(k >> 32);
    return (lo * 0x9E3779B1u) ^ (hi * 0x85EBCA77u) ^ (lo >> 15);
}

// Local coordinates of entry li of a chase tile.
template <class T>
__device__ __forceinline__ void jtile_xyz(const FieldDesc& fd, uint32_t lt, int li, int* x, int* y,
                                          int* z) {
    const int tx = (fd.nx + T::X - 1) / T::X, ty = (fd.ny + T::Y - 1) / T::Y;
    const int x0 = int(lt % uint32_t(tx)) * T::X;
    const int y0 = int((lt / uint32_t(tx)) % uint32_t(ty)) * T::Y;
    const int z0 = int(lt / (uint32_t(tx) * uint32_t(ty))) * T::Z;
    *x = x0 + li % T::X;
    *y = y0 + (li / T::X) % T::Y;
    *z = z0 + li / (T::X * T::Y);
}

// CHASE: labels from the tile-compressed pointers U/D (written back as they
// are followed).  Otherwise the labels are read from the field's desc/asc.
// O32: every vertex id of the launch is below 2^30, so U, D and the label
// arrays are addressed by 32-bit byte offsets.  STREAM: see kWholeLines.
template <class T, bool CHASE, bool O32, bool STREAM = false>
__global__ __launch_bounds__(kChaseBlock, 8) void k_chase(Fields F, uint32_t* U, uint32_t* D, int bn,
                                                  uint64_t* rec_keys, uint32_t* rec_count) {
    __shared__ uint64_t table[kHash];
    __shared__ uint16_t dense[kHash];
    __shared__ uint32_t tmp[kChaseWaves];
    __shared__ uint32_t s_base;
    uint32_t tfirst, tlast;
    block_tiles(F.dev_tiles ? gmem(F.dev_tiles)[1] : F.j_tiles, &tfirst, &tlast);
    FieldCursor<false> cursor(F);
    for (uint32_t tile = tfirst; tile < tlast; ++tile) {
        // the thread index is made opaque to the compiler once per tile, so
        // that what derives from it (lane masks, in-tile coordinates) is
        // recomputed in each tile rather than held in registers across tiles
        // (with it, the kernel fits 64 registers: eight waves per SIMD)
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int t = int(tid), lane = t & (kWave - 1), w = t / kWave;
        const FieldDesc fd = cursor.at(F, tile);
        const uint32_t lt = tile - fd.jbase;
        __syncthreads();  // the previous tile's readers of LDS are done
#pragma unroll
        for (int i = 0; i < kHash / kChaseBlock; ++i) table[t + i * kChaseBlock] = kEmpty;
        uint32_t lv[kChasePer], pu[kChasePer], pd[kChasePer];
        bool ok[kChasePer];
        // the thread's vertices: the first one's coordinates, then a fixed
        // step (in one coordinate) to each of the others
        int x0, y0, z0;
        jtile_xyz<T>(fd, lt, t, &x0, &y0, &z0);
        const uint32_t v0 = (uint32_t(z0) * uint32_t(fd.ny) + uint32_t(y0)) * uint32_t(fd.nx) + uint32_t(x0);
        const uint32_t vstep = uint32_t(T::SX) + uint32_t(T::SY) * uint32_t(fd.nx) +
                               uint32_t(T::SZ) * uint32_t(fd.nx) * uint32_t(fd.ny);
#pragma unroll
        for (int i = 0; i < kChasePer; ++i) {
            ok[i] = x0 + i * T::SX < fd.nx && y0 + i * T::SY < fd.ny && z0 + i * T::SZ < fd.nz;
            lv[i] = ok[i] ? v0 + uint32_t(i) * vstep : 0u;
            // lanes past the field's edge read its vertex 0 (lv = 0) and drop
            // the value, so the loads need no branch and issue together
            if (CHASE) {
                pu[i] = *gelem<O32>(U, fd.vbase + lv[i]);
                pd[i] = *gelem<O32>(D, fd.vbase + lv[i]);
            } else {
                pu[i] = uint32_t(*gelem<O32>(fd.desc, lv[i])) + fd.vbase;
                pd[i] = uint32_t(*gelem<O32>(fd.asc, lv[i])) + fd.vbase;
            }
        }
#pragma unroll
        for (int i = 0; i < kChasePer; ++i) {
            pu[i] = ok[i] ? pu[i] : (CHASE ? kMark : 0u);
            pd[i] = ok[i] ? pd[i] : (CHASE ? kMark : 0u);
        }
        if (CHASE) {
            // the four vertices of a thread advance together, so their
            // gathers are in flight at the same time; from the second hop on,
            // a pointer is written back so that later readers jump further
            bool pending = true;
            uint32_t hops = 0;
            while (pending && hops < kMaxHops) {
                // all gathers of the hop first, then the write-backs, so that
                // no store waits on its own load before the next is issued
                uint32_t nu[kChasePer], nd[kChasePer];
#pragma unroll
                for (int i = 0; i < kChasePer; ++i) {
                    nu[i] = pu[i];
                    nd[i] = pd[i];
                    if (!(pu[i] & kMark)) nu[i] = *gelem<O32>(U, pu[i]);
                    if (!(pd[i] & kMark)) nd[i] = *gelem<O32>(D, pd[i]);
                }
                pending = false;
#pragma unroll
                for (int i = 0; i < kChasePer; ++i) {
                    if (!(pu[i] & kMark)) {
                        if (hops) *gelem<O32>(U, fd.vbase + lv[i]) = nu[i];
                        pending = true;
                    }
                    if (!(pd[i] & kMark)) {
                        if (hops) *gelem<O32>(D, fd.vbase + lv[i]) = nd[i];
                        pending = true;
                    }
                    pu[i] = nu[i];
                    pd[i] = nd[i];
                }
                ++hops;
            }
#pragma unroll
            for (int i = 0; i < kChasePer; ++i) {
                pu[i] &= ~kMark;
                pd[i] &= ~kMark;
                if (ok[i]) {
                    const int32_t dv = int32_t(pu[i] - fd.vbase), av = int32_t(pd[i] - fd.vbase);
                    if constexpr (STREAM) {
                        __builtin_nontemporal_store(dv, gelem<O32>(fd.desc, lv[i]));
                        __builtin_nontemporal_store(av, gelem<O32>(fd.asc, lv[i]));
                    } else {
                        *gelem<O32>(fd.desc, lv[i]) = dv;
                        *gelem<O32>(fd.asc, lv[i]) = av;
                    }
                }
            }
            if (pending && fd.info) gmem(fd.info)[0] = -7;  // PLMSS_E_NOCONV
        }
        __syncthreads();
        // insert every vertex's pair; slot[i] = its hash slot.  Neighbouring
        // lanes mostly hold the same pair (MS regions span several vertices
        // of a row): only the first lane of each run of equal pairs inserts,
        // the others take its slot by a shuffle.
        const uint64_t upto_me = ~0ull >> (kWave - 1 - lane);
        uint32_t slot[kChasePer];
#pragma unroll
        for (int i = 0; i < kChasePer; ++i) {
            const uint64_t key = ok[i] ? (uint64_t(pd[i]) << bn) | uint64_t(pu[i]) : kEmpty;
            const uint32_t klo = uint32_t(key), khi = uint32_t(key >> 32);
            const uint32_t llo = uint32_t(__shfl_up(int(klo), 1)), lhi = uint32_t(__shfl_up(int(khi), 1));
            const bool first = lane == 0 || klo != llo || khi != lhi;
            uint32_t h = 0;
            if (ok[i] && first) {
                h = pair_hash(key) & (kHash - 1);
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
            }
            // the run's first lane: the highest lane at or below this one
            // that starts a run (its pair is this lane's)
            const uint64_t starts = __ballot(first);
            slot[i] = uint32_t(__shfl(int(h), top_lane(starts & upto_me)));
        }
        __syncthreads();
        // number the occupied slots: wave w scans slots [w*kHash/8, (w+1)*kHash/8)
        // row by row (64 consecutive slots per row), so LDS reads are conflict-free
        constexpr int kRows = kHash / kChaseBlock;
        uint32_t wcount = 0;
#pragma unroll
        for (int i = 0; i < kRows; ++i)
            wcount += uint32_t(__popcll(__ballot(table[w * (kHash / kChaseWaves) + i * kWave + lane] != kEmpty)));
        if (lane == 0) tmp[w] = wcount;
        __syncthreads();
        uint32_t j = 0, total = 0;
#pragma unroll
        for (int i = 0; i < kChaseWaves; ++i) {
            j += (i < w) ? tmp[i] : 0u;
            total += tmp[i];
        }
        if (t == 0) s_base = atomicAdd(rec_count, total);
        __syncthreads();
        const uint32_t base = s_base;
#pragma unroll
        for (int i = 0; i < kRows; ++i) {
            const int sl = w * (kHash / kChaseWaves) + i * kWave + lane;
            const uint64_t k = table[sl];
            const uint64_t occ = __ballot(k != kEmpty);
            if (k != kEmpty) {
                // occupied slots below this lane
                const uint32_t jj =
                    j + __builtin_amdgcn_mbcnt_hi(uint32_t(occ >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(occ), 0u));
                dense[sl] = uint16_t(jj);
                rec_keys[base + jj] = k;
            }
            j += uint32_t(__popcll(occ));
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kChasePer; ++i)
            if (ok[i]) *gelem<O32>(fd.ms, lv[i]) = int32_t(base + dense[slot[i]]);
    }
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

// ---- pair ranking ---------------------------------------------------------------------

// flag[i] = (i == 0 || key[i] != key[i-1]); rank[i] = (flags in 0..i) - 1.
// Both kernels read from indices clamped into the slice, so every load of a
// tile is issued before the first is waited for; items past the slice are
// masked afterwards.
__global__ __launch_bounds__(kBlock) void k_rank_reduce(const uint64_t* keys,
                                                        const uint32_t* count_ptr,
                                                        uint32_t* partial) {
    __shared__ uint32_t tmp[kWavesPerBlock];
    uint32_t lo, hi;
    worker_range(*count_ptr, blockIdx.x, gridDim.x, kTile, &lo, &hi);
    uint32_t s = 0;
    for (uint32_t tile = lo; tile < hi; tile += kTile) {
        uint64_t k[kItems], p[kItems];
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t idx = min(tile + uint32_t(i) * kBlock + threadIdx.x, hi - 1u);
            k[i] = keys[idx];
            p[i] = keys[idx ? idx - 1u : 0u];
        }
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t idx = tile + uint32_t(i) * kBlock + threadIdx.x;
            if (idx < hi) s += (idx == 0 || k[i] != p[i]) ? 1u : 0u;
        }
    }
    uint32_t tot;
    block_exclusive_scan(s, tmp, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// rank_of_slot[vals[i]] = rank[i].  A tile's keys are loaded coalesced into
// LDS (one padding entry per 16, so that a thread's 16 consecutive entries
// fall in different banks); each thread then scans its kItems consecutive
// keys, puts the ranks back into LDS, and the ranks are stored by their
// values in coalesced item order.
__global__ __launch_bounds__(kBlock) void k_rank_apply(const uint64_t* keys, const uint32_t* vals,
                                                       const uint32_t* count_ptr,
                                                       const uint32_t* partial,
                                                       uint32_t* rank_of_slot) {
    constexpr int kPad = kTile + kTile / 16;
    __shared__ uint64_t sk[kPad];
    __shared__ uint32_t sr[kPad];
    __shared__ uint32_t tmp[kWavesPerBlock];
    auto pad = [](uint32_t i) { return i + (i >> 4); };
    const uint32_t t = threadIdx.x;
    uint32_t lo, hi;
    worker_range(*count_ptr, blockIdx.x, gridDim.x, kTile, &lo, &hi);
    uint32_t run = partial[blockIdx.x];
    for (uint32_t tile = lo; tile < hi; tile += kTile) {
        const uint32_t tsize = min(uint32_t(kTile), hi - tile);
        uint64_t k[kItems];
        uint32_t v[kItems];
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t idx = min(tile + uint32_t(i) * kBlock + t, hi - 1u);
            k[i] = keys[idx];
            v[i] = vals[idx];
        }
        const uint64_t before = keys[tile ? tile - 1u : 0u];
        __syncthreads();  // the previous tile's readers of sk and sr are done
#pragma unroll
        for (int i = 0; i < kItems; ++i) sk[pad(uint32_t(i) * kBlock + t)] = k[i];
        __syncthreads();
        const uint32_t beg = t * kItems;
        uint32_t f[kItems], s = 0;
        uint64_t prev = beg ? sk[pad(beg - 1u)] : before;
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint64_t cur = sk[pad(beg + uint32_t(i))];
            f[i] = (beg + i < tsize && (tile + beg + i == 0 || cur != prev)) ? 1u : 0u;
            s += f[i];
            prev = cur;
        }
        uint32_t tot;
        uint32_t r = run + block_exclusive_scan(s, tmp, &tot);
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            r += f[i];
            sr[pad(beg + uint32_t(i))] = r - 1u;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const uint32_t j = uint32_t(i) * kBlock + t;
            if (j < tsize) rank_of_slot[v[i]] = sr[pad(j)];
        }
        run += tot;
    }
}

// ms[v] = MS id of its listed pair: rank_of[record] minus the field's first
// id, with the record index in ms[v] on entry.  Runs over the chase tiles, so
// every block knows its field.  STREAM: see kWholeLines.
template <class T, bool STREAM = false>
__global__ __launch_bounds__(kBlock) void k_ms_final(Fields F, const uint32_t* rank_of, const uint32_t* fbase) {
    uint32_t tfirst, tlast;
    block_tiles(F.dev_tiles ? gmem(F.dev_tiles)[1] : F.j_tiles, &tfirst, &tlast);
    if (tfirst >= tlast) return;
    FieldCursor<false> cursor(F);
    // two tiles in flight: the record indices of the next tile are loaded
    // while the ranks of the current one are gathered and stored
    struct Stage {
        int32_t* ms;
        uint32_t base;
        uint32_t lv[kJPer], sl[kJPer];
        bool ok[kJPer];
    };
    auto load = [&](uint32_t tile, Stage& st) {
        const FieldDesc fd = cursor.at(F, tile);
        const uint32_t lt = tile - fd.jbase;
        st.ms = fd.ms;
        st.base = fbase ? fbase[fd.index] : 0u;
#pragma unroll
        for (int i = 0; i < kJPer; ++i) {
            int x, y, z;
            jtile_xyz<T>(fd, lt, threadIdx.x + i * kBlock, &x, &y, &z);
            st.ok[i] = x < fd.nx && y < fd.ny && z < fd.nz;
            st.lv[i] = (uint32_t(z) * uint32_t(fd.ny) + uint32_t(y)) * uint32_t(fd.nx) + uint32_t(x);
            // vertex 0 of the field stands in for lanes past its edge, so the
            // loads need no branch and issue together; in the STREAM form
            // each record index is read past the caches, so that the
            // gathered ranks stay cached
            const auto* p = gmem(fd.ms) + (st.ok[i] ? st.lv[i] : 0u);
            if constexpr (STREAM)
                st.sl[i] = uint32_t(__builtin_nontemporal_load(p));
            else
                st.sl[i] = uint32_t(*p);
        }
    };
    Stage cur, nxt;
    load(tfirst, cur);
    for (uint32_t tile = tfirst; tile < tlast; ++tile) {
        if (tile + 1 < tlast) load(tile + 1, nxt);
        uint32_t r[kJPer];
#pragma unroll
        for (int i = 0; i < kJPer; ++i) r[i] = gmem(rank_of)[cur.ok[i] ? cur.sl[i] : 0u];
#pragma unroll
        for (int i = 0; i < kJPer; ++i)
            if (cur.ok[i]) gmem(cur.ms)[cur.lv[i]] = int32_t(r[i] - cur.base);
        cur = nxt;
    }
}

// First MS id of every field (pairs are sorted by launch-wide asc, so field
// f's pairs start at the first key >= vbase_f << bn) and its K.  One block.
__global__ __launch_bounds__(kBlock) void k_field_base(Fields F, const uint64_t* keys,
                                                       const uint32_t* vals, const uint32_t* count_ptr,
                                                       const uint32_t* k_total, const uint32_t* rank_of,
                                                       int bn, uint32_t* fbase) {
    const uint32_t nf = fields_count(F), count = *count_ptr;
    for (uint32_t f = threadIdx.x; f < nf; f += kBlock) {
        const FieldDesc fd = field_desc(F, f);
        const uint64_t target = uint64_t(fd.vbase) << bn;
        uint32_t lo = 0, hi = count;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) / 2;
            if (keys[mid] < target)
                lo = mid + 1;
            else
                hi = mid;
        }
        fbase[f] = lo < count ? rank_of[vals[lo]] : *k_total;
    }
    __syncthreads();
    for (uint32_t f = threadIdx.x; f < nf; f += kBlock) {
        const FieldDesc fd = field_desc(F, f);
        const uint32_t next = f + 1 < nf ? fbase[f + 1] : *k_total;
        if (fd.info) fd.info[3] = int32_t(next - fbase[f]);
    }
}

// info[0..3] = 0 for every field of the launch.
__global__ __launch_bounds__(kBlock) void k_init_fields(Fields F) {
    const uint32_t nf = fields_count(F);
    for (uint32_t f = blockIdx.x * kBlock + threadIdx.x; f < nf; f += gridDim.x * kBlock) {
        const FieldDesc fd = field_desc(F, f);
        if (fd.info) {
            fd.info[0] = 0;
            fd.info[1] = 0;
            fd.info[2] = 0;
            fd.info[3] = 0;
        }
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
