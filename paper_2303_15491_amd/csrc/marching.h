// Multi-label marching triangles/tetrahedra (Sec. "Multi-Label Marching
// Triangles/Tetrahedra"), in two passes as the paper splits them.  The index:
// the label code of every cell and the number of separating (or boundary)
// primitives per row of cells, then the rows' exclusive prefix.  The
// geometry: every row's primitives written at its offset.
//
// Cells: in 3-D the six Kuhn tetrahedra of every cube (the cut along the cube
// diagonal (1,1,1), the same triangulation as the neighbour scan), in 2-D
// (nz = 1) the two triangles of every square.  A cell's vertices, in
// increasing id order, are the cube's low corner, then one, two (three) unit
// steps along the axes in the order of the cell's permutation; 3-D
// permutations (x,y,z), (x,z,y), (y,x,z), (y,z,x), (z,x,y), (z,y,x) are cells
// 0..5, 2-D (x,y), (y,x) cells 0, 1.  Cell c of cube x in row r is byte
// ((r * (nx-1)) + x) * cells_per_cube + c of the code array; rows are the
// (y, z) rows of cubes, z-major (2-D: the y rows of squares).
//
// Code: a cell vertex's local label is the index of the first vertex that
// carries its label (a: 0, b: 0..1, c: 0..2, d: 0..3); code = b << 4 | c << 2
// | d for a tetrahedron, b << 2 | c for a triangle.
#pragma once

#include "common.h"

namespace plmss {

constexpr int kMarchRowsPerWave = 16;  // at most; fewer when a grid has few rows
constexpr int kMarchRowsPerBlock = kMarchRowsPerWave * kWavesPerBlock;

// Rows per wave of the count kernel: up to kMarchRowsPerWave, fewer when a
// grid has few rows (a 2-D field), so that the launch still has about 4096
// waves.
inline int march_rows_per_wave(uint64_t rows) {
    const uint64_t r = rows / 4096;
    return r < 1 ? 1 : (r > uint64_t(kMarchRowsPerWave) ? kMarchRowsPerWave : int(r));
}

// Primitives of a cell from E, the number of its vertex pairs with equal
// labels (equality is transitive, so E fixes how the labels split: for a
// tetrahedron E = 6 one label, 3 one vertex apart, 2 two and two, 1 three
// labels, 0 four; for a triangle E = 3, 1, 0 for one, two, three labels).
// Four bits per E.  Region separators of the case figures: 0, 1, 2, 5, 12
// triangles per tetrahedron and 0, 1, 3 edges per triangle; region
// boundaries: one triangle per tetrahedron with one vertex apart, one edge
// per triangle with two labels.
constexpr uint32_t kTetSep = (12u << 0) | (5u << 4) | (2u << 8) | (1u << 12);  // E = 0, 1, 2, 3; 6 -> 0
constexpr uint32_t kTetBnd = 1u << 12;                                        // E = 3
constexpr uint32_t kTriSep = (3u << 0) | (1u << 4);                           // E = 0, 1; 3 -> 0
constexpr uint32_t kTriBnd = 1u << 4;                                         // E = 1

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int d) {
    const uint32_t lo = uint32_t(__shfl_up(int(uint32_t(v)), d, kWave));
    const uint32_t hi = uint32_t(__shfl_up(int(uint32_t(v >> 32)), d, kWave));
    return (uint64_t(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_inclusive_u64(uint64_t v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t y = shfl_up_u64(v, d);
        if (lane >= d) v += y;
    }
    return v;
}

// Exclusive scan of one u64 per thread over the block; *total gets the sum.
__device__ __forceinline__ uint64_t block_exclusive_u64(uint64_t x, uint64_t* tmp, uint64_t* total) {
    const int lane = lane_id(), w = wave_id();
    const uint64_t inc = wave_inclusive_u64(x);
    if (lane == kWave - 1) tmp[w] = inc;
    __syncthreads();
    uint64_t base = 0, sum = 0;
#pragma unroll
    for (int i = 0; i < kWavesPerBlock; ++i) {
        base += i < w ? tmp[i] : 0ull;
        sum += tmp[i];
    }
    __syncthreads();
    *total = sum;
    return base + inc - x;
}

// Counts.  Each wave owns rpw (<= kMarchRowsPerWave) consecutive rows; its lanes take
// 64 consecutive cubes along x and walk the wave's rows in order, so that the
// lower y face of a cube (corners 0, 1, 4, 5; bit 0 = +x, bit 1 = +y, bit 2 =
// +z) and the label equalities on it come from the upper face of the same
// cube of the previous row (y - 1); only the first row of the wave and of each
// z slab reads it fresh.  A cell's count depends only on E (above): a
// tetrahedron (0, v1, v2, 7) has E = [0=v1] + [0=v2] + [0=7] + [v1=v2] +
// [v1=7] + [v2=7], and of these the six [0=k], [k=7] serve two tetrahedra
// each and [0=7] all six.  Every lane keeps its own running count per row in
// LDS; at the end the counts of a row are summed over the lanes, row_offsets[r]
// receives row r's count (scanned in place later) and block_sums[block] the
// block's sum.
template <bool THREE_D, int MODE, bool CODES>
__global__ __launch_bounds__(kBlock) void k_march_count(const int32_t* labels, int nx, int ny, uint32_t rows,
                                                        uint8_t* codes, uint64_t* row_offsets,
                                                        uint64_t* block_sums, int rpw) {
    __shared__ uint64_t wsum[kWavesPerBlock];
    __shared__ uint32_t rcnt[kWavesPerBlock][kMarchRowsPerWave][kWave];
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(wave_id());
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t r0 = (b * kWavesPerBlock + uint32_t(w)) * uint32_t(rpw);
    const int nrow = r0 < rows ? int(min<uint32_t>(uint32_t(rpw), rows - r0)) : 0;
    const int ncube = nx - 1;
    const uint32_t ycubes = THREE_D ? uint32_t(ny - 1) : 0xffffffffu;
    const uint32_t y0 = THREE_D ? r0 % ycubes : r0, z0 = THREE_D ? r0 / ycubes : 0u;
    const size_t plane = size_t(nx) * size_t(ny);
    constexpr int kCells = THREE_D ? 6 : 2;
    constexpr uint32_t kLut = THREE_D ? (MODE ? kTetBnd : kTetSep) : (MODE ? kTriBnd : kTriSep);
    uint32_t (&cnt)[kMarchRowsPerWave][kWave] = rcnt[w];
#pragma unroll
    for (int k = 0; k < kMarchRowsPerWave; ++k) cnt[k][lane] = 0;

    for (int x0 = 0; x0 < ncube; x0 += kWave) {
        const int x = x0 + lane;
        const bool valid = x < ncube;
        const int xc = valid ? x : ncube - 1;  // lanes past the row re-read its last cube
        // lower face: labels and equalities [0=1], [0=4], [0=5], [1=5], [4=5]
        int32_t l0 = 0, l1 = 0, l4 = 0, l5 = 0;
        bool e01 = false, e04 = false, e05 = false, e15 = false, e45 = false;
        uint32_t y = y0, z = z0;
        for (int k = 0; k < nrow; ++k) {
            const int32_t* lo = labels + (size_t(z) * size_t(ny) + y) * size_t(nx);
            const int32_t* hi = lo + nx;
            if (k == 0 || y == 0) {
                l0 = gmem(lo)[xc];
                l1 = gmem(lo)[xc + 1];
                if (THREE_D) {
                    l4 = gmem(lo + plane)[xc];
                    l5 = gmem(lo + plane)[xc + 1];
                }
                e01 = l0 == l1;
                e04 = l0 == l4;
                e05 = l0 == l5;
                e15 = l1 == l5;
                e45 = l4 == l5;
            }
            const int32_t l2 = gmem(hi)[xc];
            const int32_t l3 = gmem(hi)[xc + 1];
            uint32_t total = 0;
            uint32_t cd[kCells];
            if constexpr (THREE_D) {
                const int32_t l6 = gmem(hi + plane)[xc];
                const int32_t l7 = gmem(hi + plane)[xc + 1];
                const bool e02 = l0 == l2, e03 = l0 == l3, e06 = l0 == l6, e07 = l0 == l7;
                const bool e17 = l1 == l7, e27 = l2 == l7, e37 = l3 == l7, e47 = l4 == l7, e57 = l5 == l7,
                           e67 = l6 == l7;
                const bool e13 = l1 == l3, e23 = l2 == l3, e26 = l2 == l6, e46 = l4 == l6;
                // 4 [0=k] + 4 [k=7] per path vertex k, [0=7] folded into the table
                const uint32_t q1 = (e01 ? 4u : 0u) + (e17 ? 4u : 0u), q2 = (e02 ? 4u : 0u) + (e27 ? 4u : 0u);
                const uint32_t q4 = (e04 ? 4u : 0u) + (e47 ? 4u : 0u), q3 = (e03 ? 4u : 0u) + (e37 ? 4u : 0u);
                const uint32_t q5 = (e05 ? 4u : 0u) + (e57 ? 4u : 0u), q6 = (e06 ? 4u : 0u) + (e67 ? 4u : 0u);
                const uint32_t lut = e07 ? (kLut >> 4) : kLut;
                // tetrahedra (x,y,z) (x,z,y) (y,x,z) (y,z,x) (z,x,y) (z,y,x): paths 0-1-3-7, 0-1-5-7,
                // 0-2-3-7, 0-2-6-7, 0-4-5-7, 0-4-6-7
                total = __builtin_amdgcn_ubfe(lut, q1 + q3 + (e13 ? 4u : 0u), 4) +
                        __builtin_amdgcn_ubfe(lut, q1 + q5 + (e15 ? 4u : 0u), 4) +
                        __builtin_amdgcn_ubfe(lut, q2 + q3 + (e23 ? 4u : 0u), 4) +
                        __builtin_amdgcn_ubfe(lut, q2 + q6 + (e26 ? 4u : 0u), 4) +
                        __builtin_amdgcn_ubfe(lut, q4 + q5 + (e45 ? 4u : 0u), 4) +
                        __builtin_amdgcn_ubfe(lut, q4 + q6 + (e46 ? 4u : 0u), 4);
                if constexpr (CODES) {
                    // local labels: b = [b != a]; c = 0 | 1 (c = b) | 2; d = 0 | 1 | 2 (d = c) | 3
                    auto code = [&](bool eab, bool eac, bool ebc, bool ebd, bool ecd) {
                        const uint32_t lc = eac ? 0u : ebc ? 1u : 2u;
                        const uint32_t ld = e07 ? 0u : ebd ? 1u : ecd ? 2u : 3u;
                        return (eab ? 0u : 16u) | (lc << 2) | ld;
                    };
                    cd[0] = code(e01, e03, e13, e17, e37);
                    cd[1] = code(e01, e05, e15, e17, e57);
                    cd[2] = code(e02, e03, e23, e27, e37);
                    cd[3] = code(e02, e06, e26, e27, e67);
                    cd[4] = code(e04, e05, e45, e47, e57);
                    cd[5] = code(e04, e06, e46, e47, e67);
                }
                // the upper face is the next row's lower face
                l0 = l2, l1 = l3, l4 = l6, l5 = l7;
                e01 = e23, e04 = e26, e05 = e27, e15 = e37, e45 = e67;
            } else {
                // triangles (x,y) and (y,x): paths 0-1-3 and 0-2-3, [0=3] folded into the table
                const bool e02 = l0 == l2, e03 = l0 == l3, e13 = l1 == l3, e23 = l2 == l3;
                const uint32_t lut = e03 ? (kLut >> 4) : kLut;
                total = __builtin_amdgcn_ubfe(lut, (e01 ? 4u : 0u) + (e13 ? 4u : 0u), 4) +
                        __builtin_amdgcn_ubfe(lut, (e02 ? 4u : 0u) + (e23 ? 4u : 0u), 4);
                if constexpr (CODES) {
                    cd[0] = (e01 ? 0u : 4u) | (e03 ? 0u : e13 ? 1u : 2u);
                    cd[1] = (e02 ? 0u : 4u) | (e03 ? 0u : e23 ? 1u : 2u);
                }
                l0 = l2, l1 = l3;
                e01 = e23;
            }
            cnt[k][lane] += valid ? total : 0u;
            if (valid) {
                if constexpr (CODES) {  // a cube's codes as 16-bit stores (codes is 2-byte aligned)
                    const size_t r = r0 + uint32_t(k);
                    auto* c16 =
                        gmem(reinterpret_cast<uint16_t*>(codes + (r * size_t(ncube) + size_t(x)) * kCells));
#pragma unroll
                    for (int t = 0; t < kCells; t += 2) c16[t / 2] = uint16_t(cd[t] | (cd[t + 1] << 8));
                }
            }
            if (THREE_D && ++y == ycubes) y = 0, ++z;
            if (!THREE_D) ++y;
        }
    }
    // row sums over the wave (a row holds up to 12 * 6 * (nx - 1)): lane j adds
    // a quarter of row j / 4, then groups of four lanes combine
    __syncthreads();
    static_assert(kWave / 4 == kMarchRowsPerWave, "four lanes per row");
    const int kr = lane >> 2, q = lane & 3;
    uint64_t part = 0;
#pragma unroll
    for (int i = 0; i < kWave / 4; ++i) part += cnt[kr][q * (kWave / 4) + i];
    auto xor_u64 = [](uint64_t v, int d) {
        const uint32_t vlo = uint32_t(__shfl_xor(int(uint32_t(v)), d, kWave));
        const uint32_t vhi = uint32_t(__shfl_xor(int(uint32_t(v >> 32)), d, kWave));
        return (uint64_t(vhi) << 32) | vlo;
    };
    uint64_t row = part + xor_u64(part, 1);
    row += xor_u64(row, 2);
    if (q == 0 && kr < nrow) gmem(row_offsets)[r0 + uint32_t(kr)] = row;
    uint64_t wave_total = kr < nrow ? part : 0ull;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) wave_total += xor_u64(wave_total, d);
    if (lane == 0) wsum[w] = wave_total;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
#pragma unroll
        for (int i = 0; i < kWavesPerBlock; ++i) t += wsum[i];
        gmem(block_sums)[b] = t;
    }
}

// One block: exclusive scan of block_sums[0..n) in place, the sum to *total.
__global__ __launch_bounds__(kBlock) void k_march_scan_blocks(uint64_t* block_sums, uint32_t n, uint64_t* total) {
    __shared__ uint64_t tmp[kWavesPerBlock];
    uint64_t run = 0;
    for (uint32_t base = 0; base < n; base += kBlock * 4) {
        const uint32_t beg = base + threadIdx.x * 4;
        uint64_t c[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] = beg + i < n ? block_sums[beg + i] : 0ull;
        uint64_t tot;
        uint64_t e = run + block_exclusive_u64(c[0] + c[1] + c[2] + c[3], tmp, &tot);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (beg + i < n) block_sums[beg + i] = e;
            e += c[i];
        }
        run += tot;
    }
    if (threadIdx.x == 0) *total = run;
}

// Row counts -> exclusive row offsets: block b's rows (rpb of them, as the
// count kernel's block b) start at block_sums[b].
__global__ __launch_bounds__(kBlock) void k_march_offsets(uint64_t* row_offsets, uint32_t rows,
                                                          const uint64_t* block_sums, int rpb) {
    __shared__ uint64_t tmp[kWavesPerBlock];
    static_assert(kMarchRowsPerBlock <= kBlock, "one row per thread");
    const uint32_t b = blockIdx.x;
    const uint32_t r = b * uint32_t(rpb) + threadIdx.x;
    const bool mine = int(threadIdx.x) < rpb && r < rows;
    const uint64_t c = mine ? row_offsets[r] : 0ull;
    uint64_t tot;
    const uint64_t e = block_sums[b] + block_exclusive_u64(c, tmp, &tot);
    if (mine) row_offsets[r] = e;
}

}  // namespace plmss

namespace plmss {

// ---- geometry pass -----------------------------------------------------------------------
// The primitives of every cell, written at the offsets of the index pass.  A
// primitive is encoded in 16 bits: three (in 2-D two) point masks of 4 bits
// (bit i = cell vertex i; the point is the average of those vertices) and
// two 2-bit vertex indices u < w whose labels are the two it separates (for
// a boundary: a vertex of the equal ones, then the odd one).
struct GeoLut {
    uint8_t base[32], count[32];
    uint16_t prim[64];
};

constexpr uint16_t geo_prim(int s0, int s1, int s2, int u, int w) {
    return uint16_t(s0 | (s1 << 4) | (s2 << 8) | (u << 12) | (w << 14));
}

// Primitives of one cell from its local labels (k[i] = first vertex with
// vertex i's label): tetrahedra (nv = 4) or triangles (nv = 3).
constexpr int geo_cell(const int* k, int nv, int mode, uint16_t* out) {
    int n = 0, groups = 0, size[4] = {0, 0, 0, 0};
    for (int i = 0; i < nv; ++i) {
        size[k[i]] += 1;
        groups += k[i] == i;
    }
    int lone = -1;
    for (int i = 0; i < nv; ++i)
        if (size[k[i]] == 1 && groups == 2) lone = i;
    auto bit = [](int i) { return 1 << i; };
    if (mode == 1) {  // boundaries: the equal vertices of a cell with one vertex apart
        if (lone < 0) return 0;
        int v[3] = {0, 0, 0}, m = 0;
        for (int i = 0; i < nv; ++i)
            if (i != lone) v[m++] = i;
        out[n++] = geo_prim(bit(v[0]), bit(v[1]), nv == 4 ? bit(v[2]) : 0, v[0], lone);
        return n;
    }
    if (groups == 1) return 0;
    if (nv == 3) {
        if (groups == 2) {  // the edge between the two edges that leave the odd vertex
            int o[2] = {0, 0}, m = 0;
            for (int i = 0; i < 3; ++i)
                if (i != lone) o[m++] = i;
            out[n++] = geo_prim(bit(lone) | bit(o[0]), bit(lone) | bit(o[1]), 0, k[lone] < k[o[0]] ? k[lone] : k[o[0]],
                                k[lone] < k[o[0]] ? k[o[0]] : k[lone]);
            return n;
        }
        for (int a = 0; a < 3; ++a)  // three labels: centre to each edge midpoint
            for (int b = a + 1; b < 3; ++b) out[n++] = geo_prim(7, bit(a) | bit(b), 0, a, b);
        return n;
    }
    if (groups == 2 && lone >= 0) {
        int o[3] = {0, 0, 0}, m = 0;
        for (int i = 0; i < 4; ++i)
            if (i != lone) o[m++] = i;
        const int g0 = k[lone], g1 = k[o[0]];
        out[n++] = geo_prim(bit(lone) | bit(o[0]), bit(lone) | bit(o[1]), bit(lone) | bit(o[2]), g0 < g1 ? g0 : g1,
                            g0 < g1 ? g1 : g0);
        return n;
    }
    if (groups == 2) {  // two and two: vertex 0 with q, r < s apart
        int q = 0, r = -1, s = 0;
        for (int i = 1; i < 4; ++i) {
            if (k[i] == 0) q = i;
            else if (r < 0) r = i;
            else s = i;
        }
        out[n++] = geo_prim(bit(0) | bit(r), bit(0) | bit(s), bit(q) | bit(r), 0, r);
        out[n++] = geo_prim(bit(0) | bit(s), bit(q) | bit(r), bit(q) | bit(s), 0, r);
        return n;
    }
    if (groups == 3) {  // p < q share a label, r < s alone
        int p = -1, q = 0, r = -1, s = 0;
        for (int i = 0; i < 4; ++i) {
            if (size[k[i]] == 2) {
                if (p < 0) p = i;
                else q = i;
            } else if (r < 0) r = i;
            else s = i;
        }
        const int t1 = bit(p) | bit(r) | bit(s), t2 = bit(q) | bit(r) | bit(s);
        auto lo = [](int a, int b) { return a < b ? a : b; };
        auto hi = [](int a, int b) { return a < b ? b : a; };
        out[n++] = geo_prim(t1, t2, bit(p) | bit(r), lo(p, r), hi(p, r));
        out[n++] = geo_prim(t2, bit(p) | bit(r), bit(q) | bit(r), lo(p, r), hi(p, r));
        out[n++] = geo_prim(t1, t2, bit(r) | bit(s), r, s);
        out[n++] = geo_prim(t1, t2, bit(p) | bit(s), lo(p, s), hi(p, s));
        out[n++] = geo_prim(t2, bit(p) | bit(s), bit(q) | bit(s), lo(p, s), hi(p, s));
        return n;
    }
    // four labels: the centre, each face's centre and each of its edges
    const int faces[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
    for (int f = 0; f < 4; ++f) {
        const int a = faces[f][0], b = faces[f][1], c = faces[f][2];
        const int fm = bit(a) | bit(b) | bit(c);
        out[n++] = geo_prim(15, fm, bit(a) | bit(b), a, b);
        out[n++] = geo_prim(15, fm, bit(a) | bit(c), a, c);
        out[n++] = geo_prim(15, fm, bit(b) | bit(c), b, c);
    }
    return n;
}

// Tables over all codes (invalid codes get no primitives).
constexpr GeoLut make_geo_lut(bool three_d, int mode) {
    GeoLut t{};
    int n = 0;
    const int nv = three_d ? 4 : 3;
    for (int code = 0; code < 32; ++code) {
        int k[4] = {0, 0, 0, 0};
        if (three_d) k[1] = code >> 4, k[2] = (code >> 2) & 3, k[3] = code & 3;
        else k[1] = (code >> 2) & 1, k[2] = code & 3;
        bool valid = three_d || code < 8;
        for (int i = 0; i < nv; ++i) valid = valid && k[i] <= i && k[k[i]] == k[i];
        t.base[code] = uint8_t(n);
        const int m = valid ? geo_cell(k, nv, mode, t.prim + n) : 0;
        t.count[code] = uint8_t(m);
        n += m;
    }
    return t;
}

// The same tables expanded per cell shape (tetrahedron t of a cube, or
// triangle t of a square): each primitive's points as offsets from the cube's
// low corner in twelfths of a grid step, 4 bits per axis (point p, axis a at
// bit 12p + 4a; a point averaging |S| vertices is (12 / |S|) times the sum
// of their corner offsets), the two vertices u, w at bits 36 and 38, and
// their corners (3 bits each) at bits 40 and 43.
struct GeoTab {
    uint8_t base[32], count[32];
    uint64_t ent[6][64];
};

constexpr GeoTab make_geo_tab(bool three_d, int mode) {
    const GeoLut l = make_geo_lut(three_d, mode);
    GeoTab t{};
    for (int c = 0; c < 32; ++c) t.base[c] = l.base[c], t.count[c] = l.count[c];
    const int cells = three_d ? 6 : 2, npts = three_d ? 3 : 2, dims = three_d ? 3 : 2;
    // corners (bit 0 = +x, 1 = +y, 2 = +z) of each cell's path vertices
    const int tet[6][4] = {{0, 1, 3, 7}, {0, 1, 5, 7}, {0, 2, 3, 7}, {0, 2, 6, 7}, {0, 4, 5, 7}, {0, 4, 6, 7}};
    const int tri[2][4] = {{0, 1, 3, 0}, {0, 2, 3, 0}};
    for (int cell = 0; cell < cells; ++cell) {
        const int* cv = three_d ? tet[cell] : tri[cell];
        for (int e = 0; e < 64; ++e) {
            const uint32_t prim = l.prim[e];
            uint64_t E = 0;
            for (int p = 0; p < npts; ++p) {
                const int S = int(prim >> (4 * p)) & 15;
                int k = 0;
                for (int i = 0; i < 4; ++i) k += (S >> i) & 1;
                if (k == 0) continue;
                for (int a = 0; a < dims; ++a) {
                    int d = 0;
                    for (int i = 0; i < 4; ++i)
                        if ((S >> i) & 1) d += (cv[i] >> a) & 1;
                    E |= uint64_t((12 / k) * d) << (12 * p + 4 * a);
                }
            }
            const int u = (prim >> 12) & 3, wv = (prim >> 14) & 3;
            E |= uint64_t(u) << 36 | uint64_t(wv) << 38 | uint64_t(cv[u]) << 40 | uint64_t(cv[wv]) << 43;
            t.ent[cell][e] = E;
        }
    }
    return t;
}

__constant__ const GeoTab kGeoTab[4] = {make_geo_tab(false, 0), make_geo_tab(false, 1), make_geo_tab(true, 0),
                                        make_geo_tab(true, 1)};

constexpr int kGeoWaves = kWavesPerBlock;

// One wave per row of cubes; its lanes take 64 cubes at a time, count their
// primitives, scan the counts over the wave, keep each cube's corner labels,
// offset, cell starts and table bases in LDS, and then write the chunk's
// primitives with consecutive lanes on consecutive primitives: each lane
// finds its cube by a binary search over the offsets, then its cell from the
// cube's cell starts and its entry from the cell's table base.  The points of
// 64 primitives are staged in LDS and stored by consecutive lanes on
// consecutive floats.
template <bool THREE_D, int MODE>
__global__ __launch_bounds__(kBlock) void k_march_geometry(const int32_t* labels, int nx, int ny, uint32_t rows,
                                                           const uint64_t* row_offsets, uint64_t capacity,
                                                           float* xyz, int32_t* sides) {
    constexpr int kCells = THREE_D ? 6 : 2;
    constexpr int kCorners = THREE_D ? 8 : 4;
    constexpr int kPts = THREE_D ? 3 : 2;
    constexpr int kDim = THREE_D ? 3 : 2;
    __shared__ int32_t s_lab[kGeoWaves][kCorners][kWave];
    __shared__ uint32_t s_off[kGeoWaves][kWave + 1];
    // per cube: byte k = first primitive of cell k within the cube (k = 0..5),
    // and byte k = cell k's first entry in the table
    __shared__ uint64_t s_pre[kGeoWaves][kWave], s_bas[kGeoWaves][kWave];
    constexpr int kVals = kPts * kDim;              // floats per primitive
    __shared__ float s_xyz[kGeoWaves][kWave * kVals];
    __shared__ GeoTab s_tab;
    {
        static_assert(sizeof(GeoTab) % 4 == 0, "copied in words");
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&kGeoTab[(THREE_D ? 2 : 0) + MODE]);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&s_tab);
        for (int i = threadIdx.x; i < int(sizeof(GeoTab) / 4); i += kBlock) dst[i] = src[i];
        __syncthreads();
    }
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(wave_id());
    const uint32_t r = xcd_block(blockIdx.x, gridDim.x) * kGeoWaves + uint32_t(w);
    if (r >= rows) return;  // no block-wide barrier below
    const int ncube = nx - 1;
    const uint32_t y = THREE_D ? r % uint32_t(ny - 1) : r, z = THREE_D ? r / uint32_t(ny - 1) : 0u;
    const size_t plane = size_t(nx) * size_t(ny);
    const int32_t* p00 = labels + (size_t(z) * size_t(ny) + y) * size_t(nx);
    const bool narrow = nx < (1 << 27) && ny < (1 << 27) && y < (1u << 27) && z < (1u << 27);
    uint64_t base = gmem(row_offsets)[r];
    // the tetrahedra's second and third path vertices (corner bit 0 = +x,
    // 1 = +y, 2 = +z) and their axis order
    constexpr int v1[6] = {1, 1, 2, 2, 4, 4}, v2[6] = {3, 5, 3, 6, 5, 6};
    for (int x0 = 0; x0 < ncube; x0 += kWave) {
        const int x = x0 + lane;
        const bool valid = x < ncube;
        const int xc = valid ? x : ncube - 1;
        int32_t l[8];
        l[0] = gmem(p00)[xc];
        l[1] = gmem(p00)[xc + 1];
        l[2] = gmem(p00 + nx)[xc];
        l[3] = gmem(p00 + nx)[xc + 1];
        if (THREE_D) {
            l[4] = gmem(p00 + plane)[xc];
            l[5] = gmem(p00 + plane)[xc + 1];
            l[6] = gmem(p00 + plane + nx)[xc];
            l[7] = gmem(p00 + plane + nx)[xc + 1];
        }
        uint64_t pre = 0, bas = 0;
        uint32_t total = 0;
#pragma unroll
        for (int t = 0; t < kCells; ++t) {
            uint32_t code;
            if constexpr (THREE_D) {
                const int32_t a = l[0], b = l[v1[t]], c = l[v2[t]], d = l[7];
                code = (b == a ? 0u : 16u) | ((c == a ? 0u : c == b ? 1u : 2u) << 2) |
                       (d == a ? 0u : d == b ? 1u : d == c ? 2u : 3u);
            } else {
                const int32_t a = l[0], b = l[t == 0 ? 1 : 2], c = l[3];
                code = (b == a ? 0u : 4u) | (c == a ? 0u : c == b ? 1u : 2u);
            }
            const uint32_t m = valid ? uint32_t(s_tab.count[code]) : 0u;
            pre |= uint64_t(total) << (8 * t);
            bas |= uint64_t(s_tab.base[code]) << (8 * t);
            total += m;
        }
        // exclusive scan of the cube totals over the wave
        uint32_t inc = total;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t v = uint32_t(__shfl_up(int(inc), d, kWave));
            if (lane >= d) inc += v;
        }
        const uint32_t chunk = uint32_t(__shfl(int(inc), kWave - 1, kWave));
#pragma unroll
        for (int i = 0; i < kCorners; ++i) s_lab[w][i][lane] = l[i];
        s_off[w][lane] = inc - total;
        s_pre[w][lane] = pre;
        s_bas[w][lane] = bas;
        if (lane == 0) s_off[w][kWave] = chunk;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (uint32_t j0 = 0; j0 < chunk; j0 += kWave) {
            const uint32_t i = j0 + uint32_t(lane);
            if (i < chunk) {
                int c = 0;
#pragma unroll
                for (int step = kWave / 2; step > 0; step >>= 1)
                    if (s_off[w][c + step] <= i) c += step;
                uint32_t rem = i - s_off[w][c];  // primitive within the cube (< 128)
                const uint64_t pk = s_pre[w][c];
                // the cell: how many of the cells 1..5 start at or before rem
                // (four byte compares at once: no byte borrows, all are < 128)
                int t;
                if constexpr (THREE_D) {
                    const uint32_t starts = uint32_t(pk >> 8);
                    const uint32_t ge = (((rem * 0x01010101u) | 0x80808080u) - starts) & 0x80808080u;
                    t = __builtin_popcount(ge) + (rem >= uint32_t(pk >> 40) ? 1 : 0);
                } else {
                    t = rem >= uint32_t(pk >> 8) ? 1 : 0;
                }
                rem -= uint32_t(pk >> (8 * t)) & 0xffu;
                const uint32_t tb = uint32_t(s_bas[w][c] >> (8 * t)) & 0xffu;
                const uint64_t e = s_tab.ent[t][tb + rem];
                if (xyz) {
                    // a point: (12 * corner + its offset in twelfths) / 12,
                    // staged in LDS so that the wave's stores are contiguous
                    const double inv12 = 1.0 / 12.0;
                    const uint32_t elo = uint32_t(e), ehi = uint32_t(e >> 32);
                    auto twelfths = [&](int p, int a) {  // the 4-bit offset of point p, axis a
                        const int bit = 12 * p + 4 * a;
                        return int((bit < 32 ? elo >> bit : ehi >> (bit - 32)) & 15u);
                    };
                    if (narrow) {  // 12 * coordinate fits int32
                        const int o12[3] = {12 * (x0 + c), 12 * int(y), 12 * int(z)};
#pragma unroll
                        for (int p = 0; p < kPts; ++p)
#pragma unroll
                            for (int a = 0; a < kDim; ++a)
                                s_xyz[w][lane * kVals + p * kDim + a] =
                                    float(double(o12[a] + twelfths(p, a)) * inv12);
                    } else {
                        const int64_t o12[3] = {12 * int64_t(x0 + c), 12 * int64_t(y), 12 * int64_t(z)};
#pragma unroll
                        for (int p = 0; p < kPts; ++p)
#pragma unroll
                            for (int a = 0; a < kDim; ++a)
                                s_xyz[w][lane * kVals + p * kDim + a] =
                                    float(double(o12[a] + twelfths(p, a)) * inv12);
                    }
                }
                const uint64_t out = base + i;
                if (sides && out < capacity) {
                    const int cu = int(e >> 40) & 7, cw = int(e >> 43) & 7;
                    typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
                    gmem(reinterpret_cast<i32x2*>(sides))[out] = i32x2{s_lab[w][cu][c], s_lab[w][cw][c]};
                }
            }
            if (xyz) {  // the staged points: consecutive lanes on consecutive floats
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const uint64_t first = base + j0;
                const uint32_t nvals = min(uint32_t(kWave), chunk - j0) * uint32_t(kVals);
                const uint64_t room = capacity > first ? (capacity - first) * kVals : 0;
                const uint32_t lim = room < nvals ? uint32_t(room) : nvals;
                float* dst = xyz + first * kVals;
                if (lim == uint32_t(kWave * kVals)) {  // a full set: no per-store bound
#pragma unroll
                    for (int q = 0; q < kVals; ++q) gmem(dst)[q * kWave + lane] = s_xyz[w][q * kWave + lane];
                } else {
#pragma unroll
                    for (int q = 0; q < kVals; ++q) {
                        const uint32_t idx = uint32_t(q * kWave + lane);
                        if (idx < lim) gmem(dst)[idx] = s_xyz[w][idx];
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        base += chunk;
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace plmss
