// Multi-label marching index (Sec. "Multi-Label Marching Triangles/Tetrahedra"):
// the label code of every cell and the number of separating primitives per
// row of cells, then the rows' exclusive prefix, so that a geometry pass can
// write every row's primitives at a known offset.
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

constexpr int kMarchRowsPerWave = 16;
constexpr int kMarchRowsPerBlock = kMarchRowsPerWave * kWavesPerBlock;

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

// Counts.  Each wave owns kMarchRowsPerWave consecutive rows; its lanes take
// 64 consecutive cubes along x and walk the wave's rows in order, so that the
// lower y face of a cube (corners 0, 1, 4, 5; bit 0 = +x, bit 1 = +y, bit 2 =
// +z) and the label equalities on it come from the upper face of the cube
// below in the previous row; only the first row of the wave and of each z
// slab reads it fresh.  A cell's count depends only on E (above): a
// tetrahedron (0, v1, v2, 7) has E = [0=v1] + [0=v2] + [0=7] + [v1=v2] +
// [v1=7] + [v2=7], and of these the six [0=k], [k=7] serve two tetrahedra
// each and [0=7] all six.  Every lane keeps its own running count per row in
// LDS; at the end the counts of a row are summed over the lanes, row_offsets[r]
// receives row r's count (scanned in place later) and block_sums[block] the
// block's sum.
template <bool THREE_D, int MODE, bool CODES>
__global__ __launch_bounds__(kBlock) void k_march_count(const int32_t* labels, int nx, int ny, uint32_t rows,
                                                        uint8_t* codes, uint64_t* row_offsets,
                                                        uint64_t* block_sums) {
    __shared__ uint64_t wsum[kWavesPerBlock];
    __shared__ uint32_t rcnt[kWavesPerBlock][kMarchRowsPerWave][kWave];
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(wave_id());
    const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t r0 = b * kMarchRowsPerBlock + uint32_t(w) * kMarchRowsPerWave;
    const int nrow = r0 < rows ? int(min<uint32_t>(kMarchRowsPerWave, rows - r0)) : 0;
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

// Row counts -> exclusive row offsets: block b's rows start at block_sums[b].
__global__ __launch_bounds__(kBlock) void k_march_offsets(uint64_t* row_offsets, uint32_t rows,
                                                          const uint64_t* block_sums) {
    __shared__ uint64_t tmp[kWavesPerBlock];
    static_assert(kMarchRowsPerBlock <= kBlock, "one row per thread");
    const uint32_t b = blockIdx.x;
    const uint32_t r = b * kMarchRowsPerBlock + threadIdx.x;
    const bool mine = threadIdx.x < kMarchRowsPerBlock && r < rows;
    const uint64_t c = mine ? row_offsets[r] : 0ull;
    uint64_t tot;
    const uint64_t e = block_sums[b] + block_exclusive_u64(c, tmp, &tot);
    if (mine) row_offsets[r] = e;
}

}  // namespace plmss
