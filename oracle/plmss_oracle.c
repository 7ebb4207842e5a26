/*
 * plmss_oracle.c -- serial CPU oracle for the piecewise-linear Morse-Smale
 * segmentation (Maack et al., "Parallel Computation of Piecewise Linear
 * Morse-Smale Segmentations", arXiv 2303.15491).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  It shares no code,
 * header, table or helper with the GPU library, and only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Domain (paper, Sec. "Input Data" and the caption of Table 2): a regular
 * nx x ny x nz vertex grid, vertex id v = x + nx*(y + ny*z), cut into six
 * tetrahedra per cube.  The cut used here is the Freudenthal/Kuhn one whose
 * cube diagonal is (1,1,1); its 2-D restriction is the (+1,+1) diagonal drawn
 * in the paper's Fig. 1 (fig:wallmodes).  A vertex is joined by an edge to the
 * vertices at the offsets {(a,b,c) in {0,1}^3, not all zero} and their
 * negatives: 14 in 3-D, 6 in 2-D (nz = 1), 2 in 1-D.  No wrap-around.
 *
 * Every function is serial, allocates with malloc, and reports failure through
 * its return code (see ORC_* below).  All arrays are host memory owned by the
 * caller.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_DIMS (-2)
#define ORC_E_TOO_LARGE (-3)
#define ORC_E_NAN (-4)
#define ORC_E_NOMEM (-7)

/* The seven edge directions of the Freudenthal cube; the full neighbourhood
 * is these and their negatives. */
static const int EDGE_DIR[7][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}};

typedef struct {
    int64_t nx, ny, nz, n;
} grid_t;

static int make_grid(int64_t nx, int64_t ny, int64_t nz, grid_t* g) {
    if (nx < 1 || ny < 1 || nz < 1) return ORC_E_DIMS;
    if (nx > INT32_MAX || ny > INT32_MAX || nz > INT32_MAX) return ORC_E_TOO_LARGE;
    g->nx = nx;
    g->ny = ny;
    g->nz = nz;
    g->n = nx * ny;
    if (g->n > INT32_MAX || g->n * nz > INT32_MAX) return ORC_E_TOO_LARGE;
    g->n *= nz;
    return ORC_OK;
}

/* Writes the ids of the in-grid neighbours of v into nb[]; returns how many. */
static int neighbours(const grid_t* g, int64_t v, int64_t nb[14]) {
    int64_t x = v % g->nx, y = (v / g->nx) % g->ny, z = v / (g->nx * g->ny);
    int k = 0;
    for (int d = 0; d < 7; ++d) {
        for (int s = -1; s <= 1; s += 2) {
            int64_t xx = x + s * EDGE_DIR[d][0];
            int64_t yy = y + s * EDGE_DIR[d][1];
            int64_t zz = z + s * EDGE_DIR[d][2];
            if (xx < 0 || yy < 0 || zz < 0 || xx >= g->nx || yy >= g->ny || zz >= g->nz) continue;
            nb[k++] = xx + g->nx * (yy + g->ny * zz);
        }
    }
    return k;
}

/* Field value widened to double: exact for float32, identity for float64. */
static double value(const void* f, int dtype, int64_t v) {
    return dtype == 0 ? (double)((const float*)f)[v] : ((const double*)f)[v];
}

static int has_nan(const void* f, int dtype, int64_t n) {
    for (int64_t v = 0; v < n; ++v) {
        double a = value(f, dtype, v);
        if (a != a) return 1;
    }
    return 0;
}

/* Simulation of Simplicity comparison (paper, Sec. "Preprocessing"): u comes
 * after w in the global vertex order iff f(u) > f(w), or the values are equal
 * and u has the larger index.  IEEE comparison, so -0 and +0 are equal. */
static int sos_after(const void* f, int dtype, int64_t u, int64_t w) {
    double a = value(f, dtype, u), b = value(f, dtype, w);
    if (a > b) return 1;
    if (a < b) return 0;
    return u > w;
}

typedef struct {
    double val;
    int64_t idx;
} keyed_t;

static int cmp_keyed(const void* pa, const void* pb) {
    const keyed_t* a = (const keyed_t*)pa;
    const keyed_t* b = (const keyed_t*)pb;
    if (a->val < b->val) return -1;
    if (a->val > b->val) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

static int cmp_u64(const void* pa, const void* pb) {
    uint64_t a = *(const uint64_t*)pa, b = *(const uint64_t*)pb;
    return (a > b) - (a < b);
}

/*
 * Order field (paper, Sec. "Preprocessing"): sort the vertices by value,
 * breaking ties by vertex index, and give each vertex its position in that
 * sorted array.  perm (nullable) receives the sorted array itself.
 */
int plmss_oracle_order(const void* f, int dtype, int64_t nx, int64_t ny, int64_t nz,
                       int32_t* order, int32_t* perm) {
    grid_t g;
    int rc = make_grid(nx, ny, nz, &g);
    if (rc) return rc;
    if (!f || !order || (dtype != 0 && dtype != 1)) return ORC_E_ARG;
    if (has_nan(f, dtype, g.n)) return ORC_E_NAN;
    keyed_t* a = (keyed_t*)malloc(sizeof(keyed_t) * (size_t)g.n);
    if (!a) return ORC_E_NOMEM;
    for (int64_t v = 0; v < g.n; ++v) {
        a[v].val = value(f, dtype, v);
        a[v].idx = v;
    }
    qsort(a, (size_t)g.n, sizeof(keyed_t), cmp_keyed);
    for (int64_t i = 0; i < g.n; ++i) {
        order[a[i].idx] = (int32_t)i;
        if (perm) perm[i] = (int32_t)a[i].idx;
    }
    free(a);
    return ORC_OK;
}

/*
 * Steepest neighbours (paper, Sec. "Ascending and Descending Segmentation"):
 * up[v] is the neighbour with the largest order value, dn[v] the one with the
 * smallest.  A vertex with no larger (smaller) neighbour is a maximum
 * (minimum) and points to itself.
 */
int plmss_oracle_steepest(const int32_t* order, int64_t nx, int64_t ny, int64_t nz,
                          int32_t* up, int32_t* dn) {
    grid_t g;
    int rc = make_grid(nx, ny, nz, &g);
    if (rc) return rc;
    if (!order || !up || !dn) return ORC_E_ARG;
    int64_t nb[14];
    for (int64_t v = 0; v < g.n; ++v) {
        int k = neighbours(&g, v, nb);
        int64_t hi = v, lo = v;
        for (int i = 0; i < k; ++i) {
            if (order[nb[i]] > order[hi]) hi = nb[i];
            if (order[nb[i]] < order[lo]) lo = nb[i];
        }
        up[v] = (int32_t)hi;
        dn[v] = (int32_t)lo;
    }
    return ORC_OK;
}

/*
 * Extremum labels as the fixed point the path compression of the paper
 * converges to: desc[v] is the maximum that the chain v, up[v], up[up[v]], ...
 * ends in, asc[v] the minimum of the dn chain.  Computed by one pass over the
 * sorted vertex array: walking from the top, up[v] lies above v and has been
 * labelled already, so desc[v] = desc[up[v]]; asc symmetrically from the
 * bottom.
 */
int plmss_oracle_labels(const int32_t* perm, const int32_t* up, const int32_t* dn, int64_t n,
                        int32_t* asc, int32_t* desc) {
    if (!perm || !up || !dn || !asc || !desc || n < 1) return ORC_E_ARG;
    for (int64_t i = n - 1; i >= 0; --i) {
        int32_t v = perm[i];
        desc[v] = (up[v] == v) ? v : desc[up[v]];
    }
    for (int64_t i = 0; i < n; ++i) {
        int32_t v = perm[i];
        asc[v] = (dn[v] == v) ? v : asc[dn[v]];
    }
    return ORC_OK;
}

/*
 * Morse-Smale segmentation (paper, Sec. "Morse-Smale Segmentation"): vertices
 * with the same (minimum, maximum) pair form one region.  Regions are numbered
 * 0..K-1 by the lexicographic order of their (asc, desc) pair.
 */
int plmss_oracle_ms(const int32_t* asc, const int32_t* desc, int64_t n, int32_t* ms, int64_t* k_out) {
    if (!asc || !desc || !ms || n < 1) return ORC_E_ARG;
    uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    if (!key) return ORC_E_NOMEM;
    for (int64_t v = 0; v < n; ++v) key[v] = ((uint64_t)(uint32_t)asc[v] << 32) | (uint32_t)desc[v];
    uint64_t* uniq = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
    if (!uniq) {
        free(key);
        return ORC_E_NOMEM;
    }
    memcpy(uniq, key, sizeof(uint64_t) * (size_t)n);
    qsort(uniq, (size_t)n, sizeof(uint64_t), cmp_u64);
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i)
        if (i == 0 || uniq[i] != uniq[k - 1]) uniq[k++] = uniq[i];
    for (int64_t v = 0; v < n; ++v) {
        int64_t lo = 0, hi = k - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi) / 2;
            if (uniq[mid] < key[v])
                lo = mid + 1;
            else
                hi = mid;
        }
        ms[v] = (int32_t)lo;
    }
    if (k_out) *k_out = k;
    free(uniq);
    free(key);
    return ORC_OK;
}

/*
 * The whole segmentation of one field: order field, steepest neighbours,
 * extremum labels, MS ids.  Any output pointer except asc/desc/ms may be NULL.
 * info (nullable) receives {#minima, #maxima, K}.
 */
int plmss_oracle_segment(const void* f, int dtype, int64_t nx, int64_t ny, int64_t nz,
                         int32_t* order, int32_t* up, int32_t* dn, int32_t* asc, int32_t* desc,
                         int32_t* ms, int64_t* info) {
    grid_t g;
    int rc = make_grid(nx, ny, nz, &g);
    if (rc) return rc;
    if (!f || !asc || !desc || !ms || (dtype != 0 && dtype != 1)) return ORC_E_ARG;
    size_t bytes = sizeof(int32_t) * (size_t)g.n;
    int32_t* o = order ? order : (int32_t*)malloc(bytes);
    int32_t* perm = (int32_t*)malloc(bytes);
    int32_t* u = up ? up : (int32_t*)malloc(bytes);
    int32_t* d = dn ? dn : (int32_t*)malloc(bytes);
    if (!o || !perm || !u || !d) {
        rc = ORC_E_NOMEM;
        goto done;
    }
    rc = plmss_oracle_order(f, dtype, nx, ny, nz, o, perm);
    if (rc) goto done;
    rc = plmss_oracle_steepest(o, nx, ny, nz, u, d);
    if (rc) goto done;
    rc = plmss_oracle_labels(perm, u, d, g.n, asc, desc);
    if (rc) goto done;
    int64_t k = 0;
    rc = plmss_oracle_ms(asc, desc, g.n, ms, &k);
    if (rc) goto done;
    if (info) {
        int64_t nmin = 0, nmax = 0;
        for (int64_t v = 0; v < g.n; ++v) {
            nmin += (asc[v] == v);
            nmax += (desc[v] == v);
        }
        info[0] = nmin;
        info[1] = nmax;
        info[2] = k;
    }
done:
    if (!order) free(o);
    if (!up) free(u);
    if (!dn) free(d);
    free(perm);
    return rc;
}

/*
 * One vertex, straight from the definition of integral lines (paper, Sec.
 * "Integral Lines"): step to the highest neighbour until none is higher, and
 * to the lowest neighbour until none is lower.  "Higher" is the Simulation of
 * Simplicity comparison on (value, index); no order field is built.  Returns
 * the maximum and minimum reached and the number of steps of each walk.
 */
int plmss_oracle_trace(const void* f, int dtype, int64_t nx, int64_t ny, int64_t nz, int64_t v,
                       int64_t* max_out, int64_t* min_out, int64_t* up_steps, int64_t* dn_steps) {
    grid_t g;
    int rc = make_grid(nx, ny, nz, &g);
    if (rc) return rc;
    if (!f || v < 0 || v >= g.n || (dtype != 0 && dtype != 1)) return ORC_E_ARG;
    int64_t nb[14];
    for (int dir = 0; dir < 2; ++dir) {
        int64_t cur = v, steps = 0;
        for (;;) {
            double c = value(f, dtype, cur);
            if (c != c) return ORC_E_NAN;
            int k = neighbours(&g, cur, nb);
            int64_t best = cur;
            for (int i = 0; i < k; ++i) {
                int after = sos_after(f, dtype, nb[i], best);
                if (dir == 0 ? after : !after) best = nb[i];
            }
            if (best == cur) break;
            cur = best;
            ++steps;
        }
        if (dir == 0) {
            if (max_out) *max_out = cur;
            if (up_steps) *up_steps = steps;
        } else {
            if (min_out) *min_out = cur;
            if (dn_steps) *dn_steps = steps;
        }
    }
    return ORC_OK;
}

/*
 * Path compression as the paper states it (Sec. "Ascending and Descending
 * Segmentation", Fig. 2): L0 holds every vertex that is not its own target;
 * each iteration replaces dsc(v) by dsc(dsc(v)) for v in L0, in place, and
 * keeps in L1 the vertices with dsc(v) != dsc(dsc(v)) afterwards; then L0 = L1
 * until it is empty.  Vertices are visited in increasing id order, or in
 * decreasing order when descending != 0.  history (nullable) receives the
 * pointer array after each iteration, at most max_hist of them.  Returns the
 * number of iterations, or a negative status.
 */
int64_t plmss_oracle_compress(int32_t* dsc, int64_t n, int descending, int32_t* history,
                              int64_t max_hist) {
    if (!dsc || n < 1) return ORC_E_ARG;
    for (int64_t v = 0; v < n; ++v)
        if (dsc[v] < 0 || dsc[v] >= n) return ORC_E_ARG;
    int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!list) return ORC_E_NOMEM;
    int64_t len = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = descending ? n - 1 - i : i;
        if (dsc[v] != v) list[len++] = (int32_t)v;
    }
    int64_t iters = 0;
    while (len > 0) {
        int64_t next = 0;
        for (int64_t i = 0; i < len; ++i) {
            int32_t v = list[i];
            dsc[v] = dsc[dsc[v]];
            if (dsc[v] != dsc[dsc[v]]) list[next++] = v; /* still active: kept in order */
        }
        len = next;
        if (history && iters < max_hist) memcpy(history + iters * n, dsc, sizeof(int32_t) * (size_t)n);
        ++iters;
        if (iters > 64 + n) break; /* cannot happen for a forest; guards a malformed input */
    }
    free(list);
    return iters;
}

/* Sum over all vertices of the number of in-grid neighbours (= twice the edge
 * count of the triangulation). */
int64_t plmss_oracle_degree_sum(int64_t nx, int64_t ny, int64_t nz) {
    grid_t g;
    if (nx < 1 || ny < 1 || nz < 1) return ORC_E_DIMS;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.n = nx * ny * nz;
    int64_t nb[14], s = 0;
    for (int64_t v = 0; v < g.n; ++v) s += neighbours(&g, v, nb);
    return s;
}

/* The neighbour ids of one vertex, for tests (nb must hold 14 entries). */
int plmss_oracle_neighbours(int64_t nx, int64_t ny, int64_t nz, int64_t v, int64_t* nb) {
    grid_t g;
    int rc = make_grid(nx, ny, nz, &g);
    if (rc) return rc;
    if (!nb || v < 0 || v >= g.n) return ORC_E_ARG;
    return neighbours(&g, v, nb);
}

/* ---- multi-label marching index (Sec. "Multi-Label Marching
 * Triangles/Tetrahedra") --------------------------------------------------
 *
 * Cells: in 3-D (nx, ny, nz all > 1) the six Kuhn tetrahedra of every cube;
 * in 2-D (nz == 1 and nx, ny > 1) the two triangles of every square; no
 * cells otherwise.  A cell's vertices, in increasing id order, are the cube's
 * low corner, then one, two (and in 3-D three) unit steps along the axes in
 * the order given by the cell's permutation: 3-D permutations (x,y,z),
 * (x,z,y), (y,x,z), (y,z,x), (z,x,y), (z,y,x) are tetrahedra 0..5; 2-D
 * (x,y), (y,x) are triangles 0, 1.  Cell index: ((row * (nx-1)) + x) *
 * cells_per_cube + t, rows being the (y, z) rows of cubes (z-major), or the
 * y rows of squares in 2-D.
 *
 * The local label of a cell's i-th vertex is the index of the first vertex
 * (in that order) that carries the same label: a is always 0, b is 0 or 1,
 * c is 0, 1 or 2, d is 0..3, as in the paper's table of tetrahedron codes.
 * The code is (b << 4) | (c << 2) | d for a tetrahedron and (b << 2) | c for
 * a triangle.
 *
 * Output per cell (mode 0, region separators): the number of separating
 * triangles (3-D) or edges (2-D) of the paper's case figures: by the number
 * of distinct labels at the cell's vertices, 3-D: 1 -> 0, 2 -> 1 when one
 * vertex stands alone and 2 when the labels split two and two, 3 -> 5,
 * 4 -> 12; 2-D: 1 -> 0, 2 -> 1, 3 -> 3.  Mode 1 (region boundaries): one
 * triangle for a tetrahedron with exactly three vertices of one label and one
 * edge for a triangle with exactly two; zero otherwise.
 *
 * row_offsets[r] = number of output primitives of rows before r, and
 * row_offsets[rows] = the total.  codes may be NULL.
 */
int64_t plmss_oracle_marching_rows(int64_t nx, int64_t ny, int64_t nz) {
    if (nx > 1 && ny > 1 && nz > 1) return (ny - 1) * (nz - 1);
    if (nz == 1 && nx > 1 && ny > 1) return ny - 1;
    return 0;
}

static const int PERM3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
static const int PERM2[2][2] = {{0, 1}, {1, 0}};

int plmss_oracle_marching(const int32_t* labels, int64_t nx, int64_t ny, int64_t nz, int mode,
                          uint8_t* codes, int64_t* row_offsets) {
    if (!labels || !row_offsets || nx < 1 || ny < 1 || nz < 1 || (mode != 0 && mode != 1)) return ORC_E_ARG;
    const int64_t rows = plmss_oracle_marching_rows(nx, ny, nz);
    const int three_d = nz > 1;
    const int nv = three_d ? 4 : 3, ncells = three_d ? 6 : 2;
    int64_t total = 0;
    for (int64_t r = 0; r < rows; ++r) {
        row_offsets[r] = total;
        const int64_t y = three_d ? r % (ny - 1) : r, z = three_d ? r / (ny - 1) : 0;
        for (int64_t x = 0; x + 1 < nx; ++x) {
            for (int t = 0; t < ncells; ++t) {
                int32_t lab[4];
                int64_t p[3] = {x, y, z};
                lab[0] = labels[p[0] + nx * (p[1] + ny * p[2])];
                for (int i = 1; i < nv; ++i) {
                    const int axis = three_d ? PERM3[t][i - 1] : PERM2[t][i - 1];
                    p[axis] += 1;
                    lab[i] = labels[p[0] + nx * (p[1] + ny * p[2])];
                }
                int local[4], distinct = 0, size[4] = {0, 0, 0, 0};
                for (int i = 0; i < nv; ++i) {
                    int j = 0;
                    while (lab[j] != lab[i]) ++j;
                    local[i] = j;
                    if (j == i) ++distinct;
                    size[j] += 1;
                }
                int count;
                if (mode == 0) {
                    if (three_d) {
                        if (distinct == 1) count = 0;
                        else if (distinct == 2) {
                            int alone = 0;
                            for (int i = 0; i < 4; ++i) alone |= size[i] == 1;
                            count = alone ? 1 : 2;
                        } else if (distinct == 3) count = 5;
                        else count = 12;
                    } else {
                        count = distinct == 1 ? 0 : distinct == 2 ? 1 : 3;
                    }
                } else {
                    int big = 0;
                    for (int i = 0; i < nv; ++i) big |= size[i] == nv - 1;
                    count = (distinct == 2 && big) ? 1 : 0;
                }
                total += count;
                if (codes) {
                    const int code = three_d ? (local[1] << 4) | (local[2] << 2) | local[3]
                                             : (local[1] << 2) | local[2];
                    codes[(r * (nx - 1) + x) * ncells + t] = (uint8_t)code;
                }
            }
        }
    }
    row_offsets[rows] = total;
    return ORC_OK;
}

/* ---- multi-label marching geometry (Sec. "Multi-Label Marching
 * Triangles/Tetrahedra": the tetrahedron case figure, the triangle case
 * figure, and "Triangulation Options") ---------------------------------------
 *
 * The primitives the index above counts, written out.  Same cells, same cell
 * order (row, then x, then cell), and within a cell the order given below.
 * Points are named by the set S of the cell's vertices they average: one
 * vertex (a grid vertex), two (an edge midpoint), three (a face centre),
 * four (the tetrahedron's centre).  A point's coordinates are exact
 * multiples of 1/12 in grid units (vertex (x, y, z) sits at (x, y, z)); each
 * coordinate is stored as the float nearest to that value (the numerator,
 * an integer, divided by 12 in double precision, then rounded to float; the
 * quotient is either exact or has a repeating binary expansion, so this
 * single float rounding is the correctly rounded value).
 *
 * Cell vertices v0..v3 in path (= increasing id) order, labels L0..L3.
 * Separators, tetrahedra, by how the labels split:
 *   one label: none.
 *   one vertex p apart, the others q < r < s:  (pq, pr, ps).
 *   two and two, {v0, q} and {r, s} (r < s):  (v0r, v0s, qr), (v0s, qr, qs).
 *   three labels, p < q equal, r < s single (face centres T1 = prs,
 *   T2 = qrs):  (T1, T2, pr), (T2, pr, qr), (T1, T2, rs), (T1, T2, ps),
 *   (T2, ps, qs).
 *   four labels: for the faces 012, 013, 023, 123 in turn and each face's
 *   edges ij, ik, jk in turn: (0123, face, edge).
 * Every face of a tetrahedron is then cut as the triangle rule cuts it, so
 * that neighbouring tetrahedra agree on their common face.
 * Separators, triangles (2-D): two labels, p apart, q < r: (pq, pr); three
 * labels: (012, 01), (012, 02), (012, 12).
 * Boundaries: a tetrahedron with exactly three vertices of one label gives
 * the triangle of those three (in vertex order); a triangle with exactly two
 * labels gives the edge of its two equal vertices.
 *
 * sides[2] of a separator: the two labels it separates, the one whose first
 * vertex comes first in the cell.  Of a boundary: the label of the equal
 * vertices, then the other.
 *
 * xyz: 3-D float[T][3][3] (point, axis); 2-D float[T][2][2] (axis x, y).
 * Either output may be NULL.  capacity: primitives that fit in the outputs;
 * more is ORC_E_TOO_LARGE.  Returns the number of primitives, or a negative
 * status.
 */
typedef struct {
    float* xyz;
    int32_t* sides;
    int64_t n, cap;
    int dim, pts;  /* dim 3 / 2; points per primitive 3 / 2 */
    int64_t P[4][3];
    const int32_t* L;
} geo_out;

/* Point = the average of the cell vertices in mask S (bit i = vertex i). */
static void geo_point(const geo_out* o, int S, float* dst) {
    int k = 0;
    int64_t sum[3] = {0, 0, 0};
    for (int i = 0; i < 4; ++i)
        if (S >> i & 1) {
            ++k;
            for (int a = 0; a < 3; ++a) sum[a] += o->P[i][a];
        }
    for (int a = 0; a < o->dim; ++a) dst[a] = (float)((double)(sum[a] * (12 / k)) / 12.0);
}

static int geo_emit(geo_out* o, const int* S, int32_t side0, int32_t side1) {
    if (o->n >= o->cap) return ORC_E_TOO_LARGE;
    if (o->xyz)
        for (int p = 0; p < o->pts; ++p) geo_point(o, S[p], o->xyz + (o->n * o->pts + p) * o->dim);
    if (o->sides) {
        o->sides[2 * o->n] = side0;
        o->sides[2 * o->n + 1] = side1;
    }
    o->n += 1;
    return ORC_OK;
}

#define BIT(i) (1 << (i))

/* The two labels of vertices u and w, the one that first occurs first. */
static void first_order(const int32_t* L, int nv, int u, int w, int32_t* s0, int32_t* s1) {
    int fu = 0, fw = 0;
    while (L[fu] != L[u]) ++fu;
    while (L[fw] != L[w]) ++fw;
    (void)nv;
    *s0 = fu < fw ? L[u] : L[w];
    *s1 = fu < fw ? L[w] : L[u];
}

static int geo_cell(geo_out* o, int nv, int mode) {
    const int32_t* L = o->L;
    int size[4] = {0, 0, 0, 0}, first[4], distinct = 0;
    for (int i = 0; i < nv; ++i) {
        int j = 0;
        while (L[j] != L[i]) ++j;
        first[i] = j;
        size[j] += 1;
        if (j == i) ++distinct;
    }
    int32_t s0, s1;
    int rc = ORC_OK;
    if (mode == 1) { /* boundaries */
        if (distinct != 2) return ORC_OK;
        int lone = -1;
        for (int i = 0; i < nv; ++i)
            if (size[first[i]] == 1) lone = i;
        if (lone < 0) return ORC_OK; /* two and two */
        int S[3], k = 0, kept = -1;
        for (int i = 0; i < nv; ++i)
            if (i != lone) {
                S[k++] = BIT(i);
                if (kept < 0) kept = i;
            }
        return geo_emit(o, S, L[kept], L[lone]);
    }
    if (distinct == 1) return ORC_OK;
    if (nv == 3) { /* triangles */
        if (distinct == 2) {
            int p = 0;
            for (int i = 0; i < 3; ++i)
                if (size[first[i]] == 1) p = i;
            int q = p == 0 ? 1 : 0, r = p == 2 ? 1 : 2;
            int S[2] = {BIT(p) | BIT(q), BIT(p) | BIT(r)};
            first_order(L, nv, p, q, &s0, &s1);
            return geo_emit(o, S, s0, s1);
        }
        const int E[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (int e = 0; e < 3 && rc == ORC_OK; ++e) {
            int S[2] = {7, BIT(E[e][0]) | BIT(E[e][1])};
            first_order(L, nv, E[e][0], E[e][1], &s0, &s1);
            rc = geo_emit(o, S, s0, s1);
        }
        return rc;
    }
    if (distinct == 2) {
        int lone = -1;
        for (int i = 0; i < 4; ++i)
            if (size[first[i]] == 1) lone = i;
        if (lone >= 0) {
            int S[3], k = 0, other = -1;
            for (int i = 0; i < 4; ++i)
                if (i != lone) {
                    S[k++] = BIT(lone) | BIT(i);
                    if (other < 0) other = i;
                }
            first_order(L, 4, lone, other, &s0, &s1);
            return geo_emit(o, S, s0, s1);
        }
        /* two and two: q is v0's partner, r < s the other pair */
        int q = -1, r = -1, s = -1;
        for (int i = 1; i < 4; ++i) {
            if (L[i] == L[0]) q = i;
            else if (r < 0) r = i;
            else s = i;
        }
        first_order(L, 4, 0, r, &s0, &s1);
        int A[3] = {BIT(0) | BIT(r), BIT(0) | BIT(s), BIT(q) | BIT(r)};
        int B[3] = {BIT(0) | BIT(s), BIT(q) | BIT(r), BIT(q) | BIT(s)};
        rc = geo_emit(o, A, s0, s1);
        return rc == ORC_OK ? geo_emit(o, B, s0, s1) : rc;
    }
    if (distinct == 3) {
        int p = -1, q = -1, r = -1, s = -1;
        for (int i = 0; i < 4; ++i) {
            if (size[first[i]] == 2) {
                if (p < 0) p = i;
                else q = i;
            } else if (r < 0) r = i;
            else s = i;
        }
        const int T1 = BIT(p) | BIT(r) | BIT(s), T2 = BIT(q) | BIT(r) | BIT(s);
        const int pr = BIT(p) | BIT(r), qr = BIT(q) | BIT(r), rs = BIT(r) | BIT(s);
        const int ps = BIT(p) | BIT(s), qs = BIT(q) | BIT(s);
        int tri[5][3] = {{T1, T2, pr}, {T2, pr, qr}, {T1, T2, rs}, {T1, T2, ps}, {T2, ps, qs}};
        int sep[5][2] = {{p, r}, {p, r}, {r, s}, {p, s}, {p, s}};
        for (int t = 0; t < 5 && rc == ORC_OK; ++t) {
            first_order(L, 4, sep[t][0], sep[t][1], &s0, &s1);
            rc = geo_emit(o, tri[t], s0, s1);
        }
        return rc;
    }
    /* four labels */
    const int F[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
    for (int f = 0; f < 4 && rc == ORC_OK; ++f) {
        const int face = BIT(F[f][0]) | BIT(F[f][1]) | BIT(F[f][2]);
        const int E[3][2] = {{F[f][0], F[f][1]}, {F[f][0], F[f][2]}, {F[f][1], F[f][2]}};
        for (int e = 0; e < 3 && rc == ORC_OK; ++e) {
            int S[3] = {15, face, BIT(E[e][0]) | BIT(E[e][1])};
            rc = geo_emit(o, S, L[E[e][0]], L[E[e][1]]);
        }
    }
    return rc;
}

int64_t plmss_oracle_marching_geometry(const int32_t* labels, int64_t nx, int64_t ny, int64_t nz, int mode,
                                       float* xyz, int32_t* sides, int64_t capacity) {
    if (!labels || nx < 1 || ny < 1 || nz < 1 || (mode != 0 && mode != 1) || capacity < 0) return ORC_E_ARG;
    const int64_t rows = plmss_oracle_marching_rows(nx, ny, nz);
    const int three_d = nz > 1;
    const int nv = three_d ? 4 : 3, ncells = three_d ? 6 : 2;
    geo_out o;
    o.xyz = xyz;
    o.sides = sides;
    o.n = 0;
    o.cap = capacity;
    o.dim = three_d ? 3 : 2;
    o.pts = three_d ? 3 : 2;
    for (int64_t r = 0; r < rows; ++r) {
        const int64_t y = three_d ? r % (ny - 1) : r, z = three_d ? r / (ny - 1) : 0;
        for (int64_t x = 0; x + 1 < nx; ++x) {
            for (int t = 0; t < ncells; ++t) {
                int32_t lab[4];
                int64_t p[3] = {x, y, z};
                for (int i = 0; i < nv; ++i) {
                    if (i > 0) p[three_d ? PERM3[t][i - 1] : PERM2[t][i - 1]] += 1;
                    for (int a = 0; a < 3; ++a) o.P[i][a] = p[a];
                    lab[i] = labels[p[0] + nx * (p[1] + ny * p[2])];
                }
                o.L = lab;
                const int rc = geo_cell(&o, nv, mode);
                if (rc != ORC_OK) return rc;
            }
        }
    }
    return o.n;
}
