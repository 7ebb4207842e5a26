/*
 * plmss.h -- C ABI of the MI355X (gfx950) piecewise-linear Morse-Smale
 * segmentation library (libplmss.so).
 *
 * Method: Maack, Lukasczyk, Tierny, Hagen, Maciejewski, Garth, "Parallel
 * Computation of Piecewise Linear Morse-Smale Segmentations", arXiv 2303.15491.
 *
 * Problem (paper, Sec. "Input Data" and "Morse-Smale Segmentation"): a scalar
 * field f given on the vertices of a regular grid, which is implicitly cut
 * into simplices (six tetrahedra per cube in 3-D, two triangles per square in
 * 2-D; the cut along the (1,1,1) / (1,1) diagonal).  For every vertex v the
 * library returns
 *   desc[v]  the id of the maximum its steepest ascending integral line ends in,
 *   asc[v]   the id of the minimum its steepest descending integral line ends in,
 *   ms[v]    the id of its Morse-Smale region, i.e. of its (asc, desc) pair,
 *   order[v] (optional) its position in the Simulation-of-Simplicity vertex
 *            order (sorted by value, ties by vertex id; Sec. "Preprocessing").
 *
 * Conventions shared by every call:
 *  - Grid dims (nx, ny, nz), each >= 1; nz == 1 is a 2-D field, ny == nz == 1
 *    a 1-D field.  N = nx*ny*nz must be <= 2^31 - 1.  Vertex id
 *    v = x + nx*(y + ny*z), i.e. a C-contiguous (nz, ny, nx) array.
 *  - Neighbours of a vertex: the offsets (a,b,c) in {0,1}^3 minus (0,0,0),
 *    and their negatives (14 in 3-D, 6 in 2-D, 2 in 1-D), clipped at the
 *    border; no wrap-around.
 *  - Vertex order (Sec. "Preprocessing"): u is above w iff f(u) > f(w), or
 *    f(u) == f(w) and u > w.  IEEE comparison: -0 == +0, subnormals are
 *    ordered exactly, +-inf are allowed.  NaN is an error (f maps into R).
 *  - Labels are field-local int32 vertex ids.  MS ids run 0..K-1 in the
 *    lexicographic order of the (asc, desc) pair.
 *  - Every array argument is DEVICE memory owned by the caller unless stated
 *    otherwise.  No call allocates device memory; scratch space is a
 *    caller-provided workspace of the size the matching *_workspace_bytes call
 *    returns (plmss_segment_static instead uses one fixed library-owned array
 *    per GPU).
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  The return value reports synchronous argument checks and launch
 *    errors only.  Data-dependent errors (NaN) are written on the device to
 *    info[0]; the labels of such a field are unspecified.
 *  - Calls are re-entrant.  Two calls that run concurrently must not share a
 *    workspace.
 */
#ifndef PLMSS_H
#define PLMSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (return values, and info[0] on the device). */
#define PLMSS_OK 0
#define PLMSS_E_ARG (-1)       /* NULL pointer or bad enum value */
#define PLMSS_E_DIMS (-2)      /* a dimension < 1 */
#define PLMSS_E_TOO_LARGE (-3) /* N (or a batch's total) > 2^31 - 1 */
#define PLMSS_E_NAN (-4)       /* the field holds a NaN (device-side) */
#define PLMSS_E_WORKSPACE (-5) /* workspace NULL or smaller than required */
#define PLMSS_E_HIP (-6)       /* a HIP launch or runtime call failed */
#define PLMSS_E_NOCONV (-7)    /* path compression hit its iteration cap (device-side) */
#define PLMSS_E_INTERNAL (-8)  /* an internal invariant failed (device-side; the order field is wrong) */

/* Field element types. */
#define PLMSS_F32 0
#define PLMSS_F64 1

typedef struct {
    int64_t nx, ny, nz;
} plmss_dims;

/* One segmentation request. */
typedef struct {
    const void* field; /* device, dtype[nz][ny][nx] */
    plmss_dims dims;
    int32_t dtype;     /* PLMSS_F32 or PLMSS_F64 */
    int32_t* asc;      /* device int32[N], out */
    int32_t* desc;     /* device int32[N], out */
    int32_t* ms;       /* device int32[N], out */
    int32_t* order;    /* device int32[N], out; NULL = do not build the order field */
    int32_t* info;     /* device int32[4], out, or NULL: {status, #minima, #maxima, K} */
} plmss_job;

/* Human-readable text for a status code (static storage). */
const char* plmss_status_string(int code);

/* Library version and the GPU architecture its kernels were built for. */
const char* plmss_build_info(void);

/*
 * Full segmentation of one field (paper, Sec. "Method"): order field (only if
 * job->order != NULL), steepest neighbours, path compression, MS ids.  The
 * labels never depend on the materialised order field (the vertex order is
 * also compared in place), so with an order field the two may run
 * concurrently (PLMSS_TUNE_ORDER_CONCURRENT); the call's work is complete
 * when `stream` reaches it either way.
 * Workspace: plmss_workspace_bytes(dims, dtype, job->order != NULL) bytes of
 * device memory, 256-byte aligned (twice as much with an order field); its
 * contents on entry do not matter.
 * Returns PLMSS_OK, PLMSS_E_ARG, PLMSS_E_DIMS, PLMSS_E_TOO_LARGE,
 * PLMSS_E_WORKSPACE or PLMSS_E_HIP.
 */
size_t plmss_workspace_bytes(plmss_dims dims, int32_t dtype, int32_t with_order);
int plmss_segment(const plmss_job* job, void* workspace, size_t workspace_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): the same
 * segmentation as plmss_segment, with the same results, but without a
 * workspace argument.  Its scratch space is one library-owned device array of
 * plmss_static_scratch_bytes() bytes per GPU (the workspace of a field of
 * PLMSS_STATIC_MAX_VERTICES vertices with its order field, about 60 MiB),
 * created when the library is first used on that GPU and held until the
 * process ends.  The call itself allocates nothing.  The caller still owns
 * the field and every output (job, as for plmss_segment); the order field is
 * always built on `stream`, before the labels.
 * Every call on one GPU shares that GPU's array: two calls whose work
 * overlaps on the same GPU (other streams, other host threads) race and give
 * undefined results; calls on one stream are ordered and safe.  The array's
 * contents on entry do not matter.
 * Returns PLMSS_OK, PLMSS_E_ARG, PLMSS_E_DIMS, PLMSS_E_TOO_LARGE (also for
 * N > PLMSS_STATIC_MAX_VERTICES) or PLMSS_E_HIP.
 */
#define PLMSS_STATIC_MAX_VERTICES (1 << 21)
size_t plmss_static_scratch_bytes(void);
int plmss_segment_static(const plmss_job* job, void* stream);

/*
 * Step 0 alone -- the order field (paper, Sec. "Preprocessing"): sort the
 * vertices by value with ties broken by vertex id; order[v] = position of v.
 * A stable least-significant-digit radix sort of order-preserving integer
 * keys.  info (nullable) receives {status, 0, 0, 0}.
 */
size_t plmss_order_workspace_bytes(plmss_dims dims, int32_t dtype);
int plmss_order_field(const void* field, plmss_dims dims, int32_t dtype, int32_t* order,
                      int32_t* info, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Step 1 alone -- steepest neighbours (paper, Sec. "Ascending and Descending
 * Segmentation", first step): up[v] = the neighbour above all other
 * neighbours and above v, or v itself if v is a maximum; dn[v] likewise
 * downwards.  If order != NULL it is used as the vertex order (int32[N], a
 * permutation of 0..N-1); otherwise the order is taken from field/dtype with
 * the tie rule above.  info (nullable) receives {status, #minima, #maxima, 0}.
 * Needs no workspace.
 */
int plmss_steepest(const void* field, const int32_t* order, plmss_dims dims, int32_t dtype,
                   int32_t* up, int32_t* dn, int32_t* info, void* stream);

/*
 * Step 2 alone -- path compression (paper, same section, second step):
 * repeats p(v) <- p(p(v)) until p(p(v)) == p(v), in place, on both pointer
 * arrays.  On entry desc = up and asc = dn from step 1 (any forest whose roots
 * point to themselves is accepted); on return desc[v] is the root of v's up
 * chain and asc[v] the root of its dn chain.  n = N.  No workspace.
 */
int plmss_compress(int32_t* desc, int32_t* asc, int64_t n, void* stream);

/*
 * Step 3 alone -- Morse-Smale ids (paper, Sec. "Morse-Smale Segmentation"):
 * ms[v] = rank of (asc[v], desc[v]) among the distinct pairs of the field, in
 * lexicographic order; info (nullable) receives {status, 0, 0, K}.  n = N;
 * labels must lie in [0, n).
 */
size_t plmss_ms_workspace_bytes(int64_t n);
int plmss_ms_ids(const int32_t* asc, const int32_t* desc, int64_t n, int32_t* ms, int32_t* info,
                 void* workspace, size_t workspace_bytes, void* stream);

/*
 * Multi-label marching index (paper, Sec. "Multi-Label Marching
 * Triangles/Tetrahedra", Table of tetrahedron binary codes and the figure of
 * its case triangulations): the first pass of a geometry extraction over a
 * label field (MS, ascending or descending labels).  Nothing is triangulated
 * here; the pass says, for every cell, which labelling case it is in and how
 * many primitives it will emit, and where each row's primitives start.
 *
 * Cells.  3-D grids (nx, ny, nz > 1): the six tetrahedra of every cube along
 * its (1,1,1) diagonal (the triangulation of the neighbour scan); 2-D grids
 * (nz == 1, nx, ny > 1): the two triangles of every square along its (1,1)
 * diagonal; other grids have no cells.  A cell's vertices, in increasing id
 * order, are the cube's low corner (x, y, z) followed by one, two (three) unit
 * steps along the axes in the order of the cell's permutation: tetrahedra
 * 0..5 step (x,y,z), (x,z,y), (y,x,z), (y,z,x), (z,x,y), (z,y,x); triangles
 * 0, 1 step (x,y), (y,x).  Rows of cells are the (y, z) rows of cubes in
 * z-major order ((ny-1)(nz-1) rows of nx-1 cubes) or the y rows of squares
 * (ny-1 rows); plmss_marching_rows returns that number (0 for grids without
 * cells, -1 for invalid dims).
 *
 * codes (device uint8, nullable, 2-byte aligned): byte
 * (row * (nx-1) + x) * C + t, C = 6 (tetrahedra) or 2 (triangles), holds cell
 * t's code: with the local label of a vertex being the index of the first of
 * the cell's vertices that carries its label, code = b << 4 | c << 2 | d for
 * a tetrahedron (a, b, c, d), b << 2 | c for a triangle (a, b, c).
 *
 * mode PLMSS_MARCH_SEPARATORS counts the separating primitives of the case
 * figures: tetrahedra with 1 label 0, with 2 labels 1 (one vertex apart) or 2
 * (two and two), 3 labels 5, 4 labels 12 triangles; triangles with 1, 2, 3
 * labels 0, 1, 3 edges.  PLMSS_MARCH_BOUNDARIES counts one triangle per
 * tetrahedron with exactly three vertices of one label and one edge per
 * triangle with exactly two labels (the boundary surface of the
 * single-label variant).
 *
 * row_offsets (device uint64[rows + 1], out): row_offsets[r] = primitives of
 * rows before r; row_offsets[rows] = the total.
 * labels: device int32[N] in the field's layout (any values).  Workspace:
 * plmss_marching_workspace_bytes(dims) bytes, 256-byte aligned.
 * Returns PLMSS_OK, PLMSS_E_ARG (NULL labels/row_offsets, odd codes address,
 * bad mode), PLMSS_E_DIMS, PLMSS_E_TOO_LARGE, PLMSS_E_WORKSPACE or PLMSS_E_HIP.
 */
#define PLMSS_MARCH_SEPARATORS 0
#define PLMSS_MARCH_BOUNDARIES 1
int64_t plmss_marching_rows(plmss_dims dims);
size_t plmss_marching_workspace_bytes(plmss_dims dims);
int plmss_marching_index(const int32_t* labels, plmss_dims dims, int32_t mode, uint8_t* codes,
                         uint64_t* row_offsets, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Multi-label marching geometry (paper, same section: the tetrahedron and
 * triangle case figures, and "Triangulation Options"): the primitives that
 * plmss_marching_index counts, written at its offsets.  row_offsets is that
 * call's output for the same labels, dims and mode (device, rows + 1
 * entries); primitive j of row r is written at index row_offsets[r] + j.
 *
 * Primitives, per cell in cell order.  Points are named by the set of cell
 * vertices they average (a vertex, an edge midpoint, a face centre, the
 * tetrahedron's centre); cell vertices v0..v3 in path order.
 *   Separators, tetrahedra: one vertex p apart, others q < r < s:
 *   (pq, pr, ps); two and two {v0, q}, {r, s}: (v0r, v0s, qr),
 *   (v0s, qr, qs); three labels, p < q equal, r < s single, T1 = prs,
 *   T2 = qrs: (T1, T2, pr), (T2, pr, qr), (T1, T2, rs), (T1, T2, ps),
 *   (T2, ps, qs); four labels: for faces 012, 013, 023, 123 and each face's
 *   edges in order, (v0v1v2v3, face, edge).  Triangles (2-D): p apart,
 *   q < r: (pq, pr); three labels: (012, 01), (012, 02), (012, 12).
 *   Every tetrahedron face is thus cut as the triangle rule cuts a triangle,
 *   so that neighbouring tetrahedra agree.
 *   Boundaries: the triangle of the three equal vertices of a tetrahedron
 *   with one vertex apart; the edge of the two equal vertices of a triangle
 *   with two labels.
 *
 * xyz (device float, nullable, 4-byte aligned): 3-D float[capacity][3][3]
 * (point, axis x y z), 2-D float[capacity][2][2], in grid units (vertex
 * (x, y, z) at (x, y, z)).  Coordinates are multiples of 1/12; each is the
 * float nearest to its exact value.  sides (device int32, nullable, 8-byte
 * aligned): int32[capacity][2], the two labels a separator separates, in the
 * order of their first vertex in the cell; for a boundary, the label of the
 * equal vertices, then the other.  Primitives at indices >= capacity are not
 * written (capacity = row_offsets[rows] writes all).  No workspace.
 * Returns PLMSS_OK, PLMSS_E_ARG (NULL labels/row_offsets, bad mode,
 * misaligned outputs), PLMSS_E_DIMS, PLMSS_E_TOO_LARGE or PLMSS_E_HIP.
 */
int plmss_marching_geometry(const int32_t* labels, plmss_dims dims, int32_t mode, const uint64_t* row_offsets,
                            uint64_t capacity, float* xyz, int32_t* sides, void* stream);

/*
 * Many fields of different sizes in one pass: the same results as calling
 * plmss_segment on each job, computed by one launch per step over all fields
 * together.  jobs is a HOST array of n_jobs entries; the sum of their N must
 * be <= 2^31 - 1.  Jobs with a non-NULL order get their order field (paper,
 * Sec. "Preprocessing"): when any job asks for one, all the batch's vertices
 * are sorted together by (job index, value, vertex id), so that each field's
 * vertices fill one run of positions and each order field is its positions
 * within that run.  One field's NaN only sets that job's info[0].  Asynchronous like
 * every call: the descriptor table goes to the device through a page-locked
 * staging buffer the library keeps (reused once its copy has completed), so
 * the host neither waits for the batch nor needs to keep `jobs` alive.
 * Workspace: plmss_batch_workspace_bytes(n_jobs, jobs) bytes.
 */
size_t plmss_batch_workspace_bytes(int32_t n_jobs, const plmss_job* jobs);
int plmss_segment_batch(int32_t n_jobs, const plmss_job* jobs, void* workspace,
                        size_t workspace_bytes, void* stream);

/*
 * What a batch needs from a plan: needs[0] = total vertices, needs[1] = fields,
 * needs[2] = neighbour-scan tiles, needs[3] = chase tiles (host array of 4).
 * Returns a status.
 */
int32_t plmss_batch_needs(int32_t n_jobs, const plmss_job* jobs, int64_t* needs);

/*
 * Capacity plans: the batched segmentation with every launch sized for a
 * capacity and every total read on the device, so that one hipGraph captures
 * it once and replays it for any batch within the capacity (continuous
 * batching, serving).  Same results as plmss_segment per job.
 *   plmss_plan_create   capacity (all > 0), element type, and with_order (0 or
 *                       1): whether the plan builds the order fields its jobs
 *                       ask for (the graph then holds the order sort, run for
 *                       every batch); NULL on failure.
 *   plmss_plan_workspace_bytes  device workspace the plan's calls need.
 *   plmss_plan_set      writes the batch's descriptor tables and totals into
 *                       the workspace (asynchronous copies on `stream`, staged
 *                       through page-locked host buffers the library keeps;
 *                       the call does not wait for the device).
 *                       PLMSS_E_TOO_LARGE beyond the capacity; PLMSS_E_ARG for
 *                       a job with an order field on a plan created without.
 *   plmss_plan_launch   enqueues the kernels on `stream` (capturable).
 *   plmss_plan_launch_graph  the same through a hipGraph, captured on the
 *                       first call (and again when the workspace changes).
 * A plan is a host object; its calls must not run concurrently.
 */
typedef struct plmss_plan plmss_plan;
plmss_plan* plmss_plan_create(int64_t max_vertices, int32_t max_fields, int64_t max_scan_tiles,
                              int64_t max_chase_tiles, int32_t dtype, int32_t with_order);
void plmss_plan_destroy(plmss_plan* plan);
size_t plmss_plan_workspace_bytes(const plmss_plan* plan);
int plmss_plan_set(plmss_plan* plan, int32_t n_jobs, const plmss_job* jobs, void* workspace,
                   size_t workspace_bytes, void* stream);
int plmss_plan_launch(plmss_plan* plan, void* workspace, size_t workspace_bytes, void* stream);
int plmss_plan_launch_graph(plmss_plan* plan, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Launch tracing, for measurement.  While a trace is active on the calling
 * host thread (between plmss_trace_begin and plmss_trace_end), every kernel
 * launch made by the calls above is bracketed by two hipEvents recorded on the
 * launch's own stream; the work done is unchanged.  plmss_trace_read waits for
 * the recorded events and returns, per launch, its kernel kind and its
 * duration in milliseconds.  A trace records at most max_launches launches;
 * later ones run untraced.  Handles are host objects; create returns NULL on
 * failure; the other calls return PLMSS_OK, PLMSS_E_ARG or PLMSS_E_HIP
 * (read returns the number of launches copied, or a negative status).
 */
#define PLMSS_KERNEL_MISC 0          /* small setup / bookkeeping kernels */
#define PLMSS_KERNEL_RADIX_HIST 1    /* radix sort: per-worker digit counts */
#define PLMSS_KERNEL_RADIX_SCAN 2    /* radix sort: digit offsets */
#define PLMSS_KERNEL_RADIX_SCATTER 3 /* radix sort: stable scatter (order field, pair sort) */
#define PLMSS_KERNEL_STEEPEST 4      /* steepest neighbours */
#define PLMSS_KERNEL_JUMP 5          /* path compression (+ MS pair listing) */
#define PLMSS_KERNEL_PREFIX 6        /* prefix sums */
#define PLMSS_KERNEL_COMPACT 7       /* no longer launched (pairs are listed by the chase); the number stays reserved */
#define PLMSS_KERNEL_RANK 8          /* MS pair ranking */
#define PLMSS_KERNEL_MS_FINAL 9      /* MS id write-back */
#define PLMSS_KERNEL_ORDER_HIST 10   /* order field: per-worker digit counts */
#define PLMSS_KERNEL_ORDER_SCATTER 11 /* order field: middle passes, (key, id) to (key, id) */
#define PLMSS_KERNEL_ORDER_INVERT 12 /* order field: order[id] = position */
#define PLMSS_KERNEL_ORDER_FIRST 13  /* order field: first pass, field to (key, id) */
#define PLMSS_KERNEL_ORDER_LAST 14   /* order field: last pass (sorted ids, or (id, position) by range) */
#define PLMSS_KERNEL_ORDER_REGROUP 15 /* order field: (id, position) regrouped by id chunk */
#define PLMSS_KERNEL_MARCH 16      /* marching index: cell codes and row counts */
#define PLMSS_KERNEL_MARCH_GEOMETRY 17 /* marching geometry: primitives written out */
#define PLMSS_KERNEL_KINDS 18

typedef struct plmss_trace plmss_trace;
plmss_trace* plmss_trace_create(int32_t max_launches);
void plmss_trace_destroy(plmss_trace* trace);
int plmss_trace_begin(plmss_trace* trace);
int plmss_trace_end(plmss_trace* trace);
int32_t plmss_trace_read(plmss_trace* trace, int32_t* kinds, float* ms, int32_t max);
const char* plmss_kernel_name(int32_t kind);

/*
 * Launch-shape knobs, for the autotuner.  Process-wide; a call reads them when
 * it enqueues its kernels (a plan's hipGraph keeps the values it was captured
 * with).  Results never depend on them, only speed does.
 *   PLMSS_TUNE_ORDER_WORKERS   blocks of each order-field radix pass: 0
 *                              (default) = one per 4096-key tile, or
 *                              64..65536, each block then owning a contiguous
 *                              run of tiles.
 *   PLMSS_TUNE_ORDER_INVERT    how order[id] = position is written: 0 = by the
 *                              last radix pass itself (scattered writes over
 *                              the whole array); 1 (default) = the last pass
 *                              groups (id, position) pairs by id range, a
 *                              second launch regroups them by chunks of 32768
 *                              ids and a third inverts each chunk in LDS and
 *                              writes it as one coalesced run; w in
 *                              2..64 = the last pass writes the sorted ids and
 *                              w launches invert them, each for 1/w of the id
 *                              range.
 *   PLMSS_TUNE_ORDER_PACKED    1 (default) = 32-bit keys travel packed with
 *                              their ids in one 64-bit word (split into two
 *                              arrays for the last pass unless the inversion
 *                              is by id chunks); 64-bit keys travel as a key
 *                              array and an id array for their low four
 *                              digits, then as their high half packed with
 *                              the id; 0 = two arrays throughout.
 *   PLMSS_TUNE_ORDER_CONCURRENT  plmss_segment with an order field: 1 = the
 *                              order field is built on a
 *                              library-owned stream (one per device,
 *                              non-blocking, default priority, kept for the
 *                              life of the process) that waits for the
 *                              caller's stream, while the labels run on the
 *                              caller's stream, which then waits for the order
 *                              field; 0 (default) = everything on the caller's
 *                              stream, so that each kernel's time is its own.
 *   PLMSS_TUNE_PACKED_CODES    neighbour scan over an order field of fewer
 *                              than 2^28 vertices: 1 (default) = each rank
 *                              shares one 32-bit word with a neighbour code
 *                              and candidates are compared by plain max/min;
 *                              0 = ranks and codes apart (the form used above
 *                              that size).
 *   PLMSS_TUNE_PAIR_STREAM     loads of the MS pair sort: 0 = cached, 1 =
 *                              non-temporal (streamed past the caches), 2
 *                              (default) = streamed for batches and plans,
 *                              whose pair lists are long, and cached for a
 *                              single field, whose list usually stays in
 *                              the memory-side cache between passes.
 *   PLMSS_TUNE_SCAN_ROUNDS     in-tile path-compression sweeps of the
 *                              neighbour scan (1..8, default 3); what they
 *                              leave unfinished the cross-tile chase follows.
 *   PLMSS_TUNE_SORT_WORKERS    blocks of device-sized sorts and scans (the MS
 *                              pair sort): 64..4096, default 512.
 *   PLMSS_TUNE_PERSIST_BLOCKS  grid of a plan's persistent launches:
 *                              64..16384, default 2048.
 *   PLMSS_TUNE_SCAN_DEPTH      z-planes of a 3-D neighbour-scan tile (each
 *                              block marches through that many planes of a
 *                              64x8 column and compresses the paths inside
 *                              it): 8, 16 (default) or 32.  A plan keeps the
 *                              depth it was created with; plmss_batch_needs
 *                              counts tiles with the current depth.
 * plmss_tune_set returns PLMSS_OK, or PLMSS_E_ARG for an unknown knob or a
 * value out of range (the knob is then unchanged).  plmss_tune_get returns the
 * current value, or -1 for an unknown knob.
 */
#define PLMSS_TUNE_ORDER_WORKERS 0
#define PLMSS_TUNE_ORDER_INVERT 1
#define PLMSS_TUNE_SORT_WORKERS 2
#define PLMSS_TUNE_PERSIST_BLOCKS 3
#define PLMSS_TUNE_SCAN_DEPTH 4
#define PLMSS_TUNE_ORDER_PACKED 5
#define PLMSS_TUNE_SCAN_ROUNDS 6
#define PLMSS_TUNE_ORDER_CONCURRENT 7
#define PLMSS_TUNE_PACKED_CODES 8
#define PLMSS_TUNE_PAIR_STREAM 9
#define PLMSS_TUNE_KNOBS 10
int32_t plmss_tune_set(int32_t knob, int64_t value);
int64_t plmss_tune_get(int32_t knob);

#ifdef __cplusplus
}
#endif

#endif /* PLMSS_H */
