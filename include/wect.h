/*
 * wect.h -- C ABI of the MI355X (gfx950) weighted Euler characteristic
 * transform library (libwect.so).
 *
 * What is computed (paper: "Tensor Computation of Euler Characteristic
 * Functions and Transforms"):
 *
 *   out[b][p][q] = sum over cells c of complex b with  f_p^max(c) <= thr[q]
 *                  of (-1)^dim(c) * w(c)
 *
 * i.e. the weighted Euler characteristic (Definition "Weighted Euler
 * Characteristic") of the lower-star filtration (Definition "Lower-Star
 * Filtrations", test <=) of the height function h_p(v) = l(v) . s_p
 * (Definition "Vertex Height Functions and Directional Filtrations"),
 * sampled at the stored thresholds: the WECT of Definition "Weighted Euler
 * Characteristic Transform", computed as in Algorithm 1 / Example "WECT as a
 * special case" (filter values = coordinates times directions).
 *
 * Numerics fixed by this library:
 *   - heights are float32, round to nearest even, no fused multiply-add,
 *     evaluated as ((x*sx) + (y*sy)) + (z*sz);
 *   - a cell's value is the maximum of its vertices' heights and it enters at
 *     the first stored threshold at or above that value; a value above
 *     thr[T-1] enters at no threshold;
 *   - integer weights accumulate in int32 with wrap-around (exact whenever
 *     every result fits in int32); float32 weights are rounded once each to a
 *     64-bit fixed-point grid 2^-e (e chosen from the largest |w| and the
 *     cell count so that no sum overflows) and summed exactly, so float32
 *     results do not depend on the launch shape or the order of the work;
 *   - any number of thresholds: a histogram of all T thresholds is kept in
 *     LDS when it fits, otherwise the thresholds are processed in tiles of
 *     consecutive entries, one launch each (out[b][p][q] depends on thr[q]
 *     alone, so the tiles are exact and independent).
 *
 * Memory: every data pointer is a DEVICE pointer owned by the caller; the
 * library keeps no pointer after a call returns.  Sizes and counts in the
 * structs are HOST values.  All arrays are dense, row-major, naturally
 * aligned.
 *
 * Asynchrony: wect_forward / wect_backward / wect_batched only check the
 * host-side metadata, then enqueue kernels on `hip_stream` (a hipStream_t,
 * NULL = the null stream) and return.  They never allocate, synchronise or
 * read device memory, so they may be captured into a HIP graph.  Data
 * errors (vertex ids out of range, unsorted thresholds, NaN) are detected
 * only by wect_validate.  On any error status nothing is enqueued and the
 * outputs are untouched.  Outputs are overwritten, never accumulated.
 *
 * Thread safety: the entry points may be called concurrently from several
 * host threads on different streams with different workspaces.
 */
#ifndef WECT_H
#define WECT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WECT_OK = 0,
  WECT_ERR_ARG = 1,          /* invalid metadata: null pointer, bad size, bad enum value */
  WECT_ERR_INDEX = 2,        /* wect_validate: vertex id out of range, or inconsistent offsets/shapes */
  WECT_ERR_THRESHOLDS = 3,   /* wect_validate: thresholds not non-decreasing, or an axis not strictly increasing */
  WECT_ERR_NONFINITE = 4,    /* wect_validate: NaN or Inf in coordinates, directions, thresholds or weights */
  WECT_ERR_WORKSPACE = 5,    /* workspace pointer missing or smaller than wect_workspace_bytes() */
  WECT_ERR_UNSUPPORTED = 6,  /* valid request outside what the kernels implement (e.g. explicit
                                weights on a cubical complex) */
  WECT_ERR_DEVICE = 7        /* a HIP runtime call failed (no device, launch failure, ...) */
} wect_status;

typedef enum {
  WECT_W_ONES = 0,        /* w(c) = 1 for every cell: the Euler characteristic transform */
  WECT_W_EXPLICIT = 1,    /* simplicial: one weight per simplex, weights[i] has count[i] entries */
  WECT_W_VERTEX_MAX = 2   /* w(c) = max of its vertices' weights (caption of Figure 1);
                             simplicial: weights[0] = float32 [count[0]] vertex weights;
                             cubical: the vertex weight is the voxel intensity */
} wect_wmode;

typedef enum { WECT_I32 = 0, WECT_F32 = 1 } wect_dtype;   /* dtype of the weights == dtype of out */
typedef enum { WECT_SIMPLICIAL = 0, WECT_CUBICAL = 1 } wect_kind;

/*
 * One complex (B == 1) or a batch of B complexes stored back to back with
 * CSR offsets (the paper's input structure "Complex", Section "Computation of
 * WECFs": vertex filter data and weights, then per dimension i a list of
 * i-simplices as rows of i+1 vertex ids and their weights).
 */
typedef struct {
  int32_t kind;     /* wect_kind */
  int32_t n;        /* ambient dimension: simplicial 1..3, cubical 2 or 3 */
  int32_t B;        /* number of complexes, >= 1 */
  int32_t top_dim;  /* simplicial: highest dimension present, 0..3 */
  int32_t wmode;    /* wect_wmode */
  int32_t dtype;    /* wect_dtype; WECT_F32 requires wmode EXPLICIT or VERTEX_MAX (simplicial) */

  /* ---- simplicial ---- */
  const float* coords;              /* [count[0], n] vertex coordinates l(v) */
  const int64_t* vert_off;          /* [B+1] vertex offsets (vert_off[0] = 0); NULL allowed iff B == 1 */
  int64_t count[4];                 /* totals over the batch: vertices, edges, triangles, tetrahedra;
                                       count[i] = 0 for i > top_dim */
  const int32_t* simplices[4];      /* simplices[i]: [count[i], i+1] vertex ids, numbered locally
                                       within their complex (0 .. V_b-1); simplices[0] unused */
  const int64_t* simp_off[4];       /* simp_off[i]: [B+1] offsets of complex b's i-simplices;
                                       NULL allowed iff B == 1; simp_off[0] unused (vert_off) */
  const void* weights[4];           /* EXPLICIT: weights[i] = [count[i]] of dtype (weights[0] = vertices);
                                       VERTEX_MAX: weights[0] = float32 [count[0]]; ONES: unused */

  /* ---- cubical (implicit grid; vertex = voxel with intensity > include_above,
          every axis-aligned edge/square/cube whose corners are all vertices is
          a cell, sign (-1)^dim; VERTEX_MAX weight = max corner intensity) ---- */
  const int32_t* shape;             /* [B, 3] extents (n0, n1, n2) with axis 0 fastest; n2 = 1 when n == 2;
                                       n0*n1*n2 < 2^31 per complex */
  const int64_t* grid_off;          /* [B+1] voxel offsets into `intensity`; NULL allowed iff B == 1 */
  const uint8_t* intensity;         /* all voxels, complex after complex, axis 0 fastest */
  const float* axis;                /* per complex n0 (+ n1 (+ n2)) coordinates: axis 0, then 1, then 2,
                                       each strictly increasing */
  const int64_t* axis_off;          /* [B+1] offsets into `axis`; NULL allowed iff B == 1 */
  int64_t total_voxels;             /* sum of n0*n1*n2 over the batch */
  int32_t include_above;            /* voxel is a vertex iff intensity > include_above (-1: all) */
  int32_t reserved;
} wect_complex;

/* Sampling grid of the transform: d directions s_p (rows, used as stored,
 * not renormalised) and T thresholds thr[0] <= ... <= thr[T-1]. */
typedef struct {
  const float* dirs;   /* [d, n] */
  int32_t d;
  int32_t T;
  const float* thr;    /* [T] */
} wect_grid;

/*
 * Size in bytes of the device workspace that wect_forward (with_backward = 0),
 * wect_backward or wect_batched (with_backward = 1) need for this request on
 * the current device.  Returns 0 when the request is invalid (the call itself
 * would then return its error status) or when no workspace is needed.
 */
size_t wect_workspace_bytes(const wect_complex* c, const wect_grid* g, int with_backward);

/*
 * Forward transform (Algorithm 1 specialised to height filters, Example
 * "WECT as a special case").
 *   out: [B, d, T] int32 (dtype I32) or float32 (dtype F32), overwritten.
 *   ws:  device workspace of at least wect_workspace_bytes(c, g, 0) bytes.
 * Errors: WECT_ERR_ARG (metadata), WECT_ERR_WORKSPACE, WECT_ERR_UNSUPPORTED,
 * WECT_ERR_DEVICE (launch failed).
 */
wect_status wect_forward(const wect_complex* c, const wect_grid* g, void* out,
                         void* ws, size_t ws_bytes, void* hip_stream);

/*
 * wect_forward without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * wect_forward with ws / ws_bytes dropped: the workspace is a static device
 * array of 64 MiB inside the library, one per device, held by each device the
 * library runs on until the process ends.  It is planned without the cubical
 * forward's per-voxel records (wect_launch.cubical_records), so it needs only
 * the partial histograms.  A request whose workspace exceeds 64 MiB returns WECT_ERR_WORKSPACE
 * (wect_last_error() gives the sizes) and enqueues nothing.  The call itself
 * allocates nothing (no hipMalloc, no library allocation); the first call on
 * a device looks up that device's array address.  Calls that overlap on one
 * device (concurrent streams or threads) share the array and race: serialise
 * them.  Nothing in the array needs clearing between calls.
 */
wect_status wect_forward_noalloc(const wect_complex* c, const wect_grid* g, void* out, void* hip_stream);

/*
 * Adjoint of the forward with respect to the weights (simplicial, float32
 * weights).  The forward is linear in the cell weights, so for
 * L = sum_{b,p,q} grad_out[b][p][q] * out[b][p][q]:
 *   dL/dw(c) = (-1)^dim(c) * sum_p sum_{q : f_p^max(c) <= thr[q]} grad_out[b][p][q]
 * (a reverse scan of grad_out along the thresholds, read at each cell's
 * threshold index).  The paper lists differentiable transforms as future work
 * (Section "Discussion"); this is the derivative of its Algorithm 1 output.
 *   grad_out:    [B, d, T] float32.
 *   grad_w:      EXPLICIT: array of 4 pointers, grad_w[i] = [count[i]] float32 or NULL (skipped).
 *   grad_vertex: VERTEX_MAX: [count[0]] float32; each cell's gradient goes to the
 *                lowest-numbered vertex attaining the maximum vertex weight.
 * Gradients with respect to coordinates, directions and thresholds are zero
 * almost everywhere (the output is piecewise constant in them) and are not
 * produced.  Outputs are overwritten.  Float32 accumulation order is not fixed.
 */
wect_status wect_backward(const wect_complex* c, const wect_grid* g, const float* grad_out,
                          float* const grad_w[4], float* grad_vertex,
                          void* ws, size_t ws_bytes, void* hip_stream);

/*
 * Forward and, when grad_out != NULL, backward for a batch of complexes of
 * uneven size, each a single persistent launch over the whole batch; the call
 * sequence is capture-safe, so the pair can be replayed from one HIP graph.
 * Same arguments as wect_forward / wect_backward; ws must hold
 * wect_workspace_bytes(c, g, grad_out != NULL) bytes.
 */
wect_status wect_batched(const wect_complex* c, const wect_grid* g, void* out,
                         const float* grad_out, float* const grad_w[4], float* grad_vertex,
                         void* ws, size_t ws_bytes, void* hip_stream);

/*
 * WECF of general vertex filters on simplicial complexes (Section "Computation
 * of WECFs": Algorithm 1 takes m filter values per vertex and returns the
 * (m, T) tensor; the WECT is the case fvals = V D^T):
 *   out[b][p][q] = sum over simplices s of complex b with
 *                  max_{v in s} fvals[v][p] <= thr[q] of (-1)^dim(s) * w(s).
 * c:     as for wect_forward with kind SIMPLICIAL (weights ONES / EXPLICIT /
 *        VERTEX_MAX, CSR batch when B > 1); n and coords are not read.
 * fvals: [sum V, m] float32 device array, row-major (row = vertex in batch
 *        order, finite values).
 * thr, T: as in wect_grid (non-decreasing, finite).
 * out:   [B, m, T] int32 (integer weights) or float32 (float weights).
 * ws:    wect_wecf_workspace_bytes(c, m, T) bytes.  Work is split like
 *        wect_forward with the m columns in place of the d directions, 64 per
 *        wavefront (m below 64 leaves lanes idle).  Errors, asynchrony and
 *        capture safety as for wect_forward; the adjoint is wect_wecf_backward.
 */
size_t wect_wecf_workspace_bytes(const wect_complex* c, int32_t m, int32_t T);
wect_status wect_wecf_forward(const wect_complex* c, const float* fvals, int32_t m, const float* thr, int32_t T,
                              void* out, void* ws, size_t ws_bytes, void* hip_stream);

/*
 * Adjoint of wect_wecf_forward with respect to the weights (float32 weights,
 * EXPLICIT or VERTEX_MAX), as wect_backward with the filter values in place of
 * the heights:
 *   dL/dw(s) = (-1)^dim(s) sum_p sum_{q : max_{v in s} fvals[v][p] <= thr[q]} grad_out[b][p][q].
 * Gradients with respect to the filter values are zero almost everywhere and
 * are not produced.  grad_out [B, m, T] float32; grad_w / grad_vertex as for
 * wect_backward.  ws: at least wect_wecf_workspace_bytes(c, m, T) bytes (the
 * threshold index of every filter value is formed there first).  Asynchronous
 * and capture-safe; outputs overwritten.
 */
wect_status wect_wecf_backward(const wect_complex* c, const float* fvals, int32_t m, const float* thr, int32_t T,
                               const float* grad_out, float* const grad_w[4], float* grad_vertex, void* ws,
                               size_t ws_bytes, void* hip_stream);

/*
 * Weighted Freudenthal complexes of images, built on the device (images become
 * weighted simplicial complexes through the Freudenthal triangulation with
 * weights from the pixel intensities: the paper's Background section, after
 * the definition of weighted simplicial complexes).
 *
 * Pixel (i0, i1) of an n0 x n1 image is vertex i1 n0 + i0, at (axis0[i0],
 * axis1[i1]), with weight = its intensity (use wmode VERTEX_MAX: a simplex
 * weighs the largest intensity of its vertices).  Edges: the (n0-1) n1
 * horizontal ones (row-major), the n0 (n1-1) vertical ones, then the
 * (n0-1)(n1-1) diagonals (i0,i1)-(i0+1,i1+1).  Triangles: every
 * {(i0,i1), (i0+1,i1), (i0+1,i1+1)}, then every {(i0,i1), (i0,i1+1), (i0+1,i1+1)}.
 * Every pixel is a vertex (include_above is not read).
 *
 * wect_freudenthal_counts: host shapes [B][3] (n0, n1, 1, as in
 *   wect_complex.shape) -> total vertices, edges and triangles (host).
 * wect_freudenthal_build: c is a 2D cubical batch (shape, grid_off, intensity,
 *   axis, axis_off as for wect_forward); outputs are device arrays sized by the
 *   counts: coords [V,2] f32, vweights [V] f32, edges [E,2] and tris [F,3]
 *   int32 (vertex ids local to their image), and the CSR offsets vert_off,
 *   edge_off, tri_off [B+1] int64, ready for a wect_complex with top_dim 2.
 *   Asynchronous and capture-safe (two kernels, no allocation).
 */
wect_status wect_freudenthal_counts(int32_t B, const int32_t* shape_host, int64_t counts[3]);
wect_status wect_freudenthal_build(const wect_complex* c, float* coords, float* vweights, int32_t* edges,
                                   int32_t* tris, int64_t* vert_off, int64_t* edge_off, int64_t* tri_off,
                                   void* hip_stream);

/*
 * ECF of images and volumes with the intensity as the vertex filter: the first
 * of the two ECFs of an image in the paper's Remark on them, i.e. the WECF of
 * Section "Computation of WECFs" for one vertex filter, f(v) = intensity(v).
 *
 * c: kind CUBICAL, n = 2 or 3, dtype I32, B >= 1 images with shape [B,3] and
 *    (B > 1) grid_off [B+1]; axis and axis_off are not read.  A pixel/voxel is
 *    a vertex iff intensity > include_above (-1: all); the edges, squares and
 *    cubes whose corners are all vertices are the other cells, as for
 *    wect_forward.  A cell enters the filtration at the largest intensity of
 *    its corners.  Weight: 1 (wmode ONES: the ECF) or that largest intensity
 *    (wmode VERTEX_MAX: a WECF); EXPLICIT is WECT_ERR_UNSUPPORTED.
 * thr: [T] float32 device array, any order (each entry is read on its own; a
 *    NaN entry admits no cell).
 * out: [B, T] int32 device array (row b = image b), overwritten:
 *    out[b][q] = sum of (-1)^dim * weight over the cells of image b whose
 *    value is <= thr[q].  Integer sums wrap modulo 2^32 like int32.
 * ws:  wect_image_ecf_workspace_bytes(c) bytes of device memory (256-byte
 *    aligned, contents ignored): one 256-entry accumulator per image, so it
 *    does not depend on T.
 * Metadata errors return before anything is enqueued; data errors (shapes
 * inconsistent with grid_off or total_voxels) are reported by wect_validate
 * (with a grid of d = 0 directions).  Asynchronous on hip_stream and
 * capture-safe: three kernel launches (clear, histogram, read-out), no
 * allocation, no memset, no synchronisation.
 */
size_t wect_image_ecf_workspace_bytes(const wect_complex* c);
wect_status wect_image_ecf(const wect_complex* c, const float* thr, int32_t T, int32_t* out,
                           void* ws, size_t ws_bytes, void* hip_stream);

/*
 * Sigmoid relaxation of the WECT (simplicial complexes), a differentiable form
 * of the transform (the paper names differentiable transforms as future work,
 * Section "Discussion", and cites the differentiable ECT among related
 * software, Section "Related Work"):
 *
 *   S[b][p][q] = sum over simplices c of complex b of
 *                (-1)^dim(c) w(c) sig(lam (thr[q] - f_p^max(c))),
 *   sig(x) = 1 / (1 + exp(-x)),
 *
 * with f_p^max(c) the float32 maximum vertex height of c as in wect_forward.
 * lam >= 0 is the sharpness (finite): as lam grows S tends to the WECT away
 * from the cell values; lam = 0 gives half the weighted Euler characteristic.
 *
 * Numerics: a term with |lam (thr[q] - f)| above 17 is taken as 0 or w (error
 * below exp(-17) |w| < 2^-24 |w|); inside that window sig is evaluated in
 * float32 (hardware exp2 and reciprocal), each term w sig is rounded to a
 * fixed-point grid of 2^-e with |w| 2^e < 2^30, and the terms are summed
 * exactly in 64-bit integers, so the output does not depend on the order of
 * the work and differs from the exact value by about 30 ulp of |w| per cell.
 *
 * c:    kind SIMPLICIAL, weights ONES, EXPLICIT float32 or VERTEX_MAX (EXPLICIT
 *       int32 is WECT_ERR_UNSUPPORTED; cubical complexes likewise).
 * g:    directions and thresholds as for wect_forward (thresholds non-decreasing).
 * out:  [B, d, T] float32, overwritten.
 * ws:   wect_smooth_workspace_bytes(c, g, lam) bytes (0 possible).
 * Cost: about 34 / (lam * threshold spacing) sigmoid terms per cell and
 * direction, plus the WECT's own work.
 */
size_t wect_smooth_workspace_bytes(const wect_complex* c, const wect_grid* g, float lam);
wect_status wect_smooth_forward(const wect_complex* c, const wect_grid* g, float lam, float* out,
                                void* ws, size_t ws_bytes, void* hip_stream);

/*
 * Adjoint of wect_smooth_forward for L = sum grad_out[b][p][q] S[b][p][q]:
 *   dL/dw(c)       = (-1)^dim(c) sum_{p,q} grad_out[p][q] sig_pq(c),
 *   dL/df_p^max(c) = -(-1)^dim(c) w(c) lam sum_q grad_out[p][q] sig_pq(c) (1 - sig_pq(c)),
 * and f_p^max(c) = <l(a), s_p> for the vertex a of c attaining the maximum
 * height (the lowest vertex id among equal heights), so that the coordinates
 * of a receive dL/df s_p and the direction s_p receives dL/df l(a).
 *   grad_out:    [B, d, T] float32.
 *   grad_coords: [count[0], n] float32 or NULL (not computed).
 *   grad_dirs:   [d, n] float32 or NULL; sums over the whole batch.
 *   grad_w:      EXPLICIT: 4 pointers, grad_w[i] = [count[i]] float32 or NULL.
 *   grad_vertex: VERTEX_MAX: [count[0]] float32 or NULL; each simplex's weight
 *                gradient goes to the lowest-numbered vertex of maximum weight.
 * Window as in the forward.  Outputs are overwritten (cleared by kernels,
 * then accumulated with float32 atomics: the order of the additions is not
 * fixed).  No workspace.  Asynchronous and capture-safe.
 */
wect_status wect_smooth_backward(const wect_complex* c, const wect_grid* g, float lam, const float* grad_out,
                                 float* grad_coords, float* grad_dirs, float* const grad_w[4],
                                 float* grad_vertex, void* hip_stream);

/*
 * Lower-star index of a simplicial complex (or CSR batch): for every vertex,
 * the simplices of dimension >= 1 that contain it.  Every cell has, for each
 * direction, one vertex attaining its maximum height (lowest id among equal
 * heights), and the cells a vertex tops form its lower star (Definition
 * "Lower-Star Filtrations"); with the index, the relaxation combines those
 * cells' weights per vertex and direction and evaluates one sigmoid window per
 * vertex instead of one per cell (wect_smooth_ls_forward / _backward).
 *
 * wect_lower_star_bytes: size of the index for the complex's counts (0 on
 *   invalid metadata).  It depends only on the counts.
 * wect_lower_star_build: writes the index into `index` (device memory, at
 *   least wect_lower_star_bytes(c) bytes, 16-byte aligned, owned by the
 *   caller).  Reads the simplex lists and offsets only, so one build serves
 *   every call with the same topology (coordinates and weights may change).
 *   Asynchronous and capture-safe, no allocation: fill kernels clear the
 *   counters, then a count, a three-kernel scan, one fill per simplex
 *   dimension and the edge counts.  Vertex ids must be valid (wect_validate).
 */
size_t wect_lower_star_bytes(const wect_complex* c);
wect_status wect_lower_star_build(const wect_complex* c, void* index, size_t index_bytes, void* hip_stream);

/*
 * wect_smooth_forward / wect_smooth_backward through the lower-star index:
 * same arguments and results, plus the index built for the same complex
 * (index_bytes >= wect_lower_star_bytes(c)); the workspace size is
 * wect_smooth_ls_workspace_bytes.  Work per direction is one window per
 * vertex (float64 sum of the combined cell weights, then the fixed-point grid
 * of the forward with |combined weight| 2^e < 2^30) plus the argmax test of
 * each vertex's cofaces.  The adjoint writes each vertex's coordinate
 * gradient from its own combined weight, and adds each cell's weight
 * gradient from the vertices that top it (float32 atomics).
 */
size_t wect_smooth_ls_workspace_bytes(const wect_complex* c, const wect_grid* g, float lam);
wect_status wect_smooth_ls_forward(const wect_complex* c, const wect_grid* g, float lam, const void* index,
                                   size_t index_bytes, float* out, void* ws, size_t ws_bytes, void* hip_stream);
wect_status wect_smooth_ls_backward(const wect_complex* c, const wect_grid* g, float lam, const void* index,
                                    size_t index_bytes, const float* grad_out, float* grad_coords,
                                    float* grad_dirs, float* const grad_w[4], float* grad_vertex,
                                    void* hip_stream);

/*
 * Synchronous data check on `hip_stream`: CSR offsets and shapes consistent
 * with the counts, vertex ids in range, thresholds non-decreasing, axes
 * strictly increasing, no NaN/Inf in coordinates, directions, thresholds or
 * float weights.  Returns the first failing class (INDEX, THRESHOLDS,
 * NONFINITE) or WECT_OK.  Allocates and synchronises: not for graph capture.
 */
wect_status wect_validate(const wect_complex* c, const wect_grid* g, void* hip_stream);

/* Static, NUL-terminated description of a status code. */
const char* wect_status_string(wect_status s);

/*
 * Launch shape used by the following calls of this process (for tuning).
 * block: threads per block of the main kernels (256, 512 or 1024; 0 = default:
 *        the size giving the most resident wavefronts per compute unit);
 * blocks_per_cu: main-kernel blocks per compute unit (0 = as many as fit: 32
 *                wavefronts and 160 KiB of LDS per compute unit);
 * min_items_per_block: lower bound of stream items per block (0 = default, 256);
 * decomposition: how the forward splits its work over blocks
 *   0 = automatic,
 *   1 = stream: the (complex, direction tile, cell) stream is cut into equal
 *       contiguous ranges, one per block; groups (complex, direction tile)
 *       that a range covers whole are written by that block, the others are
 *       summed from per-block partial histograms by a second kernel,
 *   2 = one block per group: every block writes its group's output, with no
 *       partial histograms and no second kernel (balanced when the groups
 *       are of similar size and at least as many as the compute units).
 * threshold_tile: thresholds per launch (0 = automatic: all T when their
 *   LDS histogram fits, else the fewest balanced tiles that fit).  A smaller
 *   tile means a smaller histogram, so more blocks per compute unit or a
 *   larger staging area, at the price of one pass over the cells per tile.
 *   Values above what fits are lowered to the largest tile that fits.
 * directions_per_lane: the direction tile of the cubical forward is 64 times
 *   this (0 = automatic: 2 when d > 64 and two histogram columns per lane fit
 *   LDS, else 1; 1 or 2 to choose).  With 2, every staged voxel (its 3^n
 *   neighbourhood and combined weights) serves two directions per lane.
 *   Simplicial complexes always use 1.
 * cubical_records: 0 = automatic, 1 = off, 2 = on, 3 = on with two voxels
 *   per thread.  When on, the cubical forward first forms every voxel's 2^n
 *   combined weights once into records (8 bytes per voxel in 2D, 16 in 3D,
 *   part of the workspace) and stages those instead of the voxel's 3^n
 *   neighbourhood; automatic turns it on when a voxel would otherwise be
 *   staged more than once (several direction or threshold tiles).  With 3, a
 *   tile covers 1.5 staging tiles of voxels, two per thread, and the
 *   contributing ones that do not fit the stage go in a second round of the
 *   same tile (fewer tiles and block barriers per voxel); automatic does this
 *   for volumes (n = 3) when every block walks at least 16 tiles.
 *   wect_forward_noalloc never uses records.
 * cell_packing: 0 = automatic, 1 = off.  With at most 32 directions (or
 *   filter columns of the general-filter WECF) the simplicial forward packs
 *   64 / dt cells into each wavefront instruction, dt being the smallest
 *   power of two >= d: lane l serves direction l mod dt of cell l / dt and
 *   keeps its own histogram column; the copies are added together before the
 *   threshold scan, so the output is unchanged (integer and fixed-point sums
 *   are exact).  Without it, lanes past d idle.
 * stage_entries: cells (or voxels) staged per tile by the forward's main
 *   kernel (0 = automatic: one per thread as far as LDS allows, except 768
 *   for 1024-thread simplicial blocks, which measured faster than 1024; else
 *   a multiple of 64, at most 1024, lowered to what fits).  A smaller staging
 *   tile takes less LDS, which can let another block share the compute unit,
 *   at the price of more block barriers per cell.
 * Changing it changes wect_workspace_bytes().  Not to be called while other
 * threads are inside wect_* calls.
 */
typedef struct {
  int32_t block;
  int32_t blocks_per_cu;
  int32_t min_items_per_block;
  int32_t decomposition;
  int32_t threshold_tile;
  int32_t directions_per_lane;
  int32_t cubical_records;
  int32_t cell_packing;
  int32_t stage_entries;
} wect_launch;

wect_status wect_set_launch(const wect_launch* l);
wect_status wect_get_launch(wect_launch* l);

/*
 * Kernel timing for measurement.  When enabled, every following call records
 * HIP events on its own stream around its main kernel (the histogram kernel
 * of the forward, the adjoint kernel of the backward); wect_profile_read
 * synchronises those events and returns the summed durations and launch
 * counts since the last reset.  Event recording is not capture-safe: leave
 * it disabled while capturing.
 */
wect_status wect_profile_enable(int on);
wect_status wect_profile_read(double* fwd_ms, int64_t* fwd_launches,
                              double* bwd_ms, int64_t* bwd_launches, int reset);

/*
 * Measurement helpers (not part of the transform), used to calibrate what the
 * kernels are measured against.
 *
 * wect_calib_copy: copies `bytes` bytes from src to dst (device pointers,
 *   16-byte aligned, not overlapping) with one plain kernel of 16-byte loads
 *   and stores: the achievable HBM copy bandwidth, and the copy of known size
 *   against which the FETCH_SIZE / WRITE_SIZE counters are scaled.
 * wect_calib_lds_atomics: `blocks` blocks of 1024 threads; every thread
 *   issues `reps` LDS atomic adds into its lane's column of a 64 x 64 table,
 *   so the 64 lanes of a wavefront hit 64 consecutive words (the access
 *   pattern of the histogram kernels).  kind 0: 32-bit integer add, 1: 64-bit
 *   integer add, 2: float32 add.  out: device array of blocks * 64 elements of
 *   that width (row 0 of every block's table), overwritten.  Lane-level adds
 *   per second = blocks * 1024 * reps / (kernel time).
 * Both only enqueue on hip_stream; WECT_ERR_ARG on bad arguments.
 */
wect_status wect_calib_copy(void* dst, const void* src, size_t bytes, void* hip_stream);
wect_status wect_calib_lds_atomics(int32_t kind, int32_t blocks, int32_t reps, void* out, void* hip_stream);

/* Library version string, e.g. "wect 0.1 gfx950". */
const char* wect_version(void);

/* Description of the last HIP failure behind a WECT_ERR_DEVICE returned on
 * the calling thread ("" if none).  Valid until the next call on the thread. */
const char* wect_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WECT_H */
