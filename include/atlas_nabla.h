/*
 * atlas_nabla.h -- C ABI of the MI355X (gfx950) median-dual Nabla library.
 *
 * The calls follow the Grid -> Mesh -> FunctionSpace -> Field workflow of the
 * Atlas report (Section 2.3, Figure 2): a mesh is built once from a grid
 * name, fields are plain device arrays laid out as NodeColumns (one column of
 * levels per mesh node), and the Nabla operators the report lists among the
 * operations the library offers (gradient, divergence, Laplacian; Section 2.3)
 * are applied to them.  The report's own language bindings wrap each C++
 * method in one C function taking plain pointers (Section 4.1, Figure 3);
 * this header keeps that pattern: only C types, plain host or device
 * pointers and sizes cross it, and no C++ exception escapes.
 *
 * Conventions for every call
 *   - Return value: ATLAS_OK (0) or a negative status below.  On failure the
 *     thread-local message of atlas_last_error() says why.  Argument errors
 *     are detected synchronously, before anything is launched.
 *   - Fields are dense, contiguous, row-major device arrays:
 *       scalar  [nnodes][nlev]        (levels innermost)
 *       vector  [nnodes][nlev][2]     (east, north components innermost)
 *     Element type is given by atlas_dtype_t.  Pointers must be aligned to
 *     the element size (scalars) or twice the element size (vectors).
 *   - Outputs are overwritten, never accumulated into; an output may not
 *     overlap its input (the operators gather neighbour values).
 *   - nnodes * nlev must not exceed 2^32 - 1 (ATLAS_ESHAPE otherwise).
 *   - `stream` is a hipStream_t of the mesh's device passed as void*
 *     (NULL = the default stream).  Operator calls are asynchronous on it.
 *   - Node order, edge order and the dual geometry are defined by
 *     atlas_mesh_build; see the comment there.
 */
#ifndef ATLAS_NABLA_H
#define ATLAS_NABLA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ATLAS_NABLA_ABI_VERSION 1

/* ---- status codes ------------------------------------------------------ */
enum {
  ATLAS_OK = 0,
  ATLAS_EINVAL = -1,  /* bad argument: NULL, bad name, misaligned, overlap  */
  ATLAS_ENOMEM = -2,  /* host or device allocation failed                  */
  ATLAS_EHIP = -3,    /* a HIP runtime call or kernel launch failed        */
  ATLAS_ENODEV = -4,  /* no GPU, bad device ordinal, or a host-only mesh   */
  ATLAS_EDTYPE = -5,  /* unknown dtype, or dtype not supported by the call */
  ATLAS_ESHAPE = -6   /* nlev <= 0, or sizes beyond the supported range    */
};

/* ---- element types ----------------------------------------------------- */
typedef enum {
  ATLAS_F64 = 0,  /* FP64 storage and arithmetic, FP64 geometry tables      */
  ATLAS_F32 = 1,  /* FP32 storage and arithmetic; tables rounded once from
                     the FP64 geometry                                      */
  ATLAS_BF16 = 2  /* bfloat16 storage, FP32 arithmetic, FP32 tables; each
                     output is rounded to nearest-even bfloat16             */
} atlas_dtype_t;

typedef struct atlas_mesh_s* atlas_mesh_t;

/* Static version string, e.g. "atlas-nabla 0.1.0 gfx950". */
const char* atlas_version(void);

/* Message for the last non-OK status returned on this thread ("" if none).
 * The pointer stays valid until the next failing call on the thread. */
const char* atlas_last_error(void);

/* Number of visible HIP devices.  Returns ATLAS_ENODEV (and *count = 0) when
 * the HIP runtime reports none. */
int atlas_device_count(int* count);

/* ---- mesh ---------------------------------------------------------------- */

/* Build the median-dual mesh of an octahedral reduced Gaussian grid.
 *
 * grid    "O<N>", N >= 1 (the report names grids this way, Section 4.3).
 *         Row k (0..2N-1, north to south) lies at the k-th Gaussian
 *         colatitude (root of P_2N(cos t)) and holds 4*min(k+1, 2N-k)+16
 *         points at longitudes 2*pi*j/n_k; nodes are numbered row by row.
 *         Bands between rows are triangulated by an exact-integer zipper,
 *         each 20-point polar row by a ladder of 18 triangles whose 17
 *         chords are the pole edges; no node sits at a pole.
 *         V = 4N^2 + 36N nodes, E = 3V - 6 edges, T = 2V - 4 triangles.
 * radius  sphere radius in metres (> 0), e.g. 6371220.0.
 * device  HIP device ordinal that receives the operator tables, or -1 for a
 *         host-only mesh (connectivity and geometry only: the export calls
 *         work, operator calls return ATLAS_ENODEV).
 * out     receives the handle; the library owns all its memory until
 *         atlas_mesh_free.
 * Errors: ATLAS_EINVAL (name, radius, NULL out), ATLAS_ENODEV (no such
 * device), ATLAS_ENOMEM, ATLAS_EHIP, ATLAS_ESHAPE (N too large for 32-bit
 * node indices). */
int atlas_mesh_build(const char* grid, double radius, int device, atlas_mesh_t* out);

/* Release host and device memory of a mesh.  NULL is allowed.  The caller
 * must make sure no queued operator call still uses the mesh. */
void atlas_mesh_free(atlas_mesh_t mesh);

/* Sizes.  Any output pointer may be NULL.  max_slots is the largest node
 * degree (<= 7); nrows = 2N. */
int atlas_mesh_sizes(atlas_mesh_t mesh, int64_t* nnodes, int64_t* nedges,
                     int64_t* ntris, int64_t* npole_edges, int32_t* max_slots,
                     int32_t* nrows);

/* Host copies of the grid.  Caller-owned host buffers; any may be NULL.
 * row_size [nrows], row_off [nrows+1], colat [nrows] (radians),
 * lonlat [V][2] (radians), xyz [V][3] (unit sphere). */
int atlas_mesh_export_grid(atlas_mesh_t mesh, int32_t* row_size, int64_t* row_off,
                           double* colat, double* lonlat, double* xyz);

/* Host copies of the connectivity.  Caller-owned host buffers; any may be
 * NULL.  tris [T][3] (counter-clockwise seen from outside, smallest index
 * first, list sorted), edges [E][2] (a < b, sorted), csr_off [V+1],
 * nbr/eid [2E] (slots of each node ordered by neighbour index), sgn [2E]
 * (+1 if the node is the edge's first end, -1 otherwise), rev [2E] (position
 * of the node in its neighbour's slot list), is_pole [E] (1 for ladder
 * chords). */
int atlas_mesh_export_connectivity(atlas_mesh_t mesh, int32_t* tris, int32_t* edges,
                                   int64_t* csr_off, int32_t* nbr, int32_t* eid,
                                   int8_t* sgn, int8_t* rev, uint8_t* is_pole);

/* Host copies of the FP64 median-dual geometry.  Caller-owned host buffers;
 * any may be NULL.  S [E][3] dual normal of each edge in metres (integrated
 * outward conormal of the dual face, pointing from the edge's first end to
 * its second), V [V] dual cell areas in m^2, basis [V][2][3] local (east,
 * north) unit vectors, C [V][3] closure sum_e sign(i,e) S_e. */
int atlas_mesh_export_geometry(atlas_mesh_t mesh, double* S, double* V,
                               double* basis, double* C);

/* ---- operators ------------------------------------------------------------
 * All five are gathers over each node's edges (no atomics): every output
 * element is written by exactly one thread in a fixed slot order, so reruns
 * are bitwise identical.  Units follow the radius: gradient and divergence
 * per metre, Laplacian per square metre. */

/* grad_i = (1/V_i) [sum_e sign(i,e) 0.5 (f_i + f_j) S_e - f_i C_i], projected
 * on (east_i, north_i); evaluated in the equivalent difference form
 * sum_e sign(i,e) 0.5 (f_j - f_i) S_e / V_i.
 * f: scalar [V][nlev] -> grad: vector [V][nlev][2]. */
int atlas_nabla_gradient(atlas_mesh_t mesh, int dtype, int32_t nlev,
                         const void* f, void* grad, void* stream);

/* div_i = (1/V_i) sum_e sign(i,e) 0.5 (U_i + U_j) . S_e with
 * U = u east + v north.  uv: vector [V][nlev][2] -> div: scalar [V][nlev]. */
int atlas_nabla_divergence(atlas_mesh_t mesh, int dtype, int32_t nlev,
                           const void* uv, void* div, void* stream);

/* lap = div(grad f).  f, lap: scalar [V][nlev].
 * workspace == NULL: one fused pass over the precomputed two-ring stencil
 *   lap_i = sum_m W_im (f_m - f_i), W = (divergence matrix)(gradient matrix).
 * workspace != NULL: two passes through a caller-owned device buffer of
 *   V*nlev*2 elements of the dtype (gradient, then divergence). */
int atlas_nabla_laplacian(atlas_mesh_t mesh, int dtype, int32_t nlev,
                          const void* f, void* lap, void* workspace, void* stream);

/* Gradient and Laplacian of one field in one pass: grad as
 * atlas_nabla_gradient, lap as the fused atlas_nabla_laplacian, bitwise the
 * same values (up to the sign of zero) -- the two-ring differences f_m - f_i
 * serve both sums, and the field is read from memory once.  f: scalar
 * [V][nlev]; grad: vector [V][nlev][2]; lap: scalar [V][nlev]; no two of
 * them may overlap.  Runs as one kernel on the Laplacian's launch shape
 * when that is the one-tile LDS form (the default for columns of more than
 * 32 levels), else as the two calls one after the other. */
int atlas_nabla_gradient_laplacian(atlas_mesh_t mesh, int dtype, int32_t nlev,
                                   const void* f, void* grad, void* lap, void* stream);

/* Exact transpose of atlas_nabla_gradient for the plain Euclidean inner
 * product over all (node, level, component) entries:
 * sum(w * grad f) == sum(f * gradient_adjoint(w)).
 * w: vector [V][nlev][2] -> fbar: scalar [V][nlev]. */
int atlas_nabla_gradient_adjoint(atlas_mesh_t mesh, int dtype, int32_t nlev,
                                 const void* w, void* fbar, void* stream);

/* Exact transpose of atlas_nabla_divergence.
 * d: scalar [V][nlev] -> uvbar: vector [V][nlev][2]. */
int atlas_nabla_divergence_adjoint(atlas_mesh_t mesh, int dtype, int32_t nlev,
                                   const void* d, void* uvbar, void* stream);

/* Curl (vertical vorticity), the fourth operation Section 2.3 names, in the
 * same edge-based form with the tangential face vector:
 * curl_i = (1/V_i) sum_e sign(i,e) 0.5 (U_i + U_j) . T_e, T_e = m_e x S_e,
 * m_e the unit edge midpoint, U = u east + v north -- the circulation around
 * the dual cell, counter-clockwise seen from outside, per unit area.
 * uv: vector [V][nlev][2] -> zeta: scalar [V][nlev] (per metre). */
int atlas_nabla_curl(atlas_mesh_t mesh, int dtype, int32_t nlev,
                     const void* uv, void* zeta, void* stream);

/* Divergence and curl (vertical vorticity) of one vector field in one pass,
 * bitwise the values of atlas_nabla_divergence and atlas_nabla_curl (up to
 * the sign of zero); the field is read from memory once.  uv: vector
 * [V][nlev][2]; div, zeta: scalar [V][nlev]; no two of them may overlap.
 * One kernel on the divergence's launch shape when that is the one-tile LDS
 * form (the default for columns of more than 32 levels), else the two calls
 * one after the other. */
int atlas_nabla_divergence_curl(atlas_mesh_t mesh, int dtype, int32_t nlev,
                                const void* uv, void* div, void* zeta, void* stream);

/* Divergence (Section 2.3) and gradient adjoint of one vector field in one
 * pass, bitwise the values of atlas_nabla_divergence and
 * atlas_nabla_gradient_adjoint (up to the sign of zero): both combine a
 * node's own value and its 1-ring neighbours' values with one coefficient
 * pair each, so the same loads feed both sums and the field is read from
 * memory once.  uv: vector [V][nlev][2]; div, fbar: scalar [V][nlev]; no
 * two of them may overlap.  One kernel on the divergence's launch shape
 * when that is the one-tile LDS form (the default for columns of more than
 * 32 levels), else the two calls one after the other. */
int atlas_nabla_divergence_gradient_adjoint(atlas_mesh_t mesh, int dtype, int32_t nlev,
                                            const void* uv, void* div, void* fbar, void* stream);

/* Exact transpose of atlas_nabla_curl.
 * z: scalar [V][nlev] -> uvbar: vector [V][nlev][2]. */
int atlas_nabla_curl_adjoint(atlas_mesh_t mesh, int dtype, int32_t nlev,
                             const void* z, void* uvbar, void* stream);

/* Global conservation check of a divergence field: per level k,
 * out_sum[k] = sum_i V_i div_ik and out_abs[k] = sum_i |V_i div_ik|, both
 * accumulated in FP64 in a fixed order (two-pass tree), so results are
 * bitwise reproducible.  div: scalar [V][nlev] of dtype; out_sum, out_abs:
 * device FP64 arrays [nlev].  The first call on a mesh for a given nlev may
 * allocate an internal partial-sum buffer (kept until atlas_mesh_free). */
int atlas_nabla_conservation(atlas_mesh_t mesh, int dtype, int32_t nlev,
                             const void* div, double* out_sum, double* out_abs,
                             void* stream);

/* atlas_nabla_conservation for callers that cannot allocate device memory
 * (code under stream capture into a graph, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels and the same results, bit for bit,
 * with the partial sums in a 16 MiB array the library holds on each GPU
 * until the process ends, instead of a buffer allocated on first use.  It
 * makes no hipMalloc, hipFree or other allocating call.  The caller passes
 * div, out_sum and out_abs as for atlas_nabla_conservation.  Limit: the
 * partial sums, min(4096, ceil(V / 64)) x nlev x 16 bytes, must fit the
 * array (at most 256 levels on meshes of 262,144 nodes or more, e.g. O320 to
 * O1280); larger nlev returns ATLAS_ESHAPE with the limit in the message.
 * Every entry of the array a call reads is written earlier in that call, so
 * nothing needs clearing; but all calls on one GPU share the array, so
 * calls that overlap in time on that GPU (different streams, or threads)
 * race and must be serialised by the caller. */
int atlas_nabla_conservation_noalloc(atlas_mesh_t mesh, int dtype, int32_t nlev,
                                     const void* div, double* out_sum, double* out_abs,
                                     void* stream);

/* ---- grid-to-grid remapping (Section 4.3, Figures 4-6) ----------------------
 * A field on the nodes of an O-grid mesh is interpolated to the points of a
 * target grid, linearly over the source triangle each point lies in, in 3-D
 * on the sphere: the ray from the centre through the target point p meets
 * the flat triangle (a, b, c) (outward counter-clockwise) where the triple
 * products D_a = det(p,b,c), D_b = det(a,p,c), D_c = det(a,b,p) are >= 0 with
 * sum D > 0, and the weights are (D_a, D_b, D_c) / D.  Target grids: "F<M>",
 * the regular Gaussian grid (2M rows at the roots of P_2M, 4M points per row
 * at longitude 2 pi j / 4M), or "O<M>"; points numbered row by row from
 * north to south, west to east. */
typedef struct atlas_remap_s* atlas_remap_t;

/* Locates every target point on the host (FP64) and, for a mesh built on a
 * device, uploads the tables (P x 16 bytes of node indices and P x 32 / 16
 * bytes of FP64 / FP32 weights, and the transpose by source node: 8 bytes
 * per node plus 3 x (4 + 8 + 4) bytes per point).  The remap refers to
 * `mesh`, which must
 * outlive it.  *out owned by the caller; release with atlas_remap_free.
 * Statuses: ATLAS_EINVAL (NULL arguments, bad target name), ATLAS_ENOMEM,
 * ATLAS_ESHAPE (target too large), ATLAS_EHIP. */
int atlas_remap_build(atlas_mesh_t mesh, const char* target, atlas_remap_t* out);
void atlas_remap_free(atlas_remap_t remap);

/* npoints: target points P; nfallback: points that needed the exhaustive
 * search (0 on the octahedral meshes).  NULL pointers are skipped. */
int atlas_remap_sizes(atlas_remap_t remap, int64_t* npoints, int64_t* nfallback);

/* Host copies, caller-owned: nodes int32 [P][3], weights FP64 [P][3],
 * target positions xyz FP64 [P][3] (unit vectors).  NULL skips an array. */
int atlas_remap_export(atlas_remap_t remap, int32_t* nodes, double* weights, double* xyz);

/* dst[t][k] = w_t0 src[n_t0][k] + w_t1 src[n_t1][k] + w_t2 src[n_t2][k]
 * (in this order, with fused multiply-adds) for every target point t and
 * level k.  src: device [V][nlev] of dtype (any alignment of the element
 * size); dst: device [P][nlev], overwritten, must not overlap src.  FP64
 * weights for ATLAS_F64, FP32 weights and arithmetic for ATLAS_F32 and
 * ATLAS_BF16.  Asynchronous on `stream`. */
int atlas_remap_apply(atlas_remap_t remap, int dtype, int32_t nlev, const void* src, void* dst,
                      void* stream);

/* Exact transpose of atlas_remap_apply for the plain Euclidean inner
 * product (sum(dst * ybar) == sum(src * fbar)): fbar[n][k] = the sum, over
 * the target points t whose triangle has node n, in ascending t, of
 * w_tn ybar[t][k] (fused multiply-adds; 0 for nodes no point uses).
 * ybar: device [P][nlev]; fbar: device [V][nlev], overwritten, must not
 * overlap ybar.  Weights as in atlas_remap_apply.  Asynchronous on
 * `stream`. */
int atlas_remap_apply_adjoint(atlas_remap_t remap, int dtype, int32_t nlev, const void* ybar, void* fbar,
                              void* stream);

/* ---- batched multi-tracer launch ------------------------------------------
 * Many fields with different level counts go through one persistent kernel
 * launch per operator.  Per tracer, the same arithmetic per output element
 * as the single-field calls, so results are bitwise identical to them. */

enum {
  ATLAS_OP_GRADIENT = 1,
  ATLAS_OP_DIVERGENCE = 2,
  ATLAS_OP_GRADIENT_ADJOINT = 4,
  ATLAS_OP_DIVERGENCE_ADJOINT = 8,
  ATLAS_OP_LAPLACIAN = 16,  /* tuning and launch shapes only; not batchable */
  ATLAS_OP_CURL = 32,       /* tuning and launch shapes only; not batchable */
  ATLAS_OP_CURL_ADJOINT = 64 /* tuning and launch shapes only; not batchable */
};

typedef struct {
  int32_t nlev;          /* levels of this tracer, >= 1                    */
  int32_t reserved;      /* must be 0                                       */
  const void* in[4];     /* per operator bit (gradient, divergence, grad
                            adjoint, div adjoint): input field, device      */
  void* out[4];          /* per operator bit: output field, device          */
} atlas_tracer_desc_t;

/* Launch shape.  Zero fields mean "library default". */
typedef struct {
  int32_t waves_per_block;  /* 1, 2, 4, 8 or 16 (8 and 16: one-tile-per-
                               workgroup LDS tiles only, 16 except for the
                               three-slice FP64 Laplacian, which takes 8;
                               other launches use at most 4)                 */
  int32_t nodes_per_wave;   /* node groups a wave handles per workgroup       */
  int32_t blocks_per_cu;    /* persistent grid = blocks_per_cu * CU count     */
  int32_t xcd_remap;        /* 1: each XCD walks a contiguous part of the
                               node order (the default), 2: plain order      */
  int32_t lanes_per_node;   /* 16, 32 or 64 lanes share a column (nlev > 32);
                               columns of <= 32 levels always use nlev lanes */
  int32_t slices_per_iter;  /* level slices in flight per lane, 1..3         */
  int32_t band_rows;        /* rows per band of the node processing order:
                               runs of a band are visited by longitude so
                               rows above and below stay in cache (default
                               32); LDS tiles: rows per tile (default 4)      */
  int32_t run_nodes;        /* consecutive nodes of a row per run (default 16,
                               64 on the row-window walk); LDS tiles: bands
                               swept together by longitude (default 8)        */
  int32_t nt_stores;        /* 1: non-temporal output stores, 2: plain (the
                               default)                                      */
  int32_t row_window;       /* 1-ring operators on columns of more than 32
                               levels: 1 walk rows reusing the previous
                               node's column loads (the default), 2 gather
                               every slot per node                            */
  int32_t lds_tiles;        /* FP32/FP64 columns of more than 32 levels:
                               stage tiles of nodes with the columns their
                               stencils read in LDS: 1 persistent workgroups,
                               double buffered; 3 one tile per workgroup;
                               0/2 off (the default)                          */
  int32_t tile_kb;          /* LDS budget of one tile in KiB, 8..160 (0: per-
                               operator default); the persistent form holds
                               two tiles, which must fit the CU's 160 KiB     */
  int32_t tile_waves;       /* persistent tiles: computing waves, 1..15
                               (0: per-operator default)                      */
  int32_t producer_waves;   /* persistent tiles: copying waves, 1, 2, 4 or 8
                               (0: per-operator default); tile_waves +
                               producer_waves
                               <= 16, and <= 8 for FP64 (launch fails else)   */
  int32_t tile_wgs_per_cu;  /* persistent tiles: workgroups per CU, 1..4
                               (0: 1); two tile buffers each must fit LDS     */
  int32_t tile_levels;      /* LDS tiles: levels per column chunk (0: whole
                               columns when 48 (1-ring) or 96 (two-ring)
                               columns fit the budget, else equal chunks);
                               ignored if one node's stencil would not fit    */
  int32_t batch_mode;       /* batched plans: 1 (the default) one persistent
                               launch per operator over all tracers, on the
                               LDS tiles of the one-tile form (tile_kb,
                               band_rows, run_nodes, tile_levels and
                               waves_per_block shape it, tile_wgs_per_cu caps
                               its workgroups per CU; an operator whose tiles
                               do not fit runs as field launches); 2 the
                               single-field launch of each (operator, tracer)
                               with the mesh's shapes, operators outermost    */
  int32_t batch_claim;      /* batched persistent form: consecutive tiles a
                               workgroup takes per claim on its XCD's work
                               counter, 1..64 (0: 4)                          */
} atlas_tune_t;

typedef struct atlas_batch_s* atlas_batch_t;

/* Create a plan: validates descriptors (host array of ntracers entries,
 * copied), fixes the launch shape (tune may be NULL) and, for the persistent
 * form, builds each operator's LDS tiling and node records on the mesh (kept
 * with the mesh) and uploads the plan's work tables: per tracer its fields,
 * level chunk and work items (tiles x chunks), and per XCD of the GPU the
 * count of items before each tracer (each XCD takes an equal contiguous share
 * of every tracer's tiles).  op_mask is an OR of ATLAS_OP_* bits; every
 * tracer must give in/out pointers for every selected operator.  dtype:
 * ATLAS_F32 or ATLAS_F64.  The plan owns its work tables until
 * atlas_batch_free. */
int atlas_batch_create(atlas_mesh_t mesh, int dtype, const atlas_tracer_desc_t* descs,
                       int32_t ntracers, uint32_t op_mask, const atlas_tune_t* tune,
                       atlas_batch_t* out);

/* Enqueue the plan's work on `stream`, operators in the order of the bits
 * above: in the persistent form one launch per operator (as many workgroups
 * as the CUs hold at once, each walking its XCD's share of the (tracer,
 * tile, chunk) items); with batch_mode 2 the single-field launch of every
 * tracer for each operator.  A plan whose divergence and gradient adjoint
 * take the same input field in every tracer, with no output of either
 * overlapping an input, runs those two as one persistent launch on the
 * divergence's shape (as atlas_nabla_divergence_gradient_adjoint: the same
 * values; in FP64 only on shapes of at most 8 waves, else as two launches);
 * atlas_batch_tune still times them one at a time.  The
 * persistent form
 * allocates nothing and never synchronises; the field form does so only the
 * first time a (operator, dtype, level count) is used on the mesh, when it
 * builds node orders, tilings and records -- after one eager run it too may be
 * recorded into a HIP graph by stream capture. */
int atlas_batch_run(atlas_batch_t plan, void* stream);

/* Run the plan through a HIP graph owned by the plan: the first call
 * (after one eager run on `stream` in the field form, then synchronising
 * `stream`) captures atlas_batch_run and instantiates the graph, every
 * call launches it on `stream`. */
int atlas_batch_graph_launch(atlas_batch_t plan, void* stream);

void atlas_batch_free(atlas_batch_t plan);

/* Time candidate launch shapes of a plan, each operator's launch on its own
 * (`reps` runs each after one warm-up, HIP events on `stream`, which it
 * synchronises; the plan's fields are read and overwritten): the field form,
 * then the persistent form over tile LDS budgets, tiles per claim and waves
 * per workgroup.  Keeps each operator's fastest shape in the plan
 * (re-uploading its work tables), drops any captured graph, and writes
 * best[b] for each operator bit b of the plan (best has 4 entries, in the
 * order gradient, divergence, gradient adjoint, divergence adjoint; entries
 * of operators not in the plan are left as they were) and to *best_ms the
 * sum over the plan's operators of their fastest times per run, in
 * milliseconds. */
int atlas_batch_tune(atlas_batch_t plan, int32_t reps, void* stream, atlas_tune_t* best,
                     float* best_ms);

/* ---- autotuning ----------------------------------------------------------- */

/* Time candidate launch shapes of one operator (one ATLAS_OP_* bit) on
 * caller-provided device input/output fields of nlev levels (contents are
 * read/overwritten), `reps` launches per candidate after one warm-up, with
 * HIP events on `stream` (synchronises it).  Writes the fastest shape to
 * *best and its mean time per launch in milliseconds to *best_ms. */
int atlas_nabla_tune(atlas_mesh_t mesh, int dtype, uint32_t op, int32_t nlev,
                     const void* in, void* out, int32_t reps, void* stream,
                     atlas_tune_t* best, float* best_ms);

/* Set the launch shape used by the single-field calls for (op, dtype) on this
 * mesh; NULL restores the default.  op: one ATLAS_OP_* bit.  A band height
 * not used before on this mesh builds its node order on the next call (host
 * work plus one device allocation of 4 bytes per node). */
int atlas_nabla_set_tune(atlas_mesh_t mesh, int dtype, uint32_t op,
                         const atlas_tune_t* tune);

/* The one-pass calls, for atlas_nabla_describe only: the launches of
 * atlas_nabla_gradient_laplacian (on the Laplacian's shape),
 * atlas_nabla_divergence_curl and atlas_nabla_divergence_gradient_adjoint
 * (on the divergence's). */
enum {
  ATLAS_OP_GRADIENT_LAPLACIAN = 1 << 16,
  ATLAS_OP_DIVERGENCE_CURL = 1 << 17,
  ATLAS_OP_DIVERGENCE_GRADIENT_ADJOINT = 1 << 18
};

/* Describe the launch a single-field call of (op, dtype) on nlev levels
 * would make with the mesh's current shape: the shape after per-operator
 * defaults are applied (to *resolved, if not NULL) and the name of the
 * kernel it runs, e.g. "k_tile<float, 0, 3>" (to kernel, NUL-terminated and
 * truncated to len bytes, if not NULL).  op: one ATLAS_OP_* bit, or one of
 * the one-pass codes above, whose kernel name reads "two calls" when the
 * shape is not the one-tile LDS form (the call then runs its two operators
 * one after the other; a BF16 field that is not 4-byte aligned does so too).
 * Works on host-only meshes; no device work, no allocation. */
int atlas_nabla_describe(atlas_mesh_t mesh, int dtype, uint32_t op, int32_t nlev,
                         atlas_tune_t* resolved, char* kernel, int32_t len);

#ifdef __cplusplus
}
#endif

#endif /* ATLAS_NABLA_H */
