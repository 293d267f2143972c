/* quadamg: auxiliary-grid algebraic multigrid on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the method of Wang, Hu, Cohen and Xu, "A Parallel Auxiliary Grid AMG Method for GPU": an SPD system
 * A x = b from a 2D discretisation (Section 1, eq. 1) is solved by unsmoothed aggregation on a region quadtree of an
 * auxiliary grid (Section 3), with Galerkin coarse operators of fixed 9-point pattern (eq. 3-4, Section 4.4), a
 * quadtree-colored Gauss-Seidel smoother (Section 4.5) and the nonlinear AMLI-cycle (Algorithm 2.2) used as the
 * preconditioner of a flexible conjugate-gradient iteration (Algorithm 2.1).
 *
 * Conventions shared by every entry point:
 *  - Pointers marked "device" are device memory of the hierarchy's device (the device current at amg_setup);
 *    "host" pointers are ordinary host memory. Inputs are borrowed for the duration of the call only.
 *  - Arrays are 0-based; coords is n x 2 interleaved (x0, y0, x1, y1, ...); CSR is row_ptr[n+1] (int64),
 *    col_idx[nnz] (int32), vals[nnz] (float64), columns in any order inside a row, the diagonal present.
 *  - Work is enqueued on the options' stream (NULL = the default stream). Calls that return data to the host
 *    synchronise that stream.
 *  - Every call returns an amg_status; on failure no output handle is created and nothing leaks.
 *  - A hierarchy holds one solve workspace: one solve at a time per hierarchy. Distinct hierarchies may be used
 *    concurrently on different streams.
 *  - Results are deterministic: no floating-point atomics; reductions use a fixed tree that depends only on the
 *    system size.
 */
#ifndef QUADAMG_H
#define QUADAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AMG_OK = 0,
    AMG_ERR_INVALID = 1,   /* bad argument or malformed input (checked before the hierarchy is built) */
    AMG_ERR_NOMEM = 2,     /* a device or host allocation failed */
    AMG_ERR_DEVICE = 3,    /* a HIP runtime call failed */
    AMG_ERR_NOT_SPD = 4,   /* non-positive diagonal on some level, or the coarsest Cholesky failed */
    AMG_ERR_BREAKDOWN = 5, /* (p, A p) <= 0 in the outer iteration */
    AMG_ERR_NOCONV = 6     /* max_iters reached; x holds the last iterate */
} amg_status;

typedef struct amg_hierarchy amg_hierarchy;

typedef struct {
    int32_t precision;   /* 0: plain FP64 solve. 1: FP32 hierarchy, smoother and SpMV inside the preconditioner,
                            FP64 outer iteration, FP64 inner products and FP64 coarsest solve. */
    int32_t coarse_max;  /* the coarsest quadtree level is the first k <= L with 4^k <= coarse_max; a system with
                            n <= coarse_max is solved directly (default 64) */
    int32_t inner_iters; /* steps n of Algorithm 2.1 inside the cycle: 1 or 2 (default 2, the K-cycle) */
    int32_t sweeps;      /* smoothing sweeps before and after the coarse correction (default 1) */
    int32_t outer_mmax;  /* directions the outer flexible CG orthogonalises against (Algorithm 2.1, Step 2): 0 or 1
                            (default 1: the last one); -1 every earlier direction since the start or the last
                            restart, as Algorithm 2.1 is written (2 n doubles of device memory per iteration, made on
                            first use and kept by the hierarchy) */
    int32_t max_iters;   /* outer iteration cap (default 1000) */
    int32_t engine;      /* 1 (default): the small coarse levels of the cycle run inside one persistent workgroup
                            with LDS-resident operators, specialised at compile time to the level shape where the
                            levels allow it, and each larger quadtree level without same-color or overflow couplings
                            runs its presmoothing sweep with the restriction, and its first post-smoothing sweep, as
                            one launch each (16 x 16 super-cell tiles; the same values as one launch per color
                            phase); 2: the same, with the workgroup always through its generic step interpreter;
                            0: one kernel launch per step on every level */
    int32_t batch;       /* 1 (default): amg_solve_batch runs this system, when it has at most 65,536 unknowns, as
                            one workgroup of a whole-solve launch shared with the batch's other small systems;
                            0: it runs as its own amg_solve */
    int32_t smoother;    /* fine-level block smoother of Section 4.5: 0 (default) one forward (R_k) / backward
                            (R_k^t) substitution over each cell's unknowns per color phase; 1 the exact solve of
                            each cell's diagonal block (a dense Cholesky factor per cell made at setup) for cells of
                            at most 32 unknowns, the substitution for larger ones. With 1 the system never takes the
                            whole-solve workgroup of amg_solve_batch. */
    const double *box;   /* host {a1, b1, a2, b2}: the auxiliary box of eq. (5); NULL = bounding box of coords
                            (eq. 6). Points outside a given box are rejected. */
    void *stream;        /* hipStream_t used for every launch; NULL = default stream */
    void *(*alloc)(size_t bytes, void *ctx);  /* device allocator for all of the hierarchy's memory and its calls'
                            temporaries (for example a framework's caching allocator); it returns device memory of
                            the hierarchy's device usable on `stream`, or NULL on failure. NULL (default): the
                            library's own stream-ordered pool and block cache. Set alloc and dealloc together. */
    void (*dealloc)(void *ptr, void *ctx);    /* returns a block of alloc; called once the stream has drained */
    void *ctx;           /* passed to alloc and dealloc */
} amg_options;

typedef struct {
    int32_t iters;       /* outer iterations performed */
    int32_t restarts;    /* restarts from the true residual */
    int32_t status;      /* amg_status of this system's solve (per system in amg_solve_batch) */
    double relres;       /* true relative residual ||b - A x|| / ||b|| of the returned x (FP64) */
    double setup_ms;     /* wall time of amg_setup */
    double solve_ms;     /* wall time of this solve */
} amg_info;

/* Fill *opt with the defaults listed above. */
void amg_default_options(amg_options *opt);

/* Build the hierarchy (Section 3 and Sections 4.2-4.4): auxiliary box (eq. 5-6), depth L = max{l : 4^l < n}
 * (Section 3.1), level-L aggregates by cell index (eq. 9), coarse aggregates by quadtree parent (eq. 10),
 * Galerkin operators A_{k-1} = P^t A_k P (eq. 3-4, eq. 11), 4-coloring (Section 4.5) and the factorised coarsest
 * operator. coords, row_ptr, col_idx, vals: device. opt may be NULL (defaults). On success *out owns all device
 * memory it needs; the inputs may be freed afterwards. Errors: AMG_ERR_INVALID (n < 1, nnz mismatch, row_ptr not
 * monotone, column out of range, non-finite coordinate, a point outside a given box, bad option),
 * AMG_ERR_NOT_SPD, AMG_ERR_NOMEM, AMG_ERR_DEVICE. */
amg_status amg_setup(int64_t n, const double *coords, const int64_t *row_ptr, const int32_t *col_idx,
                     const double *vals, int64_t nnz, const amg_options *opt, amg_hierarchy **out);

/* The octree variant (Sections 1 and 3.1: the region quadtree generalised to three dimensions) for an SPD system from
 * a 3D discretisation: auxiliary box {a1, b1, a2, b2, a3, b3} (host; NULL = bounding box of coords), depth
 * L = max{l : 8^l < n}, level-L aggregates by the cell index of Section 4.2 on each axis, coarse aggregates by
 * octree parent (t1 >> 1, t2 >> 1, t3 >> 1), Galerkin operators with a 27-point pattern (the nine plane offsets of
 * Section 4.4 at dz = 0, +1, -1, self first) plus an overflow list, an 8-coloring (t1 & 1) + 2 (t2 & 1) + 4 (t3 & 1)
 * for the Gauss-Seidel smoother, and the same cycle and outer iteration as amg_setup. The coarsest level is the first
 * k with 8^k <= coarse_max. coords: device, n x 3 interleaved (x, y, z). opt may be NULL; opt->box must be NULL (the
 * box argument replaces it). Octree levels always run one kernel launch per step (options engine and batch have no
 * effect). amg_solve, amg_apply_precond, amg_update_values, amg_export_level (27 slots per row, lexicographic id
 * t1 + 2^k t2 + 4^k t3), amg_level_smooth, amg_level_spmv and amg_free take the hierarchy as for amg_setup. Errors
 * as amg_setup. */
amg_status amg_setup3d(int64_t n, const double *coords, const int64_t *row_ptr, const int32_t *col_idx,
                       const double *vals, int64_t nnz, const double *box, const amg_options *opt,
                       amg_hierarchy **out);

/* Replace the matrix values of h with those of a new matrix on the same sparsity pattern and the same points (a
 * time step with changed coefficients, Example 2 of Section 5): the aggregates of Section 3 depend on the points and
 * the pattern only, so only the numeric part of setup runs again (the Galerkin sums of eq. 11 on every level, the
 * smoother's data, the coarsest factor). The result is bit-identical to amg_setup on the new values with h's
 * points and options. row_ptr, col_idx, vals: device CSR of n rows with exactly the row lengths and, row by row, the
 * column order given to setup; nnz must equal setup's. Borrowed for the call. Blocks until done; later solves report
 * its wall time as setup_ms. Errors, with h unchanged: AMG_ERR_INVALID (h NULL, nnz or the pattern differs, row_ptr
 * not monotone, column out of range), AMG_ERR_NOT_SPD (a diagonal entry <= 0). Errors after the values began to
 * change (AMG_ERR_NOT_SPD from a failed cell or coarsest factor, AMG_ERR_NOMEM, AMG_ERR_DEVICE) leave h holding
 * partial values: solves on it return AMG_ERR_INVALID until an update succeeds. Temporary device memory (the
 * coarsest level's dense matrix and factor scratch, one count per cell of a level, and, when B^ is kept as a matrix,
 * its identity and step list: about 1 MB with the default coarse size) is returned before the call ends; the
 * hierarchy's own footprint does not change. Must not overlap another call on h. */
amg_status amg_update_values(amg_hierarchy *h, const int64_t *row_ptr, const int32_t *col_idx, const double *vals,
                             int64_t nnz);

/* Solve A x = b with the outer flexible CG preconditioned by the nonlinear AMLI-cycle (Algorithms 2.1 and 2.2),
 * from x = 0, until ||r|| <= tol ||b|| holds for the recurrence residual and for the true FP64 residual (the
 * iteration restarts from the true residual when only the former holds). b, x: device, n entries; x is output
 * only. b = 0 gives x = 0 and iters = 0. info may be NULL. Blocks until the solve ends. Errors:
 * AMG_ERR_NOCONV (x = last iterate), AMG_ERR_BREAKDOWN, AMG_ERR_INVALID (tol <= 0 or not finite),
 * AMG_ERR_DEVICE. */
amg_status amg_solve(amg_hierarchy *h, const double *b, double *x, double tol, amg_info *info);

/* Release every resource of h (NULL is allowed). Synchronises the hierarchy's stream first. The device blocks go to
 * a per-device cache owned by the library (at most 32 GiB per device, kept until the process ends) and serve later
 * hierarchies' allocations of exactly the same sizes; blocks beyond the cap return to the driver, and an allocation
 * that fails returns the whole cache to the driver before it tries again. */
void amg_free(amg_hierarchy *h);

/* Change the solve precision of an existing hierarchy (0 = FP64, 1 = FP32 preconditioner / FP64 outer). */
amg_status amg_set_precision(amg_hierarchy *h, int32_t precision);

/* Change the stream used by later calls on h (hipStream_t, NULL = default stream). Work already queued on the
 * previous stream is waited for first, so later calls never race with it. */
amg_status amg_set_stream(amg_hierarchy *h, void *stream);

/* Solve `count` independent systems of one device concurrently (the serving form). h, b, x, tol are host arrays of
 * `count` entries; b[i] and x[i] are device vectors of hierarchy i's size, ready once that hierarchy's stream has
 * drained (the call synchronises each stream first); info is a host array of `count` entries or NULL. The
 * hierarchies must be distinct. Small systems (options.batch, at most 65,536 unknowns) are solved together in one
 * launch, on the stream of the first of them, with one persistent workgroup per system: outer flexible CG,
 * smoother, K-cycle and convergence test all on the device. Every other system is driven by its own host thread on
 * its hierarchy's stream, overlapping with the launch (systems whose hierarchies share a stream run in turn). The
 * call returns when every system is done. A system's result does not depend on the rest of the batch (bit-identical alone and in any mix); the
 * whole-solve workgroup and amg_solve differ only by rounding (different reduction trees). Returns the first
 * non-OK status; every system is attempted. */
amg_status amg_solve_batch(amg_hierarchy *const *h, const double *const *b, double *const *x, const double *tol,
                           int32_t count, amg_info *info);

/* amg_solve_batch for callers that cannot allocate device memory (code under HIP graph capture, serving loops that
 * forbid allocation): the same whole-solve launches and results, with the per-call system descriptors and info words
 * held in a device array of the library's own (about 400 KB per device, kept until the process ends) instead of
 * memory allocated per call. No hipMalloc, hipFree or other allocating call is made. Every system must take the
 * whole-solve route (options.batch = 1, the default fine smoother, at most 65,536 unknowns); count must not exceed
 * 256. Errors, before any device work: AMG_ERR_INVALID for those conditions or the arguments amg_solve_batch
 * rejects. All calls on one device share the array: calls that overlap in time on one device race and must be
 * serialised by the caller. */
amg_status amg_solve_batch_noalloc(amg_hierarchy *const *h, const double *const *b, double *const *x,
                                   const double *tol, int32_t count, amg_info *info);

/* The library keeps the device blocks of freed hierarchies (those allocated from its own pool, not through caller
 * callbacks) in a per-device cache for reuse by the next allocation of exactly the same size; it is emptied whenever
 * one of its own allocations fails. amg_cache_control: limit_bytes >= 0 sets the cache's limit on `device` (default
 * 32 GiB) and returns the blocks beyond it to the driver, oldest first; limit_bytes < 0 leaves it. cached_bytes
 * (may be NULL) receives the bytes the cache holds afterwards. Callers that also allocate device memory outside the
 * library (and admission by memory footprint) bound it this way. AMG_ERR_INVALID for a device outside [0, 64). */
amg_status amg_cache_control(int32_t device, int64_t limit_bytes, size_t *cached_bytes);

/* Upper estimate of the device bytes a hierarchy for an n-unknown, nnz-entry system needs, workspace included
 * (used for admission by memory footprint). */
amg_status amg_estimate_bytes(int64_t n, int64_t nnz, const amg_options *opt, size_t *bytes);

/* Device bytes actually held by h. */
amg_status amg_hierarchy_bytes(const amg_hierarchy *h, size_t *bytes);

/* Number of levels: 1 (direct solve) or 1 + (L - kc + 1): the fine level then quadtree levels L, L-1, ..., kc. */
amg_status amg_num_levels(const amg_hierarchy *h, int32_t *levels);

/* Shape of a level: rows, quadtree level k (-1 for the fine level), overflow entries, depth L. */
amg_status amg_level_info(const amg_hierarchy *h, int32_t level, int64_t *n_rows, int32_t *k, int64_t *ovf_nnz,
                          int32_t *depth_L);

/* Copy a level to host buffers in canonical numbering: the caller's unknown order on the fine level,
 * lexicographic cell ids i = t1 + 2^k t2 (eq. 8) on quadtree levels. Any pointer may be NULL.
 *  level 0: agg[n] = level-L cell of each unknown (eq. 9), color[n] = color of that cell; other arrays ignored.
 *  level >= 1: agg[n] = parent cell on the next coarser level (eq. 10; -1 on the coarsest), color[n],
 *  aj[n*9] row-major in the neighbour order of Section 4.4 [i, i1, ..., i8] (-1 = outside the grid),
 *  ax[n*9] FP64 values (0 where aj = -1), ovf_ptr[n+1] / ovf_col / ovf_val: couplings that reach further than one
 *  cell, sorted by column. Empty aggregates carry the identity row. Synchronises the stream. */
amg_status amg_export_level(const amg_hierarchy *h, int32_t level, int32_t *agg_or_null, uint8_t *color,
                            int32_t *aj, double *ax, int64_t *ovf_ptr, int32_t *ovf_col, double *ovf_val);

/* FP32 values of a quadtree level (n*9, row-major, host): the round-to-nearest image of the FP64 values. */
amg_status amg_export_level_f32(const amg_hierarchy *h, int32_t level, float *ax);

/* Apply the fine-level preconditioner once (Algorithm 2.2 on the finest level): z = B^_F[r]. r, z: device, n
 * entries, caller's numbering. precision as in amg_options. */
amg_status amg_apply_precond(amg_hierarchy *h, const double *r, double *z, int32_t precision);

/* One smoothing sweep on a level (Section 4.5): forward != 0 applies R_k (colors 0..3, forward substitution in
 * each cell), else R_k^t (colors 3..0, backward), updating x in place: x <- x + R (f - A x). f, x: device, in the
 * level's canonical numbering (see amg_export_level). Not valid on the coarsest level or a single-level
 * hierarchy. */
amg_status amg_level_smooth(amg_hierarchy *h, int32_t level, const double *f, double *x, int32_t forward,
                            int32_t precision);

/* y = A_level x, device vectors in the level's canonical numbering. */
amg_status amg_level_spmv(amg_hierarchy *h, int32_t level, const double *x, double *y, int32_t precision);

/* Kernel timing of one named kernel family for roofline measurement: while enabled, every launch of that
 * kernel on h's stream is bracketed by HIP events; amg_kernel_timing_read returns the number of launches and
 * their summed device time since the last enable. name: "spmv64" (outer FP64 sliced-ELL SpMV), "gs_fine32",
 * "gs_fine64" (fine-level smoother residual pass), "resid_fine32", "resid_fine64", "engine32", "engine64" (the
 * persistent small-level workgroup of that precision). name NULL disables. bytes_per_launch is the kernel's
 * algorithmic HBM bytes per launch; for the engine kinds it is its algorithmic floating-point operations per
 * launch instead (the engine works out of LDS and L2). Timing one family takes up to 4,096 launches; later
 * launches run untimed. */
amg_status amg_kernel_timing_enable(amg_hierarchy *h, const char *name);
amg_status amg_kernel_timing_read(amg_hierarchy *h, int64_t *launches, double *total_ms, double *bytes_per_launch);

/* Configuration of the persistent small-level workgroup for a precision: the hierarchy level index of its top
 * (-1 = not used), the first level index whose operators live in LDS, the length of its step list and its dynamic
 * LDS bytes. */
amg_status amg_engine_info(const amg_hierarchy *h, int32_t precision, int32_t *top_level, int32_t *lds_level,
                           int32_t *steps, size_t *lds_bytes);

/* Human-readable name of a status. */
/* ---- P1 assembly on the device (the step before the hierarchy in time stepping) ----
 * Stiffness matrix of -div(kappa grad u) with linear triangles: element entries kappa_T (E_a . E_b) / (4 |T|), E_a
 * the edge opposite vertex a, summed per (row, column) over the triangles sharing both vertices, with every vertex
 * pair of a triangle stored (zero values included). Unknowns are the vertices with dof[v] >= 0, numbered dof[v];
 * rows and columns of the others (eliminated Dirichlet vertices) are dropped. Columns ascend inside each row. The
 * summation order is fixed (see qa_assemble.hip), so repeated assembly is bit-identical. Example 2 of Section 5
 * solves one such system per time step; the pattern is built once and each step assembles new values. */
typedef struct amg_p1_mesh amg_p1_mesh;

/* Build the pattern of a triangle mesh on the current device. points: device, nv x 2 (x, y interleaved); tris:
 * device, nt x 3 vertex ids (either orientation); dof: device, nv entries, -1 or an unknown index in [0, ndof), each
 * index used once. The handle copies what it needs (inputs borrowed for the call) and keeps about 12 bytes per
 * element entry (9 per triangle) for later assembly. stream: hipStream_t of all its work. Calls on one handle must
 * not overlap (assembly uses the handle's element buffer). Errors: AMG_ERR_INVALID (sizes, a vertex id out
 * of range, a degenerate triangle, a bad dof map, an entry summing more than 128 element entries), AMG_ERR_NOMEM,
 * AMG_ERR_DEVICE. */
amg_status amg_p1_mesh_create(int64_t nv, const double *points, int64_t nt, const int32_t *tris, const int32_t *dof,
                              int64_t ndof, void *stream, amg_p1_mesh **out);

/* The pattern: *nnz (host), and, where not NULL, row_ptr (device, ndof + 1) and col_idx (device, nnz) copied out. */
amg_status amg_p1_mesh_pattern(const amg_p1_mesh *m, int64_t *nnz, int64_t *row_ptr, int32_t *col_idx);

/* Values for per-triangle coefficients kappa (device, nt entries in the order of tris; NULL = 1) into vals (device,
 * nnz, the order of the pattern). Blocks until done. Errors: AMG_ERR_INVALID (NULL handle or vals). */
amg_status amg_p1_assemble(amg_p1_mesh *m, const double *kappa, double *vals);

/* Release the handle and its device memory (NULL is allowed). */
void amg_p1_mesh_free(amg_p1_mesh *m);

const char *amg_status_string(amg_status s);

#ifdef __cplusplus
}
#endif
#endif
