/* Oracle of the auxiliary-grid AMG method (Wang, Hu, Cohen, Xu: "A Parallel Auxiliary Grid AMG Method for GPU").
 *
 * TEST INFRASTRUCTURE ONLY. This is a plain, slow, single-threaded FP64 CPU implementation written from the paper's
 * equations and algorithms. Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it. It shares no code, header, table or helper with the HIP library.
 *
 * Numbering: the fine level keeps the caller's unknown numbering; quadtree level k uses the lexicographic cell id
 * i = t1 + 2^k t2 of Section 3.1 (eq. 8). Exported 9-slot rows use the neighbour order of Section 4.4
 * [self, i1..i8] = offsets (0,0),(1,0),(1,1),(0,1),(-1,1),(-1,0),(-1,-1),(0,-1),(1,-1), -1 for a missing neighbour.
 */
#ifndef QUADAMG_ORACLE_H
#define QUADAMG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_INVALID = 1, ORC_NOMEM = 2, ORC_NOT_SPD = 4, ORC_BREAKDOWN = 5, ORC_NOCONV = 6 };

typedef struct orc_h orc_h;

/* Depth rule of Section 3.1: single level when n <= coarse_max, else L = max{l : 4^l < n}; the coarsest quadtree
 * level is the first k (counting down from L) with 4^k <= coarse_max. Returns the number of levels (fine + quadtree
 * levels L..kc), or 1. */
int orc_depth(int64_t n, int coarse_max, int *L, int *kc);
/* The same for dim = 2 (quadtree, 4^l) or dim = 3 (octree, 8^l; the paper's 3D generalisation, Section 3.1). */
int orc_depth_dim(int64_t n, int dim, int coarse_max, int *L, int *kc);

/* Level-L aggregation of Section 4.2 (eq. 9): lexicographic cell id of each point. box = {a1,b1,a2,b2}. */
void orc_cell_index(int64_t n, const double *coords, const double *box, int L, int32_t *cell);
/* The same in dim dimensions: coords n x dim, box {a1,b1,a2,b2[,a3,b3]}, id (t3 2^L + t2) 2^L + t1. */
void orc_cell_index_dim(int64_t n, int dim, const double *coords, const double *box, int L, int32_t *cell);

/* Setup (Section 3, Section 4.2-4.4). coords n x 2 interleaved, CSR 0-based. box NULL = bounding box of coords.
 * Returns ORC_* and *out = NULL on failure. */
int orc_setup(int64_t n, const double *coords, const int64_t *row_ptr, const int32_t *col, const double *val,
              const double *box, int coarse_max, int inner_iters, int sweeps, orc_h **out);
/* The same for dim = 2 or 3 (octree: 8^k cells per level, 27 coarse slots, 8 colors): coords n x dim, box
 * {a1,b1,a2,b2[,a3,b3]}. orc_setup is orc_setup_dim with dim = 2. */
int orc_setup_dim(int64_t n, int dim, const double *coords, const int64_t *row_ptr, const int32_t *col,
                  const double *val, const double *box, int coarse_max, int inner_iters, int sweeps, orc_h **out);
void orc_free(orc_h *h);

/* Outer flexible CG (Algorithm 2.1 with the K-cycle of Algorithm 2.2 as preconditioner), x0 = 0, stop when
 * ||r|| <= tol ||b||. mmax = number of kept directions (-1 = all). */
int orc_solve(orc_h *h, const double *b, double *x, double tol, int max_iters, int mmax, int *iters,
              double *relres);

/* One application of the fine-level K-cycle preconditioner B^_F (Algorithm 2.2). */
int orc_apply_precond(orc_h *h, const double *r, double *z);

int orc_num_levels(const orc_h *h);
int orc_dim(const orc_h *h);
/* n rows, quadtree level k (-1 for the fine level), overflow entry count, depth L. */
int orc_level_info(const orc_h *h, int level, int64_t *n, int *k, int64_t *ovf_nnz, int *L);
/* Export in lexicographic numbering. level 0: agg = level-L cell per unknown, color per unknown (aj/ax ignored).
 * level >= 1: agg = parent cell at the next coarser level (NULL allowed; undefined on the coarsest), color per
 * cell, aj/ax n x 9 row-major (n x 27 in 3D: the 9-slot order at dz = 0, +1, -1), overflow CSR sorted by column.
 * Any pointer may be NULL. */
int orc_export_level(const orc_h *h, int level, int32_t *agg, uint8_t *color, int32_t *aj, double *ax,
                     int64_t *ovf_ptr, int32_t *ovf_col, double *ovf_val);
/* One smoothing sweep at a level on vectors in that level's numbering: forward = R (colors 0..3, forward
 * substitution inside cells), else R^t (colors 3..0, backward). x is updated in place. */
int orc_smooth(orc_h *h, int level, const double *f, double *x, int forward);
/* The other reading of the fine smoother (Section 4.5): on = 1 makes each cell of at most ORC_BLOCK_MAX unknowns
 * take the exact solve of its diagonal block in every color phase (a dense Cholesky factor per cell, made on the
 * first call); larger cells keep the forward / backward substitution. on = 0 returns to the substitution. */
#define ORC_BLOCK_MAX 32
int orc_set_block_smoother(orc_h *h, int on);
/* y = A_level x */
int orc_level_spmv(orc_h *h, int level, const double *x, double *y);

/* Transfer between level `level` and level + 1 (Section 4.3), vectors in those levels' numberings:
 * fc = P^t r (sum over each aggregate), u += P e (each unknown takes its aggregate's value). */
int orc_restrict(orc_h *h, int level, const double *r, double *fc);
int orc_prolong_add(orc_h *h, int level, const double *e, double *u);
/* Test knob: after `at_iter` iterations of the next orc_solve the recurrence residual is set to zero once (0 = off),
 * so the true-residual check and the restart from the true residual are exercised. */
void orc_test_force_restart(int at_iter);

/* Test hook: Algorithm 2.1 with n steps on a CSR matrix and a trivial preconditioner: mode 0 = identity,
 * mode 1 = exact inverse (dense Cholesky; small n only). */
int orc_nlpcg_test(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val, const double *f,
                   int nsteps, int mode, double *u);

#ifdef __cplusplus
}
#endif
#endif
