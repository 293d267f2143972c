/* Oracle of the auxiliary-grid AMG method: plain single-threaded FP64 C, written from the paper.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the benchmark's CPU-baseline leg; never
 * by the HIP library, which shares no code with it. Build with -O2 -ffp-contract=off (no fused multiply-add, no
 * fast-math), so every floating-point step is the plain IEEE operation written here.
 *
 * Readings taken where the paper is silent, ambiguous or garbled:
 *  R1 depth (Section 3.1): L = max{l : 4^l < N} (the stated strict constraint), not floor(log N / log 4); they
 *     differ only when N is a power of 4. Single level when N <= coarse_max.
 *  R2 cell index (Section 4.2, level-L listing): t = (x - a1)/(b1 - a1) in IEEE double, then floor(t * 2^L),
 *     clamped to 2^L - 1 so that points on the top/right edge of the box fall in the last cell; a degenerate box
 *     side (b1 == a1) puts every point in cell column 0.
 *  R3 coarse aggregation (eq. 10 and the coarse-level listing): parent(t1, t2) = (t1 >> 1, t2 >> 1).
 *  R4 empty cells: a cell without fine unknowns (or whose four children are all empty) keeps an identity row
 *     (diagonal 1, all couplings 0) and is skipped when the next coarser operator is summed.
 *  R5 pattern (Section 4.4): 9 slots in the paper's neighbour order, present iff the neighbour lies in the grid,
 *     even when the summed value is 0. Couplings that reach further than one cell (graded meshes) are kept in a
 *     per-row overflow list sorted by column.
 *  R6 summation order of eq. (4)/(11): cells in lexicographic order; inside a level-L cell its unknowns ascending,
 *     each row's entries in CSR order; below level L the four children in the order of the explicit restriction
 *     formula of Section 4.3 ((2t1,2t2), (2t1+1,2t2), (2t1+1,2t2+1), (2t1,2t2+1)), each child's 9 slots in slot
 *     order then its overflow entries.
 *  R7 smoother (Section 4.5): 4 colors, color = (t1 & 1) + 2 (t2 & 1). One sweep of R_k: for colors 0,1,2,3 the
 *     residual of that color's unknowns is taken with x as at the start of the color phase, then every cell of
 *     the color does one forward substitution over its unknowns in ascending index (a Gauss-Seidel pass inside
 *     the block) and adds the correction. R_k^t runs colors 3,2,1,0 with backward substitution. On quadtree levels
 *     each cell is one unknown, so the substitution is a division by the diagonal.
 *  R8 K-cycle (Algorithm 2.2): the coarse correction reads P B~[P^t (f - A u1)] (the printed transposes are
 *     swapped), pre-smoothing starts from zero, the coarsest level is solved exactly by Cholesky.
 *  R9 inner nonlinear PCG (Algorithm 2.1): n = inner_iters steps (2 = K-cycle), classical Gram-Schmidt against all
 *     earlier directions, and a step whose (p, Ap) <= 0 ends the iteration with the current iterate.
 *  R10 outer iteration: Algorithm 2.1 as a flexible CG at the fine level keeping the last mmax directions; stop on
 *     the recurrence residual ||r|| <= tol ||b||, confirm with the true residual, restart from it if it fails.
 *  R11 the other reading of "block-wise Gauss-Seidel" (Section 4.5), optional (orc_set_block_smoother): the cells
 *     of a color phase take the exact solve of their diagonal block, u_cell += A_cc^{-1} r_cell, through a dense
 *     Cholesky factor made once (the block in ascending unknown order, entries summed in CSR order); R_k and R_k^t
 *     then differ only in the color order. Cells of more than ORC_BLOCK_MAX unknowns keep the substitution of R7.
 *  R12 the octree (3D) variant, which the paper states only as the generalisation of the quadtree (Sections 1 and
 *     3.1: an octree, 8^L aggregates, a 27-point coarse stencil): depth L = max{l : 8^l < N} (the strict reading of
 *     R1), coarsest = first k with 8^k <= coarse_max; cell id (t3 2^k + t2) 2^k + t1; parent (t1>>1, t2>>1, t3>>1);
 *     27 slots = the 9-slot plane order of Section 4.4 at dz = 0, then at dz = +1, then at dz = -1 (self first, as
 *     Section 4.1 puts the diagonal first); 8 colors (t1 & 1) + 2 (t2 & 1) + 4 (t3 & 1), valid when couplings reach
 *     one cell; children summed in the 2D order on the lower layer (2 t3), then the same on the upper layer.
 *     Everything else (smoother, cycle, outer iteration) is the 2D method with 2^d colors and 2^d children.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* neighbour offsets of Section 4.4: self, E, NE, N, NW, W, SW, S, SE; in 3D (R12) slot 9 z + t is plane offset t at
 * dz = 0, +1, -1 for z = 0, 1, 2 */
static const int ODX[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
static const int ODY[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
static const int ODZ[3] = {0, 1, -1};
static int slot_dx(int t) { return ODX[t % 9]; }
static int slot_dy(int t) { return ODY[t % 9]; }
static int slot_dz(int t) { return ODZ[t / 9]; }

typedef struct {
    int64_t n;      /* 4^k rows (8^k in 3D) */
    int k;          /* quadtree level */
    int64_t side;   /* 2^k */
    int dim;        /* 2 or 3 */
    int ns;         /* slots per row: 9 or 27 */
    int32_t *aj;    /* n x ns, lexicographic neighbour id or -1 */
    double *ax;     /* n x ns */
    int64_t *optr;  /* overflow CSR (n + 1) */
    int32_t *ocol;
    double *oval;
    uint8_t *empty;
} olev;

struct orc_h {
    int dim;         /* 2: quadtree, 3: octree (R12) */
    int ns, nchild;  /* slots per coarse row (9 / 27), children per cell and colors (4 / 8) */
    int64_t n, nnz;
    int64_t *rp;
    int32_t *ci;
    double *va, *diag;
    int L, kc, nlev;
    double box[6];
    int32_t *cell;   /* fine unknown -> level-L cell */
    int64_t *cstart; /* cell -> first position in cdofs (4^L + 1) */
    int32_t *cdofs;  /* unknowns grouped by cell, ascending inside a cell */
    olev *lev;       /* lev[1 .. nlev-1] are quadtree levels L, L-1, ..., kc */
    double *chol;    /* Cholesky factor of the coarsest level, row-major lower */
    int64_t nc;
    int inner, sweeps;
    int block;       /* R11: exact block solves on cells of at most ORC_BLOCK_MAX unknowns */
    int64_t *boff;   /* cell -> offset of its m x m factor in bfac (4^L + 1) */
    double *bfac;
};

/* cells of a level-k grid in d dimensions: (2^d)^k */
static int64_t ncells(int dim, int k) { return (int64_t)1 << (dim * k); }

int orc_depth_dim(int64_t n, int dim, int coarse_max, int *L, int *kc) {
    if (coarse_max < 1) coarse_max = 1;
    if (n <= coarse_max) {
        *L = -1; *kc = -1;
        return 1;
    }
    int l = 0;
    while (ncells(dim, l + 1) < n) l++;
    int k = l;
    while (k > 0 && ncells(dim, k) > coarse_max) k--;
    *L = l; *kc = k;
    return 1 + (l - k + 1);
}

int orc_depth(int64_t n, int coarse_max, int *L, int *kc) { return orc_depth_dim(n, 2, coarse_max, L, kc); }

static int32_t axis_index(double v, double a, double b, int64_t s) {
    if (!(b > a)) return 0;
    double t = (v - a) / (b - a);
    double f = floor(t * (double)s);
    int64_t i = (int64_t)f;
    if (i > s - 1) i = s - 1;
    if (i < 0) i = 0;
    return (int32_t)i;
}

void orc_cell_index_dim(int64_t n, int dim, const double *coords, const double *box, int L, int32_t *cell) {
    int64_t s = (int64_t)1 << L;
    for (int64_t i = 0; i < n; i++) {
        int64_t id = 0;
        for (int a = dim - 1; a >= 0; a--)  /* (t3 s + t2) s + t1 */
            id = id * s + axis_index(coords[dim * i + a], box[2 * a], box[2 * a + 1], s);
        cell[i] = (int32_t)id;
    }
}

void orc_cell_index(int64_t n, const double *coords, const double *box, int L, int32_t *cell) {
    orc_cell_index_dim(n, 2, coords, box, L, cell);
}

/* grid coordinates (t1, t2, t3) of lexicographic cell I on a level of side s (t3 = 0 in 2D) */
static void cell_coords(int64_t I, int64_t s, int64_t t[3]) {
    t[0] = I % s;
    t[1] = (I / s) % s;
    t[2] = I / (s * s);
}

/* ------------------------------------------------------------------------------------------------------------ */
/* dense Cholesky (coarsest level, Algorithm 2.2's A_1^{-1})                                                      */

static int cholesky(double *a, int64_t n) {
    for (int64_t j = 0; j < n; j++) {
        double d = a[j * n + j];
        for (int64_t k = 0; k < j; k++) d -= a[j * n + k] * a[j * n + k];
        if (!(d > 0.0)) return ORC_NOT_SPD;
        double ljj = sqrt(d);
        a[j * n + j] = ljj;
        for (int64_t i = j + 1; i < n; i++) {
            double s = a[i * n + j];
            for (int64_t k = 0; k < j; k++) s -= a[i * n + k] * a[j * n + k];
            a[i * n + j] = s / ljj;
        }
        for (int64_t i = 0; i < j; i++) a[i * n + j] = 0.0;
    }
    return ORC_OK;
}

static void chol_solve(const double *l, int64_t n, const double *f, double *u) {
    for (int64_t i = 0; i < n; i++) {
        double s = f[i];
        for (int64_t k = 0; k < i; k++) s -= l[i * n + k] * u[k];
        u[i] = s / l[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; i--) {
        double s = u[i];
        for (int64_t k = i + 1; k < n; k++) s -= l[k * n + i] * u[k];
        u[i] = s / l[i * n + i];
    }
}

/* ------------------------------------------------------------------------------------------------------------ */
/* Galerkin construction (eq. 3-4 and eq. 11)                                                                     */

typedef struct {
    int32_t *col;
    double *val;
    int64_t cnt, cap;
} rowbuf;

typedef struct {
    int32_t *col;
    double *val;
    int64_t cnt, cap;
} ovfstore;

static int rowbuf_add(rowbuf *b, int32_t c, double v) {
    for (int64_t e = 0; e < b->cnt; e++)
        if (b->col[e] == c) {
            b->val[e] += v;
            return 0;
        }
    if (b->cnt == b->cap) {
        int64_t nc = b->cap ? 2 * b->cap : 16;
        int32_t *c2 = realloc(b->col, nc * sizeof(int32_t));
        if (!c2) return -1;
        b->col = c2;
        double *v2 = realloc(b->val, nc * sizeof(double));
        if (!v2) return -1;
        b->val = v2;
        b->cap = nc;
    }
    b->col[b->cnt] = c;
    b->val[b->cnt] = v;
    b->cnt++;
    return 0;
}

static int ovf_flush(ovfstore *s, rowbuf *b) {
    /* sort the row's overflow entries by column (insertion sort; columns are distinct) */
    for (int64_t i = 1; i < b->cnt; i++) {
        int32_t c = b->col[i];
        double v = b->val[i];
        int64_t j = i - 1;
        while (j >= 0 && b->col[j] > c) {
            b->col[j + 1] = b->col[j];
            b->val[j + 1] = b->val[j];
            j--;
        }
        b->col[j + 1] = c;
        b->val[j + 1] = v;
    }
    if (s->cnt + b->cnt > s->cap) {
        int64_t nc = s->cap ? 2 * s->cap : 64;
        while (nc < s->cnt + b->cnt) nc *= 2;
        int32_t *c2 = realloc(s->col, nc * sizeof(int32_t));
        if (!c2) return -1;
        s->col = c2;
        double *v2 = realloc(s->val, nc * sizeof(double));
        if (!v2) return -1;
        s->val = v2;
        s->cap = nc;
    }
    for (int64_t e = 0; e < b->cnt; e++) {
        s->col[s->cnt + e] = b->col[e];
        s->val[s->cnt + e] = b->val[e];
    }
    s->cnt += b->cnt;
    b->cnt = 0;
    return 0;
}

/* add coupling value v between cell I and cell J of a level: a stencil slot or the overflow row */
static int add_coupling(olev *lv, int64_t I, int64_t J, double v, rowbuf *ob) {
    int64_t ti[3], tj[3];
    cell_coords(I, lv->side, ti);
    cell_coords(J, lv->side, tj);
    int64_t dx = tj[0] - ti[0], dy = tj[1] - ti[1], dz = tj[2] - ti[2];
    if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) {
        for (int t = 0; t < lv->ns; t++)
            if (slot_dx(t) == dx && slot_dy(t) == dy && slot_dz(t) == dz) {
                lv->ax[I * lv->ns + t] += v;
                return 0;
            }
    }
    return rowbuf_add(ob, (int32_t)J, v);
}

static int level_alloc(olev *lv, int k, int dim) {
    lv->k = k;
    lv->dim = dim;
    lv->ns = dim == 3 ? 27 : 9;
    lv->side = (int64_t)1 << k;
    lv->n = ncells(dim, k);
    lv->aj = malloc(lv->n * lv->ns * sizeof(int32_t));
    lv->ax = calloc(lv->n * lv->ns, sizeof(double));
    lv->optr = calloc(lv->n + 1, sizeof(int64_t));
    lv->empty = calloc(lv->n, 1);
    lv->ocol = NULL;
    lv->oval = NULL;
    if (!lv->aj || !lv->ax || !lv->optr || !lv->empty) return ORC_NOMEM;
    int64_t s = lv->side;
    for (int64_t I = 0; I < lv->n; I++) {
        int64_t t[3];
        cell_coords(I, s, t);
        for (int q = 0; q < lv->ns; q++) {
            int64_t u1 = t[0] + slot_dx(q), u2 = t[1] + slot_dy(q), u3 = t[2] + slot_dz(q);
            int in = u1 >= 0 && u1 < s && u2 >= 0 && u2 < s && u3 >= 0 && (dim == 2 ? u3 == 0 : u3 < s);
            lv->aj[I * lv->ns + q] = in ? (int32_t)((u3 * s + u2) * s + u1) : -1;
        }
    }
    return ORC_OK;
}

/* eq. (10): the parent (t1 >> 1, t2 >> 1[, t3 >> 1]) on the level of side s / 2 */
static int64_t parent_of(int64_t J, int64_t side) {
    int64_t t[3], h = side >> 1;
    cell_coords(J, side, t);
    return ((t[2] >> 1) * h + (t[1] >> 1)) * h + (t[0] >> 1);
}

/* child c (0 .. 2^d - 1) of coarse cell (T1, T2, T3), in the order of Section 4.3's restriction formula:
 * (2T1, 2T2), (2T1+1, 2T2), (2T1+1, 2T2+1), (2T1, 2T2+1) on the layer 2 T3, then the same on the layer 2 T3 + 1 */
static int64_t child_of(const int64_t T[3], int c, int64_t fine_side) {
    static const int CX[4] = {0, 1, 1, 0}, CY[4] = {0, 0, 1, 1};
    int64_t t1 = 2 * T[0] + CX[c & 3], t2 = 2 * T[1] + CY[c & 3], t3 = 2 * T[2] + (c >> 2);
    return (t3 * fine_side + t2) * fine_side + t1;
}

/* fine CSR -> level L: (A_L)_{IJ} = sum_{i in G_I} sum_{j in G_J} a_ij */
static int galerkin_fine(orc_h *h, olev *lv) {
    rowbuf ob = {0};
    ovfstore os = {0};
    int st = ORC_OK;
    for (int64_t I = 0; I < lv->n; I++) {
        lv->empty[I] = (h->cstart[I + 1] == h->cstart[I]);
        for (int64_t a = h->cstart[I]; a < h->cstart[I + 1]; a++) {
            int32_t i = h->cdofs[a];
            for (int64_t e = h->rp[i]; e < h->rp[i + 1]; e++)
                if (add_coupling(lv, I, h->cell[h->ci[e]], h->va[e], &ob)) { st = ORC_NOMEM; goto out; }
        }
        if (ovf_flush(&os, &ob)) { st = ORC_NOMEM; goto out; }
        lv->optr[I + 1] = os.cnt;
        if (lv->empty[I]) lv->ax[I * lv->ns] = 1.0;
    }
    lv->ocol = os.col;
    lv->oval = os.val;
    os.col = NULL; os.val = NULL;
out:
    free(ob.col); free(ob.val); free(os.col); free(os.val);
    return st;
}

/* level k -> level k-1: sums over the 2^d children (the action of restriction, Section 4.4) */
static int galerkin_coarse(const olev *fl, olev *lv) {
    rowbuf ob = {0};
    ovfstore os = {0};
    int st = ORC_OK;
    const int nchild = 1 << lv->dim;
    for (int64_t I = 0; I < lv->n; I++) {
        int64_t T[3];
        cell_coords(I, lv->side, T);
        int all_empty = 1;
        for (int c = 0; c < nchild; c++) {
            int64_t C = child_of(T, c, fl->side);
            if (fl->empty[C]) continue;
            all_empty = 0;
            for (int t = 0; t < fl->ns; t++) {
                int32_t J = fl->aj[C * fl->ns + t];
                if (J < 0) continue;
                if (add_coupling(lv, I, parent_of(J, fl->side), fl->ax[C * fl->ns + t], &ob)) { st = ORC_NOMEM; goto out; }
            }
            for (int64_t e = fl->optr[C]; e < fl->optr[C + 1]; e++)
                if (add_coupling(lv, I, parent_of(fl->ocol[e], fl->side), fl->oval[e], &ob)) { st = ORC_NOMEM; goto out; }
        }
        lv->empty[I] = (uint8_t)all_empty;
        if (ovf_flush(&os, &ob)) { st = ORC_NOMEM; goto out; }
        lv->optr[I + 1] = os.cnt;
        if (all_empty) lv->ax[I * lv->ns] = 1.0;
    }
    lv->ocol = os.col;
    lv->oval = os.val;
    os.col = NULL; os.val = NULL;
out:
    free(ob.col); free(ob.val); free(os.col); free(os.val);
    return st;
}

/* ------------------------------------------------------------------------------------------------------------ */
/* level operators                                                                                                */

static int64_t level_n(const orc_h *h, int l) { return l == 0 ? h->n : h->lev[l].n; }

/* color (t1 & 1) + 2 (t2 & 1) [+ 4 (t3 & 1)] of a lexicographic cell (Section 4.5; R12 in 3D) */
static int cell_color_lex(int64_t I, int64_t side) {
    int64_t t[3];
    cell_coords(I, side, t);
    return (int)(t[0] & 1) + 2 * (int)(t[1] & 1) + 4 * (int)(t[2] & 1);
}

static double row_dot(const orc_h *h, int l, int64_t i, const double *x) {
    double acc = 0.0;
    if (l == 0) {
        for (int64_t e = h->rp[i]; e < h->rp[i + 1]; e++) acc += h->va[e] * x[h->ci[e]];
    } else {
        const olev *lv = &h->lev[l];
        for (int t = 0; t < lv->ns; t++) {
            int32_t J = lv->aj[i * lv->ns + t];
            if (J >= 0) acc += lv->ax[i * lv->ns + t] * x[J];
        }
        for (int64_t e = lv->optr[i]; e < lv->optr[i + 1]; e++) acc += lv->oval[e] * x[lv->ocol[e]];
    }
    return acc;
}

static void spmv(const orc_h *h, int l, const double *x, double *y) {
    int64_t n = level_n(h, l);
    for (int64_t i = 0; i < n; i++) y[i] = row_dot(h, l, i, x);
}

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* one colored sweep (reading R7); r and d are scratch vectors of the level's size */
static void smooth(const orc_h *h, int l, const double *f, double *x, int forward, double *r, double *d) {
    for (int ph = 0; ph < h->nchild; ph++) {
        int c = forward ? ph : h->nchild - 1 - ph;
        if (l == 0) {
            int64_t nL = ncells(h->dim, h->L), sL = (int64_t)1 << h->L;
            for (int64_t I = 0; I < nL; I++) {
                if (cell_color_lex(I, sL) != c) continue;
                for (int64_t a = h->cstart[I]; a < h->cstart[I + 1]; a++) {
                    int32_t i = h->cdofs[a];
                    r[i] = f[i] - row_dot(h, 0, i, x);
                }
            }
            for (int64_t I = 0; I < nL; I++) {
                if (cell_color_lex(I, sL) != c) continue;
                int64_t a0 = h->cstart[I], a1 = h->cstart[I + 1];
                if (h->block && a1 - a0 <= ORC_BLOCK_MAX) { /* R11: exact solve of the cell's block */
                    double rc[ORC_BLOCK_MAX], dc[ORC_BLOCK_MAX];
                    int64_t m = a1 - a0;
                    for (int64_t a = 0; a < m; a++) rc[a] = r[h->cdofs[a0 + a]];
                    chol_solve(h->bfac + h->boff[I], m, rc, dc);
                    for (int64_t a = 0; a < m; a++) x[h->cdofs[a0 + a]] += dc[a];
                    continue;
                }
                for (int64_t q = 0; q < a1 - a0; q++) {
                    int32_t i = h->cdofs[forward ? a0 + q : a1 - 1 - q];
                    double acc = r[i];
                    for (int64_t e = h->rp[i]; e < h->rp[i + 1]; e++) {
                        int32_t j = h->ci[e];
                        if (j == i || h->cell[j] != (int32_t)I) continue;
                        if (forward ? (j < i) : (j > i)) acc -= h->va[e] * d[j];
                    }
                    d[i] = acc / h->diag[i];
                }
                for (int64_t a = a0; a < a1; a++) x[h->cdofs[a]] += d[h->cdofs[a]];
            }
        } else {
            const olev *lv = &h->lev[l];
            for (int64_t I = 0; I < lv->n; I++)
                if (cell_color_lex(I, lv->side) == c) r[I] = f[I] - row_dot(h, l, I, x);
            for (int64_t I = 0; I < lv->n; I++)
                if (cell_color_lex(I, lv->side) == c) x[I] += r[I] / lv->ax[I * lv->ns];
        }
    }
}

/* f_c = P^t r (Section 4.3): level l -> level l+1 */
static void restrict_res(const orc_h *h, int l, const double *r, double *fc) {
    const olev *cl = &h->lev[l + 1];
    if (l == 0) {
        for (int64_t I = 0; I < cl->n; I++) {
            double acc = 0.0;
            for (int64_t a = h->cstart[I]; a < h->cstart[I + 1]; a++) acc += r[h->cdofs[a]];
            fc[I] = acc;
        }
    } else {
        const olev *fl = &h->lev[l];
        for (int64_t I = 0; I < cl->n; I++) {
            int64_t T[3];
            cell_coords(I, cl->side, T);
            double acc = 0.0;
            for (int c = 0; c < h->nchild; c++) acc += r[child_of(T, c, fl->side)];
            fc[I] = acc;
        }
    }
}

/* u += P e (Section 4.3): level l+1 -> level l */
static void prolong_add(const orc_h *h, int l, const double *e, double *u) {
    if (l == 0) {
        for (int64_t i = 0; i < h->n; i++) u[i] += e[h->cell[i]];
    } else {
        const olev *fl = &h->lev[l];
        for (int64_t I = 0; I < fl->n; I++) u[I] += e[parent_of(I, fl->side)];
    }
}

/* ------------------------------------------------------------------------------------------------------------ */
/* Algorithm 2.1 (nonlinear PCG) with operator callbacks                                                          */

typedef struct {
    void (*apply)(void *ctx, const double *in, double *out);
    void *ctx;
} op_t;

static int nlpcg(int64_t n, op_t A, op_t B, const double *f, int nsteps, double *u) {
    double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double));
    double *P = malloc((size_t)nsteps * n * sizeof(double)), *Q = malloc((size_t)nsteps * n * sizeof(double));
    double *D = malloc((size_t)nsteps * sizeof(double)), *beta = malloc((size_t)nsteps * sizeof(double));
    if (!r || !z || !P || !Q || !D || !beta) {
        free(r); free(z); free(P); free(Q); free(D); free(beta);
        return ORC_NOMEM;
    }
    for (int64_t i = 0; i < n; i++) { u[i] = 0.0; r[i] = f[i]; }
    for (int i = 0; i < nsteps; i++) {
        double *p = P + (size_t)i * n, *q = Q + (size_t)i * n;
        B.apply(B.ctx, r, z);
        for (int j = 0; j < i; j++) beta[j] = -dot(n, z, Q + (size_t)j * n) / D[j];
        for (int64_t t = 0; t < n; t++) p[t] = z[t];
        for (int j = 0; j < i; j++)
            for (int64_t t = 0; t < n; t++) p[t] += beta[j] * P[(size_t)j * n + t];
        A.apply(A.ctx, p, q);
        D[i] = dot(n, p, q);
        if (!(D[i] > 0.0)) break;
        double alpha = dot(n, r, p) / D[i];
        for (int64_t t = 0; t < n; t++) {
            u[t] += alpha * p[t];
            r[t] -= alpha * q[t];
        }
    }
    free(r); free(z); free(P); free(Q); free(D); free(beta);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------------------------------ */
/* Algorithm 2.2 (nonlinear AMLI-cycle)                                                                           */

typedef struct {
    orc_h *h;
    int l;
} lctx;

static int bhat(orc_h *h, int l, const double *f, double *u);

static void op_spmv(void *c, const double *in, double *out) {
    lctx *x = c;
    spmv(x->h, x->l, in, out);
}
static void op_bhat(void *c, const double *in, double *out) {
    lctx *x = c;
    bhat(x->h, x->l, in, out);
}

static int bhat(orc_h *h, int l, const double *f, double *u) {
    int64_t n = level_n(h, l);
    if (l == h->nlev - 1) {
        chol_solve(h->chol, h->nc, f, u);
        return ORC_OK;
    }
    int64_t nc = level_n(h, l + 1);
    double *r = malloc(n * sizeof(double)), *d = malloc(n * sizeof(double));
    double *fc = malloc(nc * sizeof(double)), *ec = malloc(nc * sizeof(double));
    if (!r || !d || !fc || !ec) {
        free(r); free(d); free(fc); free(ec);
        return ORC_NOMEM;
    }
    /* pre-smoothing u1 = R_k f (from zero) */
    for (int64_t i = 0; i < n; i++) u[i] = 0.0;
    for (int s = 0; s < h->sweeps; s++) smooth(h, l, f, u, 1, r, d);
    /* coarse-grid correction u2 = u1 + P B~[P^t (f - A u1)] */
    spmv(h, l, u, r);
    for (int64_t i = 0; i < n; i++) r[i] = f[i] - r[i];
    restrict_res(h, l, r, fc);
    if (l + 1 == h->nlev - 1) {
        chol_solve(h->chol, h->nc, fc, ec);
    } else {
        lctx c = {h, l + 1};
        op_t A = {op_spmv, &c}, B = {op_bhat, &c};
        int st = nlpcg(nc, A, B, fc, h->inner, ec);
        if (st) { free(r); free(d); free(fc); free(ec); return st; }
    }
    prolong_add(h, l, ec, u);
    /* post-smoothing u2 + R_k^t (f - A u2) */
    for (int s = 0; s < h->sweeps; s++) smooth(h, l, f, u, 0, r, d);
    free(r); free(d); free(fc); free(ec);
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------------------------------ */
/* setup                                                                                                          */

/* R11: factor every cell of at most ORC_BLOCK_MAX unknowns (on = 1), or return to R7 (on = 0) */
int orc_set_block_smoother(orc_h *h, int on) {
    if (!h || (on != 0 && on != 1)) return ORC_INVALID;
    h->block = 0;
    if (!on || h->nlev == 1) return ORC_OK;
    if (!h->bfac) {
        int64_t nL = ncells(h->dim, h->L);
        h->boff = calloc(nL + 1, sizeof(int64_t));
        if (!h->boff) return ORC_NOMEM;
        for (int64_t I = 0; I < nL; I++) {
            int64_t m = h->cstart[I + 1] - h->cstart[I];
            h->boff[I + 1] = h->boff[I] + (m <= ORC_BLOCK_MAX ? m * m : 0);
        }
        h->bfac = calloc(h->boff[nL] ? h->boff[nL] : 1, sizeof(double));
        if (!h->bfac) { free(h->boff); h->boff = NULL; return ORC_NOMEM; }
        for (int64_t I = 0; I < nL; I++) {
            int64_t a0 = h->cstart[I], m = h->cstart[I + 1] - a0;
            if (m > ORC_BLOCK_MAX) continue;
            double *blk = h->bfac + h->boff[I];
            for (int64_t a = 0; a < m; a++) {
                int32_t i = h->cdofs[a0 + a];
                for (int64_t e = h->rp[i]; e < h->rp[i + 1]; e++) {
                    int32_t j = h->ci[e];
                    if (h->cell[j] != (int32_t)I) continue;
                    int64_t b = 0;
                    while (h->cdofs[a0 + b] != j) b++;  /* position of j in the cell */
                    blk[a * m + b] += h->va[e];
                }
            }
            int st = cholesky(blk, m);
            if (st) { free(h->bfac); free(h->boff); h->bfac = NULL; h->boff = NULL; return st; }
        }
    }
    h->block = 1;
    return ORC_OK;
}

void orc_free(orc_h *h) {
    if (!h) return;
    free(h->rp); free(h->ci); free(h->va); free(h->diag);
    free(h->cell); free(h->cstart); free(h->cdofs); free(h->chol); free(h->boff); free(h->bfac);
    if (h->lev)
        for (int l = 1; l < h->nlev; l++) {
            olev *lv = &h->lev[l];
            free(lv->aj); free(lv->ax); free(lv->optr); free(lv->ocol); free(lv->oval); free(lv->empty);
        }
    free(h->lev);
    free(h);
}

int orc_setup_dim(int64_t n, int dim, const double *coords, const int64_t *row_ptr, const int32_t *col,
                  const double *val, const double *box, int coarse_max, int inner_iters, int sweeps, orc_h **out) {
    *out = NULL;
    if (n < 1 || (dim != 2 && dim != 3) || !coords || !row_ptr || !col || !val || inner_iters < 1 || sweeps < 1)
        return ORC_INVALID;
    if (row_ptr[0] != 0) return ORC_INVALID;
    for (int64_t i = 0; i < n; i++)
        if (row_ptr[i + 1] < row_ptr[i]) return ORC_INVALID;
    int64_t nnz = row_ptr[n];
    for (int64_t e = 0; e < nnz; e++)
        if (col[e] < 0 || col[e] >= n) return ORC_INVALID;
    for (int64_t i = 0; i < dim * n; i++)
        if (!isfinite(coords[i])) return ORC_INVALID;
    double bx[6] = {0, 0, 0, 0, 0, 0};
    if (box) {
        for (int a = 0; a < dim; a++) {
            if (!isfinite(box[2 * a]) || !isfinite(box[2 * a + 1]) || box[2 * a + 1] < box[2 * a]) return ORC_INVALID;
            for (int64_t i = 0; i < n; i++)
                if (coords[dim * i + a] < box[2 * a] || coords[dim * i + a] > box[2 * a + 1]) return ORC_INVALID;
            bx[2 * a] = box[2 * a];
            bx[2 * a + 1] = box[2 * a + 1];
        }
    } else { /* eq. (6): the bounding box */
        for (int a = 0; a < dim; a++) {
            bx[2 * a] = bx[2 * a + 1] = coords[a];
            for (int64_t i = 1; i < n; i++) {
                double v = coords[dim * i + a];
                if (v < bx[2 * a]) bx[2 * a] = v;
                if (v > bx[2 * a + 1]) bx[2 * a + 1] = v;
            }
        }
    }
    orc_h *h = calloc(1, sizeof(orc_h));
    if (!h) return ORC_NOMEM;
    h->n = n; h->nnz = nnz; h->inner = inner_iters; h->sweeps = sweeps;
    h->dim = dim;
    h->ns = dim == 3 ? 27 : 9;
    h->nchild = 1 << dim;
    memcpy(h->box, bx, sizeof bx);
    h->rp = malloc((n + 1) * sizeof(int64_t));
    h->ci = malloc((nnz ? nnz : 1) * sizeof(int32_t));
    h->va = malloc((nnz ? nnz : 1) * sizeof(double));
    h->diag = calloc(n, sizeof(double));
    if (!h->rp || !h->ci || !h->va || !h->diag) { orc_free(h); return ORC_NOMEM; }
    memcpy(h->rp, row_ptr, (n + 1) * sizeof(int64_t));
    memcpy(h->ci, col, nnz * sizeof(int32_t));
    memcpy(h->va, val, nnz * sizeof(double));
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++)
            if (col[e] == i) h->diag[i] += val[e];
    for (int64_t i = 0; i < n; i++)
        if (!(h->diag[i] > 0.0)) { orc_free(h); return ORC_NOT_SPD; }

    h->nlev = orc_depth_dim(n, dim, coarse_max, &h->L, &h->kc);
    if (h->nlev == 1) {
        h->nc = n;
        h->chol = calloc((size_t)n * n, sizeof(double));
        if (!h->chol) { orc_free(h); return ORC_NOMEM; }
        for (int64_t i = 0; i < n; i++)
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++) h->chol[i * n + col[e]] += val[e];
        int st = cholesky(h->chol, n);
        if (st) { orc_free(h); return st; }
        *out = h;
        return ORC_OK;
    }
    /* level-L aggregates, grouped by cell with a stable counting sort */
    int64_t nL = ncells(dim, h->L);
    h->cell = malloc(n * sizeof(int32_t));
    h->cstart = calloc(nL + 1, sizeof(int64_t));
    h->cdofs = malloc(n * sizeof(int32_t));
    h->lev = calloc(h->nlev, sizeof(olev));
    if (!h->cell || !h->cstart || !h->cdofs || !h->lev) { orc_free(h); return ORC_NOMEM; }
    orc_cell_index_dim(n, dim, coords, bx, h->L, h->cell);
    for (int64_t i = 0; i < n; i++) h->cstart[h->cell[i] + 1]++;
    for (int64_t I = 0; I < nL; I++) h->cstart[I + 1] += h->cstart[I];
    {
        int64_t *fill = malloc(nL * sizeof(int64_t));
        if (!fill) { orc_free(h); return ORC_NOMEM; }
        memcpy(fill, h->cstart, nL * sizeof(int64_t));
        for (int64_t i = 0; i < n; i++) h->cdofs[fill[h->cell[i]]++] = (int32_t)i;
        free(fill);
    }
    /* coarse operators */
    for (int l = 1; l < h->nlev; l++) {
        int st = level_alloc(&h->lev[l], h->L - (l - 1), dim);
        if (!st) st = (l == 1) ? galerkin_fine(h, &h->lev[1]) : galerkin_coarse(&h->lev[l - 1], &h->lev[l]);
        if (st) { orc_free(h); return st; }
        for (int64_t I = 0; I < h->lev[l].n; I++)
            if (!(h->lev[l].ax[I * h->ns] > 0.0)) { orc_free(h); return ORC_NOT_SPD; }
    }
    /* coarsest: dense Cholesky */
    olev *cl = &h->lev[h->nlev - 1];
    h->nc = cl->n;
    h->chol = calloc((size_t)cl->n * cl->n, sizeof(double));
    if (!h->chol) { orc_free(h); return ORC_NOMEM; }
    for (int64_t I = 0; I < cl->n; I++) {
        for (int t = 0; t < cl->ns; t++)
            if (cl->aj[I * cl->ns + t] >= 0) h->chol[I * cl->n + cl->aj[I * cl->ns + t]] += cl->ax[I * cl->ns + t];
        for (int64_t e = cl->optr[I]; e < cl->optr[I + 1]; e++) h->chol[I * cl->n + cl->ocol[e]] += cl->oval[e];
    }
    int st = cholesky(h->chol, cl->n);
    if (st) { orc_free(h); return st; }
    *out = h;
    return ORC_OK;
}

int orc_setup(int64_t n, const double *coords, const int64_t *row_ptr, const int32_t *col, const double *val,
              const double *box, int coarse_max, int inner_iters, int sweeps, orc_h **out) {
    return orc_setup_dim(n, 2, coords, row_ptr, col, val, box, coarse_max, inner_iters, sweeps, out);
}

/* ------------------------------------------------------------------------------------------------------------ */
/* solve                                                                                                          */

int orc_apply_precond(orc_h *h, const double *r, double *z) { return bhat(h, 0, r, z); }

/* test knob: after this many outer iterations the recurrence residual is set to zero once (a recurrence that has
 * drifted from the true residual and reports convergence), so the true-residual check and the restart from the
 * true residual run (0 = off; cleared when used) */
static int force_restart_at = 0;

void orc_test_force_restart(int at_iter) { force_restart_at = at_iter > 0 ? at_iter : 0; }

int orc_solve(orc_h *h, const double *b, double *x, double tol, int max_iters, int mmax, int *iters,
              double *relres) {
    int64_t n = h->n;
    *iters = 0;
    *relres = 0.0;
    for (int64_t i = 0; i < n; i++) x[i] = 0.0;
    double bn = sqrt(dot(n, b, b));
    if (bn == 0.0) return ORC_OK;
    int M = mmax < 0 ? (max_iters > 0 ? max_iters : 1) : mmax;
    double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double)), *t = malloc(n * sizeof(double));
    double *P = malloc((size_t)(M ? M : 1) * n * sizeof(double)), *Q = malloc((size_t)(M ? M : 1) * n * sizeof(double));
    double *D = malloc((size_t)(M ? M : 1) * sizeof(double)), *beta = malloc((size_t)(M ? M : 1) * sizeof(double));
    double *p = malloc(n * sizeof(double)), *q = malloc(n * sizeof(double));
    if (!r || !z || !t || !P || !Q || !D || !beta || !p || !q) {
        free(r); free(z); free(t); free(P); free(Q); free(D); free(beta); free(p); free(q);
        return ORC_NOMEM;
    }
    memcpy(r, b, n * sizeof(double));
    int stored = 0, head = 0; /* ring of the last M directions; head = slot of the oldest */
    int st = ORC_NOCONV, it = 0;
    while (it < max_iters) {
        int s2 = bhat(h, 0, r, z);
        if (s2) { st = s2; break; }
        for (int j = 0; j < stored; j++) {
            int slot = (head + j) % (M ? M : 1);
            beta[j] = -dot(n, z, Q + (size_t)slot * n) / D[slot];
        }
        memcpy(p, z, n * sizeof(double));
        for (int j = 0; j < stored; j++) {
            int slot = (head + j) % (M ? M : 1);
            for (int64_t i = 0; i < n; i++) p[i] += beta[j] * P[(size_t)slot * n + i];
        }
        spmv(h, 0, p, q);
        double d = dot(n, p, q);
        if (!(d > 0.0)) { st = ORC_BREAKDOWN; break; }
        double alpha = dot(n, r, p) / d;
        for (int64_t i = 0; i < n; i++) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        it++;
        if (M > 0) {
            int slot;
            if (stored < M) slot = (head + stored++) % M;
            else { slot = head; head = (head + 1) % M; }
            memcpy(P + (size_t)slot * n, p, n * sizeof(double));
            memcpy(Q + (size_t)slot * n, q, n * sizeof(double));
            D[slot] = d;
        }
        if (force_restart_at > 0 && it == force_restart_at) {
            force_restart_at = 0;
            for (int64_t i = 0; i < n; i++) r[i] = 0.0;
        }
        if (sqrt(dot(n, r, r)) <= tol * bn) {
            spmv(h, 0, x, t);
            for (int64_t i = 0; i < n; i++) t[i] = b[i] - t[i];
            if (sqrt(dot(n, t, t)) <= tol * bn) { st = ORC_OK; break; }
            memcpy(r, t, n * sizeof(double));
            stored = 0; head = 0;
        }
    }
    spmv(h, 0, x, t);
    for (int64_t i = 0; i < n; i++) t[i] = b[i] - t[i];
    *relres = sqrt(dot(n, t, t)) / bn;
    *iters = it;
    free(r); free(z); free(t); free(P); free(Q); free(D); free(beta); free(p); free(q);
    return st;
}

/* ------------------------------------------------------------------------------------------------------------ */
/* inspection and test hooks                                                                                      */

int orc_num_levels(const orc_h *h) { return h->nlev; }

int orc_dim(const orc_h *h) { return h->dim; }

int orc_level_info(const orc_h *h, int level, int64_t *n, int *k, int64_t *ovf_nnz, int *L) {
    if (level < 0 || level >= h->nlev) return ORC_INVALID;
    if (L) *L = h->L;
    if (level == 0) {
        if (n) *n = h->n;
        if (k) *k = -1;
        if (ovf_nnz) *ovf_nnz = 0;
    } else {
        const olev *lv = &h->lev[level];
        if (n) *n = lv->n;
        if (k) *k = lv->k;
        if (ovf_nnz) *ovf_nnz = lv->optr[lv->n];
    }
    return ORC_OK;
}

int orc_export_level(const orc_h *h, int level, int32_t *agg, uint8_t *color, int32_t *aj, double *ax,
                     int64_t *ovf_ptr, int32_t *ovf_col, double *ovf_val) {
    if (level < 0 || level >= h->nlev) return ORC_INVALID;
    if (level == 0) {
        if (h->nlev == 1) {
            for (int64_t i = 0; i < h->n; i++) {
                if (agg) agg[i] = -1;
                if (color) color[i] = 0;
            }
            return ORC_OK;
        }
        int64_t sL = (int64_t)1 << h->L;
        for (int64_t i = 0; i < h->n; i++) {
            if (agg) agg[i] = h->cell[i];
            if (color) color[i] = (uint8_t)cell_color_lex(h->cell[i], sL);
        }
        return ORC_OK;
    }
    const olev *lv = &h->lev[level];
    for (int64_t I = 0; I < lv->n; I++) {
        if (agg) agg[I] = (level < h->nlev - 1) ? (int32_t)parent_of(I, lv->side) : -1;
        if (color) color[I] = (uint8_t)cell_color_lex(I, lv->side);
    }
    if (aj) memcpy(aj, lv->aj, lv->n * lv->ns * sizeof(int32_t));
    if (ax) memcpy(ax, lv->ax, lv->n * lv->ns * sizeof(double));
    if (ovf_ptr) memcpy(ovf_ptr, lv->optr, (lv->n + 1) * sizeof(int64_t));
    if (ovf_col && lv->optr[lv->n]) memcpy(ovf_col, lv->ocol, lv->optr[lv->n] * sizeof(int32_t));
    if (ovf_val && lv->optr[lv->n]) memcpy(ovf_val, lv->oval, lv->optr[lv->n] * sizeof(double));
    return ORC_OK;
}

int orc_smooth(orc_h *h, int level, const double *f, double *x, int forward) {
    if (level < 0 || level >= h->nlev || (h->nlev > 1 && level == h->nlev - 1) || h->nlev == 1) return ORC_INVALID;
    int64_t n = level_n(h, level);
    double *r = malloc(n * sizeof(double)), *d = malloc(n * sizeof(double));
    if (!r || !d) { free(r); free(d); return ORC_NOMEM; }
    smooth(h, level, f, x, forward, r, d);
    free(r); free(d);
    return ORC_OK;
}

int orc_restrict(orc_h *h, int level, const double *r, double *fc) {
    if (level < 0 || level >= h->nlev - 1) return ORC_INVALID;
    restrict_res(h, level, r, fc);
    return ORC_OK;
}

int orc_prolong_add(orc_h *h, int level, const double *e, double *u) {
    if (level < 0 || level >= h->nlev - 1) return ORC_INVALID;
    prolong_add(h, level, e, u);
    return ORC_OK;
}

int orc_level_spmv(orc_h *h, int level, const double *x, double *y) {
    if (level < 0 || level >= h->nlev) return ORC_INVALID;
    spmv(h, level, x, y);
    return ORC_OK;
}

/* test hook context: a bare CSR matrix with an identity or exact-inverse preconditioner */
typedef struct {
    int64_t n;
    const int64_t *rp;
    const int32_t *ci;
    const double *va;
    double *chol;
} tctx;

static void t_spmv(void *c, const double *in, double *out) {
    tctx *t = c;
    for (int64_t i = 0; i < t->n; i++) {
        double acc = 0.0;
        for (int64_t e = t->rp[i]; e < t->rp[i + 1]; e++) acc += t->va[e] * in[t->ci[e]];
        out[i] = acc;
    }
}
static void t_ident(void *c, const double *in, double *out) {
    tctx *t = c;
    memcpy(out, in, t->n * sizeof(double));
}
static void t_exact(void *c, const double *in, double *out) {
    tctx *t = c;
    chol_solve(t->chol, t->n, in, out);
}

int orc_nlpcg_test(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val, const double *f,
                   int nsteps, int mode, double *u) {
    tctx t = {n, row_ptr, col, val, NULL};
    if (mode == 1) {
        t.chol = calloc((size_t)n * n, sizeof(double));
        if (!t.chol) return ORC_NOMEM;
        for (int64_t i = 0; i < n; i++)
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; e++) t.chol[i * n + col[e]] += val[e];
        int st = cholesky(t.chol, n);
        if (st) { free(t.chol); return st; }
    }
    op_t A = {t_spmv, &t}, B = {mode == 1 ? t_exact : t_ident, &t};
    int st = nlpcg(n, A, B, f, nsteps, u);
    free(t.chol);
    return st;
}
