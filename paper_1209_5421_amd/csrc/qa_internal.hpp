// Internal layout of the quadamg hierarchy on the device (gfx950).
//
// Numbering. Quadtree level k (side 2^k, n = 4^k cells) is stored in "color-major" order: a cell with quadtree
// coordinates (t1, t2) has Morton key m = interleave(t1 -> even bits, t2 -> odd bits), and its storage index is
// q = (m & 3) * 4^(k-1) + (m >> 2). The low two Morton bits are the cell's color (t1 & 1) + 2 (t2 & 1) of the
// 4-coloring (Section 4.5), so every color is one contiguous quarter of the vector; the four children of a
// level-(k-1) cell M (Morton) sit at q = c * 4^(k-1) + M, c = 0..3, one per quarter, so restriction reads four
// coalesced streams. The fine level is permuted the same way: rows sorted by (color-major index of their level-L
// cell, original index), so each cell's unknowns are contiguous and ascending.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <vector>

#include "quadamg.h"

namespace qa {

constexpr int kBlock = 256;        // threads per workgroup for elementwise / reduction kernels
constexpr int kSliceRows = 64;     // sliced-ELL slice height = one wavefront
constexpr int kSellWindow = 256;   // rows are sorted by length inside runs of this many positions (4 slices)
constexpr int kRedBlocksMax = 1024;
constexpr int kBlockMax = 32;      // exact-block smoother: cells of at most this many unknowns are factored
constexpr int kBigCell = 32;       // cells with more unknowns get a level-scheduled in-cell substitution
constexpr int kFuseStageRows = 512; // rows of a window the fused smoother phase stages in LDS
constexpr int kScalars = 16;       // device scalars per level
constexpr int kMaxColors = 8;      // colors of the smoother: 4 on a quadtree, 8 on an octree

// ---------------------------------------------------------------------------------------------------------------
// Morton / color-major index helpers (k <= 15)

__host__ __device__ inline uint32_t spread_bits(uint32_t v) {
  v &= 0xFFFFu;
  v = (v | (v << 8)) & 0x00FF00FFu;
  v = (v | (v << 4)) & 0x0F0F0F0Fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}
__host__ __device__ inline uint32_t compact_bits(uint32_t v) {
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0F0F0F0Fu;
  v = (v | (v >> 4)) & 0x00FF00FFu;
  v = (v | (v >> 8)) & 0x0000FFFFu;
  return v;
}
__host__ __device__ inline uint32_t morton(uint32_t t1, uint32_t t2) { return spread_bits(t1) | (spread_bits(t2) << 1); }
__host__ __device__ inline uint32_t q_of_m(uint32_t m, int k) {
  return k == 0 ? 0u : (((m & 3u) << (2 * k - 2)) | (m >> 2));
}
__host__ __device__ inline uint32_t m_of_q(uint32_t q, int k) {
  return k == 0 ? 0u : (((q & ((1u << (2 * k - 2)) - 1u)) << 2) | (q >> (2 * k - 2)));
}

// neighbour offsets of Section 4.4: self, E, NE, N, NW, W, SW, S, SE
__host__ __device__ inline int slot_dx(int s) {
  switch (s) {
    case 1: case 2: case 8: return 1;
    case 4: case 5: case 6: return -1;
    default: return 0;
  }
}
__host__ __device__ inline int slot_dy(int s) {
  switch (s) {
    case 2: case 3: case 4: return 1;
    case 6: case 7: case 8: return -1;
    default: return 0;
  }
}
// slot of offset (dx, dy), both in [-1, 1]
__host__ __device__ inline int slot_of(int dx, int dy) {
  // index (dy + 1) * 3 + (dx + 1) -> slot
  const int tab = (dy + 1) * 3 + (dx + 1);
  switch (tab) {
    case 0: return 6; case 1: return 7; case 2: return 8;
    case 3: return 5; case 4: return 0; case 5: return 1;
    case 6: return 4; case 7: return 3; default: return 2;
  }
}

// The nine stencil cells of a level-k cell in color-major numbering. Cell q = c n4 + j (n4 = 4^(k-1) = 2^sh) is child
// c = (cx, cy) of the level-(k-1) super-cell with Morton index j; each neighbour is a child of j or of one of the
// super-cells around j, found by dilated-integer +-1 on j's x bits (even) and y bits (odd). Only selects, no
// branches: when the caller passes a color that is uniform over the wavefront (one color phase, or 64 consecutive
// rows of one color) every condition below is uniform too. A neighbour outside the grid is replaced by q itself
// (its slot value is 0), so every slot can be loaded unconditionally.
__host__ __device__ inline void stencil_q(uint32_t q, uint32_t j, int c, int sh, uint32_t (&out)[9]) {
  const uint32_t n4 = 1u << sh;
  const uint32_t xm = 0x55555555u & (n4 - 1u), ym = 0xAAAAAAAAu & (n4 - 1u);
  const uint32_t jx = j & xm, jy = j & ym;
  const uint32_t xl = (jx - 1u) & xm, xr = ((jx | ~xm) + 1u) & xm;
  const uint32_t yd = (jy - 1u) & ym, yu = ((jy | ~ym) + 1u) & ym;
  const bool okl = jx != 0u, okr = jx != xm, okd = jy != 0u, oku = jy != ym;
  const int cx = c & 1, cy = c >> 1;
#pragma unroll
  for (int s = 0; s < 9; s++) {
    const int ux = cx + slot_dx(s), uy = cy + slot_dy(s);
    const uint32_t sx = ux < 0 ? xl : (ux > 1 ? xr : jx);
    const uint32_t sy = uy < 0 ? yd : (uy > 1 ? yu : jy);
    const bool ok = (ux < 0 ? okl : (ux > 1 ? okr : true)) && (uy < 0 ? okd : (uy > 1 ? oku : true));
    const uint32_t qn = (static_cast<uint32_t>((ux & 1) | ((uy & 1) << 1)) << sh) | sx | sy;
    out[s] = ok ? qn : q;
  }
}

// ---------------------------------------------------------------------------------------------------------------
// Octree (3D) levels. A cell (t1, t2, t3) of level k has Morton key m = interleave(t1 -> bits 0, 3, 6, ...,
// t2 -> bits 1, 4, ..., t3 -> bits 2, 5, ...) and storage index q = (m & 7) 8^(k-1) + (m >> 3): the low three key
// bits are its color (t1 & 1) + 2 (t2 & 1) + 4 (t3 & 1) of the 8-coloring, so every color is one contiguous eighth,
// and the eight children of a level-(k-1) cell M sit at q = c 8^(k-1) + M. The 27 coarse slots are the nine plane
// offsets of Section 4.4 (self, E, NE, N, NW, W, SW, S, SE) at dz = 0, then at dz = +1, then at dz = -1 (k <= 10).

__host__ __device__ inline uint32_t spread3(uint32_t v) {
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__host__ __device__ inline uint32_t compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030C30C3u;
  v = (v | (v >> 4)) & 0x0300F00Fu;
  v = (v | (v >> 8)) & 0x030000FFu;
  v = (v | (v >> 16)) & 0x000003FFu;
  return v;
}
__host__ __device__ inline uint32_t morton3(uint32_t t1, uint32_t t2, uint32_t t3) {
  return spread3(t1) | (spread3(t2) << 1) | (spread3(t3) << 2);
}
__host__ __device__ inline uint32_t q_of_m3(uint32_t m, int k) {
  return k == 0 ? 0u : (((m & 7u) << (3 * k - 3)) | (m >> 3));
}
__host__ __device__ inline uint32_t m_of_q3(uint32_t q, int k) {
  return k == 0 ? 0u : (((q & ((1u << (3 * k - 3)) - 1u)) << 3) | (q >> (3 * k - 3)));
}
__host__ __device__ inline int slot3_dx(int t) { return slot_dx(t % 9); }
__host__ __device__ inline int slot3_dy(int t) { return slot_dy(t % 9); }
__host__ __device__ inline int slot3_dz(int t) { return t < 9 ? 0 : (t < 18 ? 1 : -1); }
// slot of offset (dx, dy, dz), each in [-1, 1]
__host__ __device__ inline int slot3_of(int dx, int dy, int dz) {
  return (dz == 0 ? 0 : (dz > 0 ? 9 : 18)) + slot_of(dx, dy);
}
// order in which the children of a cell are summed: the 2D restriction order (0, 1, 3, 2) on the layer 2 T3, then on
// the layer 2 T3 + 1
__host__ __device__ inline int child3_order(int i) {
  const int o2[4] = {0, 1, 3, 2};
  return o2[i & 3] | (i & 4);
}

// ---------------------------------------------------------------------------------------------------------------
// hierarchy

struct QuadLevel {              // quadtree (octree in 3D) level k, color-major numbering
  int k = 0;
  int64_t n = 0;                // 4^k (8^k)
  int ns = 9;                   // slots per row: 9, or 27 on an octree level
  double *ax64 = nullptr;       // ns x n, slot-major: ax[s * n + q]
  float *ax32 = nullptr;
  uint8_t *empty = nullptr;     // 1 = aggregate without fine unknowns (identity row)
  int64_t ovf_nnz = 0;          // couplings beyond one cell: CSR over rows q, columns q, sorted by lexicographic id
  int32_t *optr = nullptr;
  int32_t *ocol = nullptr;
  double *oval64 = nullptr;
  float *oval32 = nullptr;
  int same_color_ovf = 0;       // some overflow coupling joins two cells of one color
};

struct FineLevel {
  int64_t n = 0, nnz = 0;
  int32_t *perm = nullptr;      // position p -> caller's index
  int32_t *iperm = nullptr;     // caller's index -> position p
  int64_t *rp = nullptr;        // permuted CSR (caller's entry order inside a row)
  int32_t *ci = nullptr;
  double *va = nullptr;
  // sliced ELL: each color's rows in windows (runs of whole cells whose first rows lie in one band of win_band
  // rows; 256 rows on a single level), each window in slices of 64 positions (the last one partial), column-major
  // inside a slice, diagonal first; padding entries point at the row itself with value 0
  int64_t nwin = 0;
  int win_band = 0;
  int32_t *win_q = nullptr;     // nwin + 1: first cell of each window (null on a single level)
  int32_t *win_row = nullptr;   // nwin + 1: first row of each window
  int64_t *win_slice = nullptr; // nwin + 1: first slice of each window
  int64_t *win_ent = nullptr;   // nwin + 1: first factor value (exact blocks) or in-cell coupling of each window
  int win_ent_max = 0;          // the most factor values / couplings of a window the fused phase stages
  int64_t color_win[kMaxColors + 1] = {};
  bool same_color = false;      // some row is coupled to a row of another cell of its own color
  int64_t nslices = 0;
  int64_t *slice_ptr = nullptr; // nslices + 1 (entry offsets)
  int32_t *slice_row0 = nullptr;// nslices + 1 (first row)
  int32_t *s_col = nullptr;
  int32_t *s_row = nullptr;     // SELL position -> row: rows sorted by length within runs of kSellWindow positions
                                // of a window
  double *s_val64 = nullptr;
  float *s_val32 = nullptr;
  int64_t sell_entries = 0;
  int ncolor = 4;               // 2^dim colors; each is a contiguous range of cells and rows
  int64_t color_row[kMaxColors + 1] = {};
  int64_t color_slice[kMaxColors + 1] = {};
  double *diag64 = nullptr;
  float *diag32 = nullptr;
  // couplings inside a cell (off-diagonal), caller's entry order, for the in-cell substitution
  int64_t ic_nnz = 0;
  int32_t *ic_ptr = nullptr;
  int32_t *ic_col = nullptr;
  double *ic_val64 = nullptr;
  float *ic_val32 = nullptr;
  int32_t *crow = nullptr;      // level-L cell q -> first row (4^L + 1)
  int32_t *agg_q = nullptr;     // row -> level-L cell q
  // cells of more than kBigCell unknowns: their in-cell substitution runs level by level (rows on one level of the
  // substitution's dependency graph are independent), one workgroup per cell; [0] forward, [1] backward
  int64_t nbig = 0;
  int64_t big_color[kMaxColors + 1] = {};      // first big cell of each color (big cells ascend by cell id)
  int32_t *big_cells = nullptr;                 // cell ids
  int big_max_rows = 0;                         // rows of the largest big cell
  int32_t *big_lofs[2] = {nullptr, nullptr};    // per big cell, its first entry in big_lptr (nbig + 1)
  int32_t *big_lptr[2] = {nullptr, nullptr};    // level starts as row positions, then the cell's end
  int32_t *big_sched[2] = {nullptr, nullptr};   // the big cells' rows ordered by level (indexed by row position)
  // exact-block smoother: the cell's Cholesky factor (packed lower triangle, row-major) at boff[q] for cells of at most
  // kBlockMax unknowns (empty otherwise); cells above kBlockMax are the big cells and keep the substitution
  int64_t *boff = nullptr;                      // 4^L + 1
  double *bfac64 = nullptr;
  float *bfac32 = nullptr;
  int64_t bfac_n = 0;                           // packed factor values in all (boff[4^L])
};

template <class T>
struct LevelWork {              // per level, one precision
  T *f = nullptr, *u = nullptr, *d = nullptr;  // fine level: B^ input, output, temporary
  T *g = nullptr, *e = nullptr, *r = nullptr, *p0 = nullptr, *q0 = nullptr, *p1 = nullptr, *q1 = nullptr;
};

struct Timing {
  int kind = -1;                // which kernel family is timed (see kernel_kind)
  std::vector<hipEvent_t> ev;   // pairs
  size_t used = 0;
  int64_t launches = 0;
  double total_ms = 0.0;
  double bytes_per_launch = 0.0;
};

enum KernelKind { KK_SPMV64 = 0, KK_GS_FINE32, KK_GS_FINE64, KK_RESID_FINE32, KK_RESID_FINE64, KK_ENGINE64, KK_ENGINE32,
                  KK_COUNT };

struct Chunk {                  // a device allocation that several arrays are carved from
  char *base = nullptr;
  size_t size = 0, used = 0;
};

}  // namespace qa

struct amg_hierarchy {
  int device = 0;
  int dim = 2;                          // 2: quadtree levels (4^k cells); 3: octree levels (8^k cells)
  hipStream_t stream = nullptr;
  amg_options opt{};
  double box[6] = {0, 0, 0, 0, 0, 0};   // {a1, b1, a2, b2[, a3, b3]}
  int64_t n = 0;
  int L = -1, kc = -1, nlev = 1;
  int precision = 0;
  qa::FineLevel fine;
  std::vector<qa::QuadLevel> lev;      // lev[1 .. nlev-1]
  int64_t nc = 0;                      // coarsest size
  double *ainv = nullptr;              // coarsest inverse (nc x nc), storage numbering of that level
  std::vector<qa::LevelWork<double>> w64;
  std::vector<qa::LevelWork<float>> w32;
  // outer iteration (FP64, permuted numbering)
  double *xp = nullptr, *rp = nullptr, *bp = nullptr, *zp = nullptr, *pp = nullptr, *qp = nullptr,
         *pprev = nullptr, *qprev = nullptr, *tp = nullptr;
  double *scal = nullptr;              // (nlev + 1) * kScalars device scalars
  double *partials = nullptr;          // reduction partial sums
  int64_t partials_cap = 0;
  double *host_scal = nullptr;         // pinned mirror for convergence checks
  int *dflag = nullptr;                // device error flags
  std::vector<void *> allocs;           // device chunks (freed by amg_free)
  std::vector<size_t> alloc_sizes;      // their sizes
  size_t bytes = 0;                     // device bytes held (chunks, including unused tails)
  std::vector<qa::Chunk> chunks;        // shared chunks that small arrays are carved from
  size_t chunk_unit = 8u << 20;         // size of a shared chunk (set from the size estimate at setup)
  double setup_ms = 0.0;
  int stale = 0;                        // a values update failed after it began to overwrite: solves are refused
  qa::Timing timing;
  // persistent small-level engine: top level index per precision (0 = FP64, 1 = FP32), -1 = not used
  int engine_top[2] = {-1, -1};
  int engine_lds_top[2] = {-1, -1};  // first level index whose operators and vectors live in LDS
  int engine_ainv_lds[2] = {0, 0};
  int engine_lvec[2] = {0, 0};       // work vectors of a global engine top level held in LDS (bit per vector slot)
  void *engine_ops[2] = {nullptr, nullptr};
  int engine_nops[2] = {0, 0};
  double engine_flops[2] = {0.0, 0.0};  // algorithmic floating-point operations of one engine launch
  int64_t engine_global_rows = 4096;  // a top level this small may run from global memory
  size_t engine_lds[2] = {0, 0};
  size_t lds_max = 0;
  int use_engine = 1;                 // 0 off, 1 on (specialised engine where eligible), 2 the step interpreter only
  // specialised engine (qa_engine.hip): configuration id per precision (-1 = the interpreter), its step list
  int fe_cfg[2] = {-1, -1};
  void *fe_ops[2] = {nullptr, nullptr};
  int fe_nops[2] = {0, 0};
  int use_batch = 1;
  // whole-solve workgroup (batched serving of small systems), per precision
  void *wg_ops[2] = {nullptr, nullptr};
  int wg_nops[2] = {0, 0};
  int wg_lds_top[2] = {-1, -1};
  int wg_ainv_lds[2] = {0, 0};
  size_t wg_lds[2] = {0, 0};
  // all-directions outer iteration (outer_mmax < 0): kept directions p_j, q_j = A p_j, their device address table,
  // the inner products (z, q_j) of the current step and (p_j, q_j)
  std::vector<double *> dir_p, dir_q;
  double **dir_pp = nullptr;
  double *dir_zq = nullptr;
  double *dir_d = nullptr;
  // B^ of the level above the coarsest as an explicit matrix (column-major, FP64 and FP32), or none
  int mhat_level = -1;
  int64_t mhat_n = 0;
  void *mhat[2] = {nullptr, nullptr};
};

namespace qa {

// allocation helpers (every allocation is tracked and released by amg_free)
void *dalloc(amg_hierarchy *h, size_t bytes);
template <class T>
T *dalloc_n(amg_hierarchy *h, int64_t count) {
  return static_cast<T *>(dalloc(h, sizeof(T) * static_cast<size_t>(count > 0 ? count : 1)));
}

// shared helpers implemented in qa_common.hip
amg_status scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s, amg_hierarchy *h);
amg_status scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s, amg_hierarchy *h);
amg_status release(amg_hierarchy *h);
// temporary device memory of one call on h (the caller's allocator when one is set, else the library's pool on
// stream s); tmp_free returns it on s
void *tmp_alloc(amg_hierarchy *h, hipStream_t s, size_t bytes);
void tmp_free(amg_hierarchy *h, hipStream_t s, void *p);
// the allocation state of a hierarchy, and the return to it: arrays allocated after the mark go back to the
// chunks' free tails or to the block cache (the stream is synchronised first)
struct ArenaMark {
  size_t allocs = 0;
  size_t bytes = 0;
  std::vector<size_t> used;
};
ArenaMark arena_mark(const amg_hierarchy *h);
void arena_rollback(amg_hierarchy *h, const ArenaMark &m);
amg_status borrow_events(int device, size_t count, std::vector<hipEvent_t> &out);
void return_events(int device, std::vector<hipEvent_t> &ev);
amg_status borrow_pinned_scalars(double **out);
void return_pinned_scalars(double *p);

// solve side (qa_solve.hip)
amg_status alloc_workspaces(amg_hierarchy *h);
amg_status build_mhat(amg_hierarchy *h);
amg_status plan_engine(amg_hierarchy *h);
amg_status plan_wg(amg_hierarchy *h);
amg_status plan_engine_fast(amg_hierarchy *h);   // qa_engine.hip
void launch_engine_fast(amg_hierarchy *h, int precision);
amg_status precond_apply(amg_hierarchy *h, int precision, const double *r_p, double *z_p);
amg_status level_smooth_internal(amg_hierarchy *h, int level, const double *f, double *x, int forward, int prec);
amg_status level_spmv_internal(amg_hierarchy *h, int level, const double *x, double *y, int prec);
double kernel_bytes(const amg_hierarchy *h, int kind);

}  // namespace qa

#define QA_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t qa_e_ = (call);                                                        \
    if (qa_e_ != hipSuccess) {                                                        \
      return qa_e_ == hipErrorOutOfMemory ? AMG_ERR_NOMEM : AMG_ERR_DEVICE;           \
    }                                                                                 \
  } while (0)

#define QA_TRY(call)                        \
  do {                                      \
    amg_status qa_s_ = (call);              \
    if (qa_s_ != AMG_OK) return qa_s_;      \
  } while (0)

#define QA_LAUNCH_CHECK() QA_HIP(hipGetLastError())
