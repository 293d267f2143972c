// Setup of the auxiliary-grid hierarchy (Section 3, Sections 4.2-4.4) on gfx950.
//
// Pipeline (all on the device, one stream): validate the CSR input and sum diagonals -> auxiliary box (eq. 5-6)
// -> level-L cell of every unknown by the index formula of Section 4.2 (eq. 9), turned into a color-major Morton
// index, with an integer-atomic histogram -> exclusive scan = cell row pointers -> scatter + per-cell sort (a
// stable counting sort: unknowns of a cell end up contiguous and ascending) -> permuted CSR -> sliced ELL
// (64-row slices, column-major, diagonal first, Section 4.1) and the in-cell coupling lists of the block smoother
// -> Galerkin operators: level L from the fine rows of each cell (eq. 11), level k-1 from the four children of
// each cell (Section 4.4), 9 slots plus an overflow list for couplings beyond one cell -> dense inverse of the
// coarsest operator via Cholesky (Algorithm 2.2's A_1^{-1}).
//
// This file is compiled with -ffp-contract=off: the cell index must be the IEEE sequence subtract, divide,
// multiply, floor, and the Galerkin sums are plain additions taken in a fixed order (cells, then rows ascending,
// then entries in the caller's order; children in the order of Section 4.3's restriction formula).
#include <chrono>
#include <cmath>
#include <cstring>

#include "qa_internal.hpp"

namespace qa {

enum { F_INVALID = 1, F_NOT_SPD = 2, F_SAMECOLOR = 4 };

struct Box3 {  // {a1, b1, a2, b2, a3, b3} of an octree's auxiliary box
  double v[6];
};

__device__ inline void q_to_t(uint32_t q, int k, uint32_t &t1, uint32_t &t2) {
  const uint32_t m = m_of_q(q, k);
  t1 = compact_bits(m);
  t2 = compact_bits(m >> 1);
}

// ---------------------------------------------------------------------------------------------------------------
// validation, box, cell keys

__global__ void __launch_bounds__(kBlock) k_validate(int64_t n, int64_t nnz, const double *__restrict__ coords,
                                                      const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                      const double *__restrict__ va, int has_box, double a1,
                                                      double b1, double a2, double b2, int *flag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int f = 0;
  const int64_t r0 = rp[i], r1 = rp[i + 1];
  if (i == 0 && r0 != 0) f |= F_INVALID;
  if (i == n - 1 && r1 != nnz) f |= F_INVALID;
  if (r1 < r0 || r0 < 0 || r1 > nnz) f |= F_INVALID;
  const double x = coords[2 * i], y = coords[2 * i + 1];
  if (!isfinite(x) || !isfinite(y)) f |= F_INVALID;
  if (has_box && (x < a1 || x > b1 || y < a2 || y > b2)) f |= F_INVALID;
  if (!(f & F_INVALID)) {
    double dg = 0.0;
    for (int64_t e = r0; e < r1; e++) {
      const int32_t c = ci[e];
      if (c < 0 || c >= n) f |= F_INVALID;
      else if (c == i) dg += va[e];
    }
    if (!(dg > 0.0)) f |= F_NOT_SPD;
  }
  if (f) atomicOr(flag, f);
}

// A values update's input against the stored pattern: row i of the new CSR must hold, in the same order, the
// entries that setup placed at permuted row iperm[i] (k_permute_csr keeps each row's entry order). Also the checks
// of k_validate that do not involve coordinates, and a positive diagonal of the new values.
__global__ void __launch_bounds__(kBlock) k_same_pattern(int64_t n, int64_t nnz, const int64_t *__restrict__ rp_in,
                                                          const int32_t *__restrict__ ci_in,
                                                          const double *__restrict__ va_in,
                                                          const int32_t *__restrict__ iperm,
                                                          const int64_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci, int *flag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int f = 0;
  const int64_t r0 = rp_in[i], r1 = rp_in[i + 1];
  if (i == 0 && r0 != 0) f |= F_INVALID;
  if (i == n - 1 && r1 != nnz) f |= F_INVALID;
  if (r1 < r0 || r0 < 0 || r1 > nnz) f |= F_INVALID;
  if (!f) {
    const int64_t p = iperm[i];
    const int64_t o0 = rp[p];
    if (rp[p + 1] - o0 != r1 - r0) f |= F_INVALID;
    double dg = 0.0;
    for (int64_t e = r0; e < r1 && !f; e++) {
      const int32_t c = ci_in[e];
      if (c < 0 || c >= n || iperm[c] != ci[o0 + (e - r0)]) f |= F_INVALID;
      else if (c == i) dg += va_in[e];
    }
    if (!f && !(dg > 0.0)) f |= F_NOT_SPD;
  }
  if (f) atomicOr(flag, f);
}

__global__ void __launch_bounds__(kBlock) k_bbox_partial(int64_t n, const double *__restrict__ coords,
                                                          double *__restrict__ part) {
  double mnx = INFINITY, mxx = -INFINITY, mny = INFINITY, mxy = -INFINITY;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const double x = coords[2 * i], y = coords[2 * i + 1];
    mnx = fmin(mnx, x); mxx = fmax(mxx, x); mny = fmin(mny, y); mxy = fmax(mxy, y);
  }
  __shared__ double s[4][kBlock];
  s[0][threadIdx.x] = mnx; s[1][threadIdx.x] = mxx; s[2][threadIdx.x] = mny; s[3][threadIdx.x] = mxy;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + off]);
      s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + off]);
      s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + off]);
      s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int t = 0; t < 4; t++) part[blockIdx.x * 4 + t] = s[t][0];
}

__global__ void k_bbox_final(int nb, const double *__restrict__ part, double *__restrict__ box) {
  double mnx = INFINITY, mxx = -INFINITY, mny = INFINITY, mxy = -INFINITY;
  for (int b = 0; b < nb; b++) {
    mnx = fmin(mnx, part[4 * b]); mxx = fmax(mxx, part[4 * b + 1]);
    mny = fmin(mny, part[4 * b + 2]); mxy = fmax(mxy, part[4 * b + 3]);
  }
  box[0] = mnx; box[1] = mxx; box[2] = mny; box[3] = mxy;
}

// Section 4.2: index = floor((v - a) / (b - a) * 2^L), clamped so the upper box edge belongs to the last cell.
__device__ inline uint32_t axis_cell(double v, double a, double b, int L) {
  if (!(b > a)) return 0u;
  const double t = (v - a) / (b - a);
  const double f = floor(t * static_cast<double>(1u << L));
  int64_t i = static_cast<int64_t>(f);
  const int64_t top = (static_cast<int64_t>(1) << L) - 1;
  if (i > top) i = top;
  if (i < 0) i = 0;
  return static_cast<uint32_t>(i);
}

__global__ void __launch_bounds__(kBlock) k_cell_key(int64_t n, const double *__restrict__ coords, double a1,
                                                      double b1, double a2, double b2, int L,
                                                      int32_t *__restrict__ key, int32_t *__restrict__ cnt) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t xi = axis_cell(coords[2 * i], a1, b1, L);
  const uint32_t yi = axis_cell(coords[2 * i + 1], a2, b2, L);
  const uint32_t q = q_of_m(morton(xi, yi), L);
  key[i] = static_cast<int32_t>(q);
  atomicAdd(&cnt[q], 1);
}

__global__ void __launch_bounds__(kBlock) k_scatter(int64_t n, const int32_t *__restrict__ key,
                                                     const int32_t *__restrict__ crow, int32_t *__restrict__ fill,
                                                     int32_t *__restrict__ perm) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t q = key[i];
  perm[crow[q] + atomicAdd(&fill[q], 1)] = static_cast<int32_t>(i);
}

// restore ascending caller order inside each cell (the scatter order is arbitrary): insertion sort, one thread per
// cell of at most kSortCell unknowns (larger cells: k_rank_sort_cells)
constexpr int kSortCell = 32;

__global__ void __launch_bounds__(kBlock) k_sort_cells(int64_t ncell, const int32_t *__restrict__ crow,
                                                        int32_t *__restrict__ perm) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= ncell) return;
  const int32_t a = crow[q], b = crow[q + 1];
  if (b - a > kSortCell) return;
  for (int32_t i = a + 1; i < b; i++) {
    const int32_t v = perm[i];
    int32_t j = i - 1;
    while (j >= a && perm[j] > v) {
      perm[j + 1] = perm[j];
      j--;
    }
    perm[j + 1] = v;
  }
}

// the same for one large cell per workgroup: each entry's place is the number of smaller entries in the cell (the
// entries are distinct unknown indices), read from a copy staged in LDS when the cell fits
constexpr int kRankLds = 8192;

__global__ void __launch_bounds__(kBlock) k_rank_sort_cells(const int32_t *__restrict__ cells,
                                                             const int32_t *__restrict__ crow,
                                                             const int32_t *__restrict__ in, int32_t *__restrict__ out) {
  __shared__ int32_t v[kRankLds];
  const int32_t q = cells[blockIdx.x];
  const int32_t a = crow[q], m = crow[q + 1] - a;
  const bool lds = m <= kRankLds;
  if (lds)
    for (int32_t i = threadIdx.x; i < m; i += kBlock) v[i] = in[a + i];
  __syncthreads();
  for (int32_t i = threadIdx.x; i < m; i += kBlock) {
    const int32_t x = in[a + i];
    int32_t r = 0;
    for (int32_t j = 0; j < m; j++) r += ((lds ? v[j] : in[a + j]) < x) ? 1 : 0;
    out[a + r] = x;
  }
}

__global__ void __launch_bounds__(kBlock) k_inverse_perm(int64_t n, const int32_t *__restrict__ perm,
                                                          const int32_t *__restrict__ key, int32_t *__restrict__ iperm,
                                                          int32_t *__restrict__ agg_q, const int64_t *__restrict__ rp_in,
                                                          int64_t *__restrict__ len) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t i = perm[p];
  iperm[i] = static_cast<int32_t>(p);
  if (agg_q) agg_q[p] = key[i];
  len[p] = rp_in[i + 1] - rp_in[i];
}

__global__ void __launch_bounds__(kBlock) k_permute_csr(int64_t n, const int32_t *__restrict__ perm,
                                                         const int32_t *__restrict__ iperm,
                                                         const int64_t *__restrict__ rp_in,
                                                         const int32_t *__restrict__ ci_in,
                                                         const double *__restrict__ va_in, const int64_t *__restrict__ rp,
                                                         int32_t *__restrict__ ci, double *__restrict__ va,
                                                         double *__restrict__ diag) {
  // eight lanes per row copy its entries (the rows arrive in permuted order, so a row's entries are the unit of
  // contiguous access); the diagonal is summed afterwards by k_row_diag
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t p = t >> 3;
  if (p >= n) return;
  const int32_t i = perm[p];
  const int64_t e0 = rp_in[i], o0 = rp[p];
  for (int64_t e = e0 + (t & 7); e < rp_in[i + 1]; e += 8) {
    ci[o0 + (e - e0)] = iperm[ci_in[e]];
    va[o0 + (e - e0)] = va_in[e];
  }
  (void)diag;
}

// diagonal of each permuted row: its diagonal entries summed in entry order
__global__ void __launch_bounds__(kBlock) k_row_diag(int64_t n, const int64_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci, const double *__restrict__ va,
                                                      double *__restrict__ diag) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double dg = 0.0;
  for (int64_t e = rp[p]; e < rp[p + 1]; e++)
    if (ci[e] == p) dg += va[e];
  diag[p] = dg;
}

// ---------------------------------------------------------------------------------------------------------------
// sliced ELL of the fine level

// Windows: each color's rows are cut into windows, and every window into slices of 64 positions (the last one
// partial). On a multi-level hierarchy a window is a run of whole cells of one color: consecutive cells whose first
// rows lie in one band of `band` rows (counted from the color's first row), at most kWinCells of them, and a cell of
// more than kSellWindow unknowns is a window of its own. With band = 257 - largest (the largest cell the smoother
// solves per thread) the cells it solves in a window hold at most band - 1 + largest = 256 rows, and a window at
// most band - 1 + kSellWindow < 512 rows unless it is one huge cell: the fused smoother phase takes a window per
// workgroup with its cells whole and staged in LDS. On a single level (no cells) the windows are 256 consecutive rows.
constexpr int kWinCells = 512;

// 1 if some row is coupled to a row of another cell of its own color (cells are color-major: color = cell /
// per_color)
__global__ void __launch_bounds__(kBlock) k_same_color(int64_t n, int64_t per_color, const int64_t *__restrict__ rp,
                                                        const int32_t *__restrict__ ci,
                                                        const int32_t *__restrict__ agg_q, int *__restrict__ flag) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t qp = agg_q[p];
  bool hit = false;
  for (int64_t e = rp[p]; e < rp[p + 1]; e++) {
    const int32_t qc = agg_q[ci[e]];
    hit = hit || (qc != qp && qc / per_color == qp / per_color);
  }
  if (hit) atomicOr(flag, 1);
}

// a cell starts a window when it is its color's first cell or its first row lies in another band than the
// previous cell's
__global__ void __launch_bounds__(kBlock) k_win_mark(int64_t nL, int64_t per_color, const int32_t *__restrict__ crow,
                                                      int band, int32_t *__restrict__ mark) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nL) return;
  const int64_t c0 = (q / per_color) * per_color;
  if (q == c0 || (q - c0) % kWinCells == 0) {
    mark[q] = 1;
    return;
  }
  const int32_t base = crow[c0];
  const bool big = crow[q + 1] - crow[q] > kSellWindow, prev_big = crow[q] - crow[q - 1] > kSellWindow;
  mark[q] = (big || prev_big || (crow[q] - base) / band != (crow[q - 1] - base) / band) ? 1 : 0;
}

// first cell and first row of each window; the end (nL, n) after the last
__global__ void __launch_bounds__(kBlock) k_win_fill(int64_t nL, const int32_t *__restrict__ crow,
                                                      const int32_t *__restrict__ mark,
                                                      const int32_t *__restrict__ widx, int32_t *__restrict__ win_q,
                                                      int32_t *__restrict__ win_row) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nL) return;
  if (mark[q]) {
    win_q[widx[q]] = static_cast<int32_t>(q);
    win_row[widx[q]] = crow[q];
  }
  if (q == nL - 1) {
    win_q[widx[nL]] = static_cast<int32_t>(nL);
    win_row[widx[nL]] = crow[nL];
  }
}

// single level: windows of kSellWindow consecutive rows
__global__ void __launch_bounds__(kBlock) k_win_fixed(int64_t nwin, int64_t n, int32_t *__restrict__ win_row) {
  const int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w > nwin) return;
  win_row[w] = static_cast<int32_t>(w < nwin ? w * kSellWindow : n);
}

__global__ void __launch_bounds__(kBlock) k_win_nslices(int64_t nwin, const int32_t *__restrict__ win_row,
                                                         int64_t *__restrict__ nsl) {
  const int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= nwin) return;
  nsl[w] = (win_row[w + 1] - win_row[w] + kSliceRows - 1) / kSliceRows;
}

// first position of each slice; row0[nslices] = n
__global__ void __launch_bounds__(kBlock) k_slice_starts(int64_t nwin, const int32_t *__restrict__ win_row,
                                                          const int64_t *__restrict__ win_slice,
                                                          int32_t *__restrict__ row0) {
  const int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= nwin) return;
  for (int64_t k = 0; k < win_slice[w + 1] - win_slice[w]; k++)
    row0[win_slice[w] + k] = win_row[w] + static_cast<int32_t>(k * kSliceRows);
  if (w == nwin - 1) row0[win_slice[nwin]] = win_row[nwin];
}

// Rows of each run of kSellWindow positions of a window, sorted by length (longest first, ascending row among equal
// lengths), so that the slices of a run hold rows of similar length and the padding of sliced ELL stays small
// (sliced ELL with sorting windows, "SELL-C-sigma"). One workgroup per window.
__global__ void __launch_bounds__(kSellWindow) k_sell_sort(const int32_t *__restrict__ win_row,
                                                             const int64_t *__restrict__ rp,
                                                             int32_t *__restrict__ s_row) {
  __shared__ int32_t len[kSellWindow];
  const int64_t end = win_row[blockIdx.x + 1];
  for (int64_t w0 = win_row[blockIdx.x]; w0 < end; w0 += kSellWindow) {
    const int m = static_cast<int>(min(static_cast<int64_t>(kSellWindow), end - w0));
    const int i = threadIdx.x;
    __syncthreads();
    if (i < m) len[i] = static_cast<int32_t>(rp[w0 + i + 1] - rp[w0 + i]);
    __syncthreads();
    if (i < m) {
      // place of row i: rows that are longer, or as long and earlier, come first
      const int32_t li = len[i];
      int rank = 0;
      for (int j = 0; j < m; j++) rank += (len[j] > li || (len[j] == li && j < i)) ? 1 : 0;
      s_row[w0 + rank] = static_cast<int32_t>(w0 + i);
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_slice_meta(int64_t nslices, const int32_t *__restrict__ row0,
                                                        const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                        const int32_t *__restrict__ s_row,
                                                        int64_t *__restrict__ size) {
  // one wavefront per slice: each lane counts the off-diagonal entries of one row, the width is their maximum + 1
  const int64_t s = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (s >= nslices) return;
  const int64_t r0 = row0[s], r1 = row0[s + 1];
  int w = 1;
  if (r0 + lane < r1) {
    const int64_t p = s_row[r0 + lane];
    int offd = 0;
    for (int64_t e = rp[p]; e < rp[p + 1]; e++) offd += (ci[e] != p);
    w = offd + 1;
  }
  for (int off = 32; off > 0; off >>= 1) w = max(w, __shfl_xor(w, off, 64));
  if (lane == 0) size[s] = static_cast<int64_t>(w) * kSliceRows;
}

// one thread per (slice, lane)
__global__ void __launch_bounds__(kBlock) k_fill_sell(int64_t nslices, const int32_t *__restrict__ row0,
                                                       const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                       const double *__restrict__ va, const double *__restrict__ diag,
                                                       const int64_t *__restrict__ slice_ptr,
                                                       const int32_t *__restrict__ s_row,
                                                       int32_t *__restrict__ s_col, double *__restrict__ s_val) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t s = g / kSliceRows;
  const int lane = static_cast<int>(g % kSliceRows);
  if (s >= nslices || row0[s] + lane >= row0[s + 1]) return;
  const int64_t p = s_row[row0[s] + lane];  // the row at this position
  const int64_t off = slice_ptr[s];
  const int64_t w = (slice_ptr[s + 1] - off) / kSliceRows;
  s_col[off + lane] = static_cast<int32_t>(p);
  s_val[off + lane] = diag[p];
  int64_t k = 1;
  for (int64_t e = rp[p]; e < rp[p + 1]; e++) {
    if (ci[e] == p) continue;
    s_col[off + k * kSliceRows + lane] = ci[e];
    s_val[off + k * kSliceRows + lane] = va[e];
    k++;
  }
  for (; k < w; k++) {
    s_col[off + k * kSliceRows + lane] = static_cast<int32_t>(p);
    s_val[off + k * kSliceRows + lane] = 0.0;
  }
}

// couplings between distinct unknowns of one cell (the block of the block Gauss-Seidel smoother)
__global__ void __launch_bounds__(kBlock) k_ic_count(int64_t n, const int64_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci, const int32_t *__restrict__ agg_q,
                                                      int32_t *__restrict__ cnt) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t q = agg_q[p];
  int32_t c = 0;
  for (int64_t e = rp[p]; e < rp[p + 1]; e++) c += (ci[e] != p && agg_q[ci[e]] == q);
  cnt[p] = c;
}

__global__ void __launch_bounds__(kBlock) k_ic_fill(int64_t n, const int64_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, const double *__restrict__ va,
                                                     const int32_t *__restrict__ agg_q, const int32_t *__restrict__ ptr,
                                                     int32_t *__restrict__ col, double *__restrict__ val) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t q = agg_q[p];
  int32_t o = ptr[p];
  for (int64_t e = rp[p]; e < rp[p + 1]; e++)
    if (ci[e] != p && agg_q[ci[e]] == q) {
      col[o] = ci[e];
      val[o] = va[e];
      o++;
    }
}

// Level schedule of the in-cell substitution of big cells (more than kBigCell unknowns). The forward substitution
// of a cell takes its rows in ascending order and row p uses the new values of the coupled rows c < p; its
// dependency level is 1 + the largest level among those rows (0 if none), and rows of one level are independent.
// Backward: descending order, c > p. One thread per big cell (sequential over the cell, once at setup).
__global__ void __launch_bounds__(kBlock) k_big_flag(int64_t nL, const int32_t *__restrict__ crow, int32_t threshold,
                                                      int32_t *__restrict__ flag) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q < nL) flag[q] = (crow[q + 1] - crow[q]) > threshold ? 1 : 0;
}

__global__ void __launch_bounds__(kBlock) k_big_list(int64_t nL, const int32_t *__restrict__ flag,
                                                      const int32_t *__restrict__ pos, int32_t *__restrict__ cells) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q < nL && flag[q]) cells[pos[q]] = static_cast<int32_t>(q);
}

template <bool FWD>
__global__ void __launch_bounds__(kBlock) k_big_levels(int64_t nbig, const int32_t *__restrict__ cells,
                                                        const int32_t *__restrict__ crow,
                                                        const int32_t *__restrict__ icp,
                                                        const int32_t *__restrict__ icc, int32_t *__restrict__ lv,
                                                        int32_t *__restrict__ nptr) {
  const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= nbig) return;
  const int32_t q = cells[b], a = crow[q], e = crow[q + 1];
  int32_t depth = 0;
  for (int32_t i = 0; i < e - a; i++) {
    const int32_t p = FWD ? a + i : e - 1 - i;
    int32_t m = 0;
    for (int32_t k = icp[p]; k < icp[p + 1]; k++) {
      const int32_t c = icc[k];
      if (FWD ? c < p : c > p) m = max(m, lv[c] + 1);
    }
    lv[p] = m;
    depth = max(depth, m + 1);
  }
  nptr[b] = depth + 1;  // level starts plus the end
}

__global__ void __launch_bounds__(kBlock) k_big_rows_max(int64_t nbig, const int32_t *__restrict__ cells,
                                                          const int32_t *__restrict__ crow, int *__restrict__ out) {
  const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b < nbig) atomicMax(out, crow[cells[b] + 1] - crow[cells[b]]);
}

// rows of each big cell sorted by level (stable: ascending row within a level); lptr gets the level starts
__global__ void __launch_bounds__(kBlock) k_big_sched(int64_t nbig, const int32_t *__restrict__ cells,
                                                       const int32_t *__restrict__ crow, const int32_t *__restrict__ lv,
                                                       const int32_t *__restrict__ lofs, int32_t *__restrict__ lptr,
                                                       int32_t *__restrict__ sched) {
  const int64_t b = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= nbig) return;
  const int32_t q = cells[b], a = crow[q], e = crow[q + 1];
  int32_t *ptr = lptr + lofs[b];
  const int32_t depth = lofs[b + 1] - lofs[b] - 1;
  for (int32_t l = 0; l <= depth; l++) ptr[l] = 0;
  for (int32_t p = a; p < e; p++) ptr[lv[p] + 1]++;
  ptr[0] = a;
  for (int32_t l = 1; l <= depth; l++) ptr[l] += ptr[l - 1];
  // place rows, using ptr[l] as the cursor of level l (it ends at the start of level l + 1), then shift back
  for (int32_t p = a; p < e; p++) sched[ptr[lv[p]]++] = p;
  for (int32_t l = depth; l >= 1; l--) ptr[l] = ptr[l - 1];
  ptr[0] = a;
}

// ---------------------------------------------------------------------------------------------------------------
// Galerkin operators

__device__ inline void add_slot(double (&acc)[9], int s, double v) {
#pragma unroll
  for (int j = 0; j < 9; j++) acc[j] += (j == s) ? v : 0.0;
}

__device__ inline uint32_t lex_of_q(uint32_t q, int k) {
  uint32_t t1, t2;
  q_to_t(q, k, t1, t2);
  return (t2 << k) | t1;
}

// insertion sort of an overflow row by lexicographic column
__device__ inline void sort_ovf_row(int32_t *col, double *val, int32_t a, int32_t b, int k) {
  for (int32_t i = a + 1; i < b; i++) {
    const int32_t c = col[i];
    const double v = val[i];
    const uint32_t lc = lex_of_q(static_cast<uint32_t>(c), k);
    int32_t j = i - 1;
    while (j >= a && lex_of_q(static_cast<uint32_t>(col[j]), k) > lc) {
      col[j + 1] = col[j];
      val[j + 1] = val[j];
      j--;
    }
    col[j + 1] = c;
    val[j + 1] = v;
  }
}

// fine -> level L: one thread per cell; its rows are contiguous, so its entries are the range rp[crow[q]] ..
// rp[crow[q+1]] visited in order (rows ascending, entries in the caller's order)
__global__ void __launch_bounds__(kBlock) k_galerkin_fine(int L, int64_t nL, const int32_t *__restrict__ crow,
                                                           const int64_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const double *__restrict__ va,
                                                           const int32_t *__restrict__ agg_q, double *__restrict__ ax,
                                                           uint8_t *__restrict__ empty, int32_t *__restrict__ ovf_cnt,
                                                           int *flag) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nL) return;
  uint32_t t1, t2;
  q_to_t(static_cast<uint32_t>(q), L, t1, t2);
  const int64_t e0 = rp[crow[q]], e1 = rp[crow[q + 1]];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  int32_t cnt = 0;
  // the entries are gathered kGalBatch at a time so that their loads overlap; they are still summed one by one in
  // entry order
  constexpr int kGalBatch = 8;
  for (int64_t eb = e0; eb < e1; eb += kGalBatch) {
    int32_t col[kGalBatch];
    double val[kGalBatch];
    uint32_t agq[kGalBatch];
#pragma unroll
    for (int u = 0; u < kGalBatch; u++) {
      const bool in = eb + u < e1;
      col[u] = in ? ci[eb + u] : 0;
      val[u] = in ? va[eb + u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kGalBatch; u++) agq[u] = (eb + u < e1) ? static_cast<uint32_t>(agg_q[col[u]]) : 0u;
#pragma unroll
    for (int u = 0; u < kGalBatch; u++) {
      const int64_t e = eb + u;
      if (e >= e1) break;
      const uint32_t qq = agq[u];
      uint32_t u1, u2;
      q_to_t(qq, L, u1, u2);
      const int dx = static_cast<int>(u1) - static_cast<int>(t1), dy = static_cast<int>(u2) - static_cast<int>(t2);
      if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) {
        add_slot(acc, slot_of(dx, dy), val[u]);
      } else {
        bool first = true;
        for (int64_t e2 = e0; e2 < e; e2++)
          if (static_cast<uint32_t>(agg_q[ci[e2]]) == qq) { first = false; break; }
        cnt += first;
      }
    }
  }
  const bool emp = (crow[q] == crow[q + 1]);
  empty[q] = emp ? 1 : 0;
  if (emp) acc[0] = 1.0;
#pragma unroll
  for (int j = 0; j < 9; j++) ax[j * nL + q] = acc[j];
  ovf_cnt[q] = cnt;
  if (!emp && !(acc[0] > 0.0)) atomicOr(flag, F_NOT_SPD);
}

__global__ void __launch_bounds__(kBlock) k_galerkin_fine_ovf(int L, int64_t nL, const int32_t *__restrict__ crow,
                                                               const int64_t *__restrict__ rp,
                                                               const int32_t *__restrict__ ci,
                                                               const double *__restrict__ va,
                                                               const int32_t *__restrict__ agg_q,
                                                               const int32_t *__restrict__ optr,
                                                               int32_t *__restrict__ ocol, double *__restrict__ oval,
                                                               int *flag) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nL) return;
  int32_t o = optr[q];
  if (optr[q + 1] == o) return;
  uint32_t t1, t2;
  q_to_t(static_cast<uint32_t>(q), L, t1, t2);
  const int64_t e0 = rp[crow[q]], e1 = rp[crow[q + 1]];
  const uint32_t my_color = static_cast<uint32_t>(q) >> (2 * L - 2);
  for (int64_t e = e0; e < e1; e++) {
    const uint32_t qq = static_cast<uint32_t>(agg_q[ci[e]]);
    uint32_t u1, u2;
    q_to_t(qq, L, u1, u2);
    const int dx = static_cast<int>(u1) - static_cast<int>(t1), dy = static_cast<int>(u2) - static_cast<int>(t2);
    if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
    bool first = true;
    for (int64_t e2 = e0; e2 < e; e2++)
      if (static_cast<uint32_t>(agg_q[ci[e2]]) == qq) { first = false; break; }
    if (!first) continue;
    double s = 0.0;
    for (int64_t e2 = e; e2 < e1; e2++)
      if (static_cast<uint32_t>(agg_q[ci[e2]]) == qq) s += va[e2];
    ocol[o] = static_cast<int32_t>(qq);
    oval[o] = s;
    o++;
    if ((qq >> (2 * L - 2)) == my_color) atomicOr(flag, F_SAMECOLOR);
  }
  sort_ovf_row(ocol, oval, optr[q], optr[q + 1], L);
}

// level k -> level k-1: one thread per coarse cell M (Morton at level k-1); children c in the order 0, 1, 3, 2
// ((2T1,2T2), (2T1+1,2T2), (2T1+1,2T2+1), (2T1,2T2+1)), each child's 9 slots then its overflow entries.
struct CoarseSrc {
  int k;
  int64_t n;
  const double *ax;
  const uint8_t *empty;
  const int32_t *optr;
  const int32_t *ocol;
  const double *oval;
};

__constant__ int kChildOrder[4] = {0, 1, 3, 2};

__global__ void __launch_bounds__(kBlock) k_galerkin_coarse(CoarseSrc F, double *__restrict__ ax,
                                                             uint8_t *__restrict__ empty,
                                                             int32_t *__restrict__ ovf_cnt, int *flag) {
  const int kc = F.k - 1;
  const int64_t nc = F.n >> 2;
  const int64_t M = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (M >= nc) return;
  const uint32_t T1 = compact_bits(static_cast<uint32_t>(M)), T2 = compact_bits(static_cast<uint32_t>(M) >> 1);
  const uint32_t side = 1u << F.k;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  int32_t cnt = 0;
  bool all_empty = true;
  for (int oi = 0; oi < 4; oi++) {
    const int c = kChildOrder[oi];
    const int64_t q = c * nc + M;
    if (F.empty[q]) continue;
    all_empty = false;
    const uint32_t m = (static_cast<uint32_t>(M) << 2) | static_cast<uint32_t>(c);
    const int t1 = static_cast<int>(compact_bits(m)), t2 = static_cast<int>(compact_bits(m >> 1));
#pragma unroll
    for (int s = 0; s < 9; s++) {
      const int u1 = t1 + slot_dx(s), u2 = t2 + slot_dy(s);
      if (u1 < 0 || u2 < 0 || u1 >= static_cast<int>(side) || u2 >= static_cast<int>(side)) continue;
      add_slot(acc, slot_of((u1 >> 1) - static_cast<int>(T1), (u2 >> 1) - static_cast<int>(T2)), F.ax[s * F.n + q]);
    }
    if (F.optr)
      for (int32_t e = F.optr[q]; e < F.optr[q + 1]; e++) {
        const uint32_t mm = m_of_q(static_cast<uint32_t>(F.ocol[e]), F.k);
        const uint32_t P = mm >> 2;
        const int dX = static_cast<int>(compact_bits(P)) - static_cast<int>(T1);
        const int dY = static_cast<int>(compact_bits(P >> 1)) - static_cast<int>(T2);
        if (dX >= -1 && dX <= 1 && dY >= -1 && dY <= 1) {
          add_slot(acc, slot_of(dX, dY), F.oval[e]);
        } else {
          // first occurrence of this coarse target among the far entries visited so far
          bool first = true;
          for (int oj = 0; oj <= oi && first; oj++) {
            const int64_t qj = kChildOrder[oj] * nc + M;
            if (F.empty[qj]) continue;
            const int32_t eend = (oj == oi) ? e : F.optr[qj + 1];
            for (int32_t e2 = F.optr[qj]; e2 < eend; e2++)
              if ((m_of_q(static_cast<uint32_t>(F.ocol[e2]), F.k) >> 2) == P) { first = false; break; }
          }
          cnt += first;
        }
      }
  }
  const uint32_t qc = q_of_m(static_cast<uint32_t>(M), kc);
  empty[qc] = all_empty ? 1 : 0;
  if (all_empty) acc[0] = 1.0;
#pragma unroll
  for (int j = 0; j < 9; j++) ax[j * nc + qc] = acc[j];
  ovf_cnt[qc] = cnt;
  if (!all_empty && !(acc[0] > 0.0)) atomicOr(flag, F_NOT_SPD);
}

__global__ void __launch_bounds__(kBlock) k_galerkin_coarse_ovf(CoarseSrc F, const int32_t *__restrict__ optr,
                                                                 int32_t *__restrict__ ocol,
                                                                 double *__restrict__ oval, int *flag) {
  const int kc = F.k - 1;
  const int64_t nc = F.n >> 2;
  const int64_t M = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (M >= nc) return;
  const uint32_t qc = q_of_m(static_cast<uint32_t>(M), kc);
  int32_t o = optr[qc];
  if (optr[qc + 1] == o) return;
  const uint32_t T1 = compact_bits(static_cast<uint32_t>(M)), T2 = compact_bits(static_cast<uint32_t>(M) >> 1);
  const uint32_t my_color = (kc >= 1) ? (qc >> (2 * kc - 2)) : 0u;
  for (int oi = 0; oi < 4; oi++) {
    const int64_t q = kChildOrder[oi] * nc + M;
    if (F.empty[q]) continue;
    for (int32_t e = F.optr[q]; e < F.optr[q + 1]; e++) {
      const uint32_t P = m_of_q(static_cast<uint32_t>(F.ocol[e]), F.k) >> 2;
      const int dX = static_cast<int>(compact_bits(P)) - static_cast<int>(T1);
      const int dY = static_cast<int>(compact_bits(P >> 1)) - static_cast<int>(T2);
      if (dX >= -1 && dX <= 1 && dY >= -1 && dY <= 1) continue;
      bool first = true;
      for (int oj = 0; oj <= oi && first; oj++) {
        const int64_t qj = kChildOrder[oj] * nc + M;
        if (F.empty[qj]) continue;
        const int32_t eend = (oj == oi) ? e : F.optr[qj + 1];
        for (int32_t e2 = F.optr[qj]; e2 < eend; e2++)
          if ((m_of_q(static_cast<uint32_t>(F.ocol[e2]), F.k) >> 2) == P) { first = false; break; }
      }
      if (!first) continue;
      double s = 0.0;
      for (int oj = oi; oj < 4; oj++) {
        const int64_t qj = kChildOrder[oj] * nc + M;
        if (F.empty[qj]) continue;
        const int32_t ebeg = (oj == oi) ? e : F.optr[qj];
        for (int32_t e2 = ebeg; e2 < F.optr[qj + 1]; e2++)
          if ((m_of_q(static_cast<uint32_t>(F.ocol[e2]), F.k) >> 2) == P) s += F.oval[e2];
      }
      const uint32_t target = q_of_m(P, kc);
      ocol[o] = static_cast<int32_t>(target);
      oval[o] = s;
      o++;
      if (kc >= 1 && (target >> (2 * kc - 2)) == my_color) atomicOr(flag, F_SAMECOLOR);
    }
  }
  sort_ovf_row(ocol, oval, optr[qc], optr[qc + 1], kc);
}

// ---------------------------------------------------------------------------------------------------------------
// Octree (3D) variant of the setup kernels: the same steps with three coordinates, 8^k cells, 8 children and 27
// slots (the numbering and slot order are those of qa_internal.hpp). Sums are taken in the order of the 2D kernels:
// cells in order, a cell's rows ascending and each row's entries in the caller's order; below level L the children
// in child3_order, each child's 27 slots in order, then its overflow entries.

__device__ inline void q_to_t3(uint32_t q, int k, uint32_t &t1, uint32_t &t2, uint32_t &t3) {
  const uint32_t m = m_of_q3(q, k);
  t1 = compact3(m);
  t2 = compact3(m >> 1);
  t3 = compact3(m >> 2);
}

__device__ inline uint32_t lex_of_q3(uint32_t q, int k) {
  uint32_t t1, t2, t3;
  q_to_t3(q, k, t1, t2, t3);
  return (((t3 << k) | t2) << k) | t1;
}

__device__ inline void add_slot27(double (&acc)[27], int s, double v) {
#pragma unroll
  for (int j = 0; j < 27; j++) acc[j] += (j == s) ? v : 0.0;
}

__device__ inline void sort_ovf_row3(int32_t *col, double *val, int32_t a, int32_t b, int k) {
  for (int32_t i = a + 1; i < b; i++) {
    const int32_t c = col[i];
    const double v = val[i];
    const uint32_t lc = lex_of_q3(static_cast<uint32_t>(c), k);
    int32_t j = i - 1;
    while (j >= a && lex_of_q3(static_cast<uint32_t>(col[j]), k) > lc) {
      col[j + 1] = col[j];
      val[j + 1] = val[j];
      j--;
    }
    col[j + 1] = c;
    val[j + 1] = v;
  }
}

__global__ void __launch_bounds__(kBlock) k_validate3(int64_t n, int64_t nnz, const double *__restrict__ coords,
                                                       const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                       const double *__restrict__ va, int has_box, Box3 B,
                                                       int *flag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int f = 0;
  const int64_t r0 = rp[i], r1 = rp[i + 1];
  if (i == 0 && r0 != 0) f |= F_INVALID;
  if (i == n - 1 && r1 != nnz) f |= F_INVALID;
  if (r1 < r0 || r0 < 0 || r1 > nnz) f |= F_INVALID;
  for (int a = 0; a < 3; a++) {
    const double v = coords[3 * i + a];
    if (!isfinite(v)) f |= F_INVALID;
    else if (has_box && (v < B.v[2 * a] || v > B.v[2 * a + 1])) f |= F_INVALID;
  }
  if (!(f & F_INVALID)) {
    double dg = 0.0;
    for (int64_t e = r0; e < r1; e++) {
      const int32_t c = ci[e];
      if (c < 0 || c >= n) f |= F_INVALID;
      else if (c == i) dg += va[e];
    }
    if (!(dg > 0.0)) f |= F_NOT_SPD;
  }
  if (f) atomicOr(flag, f);
}

// bounding box of 3D points: per-workgroup min / max of each coordinate, then one workgroup over those
__global__ void __launch_bounds__(kBlock) k_bbox3_partial(int64_t n, const double *__restrict__ coords,
                                                           double *__restrict__ part) {
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    for (int a = 0; a < 3; a++) {
      mn[a] = fmin(mn[a], coords[3 * i + a]);
      mx[a] = fmax(mx[a], coords[3 * i + a]);
    }
  __shared__ double sm[6][kBlock];
  for (int a = 0; a < 3; a++) {
    sm[2 * a][threadIdx.x] = mn[a];
    sm[2 * a + 1][threadIdx.x] = mx[a];
  }
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off)
      for (int a = 0; a < 3; a++) {
        sm[2 * a][threadIdx.x] = fmin(sm[2 * a][threadIdx.x], sm[2 * a][threadIdx.x + off]);
        sm[2 * a + 1][threadIdx.x] = fmax(sm[2 * a + 1][threadIdx.x], sm[2 * a + 1][threadIdx.x + off]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int t = 0; t < 6; t++) part[blockIdx.x * 6 + t] = sm[t][0];
}

__global__ void k_bbox3_final(int nb, const double *__restrict__ part, double *__restrict__ box) {
  double b[6] = {INFINITY, -INFINITY, INFINITY, -INFINITY, INFINITY, -INFINITY};
  for (int i = 0; i < nb; i++)
    for (int a = 0; a < 3; a++) {
      b[2 * a] = fmin(b[2 * a], part[6 * i + 2 * a]);
      b[2 * a + 1] = fmax(b[2 * a + 1], part[6 * i + 2 * a + 1]);
    }
  for (int t = 0; t < 6; t++) box[t] = b[t];
}

// level-L cell of each unknown (the index formula of Section 4.2 on each of the three axes), as a color-major octree
// index, with its count
__global__ void __launch_bounds__(kBlock) k_cell_key3(int64_t n, const double *__restrict__ coords, Box3 B, int L,
                                                       int32_t *__restrict__ key, int32_t *__restrict__ cnt) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t t1 = axis_cell(coords[3 * i], B.v[0], B.v[1], L);
  const uint32_t t2 = axis_cell(coords[3 * i + 1], B.v[2], B.v[3], L);
  const uint32_t t3 = axis_cell(coords[3 * i + 2], B.v[4], B.v[5], L);
  const uint32_t q = q_of_m3(morton3(t1, t2, t3), L);
  key[i] = static_cast<int32_t>(q);
  atomicAdd(&cnt[q], 1);
}

// fine -> level L on an octree: one thread per cell, its rows' entries in order, 27 slots, far couplings counted
__global__ void __launch_bounds__(kBlock) k_galerkin_fine3(int L, int64_t nL, const int32_t *__restrict__ crow,
                                                            const int64_t *__restrict__ rp,
                                                            const int32_t *__restrict__ ci,
                                                            const double *__restrict__ va,
                                                            const int32_t *__restrict__ agg_q,
                                                            double *__restrict__ ax, uint8_t *__restrict__ empty,
                                                            int32_t *__restrict__ ovf_cnt, int *flag) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nL) return;
  uint32_t t1, t2, t3;
  q_to_t3(static_cast<uint32_t>(q), L, t1, t2, t3);
  const int64_t e0 = rp[crow[q]], e1 = rp[crow[q + 1]];
  double acc[27];
#pragma unroll
  for (int j = 0; j < 27; j++) acc[j] = 0.0;
  int32_t cnt = 0;
  for (int64_t e = e0; e < e1; e++) {
    const uint32_t qq = static_cast<uint32_t>(agg_q[ci[e]]);
    uint32_t u1, u2, u3;
    q_to_t3(qq, L, u1, u2, u3);
    const int dx = static_cast<int>(u1) - static_cast<int>(t1), dy = static_cast<int>(u2) - static_cast<int>(t2),
              dz = static_cast<int>(u3) - static_cast<int>(t3);
    if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) {
      add_slot27(acc, slot3_of(dx, dy, dz), va[e]);
    } else {
      bool first = true;
      for (int64_t e2 = e0; e2 < e; e2++)
        if (static_cast<uint32_t>(agg_q[ci[e2]]) == qq) { first = false; break; }
      cnt += first;
    }
  }
  const bool emp = (crow[q] == crow[q + 1]);
  empty[q] = emp ? 1 : 0;
  if (emp) acc[0] = 1.0;
#pragma unroll
  for (int j = 0; j < 27; j++) ax[j * nL + q] = acc[j];
  ovf_cnt[q] = cnt;
  if (!emp && !(acc[0] > 0.0)) atomicOr(flag, F_NOT_SPD);
}

__global__ void __launch_bounds__(kBlock) k_galerkin_fine3_ovf(int L, int64_t nL, const int32_t *__restrict__ crow,
                                                                const int64_t *__restrict__ rp,
                                                                const int32_t *__restrict__ ci,
                                                                const double *__restrict__ va,
                                                                const int32_t *__restrict__ agg_q,
                                                                const int32_t *__restrict__ optr,
                                                                int32_t *__restrict__ ocol, double *__restrict__ oval,
                                                                int *flag) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nL) return;
  int32_t o = optr[q];
  if (optr[q + 1] == o) return;
  uint32_t t1, t2, t3;
  q_to_t3(static_cast<uint32_t>(q), L, t1, t2, t3);
  const int64_t e0 = rp[crow[q]], e1 = rp[crow[q + 1]];
  const uint32_t my_color = static_cast<uint32_t>(q) >> (3 * L - 3);
  for (int64_t e = e0; e < e1; e++) {
    const uint32_t qq = static_cast<uint32_t>(agg_q[ci[e]]);
    uint32_t u1, u2, u3;
    q_to_t3(qq, L, u1, u2, u3);
    const int dx = static_cast<int>(u1) - static_cast<int>(t1), dy = static_cast<int>(u2) - static_cast<int>(t2),
              dz = static_cast<int>(u3) - static_cast<int>(t3);
    if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) continue;
    bool first = true;
    for (int64_t e2 = e0; e2 < e; e2++)
      if (static_cast<uint32_t>(agg_q[ci[e2]]) == qq) { first = false; break; }
    if (!first) continue;
    double sum = 0.0;
    for (int64_t e2 = e; e2 < e1; e2++)
      if (static_cast<uint32_t>(agg_q[ci[e2]]) == qq) sum += va[e2];
    ocol[o] = static_cast<int32_t>(qq);
    oval[o] = sum;
    o++;
    if ((qq >> (3 * L - 3)) == my_color) atomicOr(flag, F_SAMECOLOR);
  }
  sort_ovf_row3(ocol, oval, optr[q], optr[q + 1], L);
}

// level k -> level k-1 on an octree: one thread per coarse cell M (Morton at level k-1), its 8 children in
// child3_order, each child's 27 slots then its overflow entries
__global__ void __launch_bounds__(kBlock) k_galerkin_coarse3(CoarseSrc F, double *__restrict__ ax,
                                                              uint8_t *__restrict__ empty,
                                                              int32_t *__restrict__ ovf_cnt, int *flag) {
  const int kc = F.k - 1;
  const int64_t nc = F.n >> 3;
  const int64_t M = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (M >= nc) return;
  const uint32_t Mu = static_cast<uint32_t>(M);
  const int T1 = static_cast<int>(compact3(Mu)), T2 = static_cast<int>(compact3(Mu >> 1)),
            T3 = static_cast<int>(compact3(Mu >> 2));
  const int side = 1 << F.k;
  double acc[27];
#pragma unroll
  for (int j = 0; j < 27; j++) acc[j] = 0.0;
  int32_t cnt = 0;
  bool all_empty = true;
  for (int oi = 0; oi < 8; oi++) {
    const int c = child3_order(oi);
    const int64_t q = c * nc + M;
    if (F.empty[q]) continue;
    all_empty = false;
    const uint32_t m = (Mu << 3) | static_cast<uint32_t>(c);
    const int t1 = static_cast<int>(compact3(m)), t2 = static_cast<int>(compact3(m >> 1)),
              t3 = static_cast<int>(compact3(m >> 2));
    for (int s = 0; s < 27; s++) {
      const int u1 = t1 + slot3_dx(s), u2 = t2 + slot3_dy(s), u3 = t3 + slot3_dz(s);
      if (u1 < 0 || u2 < 0 || u3 < 0 || u1 >= side || u2 >= side || u3 >= side) continue;
      add_slot27(acc, slot3_of((u1 >> 1) - T1, (u2 >> 1) - T2, (u3 >> 1) - T3), F.ax[s * F.n + q]);
    }
    if (F.optr)
      for (int32_t e = F.optr[q]; e < F.optr[q + 1]; e++) {
        const uint32_t P = m_of_q3(static_cast<uint32_t>(F.ocol[e]), F.k) >> 3;
        const int dX = static_cast<int>(compact3(P)) - T1, dY = static_cast<int>(compact3(P >> 1)) - T2,
                  dZ = static_cast<int>(compact3(P >> 2)) - T3;
        if (dX >= -1 && dX <= 1 && dY >= -1 && dY <= 1 && dZ >= -1 && dZ <= 1) {
          add_slot27(acc, slot3_of(dX, dY, dZ), F.oval[e]);
        } else {
          bool first = true;
          for (int oj = 0; oj <= oi && first; oj++) {
            const int64_t qj = child3_order(oj) * nc + M;
            if (F.empty[qj]) continue;
            const int32_t eend = (oj == oi) ? e : F.optr[qj + 1];
            for (int32_t e2 = F.optr[qj]; e2 < eend; e2++)
              if ((m_of_q3(static_cast<uint32_t>(F.ocol[e2]), F.k) >> 3) == P) { first = false; break; }
          }
          cnt += first;
        }
      }
  }
  const uint32_t qc = q_of_m3(Mu, kc);
  empty[qc] = all_empty ? 1 : 0;
  if (all_empty) acc[0] = 1.0;
#pragma unroll
  for (int j = 0; j < 27; j++) ax[j * nc + qc] = acc[j];
  ovf_cnt[qc] = cnt;
  if (!all_empty && !(acc[0] > 0.0)) atomicOr(flag, F_NOT_SPD);
}

__global__ void __launch_bounds__(kBlock) k_galerkin_coarse3_ovf(CoarseSrc F, const int32_t *__restrict__ optr,
                                                                  int32_t *__restrict__ ocol,
                                                                  double *__restrict__ oval, int *flag) {
  const int kc = F.k - 1;
  const int64_t nc = F.n >> 3;
  const int64_t M = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (M >= nc) return;
  const uint32_t Mu = static_cast<uint32_t>(M);
  const uint32_t qc = q_of_m3(Mu, kc);
  int32_t o = optr[qc];
  if (optr[qc + 1] == o) return;
  const int T1 = static_cast<int>(compact3(Mu)), T2 = static_cast<int>(compact3(Mu >> 1)),
            T3 = static_cast<int>(compact3(Mu >> 2));
  const uint32_t my_color = (kc >= 1) ? (qc >> (3 * kc - 3)) : 0u;
  for (int oi = 0; oi < 8; oi++) {
    const int64_t q = child3_order(oi) * nc + M;
    if (F.empty[q]) continue;
    for (int32_t e = F.optr[q]; e < F.optr[q + 1]; e++) {
      const uint32_t P = m_of_q3(static_cast<uint32_t>(F.ocol[e]), F.k) >> 3;
      const int dX = static_cast<int>(compact3(P)) - T1, dY = static_cast<int>(compact3(P >> 1)) - T2,
                dZ = static_cast<int>(compact3(P >> 2)) - T3;
      if (dX >= -1 && dX <= 1 && dY >= -1 && dY <= 1 && dZ >= -1 && dZ <= 1) continue;
      bool first = true;
      for (int oj = 0; oj <= oi && first; oj++) {
        const int64_t qj = child3_order(oj) * nc + M;
        if (F.empty[qj]) continue;
        const int32_t eend = (oj == oi) ? e : F.optr[qj + 1];
        for (int32_t e2 = F.optr[qj]; e2 < eend; e2++)
          if ((m_of_q3(static_cast<uint32_t>(F.ocol[e2]), F.k) >> 3) == P) { first = false; break; }
      }
      if (!first) continue;
      double sum = 0.0;
      for (int oj = oi; oj < 8; oj++) {
        const int64_t qj = child3_order(oj) * nc + M;
        if (F.empty[qj]) continue;
        const int32_t ebeg = (oj == oi) ? e : F.optr[qj];
        for (int32_t e2 = ebeg; e2 < F.optr[qj + 1]; e2++)
          if ((m_of_q3(static_cast<uint32_t>(F.ocol[e2]), F.k) >> 3) == P) sum += F.oval[e2];
      }
      const uint32_t target = q_of_m3(P, kc);
      ocol[o] = static_cast<int32_t>(target);
      oval[o] = sum;
      o++;
      if (kc >= 1 && (target >> (3 * kc - 3)) == my_color) atomicOr(flag, F_SAMECOLOR);
    }
  }
  sort_ovf_row3(ocol, oval, optr[qc], optr[qc + 1], kc);
}

__global__ void __launch_bounds__(kBlock) k_densify_level3(int k, int64_t n, const double *__restrict__ ax,
                                                            const int32_t *__restrict__ optr,
                                                            const int32_t *__restrict__ ocol,
                                                            const double *__restrict__ oval,
                                                            double *__restrict__ dense) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n) return;
  uint32_t t1, t2, t3;
  q_to_t3(static_cast<uint32_t>(q), k, t1, t2, t3);
  const int side = 1 << k;
  for (int s = 0; s < 27; s++) {
    const int u1 = static_cast<int>(t1) + slot3_dx(s), u2 = static_cast<int>(t2) + slot3_dy(s),
              u3 = static_cast<int>(t3) + slot3_dz(s);
    if (u1 < 0 || u2 < 0 || u3 < 0 || u1 >= side || u2 >= side || u3 >= side) continue;
    dense[q * n + q_of_m3(morton3(u1, u2, u3), k)] = ax[s * n + q];
  }
  if (optr)
    for (int32_t e = optr[q]; e < optr[q + 1]; e++) dense[q * n + ocol[e]] = oval[e];
}

// ---------------------------------------------------------------------------------------------------------------
// coarsest level: dense matrix, Cholesky, explicit inverse (one workgroup; n <= 1024)

__global__ void __launch_bounds__(kBlock) k_densify_level(int k, int64_t n, const double *__restrict__ ax,
                                                           const int32_t *__restrict__ optr,
                                                           const int32_t *__restrict__ ocol,
                                                           const double *__restrict__ oval, double *__restrict__ dense) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n) return;
  uint32_t t1, t2;
  q_to_t(static_cast<uint32_t>(q), k, t1, t2);
  const int side = 1 << k;
  for (int s = 0; s < 9; s++) {
    const int u1 = static_cast<int>(t1) + slot_dx(s), u2 = static_cast<int>(t2) + slot_dy(s);
    if (u1 < 0 || u2 < 0 || u1 >= side || u2 >= side) continue;
    dense[q * n + q_of_m(morton(u1, u2), k)] = ax[s * n + q];
  }
  if (optr)
    for (int32_t e = optr[q]; e < optr[q + 1]; e++) dense[q * n + ocol[e]] = oval[e];
}

__global__ void __launch_bounds__(kBlock) k_densify_csr(int64_t n, const int64_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci, const double *__restrict__ va,
                                                         double *__restrict__ dense) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t e = rp[i]; e < rp[i + 1]; e++) dense[i * n + ci[e]] += va[e];
}

constexpr int kCholLds = 64;
constexpr int kCholThreads = 1024;

// Dense inverse of the coarsest matrix through its Cholesky factor: A = L L^t, Y = L^{-1}, A^{-1} = Y^t Y. One
// workgroup; every phase is spread over all its threads, and each entry receives its updates in the same order as
// the textbook inner-product forms (increasing summation index), so the result does not depend on the thread count.
__global__ void __launch_bounds__(kCholThreads) k_chol_inverse(int n, double *__restrict__ ag,
                                                                double *__restrict__ yg, double *__restrict__ ainv,
                                                                int *flag) {
  // the factor and L^{-1} live in LDS when they fit (n <= 64: 2 x 32 KB), else in the global scratch given
  __shared__ double al[kCholLds * kCholLds], yl[kCholLds * kCholLds];
  const bool lds = n <= kCholLds;
  double *a = lds ? al : ag;
  double *y = lds ? yl : yg;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int t = tid; t < n * n; t += nt) {
    if (lds) a[t] = ag[t];
    y[t] = (t / n == t % n) ? 1.0 : 0.0;
  }
  __syncthreads();
  // right-looking factorisation: once column j is final, entry (i, k) of the trailing lower triangle subtracts
  // l_ij l_kj, so entry (i, j) sees the subtractions for k = 0, 1, ..., j-1 in order
  for (int j = 0; j < n; j++) {
    if (tid == 0) {
      double d = a[j * n + j];
      if (!(d > 0.0)) {
        atomicOr(flag, F_NOT_SPD);
        d = 1.0;
      }
      a[j * n + j] = sqrt(d);
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < n; i += nt) a[i * n + j] = a[i * n + j] / a[j * n + j];
    __syncthreads();
    const int m = n - j - 1;
    for (int t = tid; t < m * m; t += nt) {
      const int i = j + 1 + t / m, k = j + 1 + t % m;
      if (k <= i) a[i * n + k] -= a[i * n + j] * a[k * n + j];
    }
    __syncthreads();
  }
  // Y = L^{-1} by forward substitution on the identity, row by row: row i is final once divided by l_ii, and then
  // every later row r subtracts l_ri times it (entry (r, c) sees the rows c, c+1, ..., r-1 in order)
  for (int i = 0; i < n; i++) {
    for (int c = tid; c <= i; c += nt) y[i * n + c] = y[i * n + c] / a[i * n + i];
    __syncthreads();
    const int rows = n - i - 1, cols = i + 1;
    for (int t = tid; t < rows * cols; t += nt) {
      const int r = i + 1 + t / cols, c = t % cols;
      y[r * n + c] -= a[r * n + i] * y[i * n + c];
    }
    __syncthreads();
  }
  // A^{-1} = Y^t Y
  for (int idx = tid; idx < n * n; idx += nt) {
    const int i = idx / n, j = idx % n;
    double s = 0.0;
    for (int k = max(i, j); k < n; k++) s += y[k * n + i] * y[k * n + j];
    ainv[idx] = s;
  }
}

template <class S, class D>
__global__ void __launch_bounds__(kBlock) k_convert(int64_t n, const S *__restrict__ src, D *__restrict__ dst) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = static_cast<D>(src[i]);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_iota(int64_t n, T *__restrict__ v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) v[i] = static_cast<T>(i);
}

static inline unsigned nblk(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

// Section 3.1: L = max{l : (2^dim)^l < n}; the coarsest level is the first k with (2^dim)^k <= coarse_max
static int depth_rule(int64_t n, int coarse_max, int &L, int &kc, int dim = 2) {
  if (n <= coarse_max) {
    L = kc = -1;
    return 1;
  }
  int l = 0;
  while ((static_cast<int64_t>(1) << (dim * (l + 1))) < n) l++;
  int k = l;
  while (k > 0 && (static_cast<int64_t>(1) << (dim * k)) > coarse_max) k--;
  L = l;
  kc = k;
  return 1 + (l - k + 1);
}

// Small device-to-host reads of setup (counts, flags, the box) go through the hierarchy's pinned scalar slot. A copy
// into pageable memory is staged by the runtime and waits on its own, so a loop of them drains the stream once per
// value; into the pinned slot the copies of one batch are queued together and waited on once.
struct ReadBatch {
  amg_hierarchy *h;
  struct Item {
    void *dst;
    size_t off, bytes;
  };
  Item items[2 * kMaxColors + 2];
  int count = 0;
  size_t used = 0;
  explicit ReadBatch(amg_hierarchy *hh) : h(hh) {}
  amg_status add(void *dst, const void *src, size_t bytes) {
    if (!h->host_scal || count == static_cast<int>(sizeof(items) / sizeof(items[0])) ||
        used + bytes > sizeof(double) * kScalars)
      return AMG_ERR_INVALID;  // a batch larger than the slot is a bug of the caller
    QA_HIP(hipMemcpyAsync(reinterpret_cast<char *>(h->host_scal) + used, src, bytes, hipMemcpyDeviceToHost,
                          h->stream));
    items[count++] = Item{dst, used, bytes};
    used += (bytes + 7) & ~static_cast<size_t>(7);
    return AMG_OK;
  }
  amg_status finish() {
    QA_HIP(hipStreamSynchronize(h->stream));
    for (int i = 0; i < count; i++)
      std::memcpy(items[i].dst, reinterpret_cast<const char *>(h->host_scal) + items[i].off, items[i].bytes);
    count = 0;
    used = 0;
    return AMG_OK;
  }
};

static amg_status read_flag(amg_hierarchy *h, int &f) {
  ReadBatch rb(h);
  QA_TRY(rb.add(&f, h->dflag, sizeof(int)));
  return rb.finish();
}

static amg_status sell_values(amg_hierarchy *h);

// a temporary device buffer of the build, returned on every path
struct BuildTmp {
  amg_hierarchy *h;
  void *p;
  BuildTmp(amg_hierarchy *hh, size_t bytes) : h(hh), p(tmp_alloc(hh, hh->stream, std::max<size_t>(bytes, 8))) {}
  ~BuildTmp() { tmp_free(h, h->stream, p); }
  template <class T>
  T *as() const { return static_cast<T *>(p); }
};

static amg_status build_sell(amg_hierarchy *h) {
  FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  const int nc = F.ncolor;
  const int64_t n = h->n;
  // windows
  if (F.crow) {
    const int64_t nL = static_cast<int64_t>(1) << (h->dim * h->L);
    const int largest = h->opt.smoother ? kBlockMax : kBigCell;  // cells solved by one thread
    F.win_band = kSellWindow + 1 - largest;
    BuildTmp tmark(h, sizeof(int32_t) * nL), twidx(h, sizeof(int32_t) * (nL + 1));
    int32_t *mark = tmark.as<int32_t>(), *widx = twidx.as<int32_t>();
    if (!mark || !widx) return AMG_ERR_NOMEM;
    k_win_mark<<<nblk(nL), kBlock, 0, s>>>(nL, nL / nc, F.crow, F.win_band, mark);
    QA_LAUNCH_CHECK();
    QA_TRY(scan_exclusive_i32(mark, widx, nL, s, h));
    int32_t cw[kMaxColors + 1];
    ReadBatch rb(h);
    for (int c = 0; c < nc; c++) QA_TRY(rb.add(&cw[c], widx + c * (nL / nc), sizeof(int32_t)));
    QA_TRY(rb.add(&cw[nc], widx + nL, sizeof(int32_t)));
    QA_TRY(rb.finish());
    F.nwin = cw[nc];
    for (int c = 0; c <= nc; c++) F.color_win[c] = cw[c];
    F.win_q = dalloc_n<int32_t>(h, F.nwin + 1);
    F.win_row = dalloc_n<int32_t>(h, F.nwin + 1);
    if (!F.win_q || !F.win_row) return AMG_ERR_NOMEM;
    k_win_fill<<<nblk(nL), kBlock, 0, s>>>(nL, F.crow, mark, widx, F.win_q, F.win_row);
    // couplings between cells of one color: the fused smoother phase must then not read the color's own rows from u
    BuildTmp tflag(h, sizeof(int));
    int *flag = tflag.as<int>();
    if (!flag) return AMG_ERR_NOMEM;
    QA_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    k_same_color<<<nblk(n), kBlock, 0, s>>>(n, nL / nc, F.rp, F.ci, F.agg_q, flag);
    QA_LAUNCH_CHECK();
    int hf = 0;
    QA_TRY(rb.add(&hf, flag, sizeof(int)));
    QA_TRY(rb.finish());
    F.same_color = hf != 0;
  } else {
    F.win_band = kSellWindow;
    F.nwin = (n + kSellWindow - 1) / kSellWindow;
    F.color_win[0] = 0;
    for (int c = 1; c <= nc; c++) F.color_win[c] = F.nwin;
    F.win_row = dalloc_n<int32_t>(h, F.nwin + 1);
    if (!F.win_row) return AMG_ERR_NOMEM;
    k_win_fixed<<<nblk(F.nwin + 1), kBlock, 0, s>>>(F.nwin, n, F.win_row);
  }
  QA_LAUNCH_CHECK();
  // slices
  BuildTmp tnsl(h, sizeof(int64_t) * std::max<int64_t>(F.nwin, 1));
  int64_t *nsl = tnsl.as<int64_t>();
  F.win_slice = dalloc_n<int64_t>(h, F.nwin + 1);
  if (!nsl || !F.win_slice) return AMG_ERR_NOMEM;
  if (F.nwin) k_win_nslices<<<nblk(F.nwin), kBlock, 0, s>>>(F.nwin, F.win_row, nsl);
  QA_LAUNCH_CHECK();
  QA_TRY(scan_exclusive_i64(nsl, F.win_slice, F.nwin, s, h));
  {
    int64_t cs[kMaxColors + 1];
    ReadBatch rb(h);
    for (int c = 0; c <= nc; c++) QA_TRY(rb.add(&cs[c], F.win_slice + F.color_win[c], sizeof(int64_t)));
    QA_TRY(rb.finish());
    for (int c = 0; c <= nc; c++) F.color_slice[c] = cs[c];
    F.nslices = cs[nc];
  }
  int64_t *size = dalloc_n<int64_t>(h, F.nslices + 1);
  F.slice_row0 = dalloc_n<int32_t>(h, F.nslices + 1);
  F.slice_ptr = dalloc_n<int64_t>(h, F.nslices + 1);
  F.s_row = dalloc_n<int32_t>(h, std::max<int64_t>(n, 1));
  if (!size || !F.slice_row0 || !F.slice_ptr || !F.s_row) return AMG_ERR_NOMEM;
  if (F.nwin) {
    k_slice_starts<<<nblk(F.nwin), kBlock, 0, s>>>(F.nwin, F.win_row, F.win_slice, F.slice_row0);
    k_sell_sort<<<static_cast<unsigned>(F.nwin), kSellWindow, 0, s>>>(F.win_row, F.rp, F.s_row);
  } else {
    QA_HIP(hipMemsetAsync(F.slice_row0, 0, sizeof(int32_t), s));
  }
  if (F.nslices) k_slice_meta<<<nblk(64 * F.nslices), kBlock, 0, s>>>(F.nslices, F.slice_row0, F.rp, F.ci, F.s_row,
                                                                      size);
  QA_LAUNCH_CHECK();
  QA_TRY(scan_exclusive_i64(size, F.slice_ptr, F.nslices, s, h));
  {
    ReadBatch rb(h);
    QA_TRY(rb.add(&F.sell_entries, F.slice_ptr + F.nslices, sizeof(int64_t)));
    QA_TRY(rb.finish());
  }
  F.s_col = dalloc_n<int32_t>(h, F.sell_entries);
  F.s_val64 = dalloc_n<double>(h, F.sell_entries);
  F.s_val32 = dalloc_n<float>(h, F.sell_entries);
  if (!F.s_col || !F.s_val64 || !F.s_val32) return AMG_ERR_NOMEM;
  return sell_values(h);
}

// the sliced ELL's entries (columns and values, FP64 and FP32) and the FP32 diagonal from the permuted CSR
static amg_status sell_values(amg_hierarchy *h) {
  FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  if (F.nslices)
    k_fill_sell<<<nblk(64 * F.nslices), kBlock, 0, s>>>(F.nslices, F.slice_row0, F.rp, F.ci, F.va, F.diag64,
                                                        F.slice_ptr, F.s_row, F.s_col, F.s_val64);
  QA_LAUNCH_CHECK();
  k_convert<double, float><<<nblk(F.sell_entries), kBlock, 0, s>>>(F.sell_entries, F.s_val64, F.s_val32);
  QA_LAUNCH_CHECK();
  k_convert<double, float><<<nblk(F.n), kBlock, 0, s>>>(F.n, F.diag64, F.diag32);
  QA_LAUNCH_CHECK();
  return AMG_OK;
}

static amg_status build_coarsest_inverse(amg_hierarchy *h, const double *dense_src_filled, int64_t nc) {
  hipStream_t s = h->stream;
  double *y = dalloc_n<double>(h, nc * nc);
  if (!h->ainv) h->ainv = dalloc_n<double>(h, nc * nc);  // kept by a values update
  if (!y || !h->ainv) return AMG_ERR_NOMEM;
  k_chol_inverse<<<1, kCholThreads, 0, s>>>(static_cast<int>(nc), const_cast<double *>(dense_src_filled), y, h->ainv,
                                       h->dflag);
  QA_LAUNCH_CHECK();
  h->nc = nc;
  return AMG_OK;
}

static amg_status build_single_level(amg_hierarchy *h, const int64_t *row_ptr, const int32_t *col_idx,
                                     const double *vals, int64_t nnz) {
  FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  const int64_t n = h->n;
  F.perm = dalloc_n<int32_t>(h, n);
  F.iperm = dalloc_n<int32_t>(h, n);
  F.rp = dalloc_n<int64_t>(h, n + 1);
  F.ci = dalloc_n<int32_t>(h, nnz);
  F.va = dalloc_n<double>(h, nnz);
  F.diag64 = dalloc_n<double>(h, n);
  F.diag32 = dalloc_n<float>(h, n);
  int64_t *len = dalloc_n<int64_t>(h, n);
  double *dense = dalloc_n<double>(h, n * n);
  if (!F.perm || !F.iperm || !F.rp || !F.ci || !F.va || !F.diag64 || !F.diag32 || !len || !dense)
    return AMG_ERR_NOMEM;
  k_iota<int32_t><<<nblk(n), kBlock, 0, s>>>(n, F.perm);
  QA_LAUNCH_CHECK();
  k_inverse_perm<<<nblk(n), kBlock, 0, s>>>(n, F.perm, nullptr, F.iperm, nullptr, row_ptr, len);
  QA_LAUNCH_CHECK();
  QA_TRY(scan_exclusive_i64(len, F.rp, n, s, h));
  k_permute_csr<<<nblk(8 * n), kBlock, 0, s>>>(n, F.perm, F.iperm, row_ptr, col_idx, vals, F.rp, F.ci, F.va,
                                               F.diag64);
  k_row_diag<<<nblk(n), kBlock, 0, s>>>(n, F.rp, F.ci, F.va, F.diag64);
  QA_LAUNCH_CHECK();
  F.color_row[0] = 0;
  for (int c = 1; c <= F.ncolor; c++) F.color_row[c] = n;
  QA_TRY(build_sell(h));
  QA_HIP(hipMemsetAsync(dense, 0, sizeof(double) * n * n, s));
  k_densify_csr<<<nblk(n), kBlock, 0, s>>>(n, row_ptr, col_idx, vals, dense);
  QA_LAUNCH_CHECK();
  return build_coarsest_inverse(h, dense, n);
}

// cells of more than `threshold` unknowns, ascending: *cells (device), *count, and the first of each color in
// first[0..4] (first[4] = count)
static amg_status cell_list(amg_hierarchy *h, int32_t threshold, int32_t **cells, int64_t *count,
                            int64_t first[kMaxColors + 1]) {
  FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  const int64_t nL = static_cast<int64_t>(1) << (h->dim * h->L);
  const int nc = F.ncolor;
  int32_t *flag = dalloc_n<int32_t>(h, nL);
  int32_t *pos = dalloc_n<int32_t>(h, nL + 1);
  if (!flag || !pos) return AMG_ERR_NOMEM;
  k_big_flag<<<nblk(nL), kBlock, 0, s>>>(nL, F.crow, threshold, flag);
  QA_LAUNCH_CHECK();
  QA_TRY(scan_exclusive_i32(flag, pos, nL, s, h));
  int32_t bc[kMaxColors + 1];
  ReadBatch rb(h);
  for (int c = 0; c <= nc; c++) QA_TRY(rb.add(&bc[c], pos + c * (nL / nc), sizeof(int32_t)));
  QA_TRY(rb.finish());
  for (int c = 0; c <= nc; c++) first[c] = bc[c];
  *count = bc[nc];
  *cells = nullptr;
  if (*count == 0) return AMG_OK;
  *cells = dalloc_n<int32_t>(h, *count);
  if (!*cells) return AMG_ERR_NOMEM;
  k_big_list<<<nblk(nL), kBlock, 0, s>>>(nL, flag, pos, *cells);
  QA_LAUNCH_CHECK();
  return AMG_OK;
}

// factor size of a cell for the exact-block smoother (packed lower triangle, m (m + 1) / 2 for m <= kBlockMax,
// else 0)
__global__ void __launch_bounds__(kBlock) k_block_size(int64_t nL, const int32_t *__restrict__ crow,
                                                        int64_t *__restrict__ size) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nL) return;
  const int64_t m = crow[q + 1] - crow[q];
  size[q] = m <= kBlockMax ? m * (m + 1) / 2 : 0;
}

// position of (i, j), j <= i, in a packed lower triangle (row-major)
__device__ inline int packed_ij(int i, int j) { return i * (i + 1) / 2 + j; }

// The lower triangle of a cell's diagonal block (its unknowns ascending; the diagonal as summed for the smoother,
// each in-cell coupling below the diagonal added in the caller's entry order) and its Cholesky factor in place:
// column by column, each entry's inner product over the earlier columns in ascending order, then the division by
// the diagonal (the coarsest factor's order, which reads only the lower triangle). One thread per cell.
__global__ void __launch_bounds__(kBlock) k_block_factor(int64_t nL, const int32_t *__restrict__ crow,
                                                          const int32_t *__restrict__ icp,
                                                          const int32_t *__restrict__ icc,
                                                          const double *__restrict__ icv,
                                                          const double *__restrict__ diag,
                                                          const int64_t *__restrict__ boff, double *__restrict__ fac,
                                                          int *flag) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nL) return;
  const int32_t r0 = crow[q];
  const int m = crow[q + 1] - r0;
  if (m == 0 || m > kBlockMax) return;
  double *a = fac + boff[q];
  for (int i = 0; i < m; i++) {
    a[packed_ij(i, i)] = diag[r0 + i];
    for (int32_t e = icp[r0 + i]; e < icp[r0 + i + 1]; e++) {
      const int j = icc[e] - r0;
      if (j < i) a[packed_ij(i, j)] += icv[e];
    }
  }
  for (int j = 0; j < m; j++) {
    double d = a[packed_ij(j, j)];
    for (int k = 0; k < j; k++) d -= a[packed_ij(j, k)] * a[packed_ij(j, k)];
    if (!(d > 0.0)) {
      atomicOr(flag, F_NOT_SPD);
      d = 1.0;
    }
    const double ljj = sqrt(d);
    a[packed_ij(j, j)] = ljj;
    for (int i = j + 1; i < m; i++) {
      double s = a[packed_ij(i, j)];
      for (int k = 0; k < j; k++) s -= a[packed_ij(i, k)] * a[packed_ij(j, k)];
      a[packed_ij(i, j)] = s / ljj;
    }
  }
}

// in-cell couplings' values (FP64 and FP32) from the permuted CSR
static amg_status ic_values(amg_hierarchy *h) {
  FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  k_ic_fill<<<nblk(F.n), kBlock, 0, s>>>(F.n, F.rp, F.ci, F.va, F.agg_q, F.ic_ptr, F.ic_col, F.ic_val64);
  QA_LAUNCH_CHECK();
  if (F.ic_nnz) {
    k_convert<double, float><<<nblk(F.ic_nnz), kBlock, 0, s>>>(F.ic_nnz, F.ic_val64, F.ic_val32);
    QA_LAUNCH_CHECK();
  }
  return AMG_OK;
}

// the cells' packed Cholesky factors (FP64, then rounded to FP32) into the arrays sized at setup
static amg_status block_values(amg_hierarchy *h) {
  FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  const int64_t nL = static_cast<int64_t>(1) << (h->dim * h->L);
  QA_HIP(hipMemsetAsync(F.bfac64, 0, sizeof(double) * std::max<int64_t>(F.bfac_n, 1), s));
  k_block_factor<<<nblk(nL), kBlock, 0, s>>>(nL, F.crow, F.ic_ptr, F.ic_col, F.ic_val64, F.diag64, F.boff, F.bfac64,
                                             h->dflag);
  QA_LAUNCH_CHECK();
  if (F.bfac_n > 0) {
    k_convert<double, float><<<nblk(F.bfac_n), kBlock, 0, s>>>(F.bfac_n, F.bfac64, F.bfac32);
    QA_LAUNCH_CHECK();
  }
  return AMG_OK;
}

// Galerkin operator of hierarchy level l (eq. 11 from the fine level, restriction of level l-1 below it), FP64 and
// FP32. fresh: allocate the level and size its overflow list; otherwise refill the arrays in place (a values update
// on the same pattern, whose overflow positions and colour flags are unchanged).
static amg_status level_values(amg_hierarchy *h, int l, bool fresh) {
  FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  const int L = h->L;
  QuadLevel &Q = h->lev[l];
  const bool oct = h->dim == 3;
  if (fresh) {
    Q.k = L - (l - 1);
    Q.n = static_cast<int64_t>(1) << (h->dim * Q.k);
    Q.ns = oct ? 27 : 9;
    Q.ax64 = dalloc_n<double>(h, Q.ns * Q.n);
    Q.ax32 = dalloc_n<float>(h, Q.ns * Q.n);
    Q.empty = dalloc_n<uint8_t>(h, Q.n);
    Q.optr = dalloc_n<int32_t>(h, Q.n + 1);
    if (!Q.ax64 || !Q.ax32 || !Q.empty || !Q.optr) return AMG_ERR_NOMEM;
  }
  int32_t *ocnt = dalloc_n<int32_t>(h, Q.n);
  if (!ocnt) return AMG_ERR_NOMEM;
  CoarseSrc src{};
  if (l == 1) {
    if (oct)
      k_galerkin_fine3<<<nblk(Q.n), kBlock, 0, s>>>(L, Q.n, F.crow, F.rp, F.ci, F.va, F.agg_q, Q.ax64, Q.empty,
                                                     ocnt, h->dflag);
    else
      k_galerkin_fine<<<nblk(Q.n), kBlock, 0, s>>>(L, Q.n, F.crow, F.rp, F.ci, F.va, F.agg_q, Q.ax64, Q.empty, ocnt,
                                                    h->dflag);
  } else {
    const QuadLevel &P = h->lev[l - 1];
    src = CoarseSrc{P.k, P.n, P.ax64, P.empty, P.ovf_nnz ? P.optr : nullptr, P.ocol, P.oval64};
    if (oct) k_galerkin_coarse3<<<nblk(Q.n), kBlock, 0, s>>>(src, Q.ax64, Q.empty, ocnt, h->dflag);
    else k_galerkin_coarse<<<nblk(Q.n), kBlock, 0, s>>>(src, Q.ax64, Q.empty, ocnt, h->dflag);
  }
  QA_LAUNCH_CHECK();
  if (fresh) {
    QA_TRY(scan_exclusive_i32(ocnt, Q.optr, Q.n, s, h));
    int32_t on = 0;
    {
      ReadBatch rb(h);
      QA_TRY(rb.add(&on, Q.optr + Q.n, sizeof(int32_t)));
      QA_TRY(rb.finish());
    }
    Q.ovf_nnz = on;
    if (on) {
      Q.ocol = dalloc_n<int32_t>(h, on);
      Q.oval64 = dalloc_n<double>(h, on);
      Q.oval32 = dalloc_n<float>(h, on);
      if (!Q.ocol || !Q.oval64 || !Q.oval32) return AMG_ERR_NOMEM;
    }
  }
  if (Q.ovf_nnz) {
    QA_HIP(hipMemsetAsync(h->dflag + 1, 0, sizeof(int), s));
    if (l == 1 && oct)
      k_galerkin_fine3_ovf<<<nblk(Q.n), kBlock, 0, s>>>(L, Q.n, F.crow, F.rp, F.ci, F.va, F.agg_q, Q.optr, Q.ocol,
                                                         Q.oval64, h->dflag + 1);
    else if (l == 1)
      k_galerkin_fine_ovf<<<nblk(Q.n), kBlock, 0, s>>>(L, Q.n, F.crow, F.rp, F.ci, F.va, F.agg_q, Q.optr, Q.ocol,
                                                        Q.oval64, h->dflag + 1);
    else if (oct)
      k_galerkin_coarse3_ovf<<<nblk(Q.n), kBlock, 0, s>>>(src, Q.optr, Q.ocol, Q.oval64, h->dflag + 1);
    else
      k_galerkin_coarse_ovf<<<nblk(Q.n), kBlock, 0, s>>>(src, Q.optr, Q.ocol, Q.oval64, h->dflag + 1);
    QA_LAUNCH_CHECK();
    if (fresh) {
      int sc = 0;
      ReadBatch rb(h);
      QA_TRY(rb.add(&sc, h->dflag + 1, sizeof(int)));
      QA_TRY(rb.finish());
      Q.same_color_ovf = (sc & F_SAMECOLOR) ? 1 : 0;
    }
    k_convert<double, float><<<nblk(Q.ovf_nnz), kBlock, 0, s>>>(Q.ovf_nnz, Q.oval64, Q.oval32);
    QA_LAUNCH_CHECK();
  }
  k_convert<double, float><<<nblk(Q.ns * Q.n), kBlock, 0, s>>>(Q.ns * Q.n, Q.ax64, Q.ax32);
  QA_LAUNCH_CHECK();
  return AMG_OK;
}

// the coarsest level densified and inverted through its Cholesky factor
static amg_status coarsest_values(amg_hierarchy *h) {
  hipStream_t s = h->stream;
  const QuadLevel &C = h->lev[h->nlev - 1];
  double *dense = dalloc_n<double>(h, C.n * C.n);
  if (!dense) return AMG_ERR_NOMEM;
  QA_HIP(hipMemsetAsync(dense, 0, sizeof(double) * C.n * C.n, s));
  if (h->dim == 3)
    k_densify_level3<<<nblk(C.n), kBlock, 0, s>>>(C.k, C.n, C.ax64, C.ovf_nnz ? C.optr : nullptr, C.ocol,
                                                   C.oval64, dense);
  else
    k_densify_level<<<nblk(C.n), kBlock, 0, s>>>(C.k, C.n, C.ax64, C.ovf_nnz ? C.optr : nullptr, C.ocol, C.oval64,
                                                 dense);
  QA_LAUNCH_CHECK();
  return build_coarsest_inverse(h, dense, C.n);
}

static amg_status build_block_factors(amg_hierarchy *h) {
  FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  const int64_t nL = static_cast<int64_t>(1) << (h->dim * h->L);
  int64_t *size = dalloc_n<int64_t>(h, nL);
  F.boff = dalloc_n<int64_t>(h, nL + 1);
  if (!size || !F.boff) return AMG_ERR_NOMEM;
  k_block_size<<<nblk(nL), kBlock, 0, s>>>(nL, F.crow, size);
  QA_LAUNCH_CHECK();
  QA_TRY(scan_exclusive_i64(size, F.boff, nL, s, h));
  int64_t total = 0;
  {
    ReadBatch rb(h);
    QA_TRY(rb.add(&total, F.boff + nL, sizeof(int64_t)));
    QA_TRY(rb.finish());
  }
  F.bfac_n = total;
  F.bfac64 = dalloc_n<double>(h, std::max<int64_t>(total, 1));
  F.bfac32 = dalloc_n<float>(h, std::max<int64_t>(total, 1));
  if (!F.bfac64 || !F.bfac32) return AMG_ERR_NOMEM;
  return block_values(h);
}

// first cell-data entry of each window: its first cell's factor offset (exact blocks) or its first row's in-cell
// coupling offset (substitution)
__global__ void __launch_bounds__(kBlock) k_win_entries(int64_t nwin, const int32_t *__restrict__ win_q,
                                                         const int32_t *__restrict__ win_row,
                                                         const int64_t *__restrict__ boff,
                                                         const int32_t *__restrict__ icp,
                                                         int64_t *__restrict__ win_ent) {
  const int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w > nwin) return;
  win_ent[w] = boff ? boff[win_q[w]] : static_cast<int64_t>(icp[win_row[w]]);
}

// the largest cell-data count of a window the fused phase stages (at most kFuseStageRows rows and kWinCells cells)
__global__ void __launch_bounds__(kBlock) k_win_entmax(int64_t nwin, const int32_t *__restrict__ win_q,
                                                        const int32_t *__restrict__ win_row,
                                                        const int64_t *__restrict__ win_ent, int *__restrict__ out) {
  const int64_t w = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (w >= nwin) return;
  if (win_row[w + 1] - win_row[w] <= kFuseStageRows && win_q[w + 1] - win_q[w] <= kWinCells)
    atomicMax(out, static_cast<int>(win_ent[w + 1] - win_ent[w]));
}

static amg_status build_window_entries(amg_hierarchy *h) {
  FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  F.win_ent = dalloc_n<int64_t>(h, F.nwin + 1);
  if (!F.win_ent) return AMG_ERR_NOMEM;
  k_win_entries<<<nblk(F.nwin + 1), kBlock, 0, s>>>(F.nwin, F.win_q, F.win_row, h->opt.smoother ? F.boff : nullptr,
                                                     F.ic_ptr, F.win_ent);
  // the maximum goes to the device flags' slot 2, read back with them at the end of setup
  if (F.nwin) k_win_entmax<<<nblk(F.nwin), kBlock, 0, s>>>(F.nwin, F.win_q, F.win_row, F.win_ent, h->dflag + 2);
  QA_LAUNCH_CHECK();
  return AMG_OK;
}

static amg_status build_big_cells(amg_hierarchy *h) {
  FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  const int64_t n = h->n;
  // cells the smoother's per-cell kernels leave to the level-scheduled substitution
  QA_TRY(cell_list(h, h->opt.smoother ? kBlockMax : kBigCell, &F.big_cells, &F.nbig, F.big_color));
  if (F.nbig == 0) return AMG_OK;
  int32_t *lv = dalloc_n<int32_t>(h, n);
  int32_t *cnt = dalloc_n<int32_t>(h, F.nbig);
  if (!lv || !cnt) return AMG_ERR_NOMEM;
  // the largest big cell goes to the device flags' slot 3, read back with them at the end of setup
  k_big_rows_max<<<nblk(F.nbig), kBlock, 0, s>>>(F.nbig, F.big_cells, F.crow, h->dflag + 3);
  QA_LAUNCH_CHECK();
  for (int dir = 0; dir < 2; dir++) {
    if (dir == 0)
      k_big_levels<true><<<nblk(F.nbig), kBlock, 0, s>>>(F.nbig, F.big_cells, F.crow, F.ic_ptr, F.ic_col, lv, cnt);
    else
      k_big_levels<false><<<nblk(F.nbig), kBlock, 0, s>>>(F.nbig, F.big_cells, F.crow, F.ic_ptr, F.ic_col, lv, cnt);
    F.big_lofs[dir] = dalloc_n<int32_t>(h, F.nbig + 1);
    if (!F.big_lofs[dir]) return AMG_ERR_NOMEM;
    QA_TRY(scan_exclusive_i32(cnt, F.big_lofs[dir], F.nbig, s, h));
    int32_t total = 0;
    {
      ReadBatch rb(h);
      QA_TRY(rb.add(&total, F.big_lofs[dir] + F.nbig, sizeof(int32_t)));
      QA_TRY(rb.finish());
    }
    F.big_lptr[dir] = dalloc_n<int32_t>(h, total);
    F.big_sched[dir] = dalloc_n<int32_t>(h, n);
    if (!F.big_lptr[dir] || !F.big_sched[dir]) return AMG_ERR_NOMEM;
    k_big_sched<<<nblk(F.nbig), kBlock, 0, s>>>(F.nbig, F.big_cells, F.crow, lv, F.big_lofs[dir], F.big_lptr[dir],
                                                F.big_sched[dir]);
    QA_LAUNCH_CHECK();
  }
  return AMG_OK;
}

static amg_status build_multi_level(amg_hierarchy *h, const double *coords, const int64_t *row_ptr,
                                    const int32_t *col_idx, const double *vals, int64_t nnz) {
  FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  const int64_t n = h->n;
  const int L = h->L;
  const int64_t nL = static_cast<int64_t>(1) << (h->dim * L);
  // level-L cells and the stable counting sort
  int32_t *key = dalloc_n<int32_t>(h, n);
  int32_t *cnt = dalloc_n<int32_t>(h, nL);
  int32_t *fill = dalloc_n<int32_t>(h, nL);
  F.crow = dalloc_n<int32_t>(h, nL + 1);
  F.perm = dalloc_n<int32_t>(h, n);
  F.iperm = dalloc_n<int32_t>(h, n);
  F.agg_q = dalloc_n<int32_t>(h, n);
  int64_t *len = dalloc_n<int64_t>(h, n);
  F.rp = dalloc_n<int64_t>(h, n + 1);
  F.ci = dalloc_n<int32_t>(h, nnz);
  F.va = dalloc_n<double>(h, nnz);
  F.diag64 = dalloc_n<double>(h, n);
  F.diag32 = dalloc_n<float>(h, n);
  if (!key || !cnt || !fill || !F.crow || !F.perm || !F.iperm || !F.agg_q || !len || !F.rp || !F.ci || !F.va ||
      !F.diag64 || !F.diag32)
    return AMG_ERR_NOMEM;
  QA_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * nL, s));
  QA_HIP(hipMemsetAsync(fill, 0, sizeof(int32_t) * nL, s));
  if (h->dim == 3)
    k_cell_key3<<<nblk(n), kBlock, 0, s>>>(n, coords, Box3{{h->box[0], h->box[1], h->box[2], h->box[3], h->box[4],
                                                             h->box[5]}}, L, key, cnt);
  else
    k_cell_key<<<nblk(n), kBlock, 0, s>>>(n, coords, h->box[0], h->box[1], h->box[2], h->box[3], L, key, cnt);
  QA_LAUNCH_CHECK();
  QA_TRY(scan_exclusive_i32(cnt, F.crow, nL, s, h));
  k_scatter<<<nblk(n), kBlock, 0, s>>>(n, key, F.crow, fill, F.perm);
  QA_LAUNCH_CHECK();
  k_sort_cells<<<nblk(nL), kBlock, 0, s>>>(nL, F.crow, F.perm);
  QA_LAUNCH_CHECK();
  {
    int32_t *large = nullptr;
    int64_t nlarge = 0, first[kMaxColors + 1];
    QA_TRY(cell_list(h, kSortCell, &large, &nlarge, first));
    if (nlarge > 0) {
      int32_t *sorted = dalloc_n<int32_t>(h, n);
      if (!sorted) return AMG_ERR_NOMEM;
      QA_HIP(hipMemcpyAsync(sorted, F.perm, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
      k_rank_sort_cells<<<static_cast<unsigned>(nlarge), kBlock, 0, s>>>(large, F.crow, F.perm, sorted);
      QA_LAUNCH_CHECK();
      F.perm = sorted;
    }
  }
  k_inverse_perm<<<nblk(n), kBlock, 0, s>>>(n, F.perm, key, F.iperm, F.agg_q, row_ptr, len);
  QA_LAUNCH_CHECK();
  QA_TRY(scan_exclusive_i64(len, F.rp, n, s, h));
  k_permute_csr<<<nblk(8 * n), kBlock, 0, s>>>(n, F.perm, F.iperm, row_ptr, col_idx, vals, F.rp, F.ci, F.va,
                                               F.diag64);
  k_row_diag<<<nblk(n), kBlock, 0, s>>>(n, F.rp, F.ci, F.va, F.diag64);
  QA_LAUNCH_CHECK();
  // color regions: cells of color c are the range [c nL/nc, (c+1) nL/nc) of the color-major order
  {
    const int nc = F.ncolor;
    int32_t cr[kMaxColors];
    ReadBatch rb(h);
    for (int c = 0; c < nc; c++) QA_TRY(rb.add(&cr[c], F.crow + c * (nL / nc), sizeof(int32_t)));
    QA_TRY(rb.finish());
    for (int c = 0; c < nc; c++) F.color_row[c] = cr[c];
    F.color_row[nc] = n;
  }
  QA_TRY(build_sell(h));
  // in-cell couplings
  F.ic_ptr = dalloc_n<int32_t>(h, n + 1);
  int32_t *iccnt = dalloc_n<int32_t>(h, n);
  if (!F.ic_ptr || !iccnt) return AMG_ERR_NOMEM;
  k_ic_count<<<nblk(n), kBlock, 0, s>>>(n, F.rp, F.ci, F.agg_q, iccnt);
  QA_LAUNCH_CHECK();
  QA_TRY(scan_exclusive_i32(iccnt, F.ic_ptr, n, s, h));
  {
    int32_t icn = 0;
    ReadBatch rb(h);
    QA_TRY(rb.add(&icn, F.ic_ptr + n, sizeof(int32_t)));
    QA_TRY(rb.finish());
    F.ic_nnz = icn;
  }
  F.ic_col = dalloc_n<int32_t>(h, F.ic_nnz);
  F.ic_val64 = dalloc_n<double>(h, F.ic_nnz);
  F.ic_val32 = dalloc_n<float>(h, F.ic_nnz);
  if (!F.ic_col || !F.ic_val64 || !F.ic_val32) return AMG_ERR_NOMEM;
  QA_TRY(ic_values(h));
  QA_TRY(build_big_cells(h));
  if (h->opt.smoother) QA_TRY(build_block_factors(h));
  QA_TRY(build_window_entries(h));

  // Galerkin operators, level L first, then coarser
  h->lev.assign(h->nlev, QuadLevel{});
  for (int l = 1; l < h->nlev; l++) QA_TRY(level_values(h, l, true));
  return coarsest_values(h);
}

static amg_status setup_impl(amg_hierarchy *h, const double *coords, const int64_t *row_ptr, const int32_t *col_idx,
                             const double *vals, int64_t nnz) {
  hipStream_t s = h->stream;
  const int64_t n = h->n;
  h->dflag = dalloc_n<int>(h, 4);
  if (!h->dflag) return AMG_ERR_NOMEM;
  QA_HIP(hipMemsetAsync(h->dflag, 0, 4 * sizeof(int), s));
  const double *ub = h->opt.box;
  const int nbox = 2 * h->dim;
  if (h->dim == 3) {
    Box3 B{};
    for (int t = 0; t < 6 && ub; t++) B.v[t] = ub[t];
    k_validate3<<<nblk(n), kBlock, 0, s>>>(n, nnz, coords, row_ptr, col_idx, vals, ub ? 1 : 0, B, h->dflag);
  } else {
    k_validate<<<nblk(n), kBlock, 0, s>>>(n, nnz, coords, row_ptr, col_idx, vals, ub ? 1 : 0, ub ? ub[0] : 0.0,
                                           ub ? ub[1] : 0.0, ub ? ub[2] : 0.0, ub ? ub[3] : 0.0, h->dflag);
  }
  QA_LAUNCH_CHECK();
  // the validation flag and the bounding box (eq. 6) come back in one read: the box kernels only read coords[0, n)
  int f = 0;
  ReadBatch rb(h);
  QA_TRY(rb.add(&f, h->dflag, sizeof(int)));
  if (ub) {
    for (int t = 0; t < nbox; t++) h->box[t] = ub[t];
  } else if (h->dim == 3) {
    const int nb = static_cast<int>(std::min<int64_t>(nblk(n), kRedBlocksMax));
    double *part = dalloc_n<double>(h, 6 * nb + 6);
    if (!part) return AMG_ERR_NOMEM;
    k_bbox3_partial<<<nb, kBlock, 0, s>>>(n, coords, part);
    QA_LAUNCH_CHECK();
    k_bbox3_final<<<1, 1, 0, s>>>(nb, part, part + 6 * nb);
    QA_LAUNCH_CHECK();
    QA_TRY(rb.add(h->box, part + 6 * nb, 6 * sizeof(double)));
  } else {
    const int nb = static_cast<int>(std::min<int64_t>(nblk(n), kRedBlocksMax));
    double *part = dalloc_n<double>(h, 4 * nb + 4);
    if (!part) return AMG_ERR_NOMEM;
    k_bbox_partial<<<nb, kBlock, 0, s>>>(n, coords, part);
    QA_LAUNCH_CHECK();
    k_bbox_final<<<1, 1, 0, s>>>(nb, part, part + 4 * nb);
    QA_LAUNCH_CHECK();
    QA_TRY(rb.add(h->box, part + 4 * nb, 4 * sizeof(double)));
  }
  QA_TRY(rb.finish());
  if (f & F_INVALID) return AMG_ERR_INVALID;
  if (f & F_NOT_SPD) return AMG_ERR_NOT_SPD;
  h->nlev = depth_rule(n, h->opt.coarse_max, h->L, h->kc, h->dim);
  h->fine.n = n;
  h->fine.ncolor = 1 << h->dim;
  h->fine.nnz = nnz;
  if (h->nlev == 1) {
    QA_TRY(build_single_level(h, row_ptr, col_idx, vals, nnz));
    h->lev.assign(1, QuadLevel{});
  } else {
    QA_TRY(build_multi_level(h, coords, row_ptr, col_idx, vals, nnz));
  }
  {
    int fl[4] = {0, 0, 0, 0};  // error flags; [2], [3]: the largest staged window's cell data, the largest big cell
    QA_TRY(rb.add(fl, h->dflag, sizeof(fl)));
    QA_TRY(rb.finish());
    f = fl[0];
    h->fine.win_ent_max = fl[2];
    h->fine.big_max_rows = fl[3];
  }
  if (f & F_NOT_SPD) return AMG_ERR_NOT_SPD;
  QA_TRY(alloc_workspaces(h));
  QA_TRY(build_mhat(h));
  QA_TRY(plan_engine(h));
  QA_TRY(plan_wg(h));
  QA_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

// New values on the stored pattern: the numeric half of setup_impl (permuted CSR, sliced ELL, in-cell couplings,
// cell factors, Galerkin operators, coarsest inverse, B^ matrix), into the hierarchy's own arrays, with the same
// kernels and hence the same results as a setup from scratch. The aggregation, orderings, layouts and plans depend on
// the pattern only and are kept. Temporaries are returned before the call ends.
static amg_status update_impl(amg_hierarchy *h, const int64_t *row_ptr, const int32_t *col_idx, const double *vals) {
  FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  const int64_t n = h->n;
  QA_HIP(hipMemsetAsync(h->dflag, 0, 4 * sizeof(int), s));
  k_same_pattern<<<nblk(n), kBlock, 0, s>>>(n, F.nnz, row_ptr, col_idx, vals, F.iperm, F.rp, F.ci, h->dflag);
  QA_LAUNCH_CHECK();
  int f = 0;
  QA_TRY(read_flag(h, f));
  if (f & F_INVALID) return AMG_ERR_INVALID;
  if (f & F_NOT_SPD) return AMG_ERR_NOT_SPD;
  h->stale = 1;  // from here on the stored values change
  k_permute_csr<<<nblk(8 * n), kBlock, 0, s>>>(n, F.perm, F.iperm, row_ptr, col_idx, vals, F.rp, F.ci, F.va,
                                               F.diag64);
  k_row_diag<<<nblk(n), kBlock, 0, s>>>(n, F.rp, F.ci, F.va, F.diag64);
  QA_LAUNCH_CHECK();
  QA_TRY(sell_values(h));
  if (h->nlev == 1) {
    double *dense = dalloc_n<double>(h, n * n);
    if (!dense) return AMG_ERR_NOMEM;
    QA_HIP(hipMemsetAsync(dense, 0, sizeof(double) * n * n, s));
    k_densify_csr<<<nblk(n), kBlock, 0, s>>>(n, row_ptr, col_idx, vals, dense);
    QA_LAUNCH_CHECK();
    QA_TRY(build_coarsest_inverse(h, dense, n));
  } else {
    QA_TRY(ic_values(h));
    if (h->opt.smoother) QA_TRY(block_values(h));
    for (int l = 1; l < h->nlev; l++) QA_TRY(level_values(h, l, false));
    QA_TRY(coarsest_values(h));
  }
  QA_TRY(read_flag(h, f));
  if (f & F_NOT_SPD) return AMG_ERR_NOT_SPD;
  QA_TRY(build_mhat(h));
  QA_HIP(hipStreamSynchronize(s));
  h->stale = 0;
  return AMG_OK;
}

}  // namespace qa

using namespace qa;

// shared-chunk size for a hierarchy of about `estimate` bytes: an eighth of it, 4 MB to 256 MB, whole megabytes
static size_t chunk_unit_for(size_t estimate) {
  const size_t mb = static_cast<size_t>(1) << 20;
  const size_t u = std::min(std::max(estimate / 8, 4 * mb), 256 * mb);
  return (u + mb - 1) / mb * mb;
}

extern "C" amg_status amg_estimate_bytes(int64_t n, int64_t nnz, const amg_options *opt, size_t *bytes) {
  if (n < 1 || nnz < 0 || !bytes) return AMG_ERR_INVALID;
  amg_options o;
  amg_default_options(&o);
  if (opt) o = *opt;
  int L = -1, kc = -1;
  const int nlev = depth_rule(n, o.coarse_max, L, kc);
  double b = 0;
  // fine: permuted CSR (12 B/nnz + 8 B/row), sliced ELL (padding allowance 1.35) in FP64 + FP32 + columns,
  // in-cell lists (<= nnz), vectors (4 FP64 + 4 FP32 workspace, 9 FP64 outer), indices
  b += 12.0 * nnz + 8.0 * (n + 1);
  b += 1.35 * (nnz + n) * (8 + 4 + 4);
  b += 16.0 * nnz;
  b += n * (4 * 8 + 4 * 4 + 9 * 8 + 4 * 4 + 8);
  if (nlev > 1) {
    const double nL = std::ldexp(1.0, 2 * L);
    // quadtree levels: 9 FP64 + 9 FP32 + flags + 8 vectors per precision; geometric sum 4/3
    b += (4.0 / 3.0) * nL * (9 * 12 + 1 + 4 + 8 * 12 + 4);
    b += nL * 4.0 * 3;  // counting-sort temporaries and cell row pointers
    const double nc = std::ldexp(1.0, 2 * kc);
    b += 3 * nc * nc * 8;
  } else {
    b += 4.0 * n * n * 8;
  }
  // exact-block smoother: a packed factor of m (m + 1) / 2 FP64 + FP32 values per cell of m <= kBlockMax unknowns
  // (at most (kBlockMax + 1) / 2 values per unknown) and the cell offsets
  if (o.smoother == 1 && nlev > 1) b += static_cast<double>(n) * (kBlockMax + 1) * 6 + std::ldexp(1.0, 2 * L) * 16;
  b += 1 << 20;  // scalars, partial sums, alignment slack
  // arrays are carved from shared chunks of about b / 8 bytes (see chunk_unit_for): allow a chunk and a half unused
  b += 1.5 * static_cast<double>(chunk_unit_for(static_cast<size_t>(b)));
  *bytes = static_cast<size_t>(b);
  return AMG_OK;
}

// shared by the quadtree (dim 2) and octree (dim 3) entry points; box: 2 dim values or NULL
static amg_status setup_dim(int dim, int64_t n, const double *coords, const int64_t *row_ptr, const int32_t *col_idx,
                            const double *vals, int64_t nnz, const double *box, const amg_options *opt,
                            amg_hierarchy **out) {
  if (!out) return AMG_ERR_INVALID;
  *out = nullptr;
  amg_options o;
  amg_default_options(&o);
  if (opt) o = *opt;
  if (n < 1 || n > (static_cast<int64_t>(1) << 31) - 2 || nnz < 0 || !coords || !row_ptr || !col_idx || !vals)
    return AMG_ERR_INVALID;
  if ((o.precision != 0 && o.precision != 1) || o.coarse_max < 4 || o.coarse_max > 1024 || o.inner_iters < 1 ||
      o.inner_iters > 2 || o.sweeps < 1 || o.sweeps > 8 || (o.outer_mmax < -1 || o.outer_mmax > 1) ||
      o.max_iters < 1 || (o.smoother != 0 && o.smoother != 1) || o.engine < 0 || o.engine > 2 ||
      !o.alloc != !o.dealloc)
    return AMG_ERR_INVALID;
  if (box) {
    for (int t = 0; t < 2 * dim; t++)
      if (!std::isfinite(box[t])) return AMG_ERR_INVALID;
    for (int a = 0; a < dim; a++)
      if (box[2 * a + 1] < box[2 * a]) return AMG_ERR_INVALID;
  }
  const auto t0 = std::chrono::steady_clock::now();
  amg_hierarchy *h = new (std::nothrow) amg_hierarchy();
  if (!h) return AMG_ERR_NOMEM;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return AMG_ERR_DEVICE;
  }
  h->dim = dim;
  h->opt = o;
  h->opt.box = nullptr;  // borrowed pointer: do not keep
  h->stream = static_cast<hipStream_t>(o.stream);
  h->precision = o.precision;
  // the persistent small-level workgroups and the batched whole-solve route carry the quadtree's 9-point levels
  h->use_engine = dim == 2 ? o.engine : 0;
  h->use_batch = (dim == 2 && o.batch) ? 1 : 0;
  h->n = n;
  {
    size_t est = 0;
    amg_options eo = o;
    eo.box = nullptr;
    if (amg_estimate_bytes(n, nnz, &eo, &est) == AMG_OK)
      h->chunk_unit = chunk_unit_for(dim == 3 ? est + est / 2 : est);
  }
  h->opt.box = box;
  amg_status st = borrow_pinned_scalars(&h->host_scal);  // the readbacks of setup use it first
  if (st == AMG_OK) st = setup_impl(h, coords, row_ptr, col_idx, vals, nnz);
  h->opt.box = nullptr;
  if (st != AMG_OK) {
    (void)hipStreamSynchronize(h->stream);
    release(h);
    delete h;
    return st;
  }
  h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h;
  return AMG_OK;
}

extern "C" amg_status amg_setup(int64_t n, const double *coords, const int64_t *row_ptr, const int32_t *col_idx,
                                const double *vals, int64_t nnz, const amg_options *opt, amg_hierarchy **out) {
  return setup_dim(2, n, coords, row_ptr, col_idx, vals, nnz, opt ? opt->box : nullptr, opt, out);
}

extern "C" amg_status amg_setup3d(int64_t n, const double *coords, const int64_t *row_ptr, const int32_t *col_idx,
                                  const double *vals, int64_t nnz, const double *box, const amg_options *opt,
                                  amg_hierarchy **out) {
  if (opt && opt->box) return AMG_ERR_INVALID;  // the octree's box is the box argument
  return setup_dim(3, n, coords, row_ptr, col_idx, vals, nnz, box, opt, out);
}

extern "C" amg_status amg_update_values(amg_hierarchy *h, const int64_t *row_ptr, const int32_t *col_idx,
                                        const double *vals, int64_t nnz) {
  if (!h || !row_ptr || !col_idx || !vals || nnz != h->fine.nnz) return AMG_ERR_INVALID;
  QA_HIP(hipSetDevice(h->device));
  const auto t0 = std::chrono::steady_clock::now();
  const ArenaMark mark = arena_mark(h);
  const amg_status st = update_impl(h, row_ptr, col_idx, vals);
  arena_rollback(h, mark);
  if (st == AMG_OK)
    h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

// ---------------------------------------------------------------------------------------------------------------
// export in canonical numbering (host-side rearrangement of device arrays)

extern "C" amg_status amg_level_info(const amg_hierarchy *h, int32_t level, int64_t *n_rows, int32_t *k,
                                     int64_t *ovf_nnz, int32_t *depth_L) {
  if (!h || level < 0 || level >= h->nlev) return AMG_ERR_INVALID;
  if (depth_L) *depth_L = h->L;
  if (level == 0) {
    if (n_rows) *n_rows = h->n;
    if (k) *k = -1;
    if (ovf_nnz) *ovf_nnz = 0;
  } else {
    const QuadLevel &Q = h->lev[level];
    if (n_rows) *n_rows = Q.n;
    if (k) *k = Q.k;
    if (ovf_nnz) *ovf_nnz = Q.ovf_nnz;
  }
  return AMG_OK;
}

template <class T>
static amg_status to_host(std::vector<T> &v, const T *d, int64_t count, hipStream_t s) {
  v.resize(static_cast<size_t>(count > 0 ? count : 0));
  if (count > 0) QA_HIP(hipMemcpyAsync(v.data(), d, sizeof(T) * count, hipMemcpyDeviceToHost, s));
  return AMG_OK;
}

// lexicographic id (eq. 8: t1 + 2^k t2 [+ 4^k t3]) <-> color-major storage index on a level of dimension dim
static uint32_t host_q_of_lex(uint32_t lex, int k, int dim = 2) {
  const uint32_t mask = (1u << k) - 1u;
  if (dim == 3) return q_of_m3(morton3(lex & mask, (lex >> k) & mask, lex >> (2 * k)), k);
  return q_of_m(morton(lex & mask, lex >> k), k);
}
static uint32_t host_lex_of_q(uint32_t q, int k, int dim = 2) {
  if (dim == 3) {
    const uint32_t m = m_of_q3(q, k);
    return (((compact3(m >> 2) << k) | compact3(m >> 1)) << k) | compact3(m);
  }
  const uint32_t m = m_of_q(q, k);
  return (compact_bits(m >> 1) << k) | compact_bits(m);
}
// grid coordinates of lexicographic cell I of side `side`
static void host_coords(uint32_t I, uint32_t side, int dim, int t[3]) {
  t[0] = static_cast<int>(I % side);
  t[1] = static_cast<int>((I / side) % side);
  t[2] = dim == 3 ? static_cast<int>(I / side / side) : 0;
}
static int host_slot_d(int sl, int a, int dim) {
  if (dim == 3) return a == 0 ? slot3_dx(sl) : (a == 1 ? slot3_dy(sl) : slot3_dz(sl));
  return a == 0 ? slot_dx(sl) : (a == 1 ? slot_dy(sl) : 0);
}
// lexicographic neighbour of I in slot sl, or -1 outside the grid
static int32_t host_neighbour(uint32_t I, int sl, uint32_t side, int dim) {
  int t[3];
  host_coords(I, side, dim, t);
  int u[3];
  for (int a = 0; a < 3; a++) {
    u[a] = t[a] + host_slot_d(sl, a, dim);
    if (u[a] < 0 || (a < dim && u[a] >= static_cast<int>(side)) || (a >= dim && u[a] != 0)) return -1;
  }
  return static_cast<int32_t>((static_cast<uint32_t>(u[2]) * side + static_cast<uint32_t>(u[1])) * side +
                              static_cast<uint32_t>(u[0]));
}

template <class V>
static amg_status export_values(const amg_hierarchy *h, int32_t level, const V *dev_ax, V *ax) {
  const QuadLevel &Q = h->lev[level];
  const int ns = Q.ns, dim = h->dim;
  std::vector<V> hax;
  QA_TRY(to_host(hax, dev_ax, ns * Q.n, h->stream));
  QA_HIP(hipStreamSynchronize(h->stream));
  const uint32_t side = 1u << Q.k;
  for (uint32_t I = 0; I < static_cast<uint32_t>(Q.n); I++) {
    const uint32_t q = host_q_of_lex(I, Q.k, dim);
    for (int sl = 0; sl < ns; sl++)
      ax[static_cast<size_t>(I) * ns + sl] =
          host_neighbour(I, sl, side, dim) >= 0 ? hax[static_cast<size_t>(sl) * Q.n + q] : V(0);
  }
  return AMG_OK;
}

extern "C" amg_status amg_export_level(const amg_hierarchy *h, int32_t level, int32_t *agg, uint8_t *color,
                                       int32_t *aj, double *ax, int64_t *ovf_ptr, int32_t *ovf_col,
                                       double *ovf_val) {
  if (!h || level < 0 || level >= h->nlev) return AMG_ERR_INVALID;
  QA_HIP(hipSetDevice(h->device));
  hipStream_t s = h->stream;
  if (level == 0) {
    if (h->nlev == 1) {
      for (int64_t i = 0; i < h->n; i++) {
        if (agg) agg[i] = -1;
        if (color) color[i] = 0;
      }
      return AMG_OK;
    }
    std::vector<int32_t> iperm, aggq;
    QA_TRY(to_host(iperm, h->fine.iperm, h->n, s));
    QA_TRY(to_host(aggq, h->fine.agg_q, h->n, s));
    QA_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < h->n; i++) {
      const uint32_t q = static_cast<uint32_t>(aggq[iperm[i]]);
      if (agg) agg[i] = static_cast<int32_t>(host_lex_of_q(q, h->L, h->dim));
      if (color) color[i] = static_cast<uint8_t>(h->dim == 3 ? (m_of_q3(q, h->L) & 7u) : (m_of_q(q, h->L) & 3u));
    }
    return AMG_OK;
  }
  const QuadLevel &Q = h->lev[level];
  const int dim = h->dim, ns = Q.ns;
  const uint32_t side = 1u << Q.k, half = side >> 1;
  for (uint32_t I = 0; I < static_cast<uint32_t>(Q.n); I++) {
    int t[3];
    host_coords(I, side, dim, t);
    if (agg) {  // eq. (10): the parent (t1 >> 1, t2 >> 1[, t3 >> 1])
      const uint32_t p1 = static_cast<uint32_t>(t[0]) >> 1, p2 = static_cast<uint32_t>(t[1]) >> 1,
                     p3 = static_cast<uint32_t>(t[2]) >> 1;
      agg[I] = (level < h->nlev - 1) ? static_cast<int32_t>((p3 * half + p2) * half + p1) : -1;
    }
    if (color) color[I] = static_cast<uint8_t>((t[0] & 1) + 2 * (t[1] & 1) + 4 * (t[2] & 1));
    if (aj)
      for (int sl = 0; sl < ns; sl++) aj[static_cast<size_t>(I) * ns + sl] = host_neighbour(I, sl, side, dim);
  }
  if (ax) QA_TRY(export_values<double>(h, level, Q.ax64, ax));
  if (ovf_ptr || ovf_col || ovf_val) {
    std::vector<int32_t> optr, ocol;
    std::vector<double> oval;
    QA_TRY(to_host(optr, Q.optr, Q.n + 1, s));
    QA_TRY(to_host(ocol, Q.ocol, Q.ovf_nnz, s));
    QA_TRY(to_host(oval, Q.oval64, Q.ovf_nnz, s));
    QA_HIP(hipStreamSynchronize(s));
    int64_t o = 0;
    if (ovf_ptr) ovf_ptr[0] = 0;
    for (uint32_t I = 0; I < static_cast<uint32_t>(Q.n); I++) {
      const uint32_t q = host_q_of_lex(I, Q.k, dim);
      for (int32_t e = optr[q]; e < optr[q + 1]; e++, o++) {
        if (ovf_col) ovf_col[o] = static_cast<int32_t>(host_lex_of_q(static_cast<uint32_t>(ocol[e]), Q.k, dim));
        if (ovf_val) ovf_val[o] = oval[e];
      }
      if (ovf_ptr) ovf_ptr[I + 1] = o;
    }
  }
  return AMG_OK;
}

extern "C" amg_status amg_export_level_f32(const amg_hierarchy *h, int32_t level, float *ax) {
  if (!h || level < 1 || level >= h->nlev || !ax) return AMG_ERR_INVALID;
  QA_HIP(hipSetDevice(h->device));
  return export_values<float>(h, level, h->lev[level].ax32, ax);
}
