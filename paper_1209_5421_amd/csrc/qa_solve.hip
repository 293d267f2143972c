// Solve phase on gfx950: the nonlinear AMLI-cycle (Algorithm 2.2) with the nonlinear PCG of Algorithm 2.1 as its
// coarse-level accelerator, used as the preconditioner of an outer flexible CG at the fine level.
//
// Kernels are templated on the storage/arithmetic type T (double for the plain solve, float for the
// preconditioner of the mixed form); every inner product accumulates in double with a fixed reduction tree
// (wavefront shuffles, then the four waves of a workgroup, then the workgroup partials summed in order by the last
// workgroup to finish), so results depend only on the system size, never on scheduling.
//
// Fine level: sliced ELL (64-row slices = one wavefront, column-major, so every load of a slice row step is one
// coalesced 256/512-byte access). The colored block Gauss-Seidel phase (Section 4.5) is split in two kernels: the
// residual of the color's rows (sliced-ELL pass), then one thread per cell doing the forward/backward
// substitution over the cell's unknowns with the in-cell couplings. The kernel boundary between the two is what
// makes every residual of a color see the iterate at phase start.
//
// Quadtree levels: values only (9 per row, slot-major so each slot is a coalesced stream), neighbour indices
// recomputed from the color-major Morton index; overflow couplings from a small CSR.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>
#include <type_traits>

#include <hip/hip_ext.h>

#include "qa_internal.hpp"

namespace qa {

// ---------------------------------------------------------------------------------------------------------------
// scalar slots (per level, kScalars doubles; the outer iteration uses slot block nlev)

enum {
  S_D0 = 0, S_S0 = 1, S_A0 = 2, S_STOP = 3, S_T = 4, S_BETA = 5, S_D1 = 6, S_S1 = 7, S_A1 = 8,
  O_D = 0, O_S = 1, O_ALPHA = 2, O_BREAK = 3, O_ZQ = 4, O_BETA = 5, O_RR = 6, O_TT = 7, O_BB = 8
};
enum Epi { EPI_ALPHA0, EPI_BETA, EPI_ALPHA1, EPI_OUT_ALPHA, EPI_OUT_BETA, EPI_STORE };

struct Red {
  double *partials;
  double *sc;
  int epi;
  int slot;
};

// sum over the workgroup (fixed order); valid in thread 0
template <int ND>
__device__ inline void block_sum(double (&v)[ND]) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int j = 0; j < ND; j++) v[j] += __shfl_down(v[j], off, 64);
  __shared__ double s[ND][kBlock / 64];
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int j = 0; j < ND; j++) s[j][threadIdx.x >> 6] = v[j];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < ND; j++) v[j] = (s[j][0] + s[j][1]) + (s[j][2] + s[j][3]);
}

__device__ inline void epilogue(const double *acc, const Red &R) {
  double *sc = R.sc;
  switch (R.epi) {
    case EPI_ALPHA0: {
      const double d = acc[0], s = acc[1];
      const bool stop = !(d > 0.0);
      sc[S_D0] = d; sc[S_S0] = s; sc[S_STOP] = stop ? 1.0 : 0.0; sc[S_A0] = stop ? 0.0 : s / d;
      break;
    }
    case EPI_BETA:
      sc[S_T] = acc[0];
      sc[S_BETA] = (sc[S_STOP] != 0.0) ? 0.0 : -acc[0] / sc[S_D0];
      break;
    case EPI_ALPHA1: {
      const double d = acc[0], s = acc[1];
      sc[S_D1] = d; sc[S_S1] = s;
      sc[S_A1] = (sc[S_STOP] != 0.0 || !(d > 0.0)) ? 0.0 : s / d;
      break;
    }
    case EPI_OUT_ALPHA: {
      const double d = acc[0], s = acc[1];
      const bool ok = d > 0.0;
      sc[O_D] = d; sc[O_S] = s; sc[O_ALPHA] = ok ? s / d : 0.0; sc[O_BREAK] = ok ? 0.0 : 1.0;
      break;
    }
    case EPI_OUT_BETA:
      sc[O_ZQ] = acc[0];
      sc[O_BETA] = -acc[0] / sc[O_D];
      break;
    default:
      sc[R.slot] = acc[0];
  }
}

// Every thread of every workgroup must call this (no early returns in reduction kernels). A single-workgroup
// launch applies the epilogue directly; otherwise each workgroup stores its partial sums and a one-workgroup
// k_finish launched right after sums them in workgroup order. The kernel boundary orders the two, so no
// device-scope fence is needed (on this multi-XCD part such a fence writes back the L2 of every workgroup).
template <int ND>
__device__ inline void reduce_finish(double (&v)[ND], const Red &R) {
  block_sum<ND>(v);
  if (threadIdx.x == 0) {
    if (gridDim.x == 1) {
      epilogue(v, R);
    } else {
#pragma unroll
      for (int j = 0; j < ND; j++) R.partials[static_cast<size_t>(blockIdx.x) * ND + j] = v[j];
    }
  }
}

template <int ND>
__global__ void __launch_bounds__(kBlock) k_finish(unsigned nb, Red R) {
  double acc[ND];
#pragma unroll
  for (int j = 0; j < ND; j++) acc[j] = 0.0;
  for (unsigned b = threadIdx.x; b < nb; b += kBlock)
#pragma unroll
    for (int j = 0; j < ND; j++) acc[j] += R.partials[static_cast<size_t>(b) * ND + j];
  block_sum<ND>(acc);
  if (threadIdx.x == 0) epilogue(acc, R);
}

// r = g - a0 q0 of the first inner update of Algorithm 2.1 (one expression, so the separate and the folded forms
// round alike)
template <class T>
__device__ __forceinline__ T upd1_r(T g, T a0, T q0) {
  return g - a0 * q0;
}

// the first inner update e = a0 p0, r = g - a0 q0 left for the first relaxation of the second B^ (null sc: none):
// that kernel writes e and r and reads its right-hand side r formed on the fly
template <class T>
struct Upd1 {
  const double *sc;
  const T *g, *q0, *p0;
  T *e, *r;
  __device__ T a0() const { return static_cast<T>(sc[S_A0]); }
  __device__ T rv(T a, uint32_t i) const { return upd1_r(g[i], a, q0[i]); }
  __device__ void store(T a, int64_t i) const {
    e[i] = a * p0[i];
    r[i] = upd1_r(g[i], a, q0[i]);
  }
};

// the child's pending last update e_c + a1 (p1 + beta p0) of Algorithm 2.1, formed where the prolongation reads e_c
// (null sc: nothing pending)
template <class T>
struct Pending {
  const double *sc;
  const T *p1, *p0;
  __device__ T mix(T em, T p1m, T p0m) const {
    const T a1 = static_cast<T>(sc[S_A1]), beta = static_cast<T>(sc[S_BETA]);
    return em + a1 * (p1m + beta * p0m);
  }
  __device__ T apply(const T *e, uint32_t m) const {
    if (!sc) return e[m];
    return mix(e[m], p1[m], p0[m]);
  }
};

// ---------------------------------------------------------------------------------------------------------------
// fine level kernels

template <class T>
struct SellView {
  const int64_t *ptr;
  const int32_t *row0;    // first position of each slice
  const int32_t *srow;    // position -> row
  const int32_t *col;
  const T *val;
};

// (A x)_row for the row of `lane` in a slice of width w starting at entry `off`: the loop is unrolled by four with the
// column and value loads of a group issued before its gathers, so each wavefront keeps several gathers in flight
// sum over a slice row's entries of value x gathered entry, in entry order. Entries go in batches of kSellBatch:
// a batch's columns and values are loaded together, then its gathers, then its products are added one by one, so a
// row waits on two memory round trips per batch. The last batch's loads past the row's width are clamped to its last
// entry and their products skipped, so the sum is the plain loop's bit for bit. get(c) returns the gathered entry.
constexpr int kSellBatch = 8;
template <class T, class XT, class Get>
__device__ __forceinline__ XT sell_row_batched(const SellView<T> &S, int64_t off, int w, int lane, Get get) {
  const T *vp = S.val + off + lane;
  const int32_t *cp = S.col + off + lane;
  XT acc = 0;
  for (int k = 0; k < w; k += kSellBatch) {
    int32_t c[kSellBatch];
    T v[kSellBatch];
    XT xv[kSellBatch];
#pragma unroll
    for (int u = 0; u < kSellBatch; u++) {
      const int e = min(k + u, w - 1) * 64;
      c[u] = cp[e];
      v[u] = vp[e];
    }
#pragma unroll
    for (int u = 0; u < kSellBatch; u++) xv[u] = get(c[u]);
#pragma unroll
    for (int u = 0; u < kSellBatch; u++)
      if (k + u < w) acc += v[u] * xv[u];
  }
  return acc;
}

template <class T, class XT>
__device__ inline XT sell_row(const SellView<T> &S, int64_t off, int w, int lane, const XT *__restrict__ x) {
  return sell_row_batched<T, XT>(S, off, w, lane, [&](int32_t c) -> XT { return x[c]; });
}

// sell_row with the entries of columns in [lo, hi) taken from alt (from zero when alt is null) instead of x: the
// same products in the same order, so with alt holding what x held there the result is the same bit for bit
template <class T>
__device__ inline T sell_row_split(const SellView<T> &S, int64_t off, int w, int lane, const T *__restrict__ x,
                                   const T *__restrict__ alt, int32_t lo, int32_t hi) {
  return sell_row_batched<T, T>(S, off, w, lane, [&](int32_t c) -> T {
    return (c >= lo && c < hi) ? (alt ? alt[c] : T(0)) : x[c];
  });
}

// Which slices a launch over the colors [c0, c1) gives to which workgroup. Workgroups are dispatched to the eight
// XCDs round-robin (workgroup b runs on XCD b mod 8) and every XCD has an L2 of its own. In the XCD-aware order,
// workgroup b takes its slices from chunk b mod 8 of every color in [c0, c1), the same eighth of the Morton range in
// each color. A row's couplings reach the other colors at nearby Morton positions, so each XCD gathers mostly its
// own eighth of x instead of all of it. Small passes keep the plain order (one grid-ordered run of slices, which also
// keeps single-workgroup reductions in one launch).
struct SliceSched {
  int64_t cs[kMaxColors + 1];  // first slice of each color; cs[ncolor] = number of slices
  int c0, c1;
  int xcd;        // 1: XCD-aware order (grid = 8 x the largest per-XCD share), 0: slices in grid order
  int ilv;        // XCD-aware order only: > 0, the colors' shares taken in turns of ilv slices; 0, color by color
};

// slice of this thread's wavefront (4 per workgroup), or -1
__device__ inline int64_t sched_slice(const SliceSched &S) {
  const int w = static_cast<int>(threadIdx.x >> 6);
  if (!S.xcd) {
    const int64_t s = S.cs[S.c0] + static_cast<int64_t>(blockIdx.x) * (kBlock / 64) + w;
    return s < S.cs[S.c1] ? s : -1;
  }
  const int64_t x = blockIdx.x & 7u;
  int64_t p = static_cast<int64_t>(blockIdx.x >> 3) * (kBlock / 64) + w;
  int64_t skip = 0;  // slices of each color's share already taken in turns
  if (S.ilv > 0) {
    // turns: ilv slices of every color's share at the same position, while every share has ilv slices left, so
    // the rows gathering one stretch of x from all colors run close together in time on the XCD
    int64_t shortest = INT64_MAX;
    for (int c = S.c0; c < S.c1; c++) {
      const int64_t len = S.cs[c + 1] - S.cs[c];
      const int64_t share = len * (x + 1) / 8 - len * x / 8;
      shortest = share < shortest ? share : shortest;
    }
    const int64_t nc = S.c1 - S.c0, turns = shortest / S.ilv, in_turns = turns * nc * S.ilv;
    if (p < in_turns) {
      const int64_t t = p / (nc * S.ilv), q = p % (nc * S.ilv);
      const int c = S.c0 + static_cast<int>(q / S.ilv);
      const int64_t len = S.cs[c + 1] - S.cs[c];
      return S.cs[c] + len * x / 8 + t * S.ilv + q % S.ilv;
    }
    p -= in_turns;
    skip = turns * S.ilv;
  }
  for (int c = S.c0; c < S.c1; c++) {  // the rest color by color
    const int64_t len = S.cs[c + 1] - S.cs[c];
    const int64_t b0 = len * x / 8 + skip, b1 = len * (x + 1) / 8;
    if (p < b1 - b0) return S.cs[c] + b0 + p;
    p -= b1 - b0;
  }
  return -1;
}

// d[p] = f[p] - (A x)[p] for the rows of the scheduled slices; one wavefront per slice
template <class T>
__device__ inline void fine_resid_body(const SellView<T> &S, const SliceSched &Z, const T *__restrict__ f,
                                       const T *__restrict__ x, T *__restrict__ d) {
  const int64_t s = sched_slice(Z);
  if (s < 0) return;
  const int lane = threadIdx.x & 63;
  const int32_t r0 = S.row0[s], r1 = S.row0[s + 1];
  if (r0 + lane >= r1) return;
  const int32_t row = S.srow[r0 + lane];
  const int64_t off = S.ptr[s];
  const int w = static_cast<int>((S.ptr[s + 1] - off) >> 6);
  const T acc = sell_row<T, T>(S, off, w, lane, x);
  d[row] = f[row] - acc;
}

// residual of one color's rows, for a smoother phase whose color has couplings between its own cells (the fused
// phase below then reads it from d)
template <class T>
__global__ void __launch_bounds__(kBlock) k_fine_resid(SellView<T> S, SliceSched Z, const T *__restrict__ f,
                                                        const T *__restrict__ x, T *__restrict__ d) {
  fine_resid_body(S, Z, f, x, d);
}

// residual of all rows (input of the restriction); a kernel of its own so its launches are timed separately
template <class T>
__global__ void __launch_bounds__(kBlock) k_fine_resid_full(SellView<T> S, SliceSched Z, const T *__restrict__ f,
                                                             const T *__restrict__ x, T *__restrict__ d) {
  fine_resid_body(S, Z, f, x, d);
}

// y = A x over the scheduled slices (level hook)
template <class T>
__global__ void __launch_bounds__(kBlock) k_fine_apply(SellView<T> S, SliceSched Z, const T *__restrict__ x,
                                                        T *__restrict__ y) {
  const int64_t s = sched_slice(Z);
  if (s < 0) return;
  const int lane = threadIdx.x & 63;
  if (S.row0[s] + lane >= S.row0[s + 1]) return;
  const int32_t row = S.srow[S.row0[s] + lane];
  const int64_t off = S.ptr[s];
  const int w = static_cast<int>((S.ptr[s + 1] - off) >> 6);
  const T acc = sell_row<T, T>(S, off, w, lane, x);
  y[row] = acc;
}

// L L^t v = v in place, L packed lower triangle (row i holds L_i0 .. L_ii), v with the given element stride
template <class T>
__device__ inline void block_solve(const T *Lf, int m, T *v, int stride) {
  for (int i = 0; i < m; i++) {
    const T *Li = Lf + i * (i + 1) / 2;
    T s = v[i * stride];
    for (int k = 0; k < i; k++) s -= Li[k] * v[k * stride];
    v[i * stride] = s / Li[i];
  }
  for (int i = m - 1; i >= 0; i--) {
    T s = v[i * stride];
    for (int k = m - 1; k > i; k--) s -= Lf[k * (k + 1) / 2 + i] * v[k * stride];
    v[i * stride] = s / Lf[i * (i + 1) / 2 + i];
  }
}

// block_solve with the cell's vector in registers, for cells of at most MC unknowns: the same operations in the same
// order (the loops are unrolled to MC and guarded by m), so the results are identical, but the substitutions wait on
// register operands instead of a chain of LDS round trips; only the factor values are read from memory.
template <class T, int MC>
__device__ __forceinline__ void block_solve_reg(const T *Lf, int m, T *v) {
  T y[MC];
#pragma unroll
  for (int i = 0; i < MC; i++) y[i] = i < m ? v[i] : T(0);
#pragma unroll
  for (int i = 0; i < MC; i++) {
    if (i < m) {
      const T *Li = Lf + i * (i + 1) / 2;
      T s = y[i];
#pragma unroll
      for (int k = 0; k < i; k++) s -= Li[k] * y[k];
      y[i] = s / Li[i];
    }
    __builtin_amdgcn_sched_barrier(0);  // one row's factor values in flight at a time
  }
  // backward by columns: x_k is final once the columns above it are subtracted; row k of the factor then updates
  // the rows below it (each row's subtractions in descending k, the order of block_solve)
#pragma unroll
  for (int k = MC - 1; k >= 0; k--) {
    if (k < m) {
      const T *Lk = Lf + k * (k + 1) / 2;
      y[k] = y[k] / Lk[k];
#pragma unroll
      for (int i = 0; i < k; i++) y[i] -= Lk[i] * y[k];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int i = 0; i < MC; i++)
    if (i < m) v[i] = y[i];
}

// register classes up to kRegCell unknowns, the cells one thread solves in the fused phase (a 32-unknown class needs
// more registers than a thread holds without spilling)
constexpr int kRegCell = 16;
template <class T>
__device__ inline void block_solve_small(const T *Lf, int m, T *v) {
  static_assert(kRegCell == 16, "register classes 4, 8, 16");
  if (m <= 4) block_solve_reg<T, 4>(Lf, m, v);
  else if (m <= 8) block_solve_reg<T, 8>(Lf, m, v);
  else block_solve_reg<T, 16>(Lf, m, v);
}

template <class T>
__device__ __forceinline__ T wave_lane_value(T v, int k) {  // v of lane k (k uniform over the wavefront)
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
  } else {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), k);
    const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), k);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
  }
}

// block_solve by one wavefront, lane i holding row i (m <= kBlockMax <= 64): column k is finished, broadcast, and
// subtracted from the rows it couples to, so each row sees the same subtractions in the same order as block_solve
// (columns ascending forward, descending backward) and the results are identical; the dependent chain is 2 m
// broadcast steps instead of m^2 dependent memory operations of one thread.
template <class T>
__device__ inline void block_solve_wave(const T *Lf, int m, T *v, int lane) {
  static_assert(kBlockMax <= 64, "one row per lane");
  T y = lane < m ? v[lane] : T(0);
#pragma unroll 2
  for (int k = 0; k < m; k++) {
    const T yk = wave_lane_value(y, k) / Lf[k * (k + 1) / 2 + k];
    if (lane == k) y = yk;
    else if (lane > k && lane < m) y -= Lf[lane * (lane + 1) / 2 + k] * yk;
  }
#pragma unroll 2
  for (int k = m - 1; k >= 0; k--) {
    const T xk = wave_lane_value(y, k) / Lf[k * (k + 1) / 2 + k];
    if (lane == k) y = xk;
    else if (lane < k) y -= Lf[k * (k + 1) / 2 + lane] * xk;
  }
  if (lane < m) v[lane] = y;
}

// One color phase of the fine-level smoother (Section 4.5), fused: a workgroup per window (a run of whole cells of
// the color and the sliced-ELL slices of exactly their rows).
//  1. The residual r = f - A u of the window's rows, one wavefront per slice with the residual pass's arithmetic,
//     kept in LDS; with GIVEN, r is read from src instead (f for the first phase of a sweep from zero, or d filled
//     by k_fine_resid when cells of the color are coupled to each other, which a fused residual would race with).
//  2. Each cell of at most CMAX unknowns is solved there by one thread: SM = 1, the exact block L L^t delta = r with
//     the cell's Cholesky factor; SM = 0, the in-cell substitution, delta_p = (r_p - sum a_pc delta_c) / a_pp over
//     the cell's rows ascending (FWD, c < p) or descending (c > p).
//  3. u += delta with coalesced stores. The rows of larger cells get r in d instead, for k_fine_subst_big.
// The window's cell bounds, rows of u, factor values and in-cell couplings are contiguous and staged in LDS with
// coalesced loads issued together with the residual's, so the kernel waits on few dependent round trips to memory.
// A window holds at most kFuseStageRows rows and kFuseCells cells unless it is a single cell of more unknowns than a
// fused window stages; its factor values or in-cell couplings go to dynamic LDS sized by the setup's largest window
// (at most kFuseDynBytes). A window that exceeds the staging arrays takes the same arithmetic on global memory; a
// window of one cell too large to solve here has, with GIVEN, nothing to do (k_fine_subst_big reads the given
// residual itself). Without GIVEN either the color's cells are not coupled to each other, or (split) the residual
// reads the color's own rows from alt, which holds their values from before the phase (zero in a sweep from zero;
// the copy the prolongation makes before the backward sweep), so no workgroup reads another's corrections and the
// residual is the separate pass's value for value; u of a window's rows changes only in its own workgroup.
constexpr int kFuseRows = kFuseStageRows;
constexpr int kFuseCells = 512;
constexpr int kFuseDynBytes = 48 * 1024;
template <class T, int SM>
constexpr int fuse_ent_bytes() {  // LDS bytes per staged factor value (exact blocks) or in-cell coupling
  return SM ? static_cast<int>(sizeof(T)) : static_cast<int>(sizeof(T) + sizeof(int16_t));
}

// r_p - sum of a_pc x_c over the in-cell couplings k0 <= k < k1 of row p with c < p (FWD) or c > p, in entry order:
// the couplings of a chunk are read together, then the x_c they need, then the products are subtracted in order, so
// a row waits on two LDS round trips per chunk of kSubstChunk couplings instead of two per coupling
constexpr int kSubstChunk = 8;
template <class T, bool FWD>
__device__ __forceinline__ T subst_row(T acc, int k0, int k1, int p, const int16_t *s_col, const T *s_val,
                                       const T *s_x) {
  for (int kb = k0; kb < k1; kb += kSubstChunk) {
    int c[kSubstChunk];
    T v[kSubstChunk], x[kSubstChunk];
#pragma unroll
    for (int u = 0; u < kSubstChunk; u++) {
      c[u] = p;
      v[u] = T(0);
      if (kb + u < k1) {
        c[u] = s_col[kb + u];
        v[u] = s_val[kb + u];
      }
    }
#pragma unroll
    for (int u = 0; u < kSubstChunk; u++) x[u] = (FWD ? c[u] < p : c[u] > p) ? s_x[c[u]] : T(0);
#pragma unroll
    for (int u = 0; u < kSubstChunk; u++)
      if (FWD ? c[u] < p : c[u] > p) acc -= v[u] * x[u];
  }
  return acc;
}

template <class T>
struct FuseArgs {
  const int32_t *win_q, *win_row, *crow;
  const int64_t *win_slice, *win_ent;
  int64_t win0, nwin;            // this color's windows
  int xcd;                       // 1: XCD-aware window order (grid = 8 x the largest per-XCD share)
  int big;                       // the color has cells left to k_fine_subst_big: write their residual to d
  int ent_cap;                   // factor values / couplings the dynamic LDS holds
  int split;                     // 1: the residual reads the color's own rows [clo, chi) from alt (zero when null)
  int32_t clo, chi;
  const T *alt;
  const T *f, *src;              // src: the given residual (GIVEN)
  T *u, *d;
  const T *diag, *icv, *fac;
  const int32_t *icp, *icc;
  const int64_t *boff;
};

template <class T, int SM, bool FWD, bool GIVEN>
__global__ void __launch_bounds__(kBlock) k_fine_gs(SellView<T> S, FuseArgs<T> A) {
  constexpr int CMAX = SM ? kBlockMax : kBigCell;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ T s_r[kFuseRows];                   // residual (SM = 1: then the delta, in place)
  __shared__ T s_u[kFuseRows];                   // u of the window's rows
  __shared__ T s_dx[SM ? 1 : kFuseRows];         // the deltas (SM = 0)
  __shared__ T s_dg[SM ? 1 : kFuseRows];
  __shared__ int32_t s_ep[SM ? 1 : kFuseRows + 1];
  T *s_x = SM ? reinterpret_cast<T *>(smem) : s_dx;        // factor values (SM = 1) or the deltas (SM = 0)
  T *s_val = reinterpret_cast<T *>(smem);                  // in-cell couplings (SM = 0)
  int16_t *s_col = reinterpret_cast<int16_t *>(smem + sizeof(T) * A.ent_cap);
  __shared__ int32_t s_cr[kFuseCells + 1];       // cell bounds relative to the first row
  __shared__ int32_t s_cf[SM ? kFuseCells + 1 : 1];  // factor offsets relative to the first value
  __shared__ uint8_t s_mine[kFuseRows];
  constexpr int kTeamCells = kFuseRows / (kRegCell + 1) + 1;  // cells a wavefront solves (more than kRegCell rows)
  __shared__ int16_t s_team[SM ? kTeamCells : 1];
  __shared__ int s_nteam;
  int64_t w;
  if (A.xcd) {
    const int64_t x = blockIdx.x & 7u, p = blockIdx.x >> 3;
    const int64_t b0 = A.nwin * x / 8, b1 = A.nwin * (x + 1) / 8;
    if (p >= b1 - b0) return;
    w = A.win0 + b0 + p;
  } else {
    w = A.win0 + blockIdx.x;
  }
  const int t = threadIdx.x, lane = t & 63;
  const int32_t q0 = A.win_q[w], q1 = A.win_q[w + 1];
  const int32_t r0 = A.win_row[w], r1 = A.win_row[w + 1];
  const int64_t sl0 = A.win_slice[w], sl1 = A.win_slice[w + 1];
  const int64_t e0 = A.win_ent[w], ne = A.win_ent[w + 1] - e0;
  const int nr = r1 - r0, nq = q1 - q0;
  if (GIVEN && nq == 1 && nr > CMAX) return;  // one cell left to k_fine_subst_big, which reads src
  const bool staged = nr <= kFuseRows && ne <= A.ent_cap && nq <= kFuseCells;  // uniform over the workgroup
  if (staged) {
    // every thread issues all its loads of a batch before its LDS stores, so the staging waits on one round trip to
    // memory per batch instead of one per element
    constexpr int kCellIt = (kFuseCells + 1 + kBlock - 1) / kBlock, kRowIt = kFuseRows / kBlock, kEntBatch = 8;
    {
      int32_t cr[kCellIt];
      int64_t cf[kCellIt];
#pragma unroll
      for (int u = 0; u < kCellIt; u++) {
        const int k = t + u * kBlock;
        if (k <= nq) {
          cr[u] = A.crow[q0 + k];
          if constexpr (SM) cf[u] = A.boff[q0 + k];
        }
      }
#pragma unroll
      for (int u = 0; u < kCellIt; u++) {
        const int k = t + u * kBlock;
        if (k <= nq) {
          s_cr[k] = cr[u] - r0;
          if constexpr (SM) s_cf[k] = static_cast<int32_t>(cf[u] - e0);
        }
      }
    }
    for (int kb = t; kb < ne; kb += kEntBatch * kBlock) {
      T v[kEntBatch];
      int32_t c[kEntBatch];
#pragma unroll
      for (int u = 0; u < kEntBatch; u++) {
        const int k = kb + u * kBlock;
        if (k < ne) {
          if constexpr (SM) {
            v[u] = A.fac[e0 + k];
          } else {
            c[u] = A.icc[e0 + k];
            v[u] = A.icv[e0 + k];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kEntBatch; u++) {
        const int k = kb + u * kBlock;
        if (k < ne) {
          if constexpr (SM) {
            s_x[k] = v[u];
          } else {
            s_col[k] = static_cast<int16_t>(c[u] - r0);
            s_val[k] = v[u];
          }
        }
      }
    }
    {
      T uu[kRowIt], dg[kRowIt], rr[kRowIt];
      int32_t ep[kRowIt];
#pragma unroll
      for (int u = 0; u < kRowIt; u++) {
        const int i = t + u * kBlock;
        if (i < nr) {
          uu[u] = A.u[r0 + i];
          if constexpr (!SM) {
            dg[u] = A.diag[r0 + i];
            ep[u] = A.icp[r0 + i];
          }
          if constexpr (GIVEN) rr[u] = A.src[r0 + i];
        }
      }
#pragma unroll
      for (int u = 0; u < kRowIt; u++) {
        const int i = t + u * kBlock;
        if (i < nr) {
          s_u[i] = uu[u];
          if constexpr (!SM) {
            s_dg[i] = dg[u];
            s_ep[i] = static_cast<int32_t>(ep[u] - e0);
          }
          if constexpr (GIVEN) s_r[i] = rr[u];
          s_mine[i] = 0;
        }
      }
    }
    if constexpr (!SM)
      if (t == 0) s_ep[nr] = static_cast<int32_t>(ne);
    if constexpr (SM)
      if (t == 0) s_nteam = 0;
  }
  if constexpr (!GIVEN) {
    // slice k of the window holds the positions r0 + 64 k .. (rows of the window, sorted by length)
    for (int64_t sl = sl0 + (t >> 6); sl < sl1; sl += kBlock / 64) {
      const int32_t p = r0 + static_cast<int32_t>(sl - sl0) * kSliceRows + lane;
      if (p < r1) {
        const int32_t row = S.srow[p];
        const int64_t off = S.ptr[sl];
        const int wd = static_cast<int>((S.ptr[sl + 1] - off) >> 6);
        const T r = A.f[row] - (A.split ? sell_row_split<T>(S, off, wd, lane, A.u, A.alt, A.clo, A.chi)
                                        : sell_row<T, T>(S, off, wd, lane, A.u));
        if (staged) s_r[row - r0] = r;
        else A.d[row] = r;
      }
    }
  } else {
    if (!staged && A.src != A.d)
      for (int i = t; i < nr; i += kBlock) A.d[r0 + i] = A.src[r0 + i];
  }
  __syncthreads();  // also orders the global residual writes of the unstaged path within the workgroup
  for (int j = t; j < nq; j += kBlock) {
    if (staged) {
      const int a = s_cr[j], b = s_cr[j + 1];
      const int m = b - a;
      if (m == 0 || m > CMAX) continue;
      if constexpr (SM) {
        if (m > kRegCell) s_team[atomicAdd(&s_nteam, 1)] = static_cast<int16_t>(j);
        else block_solve_small<T>(s_x + s_cf[j], m, s_r + a);
      } else {
        for (int i = 0; i < m; i++) {
          const int p = FWD ? a + i : b - 1 - i;
          s_x[p] = subst_row<T, FWD>(s_r[p], s_ep[p], s_ep[p + 1], p, s_col, s_val, s_x) / s_dg[p];
        }
      }
      for (int i = a; i < b; i++) s_mine[i] = 1;
    } else {
      const int32_t ca = A.crow[q0 + j], cb = A.crow[q0 + j + 1];
      const int m = cb - ca;
      if (m == 0 || m > CMAX) continue;
      T *dd = A.d;
      if constexpr (SM) {
        block_solve<T>(A.fac + A.boff[q0 + j], m, dd + ca, 1);
      } else if constexpr (FWD) {
        for (int32_t p = ca; p < cb; p++) {
          T acc = dd[p];
          for (int32_t e = A.icp[p]; e < A.icp[p + 1]; e++) {
            const int32_t c = A.icc[e];
            if (c < p) acc -= A.icv[e] * dd[c];
          }
          dd[p] = acc / A.diag[p];
        }
      } else {
        for (int32_t p = cb - 1; p >= ca; p--) {
          T acc = dd[p];
          for (int32_t e = A.icp[p]; e < A.icp[p + 1]; e++) {
            const int32_t c = A.icc[e];
            if (c > p) acc -= A.icv[e] * dd[c];
          }
          dd[p] = acc / A.diag[p];
        }
      }
      for (int32_t p = ca; p < cb; p++) A.u[p] += dd[p];
    }
  }
  if (!staged) return;
  __syncthreads();
  if constexpr (SM) {  // the window's larger cells, one wavefront each
    const int nt = s_nteam;
    if (nt > 0) {
      for (int k = t >> 6; k < nt; k += kBlock / 64) {
        const int j = s_team[k];
        const int a = s_cr[j];
        block_solve_wave<T>(s_x + s_cf[j], s_cr[j + 1] - a, s_r + a, lane);
      }
      __syncthreads();
    }
  }
  for (int i = t; i < nr; i += kBlock) {
    if (s_mine[i]) A.u[r0 + i] = s_u[i] + (SM ? s_r[i] : s_x[i]);
    else if (A.big && !GIVEN) A.d[r0 + i] = s_r[i];
  }
}

// The same substitution for the big cells of one color, one workgroup per cell: rows are taken level by level of the
// cell's dependency schedule (the rows of a level use only values of earlier levels), with a barrier between levels;
// each row's arithmetic is the thread-per-cell kernel's (the same couplings in the same order), so the results are
// identical. The cell's vector lives in LDS while it is solved, and each thread loads the rows of its first
// kSubstRegRows schedule positions (row, diagonal, first kSubstRegCouplings in-cell couplings) into registers before
// the first level, so a level costs LDS reads and a barrier instead of a chain of dependent global loads. A cell of
// more rows than the LDS holds, or with a deeper schedule than kSubstLevels, takes the same arithmetic on global
// memory (coherent within a workgroup at the barrier: all its wavefronts share one CU).
constexpr int kSubstLanes = 256;
constexpr int kSubstRegRows = 4;
constexpr int kSubstRegCouplings = 8;
constexpr int kSubstLevels = 256;
constexpr int kSubstDynBytes = 48 * 1024;

template <class T, bool FWD>
__global__ void __launch_bounds__(kSubstLanes) k_fine_subst_big(const int32_t *__restrict__ crow,
                                                            const int32_t *__restrict__ icp,
                                                            const int32_t *__restrict__ icc,
                                                            const T *__restrict__ icv, const T *__restrict__ diag,
                                                            const T *src, T *d, T *__restrict__ x,
                                                            const int32_t *__restrict__ cells, int64_t b_begin,
                                                            const int32_t *__restrict__ lofs,
                                                            const int32_t *__restrict__ lptr,
                                                            const int32_t *__restrict__ sched, int lds_rows) {
  constexpr int R = kSubstRegRows, KM = kSubstRegCouplings;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int32_t s_lp[kSubstLevels + 1];
  T *s_d = reinterpret_cast<T *>(smem);
  const int32_t t = static_cast<int32_t>(threadIdx.x);
  const int64_t b = b_begin + blockIdx.x;
  const int32_t q = cells[b];
  const int32_t a = crow[q], e = crow[q + 1];
  const int32_t l0 = lofs[b], l1 = lofs[b + 1];
  const int32_t nl = l1 - l0;  // level starts and the end
  if (e - a > lds_rows || nl > kSubstLevels + 1) {
    for (int32_t lv = l0; lv + 1 < l1; lv++) {
      for (int32_t i = lptr[lv] + t; i < lptr[lv + 1]; i += kSubstLanes) {
        const int32_t p = sched[i];
        T acc = src[p];
        for (int32_t k = icp[p]; k < icp[p + 1]; k++) {
          const int32_t c = icc[k];
          if (FWD ? c < p : c > p) acc -= icv[k] * d[c];
        }
        d[p] = acc / diag[p];
      }
      __syncthreads();
    }
    for (int32_t p = a + t; p < e; p += kSubstLanes) x[p] += d[p];
    return;
  }
  for (int32_t p0 = a + t; p0 < e; p0 += 4 * kSubstLanes) {  // four loads in flight per thread
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; u++)
      if (p0 + u * kSubstLanes < e) v[u] = src[p0 + u * kSubstLanes];
#pragma unroll
    for (int u = 0; u < 4; u++)
      if (p0 + u * kSubstLanes < e) s_d[p0 + u * kSubstLanes - a] = v[u];
  }
  for (int32_t k = t; k < nl; k += kSubstLanes) s_lp[k] = lptr[l0 + k];
  // schedule positions a + t + kSubstLanes j (j < R), rows and couplings relative to a
  int32_t rp[R], rk[R], rn[R], rc[R][KM];
  T rdg[R], rv[R][KM];
#pragma unroll
  for (int j = 0; j < R; j++) {
    const int32_t i = a + t + kSubstLanes * j;
    rp[j] = 0;
    rk[j] = 0;
    rn[j] = 0;
    rdg[j] = T(1);
#pragma unroll
    for (int k = 0; k < KM; k++) {
      rc[j][k] = 0;
      rv[j][k] = T(0);
    }
    if (i < e) {
      const int32_t p = sched[i];
      rp[j] = p - a;
      rdg[j] = diag[p];
      rk[j] = icp[p];
      rn[j] = icp[p + 1] - rk[j];
#pragma unroll
      for (int k = 0; k < KM; k++)
        if (k < rn[j]) {
          rc[j][k] = icc[rk[j] + k] - a;
          rv[j][k] = icv[rk[j] + k];
        }
    }
  }
  __syncthreads();
  for (int32_t lv = 0; lv + 1 < nl; lv++) {
    const int32_t lo = s_lp[lv], hi = s_lp[lv + 1];
#pragma unroll
    for (int j = 0; j < R; j++) {
      const int32_t i = a + t + kSubstLanes * j;
      if (i >= lo && i < hi) {
        const int32_t p = rp[j];
        T acc = s_d[p];
#pragma unroll
        for (int k = 0; k < KM; k++)
          if (k < rn[j]) {
            const int32_t c = rc[j][k];
            if (FWD ? c < p : c > p) acc -= rv[j][k] * s_d[c];
          }
        for (int32_t k = rk[j] + KM; k < rk[j] + rn[j]; k++) {
          const int32_t c = icc[k] - a;
          if (FWD ? c < p : c > p) acc -= icv[k] * s_d[c];
        }
        s_d[p] = acc / rdg[j];
      }
    }
    // positions past the register-held ones
    int32_t i = a + t + kSubstLanes * R;
    if (i < lo) i += (lo - i + kSubstLanes - 1) / kSubstLanes * kSubstLanes;
    for (; i < hi; i += kSubstLanes) {
      const int32_t pa = sched[i], p = pa - a;
      T acc = s_d[p];
      for (int32_t k = icp[pa]; k < icp[pa + 1]; k++) {
        const int32_t c = icc[k] - a;
        if (FWD ? c < p : c > p) acc -= icv[k] * s_d[c];
      }
      s_d[p] = acc / diag[pa];
    }
    __syncthreads();
  }
  for (int32_t p = a + t; p < e; p += kSubstLanes) {
    const T v = s_d[p - a];
    d[p] = v;
    x[p] += v;
  }
}

// g[q] = sum of d over the rows of level-L cell q (rows ascending); cells of more than `big` rows are left to
// k_fine_restrict_big
template <class T>
__global__ void __launch_bounds__(kBlock) k_fine_restrict(int64_t nL, const int32_t *__restrict__ crow,
                                                           const T *__restrict__ d, T *__restrict__ g, int big) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= nL) return;
  const int32_t a = crow[q], b = crow[q + 1];
  if (b - a > big) return;
  T acc = 0;
  for (int32_t p = a; p < b; p++) acc += d[p];
  g[q] = acc;
}

// the same sum for the listed cells, one wavefront per cell: the wavefront stages the cell's d in LDS with coalesced
// loads, 1,024 rows at a time, and lane 0 adds them in ascending order (the thread-per-cell order), so a cell of a
// thousand rows costs LDS reads instead of a chain of dependent global loads
constexpr int kRestrictChunk = 1024;

template <class T>
__global__ void __launch_bounds__(64) k_fine_restrict_big(const int32_t *__restrict__ cells,
                                                           const int32_t *__restrict__ crow,
                                                           const T *__restrict__ d, T *__restrict__ g) {
  __shared__ T s_d[kRestrictChunk];
  const int32_t q = cells[blockIdx.x];
  const int32_t a = crow[q], b = crow[q + 1];
  T acc = 0;
  for (int32_t c0 = a; c0 < b; c0 += kRestrictChunk) {
    const int m = min(kRestrictChunk, b - c0);
    __syncthreads();
    T v[kRestrictChunk / 64];  // all loads of the chunk in flight before the LDS stores
#pragma unroll
    for (int u = 0; u < kRestrictChunk / 64; u++) {
      const int i = static_cast<int>(threadIdx.x) + 64 * u;
      if (i < m) v[u] = d[c0 + i];
    }
#pragma unroll
    for (int u = 0; u < kRestrictChunk / 64; u++) {
      const int i = static_cast<int>(threadIdx.x) + 64 * u;
      if (i < m) s_d[i] = v[u];
    }
    __syncthreads();
    if (threadIdx.x == 0)
      for (int i = 0; i < m; i++) acc += s_d[i];
  }
  if (threadIdx.x == 0) g[q] = acc;
}

// u += P e on the fine level; snap (when not null) gets a copy of the new u
template <class T>
__global__ void __launch_bounds__(kBlock) k_fine_prolong(int64_t n, const int32_t *__restrict__ agg_q,
                                                          const T *__restrict__ e, Pending<T> pend,
                                                          T *__restrict__ u, T *__restrict__ snap) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const T em = pend.apply(e, static_cast<uint32_t>(agg_q[p]));
  const T v = u[p] + em;
  u[p] = v;
  if (snap) snap[p] = v;
}

// ---------------------------------------------------------------------------------------------------------------
// quadtree level kernels

template <class T>
struct QView {
  int k;
  int64_t n;
  const T *ax;       // 9 x n slot-major
  const int32_t *optr;  // null when the level has no overflow
  const int32_t *ocol;
  const T *oval;
};

// (A x)_q for row q = c n/4 + j of a quadtree level (slots in order 0..8, then overflow entries). A slot whose
// neighbour lies outside the grid holds the value 0, so its product is taken with x[q] instead of being branched
// around: all nine loads are independent and issue back to back.
template <class T, class XV>
__device__ inline T row_apply_f(const QView<T> &Q, uint32_t q, int c, XV xv) {
  const int sh = 2 * Q.k - 2;
  uint32_t nb[9];
  stencil_q(q, q & ((1u << sh) - 1u), c, sh, nb);
  T acc = 0;
#pragma unroll
  for (int s = 0; s < 9; s++) acc += Q.ax[s * Q.n + q] * xv(nb[s]);
  if (Q.optr)
    for (int32_t e = Q.optr[q]; e < Q.optr[q + 1]; e++) acc += Q.oval[e] * xv(static_cast<uint32_t>(Q.ocol[e]));
  return acc;
}

template <class T>
__device__ inline T row_apply(const QView<T> &Q, uint32_t q, int c, const T *__restrict__ x) {
  return row_apply_f<T>(Q, q, c, [x](uint32_t i) { return x[i]; });
}

// color of row q (sh = 2k - 2); uniform over a wavefront of consecutive rows when a color block holds >= 64 rows
__device__ inline int row_color(uint32_t q, int sh) {
  const int c = static_cast<int>(q >> sh);
  return sh >= 6 ? __builtin_amdgcn_readfirstlane(c) : c;
}

// first phase of a sweep from zero: x = f / diag on color 0, zero elsewhere (UPD: f is the pending update's r)
template <class T, bool UPD>
__global__ void __launch_bounds__(kBlock) k_cgs_first(QView<T> Q, const T *__restrict__ f, T *__restrict__ x,
                                                       Upd1<T> U) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= Q.n) return;
  if constexpr (UPD) {
    const T a = U.a0();
    x[q] = (q < (Q.n >> 2)) ? U.rv(a, static_cast<uint32_t>(q)) / Q.ax[q] : T(0);
    U.store(a, q);
  } else {
    x[q] = (q < (Q.n >> 2)) ? f[q] / Q.ax[q] : T(0);
  }
}

// the first two phases of a sweep from zero (levels without same-color couplings): x = f / diag on color 0, zero on
// colors 2 and 3, and the color-1 rows relaxed against the color-0 values formed on the fly (nothing reads x here)
template <class T, class FV>
__device__ inline void cgs_first2_row(const QView<T> &Q, int64_t q, FV fv, T *__restrict__ x) {
  const int64_t n4 = Q.n >> 2;
  if (q < n4) {
    x[q] = fv(static_cast<uint32_t>(q)) / Q.ax[q];
  } else if (q < 2 * n4) {
    const uint32_t n4u = static_cast<uint32_t>(n4);
    const T *ax = Q.ax;
    auto first = [fv, ax, n4u](uint32_t i) { return i < n4u ? fv(i) / ax[i] : T(0); };
    x[q] = T(0) + (fv(static_cast<uint32_t>(q)) - row_apply_f<T>(Q, static_cast<uint32_t>(q), 1, first)) / Q.ax[q];
  } else {
    x[q] = T(0);
  }
}

template <class T, bool UPD>
__global__ void __launch_bounds__(kBlock) k_cgs_first2(QView<T> Q, const T *__restrict__ f, T *__restrict__ x,
                                                        Upd1<T> U) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= Q.n) return;
  if constexpr (UPD) {
    const T a = U.a0();
    cgs_first2_row<T>(Q, q, [U, a](uint32_t i) { return U.rv(a, i); }, x);
    U.store(a, q);
  } else {
    cgs_first2_row<T>(Q, q, [f](uint32_t i) { return f[i]; }, x);
  }
}

// one color phase of the pointwise 4-color Gauss-Seidel: rows q = c n/4 + j, Morton m = 4 j + c.
// delta == nullptr: update in place (valid when no coupling joins two cells of color c); else write delta only.
template <class T>
__global__ void __launch_bounds__(kBlock) k_cgs(QView<T> Q, const T *__restrict__ f, T *__restrict__ x,
                                                T *__restrict__ delta, int c) {
  const int64_t n4 = Q.n >> 2;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n4) return;
  const uint32_t q = static_cast<uint32_t>(c * n4 + j);
  const T dl = (f[q] - row_apply(Q, q, c, x)) / Q.ax[q];
  if (delta) delta[q] = dl;
  else x[q] += dl;
}

// the last color phase (c = 0) of the second B^ with the inner product (p1, q0) of Algorithm 2.1 for beta: thread j
// relaxes row j and adds the products of rows j + c n/4 of all four colors (colors 1 to 3 are final already)
template <class T>
__global__ void __launch_bounds__(kBlock) k_cgs0_beta(QView<T> Q, const T *__restrict__ f, T *__restrict__ x,
                                                      const T *__restrict__ q0, Red R) {
  const int64_t n4 = Q.n >> 2;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double v[1] = {0.0};
  if (j < n4) {
    const uint32_t q = static_cast<uint32_t>(j);
    const T xn = x[q] + (f[q] - row_apply(Q, q, 0, x)) / Q.ax[q];
    x[q] = xn;
    v[0] = static_cast<double>(xn) * static_cast<double>(q0[q]);
#pragma unroll
    for (int c = 1; c < 4; c++) v[0] += static_cast<double>(x[c * n4 + j]) * static_cast<double>(q0[c * n4 + j]);
  }
  reduce_finish<1>(v, R);
}

// A color phase of the first post-smoothing sweep (no same-color couplings) with the prolongation u += P e_c folded
// in: the rows of colors <= C have not been corrected yet (the backward sweep has only passed colors > C), so their
// values are read as u + (P e_c) formed on the fly, each equal to what the separate prolongation stores; the phase
// stores the corrected and relaxed values of its own rows. With BETA (C = 0, the last phase of the second B^) it also
// forms (p1, q0) for beta over the rows j + c n/4 of the four colors.
template <class T, int C, bool BETA>
__global__ void __launch_bounds__(kBlock) k_cgs_post(QView<T> Q, const T *__restrict__ f, T *__restrict__ x,
                                                     const T *__restrict__ ec, Pending<T> pend,
                                                     const T *__restrict__ q0, Red R) {
  const int64_t n4 = Q.n >> 2;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int sh = 2 * Q.k - 2;
  const uint32_t mask = static_cast<uint32_t>(n4 - 1);
  const int kc = Q.k - 1;
  auto pe = [ec, pend, mask, kc](uint32_t i) { return pend.apply(ec, q_of_m(i & mask, kc)); };
  double v[1] = {0.0};
  if (j < n4) {
    const uint32_t q = static_cast<uint32_t>(C * n4 + j);
    uint32_t nb[9];
    stencil_q(q, static_cast<uint32_t>(j), C, sh, nb);
    T acc = 0;
#pragma unroll
    for (int s = 0; s < 9; s++) {
      const int cn = (((C & 1) + slot_dx(s)) & 1) | ((((C >> 1) + slot_dy(s)) & 1) << 1);
      const T xn = x[nb[s]];
      acc += Q.ax[s * Q.n + q] * (cn <= C ? xn + pe(nb[s]) : xn);
    }
    if (Q.optr)
      for (int32_t e = Q.optr[q]; e < Q.optr[q + 1]; e++) {
        const uint32_t i = static_cast<uint32_t>(Q.ocol[e]);
        const T xn = x[i];
        acc += Q.oval[e] * (static_cast<int>(i >> sh) <= C ? xn + pe(i) : xn);
      }
    const T xq = x[q] + pe(q);
    const T xr = xq + (f[q] - acc) / Q.ax[q];
    x[q] = xr;
    if constexpr (BETA) {
      v[0] = static_cast<double>(xr) * static_cast<double>(q0[q]);
#pragma unroll
      for (int c = 1; c < 4; c++) v[0] += static_cast<double>(x[c * n4 + j]) * static_cast<double>(q0[c * n4 + j]);
    }
  }
  if constexpr (BETA) reduce_finish<1>(v, R);
}

// Tiles of the per-step path. Workgroup b owns the 16 x 16 super-cells j in [256 b, 256 b + 256), a Morton-aligned
// square, and stages the values of the square and four rings of super-cells around it in LDS. A stencil reaches one
// super-cell further, so a chain of color phases runs on shrinking rings: each phase relaxes the rows that the later
// phases of the square's rows read (ring rows again in the neighbouring workgroups, from the same values). Each row
// takes the values, slot order and arithmetic of the one-launch-per-phase kernels, so the square's rows equal
// theirs bit for bit.
constexpr int kTileSide = 16;                          // super-cells per side of a workgroup's square
constexpr int kTileRings = 4;                          // rings staged around it
constexpr int kTileStage = kTileSide + 2 * kTileRings;  // 24
constexpr int kTileCells = kTileSide * kTileSide;       // 256: thread t < 256 holds super-cell 256 b + t
constexpr int kTileThreads = 512;                      // threads of a tile workgroup: one row slot per thread and
                                                       // phase, so a wavefront's prologue loads stay in flight together
static_assert(kTileCells == kBlock, "the square's partial sums are those of a kBlock-thread per-phase launch");
static_assert(kTileStage == 24 && kTileRings == 4, "the staged square is 6 x 6 blocks of 4 x 4 super-cells");

template <int RG>
struct RingRows {  // row slots per thread of a phase over the square and its RG innermost rings
  static constexpr int side = kTileSide + 2 * RG;
  static constexpr int count = side * side;
  static constexpr int slots = (count + kTileThreads - 1) / kTileThreads;
};

constexpr int kStageSlots = (kTileStage * kTileStage + kTileThreads - 1) / kTileThreads;  // 2

// staging slot i of this thread (the 6 x 6 blocks of 4 x 4 super-cells in turn, Morton order inside a block, so a
// wavefront reads four contiguous runs): its staged index, -1 outside the grid, and its super-cell's Morton index
__device__ inline int stage_slot(int i, int px0, int py0, int np, uint32_t &jm) {
  const int e = static_cast<int>(threadIdx.x) + i * kTileThreads;
  const int blk = e >> 4, w = e & 15;
  const int lx = 4 * (blk % 6) + static_cast<int>(compact_bits(static_cast<uint32_t>(w)));
  const int ly = 4 * (blk / 6) + static_cast<int>(compact_bits(static_cast<uint32_t>(w) >> 1));
  const int px = px0 + lx, py = py0 + ly;
  const bool ok = e < kTileStage * kTileStage && px >= 0 && px < np && py >= 0 && py < np;
  jm = ok ? morton(static_cast<uint32_t>(px), static_cast<uint32_t>(py)) : 0u;
  return ok ? ly * kTileStage + lx : -1;
}

template <class T, int RG>
struct RingData {
  T a[RingRows<RG>::slots][9];
  T f[RingRows<RG>::slots];
  T f2[RingRows<RG>::slots];  // with a pending first inner update: q0 of the row (f holds g until rhs_upd)
  int l[RingRows<RG>::slots];  // staged index of the row's super-cell, -1 when the slot has no row
};

// staged super-cell (lx, ly) of slot i. The staged square is 6 x 6 Morton-contiguous blocks of 4 x 4 super-cells;
// the rows of a region are taken block by block (bands of block rows, blocks across a band, row-major inside the
// part of a block in the region), so that a wavefront's loads touch a few blocks. For the square alone (RG = 0):
// its Morton order, so that thread t holds super-cell 256 b + t (threads from 256 on hold no row).
template <int RG>
__device__ inline void ring_slot_xy(int i, int &lx, int &ly) {
  const int r = static_cast<int>(threadIdx.x) + i * kTileThreads;
  if constexpr (RG == 0) {
    lx = static_cast<int>(compact_bits(static_cast<uint32_t>(r))) + kTileRings;
    ly = static_cast<int>(compact_bits(static_cast<uint32_t>(r) >> 1)) + kTileRings;
  } else {
    constexpr int W = RingRows<RG>::side;
    constexpr int band0 = W * RG, bandm = W * 4;  // rows of the outer and of an inner band of blocks
    int by, rb, h;
    if (r < band0) {
      by = 0, rb = r, h = RG;
    } else if (r < band0 + 4 * bandm) {
      const int t = r - band0;
      by = 1 + t / bandm, rb = t % bandm, h = 4;
    } else {
      by = 5, rb = r - band0 - 4 * bandm, h = RG;
    }
    int bx, rs, w;
    if (rb < RG * h) {
      bx = 0, rs = rb, w = RG;
    } else if (rb < RG * h + 16 * h) {
      const int t = rb - RG * h;
      bx = 1 + t / (4 * h), rs = t % (4 * h), w = 4;
    } else {
      bx = 5, rs = rb - RG * h - 16 * h, w = RG;
    }
    lx = (bx == 0 ? kTileRings - RG : 4 * bx) + rs % w;
    ly = (by == 0 ? kTileRings - RG : 4 * by) + rs / w;
  }
}

// the operator rows and right-hand sides of the color-C rows of the region. UPD: f and f2 take g and q0 of the
// pending first inner update, combined by rhs_upd once every load has been issued.
template <class T, int RG, int C, bool UPD>
__device__ inline void ring_load(const QView<T> &Q, const T *__restrict__ f, const Upd1<T> &U, int px0, int py0,
                                 int np, uint32_t n4, RingData<T, RG> &D) {
#pragma unroll
  for (int i = 0; i < RingRows<RG>::slots; i++) {
    int lx, ly;
    ring_slot_xy<RG>(i, lx, ly);
    const int r = static_cast<int>(threadIdx.x) + i * kTileThreads;
    const int px = px0 + lx, py = py0 + ly;
    const bool ok = r < RingRows<RG>::count && px >= 0 && px < np && py >= 0 && py < np;
    D.l[i] = ok ? ly * kTileStage + lx : -1;
    // loads without branches (a slot without a row reads row C n/4 and ignores it), so that none waits for another
    const uint32_t jm = ok ? morton(static_cast<uint32_t>(px), static_cast<uint32_t>(py)) : 0u;
    const uint32_t q = static_cast<uint32_t>(C) * n4 + jm;
#pragma unroll
    for (int s = 0; s < 9; s++) D.a[i][s] = Q.ax[s * Q.n + q];
    if constexpr (UPD) {
      D.f[i] = U.g[q];
      D.f2[i] = U.q0[q];
    } else {
      D.f[i] = f[q];
    }
  }
}

// r = g - a0 q0 of the pending first inner update as the right-hand side of the region's rows
template <class T, int RG>
__device__ inline void rhs_upd(RingData<T, RG> &D, T a0) {
#pragma unroll
  for (int i = 0; i < RingRows<RG>::slots; i++)
    if (D.l[i] >= 0) D.f[i] = upd1_r(D.f[i], a0, D.f2[i]);
}

// sum over the nine slots of a color-C row at staged index l (a slot outside the grid holds 0: its product is taken
// with the row's own value, as the per-phase kernels do)
template <class T, int C>
__device__ inline T ring_row(const T (&a)[9], int l, int px0, int py0, int np, const T (*sv)[kTileStage * kTileStage]) {
  constexpr int cx = C & 1, cy = C >> 1;
  const int lx = l % kTileStage, ly = l / kTileStage;
  T acc = 0;
#pragma unroll
  for (int s = 0; s < 9; s++) {
    const int ux = cx + slot_dx(s), uy = cy + slot_dy(s);
    const int cn = (ux & 1) | ((uy & 1) << 1);
    const int nx = lx + (ux >> 1), ny = ly + (uy >> 1);
    const int gx = px0 + nx, gy = py0 + ny;
    const bool in = gx >= 0 && gx < np && gy >= 0 && gy < np;
    acc += a[s] * (in ? sv[cn][ny * kTileStage + nx] : sv[C][l]);
  }
  return acc;
}

// one color phase: x_q + (f_q - (A x)_q) / a_qq for the color-C rows of the region
template <class T, int RG, int C>
__device__ inline void ring_phase(const RingData<T, RG> &D, int px0, int py0, int np, T (*sv)[kTileStage * kTileStage]) {
#pragma unroll
  for (int i = 0; i < RingRows<RG>::slots; i++) {
    const int l = D.l[i];
    if (l < 0) continue;
    const T acc = ring_row<T, C>(D.a[i], l, px0, py0, np, sv);
    const T xq = sv[C][l];
    sv[C][l] = xq + (D.f[i] - acc) / D.a[i][0];
  }
}

// residuals f_q - (A x)_q of the square's color-C rows among the region's rows, by the square's Morton index
template <class T, int RG, int C>
__device__ inline void ring_resid(const RingData<T, RG> &D, int px0, int py0, int np,
                                  const T (*sv)[kTileStage * kTileStage], T *res) {
#pragma unroll
  for (int i = 0; i < RingRows<RG>::slots; i++) {
    const int l = D.l[i];
    if (l < 0) continue;
    const int tx = l % kTileStage - kTileRings, ty = l / kTileStage - kTileRings;
    if (tx < 0 || tx >= kTileSide || ty < 0 || ty >= kTileSide) continue;
    const T acc = ring_row<T, C>(D.a[i], l, px0, py0, np, sv);
    res[morton(static_cast<uint32_t>(tx), static_cast<uint32_t>(ty))] = D.f[i] - acc;
  }
}

// (p1, q0) partial of the square: the sum over threads 0..255 in block_sum's order, stored as reduce_finish stores
// it (every thread of the workgroup calls this)
__device__ inline void tile_reduce_finish(double v, const Red &R) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  __shared__ double s[kTileThreads / 64];
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc[1] = {(s[0] + s[1]) + (s[2] + s[3])};
    if (gridDim.x == 1) epilogue(acc, R);
    else R.partials[blockIdx.x] = acc[0];
  }
}

// The whole first post-smoothing sweep (color phases 3, 2, 1, 0, the prolongation folded in as in k_cgs_post) of a
// level without same-color couplings or overflow entries, in one launch: u + P e_c staged over the square and its
// rings, phase C on the color-C rows of the square and its C innermost rings. With BETA thread t forms (p1, q0) over
// rows j + c n/4 of super-cell j = 256 b + t, as k_cgs_post<T, 0, true> does, so the partials are the same.
template <class T, bool BETA>
__global__ void __launch_bounds__(kTileThreads) k_cgs_post4(QView<T> Q, const T *__restrict__ f, T *__restrict__ x,
                                                      const T *__restrict__ ec, Pending<T> pend,
                                                      const T *__restrict__ q0, Red R) {
  __shared__ T sv[4][kTileStage * kTileStage];
  const int kc = Q.k - 1;
  const int np = 1 << kc;
  const uint32_t n4 = static_cast<uint32_t>(Q.n >> 2);
  const uint32_t j0 = blockIdx.x * static_cast<uint32_t>(kTileCells);
  const int px0 = static_cast<int>(compact_bits(j0)) - kTileRings;
  const int py0 = static_cast<int>(compact_bits(j0 >> 1)) - kTileRings;
  // every load of the prologue is issued before the first value is formed
  // (branch-free: a slot outside the grid reads super-cell 0 and ignores it)
  int sl[kStageSlots];
  T sx[kStageSlots][4], se[kStageSlots], s1[kStageSlots], s0[kStageSlots];
  const T *p1p = pend.sc ? pend.p1 : ec, *p0p = pend.sc ? pend.p0 : ec;
#pragma unroll
  for (int i = 0; i < kStageSlots; i++) {
    uint32_t jm;
    sl[i] = stage_slot(i, px0, py0, np, jm);
#pragma unroll
    for (int c = 0; c < 4; c++) sx[i][c] = x[c * n4 + jm];
    const uint32_t m = q_of_m(jm, kc);
    se[i] = ec[m];
    s1[i] = p1p[m];
    s0[i] = p0p[m];
  }
  T q0v[4];
  const int t = static_cast<int>(threadIdx.x);
  const uint32_t jt = j0 + static_cast<uint32_t>(t & (kTileCells - 1));  // clamped for threads without a super-cell
  if constexpr (BETA) {
#pragma unroll
    for (int c = 0; c < 4; c++) q0v[c] = q0[c * n4 + jt];
  }
  const Upd1<T> none{};
  RingData<T, 3> D3;
  RingData<T, 2> D2;
  RingData<T, 1> D1;
  RingData<T, 0> D0;
  ring_load<T, 3, 3, false>(Q, f, none, px0, py0, np, n4, D3);
  ring_load<T, 2, 2, false>(Q, f, none, px0, py0, np, n4, D2);
  ring_load<T, 1, 1, false>(Q, f, none, px0, py0, np, n4, D1);
  ring_load<T, 0, 0, false>(Q, f, none, px0, py0, np, n4, D0);
  // u + P e_c as k_cgs_post forms it
#pragma unroll
  for (int i = 0; i < kStageSlots; i++)
    if (sl[i] >= 0) {
      const T em = pend.sc ? pend.mix(se[i], s1[i], s0[i]) : se[i];
#pragma unroll
      for (int c = 0; c < 4; c++) sv[c][sl[i]] = sx[i][c] + em;
    }
  __syncthreads();
  ring_phase<T, 3, 3>(D3, px0, py0, np, sv);
  __syncthreads();
  ring_phase<T, 2, 2>(D2, px0, py0, np, sv);
  __syncthreads();
  ring_phase<T, 1, 1>(D1, px0, py0, np, sv);
  __syncthreads();
  ring_phase<T, 0, 0>(D0, px0, py0, np, sv);  // thread t's own row: read back below by thread t alone
  const int lj = D0.l[0];
  double v = 0.0;
  if (t < kTileCells) {
#pragma unroll
    for (int c = 0; c < 4; c++) x[c * n4 + jt] = sv[c][lj];
    if constexpr (BETA) {
      v = static_cast<double>(sv[0][lj]) * static_cast<double>(q0v[0]);
#pragma unroll
      for (int c = 1; c < 4; c++) v += static_cast<double>(sv[c][lj]) * static_cast<double>(q0v[c]);
    }
  }
  if constexpr (BETA) tile_reduce_finish(v, R);
}

// The whole presmoothing sweep from zero and the restriction (k_cgs_first2, the color phases 2 and 3, k_cres_restrict)
// of a level without same-color couplings or overflow entries, in one launch: color 0 = f / diag staged over the
// square and its rings (colors 1 to 3 zero), then color 1 on three rings, color 2 on two, color 3 on one, and the
// square's residuals summed over the four children in the order 0, 1, 3, 2 into the parent's slot. UPD: the right-hand
// side is the pending first inner update's r, formed on the fly, and the update's e and r are stored for the square.
template <class T, bool UPD>
__global__ void __launch_bounds__(kTileThreads) k_cgs_pre4(QView<T> Q, const T *__restrict__ f, T *__restrict__ x, Upd1<T> U,
                                                     T *__restrict__ gc) {
  __shared__ T sv[4][kTileStage * kTileStage];
  __shared__ T res[4][kTileCells];
  const int kc = Q.k - 1;
  const int np = 1 << kc;
  const uint32_t n4 = static_cast<uint32_t>(Q.n >> 2);
  const uint32_t j0 = blockIdx.x * static_cast<uint32_t>(kTileCells);
  const int px0 = static_cast<int>(compact_bits(j0)) - kTileRings;
  const int py0 = static_cast<int>(compact_bits(j0 >> 1)) - kTileRings;
  const T a0 = UPD ? U.a0() : T(0);
  // every load of the prologue is issued before the first value is formed
  int sl[kStageSlots];
  T sf[kStageSlots], sq[kStageSlots], sd[kStageSlots];
#pragma unroll
  for (int i = 0; i < kStageSlots; i++) {  // branch-free, as in k_cgs_post4
    uint32_t jm;
    sl[i] = stage_slot(i, px0, py0, np, jm);
    if constexpr (UPD) {
      sf[i] = U.g[jm];
      sq[i] = U.q0[jm];
    } else {
      sf[i] = f[jm];
    }
    sd[i] = Q.ax[jm];
  }
  T up[4], ug[4], uq[4];  // p0, g, q0 of the square's rows for the update's e and r
  const int t = static_cast<int>(threadIdx.x);
  const uint32_t jt = j0 + static_cast<uint32_t>(t & (kTileCells - 1));  // clamped for threads without a super-cell
  if constexpr (UPD) {
#pragma unroll
    for (int c = 0; c < 4; c++) {
      up[c] = U.p0[c * n4 + jt];
      ug[c] = U.g[c * n4 + jt];
      uq[c] = U.q0[c * n4 + jt];
    }
  }
  RingData<T, 3> D1;
  RingData<T, 2> D2;
  RingData<T, 1> D3;
  RingData<T, 0> D0;
  ring_load<T, 3, 1, UPD>(Q, f, U, px0, py0, np, n4, D1);
  ring_load<T, 2, 2, UPD>(Q, f, U, px0, py0, np, n4, D2);
  ring_load<T, 1, 3, UPD>(Q, f, U, px0, py0, np, n4, D3);
  ring_load<T, 0, 0, UPD>(Q, f, U, px0, py0, np, n4, D0);
  if constexpr (UPD) {
    rhs_upd<T, 3>(D1, a0);
    rhs_upd<T, 2>(D2, a0);
    rhs_upd<T, 1>(D3, a0);
    rhs_upd<T, 0>(D0, a0);
  }
  // color 0 = f / diag as k_cgs_first2 forms it, colors 1 to 3 zero
#pragma unroll
  for (int i = 0; i < kStageSlots; i++)
    if (sl[i] >= 0) {
      T fi;
      if constexpr (UPD) fi = upd1_r(sf[i], a0, sq[i]);
      else fi = sf[i];
      sv[0][sl[i]] = fi / sd[i];
      sv[1][sl[i]] = T(0);
      sv[2][sl[i]] = T(0);
      sv[3][sl[i]] = T(0);
    }
  if (UPD && t < kTileCells) {  // the update's e and r of the square's rows as Upd1::store forms them (independent
                                // of the sweep)
#pragma unroll
    for (int c = 0; c < 4; c++) {
      U.e[c * n4 + jt] = a0 * up[c];
      U.r[c * n4 + jt] = upd1_r(ug[c], a0, uq[c]);
    }
  }
  __syncthreads();
  ring_phase<T, 3, 1>(D1, px0, py0, np, sv);
  __syncthreads();
  ring_phase<T, 2, 2>(D2, px0, py0, np, sv);
  __syncthreads();
  ring_phase<T, 1, 3>(D3, px0, py0, np, sv);
  __syncthreads();
  ring_resid<T, 0, 0>(D0, px0, py0, np, sv, res[0]);
  ring_resid<T, 3, 1>(D1, px0, py0, np, sv, res[1]);
  ring_resid<T, 2, 2>(D2, px0, py0, np, sv, res[2]);
  ring_resid<T, 1, 3>(D3, px0, py0, np, sv, res[3]);
  __syncthreads();
  if (t >= kTileCells) return;
  const int lj = D0.l[0];
  const int order[4] = {0, 1, 3, 2};
  T acc = 0;
#pragma unroll
  for (int oi = 0; oi < 4; oi++) acc += res[order[oi]][t];
  gc[q_of_m(jt, kc)] = acc;
#pragma unroll
  for (int c = 0; c < 4; c++) x[c * n4 + jt] = sv[c][lj];
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_add_range(int64_t begin, int64_t count, const T *__restrict__ delta,
                                                       T *__restrict__ x) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) x[begin + i] += delta[begin + i];
}

// residual of the four children of coarse cell M, summed in the order 0, 1, 3, 2 (Section 4.3's explicit
// restriction), written to the parent's color-major slot
template <class T>
__global__ void __launch_bounds__(kBlock) k_cres_restrict(QView<T> Q, const T *__restrict__ f,
                                                           const T *__restrict__ u, T *__restrict__ g) {
  const int64_t n4 = Q.n >> 2;
  const int64_t M = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (M >= n4) return;
  const int order[4] = {0, 1, 3, 2};
  T acc = 0;
#pragma unroll
  for (int oi = 0; oi < 4; oi++) {
    const int c = order[oi];
    const uint32_t q = static_cast<uint32_t>(c * n4 + M);
    acc += f[q] - row_apply(Q, q, c, u);
  }
  g[q_of_m(static_cast<uint32_t>(M), Q.k - 1)] = acc;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_cprolong(int k, int64_t n, const T *__restrict__ e, Pending<T> pend,
                                                      T *__restrict__ u) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n) return;
  // children of M are q = c n/4 + M: the parent's Morton index is q mod n/4
  const uint32_t M = static_cast<uint32_t>(q & ((n >> 2) - 1));
  const T em = pend.apply(e, q_of_m(M, k - 1));
  u[q] += em;
}

// y = A x on a quadtree level with two inner products (x, y) and (w, x); grid-stride, fixed grid
template <class T>
__global__ void __launch_bounds__(kBlock) k_cspmv_dot(QView<T> Q, const T *__restrict__ x, T *__restrict__ y,
                                                       const T *__restrict__ w, Red R) {
  double v[2] = {0.0, 0.0};
  for (int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; q < Q.n;
       q += static_cast<int64_t>(gridDim.x) * kBlock) {
    const T yq = row_apply(Q, static_cast<uint32_t>(q), row_color(static_cast<uint32_t>(q), 2 * Q.k - 2), x);
    y[q] = yq;
    const double xq = static_cast<double>(x[q]);
    v[0] += xq * static_cast<double>(yq);
    v[1] += static_cast<double>(w[q]) * xq;
  }
  reduce_finish<2>(v, R);
}

// the second inner step of Algorithm 2.1: A d with the direction d = p1 + beta p0 formed on the fly (never stored),
// inner products (d, A d) and (r, d)
template <class T>
__global__ void __launch_bounds__(kBlock) k_cspmv_dir(QView<T> Q, const double *__restrict__ sc,
                                                       const T *__restrict__ p1, const T *__restrict__ p0,
                                                       const T *__restrict__ r, Red R) {
  const T beta = static_cast<T>(sc[S_BETA]);
  auto dir = [p1, p0, beta](uint32_t i) { return p1[i] + beta * p0[i]; };
  double v[2] = {0.0, 0.0};
  for (int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; q < Q.n;
       q += static_cast<int64_t>(gridDim.x) * kBlock) {
    const uint32_t qu = static_cast<uint32_t>(q);
    const T yq = row_apply_f<T>(Q, qu, row_color(qu, 2 * Q.k - 2), dir);
    const double dq = static_cast<double>(dir(qu));
    v[0] += dq * static_cast<double>(yq);
    v[1] += static_cast<double>(r[q]) * dq;
  }
  reduce_finish<2>(v, R);
}

// ---------------------------------------------------------------------------------------------------------------
// octree (3D) level kernels: 27 slots, 8 colors, 8 children (numbering of qa_internal.hpp). Neighbour indices are
// recomputed from the row's grid coordinates; a neighbour outside the grid is replaced by the row itself (its slot
// holds 0), as on quadtree levels.

template <class T, class XV>
__device__ inline T row_apply3_f(const QView<T> &Q, uint32_t q, XV xv) {
  const uint32_t m = m_of_q3(q, Q.k);
  const int t1 = static_cast<int>(compact3(m)), t2 = static_cast<int>(compact3(m >> 1)),
            t3 = static_cast<int>(compact3(m >> 2));
  const int side = 1 << Q.k;
  T acc = 0;
#pragma unroll 9
  for (int s = 0; s < 27; s++) {
    const int u1 = t1 + slot3_dx(s), u2 = t2 + slot3_dy(s), u3 = t3 + slot3_dz(s);
    const bool in = u1 >= 0 && u2 >= 0 && u3 >= 0 && u1 < side && u2 < side && u3 < side;
    const uint32_t qn = in ? q_of_m3(morton3(static_cast<uint32_t>(u1), static_cast<uint32_t>(u2),
                                             static_cast<uint32_t>(u3)), Q.k)
                           : q;
    acc += Q.ax[s * Q.n + q] * xv(qn);
  }
  if (Q.optr)
    for (int32_t e = Q.optr[q]; e < Q.optr[q + 1]; e++) acc += Q.oval[e] * xv(static_cast<uint32_t>(Q.ocol[e]));
  return acc;
}

template <class T>
__device__ inline T row_apply3(const QView<T> &Q, uint32_t q, const T *__restrict__ x) {
  return row_apply3_f<T>(Q, q, [x](uint32_t i) { return x[i]; });
}

// one color phase of the pointwise 8-color Gauss-Seidel on an octree level (delta: see k_cgs)
template <class T>
__global__ void __launch_bounds__(kBlock) k_cgs3(QView<T> Q, const T *__restrict__ f, T *__restrict__ x,
                                                 T *__restrict__ delta, int c) {
  const int64_t n8 = Q.n >> 3;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n8) return;
  const uint32_t q = static_cast<uint32_t>(c * n8 + j);
  const T dl = (f[q] - row_apply3(Q, q, x)) / Q.ax[q];
  if (delta) delta[q] = dl;
  else x[q] += dl;
}

// One sweep of the eight color phases of a small octree level inside one workgroup: each row's arithmetic is
// k_cgs3's (and k_add_range's where cells of a color are coupled), the phases in the same order, with a barrier where
// the launches ended, so the result is theirs bit for bit.
constexpr int kOctSweepThreads = 1024;
constexpr int64_t kOctSweepMax = 8 * 2048;  // levels of at most this many cells sweep in one workgroup
template <class T, bool FWD, class Apply>
__device__ inline void oct_sweep(const QView<T> &Q, const T *__restrict__ f, T *x, T *delta, Apply apply) {
  const int64_t n8 = Q.n >> 3;
  for (int cc = 0; cc < 8; cc++) {
    const int c = FWD ? cc : 7 - cc;
    for (int64_t j = threadIdx.x; j < n8; j += kOctSweepThreads) {
      const uint32_t q = static_cast<uint32_t>(c * n8 + j);
      const T dl = (f[q] - apply(q, x)) / Q.ax[q];
      if (delta) delta[q] = dl;
      else x[q] += dl;
    }
    if (delta) {
      __syncthreads();
      for (int64_t j = threadIdx.x; j < n8; j += kOctSweepThreads) x[c * n8 + j] += delta[c * n8 + j];
    }
    __syncthreads();
  }
}

// the residual of coarse cell M's eight children, summed in child3_order (Section 4.3's restriction order on each
// layer), into the parent's color-major slot (k_cres_restrict3's row)
template <class T, class Apply>
__device__ inline void oct_restrict(const QView<T> &Q, const T *__restrict__ f, const T *u, T *gc, int64_t M,
                                    Apply apply) {
  const int64_t n8 = Q.n >> 3;
  T acc = 0;
  for (int o = 0; o < 8; o++) {
    const uint32_t q = static_cast<uint32_t>(child3_order(o) * n8 + M);
    acc += f[q] - apply(q, u);
  }
  gc[q_of_m3(static_cast<uint32_t>(M), Q.k - 1)] = acc;
}

// B^ of a small octree level (Algorithm 2.2) in one workgroup, its steps those of the per-step launches in their
// order with a barrier for each launch boundary: u = 0; `sweeps` forward sweeps; the restricted residual into gc;
// then, when the next level is the coarsest (whole), e_c = A_c^{-1} g_c with k_dense_solve's sums, u += P e_c and the
// backward sweeps. Without whole the kernel ends after the restriction (pre) or starts at the prolongation (post),
// and the next level's B~ runs between the two.
template <class T, int PART>  // PART 0: whole, 1: pre, 2: post
__global__ void __launch_bounds__(kOctSweepThreads) k_bhat3_small(QView<T> Q, const T *__restrict__ f, T *u, T *dl,
                                                                   T *gc, T *ec, const double *__restrict__ ainv,
                                                                   int nc, int sweeps) {
  __shared__ double sg[1024];
  const int64_t n = Q.n, n8 = n >> 3;
  const int tid = static_cast<int>(threadIdx.x);
  auto ap = [&Q](uint32_t q, const T *x) { return row_apply3(Q, q, x); };
  if (PART != 2) {
    for (int64_t q = tid; q < n; q += kOctSweepThreads) u[q] = T(0);
    __syncthreads();
    for (int sw = 0; sw < sweeps; sw++) oct_sweep<T, true>(Q, f, u, dl, ap);
    for (int64_t M = tid; M < n8; M += kOctSweepThreads) oct_restrict<T>(Q, f, u, gc, M, ap);
    if (PART == 1) return;
    __syncthreads();
    for (int i = tid; i < nc; i += kOctSweepThreads) sg[i] = static_cast<double>(gc[i]);
    __syncthreads();
    for (int i = tid; i < nc; i += kOctSweepThreads) {
      double acc = 0.0;
      for (int j = 0; j < nc; j++) acc += ainv[static_cast<size_t>(i) * nc + j] * sg[j];
      ec[i] = static_cast<T>(acc);
    }
    __syncthreads();
  }
  for (int64_t q = tid; q < n; q += kOctSweepThreads) u[q] += ec[q_of_m3(static_cast<uint32_t>(q & (n8 - 1)), Q.k - 1)];
  __syncthreads();
  for (int sw = 0; sw < sweeps; sw++) oct_sweep<T, false>(Q, f, u, dl, ap);
}

// residual of the eight children of coarse cell M, summed in child3_order (Section 4.3's restriction order on each
// layer), into the parent's color-major slot
template <class T>
__global__ void __launch_bounds__(kBlock) k_cres_restrict3(QView<T> Q, const T *__restrict__ f,
                                                           const T *__restrict__ u, T *__restrict__ gc) {
  const int64_t n8 = Q.n >> 3;
  const int64_t M = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (M >= n8) return;
  T acc = 0;
  for (int o = 0; o < 8; o++) {
    const uint32_t q = static_cast<uint32_t>(child3_order(o) * n8 + M);
    acc += f[q] - row_apply3(Q, q, u);
  }
  gc[q_of_m3(static_cast<uint32_t>(M), Q.k - 1)] = acc;
}

// The whole B^ of k_bhat3_small (PART 0) with the level's operator, u, f, the coarse vectors and a table of each row's
// 27 neighbours in LDS, made once: every step's gathers and operator values then come from LDS instead of L2, and
// no step recomputes the 3D neighbour rule (the overflow lists stay in global memory). The same steps, arithmetic and
// order as k_bhat3_small, so the same results bit for bit; u goes back to global memory at the end.
template <class T>
__global__ void __launch_bounds__(kOctSweepThreads) k_bhat3_lds(QView<T> Q, const T *__restrict__ f, T *u,
                                                                 const double *__restrict__ ainv, int nc, int sweeps,
                                                                 int use_delta) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t n = Q.n, n8 = n >> 3;
  const int tid = static_cast<int>(threadIdx.x);
  double *s_g = reinterpret_cast<double *>(smem);  // nc
  T *s_ax = reinterpret_cast<T *>(s_g + nc);       // 27 n
  T *s_u = s_ax + 27 * n, *s_f = s_u + n, *s_dl = s_f + n, *s_gt = s_dl + n, *s_e = s_gt + nc;
  uint16_t *s_nb = reinterpret_cast<uint16_t *>(s_e + nc);  // 27 n: row q's neighbour in slot s (q itself outside)
  for (int64_t i = tid; i < 27 * n; i += kOctSweepThreads) s_ax[i] = Q.ax[i];
  for (int64_t i = tid; i < n; i += kOctSweepThreads) {
    s_f[i] = f[i];
    s_u[i] = T(0);
    // the neighbour rule of row_apply3_f, once per row instead of once per row and step
    const uint32_t q = static_cast<uint32_t>(i), m = m_of_q3(q, Q.k);
    const int t1 = static_cast<int>(compact3(m)), t2 = static_cast<int>(compact3(m >> 1)),
              t3 = static_cast<int>(compact3(m >> 2));
    const int side = 1 << Q.k;
    for (int s = 0; s < 27; s++) {
      const int u1 = t1 + slot3_dx(s), u2 = t2 + slot3_dy(s), u3 = t3 + slot3_dz(s);
      const bool in = u1 >= 0 && u2 >= 0 && u3 >= 0 && u1 < side && u2 < side && u3 < side;
      s_nb[s * n + i] = static_cast<uint16_t>(
          in ? q_of_m3(morton3(static_cast<uint32_t>(u1), static_cast<uint32_t>(u2), static_cast<uint32_t>(u3)), Q.k)
             : q);
    }
  }
  __syncthreads();
  QView<T> QL = Q;
  QL.ax = s_ax;
  // row_apply3's sum (slots 0..26, then the overflow entries) with the neighbours from the table
  auto ap = [&](uint32_t q, const T *x) {
    T acc = 0;
    for (int s = 0; s < 27; s++) acc += s_ax[s * n + q] * x[s_nb[s * n + q]];
    if (Q.optr)
      for (int32_t e = Q.optr[q]; e < Q.optr[q + 1]; e++) acc += Q.oval[e] * x[static_cast<uint32_t>(Q.ocol[e])];
    return acc;
  };
  for (int sw = 0; sw < sweeps; sw++) oct_sweep<T, true>(QL, s_f, s_u, use_delta ? s_dl : nullptr, ap);
  for (int64_t M = tid; M < n8; M += kOctSweepThreads) oct_restrict<T>(QL, s_f, s_u, s_gt, M, ap);
  __syncthreads();
  for (int i = tid; i < nc; i += kOctSweepThreads) s_g[i] = static_cast<double>(s_gt[i]);
  __syncthreads();
  for (int i = tid; i < nc; i += kOctSweepThreads) {
    double acc = 0.0;
    for (int j = 0; j < nc; j++) acc += ainv[static_cast<size_t>(i) * nc + j] * s_g[j];
    s_e[i] = static_cast<T>(acc);
  }
  __syncthreads();
  for (int64_t q = tid; q < n; q += kOctSweepThreads)
    s_u[q] += s_e[q_of_m3(static_cast<uint32_t>(q & (n8 - 1)), Q.k - 1)];
  __syncthreads();
  for (int sw = 0; sw < sweeps; sw++) oct_sweep<T, false>(QL, s_f, s_u, use_delta ? s_dl : nullptr, ap);
  for (int64_t q = tid; q < n; q += kOctSweepThreads) u[q] = s_u[q];
}

template <class T>
static size_t bhat3_lds_bytes(int64_t n, int nc) {
  if (n > 65536) return SIZE_MAX;  // the neighbour table holds 16-bit rows
  return sizeof(double) * static_cast<size_t>(nc) + sizeof(T) * static_cast<size_t>(30 * n + 2 * nc) +
         sizeof(uint16_t) * static_cast<size_t>(27 * n);
}

// the LDS a launch of k_bhat3_lds may take on this device (set once per device: above 64 KB it must be asked for)
static int bhat3_lds_limit(int device) {
  static std::once_flag once[64];
  static int limit[64] = {};
  if (device < 0 || device >= 64) return 0;
  std::call_once(once[device], [&]() {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) return;
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(k_bhat3_lds<float>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void *>(k_bhat3_lds<double>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
      return;
    limit[device] = lds;
  });
  return limit[device];
}

// u += P e_c: row q = c 8^(k-1) + M takes its parent's value
template <class T>
__global__ void __launch_bounds__(kBlock) k_cprolong3(int k, int64_t n, const T *__restrict__ e, T *__restrict__ u) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= n) return;
  u[q] += e[q_of_m3(static_cast<uint32_t>(q & ((n >> 3) - 1)), k - 1)];
}

// y = A x on an octree level with (x, y) and (w, x)
template <class T>
__global__ void __launch_bounds__(kBlock) k_cspmv_dot3(QView<T> Q, const T *__restrict__ x, T *__restrict__ y,
                                                       const T *__restrict__ w, Red R) {
  double v[2] = {0.0, 0.0};
  for (int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; q < Q.n;
       q += static_cast<int64_t>(gridDim.x) * kBlock) {
    const T yq = row_apply3(Q, static_cast<uint32_t>(q), x);
    y[q] = yq;
    const double xq = static_cast<double>(x[q]);
    v[0] += xq * static_cast<double>(yq);
    v[1] += static_cast<double>(w[q]) * xq;
  }
  reduce_finish<2>(v, R);
}

// A d for d = p1 + beta p0 formed on the fly, with (d, A d) and (r, d)
template <class T>
__global__ void __launch_bounds__(kBlock) k_cspmv_dir3(QView<T> Q, const double *__restrict__ sc,
                                                       const T *__restrict__ p1, const T *__restrict__ p0,
                                                       const T *__restrict__ r, Red R) {
  const T beta = static_cast<T>(sc[S_BETA]);
  auto dir = [p1, p0, beta](uint32_t i) { return p1[i] + beta * p0[i]; };
  double v[2] = {0.0, 0.0};
  for (int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; q < Q.n;
       q += static_cast<int64_t>(gridDim.x) * kBlock) {
    const uint32_t qu = static_cast<uint32_t>(q);
    const T yq = row_apply3_f<T>(Q, qu, dir);
    const double dq = static_cast<double>(dir(qu));
    v[0] += dq * static_cast<double>(yq);
    v[1] += static_cast<double>(r[q]) * dq;
  }
  reduce_finish<2>(v, R);
}

// y = A x on an octree level (level hook)
template <class T>
__global__ void __launch_bounds__(kBlock) k_capply3(QView<T> Q, const T *__restrict__ x, T *__restrict__ y) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q < Q.n) y[q] = row_apply3(Q, static_cast<uint32_t>(q), x);
}

// ---------------------------------------------------------------------------------------------------------------
// vector kernels of Algorithm 2.1 (n = 2); scalars are read from device memory

template <class T>
__global__ void __launch_bounds__(kBlock) k_update1(int64_t n, const double *__restrict__ sc,
                                                     const T *__restrict__ p0, const T *__restrict__ q0,
                                                     const T *__restrict__ g, T *__restrict__ e, T *__restrict__ r) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T a = static_cast<T>(sc[S_A0]);
  e[i] = a * p0[i];
  r[i] = upd1_r(g[i], a, q0[i]);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_dot(int64_t n, const T *__restrict__ a, const T *__restrict__ b, Red R) {
  double v[1] = {0.0};
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    v[0] += static_cast<double>(a[i]) * static_cast<double>(b[i]);
  reduce_finish<1>(v, R);
}

// e += a1 (p1 + beta p0): the last update of Algorithm 2.1 with the direction formed on the fly
template <class T>
__global__ void __launch_bounds__(kBlock) k_update2(int64_t n, const double *__restrict__ sc, const T *__restrict__ p1,
                                                     const T *__restrict__ p0, T *__restrict__ e) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T a1 = static_cast<T>(sc[S_A1]), beta = static_cast<T>(sc[S_BETA]);
  e[i] += a1 * (p1[i] + beta * p0[i]);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_fill(int64_t n, T *__restrict__ v, T val) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) v[i] = val;
}

// e = A^{-1} g on the coarsest level (FP64 arithmetic whatever T is); one workgroup
template <class T>
__global__ void __launch_bounds__(kBlock) k_dense_solve(int n, const double *__restrict__ ainv,
                                                         const T *__restrict__ g, T *__restrict__ e) {
  __shared__ double sg[1024];
  for (int i = threadIdx.x; i < n; i += kBlock) sg[i] = static_cast<double>(g[i]);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kBlock) {
    double acc = 0.0;
    for (int j = 0; j < n; j++) acc += ainv[static_cast<size_t>(i) * n + j] * sg[j];
    e[i] = static_cast<T>(acc);
  }
}

// ---------------------------------------------------------------------------------------------------------------
// outer flexible CG kernels (FP64, permuted numbering)

// q = A p over all slices, with (p, q) and (r, p); one wavefront per slice
__global__ void __launch_bounds__(kBlock) k_outer_spmv_dot(SellView<double> S, SliceSched Z,
                                                            const double *__restrict__ p, double *__restrict__ q,
                                                            const double *__restrict__ r, Red R) {
  const int64_t s = sched_slice(Z);
  const int lane = threadIdx.x & 63;
  double v[2] = {0.0, 0.0};
  if (s >= 0) {
    if (S.row0[s] + lane < S.row0[s + 1]) {
      const int32_t row = S.srow[S.row0[s] + lane];
      const int64_t off = S.ptr[s];
      const int w = static_cast<int>((S.ptr[s + 1] - off) >> 6);
      const double acc = sell_row<double, double>(S, off, w, lane, p);
      q[row] = acc;
      v[0] = p[row] * acc;
      v[1] = r[row] * p[row];
    }
  }
  reduce_finish<2>(v, R);
}

// t = b - A x with (t, t)
__global__ void __launch_bounds__(kBlock) k_outer_true_resid(SellView<double> S, SliceSched Z,
                                                              const double *__restrict__ b,
                                                              const double *__restrict__ x, double *__restrict__ t,
                                                              Red R) {
  const int64_t s = sched_slice(Z);
  const int lane = threadIdx.x & 63;
  double v[1] = {0.0};
  if (s >= 0) {
    if (S.row0[s] + lane < S.row0[s + 1]) {
      const int32_t row = S.srow[S.row0[s] + lane];
      const int64_t off = S.ptr[s];
      const int w = static_cast<int>((S.ptr[s + 1] - off) >> 6);
      const double acc = sell_row<double, double>(S, off, w, lane, x);
      const double tr = b[row] - acc;
      t[row] = tr;
      v[0] = tr * tr;
    }
  }
  reduce_finish<1>(v, R);
}

// x += alpha p, r -= alpha q, with (r, r)
__global__ void __launch_bounds__(kBlock) k_outer_update(int64_t n, const double *__restrict__ sc,
                                                          const double *__restrict__ p, const double *__restrict__ q,
                                                          double *__restrict__ x, double *__restrict__ r, Red R) {
  const double a = sc[O_ALPHA];
  double v[1] = {0.0};
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    x[i] += a * p[i];
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    v[0] += ri * ri;
  }
  reduce_finish<1>(v, R);
}

// p = z + beta pprev (beta from the scalar block when use_beta)
template <class T>
__global__ void __launch_bounds__(kBlock) k_outer_dir(int64_t n, const double *__restrict__ sc,
                                                       const T *__restrict__ z, const double *__restrict__ pprev,
                                                       double *__restrict__ p, int use_beta) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double zi = static_cast<double>(z[i]);
  p[i] = use_beta ? zi + sc[O_BETA] * pprev[i] : zi;
}

// p = z + sum_j beta_j P_j over all m stored directions, beta_j = -(z, Q_j) / (P_j, Q_j) (Algorithm 2.1, Step 2, as
// written: z is orthogonalised against every earlier direction; the terms are added in order j = 0, 1, ...)
__global__ void __launch_bounds__(kBlock) k_outer_dir_all(int64_t n, const double *__restrict__ z,
                                                           const double *const *__restrict__ P,
                                                           const double *__restrict__ zq,
                                                           const double *__restrict__ d, int m,
                                                           double *__restrict__ p) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double pi = z[i];
  for (int j = 0; j < m; j++) pi += (-zq[j] / d[j]) * P[j][i];
  p[i] = pi;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_dot_mixed(int64_t n, const T *__restrict__ a, const double *__restrict__ b,
                                                       Red R) {
  double v[1] = {0.0};
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock)
    v[0] += static_cast<double>(a[i]) * b[i];
  reduce_finish<1>(v, R);
}

template <class S, class D>
__global__ void __launch_bounds__(kBlock) k_gather(int64_t n, const int32_t *__restrict__ perm,
                                                    const S *__restrict__ src, D *__restrict__ dst) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) dst[p] = static_cast<D>(src[perm[p]]);
}

template <class S, class D>
__global__ void __launch_bounds__(kBlock) k_scatter_back(int64_t n, const int32_t *__restrict__ perm,
                                                          const S *__restrict__ src, D *__restrict__ dst) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < n) dst[perm[p]] = static_cast<D>(src[p]);
}

template <class S, class D>
__global__ void __launch_bounds__(kBlock) k_cast(int64_t n, const S *__restrict__ src, D *__restrict__ dst) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = static_cast<D>(src[i]);
}

// lexicographic <-> color-major numbering of a quadtree level (tests and level hooks)
template <class S, class D>
__global__ void __launch_bounds__(kBlock) k_lex_to_q(int k, int64_t n, const S *__restrict__ src, D *__restrict__ dst,
                                                      int inverse, int dim = 2) {
  const int64_t I = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (I >= n) return;
  const uint32_t mask = (1u << k) - 1u, Iu = static_cast<uint32_t>(I);
  const uint32_t q = dim == 3 ? q_of_m3(morton3(Iu & mask, (Iu >> k) & mask, Iu >> (2 * k)), k)
                              : q_of_m(morton(Iu & mask, Iu >> k), k);
  if (inverse) dst[I] = static_cast<D>(src[q]);
  else dst[q] = static_cast<D>(src[I]);
}

// ---------------------------------------------------------------------------------------------------------------
// host orchestration

static inline unsigned nblk(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }
static inline unsigned nred(int64_t n) { return static_cast<unsigned>(std::min<int64_t>(nblk(n), kRedBlocksMax)); }

template <class T> struct P;
template <> struct P<double> {
  static std::vector<LevelWork<double>> &W(amg_hierarchy *h) { return h->w64; }
  static const double *ax(const QuadLevel &Q) { return Q.ax64; }
  static const double *oval(const QuadLevel &Q) { return Q.oval64; }
  static const double *sval(const FineLevel &F) { return F.s_val64; }
  static const double *diag(const FineLevel &F) { return F.diag64; }
  static const double *icv(const FineLevel &F) { return F.ic_val64; }
  static const double *bfac(const FineLevel &F) { return F.bfac64; }
  static constexpr int kResid = KK_RESID_FINE64, kGs = KK_GS_FINE64;
};
template <> struct P<float> {
  static std::vector<LevelWork<float>> &W(amg_hierarchy *h) { return h->w32; }
  static const float *ax(const QuadLevel &Q) { return Q.ax32; }
  static const float *oval(const QuadLevel &Q) { return Q.oval32; }
  static const float *sval(const FineLevel &F) { return F.s_val32; }
  static const float *diag(const FineLevel &F) { return F.diag32; }
  static const float *icv(const FineLevel &F) { return F.ic_val32; }
  static const float *bfac(const FineLevel &F) { return F.bfac32; }
  static constexpr int kResid = KK_RESID_FINE32, kGs = KK_GS_FINE32;
};

template <class T>
static QView<T> qview(const QuadLevel &Q) {
  return QView<T>{Q.k, Q.n, P<T>::ax(Q), Q.ovf_nnz ? Q.optr : nullptr, Q.ocol, P<T>::oval(Q)};
}
template <class T>
static SellView<T> sview(const FineLevel &F, const T *val) {
  return SellView<T>{F.slice_ptr, F.slice_row0, F.s_row, F.s_col, val};
}
static Red red(amg_hierarchy *h, int l, int epi, int slot = 0) {
  return Red{h->partials, h->scal + static_cast<size_t>(l) * kScalars, epi, slot};
}

// second stage of a multi-workgroup reduction (no-op for a single-workgroup launch)
template <int ND>
static void finish(amg_hierarchy *h, unsigned nb, const Red &R) {
  if (nb > 1) k_finish<ND><<<1, kBlock, 0, h->stream>>>(nb, R);
}

// Schedule of a fine-level pass over colors [c0, c1); the XCD-aware order from 256 slices (16,384 rows) up.
constexpr int64_t kMallBytes = int64_t(256) << 20;  // Infinity Cache

static SliceSched slice_sched(const FineLevel &F, int c0, int c1) {
  SliceSched Z{};
  for (int c = 0; c <= F.ncolor; c++) Z.cs[c] = F.color_slice[c];
  Z.c0 = c0;
  Z.c1 = c1;
  Z.xcd = (Z.cs[c1] - Z.cs[c0]) >= 256 ? 1 : 0;
  // a pass over several colors whose FP32 operands exceed the 256 MB Infinity Cache takes the colors in turns of
  // 16 slices (measured: the graded 4.0M-unknown mesh's full residual 74.5 -> 70.1 us; on operands the cache holds
  // the turns cost more than they save: 18.0 -> 20.3 us on the 1M-unknown mesh)
  const double fp32_bytes = 8.0 * static_cast<double>(F.nnz) + 12.0 * static_cast<double>(F.n);
  Z.ilv = (Z.xcd && c1 - c0 > 1 && fp32_bytes > static_cast<double>(kMallBytes)) ? 16 : 0;
  return Z;
}

// workgroups of a scheduled pass (4 slices each)
static unsigned sched_grid(const SliceSched &Z) {
  if (!Z.xcd) return static_cast<unsigned>((Z.cs[Z.c1] - Z.cs[Z.c0] + 3) / 4);
  int64_t most = 0;
  for (int64_t x = 0; x < 8; x++) {
    int64_t mine = 0;
    for (int c = Z.c0; c < Z.c1; c++) {
      const int64_t len = Z.cs[c + 1] - Z.cs[c];
      mine += len * (x + 1) / 8 - len * x / 8;
    }
    most = std::max(most, mine);
  }
  return static_cast<unsigned>(8 * ((most + 3) / 4));
}

// Launch `kern` on the hierarchy's stream with kBlock threads per workgroup. When its family is the one being timed,
// the launch goes through hipExtLaunchKernelGGL with a start/stop event pair: the runtime stamps both events from
// the dispatch packet itself, so the interval is the kernel's own execution window (the same span a kernel-trace
// profiler reports), not the gap between two markers queued around it.
template <typename F, typename... Args>
static void launch_timed_lds(amg_hierarchy *h, int kind, F kern, unsigned grid, size_t lds, Args... args) {
  Timing &t = h->timing;
  if (kind >= 0 && t.kind == kind && t.used + 2 <= t.ev.size()) {
    hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, h->stream, t.ev[t.used], t.ev[t.used + 1], 0,
                          args...);
    t.used += 2;
  } else {
    kern<<<grid, kBlock, lds, h->stream>>>(args...);
  }
}

template <class F, class... Args>
static void launch_timed(amg_hierarchy *h, int kind, F kern, unsigned grid, Args... args) {
  launch_timed_lds(h, kind, kern, grid, 0, args...);
}

// ---------------------------------------------------------------------------------------------------------------
// Persistent small-level engine. Below a size threshold the cycle is latency-bound: level k - j is visited 2^(j+1)
// times per outer iteration, each visit a chain of ~10 dependent steps on a few thousand rows. One workgroup runs
// B~ of the engine's top level and everything below it (B^, restriction, prolongation, the inner nonlinear PCG,
// the coarsest solve) in a single launch. The host emits the step list of that recursion once per hierarchy; the
// workgroup interprets it with a barrier after every step. Levels below the top keep operators and vectors in
// LDS; the top level stays in global memory when it does not fit. Inner products are workgroup reductions in
// double with a fixed tree.

constexpr int kEngThreads = 1024;
constexpr int kEngWaves = kEngThreads / 64;
constexpr int kEngMaxLevels = 8;
constexpr int kEngMaxOps = 512;  // step list staged in LDS (24 bytes each)
constexpr int kEngRows = 4;      // rows per thread whose loads an SpMV step issues together

enum EngOpType : int32_t {
  EO_GS_FIRST = 0, EO_GS, EO_RES_RESTRICT, EO_DENSE, EO_PROLONG, EO_SPMV_DOT0, EO_UPDATE1, EO_DOT_BETA,
  EO_AXPY_BETA, EO_SPMV_DOT1, EO_UPDATE2, EO_BHAT_M, EO_GS_FIRST2
};
// engine scalars of a level (8 per level)
enum EngScalar : int { ES_D0 = 0, ES_A0 = 2, ES_STOP = 3, ES_BETA = 5, ES_A1 = 6 };
constexpr int kMhatMaxRows = 256;   // B^ kept as a matrix when the level above the coarsest has at most this many rows
constexpr int kMhatPart = 4096;     // LDS partial sums of the matrix-vector product (T units)
enum EngVec : int32_t { EV_G = 0, EV_E, EV_R, EV_P0, EV_Q0, EV_P1, EV_Q1, EV_D, EV_COUNT };

struct EngOp {
  int32_t type, lvl, color, f, u;  // f, u: vector slots of level lvl
  int32_t fuse;                    // EngFuse bits
};
// Steps folded into their neighbours in the step list of B~ (each value equal to what the separate step stores):
// FUSE_UPD1 on the first step of the second B^: the update e = a0 p0, r = g - a0 q0 is written there, and that
// step reads its right-hand side r as g - a0 q0 formed on the fly; FUSE_BETA on the last step of that B^: the inner
// product (p1, q0) and beta are formed after a barrier at its end.
enum EngFuse : int32_t { FUSE_UPD1 = 1, FUSE_BETA = 2 };

template <class T>
struct EngLevel {
  int k, n;
  int in_lds;
  const T *ax;                 // global 9 x n
  const int32_t *optr, *ocol;  // overflow in global (null when none)
  const T *oval;
  int same_color;
  int ax_off, vec_off;         // LDS offsets (T units) of the 9 x n operator and of the vectors when in_lds
  T *vec[EV_COUNT];            // global vectors when not in LDS
  // a level run from global memory may still hold some of its work vectors in LDS: the vectors whose bits are set
  // lie at vec_off, one after another in slot order, and the workgroup points vec[] at them when it starts
  int lvec_mask;
};

template <class T>
struct EngPlan {
  int nlev, nops, nc, ainv_in_lds;
  int t_base;                  // byte offset of the T arrays in dynamic LDS
  const EngOp *ops;
  const double *ainv;
  const T *g_in;
  T *e_out;
  int64_t batch_stride;        // workgroup b reads g_in + b * stride, writes e_out + b * stride (0: one system)
  const T *mhat;               // B^ of the level above the coarsest, column-major (EO_BHAT_M), or null
  int mhat_parts;              // threads per row of its product
  int mpart_off;               // LDS offset (T units) of the partial sums
  EngLevel<T> lv[kEngMaxLevels];
};

template <int ND>
__device__ inline void eng_reduce(double (&v)[ND], double *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int j = 0; j < ND; j++) v[j] += __shfl_down(v[j], off, 64);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int j = 0; j < ND; j++) red[j * kEngWaves + (threadIdx.x >> 6)] = v[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ND; j++) {
    double acc = 0.0;
#pragma unroll
    for (int w = 0; w < kEngWaves; w++) acc += red[j * kEngWaves + w];
    v[j] = acc;  // every thread sums the same values in the same order
  }
}

// The same sum delivered to thread 0 only, for steps whose result thread 0 stores: waves at or past `waves` hold
// zeros (their threads had no rows) and skip the shuffles, and one thread adds the wave sums, so the waves that do
// the work do not share their SIMDs with idle ones. The sum equals eng_reduce's (adding zeros changes nothing).
template <int ND>
__device__ inline void eng_reduce_t0(double (&v)[ND], double *red, int waves) {
  if (static_cast<int>(threadIdx.x >> 6) < waves) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int j = 0; j < ND; j++) v[j] += __shfl_down(v[j], off, 64);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int j = 0; j < ND; j++) red[j * kEngWaves + (threadIdx.x >> 6)] = v[j];
  }
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < ND; j++) {
      double acc = 0.0;
      for (int w = 0; w < waves; w++) acc += red[j * kEngWaves + w];
      v[j] = acc;
    }
}

// waves of the workgroup that hold rows of an n-row level (threads tid < n)
__device__ inline int eng_waves(int n) {
  return n >= kEngThreads ? kEngWaves : (n + 63) >> 6;
}

// (A x)_q on an engine level, x given by a function of the index (a stored vector, or values formed on the fly)
template <class T, class XV>
__device__ __forceinline__ T eng_row_f(int k, int n, const T *ax, const int32_t *optr, const int32_t *ocol, const T *oval,
                              uint32_t q, int c, XV xv) {
  const int sh = 2 * k - 2;
  uint32_t nb[9];
  stencil_q(q, q & ((1u << sh) - 1u), c, sh, nb);
  T acc = 0;
#pragma unroll
  for (int s = 0; s < 9; s++) acc += ax[s * n + q] * xv(nb[s]);  // absent slots hold 0
  if (optr)
    for (int32_t e = optr[q]; e < optr[q + 1]; e++) acc += oval[e] * xv(static_cast<uint32_t>(ocol[e]));
  return acc;
}

template <class T>
__device__ __forceinline__ T eng_row(int k, int n, const T *ax, const int32_t *optr, const int32_t *ocol, const T *oval,
                            uint32_t q, int c, const T *x) {
  return eng_row_f<T>(k, n, ax, optr, ocol, oval, q, c, [x](uint32_t i) { return x[i]; });
}

// Vector and operator access of one engine level: LDS levels are addressed as offsets into the dynamic shared
// array (so the compiler emits LDS instructions), the global top level through its device pointers.
template <class T, bool LDS>
struct EngMem {
  T *S;
  const EngLevel<T> &L;
  __device__ T *vec(int v) const { return LDS ? S + L.vec_off + v * L.n : L.vec[v]; }
  __device__ const T *ax() const { return LDS ? S + L.ax_off : L.ax; }
};

struct EngCtx {
  double *sc;       // this level's scalars
  double *sc_child; // the next coarser level's scalars
  double *red;
};

// the first inner update of Algorithm 2.1 on an engine level, as a value source (r) and a store of e and r
template <class T, bool LDS>
struct EngUpd1 {
  T a0;
  const T *g, *q0, *p0;
  T *e, *r;
  __device__ EngUpd1(const EngMem<T, LDS> &M, const EngCtx &C)
      : a0(static_cast<T>(C.sc[ES_A0])), g(M.vec(EV_G)), q0(M.vec(EV_Q0)), p0(M.vec(EV_P0)), e(M.vec(EV_E)),
        r(M.vec(EV_R)) {}
  __device__ T rv(uint32_t i) const { return upd1_r(g[i], a0, q0[i]); }
  __device__ void store(int i) const {
    e[i] = a0 * p0[i];
    r[i] = upd1_r(g[i], a0, q0[i]);
  }
};

// beta = -(p1, q0) / d0 of Algorithm 2.1 (every thread calls it; the reduction tree is fixed)
template <class T, bool LDS>
__device__ __forceinline__ void eng_dot_beta(const EngMem<T, LDS> &M, int n, const EngCtx &C) {
  const T *p1 = M.vec(EV_P1), *q0 = M.vec(EV_Q0);
  double t[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += kEngThreads) t[0] += static_cast<double>(p1[i]) * static_cast<double>(q0[i]);
  eng_reduce_t0<1>(t, C.red, eng_waves(n));
  if (threadIdx.x == 0) C.sc[ES_BETA] = (C.sc[ES_STOP] != 0.0) ? 0.0 : -t[0] / C.sc[ES_D0];
}

// the first two phases of a sweep from zero (levels without same-color couplings): color 0 takes u = f / diag, and
// the color-1 rows read those values formed on the fly (colors 2 and 3 are still 0); no thread reads u here, so
// the writes of colors 0, 2 and 3 go alongside. `each` runs once per row (the folded first inner update).
template <class T, class FV, class EACH>
__device__ __forceinline__ void eng_gs_first2(const EngLevel<T> &L, int k, int n, const T *ax, T *u, FV fv,
                                              EACH each) {
  const int tid = static_cast<int>(threadIdx.x);
  const int n4 = n >> 2;
  const uint32_t n4u = static_cast<uint32_t>(n4);
  auto first = [fv, ax, n4u](uint32_t i) { return i < n4u ? fv(i) / ax[i] : T(0); };
  for (int j = tid; j < n4; j += kEngThreads) {
    const uint32_t q = static_cast<uint32_t>(n4 + j);
    u[q] = T(0) + (fv(q) - eng_row_f<T>(k, n, ax, L.optr, L.ocol, L.oval, q, 1, first)) / ax[q];
  }
  for (int q = tid; q < n; q += kEngThreads) {
    if (q < n4) u[q] = fv(static_cast<uint32_t>(q)) / ax[q];
    else if (q >= 2 * n4) u[q] = T(0);
    each(q);
  }
}

// u = B^ f with B^ precomputed as a matrix (column-major, global memory). A thread owns four consecutive rows
// (one 16-byte load per column in FP32, two in FP64) for a run of columns; the workgroup splits the columns into
// mhat_parts runs, and the partial sums of a row are added in a fixed order.
template <class T, class FV, class EACH>
__device__ __forceinline__ void eng_bhat_m(const EngPlan<T> &P, int n, T *S, T *u, FV fv, EACH each) {
  const int tid = static_cast<int>(threadIdx.x);
  T *part = S + P.mpart_off;
  const int groups = n >> 2;
  const int parts = P.mhat_parts;
  const int cols = n / parts;
  if (tid < groups * parts) {
    const int g = tid % groups;
    const int b = tid / groups;
    const T *mc = P.mhat + static_cast<size_t>(b) * cols * n + 4 * g;
    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int i = 0; i < cols; i++) {
      const T *col = mc + static_cast<size_t>(i) * n;
      const T fi = fv(static_cast<uint32_t>(b * cols + i));
      if constexpr (std::is_same<T, float>::value) {
        const float4 v = *reinterpret_cast<const float4 *>(col);
        a0 += v.x * fi; a1 += v.y * fi; a2 += v.z * fi; a3 += v.w * fi;
      } else {
        const double2 v0 = *reinterpret_cast<const double2 *>(col);
        const double2 v1 = *reinterpret_cast<const double2 *>(col + 2);
        a0 += v0.x * fi; a1 += v0.y * fi; a2 += v1.x * fi; a3 += v1.y * fi;
      }
    }
    T *pb = part + b * n + 4 * g;
    pb[0] = a0; pb[1] = a1; pb[2] = a2; pb[3] = a3;
  }
  __syncthreads();
  for (int r = tid; r < n; r += kEngThreads) {
    T acc = part[r];
    for (int b = 1; b < parts; b++) acc += part[b * n + r];
    u[r] = acc;
    each(r);
  }
}

// One step of the interpreter, run by the whole workgroup. LDS / LDS_CHILD: where this level's and its child's
// vectors live.
template <class T, bool LDS, bool LDS_CHILD>
__device__ __forceinline__ void eng_step(const EngOp &op, const EngLevel<T> *LV, const EngPlan<T> &P, T *S,
                                const double *Ainv, EngCtx C) {
  constexpr int kStride = kEngThreads;
  const int tid = static_cast<int>(threadIdx.x);
  const int l = op.lvl;
  const EngLevel<T> &L = LV[l];
  const EngMem<T, LDS> M{S, L};
  const int k = L.k, n = L.n, n4 = n >> 2;
  const T *ax = M.ax();
  switch (op.type) {
    case EO_GS_FIRST: {
      T *u = M.vec(op.u);
      if (op.fuse & FUSE_UPD1) {
        const EngUpd1<T, LDS> U(M, C);
        for (int q = tid; q < n; q += kStride) {
          u[q] = (q < n4) ? U.rv(static_cast<uint32_t>(q)) / ax[q] : T(0);
          U.store(q);
        }
      } else {
        const T *f = M.vec(op.f);
        for (int q = tid; q < n; q += kStride) u[q] = (q < n4) ? f[q] / ax[q] : T(0);
      }
      break;
    }
    case EO_GS_FIRST2: {
      T *u = M.vec(op.u);
      if (op.fuse & FUSE_UPD1) {
        const EngUpd1<T, LDS> U(M, C);
        eng_gs_first2<T>(L, k, n, ax, u, [U](uint32_t i) { return U.rv(i); }, [U](int i) { U.store(i); });
      } else {
        const T *f = M.vec(op.f);
        eng_gs_first2<T>(L, k, n, ax, u, [f](uint32_t i) { return f[i]; }, [](int) {});
      }
      break;
    }
    case EO_GS: {
      const T *f = M.vec(op.f);
      T *u = M.vec(op.u);
      T *d = M.vec(EV_D);
      const int c = __builtin_amdgcn_readfirstlane(op.color);
      for (int j = tid; j < n4; j += kStride) {
        const uint32_t q = static_cast<uint32_t>(c * n4 + j);
        const T dl = (f[q] - eng_row(k, n, ax, L.optr, L.ocol, L.oval, q, c, u)) / ax[q];
        if (L.same_color) d[q] = dl;
        else u[q] += dl;
      }
      if (L.same_color) {
        __syncthreads();
        for (int j = tid; j < n4; j += kStride) u[c * n4 + j] += d[c * n4 + j];
      }
      if (op.fuse & FUSE_BETA) {
        __syncthreads();
        eng_dot_beta<T, LDS>(M, n, C);
      }
      break;
    }
    case EO_RES_RESTRICT: {
      const T *f = M.vec(op.f);
      const T *u = M.vec(op.u);
      const EngMem<T, LDS_CHILD> MC{S, LV[l + 1]};
      T *gc = MC.vec(EV_G);
      const int order[4] = {0, 1, 3, 2};
      for (int m = tid; m < n4; m += kStride) {
        T r[4];
#pragma unroll
        for (int o = 0; o < 4; o++) {
          const uint32_t q = static_cast<uint32_t>(order[o] * n4 + m);
          r[o] = f[q] - eng_row(k, n, ax, L.optr, L.ocol, L.oval, q, order[o], u);
        }
        T acc = 0;
#pragma unroll
        for (int o = 0; o < 4; o++) acc += r[o];
        gc[q_of_m(static_cast<uint32_t>(m), k - 1)] = acc;
      }
      break;
    }
    case EO_DENSE: {
      // 16 threads per row: strided partial sums, then a fixed butterfly over the 16 lanes
      const T *g = M.vec(EV_G);
      T *e = M.vec(EV_E);
      const int part = tid & 15;
      for (int i0 = 0; i0 < P.nc; i0 += kStride / 16) {
        const int i = i0 + (tid >> 4);
        double acc = 0.0;
        if (i < P.nc)
          for (int j = part; j < P.nc; j += 16) acc += Ainv[i * P.nc + j] * static_cast<double>(g[j]);
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
        if (i < P.nc && part == 0) e[i] = static_cast<T>(acc);
      }
      break;
    }
    case EO_BHAT_M: {
      T *u = M.vec(op.u);
      if (op.fuse & FUSE_UPD1) {
        const EngUpd1<T, LDS> U(M, C);
        eng_bhat_m<T>(P, n, S, u, [U](uint32_t i) { return U.rv(i); }, [U](int i) { U.store(i); });
      } else {
        const T *f = M.vec(op.f);
        eng_bhat_m<T>(P, n, S, u, [f](uint32_t i) { return f[i]; }, [](int) {});
      }
      if (op.fuse & FUSE_BETA) {
        __syncthreads();
        eng_dot_beta<T, LDS>(M, n, C);
      }
      break;
    }
    case EO_PROLONG: {
      // u += P e_c; with op.color = 1 the child's last update e_c += a1 (p1 + beta p0) (UPDATE2, deferred) is
      // formed here, value for value as that step would have stored it
      T *u = M.vec(op.u);
      const EngMem<T, LDS_CHILD> MC{S, LV[l + 1]};
      const T *ec = MC.vec(EV_E);
      if (op.color) {
        const T a1 = static_cast<T>(C.sc_child[ES_A1]), beta = static_cast<T>(C.sc_child[ES_BETA]);
        const T *p1c = MC.vec(EV_P1), *p0c = MC.vec(EV_P0);
        for (int q = tid; q < n; q += kStride) {
          const uint32_t m = q_of_m(static_cast<uint32_t>(q & (n4 - 1)), k - 1);
          const T ecm = ec[m] + a1 * (p1c[m] + beta * p0c[m]);
          u[q] += ecm;
        }
      } else {
        for (int q = tid; q < n; q += kStride) u[q] += ec[q_of_m(static_cast<uint32_t>(q & (n4 - 1)), k - 1)];
      }
      break;
    }
    case EO_SPMV_DOT0: {
      const T *x = M.vec(EV_P0);
      T *y = M.vec(EV_Q0);
      const T *w = M.vec(EV_G);
      double v[2] = {0.0, 0.0};
      // a thread's rows (up to kEngRows per pass) are all loaded before any is stored, so their loads overlap
      for (int q0 = tid; q0 < n; q0 += kEngRows * kStride) {
        T yq[kEngRows];
#pragma unroll
        for (int r = 0; r < kEngRows; r++) {
          const int q = q0 + r * kStride;
          if (q < n)
            yq[r] = eng_row(k, n, ax, L.optr, L.ocol, L.oval, static_cast<uint32_t>(q),
                            row_color(static_cast<uint32_t>(q), 2 * k - 2), x);
        }
#pragma unroll
        for (int r = 0; r < kEngRows; r++) {
          const int q = q0 + r * kStride;
          if (q < n) {
            y[q] = yq[r];
            v[0] += static_cast<double>(x[q]) * static_cast<double>(yq[r]);
            v[1] += static_cast<double>(w[q]) * static_cast<double>(x[q]);
          }
        }
      }
      eng_reduce_t0<2>(v, C.red, eng_waves(n));
      if (tid == 0) {
        const bool stop = !(v[0] > 0.0);
        C.sc[ES_D0] = v[0];
        C.sc[ES_STOP] = stop ? 1.0 : 0.0;
        C.sc[ES_A0] = stop ? 0.0 : v[1] / v[0];
      }
      break;
    }
    case EO_SPMV_DOT1: {
      // A p1 with the direction update p1 + beta p0 formed on the fly (it is never stored: UPDATE2 forms it too);
      // only the two inner products are kept
      const T beta = static_cast<T>(C.sc[ES_BETA]);
      const T *p1 = M.vec(EV_P1), *p0 = M.vec(EV_P0);
      const T *w = M.vec(EV_R);
      auto dir = [p1, p0, beta](uint32_t i) { return p1[i] + beta * p0[i]; };
      double v[2] = {0.0, 0.0};
      for (int q0 = tid; q0 < n; q0 += kEngRows * kStride) {
        T yq[kEngRows], xq[kEngRows], wq[kEngRows];
#pragma unroll
        for (int r = 0; r < kEngRows; r++) {
          const int q = q0 + r * kStride;
          if (q < n) {
            yq[r] = eng_row_f<T>(k, n, ax, L.optr, L.ocol, L.oval, static_cast<uint32_t>(q),
                                 row_color(static_cast<uint32_t>(q), 2 * k - 2), dir);
            xq[r] = dir(static_cast<uint32_t>(q));
            wq[r] = w[q];
          }
        }
#pragma unroll
        for (int r = 0; r < kEngRows; r++)
          if (q0 + r * kStride < n) {
            v[0] += static_cast<double>(xq[r]) * static_cast<double>(yq[r]);
            v[1] += static_cast<double>(wq[r]) * static_cast<double>(xq[r]);
          }
      }
      eng_reduce_t0<2>(v, C.red, eng_waves(n));
      if (tid == 0) C.sc[ES_A1] = (C.sc[ES_STOP] != 0.0 || !(v[0] > 0.0)) ? 0.0 : v[1] / v[0];
      break;
    }
    case EO_UPDATE1: {
      const EngUpd1<T, LDS> U(M, C);
      for (int i = tid; i < n; i += kStride) U.store(i);
      break;
    }
    case EO_DOT_BETA:
      eng_dot_beta<T, LDS>(M, n, C);
      break;
    case EO_UPDATE2: {
      const T a1 = static_cast<T>(C.sc[ES_A1]), beta = static_cast<T>(C.sc[ES_BETA]);
      const T *p1 = M.vec(EV_P1), *p0 = M.vec(EV_P0);
      T *e = M.vec(EV_E);
      for (int i = tid; i < n; i += kStride) e[i] += a1 * (p1[i] + beta * p0[i]);
      break;
    }
    default:
      break;
  }
}

// Interpret a step list (operators and step list already staged in LDS).
template <class T>
__device__ __forceinline__ void eng_run(const EngPlan<T> &P, const EngOp *ops, const EngLevel<T> *LV, T *S,
                               const double *Ainv, double (*sc)[8], double *red) {
  for (int oi = 0; oi < P.nops; oi++) {
    const EngOp op = ops[oi];
    const EngCtx C{sc[op.lvl], sc[op.lvl + 1 < kEngMaxLevels ? op.lvl + 1 : op.lvl], red};
    const bool lds = LV[op.lvl].in_lds != 0;
    const bool lds_child = (op.lvl + 1 < P.nlev) && LV[op.lvl + 1].in_lds != 0;
    if (lds) eng_step<T, true, true>(op, LV, P, S, Ainv, C);
    else if (lds_child) eng_step<T, false, true>(op, LV, P, S, Ainv, C);
    else eng_step<T, false, false>(op, LV, P, S, Ainv, C);
    __syncthreads();
  }
}

// Copy the step list, level table, coarsest inverse and LDS-resident operators into LDS.
template <class T>
__device__ inline void eng_stage(const EngPlan<T> &P, EngOp *ops, EngLevel<T> *LV, T *S, double *ainv_lds) {
  const int tid = threadIdx.x;
  for (int i = tid; i < P.nops; i += kEngThreads) ops[i] = P.ops[i];
  if (tid < P.nlev) {
    EngLevel<T> L = P.lv[tid];
    for (int v = 0, j = 0; v < EV_COUNT; v++)
      if ((L.lvec_mask >> v) & 1) L.vec[v] = S + L.vec_off + (j++) * L.n;
    LV[tid] = L;
  }
  if (P.ainv_in_lds)
    for (int i = tid; i < P.nc * P.nc; i += kEngThreads) ainv_lds[i] = P.ainv[i];
  for (int l = 0; l < P.nlev; l++) {
    const EngLevel<T> &L = P.lv[l];
    if (L.in_lds && l + 1 < P.nlev)
      for (int i = tid; i < 9 * L.n; i += kEngThreads) S[L.ax_off + i] = L.ax[i];
  }
}

template <class T>
__global__ void __launch_bounds__(kEngThreads) k_engine(EngPlan<T> P) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sc[kEngMaxLevels][8];
  __shared__ double red[2 * kEngWaves];
  __shared__ EngOp ops[kEngMaxOps];
  __shared__ EngLevel<T> LV[kEngMaxLevels];
  const int tid = threadIdx.x;
  T *S = reinterpret_cast<T *>(smem + P.t_base);
  double *ainv_lds = reinterpret_cast<double *>(smem);
  const T *g_in = P.g_in + blockIdx.x * P.batch_stride;
  T *e_out = P.e_out + blockIdx.x * P.batch_stride;
  eng_stage(P, ops, LV, S, ainv_lds);
  if (P.lv[0].in_lds)
    for (int i = tid; i < P.lv[0].n; i += kEngThreads) S[P.lv[0].vec_off + EV_G * P.lv[0].n + i] = g_in[i];
  __syncthreads();
  eng_run(P, ops, LV, S, P.ainv_in_lds ? ainv_lds : P.ainv, sc, red);
  if (P.lv[0].in_lds)
    for (int i = tid; i < P.lv[0].n; i += kEngThreads) e_out[i] = S[P.lv[0].vec_off + EV_E * P.lv[0].n + i];
}

// Step list of B~ at engine level l; mirrors btilde / bhat_coarse below.
struct EmitCtx {
  int nl, sweeps, inner;
  int mhat;               // B^ of the level above the coarsest is one EO_BHAT_M step
  const int *same_color;  // per engine level: some coupling joins two cells of one color
};

static void emit_btilde(std::vector<EngOp> &ops, const EmitCtx &E, int l, bool defer_update2);

// B^ of Algorithm 2.2 on engine level l (f, u: vector slots). The first two phases of the first sweep are one step
// where no coupling joins cells of one color; with a second inner iteration below, the child's last update is
// folded into this level's prolongation.
static void emit_bhat(std::vector<EngOp> &ops, const EmitCtx &E, int l, int f, int u) {
  if (E.mhat && l + 1 == E.nl - 1) {
    ops.push_back({EO_BHAT_M, l, 0, f, u});
    return;
  }
  for (int sw = 0; sw < E.sweeps; sw++)
    for (int c = 0; c < 4; c++) {
      if (sw == 0 && c == 0 && !E.same_color[l]) {
        ops.push_back({EO_GS_FIRST2, l, 1, f, u});
        c = 1;
      } else {
        ops.push_back({(sw == 0 && c == 0) ? EO_GS_FIRST : EO_GS, l, c, f, u});
      }
    }
  ops.push_back({EO_RES_RESTRICT, l, 0, f, u});
  const bool defer = l + 1 < E.nl - 1 && E.inner >= 2;
  if (l + 1 == E.nl - 1) ops.push_back({EO_DENSE, l + 1, 0, 0, 0});
  else emit_btilde(ops, E, l + 1, defer);
  ops.push_back({EO_PROLONG, l, defer ? 1 : 0, f, u});
  for (int sw = 0; sw < E.sweeps; sw++)
    for (int c = 3; c >= 0; c--) ops.push_back({EO_GS, l, c, f, u});
}

// B~ of Algorithm 2.1 with n = inner iterations on engine level l
static void emit_btilde(std::vector<EngOp> &ops, const EmitCtx &E, int l, bool defer_update2) {
  emit_bhat(ops, E, l, EV_G, EV_P0);
  ops.push_back({EO_SPMV_DOT0, l, 0, 0, 0});
  if (E.inner < 2) {
    ops.push_back({EO_UPDATE1, l, 0, 0, 0});
    return;
  }
  // the update folds into the first step of the second B^ and the inner product for beta into its last, when those
  // are steps on this level that take the fold (a relaxation from zero or the B^ matrix; a color phase or the B^
  // matrix)
  const size_t first = ops.size();
  emit_bhat(ops, E, l, EV_R, EV_P1);
  EngOp &a = ops[first];
  if (a.lvl == l && (a.type == EO_GS_FIRST || a.type == EO_GS_FIRST2 || a.type == EO_BHAT_M)) {
    a.fuse |= FUSE_UPD1;
  } else {
    ops.insert(ops.begin() + static_cast<std::ptrdiff_t>(first), EngOp{EO_UPDATE1, l, 0, 0, 0, 0});
  }
  EngOp &z = ops.back();
  if (z.lvl == l && (z.type == EO_GS || z.type == EO_BHAT_M)) z.fuse |= FUSE_BETA;
  else ops.push_back({EO_DOT_BETA, l, 0, 0, 0});
  ops.push_back({EO_SPMV_DOT1, l, 0, 0, 0});
  if (!defer_update2) ops.push_back({EO_UPDATE2, l, 0, 0, 0});
}

// same-color flags of the levels from `top` down, indexed from 0
static std::vector<int> same_color_from(const amg_hierarchy *h, int top) {
  std::vector<int> v;
  for (int l = top; l < h->nlev; l++) v.push_back(l >= 1 ? h->lev[l].same_color_ovf : 0);
  return v;
}

template <class T> struct WgSys;
template <class T> __global__ void k_solve_wg(const WgSys<T> *systems);

// Dynamic LDS limit of the persistent kernels: set once per device, to all the device allows beside their static
// arrays, so that hierarchies set up concurrently on several host threads never lower it under one another's launch.
static amg_status engine_lds_limits(amg_hierarchy *h) {
  static std::once_flag once[64];
  if (h->device < 0 || h->device >= 64) return AMG_ERR_DEVICE;
  amg_status st = AMG_OK;
  std::call_once(once[h->device], [&]() {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) != hipSuccess) {
      st = AMG_ERR_DEVICE;
      return;
    }
    const int dyn = lds - static_cast<int>(sizeof(EngOp) * kEngMaxOps + 4096);
    const void *kernels[4] = {reinterpret_cast<const void *>(k_engine<double>),
                              reinterpret_cast<const void *>(k_engine<float>),
                              reinterpret_cast<const void *>(k_solve_wg<double>),
                              reinterpret_cast<const void *>(k_solve_wg<float>)};
    for (const void *k : kernels)
      if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn) != hipSuccess) st = AMG_ERR_DEVICE;
  });
  return st;
}

// Algorithmic floating-point operations of one launch of a step list whose level 0 is hierarchy level `top`: each
// add, multiply or divide counts one (a fused multiply-add two), once per value the step defines, whatever the
// kernel recomputes on the fly. A nine-slot row is 18.
static double engine_flops(const amg_hierarchy *h, int top, const std::vector<EngOp> &ops) {
  double f = 0.0;
  for (const EngOp &op : ops) {
    const double n = static_cast<double>(h->lev[top + op.lvl].n), n4 = n / 4;
    switch (op.type) {
      case EO_GS_FIRST: f += n4; break;                           // u = f / a on color 0
      case EO_GS_FIRST2: f += n4 + n4 * 20; break;                // color 0, then color 1 against it
      case EO_GS: f += n4 * 21; break;                            // f - A u, / a, +
      case EO_RES_RESTRICT: f += n * 19 + n; break;               // f - A u, four children summed
      case EO_DENSE: f += 2.0 * static_cast<double>(h->nc) * static_cast<double>(h->nc); break;
      case EO_BHAT_M: f += 2.0 * n * n; break;
      case EO_PROLONG: f += op.color ? 5 * n : n; break;          // with the child's deferred update: 4 more
      case EO_SPMV_DOT0: f += n * 18 + 4 * n; break;
      case EO_SPMV_DOT1: f += 2 * n + n * 18 + 4 * n; break;      // direction, A d, two inner products
      case EO_UPDATE1: f += 3 * n; break;
      case EO_DOT_BETA: f += 2 * n; break;
      case EO_UPDATE2: f += 4 * n; break;
      default: break;
    }
    if (op.fuse & FUSE_UPD1) f += 3 * n;
    if (op.fuse & FUSE_BETA) f += 2 * n;
  }
  return f;
}

amg_status plan_engine(amg_hierarchy *h) {
  h->engine_top[0] = h->engine_top[1] = -1;
  // nothing between the fine level and the coarsest; octree levels run per step
  if (h->nlev < 3 || h->dim != 2) return AMG_OK;
  int lds = 0;
  QA_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
  h->lds_max = static_cast<size_t>(lds);
  // room for the static shared arrays (step list, pointer tables, scalars)
  const size_t stat = sizeof(EngOp) * kEngMaxOps + 4096;
  const size_t budget = h->lds_max > stat ? h->lds_max - stat : 0;
  const int mhat = h->mhat_level >= 0 ? 1 : 0;
  for (int pi = 0; pi < 2; pi++) {
    const size_t ts = pi == 0 ? sizeof(double) : sizeof(float);
    const size_t extra = mhat ? static_cast<size_t>(kMhatPart) * ts : 0;  // partial sums of EO_BHAT_M
    // deepest levels first: the largest set of LDS-resident levels (coarsest included)
    size_t bytes = static_cast<size_t>(h->nc) * 2 * ts + extra;
    int lds_top = h->nlev - 1;
    while (lds_top - 1 >= 1 && bytes + static_cast<size_t>(h->lev[lds_top - 1].n) * 17 * ts <= budget) {
      lds_top--;
      bytes += static_cast<size_t>(h->lev[lds_top].n) * 17 * ts;
    }
    int top = lds_top;
    // one more level above may run from global memory (L2-resident) when it is small enough
    if (top - 1 >= 1 && h->lev[top - 1].n <= h->engine_global_rows) top--;
    std::vector<EngOp> ops;
    std::vector<int> same_top;
    for (;; top++) {
      same_top = same_color_from(h, top);
      if (top >= h->nlev - 1) break;
      ops.clear();
      if (h->nlev - top <= kEngMaxLevels)
        emit_btilde(ops, EmitCtx{h->nlev - top, h->opt.sweeps, h->opt.inner_iters, mhat, same_top.data()}, 0, false);
      if (!ops.empty() && ops.size() <= static_cast<size_t>(kEngMaxOps)) break;
    }
    if (top >= h->nlev - 1) continue;  // no engine for this precision
    if (lds_top < top) {               // LDS holds exactly the engine's levels from top down
      lds_top = top;
      bytes = static_cast<size_t>(h->nc) * 2 * ts + extra;
      for (int l = top; l < h->nlev - 1; l++) bytes += static_cast<size_t>(h->lev[l].n) * 17 * ts;
    }
    // the coarsest inverse is staged into LDS only when the step list uses it (no B^ matrix)
    const bool ainv = !mhat && bytes + static_cast<size_t>(h->nc * h->nc) * 8 <= budget;
    const size_t ainv_bytes = ainv ? static_cast<size_t>(h->nc * h->nc) * 8 : 0;
    // an FP32 top level run from global memory keeps the work vectors it gathers most (the two B^ outputs, then q0
    // and r) in whatever LDS is left; g and e stay in global memory, where the caller reads and writes them (in
    // FP64 the generic accesses this needs measured slower than the L2-resident vectors)
    int lvec = 0;
    if (top < lds_top && pi == 1) {
      const size_t vb = static_cast<size_t>(h->lev[top].n) * ts;
      for (int v : {EV_P0, EV_P1, EV_Q0, EV_R})
        if (bytes + ainv_bytes + vb <= budget) {
          lvec |= 1 << v;
          bytes += vb;
        }
    }
    EngOp *d = static_cast<EngOp *>(dalloc(h, sizeof(EngOp) * ops.size()));
    if (!d) return AMG_ERR_NOMEM;
    QA_HIP(hipMemcpyAsync(d, ops.data(), sizeof(EngOp) * ops.size(), hipMemcpyHostToDevice, h->stream));
    QA_HIP(hipStreamSynchronize(h->stream));
    h->engine_top[pi] = top;
    h->engine_lds_top[pi] = lds_top;
    h->engine_ainv_lds[pi] = ainv ? 1 : 0;
    h->engine_lvec[pi] = lvec;
    h->engine_lds[pi] = bytes + ainv_bytes;
    h->engine_ops[pi] = d;
    h->engine_nops[pi] = static_cast<int>(ops.size());
    h->engine_flops[pi] = engine_flops(h, top, ops);
  }
  QA_TRY(engine_lds_limits(h));
  // the specialised engine replaces the interpreter where the levels have its shape
  return plan_engine_fast(h);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_identity(int64_t n, T *__restrict__ a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n * n) a[i] = (i / n == i % n) ? T(1) : T(0);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_round(int64_t n, const double *__restrict__ a, T *__restrict__ b) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = static_cast<T>(a[i]);
}

template <class T>
static void fill_engine(amg_hierarchy *h, int top, int lds_top, int ainv_lds, EngPlan<T> &E, int lvec = 0);

// B^ on the level just above the coarsest is linear (smoothing, restriction, the exact coarsest solve, prolongation,
// smoothing: Algorithm 2.2 with no nonlinear inner iteration below it). When that level is small it is evaluated
// once here, column by column, by running its own step list on the unit vectors (one workgroup per column, FP64),
// and kept as an n x n matrix; the cycle then applies it as one matrix-vector product instead of ten dependent
// steps. The FP32 copy is the rounded FP64 matrix.
amg_status build_mhat(amg_hierarchy *h) {
  h->mhat_level = -1;
  if (h->nlev < 3 || h->dim != 2) return AMG_OK;
  const int l = h->nlev - 2;
  const int64_t n = h->lev[l].n;
  if (n > kMhatMaxRows) return AMG_OK;
  hipStream_t s = h->stream;
  int lds = 0;
  QA_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
  const size_t bytes = static_cast<size_t>(n) * 17 * sizeof(double) + static_cast<size_t>(h->nc) * 2 * sizeof(double) +
                       static_cast<size_t>(h->nc * h->nc) * 8;
  const size_t stat = sizeof(EngOp) * kEngMaxOps + 4096;
  if (bytes + stat > static_cast<size_t>(lds)) return AMG_OK;
  std::vector<EngOp> ops;
  const std::vector<int> same_l = same_color_from(h, l);
  emit_bhat(ops, EmitCtx{2, h->opt.sweeps, h->opt.inner_iters, 0, same_l.data()}, 0, EV_G, EV_E);
  if (ops.size() > static_cast<size_t>(kEngMaxOps)) return AMG_OK;
  double *ident = dalloc_n<double>(h, n * n);
  // a values update refills the matrices made at setup
  double *m64 = h->mhat[0] ? static_cast<double *>(h->mhat[0]) : dalloc_n<double>(h, n * n);
  float *m32 = h->mhat[1] ? static_cast<float *>(h->mhat[1]) : dalloc_n<float>(h, n * n);
  EngOp *d = static_cast<EngOp *>(dalloc(h, sizeof(EngOp) * ops.size()));
  if (!ident || !m64 || !m32 || !d) return AMG_ERR_NOMEM;
  QA_HIP(hipMemcpyAsync(d, ops.data(), sizeof(EngOp) * ops.size(), hipMemcpyHostToDevice, s));
  k_identity<double><<<nblk(n * n), kBlock, 0, s>>>(n, ident);
  EngPlan<double> E{};
  fill_engine(h, l, l, 1, E);  // both levels and the coarsest inverse in LDS
  E.nops = static_cast<int>(ops.size());
  E.ops = d;
  E.g_in = ident;
  E.e_out = m64;
  E.batch_stride = n;
  QA_TRY(engine_lds_limits(h));
  k_engine<double><<<static_cast<unsigned>(n), kEngThreads, bytes, s>>>(E);
  k_round<float><<<nblk(n * n), kBlock, 0, s>>>(n * n, m64, m32);
  QA_LAUNCH_CHECK();
  QA_HIP(hipStreamSynchronize(s));
  h->mhat_level = l;
  h->mhat_n = n;
  h->mhat[0] = m64;
  h->mhat[1] = m32;
  return AMG_OK;
}

// Level table of an engine whose top is hierarchy level `top`, levels from `lds_top` down LDS-resident.
template <class T>
static void fill_engine(amg_hierarchy *h, int top, int lds_top, int ainv_lds, EngPlan<T> &E, int lvec) {
  const int pi = std::is_same<T, float>::value ? 1 : 0;
  E.nlev = h->nlev - top;
  E.nc = static_cast<int>(h->nc);
  E.ainv_in_lds = ainv_lds;
  E.ainv = h->ainv;
  E.t_base = E.ainv_in_lds ? static_cast<int>(h->nc * h->nc * 8) : 0;
  int off = 0;
  std::vector<LevelWork<T>> &W = P<T>::W(h);
  for (int i = 0; i < E.nlev; i++) {
    const int l = top + i;
    const QuadLevel &Q = h->lev[l];
    EngLevel<T> &L = E.lv[i];
    L.k = Q.k;
    L.n = static_cast<int>(Q.n);
    L.ax = P<T>::ax(Q);
    L.optr = Q.ovf_nnz ? Q.optr : nullptr;
    L.ocol = Q.ocol;
    L.oval = P<T>::oval(Q);
    L.same_color = Q.same_color_ovf;
    L.in_lds = l >= lds_top ? 1 : 0;
    L.lvec_mask = 0;
    if (L.in_lds) {
      if (i + 1 < E.nlev) {  // operator and the eight vectors
        L.ax_off = off;
        L.vec_off = off + 9 * L.n;
        off += 17 * L.n;
      } else {               // coarsest: g and e only (slot pointers beyond EV_E are never used there)
        L.ax_off = off;
        L.vec_off = off;
        off += 2 * L.n;
      }
    } else {
      L.vec[EV_G] = W[l].g; L.vec[EV_E] = W[l].e; L.vec[EV_R] = W[l].r; L.vec[EV_P0] = W[l].p0;
      L.vec[EV_Q0] = W[l].q0; L.vec[EV_P1] = W[l].p1; L.vec[EV_Q1] = W[l].q1; L.vec[EV_D] = W[l].d;
    }
  }
  E.batch_stride = 0;
  E.mhat = nullptr;
  if (h->mhat_level >= top) {
    const int n = static_cast<int>(h->mhat_n);
    E.mhat = static_cast<const T *>(h->mhat[pi]);
    // four rows per thread: n / 4 row groups, the columns split over the rest of the workgroup (at most n runs)
    E.mhat_parts = std::max(1, std::min(kEngThreads / std::max(n / 4, 1), std::min(n, kMhatPart / n)));
    E.mpart_off = off;
    off += kMhatPart;
  }
  // the work vectors of a global top level held in LDS (lvec: bit per vector slot) come last
  if (!E.lv[0].in_lds && lvec) {
    E.lv[0].lvec_mask = lvec;
    E.lv[0].vec_off = off;
  }
}

template <class T>
static void launch_engine(amg_hierarchy *h, int top) {
  const int pi = std::is_same<T, float>::value ? 1 : 0;
  if (h->fe_cfg[pi] >= 0) {
    launch_engine_fast(h, pi);
    return;
  }
  EngPlan<T> E{};
  fill_engine(h, top, h->engine_lds_top[pi], h->engine_ainv_lds[pi], E, h->engine_lvec[pi]);
  E.nops = h->engine_nops[pi];
  E.ops = static_cast<const EngOp *>(h->engine_ops[pi]);
  std::vector<LevelWork<T>> &W = P<T>::W(h);
  E.g_in = W[top].g;
  E.e_out = W[top].e;
  Timing &t = h->timing;
  const int kind = pi ? KK_ENGINE32 : KK_ENGINE64;
  if (t.kind == kind && t.used + 2 <= t.ev.size()) {  // dispatch-stamped start / stop, as launch_timed
    hipExtLaunchKernelGGL(k_engine<T>, dim3(1), dim3(kEngThreads), h->engine_lds[pi], h->stream, t.ev[t.used],
                          t.ev[t.used + 1], 0, E);
    t.used += 2;
  } else {
    k_engine<T><<<1, kEngThreads, h->engine_lds[pi], h->stream>>>(E);
  }
}

// ---------------------------------------------------------------------------------------------------------------
// Whole-solve workgroup: the serving form for small systems. One workgroup runs a complete solve of one system
// (outer flexible CG, fine-level block smoother, the coarse cycle through the step interpreter, the convergence
// test) with no host round trip; a batch of systems is one launch with one workgroup per system, so the result of
// a system does not depend on what else is in the batch.

constexpr int64_t kWgMaxRows = 65536;

template <class T>
struct WgSys {
  int n, L, nslices;
  int64_t color_row[5], color_slice[5];
  const int64_t *slice_ptr;
  const int32_t *slice_row0, *s_row, *s_col;
  const T *s_val;             // preconditioner precision
  const double *s_val64;      // outer FP64 operator
  const T *diag;
  const int32_t *ic_ptr, *ic_col;
  const T *ic_val;
  const int32_t *crow, *agg_q, *perm;
  const double *b;            // caller numbering
  double *x;
  double *xp, *rp, *bp, *zp, *tp, *pv[2], *qv[2];
  T *f, *u, *d;               // preconditioner input / output / temporary (f, u alias rp, zp in FP64)
  double *info;               // status, iterations, restarts, relative residual
  double tol;
  int max_iters, mmax, sweeps;
  EngPlan<T> E;               // coarse levels: engine level 0 = hierarchy level 1
};

// residual of the rows of slices [s0, s1) (one wavefront per slice, strided over the workgroup's wavefronts)
template <class V, class X>
__device__ inline void wg_resid(const int64_t *sp, const int32_t *r0, const int32_t *srow, const int32_t *col,
                                const V *val, const X *f, const X *x, X *d, int64_t s0, int64_t s1) {
  const int lane = threadIdx.x & 63;
  for (int64_t s = s0 + (threadIdx.x >> 6); s < s1; s += kEngWaves) {
    if (r0[s] + lane >= r0[s + 1]) continue;
    const int32_t row = srow[r0[s] + lane];
    const int64_t off = sp[s];
    const int w = static_cast<int>((sp[s + 1] - off) >> 6);
    X acc = 0;
    for (int k = 0; k < w; k++) {
      const int64_t e = off + static_cast<int64_t>(k) * 64 + lane;
      acc += val[e] * x[col[e]];
    }
    d[row] = f[row] - acc;
  }
}

template <class T>
__device__ inline void wg_subst(const WgSys<T> &Y, const T *src, T *d, T *x, int c, bool fwd) {
  const int64_t nL4 = Y.E.lv[0].n >> 2;
  for (int64_t q = c * nL4 + threadIdx.x; q < (c + 1) * nL4; q += kEngThreads) {
    const int32_t a = Y.crow[q], b = Y.crow[q + 1];
    if (fwd) {
      for (int32_t p = a; p < b; p++) {
        T acc = src[p];
        for (int32_t e = Y.ic_ptr[p]; e < Y.ic_ptr[p + 1]; e++)
          if (Y.ic_col[e] < p) acc -= Y.ic_val[e] * d[Y.ic_col[e]];
        d[p] = acc / Y.diag[p];
      }
    } else {
      for (int32_t p = b - 1; p >= a; p--) {
        T acc = src[p];
        for (int32_t e = Y.ic_ptr[p]; e < Y.ic_ptr[p + 1]; e++)
          if (Y.ic_col[e] > p) acc -= Y.ic_val[e] * d[Y.ic_col[e]];
        d[p] = acc / Y.diag[p];
      }
    }
    for (int32_t p = a; p < b; p++) x[p] += d[p];
  }
}

template <class T>
__device__ inline void wg_fine_phase(const WgSys<T> &Y, const T *f, T *u, int c, bool fwd, bool from_f) {
  if (!from_f) {
    wg_resid(Y.slice_ptr, Y.slice_row0, Y.s_row, Y.s_col, Y.s_val, f, u, Y.d, Y.color_slice[c], Y.color_slice[c + 1]);
    __syncthreads();
  }
  wg_subst(Y, from_f ? f : Y.d, Y.d, u, c, fwd);
  __syncthreads();
}

template <class T>
__device__ inline T *wg_engine_vec(const EngLevel<T> &L, T *S, int v) {
  return L.in_lds ? S + L.vec_off + v * L.n : L.vec[v];
}

// z = B^_F[f] on the fine level (Algorithm 2.2), the coarse B~ through the step interpreter
template <class T>
__device__ void wg_bhat_fine(const WgSys<T> &Y, const EngOp *ops, const EngLevel<T> *LV, T *S, const double *Ainv,
                             double (*sc)[8], double *red, const T *f, T *u) {
  const int tid = threadIdx.x;
  for (int i = tid; i < Y.n; i += kEngThreads) u[i] = T(0);
  __syncthreads();
  for (int sw = 0; sw < Y.sweeps; sw++)
    for (int c = 0; c < 4; c++) wg_fine_phase(Y, f, u, c, true, sw == 0 && c == 0);
  wg_resid(Y.slice_ptr, Y.slice_row0, Y.s_row, Y.s_col, Y.s_val, f, u, Y.d, 0, Y.nslices);
  __syncthreads();
  T *g0 = wg_engine_vec(LV[0], S, EV_G);
  const int nL = LV[0].n;
  for (int q = tid; q < nL; q += kEngThreads) {
    T acc = 0;
    for (int32_t p = Y.crow[q]; p < Y.crow[q + 1]; p++) acc += Y.d[p];
    g0[q] = acc;
  }
  __syncthreads();
  eng_run(Y.E, ops, LV, S, Ainv, sc, red);
  const T *e0 = wg_engine_vec(LV[0], S, EV_E);
  for (int i = tid; i < Y.n; i += kEngThreads) u[i] += e0[Y.agg_q[i]];
  __syncthreads();
  for (int sw = 0; sw < Y.sweeps; sw++)
    for (int c = 3; c >= 0; c--) wg_fine_phase(Y, f, u, c, false, false);
}

// q = A p (FP64) with (p, q) and (r, p), or the true residual t = b - A x with (t, t)
__device__ inline void wg_spmv64(const int64_t *sp, const int32_t *r0, const int32_t *srow, const int32_t *col,
                                 const double *val, int64_t ns, const double *p, double *q, const double *r,
                                 double (&v)[2]) {
  const int lane = threadIdx.x & 63;
  v[0] = 0.0; v[1] = 0.0;
  for (int64_t s = threadIdx.x >> 6; s < ns; s += kEngWaves) {
    if (r0[s] + lane >= r0[s + 1]) continue;
    const int32_t row = srow[r0[s] + lane];
    const int64_t off = sp[s];
    const int w = static_cast<int>((sp[s + 1] - off) >> 6);
    double acc = 0.0;
    for (int k = 0; k < w; k++) {
      const int64_t e = off + static_cast<int64_t>(k) * 64 + lane;
      acc += val[e] * p[col[e]];
    }
    q[row] = acc;
    v[0] += p[row] * acc;
    v[1] += r[row] * p[row];
  }
}

template <class T>
__global__ void __launch_bounds__(kEngThreads) k_solve_wg(const WgSys<T> *systems) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sc[kEngMaxLevels][8];
  __shared__ double red[2 * kEngWaves];
  __shared__ EngOp ops[kEngMaxOps];
  __shared__ EngLevel<T> LV[kEngMaxLevels];
  const WgSys<T> &Y = systems[blockIdx.x];
  const int tid = threadIdx.x;
  const int n = Y.n;
  T *S = reinterpret_cast<T *>(smem + Y.E.t_base);
  double *ainv_lds = reinterpret_cast<double *>(smem);
  eng_stage(Y.E, ops, LV, S, ainv_lds);
  const double *Ainv = Y.E.ainv_in_lds ? ainv_lds : Y.E.ainv;
  // x = 0, r = b (permuted)
  double v1[1] = {0.0};
  for (int i = tid; i < n; i += kEngThreads) {
    const double bi = Y.b[Y.perm[i]];
    Y.bp[i] = bi;
    Y.rp[i] = bi;
    Y.xp[i] = 0.0;
    v1[0] += bi * bi;
  }
  eng_reduce<1>(v1, red);  // includes the barrier that publishes the staging above
  const double bn = sqrt(v1[0]);
  double status = 6.0;  // NOCONV unless something else happens
  int it = 0, restarts = 0, par = 0;
  bool have_prev = false;
  double dprev = 0.0;
  if (bn == 0.0) {
    status = 0.0;
  } else {
    while (it < Y.max_iters) {
      // z = B^_F[r]
      if constexpr (std::is_same<T, double>::value) {
        wg_bhat_fine(Y, ops, LV, S, Ainv, sc, red, Y.rp, Y.zp);
      } else {
        for (int i = tid; i < n; i += kEngThreads) Y.f[i] = static_cast<T>(Y.rp[i]);
        __syncthreads();
        wg_bhat_fine(Y, ops, LV, S, Ainv, sc, red, Y.f, Y.u);
        for (int i = tid; i < n; i += kEngThreads) Y.zp[i] = static_cast<double>(Y.u[i]);
        __syncthreads();
      }
      double *p = Y.pv[par], *q = Y.qv[par];
      const double *pprev = Y.pv[1 - par], *qprev = Y.qv[1 - par];
      double beta = 0.0;
      if (have_prev && Y.mmax == 1) {
        double t1[1] = {0.0};
        for (int i = tid; i < n; i += kEngThreads) t1[0] += Y.zp[i] * qprev[i];
        eng_reduce<1>(t1, red);
        beta = -t1[0] / dprev;
      }
      for (int i = tid; i < n; i += kEngThreads) p[i] = (have_prev && Y.mmax == 1) ? Y.zp[i] + beta * pprev[i] : Y.zp[i];
      __syncthreads();
      double v2[2];
      wg_spmv64(Y.slice_ptr, Y.slice_row0, Y.s_row, Y.s_col, Y.s_val64, Y.nslices, p, q, Y.rp, v2);
      eng_reduce<2>(v2, red);
      const double d = v2[0];
      if (!(d > 0.0)) {
        status = 5.0;  // BREAKDOWN
        break;
      }
      const double alpha = v2[1] / d;
      double v3[1] = {0.0};
      for (int i = tid; i < n; i += kEngThreads) {
        Y.xp[i] += alpha * p[i];
        const double ri = Y.rp[i] - alpha * q[i];
        Y.rp[i] = ri;
        v3[0] += ri * ri;
      }
      eng_reduce<1>(v3, red);
      it++;
      have_prev = true;
      dprev = d;
      par ^= 1;
      if (sqrt(v3[0]) <= Y.tol * bn) {
        double v4[2];
        wg_spmv64(Y.slice_ptr, Y.slice_row0, Y.s_row, Y.s_col, Y.s_val64, Y.nslices, Y.xp, Y.tp, Y.xp, v4);
        __syncthreads();
        double v5[1] = {0.0};
        for (int i = tid; i < n; i += kEngThreads) {
          const double ti = Y.bp[i] - Y.tp[i];
          Y.tp[i] = ti;
          v5[0] += ti * ti;
        }
        eng_reduce<1>(v5, red);
        if (sqrt(v5[0]) <= Y.tol * bn) {
          status = 0.0;
          break;
        }
        for (int i = tid; i < n; i += kEngThreads) Y.rp[i] = Y.tp[i];
        __syncthreads();
        have_prev = false;
        restarts++;
      }
    }
  }
  // true relative residual and the solution in the caller's numbering
  double v6[2];
  wg_spmv64(Y.slice_ptr, Y.slice_row0, Y.s_row, Y.s_col, Y.s_val64, Y.nslices, Y.xp, Y.tp, Y.xp, v6);
  __syncthreads();
  double v7[1] = {0.0};
  for (int i = tid; i < n; i += kEngThreads) {
    const double ti = Y.bp[i] - Y.tp[i];
    v7[0] += ti * ti;
    Y.x[Y.perm[i]] = Y.xp[i];
  }
  eng_reduce<1>(v7, red);
  if (tid == 0) {
    Y.info[0] = status;
    Y.info[1] = it;
    Y.info[2] = restarts;
    Y.info[3] = bn == 0.0 ? 0.0 : sqrt(v7[0]) / bn;
  }
}

// Plan of the whole-solve workgroup for one precision: all quadtree levels run through the step interpreter, the
// deepest ones from LDS.
amg_status plan_wg(amg_hierarchy *h) {
  h->wg_nops[0] = h->wg_nops[1] = 0;
  // the whole-solve workgroup carries the substitution smoother and at most one kept direction only
  if (h->nlev < 3 || h->n > kWgMaxRows || h->opt.smoother || h->opt.outer_mmax < 0 || h->dim != 2) return AMG_OK;
  if (h->lds_max == 0) {
    int lds = 0;
    QA_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device));
    h->lds_max = static_cast<size_t>(lds);
  }
  const size_t stat = sizeof(EngOp) * kEngMaxOps + 4096;
  const size_t budget = h->lds_max > stat ? h->lds_max - stat : 0;
  std::vector<EngOp> ops;
  const int mhat = h->mhat_level >= 0 ? 1 : 0;
  const std::vector<int> same1 = same_color_from(h, 1);
  emit_btilde(ops, EmitCtx{h->nlev - 1, h->opt.sweeps, h->opt.inner_iters, mhat, same1.data()}, 0, false);
  if (ops.size() > static_cast<size_t>(kEngMaxOps) || h->nlev - 1 > kEngMaxLevels) return AMG_OK;
  for (int pi = 0; pi < 2; pi++) {
    const size_t ts = pi == 0 ? sizeof(double) : sizeof(float);
    const size_t extra = mhat ? static_cast<size_t>(kMhatPart) * ts : 0;
    size_t bytes = static_cast<size_t>(h->nc) * 2 * ts + extra;
    int lds_top = h->nlev - 1;
    while (lds_top - 1 >= 1 && bytes + static_cast<size_t>(h->lev[lds_top - 1].n) * 17 * ts <= budget) {
      lds_top--;
      bytes += static_cast<size_t>(h->lev[lds_top].n) * 17 * ts;
    }
    const bool ainv = !mhat && bytes + static_cast<size_t>(h->nc * h->nc) * 8 <= budget;
    EngOp *d = static_cast<EngOp *>(dalloc(h, sizeof(EngOp) * ops.size()));
    if (!d) return AMG_ERR_NOMEM;
    QA_HIP(hipMemcpyAsync(d, ops.data(), sizeof(EngOp) * ops.size(), hipMemcpyHostToDevice, h->stream));
    QA_HIP(hipStreamSynchronize(h->stream));
    h->wg_ops[pi] = d;
    h->wg_nops[pi] = static_cast<int>(ops.size());
    h->wg_lds_top[pi] = lds_top;
    h->wg_ainv_lds[pi] = ainv ? 1 : 0;
    h->wg_lds[pi] = bytes + (ainv ? static_cast<size_t>(h->nc * h->nc) * 8 : 0);
  }
  return engine_lds_limits(h);
}

template <class T> static void btilde(amg_hierarchy *h, int l, const T *g, T *e, bool defer_update2);
template <class T> static void btilde_oct(amg_hierarchy *h, int l, const T *g, T *e);

// Solve or cycle on level l for the correction of level l - 1. Returns the pending last update of B~ on level l when
// it was left for the parent's prolongation (only levels that run per step, with two inner iterations).
template <class T>
static Pending<T> coarse_solve_or_cycle(amg_hierarchy *h, int l) {
  LevelWork<T> &w = P<T>::W(h)[l];
  const int pi = std::is_same<T, float>::value ? 1 : 0;
  if (l == h->nlev - 1) {
    k_dense_solve<T><<<1, kBlock, 0, h->stream>>>(static_cast<int>(h->nc), h->ainv, w.g, w.e);
  } else if (h->dim == 3) {
    btilde_oct<T>(h, l, w.g, w.e);
  } else if (h->use_engine && l == h->engine_top[pi]) {
    launch_engine<T>(h, l);
  } else {
    const bool defer = h->opt.inner_iters >= 2;
    btilde<T>(h, l, w.g, w.e, defer);
    if (defer) return Pending<T>{h->scal + static_cast<size_t>(l) * kScalars, w.p1, w.p0};
  }
  return Pending<T>{nullptr, nullptr, nullptr};
}

template <class T>
static void gs_phase_coarse(amg_hierarchy *h, int l, const T *f, T *u, int c) {
  const QuadLevel &Q = h->lev[l];
  const int64_t n4 = Q.n >> 2;
  if (Q.same_color_ovf) {
    T *dl = P<T>::W(h)[l].d;
    k_cgs<T><<<nblk(n4), kBlock, 0, h->stream>>>(qview<T>(Q), f, u, dl, c);
    k_add_range<T><<<nblk(n4), kBlock, 0, h->stream>>>(c * n4, n4, dl, u);
  } else {
    k_cgs<T><<<nblk(n4), kBlock, 0, h->stream>>>(qview<T>(Q), f, u, nullptr, c);
  }
}

// B^_l for a quadtree level l (not the coarsest): Algorithm 2.2. `upd` (sc non-null): the pending first inner update
// of the caller, done by the first relaxation (needs sweeps >= 1). `beta` (non-null): the last color phase also
// forms (p1, q0) for beta (needs sweeps >= 1 and no same-color couplings).
template <class T>
static void bhat_coarse(amg_hierarchy *h, int l, const T *f, T *u, const Upd1<T> &upd = Upd1<T>{},
                        const T *beta_q0 = nullptr) {
  const QuadLevel &Q = h->lev[l];
  hipStream_t s = h->stream;
  const int sweeps = h->opt.sweeps;
  const bool U = upd.sc != nullptr;
  const int64_t n4 = Q.n >> 2;
  LevelWork<T> &wc = P<T>::W(h)[l + 1];
  // the per-step path keeps one launch per color phase; with tiles the presmoothing sweep and the restriction take
  // one launch, and so does the first post-smoothing sweep
  const bool tiles = h->use_engine != 0 && !Q.same_color_ovf && Q.ovf_nnz == 0 && n4 >= kTileCells;
  const bool tiled_pre = tiles && sweeps == 1;
  if (tiled_pre) {
    const unsigned grid = static_cast<unsigned>(n4 / kTileCells);
    if (U) k_cgs_pre4<T, true><<<grid, kTileThreads, 0, s>>>(qview<T>(Q), f, u, upd, wc.g);
    else k_cgs_pre4<T, false><<<grid, kTileThreads, 0, s>>>(qview<T>(Q), f, u, upd, wc.g);
  }
  for (int sw = 0; sw < (tiled_pre ? 0 : sweeps); sw++)
    for (int c = 0; c < 4; c++) {
      if (sw == 0 && c == 0 && !Q.same_color_ovf) {
        if (U) k_cgs_first2<T, true><<<nblk(Q.n), kBlock, 0, s>>>(qview<T>(Q), f, u, upd);
        else k_cgs_first2<T, false><<<nblk(Q.n), kBlock, 0, s>>>(qview<T>(Q), f, u, upd);
        c = 1;
      } else if (sw == 0 && c == 0) {
        if (U) k_cgs_first<T, true><<<nblk(Q.n), kBlock, 0, s>>>(qview<T>(Q), f, u, upd);
        else k_cgs_first<T, false><<<nblk(Q.n), kBlock, 0, s>>>(qview<T>(Q), f, u, upd);
      } else {
        gs_phase_coarse<T>(h, l, f, u, c);
      }
    }
  if (!tiled_pre) k_cres_restrict<T><<<nblk(Q.n >> 2), kBlock, 0, s>>>(qview<T>(Q), f, u, wc.g);
  const Pending<T> pend = coarse_solve_or_cycle<T>(h, l + 1);
  // without same-color couplings the prolongation folds into the first post-smoothing sweep
  const bool fold_prolong = !Q.same_color_ovf && sweeps >= 1;
  if (!fold_prolong) k_cprolong<T><<<nblk(Q.n), kBlock, 0, s>>>(Q.k, Q.n, wc.e, pend, u);
  const Red rb = red(h, l, EPI_BETA);
  const bool tiled = tiles && fold_prolong;
  if (tiled) {
    const QView<T> V = qview<T>(Q);
    const unsigned grid = static_cast<unsigned>(n4 / kTileCells);
    if (beta_q0 && sweeps == 1) {
      k_cgs_post4<T, true><<<grid, kTileThreads, 0, s>>>(V, f, u, wc.e, pend, beta_q0, rb);
      finish<1>(h, nblk(n4), rb);
    } else {
      k_cgs_post4<T, false><<<grid, kTileThreads, 0, s>>>(V, f, u, wc.e, pend, beta_q0, rb);
    }
  }
  for (int sw = tiled ? 1 : 0; sw < sweeps; sw++)
    for (int c = 3; c >= 0; c--) {
      const bool beta_here = beta_q0 && sw == sweeps - 1 && c == 0;
      if (fold_prolong && sw == 0) {
        const QView<T> V = qview<T>(Q);
        switch (c) {
          case 3: k_cgs_post<T, 3, false><<<nblk(n4), kBlock, 0, s>>>(V, f, u, wc.e, pend, beta_q0, rb); break;
          case 2: k_cgs_post<T, 2, false><<<nblk(n4), kBlock, 0, s>>>(V, f, u, wc.e, pend, beta_q0, rb); break;
          case 1: k_cgs_post<T, 1, false><<<nblk(n4), kBlock, 0, s>>>(V, f, u, wc.e, pend, beta_q0, rb); break;
          default:
            if (beta_here) k_cgs_post<T, 0, true><<<nblk(n4), kBlock, 0, s>>>(V, f, u, wc.e, pend, beta_q0, rb);
            else k_cgs_post<T, 0, false><<<nblk(n4), kBlock, 0, s>>>(V, f, u, wc.e, pend, beta_q0, rb);
        }
      } else if (beta_here) {
        k_cgs0_beta<T><<<nblk(n4), kBlock, 0, s>>>(qview<T>(Q), f, u, beta_q0, rb);
      } else {
        gs_phase_coarse<T>(h, l, f, u, c);
      }
      if (beta_here) finish<1>(h, nblk(n4), rb);
    }
}

template <class T>
static void fine_resid(amg_hierarchy *h, const T *f, const T *x, T *d, int c0, int c1, int kind) {
  const SliceSched Z = slice_sched(h->fine, c0, c1);
  const unsigned grid = sched_grid(Z);
  if (grid == 0) return;
  if (kind == P<T>::kResid)
    launch_timed(h, kind, k_fine_resid_full<T>, grid, sview<T>(h->fine, P<T>::sval(h->fine)), Z, f, x, d);
  else
    launch_timed(h, kind, k_fine_resid<T>, grid, sview<T>(h->fine, P<T>::sval(h->fine)), Z, f, x, d);
}

template <class T, int SM, bool FWD, bool GIVEN>
static void fine_gs_launch(amg_hierarchy *h, unsigned grid, FuseArgs<T> A) {
  A.ent_cap = std::min(h->fine.win_ent_max, kFuseDynBytes / fuse_ent_bytes<T, SM>());
  const size_t lds = (static_cast<size_t>(A.ent_cap) * fuse_ent_bytes<T, SM>() + 15) / 16 * 16;
  launch_timed_lds(h, P<T>::kGs, k_fine_gs<T, SM, FWD, GIVEN>, grid, lds, sview<T>(h->fine, P<T>::sval(h->fine)),
                   A);
}

// One color phase of the fine smoother: the fused residual and cell solves (k_fine_gs), then the cells left to the
// level-scheduled substitution. from_f: the first phase of a sweep from zero, whose residual is f. Where cells of a
// color are coupled to each other, `old` says where the values of the color's rows from before the phase are:
// kOldZero (a sweep from zero: still zero) or kOldSnap (the fine workspace's snapshot) let the fused phase form the
// residual itself; kOldNone takes a separate residual pass first.
enum { kOldNone = 0, kOldZero = 1, kOldSnap = 2 };
template <class T>
static void fine_phase(amg_hierarchy *h, const T *f, T *u, T *d, int c, bool fwd, bool from_f, int old = kOldNone) {
  const FineLevel &F = h->fine;
  const T *src = from_f ? f : d;
  const bool split = !from_f && F.same_color && old != kOldNone;
  const bool given = from_f || (F.same_color && !split);
  if (!from_f && F.same_color && !split) fine_resid<T>(h, f, u, d, c, c + 1, -1);
  const int64_t b0 = F.big_color[c], nb = F.big_color[c + 1] - b0;
  FuseArgs<T> A{};
  A.win_q = F.win_q;
  A.win_row = F.win_row;
  A.crow = F.crow;
  A.win_slice = F.win_slice;
  A.win_ent = F.win_ent;
  A.win0 = F.color_win[c];
  A.nwin = F.color_win[c + 1] - F.color_win[c];
  A.xcd = A.nwin >= 64 ? 1 : 0;
  A.big = nb > 0 ? 1 : 0;
  A.f = f;
  A.src = src;
  A.u = u;
  A.d = d;
  A.diag = P<T>::diag(F);
  A.icv = P<T>::icv(F);
  A.fac = P<T>::bfac(F);
  A.icp = F.ic_ptr;
  A.icc = F.ic_col;
  A.boff = F.boff;
  A.split = split ? 1 : 0;
  A.clo = static_cast<int32_t>(F.color_row[c]);
  A.chi = static_cast<int32_t>(F.color_row[c + 1]);
  A.alt = old == kOldSnap ? P<T>::W(h)[0].r : nullptr;
  if (A.nwin > 0) {
    const unsigned grid = static_cast<unsigned>(A.xcd ? 8 * ((A.nwin + 7) / 8) : A.nwin);
    if (h->opt.smoother) {
      if (given) fine_gs_launch<T, 1, true, true>(h, grid, A);
      else fine_gs_launch<T, 1, true, false>(h, grid, A);
    } else if (fwd) {
      if (given) fine_gs_launch<T, 0, true, true>(h, grid, A);
      else fine_gs_launch<T, 0, true, false>(h, grid, A);
    } else {
      if (given) fine_gs_launch<T, 0, false, true>(h, grid, A);
      else fine_gs_launch<T, 0, false, false>(h, grid, A);
    }
  }
  if (nb > 0) {
    const int dir = fwd ? 0 : 1;
    const int lds_rows = std::min(F.big_max_rows, kSubstDynBytes / static_cast<int>(sizeof(T)));
    const size_t lds = (static_cast<size_t>(lds_rows) * sizeof(T) + 15) / 16 * 16;
    if (fwd)
      k_fine_subst_big<T, true><<<static_cast<unsigned>(nb), kSubstLanes, lds, h->stream>>>(
          F.crow, F.ic_ptr, F.ic_col, P<T>::icv(F), P<T>::diag(F), src, d, u, F.big_cells, b0, F.big_lofs[dir],
          F.big_lptr[dir], F.big_sched[dir], lds_rows);
    else
      k_fine_subst_big<T, false><<<static_cast<unsigned>(nb), kSubstLanes, lds, h->stream>>>(
          F.crow, F.ic_ptr, F.ic_col, P<T>::icv(F), P<T>::diag(F), src, d, u, F.big_cells, b0, F.big_lofs[dir],
          F.big_lptr[dir], F.big_sched[dir], lds_rows);
  }
}

// B^_F on the fine level (f, u in permuted numbering)
template <class T>
static void bhat_fine(amg_hierarchy *h, const T *f, T *u) {
  const FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  LevelWork<T> &w = P<T>::W(h)[0];
  k_fill<T><<<nblk(F.n), kBlock, 0, s>>>(F.n, u, T(0));
  const int sweeps = h->opt.sweeps;
  const int nc = F.ncolor;
  // one sweep each way: the pre-smoothing's color rows are zero before their phase, and the post-smoothing's hold
  // the prolongation's values, which it copies to the snapshot
  const bool one = sweeps == 1 && F.same_color;
  for (int sw = 0; sw < sweeps; sw++)
    for (int c = 0; c < nc; c++)
      fine_phase<T>(h, f, u, w.d, c, true, sw == 0 && c == 0, one ? kOldZero : kOldNone);
  LevelWork<T> &wc = P<T>::W(h)[1];
  fine_resid<T>(h, f, u, w.d, 0, F.ncolor, P<T>::kResid);
  const int64_t nL = static_cast<int64_t>(1) << (h->dim * h->L);
  const int big = h->opt.smoother ? kBlockMax : kBigCell;  // the big-cell list's threshold
  k_fine_restrict<T><<<nblk(nL), kBlock, 0, s>>>(nL, F.crow, w.d, wc.g, F.nbig ? big : INT32_MAX);
  if (F.nbig) k_fine_restrict_big<T><<<static_cast<unsigned>(F.nbig), 64, 0, s>>>(F.big_cells, F.crow, w.d, wc.g);
  const Pending<T> pend = coarse_solve_or_cycle<T>(h, 1);
  k_fine_prolong<T><<<nblk(F.n), kBlock, 0, s>>>(F.n, F.agg_q, wc.e, pend, u, one ? w.r : nullptr);
  for (int sw = 0; sw < sweeps; sw++)
    for (int c = nc - 1; c >= 0; c--) fine_phase<T>(h, f, u, w.d, c, false, false, one ? kOldSnap : kOldNone);
}

template <class T>
static void bhat(amg_hierarchy *h, int l, const T *f, T *u) {
  if (l == 0) bhat_fine<T>(h, f, u);
  else bhat_coarse<T>(h, l, f, u);
}

// B~_l: Algorithm 2.1 with n = inner_iters (1 or 2) steps and B^_l as preconditioner
template <class T>
static void btilde(amg_hierarchy *h, int l, const T *g, T *e, bool defer_update2) {
  const QuadLevel &Q = h->lev[l];
  LevelWork<T> &w = P<T>::W(h)[l];
  hipStream_t s = h->stream;
  const double *sc = h->scal + static_cast<size_t>(l) * kScalars;
  bhat<T>(h, l, g, w.p0);
  k_cspmv_dot<T><<<nred(Q.n), kBlock, 0, s>>>(qview<T>(Q), w.p0, w.q0, g, red(h, l, EPI_ALPHA0));
  finish<2>(h, nred(Q.n), red(h, l, EPI_ALPHA0));
  // with two inner steps the update below and the inner product for beta fold into the second B^ (first and last
  // relaxation) where its sweeps allow
  const bool two = h->opt.inner_iters >= 2;
  const bool fold_upd = two && h->opt.sweeps >= 1;
  const bool fold_beta = two && h->opt.sweeps >= 1 && !Q.same_color_ovf;
  if (!fold_upd) k_update1<T><<<nblk(Q.n), kBlock, 0, s>>>(Q.n, sc, w.p0, w.q0, g, e, w.r);
  if (!two) return;
  bhat_coarse<T>(h, l, w.r, w.p1, fold_upd ? Upd1<T>{sc, g, w.q0, w.p0, e, w.r} : Upd1<T>{},
                 fold_beta ? w.q0 : nullptr);
  if (!fold_beta) {
    k_dot<T><<<nred(Q.n), kBlock, 0, s>>>(Q.n, w.p1, w.q0, red(h, l, EPI_BETA));
    finish<1>(h, nred(Q.n), red(h, l, EPI_BETA));
  }
  k_cspmv_dir<T><<<nred(Q.n), kBlock, 0, s>>>(qview<T>(Q), sc, w.p1, w.p0, w.r, red(h, l, EPI_ALPHA1));
  finish<2>(h, nred(Q.n), red(h, l, EPI_ALPHA1));
  if (!defer_update2) k_update2<T><<<nblk(Q.n), kBlock, 0, s>>>(Q.n, sc, w.p1, w.p0, e);
}

// Octree levels (per-step launches): one color phase, B^ (Algorithm 2.2) and B~ (Algorithm 2.1 with n = inner
// iterations), with the same readings as the quadtree levels; a small level's B^ runs in one workgroup
// (k_bhat3_small).
template <class T>
static void gs_phase_oct(amg_hierarchy *h, int l, const T *f, T *u, int c) {
  const QuadLevel &Q = h->lev[l];
  const int64_t n8 = Q.n >> 3;
  if (Q.same_color_ovf) {
    T *dl = P<T>::W(h)[l].d;
    k_cgs3<T><<<nblk(n8), kBlock, 0, h->stream>>>(qview<T>(Q), f, u, dl, c);
    k_add_range<T><<<nblk(n8), kBlock, 0, h->stream>>>(c * n8, n8, dl, u);
  } else {
    k_cgs3<T><<<nblk(n8), kBlock, 0, h->stream>>>(qview<T>(Q), f, u, nullptr, c);
  }
}

template <class T> static void btilde_oct(amg_hierarchy *h, int l, const T *g, T *e);

template <class T>
static void bhat_oct(amg_hierarchy *h, int l, const T *f, T *u) {
  const QuadLevel &Q = h->lev[l];
  hipStream_t s = h->stream;
  const bool small = Q.n <= kOctSweepMax;
  T *dl = Q.same_color_ovf ? P<T>::W(h)[l].d : nullptr;
  LevelWork<T> &wc = P<T>::W(h)[l + 1];
  if (small) {  // B^ in one workgroup: whole when the next level is the coarsest, else around its B~
    const bool whole = l + 1 == h->nlev - 1;
    const int nc = whole ? static_cast<int>(h->nc) : 0, sw = h->opt.sweeps;
    const size_t lds = bhat3_lds_bytes<T>(Q.n, nc);
    if (whole && lds <= static_cast<size_t>(bhat3_lds_limit(h->device))) {
      k_bhat3_lds<T><<<1, kOctSweepThreads, lds, s>>>(qview<T>(Q), f, u, h->ainv, nc, sw, dl ? 1 : 0);
    } else if (whole) {
      k_bhat3_small<T, 0><<<1, kOctSweepThreads, 0, s>>>(qview<T>(Q), f, u, dl, wc.g, wc.e, h->ainv, nc, sw);
    } else {
      k_bhat3_small<T, 1><<<1, kOctSweepThreads, 0, s>>>(qview<T>(Q), f, u, dl, wc.g, wc.e, nullptr, 0, sw);
      btilde_oct<T>(h, l + 1, wc.g, wc.e);
      k_bhat3_small<T, 2><<<1, kOctSweepThreads, 0, s>>>(qview<T>(Q), f, u, dl, wc.g, wc.e, nullptr, 0, sw);
    }
    return;
  }
  k_fill<T><<<nblk(Q.n), kBlock, 0, s>>>(Q.n, u, T(0));
  for (int sw = 0; sw < h->opt.sweeps; sw++)
    for (int c = 0; c < 8; c++) gs_phase_oct<T>(h, l, f, u, c);
  k_cres_restrict3<T><<<nblk(Q.n >> 3), kBlock, 0, s>>>(qview<T>(Q), f, u, wc.g);
  if (l + 1 == h->nlev - 1)
    k_dense_solve<T><<<1, kBlock, 0, s>>>(static_cast<int>(h->nc), h->ainv, wc.g, wc.e);
  else
    btilde_oct<T>(h, l + 1, wc.g, wc.e);
  k_cprolong3<T><<<nblk(Q.n), kBlock, 0, s>>>(Q.k, Q.n, wc.e, u);
  for (int sw = 0; sw < h->opt.sweeps; sw++)
    for (int c = 7; c >= 0; c--) gs_phase_oct<T>(h, l, f, u, c);
}

template <class T>
static void btilde_oct(amg_hierarchy *h, int l, const T *g, T *e) {
  const QuadLevel &Q = h->lev[l];
  LevelWork<T> &w = P<T>::W(h)[l];
  hipStream_t s = h->stream;
  const double *sc = h->scal + static_cast<size_t>(l) * kScalars;
  bhat_oct<T>(h, l, g, w.p0);
  k_cspmv_dot3<T><<<nred(Q.n), kBlock, 0, s>>>(qview<T>(Q), w.p0, w.q0, g, red(h, l, EPI_ALPHA0));
  finish<2>(h, nred(Q.n), red(h, l, EPI_ALPHA0));
  k_update1<T><<<nblk(Q.n), kBlock, 0, s>>>(Q.n, sc, w.p0, w.q0, g, e, w.r);
  if (h->opt.inner_iters < 2) return;
  bhat_oct<T>(h, l, w.r, w.p1);
  k_dot<T><<<nred(Q.n), kBlock, 0, s>>>(Q.n, w.p1, w.q0, red(h, l, EPI_BETA));
  finish<1>(h, nred(Q.n), red(h, l, EPI_BETA));
  k_cspmv_dir3<T><<<nred(Q.n), kBlock, 0, s>>>(qview<T>(Q), sc, w.p1, w.p0, w.r, red(h, l, EPI_ALPHA1));
  finish<2>(h, nred(Q.n), red(h, l, EPI_ALPHA1));
  k_update2<T><<<nblk(Q.n), kBlock, 0, s>>>(Q.n, sc, w.p1, w.p0, e);
}

// z = B^_F[r] in the requested precision (r, z: FP64, permuted numbering)
amg_status precond_apply(amg_hierarchy *h, int precision, const double *r, double *z) {
  const int64_t n = h->n;
  hipStream_t s = h->stream;
  if (h->nlev == 1) {
    k_dense_solve<double><<<1, kBlock, 0, s>>>(static_cast<int>(h->nc), h->ainv, r, z);
    QA_LAUNCH_CHECK();
    return AMG_OK;
  }
  if (precision == 1) {
    LevelWork<float> &w = h->w32[0];
    k_cast<double, float><<<nblk(n), kBlock, 0, s>>>(n, r, w.f);
    bhat_fine<float>(h, w.f, w.u);
    k_cast<float, double><<<nblk(n), kBlock, 0, s>>>(n, w.u, z);
  } else {
    bhat_fine<double>(h, r, z);
  }
  QA_LAUNCH_CHECK();
  return AMG_OK;
}

amg_status alloc_workspaces(amg_hierarchy *h) {
  const int64_t n = h->n;
  h->w64.assign(h->nlev, LevelWork<double>{});
  h->w32.assign(h->nlev, LevelWork<float>{});
  {
    auto mk = [&](auto &W) -> bool {
      using T = std::remove_pointer_t<decltype(W[0].f)>;
      W[0].f = dalloc_n<T>(h, n);
      W[0].u = dalloc_n<T>(h, n);
      W[0].d = dalloc_n<T>(h, n);
      if (!W[0].f || !W[0].u || !W[0].d) return false;
      if (h->fine.same_color) {  // the fine smoother's snapshot of u before the backward sweep
        W[0].r = dalloc_n<T>(h, n);
        if (!W[0].r) return false;
      }
      for (int l = 1; l < h->nlev; l++) {
        const int64_t m = h->lev[l].n;
        W[l].g = dalloc_n<T>(h, m);
        W[l].e = dalloc_n<T>(h, m);
        if (!W[l].g || !W[l].e) return false;
        if (l < h->nlev - 1) {
          W[l].r = dalloc_n<T>(h, m);
          W[l].p0 = dalloc_n<T>(h, m);
          W[l].q0 = dalloc_n<T>(h, m);
          W[l].p1 = dalloc_n<T>(h, m);
          W[l].q1 = dalloc_n<T>(h, m);
          W[l].d = dalloc_n<T>(h, m);
          if (!W[l].r || !W[l].p0 || !W[l].q0 || !W[l].p1 || !W[l].q1 || !W[l].d) return false;
        }
      }
      return true;
    };
    if (!mk(h->w64) || !mk(h->w32)) return AMG_ERR_NOMEM;
  }
  double **outer[] = {&h->xp, &h->rp, &h->bp, &h->zp, &h->pp, &h->qp, &h->pprev, &h->qprev, &h->tp};
  for (double **v : outer) {
    *v = dalloc_n<double>(h, n);
    if (!*v) return AMG_ERR_NOMEM;
  }
  h->scal = dalloc_n<double>(h, (h->nlev + 1) * kScalars);
  // two values per workgroup of the largest reduction launch (a scheduled pass over all slices)
  h->partials_cap = std::max<int64_t>(kRedBlocksMax, sched_grid(slice_sched(h->fine, 0, h->fine.ncolor)) + 1) * 2;
  h->partials = dalloc_n<double>(h, h->partials_cap);
  if (!h->scal || !h->partials) return AMG_ERR_NOMEM;
  QA_HIP(hipMemsetAsync(h->scal, 0, sizeof(double) * (h->nlev + 1) * kScalars, h->stream));
  if (!h->host_scal) QA_TRY(borrow_pinned_scalars(&h->host_scal));
  return AMG_OK;
}

double kernel_bytes(const amg_hierarchy *h, int kind) {
  const double n = static_cast<double>(h->n), nnz = static_cast<double>(h->fine.nnz);
  const bool given_resid = h->fine.same_color && h->opt.sweeps != 1;
  switch (kind) {
    case KK_SPMV64: return 12.0 * nnz + 24.0 * n;   // values + columns, x, q written, r read for (r, p)
    case KK_RESID_FINE64: return 12.0 * nnz + 24.0 * n;
    case KK_RESID_FINE32: return 8.0 * nnz + 12.0 * n;
    // one fused color phase: the color's share of the residual pass (f read, x read, x written) and of the cell
    // solves' data (factor values, or in-cell couplings and the diagonal); where the colour's cells are coupled to
    // each other and the smoother makes more than one sweep, the residual comes from a separate pass, and the phase
    // reads it (4 or 8 B per row) instead
    case KK_GS_FINE64:  // the residual is given only where coupled cells of a color take a separate pass
      return ((given_resid ? 24.0 * n : 12.0 * nnz + 24.0 * n) +
              (h->opt.smoother ? 8.0 * h->fine.bfac_n : 12.0 * h->fine.ic_nnz + 8.0 * n)) / h->fine.ncolor;
    case KK_GS_FINE32:
      return ((given_resid ? 12.0 * n : 8.0 * nnz + 12.0 * n) +
              (h->opt.smoother ? 4.0 * h->fine.bfac_n : 8.0 * h->fine.ic_nnz + 4.0 * n)) / h->fine.ncolor;
    case KK_ENGINE64: return h->engine_flops[0];
    case KK_ENGINE32: return h->engine_flops[1];
  }
  return 0.0;
}

static amg_status read_scalars(amg_hierarchy *h, int first, int count) {
  const double *src = h->scal + static_cast<size_t>(h->nlev) * kScalars + first;
  QA_HIP(hipMemcpyAsync(h->host_scal + first, src, sizeof(double) * count, hipMemcpyDeviceToHost, h->stream));
  QA_HIP(hipStreamSynchronize(h->stream));
  return AMG_OK;
}

// Direction storage of the all-directions outer iteration (outer_mmax < 0): pairs (p_j, A p_j) of n doubles, made
// when first needed and kept by the hierarchy for later solves, with a device table of their addresses.
static amg_status outer_dirs_reserve(amg_hierarchy *h, int count) {
  const int cap = h->opt.max_iters;
  if (!h->dir_pp) {
    h->dir_pp = dalloc_n<double *>(h, cap);
    h->dir_zq = dalloc_n<double>(h, cap);
    h->dir_d = dalloc_n<double>(h, cap);
    if (!h->dir_pp || !h->dir_zq || !h->dir_d) return AMG_ERR_NOMEM;
  }
  if (count > cap) return AMG_ERR_INVALID;
  while (static_cast<int>(h->dir_p.size()) < count) {
    double *pj = dalloc_n<double>(h, h->n), *qj = dalloc_n<double>(h, h->n);
    if (!pj || !qj) return AMG_ERR_NOMEM;
    h->dir_p.push_back(pj);
    h->dir_q.push_back(qj);
    const size_t j = h->dir_p.size() - 1;
    QA_HIP(hipMemcpyAsync(h->dir_pp + j, &h->dir_p[j], sizeof(double *), hipMemcpyHostToDevice, h->stream));
    QA_HIP(hipStreamSynchronize(h->stream));  // the source is a host vector that may grow
  }
  return AMG_OK;
}

static amg_status solve_impl(amg_hierarchy *h, const double *b, double *x, double tol, amg_info *info) {
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t n = h->n;
  const FineLevel &F = h->fine;
  hipStream_t s = h->stream;
  const int L0 = h->nlev;  // outer scalar block
  const double *osc = h->scal + static_cast<size_t>(L0) * kScalars;
  const SliceSched Zall = slice_sched(F, 0, F.ncolor);
  const unsigned nsl_blocks = sched_grid(Zall);
  SellView<double> A64 = sview<double>(F, F.s_val64);
  amg_info inf{};
  inf.setup_ms = h->setup_ms;

  k_gather<double, double><<<nblk(n), kBlock, 0, s>>>(n, F.perm, b, h->bp);
  k_dot<double><<<nred(n), kBlock, 0, s>>>(n, h->bp, h->bp, red(h, L0, EPI_STORE, O_BB));
  finish<1>(h, nred(n), red(h, L0, EPI_STORE, O_BB));
  k_fill<double><<<nblk(n), kBlock, 0, s>>>(n, h->xp, 0.0);
  QA_LAUNCH_CHECK();
  QA_TRY(read_scalars(h, O_BB, 1));
  const double bn = std::sqrt(h->host_scal[O_BB]);
  if (bn == 0.0) {
    k_fill<double><<<nblk(n), kBlock, 0, s>>>(n, x, 0.0);
    QA_HIP(hipStreamSynchronize(s));
    inf.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return AMG_OK;
  }
  QA_HIP(hipMemcpyAsync(h->rp, h->bp, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  amg_status st = AMG_ERR_NOCONV;
  int it = 0;
  bool have_prev = false;
  double *p = h->pp, *q = h->qp, *pprev = h->pprev, *qprev = h->qprev;
  const int prec = h->precision;
  const bool all_dirs = h->opt.outer_mmax < 0;
  int stored = 0;  // all-directions form: directions kept since the start or the last restart
  while (it < h->opt.max_iters) {
    QA_TRY(precond_apply(h, prec, h->rp, h->zp));
    if (all_dirs) {
      QA_TRY(outer_dirs_reserve(h, stored + 1));
      p = h->dir_p[stored];
      q = h->dir_q[stored];
      for (int j = 0; j < stored; j++) {
        const Red R{h->partials, h->dir_zq, EPI_STORE, j};
        k_dot<double><<<nred(n), kBlock, 0, s>>>(n, h->zp, h->dir_q[j], R);
        finish<1>(h, nred(n), R);
      }
      k_outer_dir_all<<<nblk(n), kBlock, 0, s>>>(n, h->zp, h->dir_pp, h->dir_zq, h->dir_d, stored, p);
    } else {
      const bool use_beta = have_prev && h->opt.outer_mmax == 1;
      if (use_beta) {
        k_dot<double><<<nred(n), kBlock, 0, s>>>(n, h->zp, qprev, red(h, L0, EPI_OUT_BETA));
        finish<1>(h, nred(n), red(h, L0, EPI_OUT_BETA));
      }
      k_outer_dir<double><<<nblk(n), kBlock, 0, s>>>(n, osc, h->zp, pprev, p, use_beta ? 1 : 0);
    }
    launch_timed(h, KK_SPMV64, k_outer_spmv_dot, nsl_blocks, A64, Zall, static_cast<const double *>(p), q,
                 static_cast<const double *>(h->rp), red(h, L0, EPI_OUT_ALPHA));
    finish<2>(h, nsl_blocks, red(h, L0, EPI_OUT_ALPHA));
    k_outer_update<<<nred(n), kBlock, 0, s>>>(n, osc, p, q, h->xp, h->rp, red(h, L0, EPI_STORE, O_RR));
    finish<1>(h, nred(n), red(h, L0, EPI_STORE, O_RR));
    QA_LAUNCH_CHECK();
    QA_TRY(read_scalars(h, 0, O_BB));
    if (h->host_scal[O_BREAK] != 0.0) {
      st = AMG_ERR_BREAKDOWN;
      break;
    }
    it++;
    if (all_dirs) {  // keep (p, q) and (p, A p) of this step
      QA_HIP(hipMemcpyAsync(h->dir_d + stored, osc + O_D, sizeof(double), hipMemcpyDeviceToDevice, s));
      stored++;
    } else {
      have_prev = true;
      std::swap(p, pprev);
      std::swap(q, qprev);
    }
    if (std::sqrt(h->host_scal[O_RR]) <= tol * bn) {
      k_outer_true_resid<<<nsl_blocks, kBlock, 0, s>>>(A64, Zall, h->bp, h->xp, h->tp,
                                                        red(h, L0, EPI_STORE, O_TT));
      finish<1>(h, nsl_blocks, red(h, L0, EPI_STORE, O_TT));
      QA_LAUNCH_CHECK();
      QA_TRY(read_scalars(h, O_TT, 1));
      if (std::sqrt(h->host_scal[O_TT]) <= tol * bn) {
        st = AMG_OK;
        break;
      }
      QA_HIP(hipMemcpyAsync(h->rp, h->tp, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
      have_prev = false;
      stored = 0;
      inf.restarts++;
    }
  }
  k_outer_true_resid<<<nsl_blocks, kBlock, 0, s>>>(A64, Zall, h->bp, h->xp, h->tp, red(h, L0, EPI_STORE, O_TT));
  finish<1>(h, nsl_blocks, red(h, L0, EPI_STORE, O_TT));
  k_scatter_back<double, double><<<nblk(n), kBlock, 0, s>>>(n, F.perm, h->xp, x);
  QA_LAUNCH_CHECK();
  QA_TRY(read_scalars(h, O_TT, 1));
  inf.iters = it;
  inf.relres = std::sqrt(h->host_scal[O_TT]) / bn;
  inf.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return st;
}

// ---------------------------------------------------------------------------------------------------------------
// level hooks (tests): vectors in canonical numbering

template <class T>
static amg_status level_smooth_t(amg_hierarchy *h, int level, const double *f, double *x, int forward) {
  hipStream_t s = h->stream;
  std::vector<LevelWork<T>> &W = P<T>::W(h);
  if (level == 0) {
    const FineLevel &F = h->fine;
    const int64_t n = F.n;
    T *ff = W[0].f, *xx = W[0].u;
    k_gather<double, T><<<nblk(n), kBlock, 0, s>>>(n, F.perm, f, ff);
    k_gather<double, T><<<nblk(n), kBlock, 0, s>>>(n, F.perm, x, xx);
    const int nc = h->fine.ncolor;
    for (int c = 0; c < nc; c++) fine_phase<T>(h, ff, xx, W[0].d, forward ? c : nc - 1 - c, forward != 0, false);
    k_scatter_back<T, double><<<nblk(n), kBlock, 0, s>>>(n, F.perm, xx, x);
  } else {
    const QuadLevel &Q = h->lev[level];
    const int dim = h->dim, nc = 1 << dim;
    T *ff = W[level].r, *xx = W[level].p0;
    k_lex_to_q<double, T><<<nblk(Q.n), kBlock, 0, s>>>(Q.k, Q.n, f, ff, 0, dim);
    k_lex_to_q<double, T><<<nblk(Q.n), kBlock, 0, s>>>(Q.k, Q.n, x, xx, 0, dim);
    for (int c = 0; c < nc; c++) {
      if (dim == 3) gs_phase_oct<T>(h, level, ff, xx, forward ? c : nc - 1 - c);
      else gs_phase_coarse<T>(h, level, ff, xx, forward ? c : nc - 1 - c);
    }
    k_lex_to_q<T, double><<<nblk(Q.n), kBlock, 0, s>>>(Q.k, Q.n, xx, x, 1, dim);
  }
  QA_LAUNCH_CHECK();
  QA_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

amg_status level_smooth_internal(amg_hierarchy *h, int level, const double *f, double *x, int forward, int prec) {
  return prec == 1 ? level_smooth_t<float>(h, level, f, x, forward) : level_smooth_t<double>(h, level, f, x, forward);
}

template <class T>
static amg_status level_spmv_t(amg_hierarchy *h, int level, const double *x, double *y) {
  hipStream_t s = h->stream;
  std::vector<LevelWork<T>> &W = P<T>::W(h);
  if (level == 0) {
    const FineLevel &F = h->fine;
    const int64_t n = F.n;
    T *xx = W[0].f, *yy = W[0].u;
    k_gather<double, T><<<nblk(n), kBlock, 0, s>>>(n, F.perm, x, xx);
    const SliceSched Z = slice_sched(F, 0, F.ncolor);
    k_fine_apply<T><<<sched_grid(Z), kBlock, 0, s>>>(sview<T>(F, P<T>::sval(F)), Z, xx, yy);
    k_scatter_back<T, double><<<nblk(n), kBlock, 0, s>>>(n, F.perm, yy, y);
    QA_LAUNCH_CHECK();
    QA_HIP(hipStreamSynchronize(s));
    return AMG_OK;
  }
  const QuadLevel &Q = h->lev[level];
  const int dim = h->dim;
  T *xx = W[level].g, *yy = W[level].e;
  k_lex_to_q<double, T><<<nblk(Q.n), kBlock, 0, s>>>(Q.k, Q.n, x, xx, 0, dim);
  if (dim == 3) {
    k_capply3<T><<<nblk(Q.n), kBlock, 0, s>>>(qview<T>(Q), xx, yy);
  } else {
    // reuse the dot kernel's SpMV (the inner products are discarded into the scratch slot of level 0)
    k_cspmv_dot<T><<<nred(Q.n), kBlock, 0, s>>>(qview<T>(Q), xx, yy, xx, red(h, h->nlev, EPI_STORE, 15));
    finish<2>(h, nred(Q.n), red(h, h->nlev, EPI_STORE, 15));
  }
  k_lex_to_q<T, double><<<nblk(Q.n), kBlock, 0, s>>>(Q.k, Q.n, yy, y, 1, dim);
  QA_LAUNCH_CHECK();
  QA_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

amg_status level_spmv_internal(amg_hierarchy *h, int level, const double *x, double *y, int prec) {
  return prec == 1 ? level_spmv_t<float>(h, level, x, y) : level_spmv_t<double>(h, level, x, y);
}

}  // namespace qa

using namespace qa;

extern "C" amg_status amg_solve(amg_hierarchy *h, const double *b, double *x, double tol, amg_info *info) {
  if (!h || !b || !x || !(tol > 0.0) || !std::isfinite(tol) || h->stale) return AMG_ERR_INVALID;
  QA_HIP(hipSetDevice(h->device));
  const amg_status st = solve_impl(h, b, x, tol, info);
  if (info) info->status = st;
  return st;
}

extern "C" amg_status amg_apply_precond(amg_hierarchy *h, const double *r, double *z, int32_t precision) {
  if (!h || !r || !z || (precision != 0 && precision != 1) || h->stale) return AMG_ERR_INVALID;
  QA_HIP(hipSetDevice(h->device));
  const int64_t n = h->n;
  hipStream_t s = h->stream;
  k_gather<double, double><<<nblk(n), kBlock, 0, s>>>(n, h->fine.perm, r, h->tp);
  QA_TRY(precond_apply(h, precision, h->tp, h->zp));
  k_scatter_back<double, double><<<nblk(n), kBlock, 0, s>>>(n, h->fine.perm, h->zp, z);
  QA_LAUNCH_CHECK();
  QA_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

extern "C" amg_status amg_level_smooth(amg_hierarchy *h, int32_t level, const double *f, double *x, int32_t forward,
                                       int32_t precision) {
  if (!h || !f || !x || level < 0 || level >= h->nlev - 1 || h->nlev == 1 || (precision != 0 && precision != 1) ||
      h->stale)
    return AMG_ERR_INVALID;
  QA_HIP(hipSetDevice(h->device));
  return level_smooth_internal(h, level, f, x, forward, precision);
}

extern "C" amg_status amg_level_spmv(amg_hierarchy *h, int32_t level, const double *x, double *y, int32_t precision) {
  if (!h || !x || !y || level < 0 || level >= h->nlev || (precision != 0 && precision != 1) || h->stale)
    return AMG_ERR_INVALID;
  if (level == 0 && h->nlev == 1 && precision == 1) return AMG_ERR_INVALID;
  QA_HIP(hipSetDevice(h->device));
  return level_spmv_internal(h, level, x, y, precision);
}

namespace qa {

template <class T>
static void fill_wg(amg_hierarchy *h, const double *b, double *x, double tol, double *info, WgSys<T> &Y) {
  const int pi = std::is_same<T, float>::value ? 1 : 0;
  const FineLevel &F = h->fine;
  Y.n = static_cast<int>(h->n);
  Y.L = h->L;
  Y.nslices = static_cast<int>(F.nslices);
  for (int c = 0; c < 5; c++) { Y.color_row[c] = F.color_row[c]; Y.color_slice[c] = F.color_slice[c]; }
  Y.slice_ptr = F.slice_ptr; Y.slice_row0 = F.slice_row0; Y.s_row = F.s_row; Y.s_col = F.s_col;
  Y.s_val = P<T>::sval(F); Y.s_val64 = F.s_val64; Y.diag = P<T>::diag(F);
  Y.ic_ptr = F.ic_ptr; Y.ic_col = F.ic_col; Y.ic_val = P<T>::icv(F);
  Y.crow = F.crow; Y.agg_q = F.agg_q; Y.perm = F.perm;
  Y.b = b; Y.x = x;
  Y.xp = h->xp; Y.rp = h->rp; Y.bp = h->bp; Y.zp = h->zp; Y.tp = h->tp;
  Y.pv[0] = h->pp; Y.pv[1] = h->pprev; Y.qv[0] = h->qp; Y.qv[1] = h->qprev;
  LevelWork<T> &w0 = P<T>::W(h)[0];
  Y.f = w0.f; Y.u = w0.u; Y.d = w0.d;
  Y.info = info;
  Y.tol = tol;
  Y.max_iters = h->opt.max_iters;
  Y.mmax = h->opt.outer_mmax;
  Y.sweeps = h->opt.sweeps;
  Y.E = EngPlan<T>{};
  fill_engine(h, 1, h->wg_lds_top[pi], h->wg_ainv_lds[pi], Y.E);
  Y.E.nops = h->wg_nops[pi];
  Y.E.ops = static_cast<const EngOp *>(h->wg_ops[pi]);
}

// one launch, one workgroup per system; info of system i -> out[4 i .. 4 i + 3]. buf: device memory of at least
// wg_batch_bytes<T>(ids.size()) bytes for the system descriptors and the info words.
template <class T>
static size_t wg_batch_bytes(size_t m) {
  return sizeof(WgSys<T>) * m + sizeof(double) * 4 * m;
}

// sys: host staging for the m descriptors, out: 4 m doubles
template <class T>
static amg_status launch_wg_batch_in(amg_hierarchy *const *hs, const double *const *b, double *const *x,
                                     const double *tol, const int *ids, int m, void *buf, WgSys<T> *sys,
                                     double *out) {
  const int pi = std::is_same<T, float>::value ? 1 : 0;
  hipStream_t s = hs[ids[0]]->stream;
  const size_t sys_bytes = sizeof(WgSys<T>) * m;
  double *info_d = reinterpret_cast<double *>(static_cast<char *>(buf) + sys_bytes);
  size_t lds = 0;
  for (int j = 0; j < m; j++) {
    const int i = ids[j];
    fill_wg<T>(hs[i], b[i], x[i], tol[i], info_d + 4 * j, sys[j]);
    lds = std::max(lds, hs[i]->wg_lds[pi]);
  }
  QA_HIP(hipMemcpyAsync(buf, sys, sys_bytes, hipMemcpyHostToDevice, s));
  k_solve_wg<T><<<m, kEngThreads, lds, s>>>(static_cast<const WgSys<T> *>(buf));
  QA_LAUNCH_CHECK();
  for (int j = 0; j < 4 * m; j++) out[j] = 0.0;
  QA_HIP(hipMemcpyAsync(out, info_d, sizeof(double) * 4 * m, hipMemcpyDeviceToHost, s));
  QA_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

template <class T>
static amg_status launch_wg_batch(amg_hierarchy *const *hs, const double *const *b, double *const *x,
                                  const double *tol, const std::vector<int> &ids, std::vector<double> &out) {
  QA_HIP(hipSetDevice(hs[ids[0]]->device));
  hipStream_t s = hs[ids[0]]->stream;
  void *buf = tmp_alloc(hs[ids[0]], s, wg_batch_bytes<T>(ids.size()));
  if (!buf) return AMG_ERR_NOMEM;
  std::vector<WgSys<T>> sys(ids.size());
  out.assign(4 * ids.size(), 0.0);
  const amg_status st =
      launch_wg_batch_in<T>(hs, b, x, tol, ids.data(), static_cast<int>(ids.size()), buf, sys.data(), out.data());
  tmp_free(hs[ids[0]], s, buf);  // on every path
  return st;
}

// Per-system results of whole-solve launches into st / inf.
static void wg_results(amg_hierarchy *const *hs, const int *ids, int m, const double *out, double ms,
                       amg_status *st, amg_info *inf) {
  for (int j = 0; j < m; j++) {
    const int i = ids[j];
    st[i] = static_cast<amg_status>(static_cast<int>(out[4 * j]));
    inf[i].iters = static_cast<int32_t>(out[4 * j + 1]);
    inf[i].restarts = static_cast<int32_t>(out[4 * j + 2]);
    inf[i].relres = out[4 * j + 3];
    inf[i].setup_ms = hs[i]->setup_ms;
    inf[i].solve_ms = ms;
  }
}

// Arguments of a batch call: each hierarchy given once, all on one device, every input present.
static amg_status check_batch_args(amg_hierarchy *const *hs, const double *const *b, double *const *x,
                                   const double *tol, int32_t count) {
  if (count < 0 || (count > 0 && (!hs || !b || !x || !tol))) return AMG_ERR_INVALID;
  for (int32_t i = 0; i < count; i++) {
    if (!hs[i] || !b[i] || !x[i] || !(tol[i] > 0.0) || !std::isfinite(tol[i]) || hs[i]->stale) return AMG_ERR_INVALID;
    for (int32_t j = 0; j < i; j++)
      if (hs[j] == hs[i]) return AMG_ERR_INVALID;  // one workspace per hierarchy
    if (hs[i]->device != hs[0]->device) return AMG_ERR_INVALID;
  }
  return AMG_OK;
}

// ---------------------------------------------------------------------------------------------------------------
// Batch solve without allocation. The system descriptors and info words of the whole-solve launches live in a
// file-scope device array instead of memory allocated per call. The array's name is only a host-side handle: its
// device address is looked up once per device (with that device current) and every use goes through that address.

constexpr int kNoAllocMaxSystems = 256;
constexpr size_t kNoAllocBytes =
    (std::max(sizeof(WgSys<double>), sizeof(WgSys<float>)) + sizeof(double) * 4) * kNoAllocMaxSystems;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];
static std::once_flag g_scratch_once[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices];

// device address of `scratch` on `device` (made current by the caller), or null
static void *scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::call_once(g_scratch_once[device], [device]() {
    void *p = nullptr;
    g_scratch_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[device] = g_scratch_err[device] == hipSuccess ? p : nullptr;
  });
  return g_scratch_ptr[device];
}

// Host staging of the calls, also static (no heap use per call). Calls are serialised by g_noalloc_mu: they share
// these arrays and, on one device, the device array.
struct NoAllocStage {
  WgSys<double> sys64[kNoAllocMaxSystems];
  WgSys<float> sys32[kNoAllocMaxSystems];
  double out[4 * kNoAllocMaxSystems];
  int ids[2][kNoAllocMaxSystems];
  amg_status st[kNoAllocMaxSystems];
  amg_info inf[kNoAllocMaxSystems];
};
static NoAllocStage g_stage;
static std::mutex g_noalloc_mu;

}  // namespace qa

extern "C" amg_status amg_solve_batch(amg_hierarchy *const *hs, const double *const *b, double *const *x,
                                      const double *tol, int32_t count, amg_info *info) {
  QA_TRY(check_batch_args(hs, b, x, tol, count));
  if (count == 0) return AMG_OK;
  const auto t0 = std::chrono::steady_clock::now();
  // inputs are complete once each hierarchy's stream has drained
  for (int32_t i = 0; i < count; i++) {
    QA_HIP(hipSetDevice(hs[i]->device));
    QA_HIP(hipStreamSynchronize(hs[i]->stream));
  }
  std::vector<int> small[2], large;
  for (int32_t i = 0; i < count; i++) {
    const int pi = hs[i]->precision;
    if (hs[i]->use_batch && hs[i]->wg_nops[pi] > 0) small[pi].push_back(i);
    else large.push_back(i);
  }
  std::vector<amg_status> st(count, AMG_OK);
  std::vector<amg_info> inf(count);
  std::vector<std::thread> threads;
  for (int i : large)
    threads.emplace_back([&, i]() {
      if (hipSetDevice(hs[i]->device) != hipSuccess) { st[i] = AMG_ERR_DEVICE; return; }
      st[i] = amg_solve(hs[i], b[i], x[i], tol[i], &inf[i]);
    });
  amg_status launch_st = AMG_OK;
  for (int pi = 0; pi < 2 && launch_st == AMG_OK; pi++) {
    if (small[pi].empty()) continue;
    std::vector<double> out;
    launch_st = pi == 0 ? launch_wg_batch<double>(hs, b, x, tol, small[pi], out)
                        : launch_wg_batch<float>(hs, b, x, tol, small[pi], out);
    if (launch_st != AMG_OK) break;
    wg_results(hs, small[pi].data(), static_cast<int>(small[pi].size()), out.data(),
               std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count(), st.data(),
               inf.data());
  }
  for (auto &t : threads) t.join();
  amg_status first = launch_st;
  for (int32_t i = 0; i < count; i++) {
    if (launch_st != AMG_OK && std::find(large.begin(), large.end(), i) == large.end()) st[i] = launch_st;
    inf[i].status = st[i];
    if (info) info[i] = inf[i];
    if (first == AMG_OK && st[i] != AMG_OK) first = st[i];
  }
  return first;
}

extern "C" amg_status amg_solve_batch_noalloc(amg_hierarchy *const *hs, const double *const *b, double *const *x,
                                              const double *tol, int32_t count, amg_info *info) {
  QA_TRY(check_batch_args(hs, b, x, tol, count));
  if (count > kNoAllocMaxSystems) return AMG_ERR_INVALID;
  if (count == 0) return AMG_OK;
  for (int32_t i = 0; i < count; i++) {
    const int pi = hs[i]->precision;
    if (!(hs[i]->use_batch && hs[i]->wg_nops[pi] > 0)) return AMG_ERR_INVALID;  // only whole-solve systems
  }
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  NoAllocStage &G = g_stage;
  int nsmall[2] = {0, 0};
  for (int32_t i = 0; i < count; i++) {
    const int pi = hs[i]->precision;
    G.ids[pi][nsmall[pi]++] = i;
    G.st[i] = AMG_OK;
    G.inf[i] = amg_info{};
  }
  const auto t0 = std::chrono::steady_clock::now();
  QA_HIP(hipSetDevice(hs[0]->device));
  char *base = static_cast<char *>(scratch_ptr(hs[0]->device));
  if (!base) return AMG_ERR_DEVICE;
  for (int32_t i = 0; i < count; i++) QA_HIP(hipStreamSynchronize(hs[i]->stream));
  // the FP64 group's descriptors first, the FP32 group's after them: disjoint parts of the array
  const size_t off[2] = {0, wg_batch_bytes<double>(nsmall[0])};
  amg_status first = AMG_OK;
  for (int pi = 0; pi < 2 && first == AMG_OK; pi++) {
    if (nsmall[pi] == 0) continue;
    first = pi == 0 ? launch_wg_batch_in<double>(hs, b, x, tol, G.ids[0], nsmall[0], base + off[0], G.sys64, G.out)
                    : launch_wg_batch_in<float>(hs, b, x, tol, G.ids[1], nsmall[1], base + off[1], G.sys32, G.out);
    if (first == AMG_OK)
      wg_results(hs, G.ids[pi], nsmall[pi], G.out,
                 std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count(), G.st,
                 G.inf);
  }
  for (int32_t i = 0; i < count; i++) {
    if (first != AMG_OK) G.st[i] = first;
    G.inf[i].status = G.st[i];
    if (info) info[i] = G.inf[i];
    if (first == AMG_OK && G.st[i] != AMG_OK) first = G.st[i];
  }
  return first;
}

extern "C" amg_status amg_kernel_timing_enable(amg_hierarchy *h, const char *name) {
  if (!h) return AMG_ERR_INVALID;
  int kind = -1;
  if (name) {
    if (!std::strcmp(name, "spmv64")) kind = KK_SPMV64;
    else if (!std::strcmp(name, "gs_fine32")) kind = KK_GS_FINE32;
    else if (!std::strcmp(name, "gs_fine64")) kind = KK_GS_FINE64;
    else if (!std::strcmp(name, "resid_fine32")) kind = KK_RESID_FINE32;
    else if (!std::strcmp(name, "resid_fine64")) kind = KK_RESID_FINE64;
    else if (!std::strcmp(name, "engine32")) kind = KK_ENGINE32;
    else if (!std::strcmp(name, "engine64")) kind = KK_ENGINE64;
    else return AMG_ERR_INVALID;
  }
  QA_HIP(hipSetDevice(h->device));
  QA_HIP(hipStreamSynchronize(h->stream));
  Timing &t = h->timing;
  if (kind >= 0 && t.ev.empty()) QA_TRY(borrow_events(h->device, 2 * 4096, t.ev));
  if (kind < 0) return_events(h->device, t.ev);
  t.kind = kind;
  t.used = 0;
  t.launches = 0;
  t.total_ms = 0.0;
  t.bytes_per_launch = kind >= 0 ? kernel_bytes(h, kind) : 0.0;
  return AMG_OK;
}

extern "C" amg_status amg_kernel_timing_read(amg_hierarchy *h, int64_t *launches, double *total_ms,
                                             double *bytes_per_launch) {
  if (!h) return AMG_ERR_INVALID;
  QA_HIP(hipSetDevice(h->device));
  QA_HIP(hipStreamSynchronize(h->stream));
  Timing &t = h->timing;
  for (size_t i = 0; i + 1 < t.used; i += 2) {
    float ms = 0.f;
    QA_HIP(hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1]));
    t.total_ms += ms;
    t.launches++;
  }
  t.used = 0;
  if (launches) *launches = t.launches;
  if (total_ms) *total_ms = t.total_ms;
  if (bytes_per_launch) *bytes_per_launch = t.bytes_per_launch;
  return AMG_OK;
}

extern "C" amg_status amg_engine_info(const amg_hierarchy *h, int32_t precision, int32_t *top_level,
                                      int32_t *lds_level, int32_t *steps, size_t *lds_bytes) {
  if (!h || (precision != 0 && precision != 1)) return AMG_ERR_INVALID;
  const int pi = precision;
  if (top_level) *top_level = h->use_engine ? h->engine_top[pi] : -1;
  if (lds_level) *lds_level = h->engine_lds_top[pi];
  if (steps) *steps = h->engine_nops[pi];
  if (lds_bytes) *lds_bytes = h->engine_lds[pi];
  return AMG_OK;
}
