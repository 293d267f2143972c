// Linear-element (P1) stiffness assembly on the device for a fixed triangle mesh: the step before the hierarchy in
// time stepping (Example 2 of Section 5 advances one time step per solve). The pattern is built once per mesh; each
// step then assembles new values for new coefficients, to be handed to amg_update_values.
//
// Element matrix of -div(kappa grad u) on triangle T with vertices P0, P1, P2 (counter-clockwise after orientation):
// K_ab = kappa_T (E_a . E_b) / (4 |T|), E_a the edge opposite vertex a (E_0 = P2 - P1, E_1 = P0 - P2, E_2 = P1 - P0).
// Entries whose row or column vertex is eliminated (no unknown) are dropped; the rest are summed per (row, column).
//
// Fixed evaluation order (this file is compiled without floating-point contraction): element entry
// ((kappa * (E_a.x E_b.x + E_a.y E_b.y)) / (2 |2 area|)); the element entries of one stored (row, column) taken in
// the order (a, b, triangle), ascending; their sum is the first entry plus the sum of the others, that sum being
// sequential from 0 below eight terms and, from eight to 128 terms, eight interleaved partial sums combined as
// ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7)) followed by the remainder in order (pairwise summation with
// eight accumulators). This is the order of a stable sort of the element entries by (row, column) followed by
// NumPy's add.reduceat over the segments, so the host generator's assembly and this one agree bit for bit.
//
// The sort is a counting sort by row: each vertex's corners count their kept entries into the row of the vertex's
// unknown, an exclusive scan gives each row's first position, the corners drop their entries into their row's
// range in any order, and each entry's final place in its row is the number of entries of that row with a smaller
// (column, entry index) pair. The (row, column, entry index) order that results is the stable sort's, whatever
// order the atomics took.

#include <algorithm>

#include "qa_internal.hpp"

using namespace qa;

struct amg_p1_mesh {
  amg_hierarchy arena;       // used for its allocator only: device, stream and the tracked device blocks
  int64_t nv = 0, nt = 0, ndof = 0, nnz = 0, m = 0;  // m = 9 nt element entries
  int32_t *tri = nullptr;    // nt x 3 vertex ids, counter-clockwise
  double *pts = nullptr;     // nv x 2
  double *elem = nullptr;    // element entries, entry (a, b) of triangle t at (3 a + b) nt + t
  int32_t *perm = nullptr;   // element entry of each sorted position (stored entries' terms contiguous)
  int64_t *seg = nullptr;    // nnz + 1: first sorted position of each stored entry
  int64_t *row_ptr = nullptr;
  int32_t *col = nullptr;
};

namespace {

enum { F_INVALID = 1 };  // device error flag
constexpr int kAsmBlock = 256;
constexpr int64_t kMaxTerms = 128;  // element entries summed into one stored entry

inline unsigned ablk(int64_t n) { return static_cast<unsigned>((n + kAsmBlock - 1) / kAsmBlock); }

__device__ inline double area2_signed(const double *p, int32_t a, int32_t b, int32_t c) {
  const double ax = p[2 * a], ay = p[2 * a + 1];
  return (p[2 * b] - ax) * (p[2 * c + 1] - ay) - (p[2 * b + 1] - ay) * (p[2 * c] - ax);
}

// vertex ids in range, non-degenerate triangles, counter-clockwise order (vertices 1 and 2 swapped otherwise)
__global__ void __launch_bounds__(kAsmBlock) k_tri_orient(int64_t nt, int64_t nv, const int32_t *__restrict__ in,
                                                           const double *__restrict__ pts, int32_t *__restrict__ out,
                                                           int *flag) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  int32_t v[3];
  for (int k = 0; k < 3; k++) {
    v[k] = in[3 * t + k];
    if (v[k] < 0 || v[k] >= nv) {
      atomicOr(flag, F_INVALID);
      return;
    }
  }
  const double s = area2_signed(pts, v[0], v[1], v[2]);
  if (!(s != 0.0) || !isfinite(s)) atomicOr(flag, F_INVALID);
  out[3 * t] = v[0];
  out[3 * t + 1] = s < 0.0 ? v[2] : v[1];
  out[3 * t + 2] = s < 0.0 ? v[1] : v[2];
}

// unknown numbering: each entry -1 or in [0, ndof), each unknown taken by exactly one vertex
__global__ void __launch_bounds__(kAsmBlock) k_dof_count(int64_t nv, int64_t ndof, const int32_t *__restrict__ dof,
                                                          int32_t *__restrict__ cnt, int *flag) {
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  const int32_t d = dof[v];
  if (d < -1 || d >= ndof) atomicOr(flag, F_INVALID);
  else if (d >= 0) atomicAdd(&cnt[d], 1);
}

__global__ void __launch_bounds__(kAsmBlock) k_dof_once(int64_t ndof, const int32_t *__restrict__ cnt, int *flag) {
  const int64_t d = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (d < ndof && cnt[d] != 1) atomicOr(flag, F_INVALID);
}

// kept entries (a, b, t) of corner (a, t) whose vertex has an unknown: the b with an unknown
__device__ inline int corner_kept(const int32_t *tri, const int32_t *dof, int64_t t) {
  return (dof[tri[3 * t]] >= 0) + (dof[tri[3 * t + 1]] >= 0) + (dof[tri[3 * t + 2]] >= 0);
}

// per row, the number of kept element entries (corner i = a nt + t)
__global__ void __launch_bounds__(kAsmBlock) k_row_counts(int64_t nt, const int32_t *__restrict__ tri,
                                                           const int32_t *__restrict__ dof,
                                                           int32_t *__restrict__ cnt) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= 3 * nt) return;
  const int64_t t = i % nt;
  const int a = static_cast<int>(i / nt);
  const int32_t r = dof[tri[3 * t + a]];
  if (r >= 0) atomicAdd(&cnt[r], corner_kept(tri, dof, t));
}

// each corner's kept entries into its row's range, in arrival order: the pair (column, entry index) packed as
// column << 32 | index (both below 2^31) and the row of each position
__global__ void __launch_bounds__(kAsmBlock) k_row_fill(int64_t nt, const int32_t *__restrict__ tri,
                                                         const int32_t *__restrict__ dof,
                                                         const int32_t *__restrict__ start, int32_t *__restrict__ fill,
                                                         uint64_t *__restrict__ ckey, int32_t *__restrict__ rowid) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= 3 * nt) return;
  const int64_t t = i % nt;
  const int a = static_cast<int>(i / nt);
  const int32_t r = dof[tri[3 * t + a]];
  if (r < 0) return;
  int32_t p = start[r] + atomicAdd(&fill[r], corner_kept(tri, dof, t));
  for (int b = 0; b < 3; b++) {
    const int32_t c = dof[tri[3 * t + b]];
    if (c < 0) continue;
    const uint64_t e = static_cast<uint64_t>((3 * a + b) * nt + t);
    ckey[p] = (static_cast<uint64_t>(c) << 32) | e;
    rowid[p] = r;
    p++;
  }
}

// each kept entry to its place: its row's first position plus the number of that row's entries with a smaller
// (column, entry index); the sorted key row * ndof + column and the entry index
__global__ void __launch_bounds__(kAsmBlock) k_row_rank(int64_t mk, int64_t ndof, const int32_t *__restrict__ start,
                                                         const uint64_t *__restrict__ ckey,
                                                         const int32_t *__restrict__ rowid,
                                                         uint64_t *__restrict__ key, int32_t *__restrict__ perm) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= mk) return;
  const int32_t r = rowid[p];
  const uint64_t k = ckey[p];
  const int32_t lo = start[r], hi = start[r + 1];
  int32_t rank = 0;
  for (int32_t q = lo; q < hi; q++) rank += ckey[q] < k;
  key[lo + rank] = static_cast<uint64_t>(r) * static_cast<uint64_t>(ndof) + (k >> 32);
  perm[lo + rank] = static_cast<int32_t>(k & 0xffffffffu);
}

// positions past the kept entries: key `drop` (they close the last segment), entry index 0 (never summed)
__global__ void __launch_bounds__(kAsmBlock) k_drop_tail(int64_t mk, int64_t m, uint64_t drop,
                                                          uint64_t *__restrict__ key, int32_t *__restrict__ perm) {
  const int64_t p = mk + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= m) return;
  key[p] = drop;
  perm[p] = 0;
}

// first sorted position of each distinct kept key
__global__ void __launch_bounds__(kAsmBlock) k_heads(int64_t m, const uint64_t *__restrict__ key, uint64_t drop,
                                                      int32_t *__restrict__ head) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  head[i] = (key[i] != drop && (i == 0 || key[i] != key[i - 1])) ? 1 : 0;
}

// stored entry s = pos[i] of each head i: its column, first position and its row's count; the end of the kept keys
// closes the last segment
__global__ void __launch_bounds__(kAsmBlock) k_segments(int64_t m, int64_t ndof, int64_t nnz,
                                                         const uint64_t *__restrict__ key, uint64_t drop,
                                                         const int32_t *__restrict__ head,
                                                         const int32_t *__restrict__ pos, int64_t *__restrict__ seg,
                                                         int32_t *__restrict__ col, int64_t *__restrict__ rowcnt) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint64_t k = key[i];
  if (head[i]) {
    const int64_t s = pos[i];
    seg[s] = i;
    col[s] = static_cast<int32_t>(k % static_cast<uint64_t>(ndof));
    atomicAdd(reinterpret_cast<unsigned long long *>(&rowcnt[k / static_cast<uint64_t>(ndof)]), 1ull);
  }
  if (k != drop && (i == m - 1 || key[i + 1] == drop)) seg[nnz] = i + 1;
}

__global__ void __launch_bounds__(kAsmBlock) k_seg_limit(int64_t nnz, const int64_t *__restrict__ seg, int *flag) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s < nnz && seg[s + 1] - seg[s] > kMaxTerms) atomicOr(flag, F_INVALID);
}

// the nine element entries of each triangle
__global__ void __launch_bounds__(kAsmBlock) k_elements(int64_t nt, const int32_t *__restrict__ tri,
                                                         const double *__restrict__ pts,
                                                         const double *__restrict__ kappa,
                                                         double *__restrict__ elem) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const int32_t v0 = tri[3 * t], v1 = tri[3 * t + 1], v2 = tri[3 * t + 2];
  const double denom = 2.0 * fabs(area2_signed(pts, v0, v1, v2));
  const double ex[3] = {pts[2 * v2] - pts[2 * v1], pts[2 * v0] - pts[2 * v2], pts[2 * v1] - pts[2 * v0]};
  const double ey[3] = {pts[2 * v2 + 1] - pts[2 * v1 + 1], pts[2 * v0 + 1] - pts[2 * v2 + 1],
                        pts[2 * v1 + 1] - pts[2 * v0 + 1]};
  const double kap = kappa ? kappa[t] : 1.0;
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) elem[(3 * a + b) * nt + t] = kap * (ex[a] * ex[b] + ey[a] * ey[b]) / denom;
}

// each stored entry: the first term plus the others' sum, in the order stated at the top of this file
__global__ void __launch_bounds__(kAsmBlock) k_entry_sums(int64_t nnz, const int64_t *__restrict__ seg,
                                                           const int32_t *__restrict__ perm,
                                                           const double *__restrict__ elem,
                                                           double *__restrict__ val) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= nnz) return;
  const int64_t a = seg[s], n = seg[s + 1] - a - 1;  // n terms after the first
  const double first = elem[perm[a]];
  const int32_t *q = perm + a + 1;
  double rest = 0.0;
  if (n < 8) {
    for (int64_t i = 0; i < n; i++) rest += elem[q[i]];
  } else {
    double p[8];
    for (int j = 0; j < 8; j++) p[j] = elem[q[j]];
    int64_t i = 8;
    for (; i + 8 <= n; i += 8)
      for (int j = 0; j < 8; j++) p[j] += elem[q[i + j]];
    rest = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
    for (; i < n; i++) rest += elem[q[i]];
  }
  val[s] = n > 0 ? first + rest : first;
}

// stream-ordered temporary device buffer, returned when it leaves scope
struct Temp {
  void *p = nullptr;
  hipStream_t s;
  explicit Temp(hipStream_t st) : s(st) {}
  bool get(size_t bytes) { return hipMallocAsync(&p, std::max<size_t>(bytes, 256), s) == hipSuccess; }
  ~Temp() {
    if (p) (void)hipFreeAsync(p, s);
  }
  template <class T>
  T *as() const { return static_cast<T *>(p); }
};

amg_status read_flag(amg_p1_mesh *M, int *dflag, int &f) {
  QA_HIP(hipMemcpyAsync(&f, dflag, sizeof(int), hipMemcpyDeviceToHost, M->arena.stream));
  QA_HIP(hipStreamSynchronize(M->arena.stream));
  return AMG_OK;
}

amg_status mesh_build(amg_p1_mesh *M, const double *points, const int32_t *tris, const int32_t *dof) {
  amg_hierarchy *h = &M->arena;
  hipStream_t s = h->stream;
  const int64_t nv = M->nv, nt = M->nt, ndof = M->ndof, m = M->m;
  int *dflag = dalloc_n<int>(h, 1);
  M->pts = dalloc_n<double>(h, 2 * nv);
  M->tri = dalloc_n<int32_t>(h, 3 * nt);
  M->elem = dalloc_n<double>(h, m);
  M->perm = dalloc_n<int32_t>(h, m);
  M->row_ptr = dalloc_n<int64_t>(h, ndof + 1);
  if (!dflag || !M->pts || !M->tri || !M->elem || !M->perm || !M->row_ptr) return AMG_ERR_NOMEM;
  QA_HIP(hipMemsetAsync(dflag, 0, sizeof(int), s));
  QA_HIP(hipMemcpyAsync(M->pts, points, sizeof(double) * 2 * nv, hipMemcpyDeviceToDevice, s));
  Temp cnt(s), start(s), key2(s), ckey(s), rowid(s), head(s), pos(s), rowcnt(s);
  if (!cnt.get(sizeof(int32_t) * ndof)) return AMG_ERR_NOMEM;
  QA_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * ndof, s));
  k_tri_orient<<<ablk(nt), kAsmBlock, 0, s>>>(nt, nv, tris, M->pts, M->tri, dflag);
  k_dof_count<<<ablk(nv), kAsmBlock, 0, s>>>(nv, ndof, dof, cnt.as<int32_t>(), dflag);
  k_dof_once<<<ablk(ndof), kAsmBlock, 0, s>>>(ndof, cnt.as<int32_t>(), dflag);
  QA_LAUNCH_CHECK();
  int f = 0;
  QA_TRY(read_flag(M, dflag, f));
  if (f) return AMG_ERR_INVALID;
  // stable sort of the element entries by (row, column): equal keys keep the (a, b, triangle) order; entries with
  // a vertex without unknown are dropped (key `drop` after the kept ones)
  const uint64_t drop = static_cast<uint64_t>(ndof) * static_cast<uint64_t>(ndof);
  if (!start.get(4 * (ndof + 1)) || !key2.get(8 * m)) return AMG_ERR_NOMEM;
  QA_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * ndof, s));
  k_row_counts<<<ablk(3 * nt), kAsmBlock, 0, s>>>(nt, M->tri, dof, cnt.as<int32_t>());
  QA_LAUNCH_CHECK();
  QA_TRY(scan_exclusive_i32(cnt.as<int32_t>(), start.as<int32_t>(), ndof, s, h));
  int32_t mk = 0;
  QA_HIP(hipMemcpyAsync(&mk, start.as<int32_t>() + ndof, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  QA_HIP(hipStreamSynchronize(s));
  if (mk < 0 || mk > m) return AMG_ERR_INVALID;
  if (!ckey.get(8 * static_cast<size_t>(mk)) || !rowid.get(4 * static_cast<size_t>(mk))) return AMG_ERR_NOMEM;
  QA_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * ndof, s));  // reused as the fill counters
  k_row_fill<<<ablk(3 * nt), kAsmBlock, 0, s>>>(nt, M->tri, dof, start.as<int32_t>(), cnt.as<int32_t>(),
                                                ckey.as<uint64_t>(), rowid.as<int32_t>());
  if (mk) k_row_rank<<<ablk(mk), kAsmBlock, 0, s>>>(mk, ndof, start.as<int32_t>(), ckey.as<uint64_t>(),
                                                    rowid.as<int32_t>(), key2.as<uint64_t>(), M->perm);
  if (mk < m) k_drop_tail<<<ablk(m - mk), kAsmBlock, 0, s>>>(mk, m, drop, key2.as<uint64_t>(), M->perm);
  // distinct kept keys are the stored entries, already in row-major, column-ascending order
  if (!head.get(4 * m) || !pos.get(4 * (m + 1)) || !rowcnt.get(8 * ndof)) return AMG_ERR_NOMEM;
  k_heads<<<ablk(m), kAsmBlock, 0, s>>>(m, key2.as<uint64_t>(), drop, head.as<int32_t>());
  QA_LAUNCH_CHECK();
  QA_TRY(scan_exclusive_i32(head.as<int32_t>(), pos.as<int32_t>(), m, s, h));
  int32_t nnz = 0;
  QA_HIP(hipMemcpyAsync(&nnz, pos.as<int32_t>() + m, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  QA_HIP(hipStreamSynchronize(s));
  M->nnz = nnz;
  M->seg = dalloc_n<int64_t>(h, M->nnz + 1);
  M->col = dalloc_n<int32_t>(h, M->nnz);
  if (!M->seg || !M->col) return AMG_ERR_NOMEM;
  QA_HIP(hipMemsetAsync(M->seg, 0, sizeof(int64_t) * (M->nnz + 1), s));
  QA_HIP(hipMemsetAsync(rowcnt.p, 0, sizeof(int64_t) * ndof, s));
  k_segments<<<ablk(m), kAsmBlock, 0, s>>>(m, ndof, M->nnz, key2.as<uint64_t>(), drop, head.as<int32_t>(),
                                           pos.as<int32_t>(), M->seg, M->col, rowcnt.as<int64_t>());
  if (M->nnz) k_seg_limit<<<ablk(M->nnz), kAsmBlock, 0, s>>>(M->nnz, M->seg, dflag);
  QA_LAUNCH_CHECK();
  QA_TRY(scan_exclusive_i64(rowcnt.as<int64_t>(), M->row_ptr, ndof, s, h));
  QA_TRY(read_flag(M, dflag, f));
  if (f) return AMG_ERR_INVALID;  // a stored entry would sum more than kMaxTerms element entries
  return AMG_OK;
}

}  // namespace

extern "C" amg_status amg_p1_mesh_create(int64_t nv, const double *points, int64_t nt, const int32_t *tris,
                                         const int32_t *dof, int64_t ndof, void *stream, amg_p1_mesh **out) {
  if (!out) return AMG_ERR_INVALID;
  *out = nullptr;
  if (nv < 1 || nt < 1 || ndof < 1 || ndof > nv || nv > (static_cast<int64_t>(1) << 31) - 2 ||
      9 * nt > (static_cast<int64_t>(1) << 31) - 2 || !points || !tris || !dof)
    return AMG_ERR_INVALID;
  amg_p1_mesh *M = new (std::nothrow) amg_p1_mesh();
  if (!M) return AMG_ERR_NOMEM;
  if (hipGetDevice(&M->arena.device) != hipSuccess) {
    delete M;
    return AMG_ERR_DEVICE;
  }
  M->arena.stream = static_cast<hipStream_t>(stream);
  M->arena.chunk_unit = static_cast<size_t>(4) << 20;
  M->nv = nv;
  M->nt = nt;
  M->ndof = ndof;
  M->m = 9 * nt;
  const amg_status st = mesh_build(M, points, tris, dof);
  (void)hipStreamSynchronize(M->arena.stream);  // the temporaries' frees are ordered after their last use
  if (st != AMG_OK) {
    release(&M->arena);
    delete M;
    return st;
  }
  *out = M;
  return AMG_OK;
}

extern "C" amg_status amg_p1_mesh_pattern(const amg_p1_mesh *M, int64_t *nnz, int64_t *row_ptr, int32_t *col_idx) {
  if (!M || !nnz) return AMG_ERR_INVALID;
  *nnz = M->nnz;
  QA_HIP(hipSetDevice(M->arena.device));
  hipStream_t s = M->arena.stream;
  if (row_ptr)
    QA_HIP(hipMemcpyAsync(row_ptr, M->row_ptr, sizeof(int64_t) * (M->ndof + 1), hipMemcpyDeviceToDevice, s));
  if (col_idx && M->nnz)
    QA_HIP(hipMemcpyAsync(col_idx, M->col, sizeof(int32_t) * M->nnz, hipMemcpyDeviceToDevice, s));
  QA_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

extern "C" amg_status amg_p1_assemble(amg_p1_mesh *M, const double *kappa, double *vals) {
  if (!M || !vals) return AMG_ERR_INVALID;
  QA_HIP(hipSetDevice(M->arena.device));
  hipStream_t s = M->arena.stream;
  k_elements<<<ablk(M->nt), kAsmBlock, 0, s>>>(M->nt, M->tri, M->pts, kappa, M->elem);
  if (M->nnz) k_entry_sums<<<ablk(M->nnz), kAsmBlock, 0, s>>>(M->nnz, M->seg, M->perm, M->elem, vals);
  QA_LAUNCH_CHECK();
  QA_HIP(hipStreamSynchronize(s));
  return AMG_OK;
}

extern "C" void amg_p1_mesh_free(amg_p1_mesh *M) {
  if (!M) return;
  (void)hipSetDevice(M->arena.device);
  release(&M->arena);
  delete M;
}
