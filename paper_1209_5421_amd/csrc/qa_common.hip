// Runtime pieces shared by setup and solve: tracked device allocation, exclusive scans, release, status names.
#include <algorithm>
#include <mutex>

#include "qa_internal.hpp"

namespace qa {

static std::mutex g_pool_mu;  // guards the per-device pools below (setups may run on several host threads)

// Hierarchy memory comes from a library-owned stream-ordered pool per device that keeps freed blocks cached, so
// repeated setup / free cycles (a request stream) do not pay hipMalloc / hipFree each time.
static hipMemPool_t pool_for(int device) {
  static hipMemPool_t pools[64] = {};
  static bool ready[64] = {};
  if (device < 0 || device >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(g_pool_mu);
  if (!ready[device]) {
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = device;
    hipMemPool_t p = nullptr;
    if (hipMemPoolCreate(&p, &props) == hipSuccess) {
      uint64_t keep = ~0ull;
      (void)hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep);
      pools[device] = p;
    }
    ready[device] = true;
  }
  return pools[device];
}

// Allocations of freed hierarchies are kept per device (up to kCacheCap bytes) and handed to the next allocation of
// exactly the same size: a request stream re-creates hierarchies of the sizes it has seen (repeated meshes, the
// benchmark's steps), and each stream-ordered free and allocation costs tens of microseconds of driver time. A block
// enters the cache only after its hierarchy's stream has drained (release), so any stream may reuse it at once.
constexpr size_t kCacheCap = static_cast<size_t>(32) << 30;
struct CachedBlock {
  void *p;
  size_t size;
};
static std::vector<CachedBlock> g_cache[64];
static size_t g_cache_bytes[64];
static size_t g_cache_cap[64];  // 0: the default kCacheCap

static size_t cache_cap(int device) { return g_cache_cap[device] ? g_cache_cap[device] - 1 : kCacheCap; }

static void *cached_block(int device, size_t bytes) {
  if (device < 0 || device >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(g_pool_mu);
  std::vector<CachedBlock> &c = g_cache[device];
  for (size_t i = c.size(); i-- > 0;)
    if (c[i].size == bytes) {
      void *p = c[i].p;
      c.erase(c.begin() + static_cast<std::ptrdiff_t>(i));
      g_cache_bytes[device] -= bytes;
      return p;
    }
  return nullptr;
}

static bool cache_block(int device, void *p, size_t bytes) {
  if (device < 0 || device >= 64) return false;
  std::lock_guard<std::mutex> lock(g_pool_mu);
  if (g_cache_bytes[device] + bytes > cache_cap(device)) return false;
  g_cache[device].push_back(CachedBlock{p, bytes});
  g_cache_bytes[device] += bytes;
  return true;
}

// return every cached block of a device to the driver (an allocation failed: the cache must not be what starves it)
static void flush_cache(int device) {
  std::vector<CachedBlock> blocks;
  {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    blocks.swap(g_cache[device]);
    g_cache_bytes[device] = 0;
  }
  hipMemPool_t pool = pool_for(device);
  const bool pooled = pool != nullptr;  // then every block came from the device's pool
  for (const CachedBlock &b : blocks) (void)(pooled ? hipFreeAsync(b.p, nullptr) : hipFree(b.p));
  if (pooled) {
    (void)hipStreamSynchronize(nullptr);
    // the pool keeps what it was given back (its release threshold is unlimited); hand it to the driver now
    (void)hipMemPoolTrimTo(pool, 0);
  }
}

static void *fresh_block(amg_hierarchy *h, size_t bytes) {
  void *p = nullptr;
  hipMemPool_t pool = pool_for(h->device);
  if (pool) {
    if (hipMallocFromPoolAsync(&p, bytes, pool, h->stream) != hipSuccess) return nullptr;
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    return nullptr;
  }
  return p;
}

static void *raw_alloc(amg_hierarchy *h, size_t bytes) {
  if (h->opt.alloc) {  // the caller's device allocator: no cache, no pool
    void *p = h->opt.alloc(bytes, h->opt.ctx);
    if (!p) return nullptr;
    h->allocs.push_back(p);
    h->alloc_sizes.push_back(bytes);
    h->bytes += bytes;
    return p;
  }
  void *p = cached_block(h->device, bytes);
  if (!p) p = fresh_block(h, bytes);
  if (!p && h->device >= 0 && h->device < 64) {
    (void)hipGetLastError();  // clear the failed allocation's error before retrying
    flush_cache(h->device);
    p = fresh_block(h, bytes);
  }
  if (!p) return nullptr;
  h->allocs.push_back(p);
  h->alloc_sizes.push_back(bytes);
  h->bytes += bytes;
  return p;
}

// A hierarchy holds a few hundred device arrays; one pool allocation and one free for each would cost more than the
// setup's kernels. Arrays up to half a chunk are therefore carved (256-byte aligned, first fit) from shared chunks
// of chunk_unit bytes, about an eighth of the hierarchy's estimated size; larger arrays get an allocation of their
// own. A hierarchy then makes a few dozen allocations.
void *dalloc(amg_hierarchy *h, size_t bytes) {
  bytes = (bytes + 255) & ~static_cast<size_t>(255);
  if (bytes > h->chunk_unit / 2) return raw_alloc(h, bytes);
  for (Chunk &c : h->chunks)
    if (c.used + bytes <= c.size) {
      void *p = c.base + c.used;
      c.used += bytes;
      return p;
    }
  char *base = static_cast<char *>(raw_alloc(h, h->chunk_unit));
  if (!base) return nullptr;
  h->chunks.push_back(Chunk{base, h->chunk_unit, bytes});
  return base;
}

// give one of h's blocks back: to the caller's allocator, the block cache, or the pool / driver; true when it went to
// the pool or the driver (the caller then synchronises the stream)
static bool give_back(amg_hierarchy *h, void *p, size_t bytes, bool pooled) {
  if (h->opt.dealloc) {
    h->opt.dealloc(p, h->opt.ctx);
    return false;
  }
  if (cache_block(h->device, p, bytes)) return false;
  (void)(pooled ? hipFreeAsync(p, h->stream) : hipFree(p));
  return true;
}

void *tmp_alloc(amg_hierarchy *h, hipStream_t s, size_t bytes) {
  void *p = nullptr;
  if (h && h->opt.alloc) return h->opt.alloc(bytes, h->opt.ctx);
  hipMemPool_t pool = h ? pool_for(h->device) : nullptr;
  if (pool) {
    if (hipMallocFromPoolAsync(&p, bytes, pool, s) != hipSuccess) {
      (void)hipGetLastError();
      flush_cache(h->device);
      p = nullptr;
      if (hipMallocFromPoolAsync(&p, bytes, pool, s) != hipSuccess) return nullptr;
    }
    return p;
  }
  return hipMallocAsync(&p, bytes, s) == hipSuccess ? p : nullptr;
}

void tmp_free(amg_hierarchy *h, hipStream_t s, void *p) {
  if (!p) return;
  if (h && h->opt.dealloc) {
    (void)hipStreamSynchronize(s);  // the temporary's last reader has finished before the caller reuses it
    h->opt.dealloc(p, h->opt.ctx);
    return;
  }
  (void)hipFreeAsync(p, s);
}

amg_status release(amg_hierarchy *h) {
  const bool pooled = pool_for(h->device) != nullptr;
  (void)hipStreamSynchronize(h->stream);  // the hierarchy's work has drained: its blocks are idle
  bool freed = false;
  for (size_t i = 0; i < h->allocs.size(); i++) freed |= give_back(h, h->allocs[i], h->alloc_sizes[i], pooled);
  if (pooled && freed) (void)hipStreamSynchronize(h->stream);
  h->allocs.clear();
  h->alloc_sizes.clear();
  h->chunks.clear();
  if (h->host_scal) return_pinned_scalars(h->host_scal);
  h->host_scal = nullptr;
  return_events(h->device, h->timing.ev);
  return AMG_OK;
}

ArenaMark arena_mark(const amg_hierarchy *h) {
  ArenaMark m;
  m.allocs = h->allocs.size();
  m.bytes = h->bytes;
  for (const Chunk &c : h->chunks) m.used.push_back(c.used);
  return m;
}

void arena_rollback(amg_hierarchy *h, const ArenaMark &m) {
  (void)hipStreamSynchronize(h->stream);  // the temporaries' last readers have finished
  const bool pooled = pool_for(h->device) != nullptr;
  bool freed = false;
  for (size_t i = m.allocs; i < h->allocs.size(); i++) freed |= give_back(h, h->allocs[i], h->alloc_sizes[i], pooled);
  if (pooled && freed) (void)hipStreamSynchronize(h->stream);
  h->allocs.resize(m.allocs);
  h->alloc_sizes.resize(m.allocs);
  h->bytes = m.bytes;
  h->chunks.resize(m.used.size());  // chunks opened after the mark were among the blocks just released
  for (size_t c = 0; c < m.used.size(); c++) h->chunks[c].used = m.used[c];
}

// Timing events are kept in a process-wide pool per device: a hierarchy borrows a block while kernel timing is on
// and returns it when freed, so a stream of short-lived timed hierarchies creates events only once.
static std::vector<hipEvent_t> g_free_events[64];

amg_status borrow_events(int device, size_t count, std::vector<hipEvent_t> &out) {
  if (device < 0 || device >= 64) return AMG_ERR_INVALID;
  std::lock_guard<std::mutex> lock(g_pool_mu);
  std::vector<hipEvent_t> &fl = g_free_events[device];
  while (fl.size() < count) {
    hipEvent_t e = nullptr;
    QA_HIP(hipEventCreate(&e));
    fl.push_back(e);
  }
  out.assign(fl.end() - static_cast<std::ptrdiff_t>(count), fl.end());
  fl.resize(fl.size() - count);
  return AMG_OK;
}

// Pinned host mirrors of the convergence scalars (kScalars doubles each) come from a process-wide free list filled
// in chunks that are never freed: pinning and unpinning host memory costs milliseconds, far more than a solve's
// bookkeeping, and a request stream creates and frees hierarchies continually.
static std::vector<double *> g_free_pinned;

amg_status borrow_pinned_scalars(double **out) {
  std::lock_guard<std::mutex> lock(g_pool_mu);
  if (g_free_pinned.empty()) {
    constexpr int kPerChunk = 64;
    double *chunk = nullptr;
    QA_HIP(hipHostMalloc(reinterpret_cast<void **>(&chunk), sizeof(double) * kScalars * kPerChunk,
                         hipHostMallocDefault));
    for (int i = kPerChunk - 1; i >= 0; i--) g_free_pinned.push_back(chunk + static_cast<size_t>(i) * kScalars);
  }
  *out = g_free_pinned.back();
  g_free_pinned.pop_back();
  return AMG_OK;
}

void return_pinned_scalars(double *p) {
  std::lock_guard<std::mutex> lock(g_pool_mu);
  g_free_pinned.push_back(p);
}

void return_events(int device, std::vector<hipEvent_t> &ev) {
  if (ev.empty()) return;
  if (device >= 0 && device < 64) {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    g_free_events[device].insert(g_free_events[device].end(), ev.begin(), ev.end());
  } else {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  ev.clear();
}

// ---------------------------------------------------------------------------------------------------------------
// Exclusive scan: out[i] = sum_{j<i} in[j], out[n] = total. Blocks of 256 threads x 8 items; block totals are
// scanned recursively and added back.

constexpr int kScanItems = 8;
constexpr int kScanChunk = kBlock * kScanItems;

template <class T>
__global__ void __launch_bounds__(kBlock) k_scan_block(const T *__restrict__ in, T *__restrict__ out,
                                                        T *__restrict__ bsum, int64_t n) {
  __shared__ T s_tot[kBlock];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanChunk + static_cast<int64_t>(threadIdx.x) * kScanItems;
  T v[kScanItems];
  T run = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; i++) {
    v[i] = (base + i < n) ? in[base + i] : T(0);
    T t = v[i];
    v[i] = run;
    run += t;
  }
  s_tot[threadIdx.x] = run;
  __syncthreads();
  // Hillis-Steele inclusive scan of the thread totals
  for (int off = 1; off < kBlock; off <<= 1) {
    T add = (threadIdx.x >= off) ? s_tot[threadIdx.x - off] : T(0);
    __syncthreads();
    s_tot[threadIdx.x] += add;
    __syncthreads();
  }
  const T excl = (threadIdx.x > 0) ? s_tot[threadIdx.x - 1] : T(0);
#pragma unroll
  for (int i = 0; i < kScanItems; i++)
    if (base + i < n) out[base + i] = excl + v[i];
  if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = s_tot[kBlock - 1];
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_scan_add(T *__restrict__ out, const T *__restrict__ bsum_ex, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) out[i] += bsum_ex[i / kScanChunk];
  if (i == 0) out[n] = bsum_ex[(n + kScanChunk - 1) / kScanChunk];
}

template <class T>
__global__ void k_scan_single_tail(T *__restrict__ out, const T *__restrict__ bsum, int64_t n) {
  out[n] = bsum[0];
}

template <class T>
static amg_status scan_impl(const T *in, T *out, int64_t n, hipStream_t s, amg_hierarchy *h) {
  if (n <= 0) {
    T zero = 0;
    QA_HIP(hipMemcpyAsync(out, &zero, sizeof(T), hipMemcpyHostToDevice, s));
    QA_HIP(hipStreamSynchronize(s));
    return AMG_OK;
  }
  const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
  T *bsum = static_cast<T *>(tmp_alloc(h, s, sizeof(T) * (2 * nb + 2)));
  if (!bsum) return AMG_ERR_NOMEM;
  T *bsum_ex = bsum + nb;
  amg_status st = AMG_OK;
  k_scan_block<T><<<nb, kBlock, 0, s>>>(in, out, bsum, n);
  if (hipGetLastError() != hipSuccess) st = AMG_ERR_DEVICE;
  if (st == AMG_OK && nb == 1) {
    k_scan_single_tail<T><<<1, 1, 0, s>>>(out, bsum, n);
    if (hipGetLastError() != hipSuccess) st = AMG_ERR_DEVICE;
  } else if (st == AMG_OK) {
    st = scan_impl<T>(bsum, bsum_ex, nb, s, h);
    if (st == AMG_OK) {
      k_scan_add<T><<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(out, bsum_ex, n);
      if (hipGetLastError() != hipSuccess) st = AMG_ERR_DEVICE;
    }
  }
  tmp_free(h, s, bsum);  // on every path
  return st;
}

amg_status scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s, amg_hierarchy *h) {
  return scan_impl<int64_t>(in, out, n, s, h);
}
amg_status scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, hipStream_t s, amg_hierarchy *h) {
  return scan_impl<int32_t>(in, out, n, s, h);
}

}  // namespace qa

extern "C" {

amg_status amg_cache_control(int32_t device, int64_t limit_bytes, size_t *cached_bytes) {
  if (device < 0 || device >= 64) return AMG_ERR_INVALID;
  if (limit_bytes >= 0) {
    std::vector<qa::CachedBlock> out;
    {
      std::lock_guard<std::mutex> lock(qa::g_pool_mu);
      qa::g_cache_cap[device] = static_cast<size_t>(limit_bytes) + 1;
      std::vector<qa::CachedBlock> &c = qa::g_cache[device];
      // the oldest blocks go first
      while (!c.empty() && qa::g_cache_bytes[device] > static_cast<size_t>(limit_bytes)) {
        out.push_back(c.front());
        qa::g_cache_bytes[device] -= c.front().size;
        c.erase(c.begin());
      }
    }
    if (!out.empty()) {
      int cur = 0;
      if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(device) != hipSuccess) return AMG_ERR_DEVICE;
      hipMemPool_t pool = qa::pool_for(device);
      for (const qa::CachedBlock &b : out) (void)(pool ? hipFreeAsync(b.p, nullptr) : hipFree(b.p));
      if (pool) {
        (void)hipStreamSynchronize(nullptr);
        (void)hipMemPoolTrimTo(pool, 0);
      }
      (void)hipSetDevice(cur);
    }
  }
  if (cached_bytes) {
    std::lock_guard<std::mutex> lock(qa::g_pool_mu);
    *cached_bytes = qa::g_cache_bytes[device];
  }
  return AMG_OK;
}

void amg_default_options(amg_options *opt) {
  if (!opt) return;
  opt->precision = 0;
  opt->coarse_max = 64;
  opt->inner_iters = 2;
  opt->sweeps = 1;
  opt->outer_mmax = 1;
  opt->max_iters = 1000;
  opt->engine = 1;
  opt->batch = 1;
  opt->smoother = 0;
  opt->box = nullptr;
  opt->stream = nullptr;
  opt->alloc = nullptr;
  opt->dealloc = nullptr;
  opt->ctx = nullptr;
}

const char *amg_status_string(amg_status s) {
  switch (s) {
    case AMG_OK: return "AMG_OK";
    case AMG_ERR_INVALID: return "AMG_ERR_INVALID";
    case AMG_ERR_NOMEM: return "AMG_ERR_NOMEM";
    case AMG_ERR_DEVICE: return "AMG_ERR_DEVICE";
    case AMG_ERR_NOT_SPD: return "AMG_ERR_NOT_SPD";
    case AMG_ERR_BREAKDOWN: return "AMG_ERR_BREAKDOWN";
    case AMG_ERR_NOCONV: return "AMG_ERR_NOCONV";
  }
  return "AMG_ERR_UNKNOWN";
}

void amg_free(amg_hierarchy *h) {
  if (!h) return;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  qa::release(h);
  delete h;
}

amg_status amg_hierarchy_bytes(const amg_hierarchy *h, size_t *bytes) {
  if (!h || !bytes) return AMG_ERR_INVALID;
  *bytes = h->bytes;
  return AMG_OK;
}

amg_status amg_num_levels(const amg_hierarchy *h, int32_t *levels) {
  if (!h || !levels) return AMG_ERR_INVALID;
  *levels = h->nlev;
  return AMG_OK;
}

amg_status amg_set_precision(amg_hierarchy *h, int32_t precision) {
  if (!h || (precision != 0 && precision != 1)) return AMG_ERR_INVALID;
  h->precision = precision;
  return AMG_OK;
}

amg_status amg_set_stream(amg_hierarchy *h, void *stream) {
  if (!h) return AMG_ERR_INVALID;
  if (static_cast<hipStream_t>(stream) == h->stream) return AMG_OK;
  QA_HIP(hipSetDevice(h->device));
  QA_HIP(hipStreamSynchronize(h->stream));
  h->stream = static_cast<hipStream_t>(stream);
  return AMG_OK;
}

}  // extern "C"
