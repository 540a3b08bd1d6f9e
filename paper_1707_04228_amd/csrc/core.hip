// Context management, error reporting and a device exclusive prefix sum.
#include "gx_internal.h"

namespace gx {

thread_local gx_ctx* tls_ctx = nullptr;
thread_local hipStream_t tls_stream = nullptr;     // overrides the context's stream if set
thread_local bool tls_idle = false;                // releases happen on an idle device

CtxScope::CtxScope(gx_ctx* c) : prev(tls_ctx), prev_stream(tls_stream) {
  tls_ctx = c;
  tls_stream = nullptr;
}
CtxScope::~CtxScope() {
  tls_ctx = prev;
  tls_stream = prev_stream;
}
StreamScope::StreamScope(hipStream_t s) : prev(tls_stream) { tls_stream = s; }
StreamScope::~StreamScope() { tls_stream = prev; }

namespace {
constexpr size_t CACHE_MIN = (size_t)64 << 20;   // large blocks: cached whoever frees them
constexpr size_t SMALL_CAP = (size_t)1 << 30;    // small blocks kept per device

// What a cached block may still be used by: nothing (idle), the work its owner's stream
// had queued when it was released (owner, ev), or unknown work (neither: a device
// synchronisation before reuse).
struct CachedBlock {
  int dev;
  size_t bytes;
  void* p;
  const gx_ctx* owner;
  hipStream_t st;                                // the stream its last kernels ran on
  hipEvent_t ev;                                 // recorded on st at release
  bool idle;
  uint64_t seq;                                  // release order (large blocks: eviction)
};

// The stream a context's work on this thread goes to (null outside any context).
hipStream_t cur_stream(const gx_ctx* me) { return tls_stream ? tls_stream : me ? me->stream : nullptr; }

std::mutex cache_mu;
std::vector<CachedBlock> cache_blocks;
std::vector<size_t> cache_bytes, cache_cap, small_bytes;   // per device
uint64_t release_seq = 0;

void ensure_dev(int dev) {                         // caller holds cache_mu
  if ((int)cache_bytes.size() <= dev) {
    cache_bytes.resize(dev + 1, 0);
    cache_cap.resize(dev + 1, 0);
    small_bytes.resize(dev + 1, 0);
  }
  if (!cache_cap[dev]) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) cache_cap[dev] = tot / 4 * 3;
  }
}

void drop_block(size_t i) {                        // caller holds cache_mu; counters only
  const CachedBlock& c = cache_blocks[i];
  if (c.bytes >= CACHE_MIN)
    cache_bytes[c.dev] -= c.bytes;
  else
    small_bytes[c.dev] -= c.bytes;
  cache_blocks[i] = cache_blocks.back();
  cache_blocks.pop_back();
}

void trim_cache(int dev) {                          // caller holds cache_mu
  (void)hipDeviceSynchronize();
  for (size_t i = 0; i < cache_blocks.size();) {
    if (cache_blocks[i].dev == dev) {
      if (cache_blocks[i].ev) (void)hipEventDestroy(cache_blocks[i].ev);
      (void)hipFree(cache_blocks[i].p);
      drop_block(i);
    } else {
      ++i;
    }
  }
}

// preference among reusable blocks: 0 no wait (own stream, or idle), 1 a host wait for the
// owner's event, 2 a device synchronisation
int wait_class(const CachedBlock& c, const gx_ctx* me) {
  if (c.idle || (me && c.owner == me && c.st == cur_stream(me))) return 0;
  return c.ev ? 1 : 2;
}
}  // namespace

void* dev_alloc(size_t bytes, int* dev, hipError_t* err) {
  int d = 0;
  (void)hipGetDevice(&d);
  *dev = d;
  const gx_ctx* me = tls_ctx && tls_ctx->device == d ? tls_ctx : nullptr;
  const bool large = bytes >= CACHE_MIN;
  {
    std::unique_lock<std::mutex> lk(cache_mu);
    ensure_dev(d);
    int best = -1, best_w = 3;
    for (int i = 0; i < (int)cache_blocks.size(); ++i) {
      const CachedBlock& c = cache_blocks[i];
      if (c.dev != d || c.bytes < bytes || (c.bytes >= CACHE_MIN) != large) continue;
      if (large ? c.bytes > bytes + bytes / 8 + CACHE_MIN : c.bytes > 2 * bytes + 4096) continue;
      const int w = wait_class(c, me);
      if (!large && w == 2) continue;              // small blocks: never a device sync
      if (best < 0 || w < best_w || (w == best_w && c.bytes < cache_blocks[best].bytes)) {
        best = i;
        best_w = w;
      }
    }
    if (best >= 0) {
      const CachedBlock c = cache_blocks[best];
      drop_block(best);
      lk.unlock();
      // the block's earlier users must be done with it before anything of ours runs
      *err = hipSuccess;
      if (best_w == 1)
        *err = hipEventSynchronize(c.ev);          // the owner's work up to the release
      else if (best_w == 2)
        *err = hipDeviceSynchronize();
      if (c.ev) (void)hipEventDestroy(c.ev);
      if (*err != hipSuccess) {
        (void)hipDeviceSynchronize();
        (void)hipFree(c.p);
        return nullptr;
      }
      // (released again, it is filed under the requested size, never more than it has)
      return c.p;
    }
  }
  void* p = nullptr;
  *err = hipMalloc(&p, bytes);
  if (*err == hipErrorOutOfMemory) {
    {
      std::lock_guard<std::mutex> lk(cache_mu);
      trim_cache(d);
    }
    (void)hipGetLastError();
    *err = hipMalloc(&p, bytes);
  }
  return *err == hipSuccess ? p : nullptr;
}

void dev_free(void* p, size_t bytes, int dev) {
  if (!p) return;
  const gx_ctx* me = tls_ctx && tls_ctx->device == dev ? tls_ctx : nullptr;
  if (dev >= 0) {
    std::lock_guard<std::mutex> lk(cache_mu);
    ensure_dev(dev);
    const bool large = bytes >= CACHE_MIN;
    if (large && cache_bytes[dev] + bytes > cache_cap[dev] && bytes <= cache_cap[dev]) {
      // the latest release is the likeliest to be asked for again (the next solve of the
      // same problem): make room by freeing the large blocks released longest ago
      (void)hipDeviceSynchronize();
      while (cache_bytes[dev] + bytes > cache_cap[dev]) {
        int old = -1;
        for (int i = 0; i < (int)cache_blocks.size(); ++i) {
          const CachedBlock& c = cache_blocks[i];
          if (c.dev == dev && c.bytes >= CACHE_MIN &&
              (old < 0 || c.seq < cache_blocks[old].seq))
            old = i;
        }
        if (old < 0) break;
        if (cache_blocks[old].ev) (void)hipEventDestroy(cache_blocks[old].ev);
        (void)hipFree(cache_blocks[old].p);
        drop_block(old);
      }
    }
    const bool room = large ? cache_bytes[dev] + bytes <= cache_cap[dev]
                            : (me || tls_idle) && small_bytes[dev] + bytes <= SMALL_CAP;
    if (room) {
      CachedBlock c{dev, bytes, p, nullptr, nullptr, nullptr, tls_idle, ++release_seq};
      if (!tls_idle && me) {
        // tag with the owner's stream position; without an event the block stays untagged
        hipEvent_t ev = nullptr;
        const hipStream_t st = cur_stream(me);
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
          if (hipEventRecord(ev, st) == hipSuccess) {
            c.owner = me;
            c.st = st;
            c.ev = ev;
          } else {
            (void)hipEventDestroy(ev);
          }
        }
      }
      if (large || c.owner || c.idle) {
        cache_blocks.push_back(c);
        (large ? cache_bytes : small_bytes)[dev] += bytes;
        return;
      }
    }
  }
  (void)hipFree(p);
}

void dev_forget(const gx_ctx* c) {
  std::lock_guard<std::mutex> lk(cache_mu);
  for (CachedBlock& b : cache_blocks)
    if (b.owner == c) {                            // its stream is idle: nothing pending
      if (b.ev) (void)hipEventDestroy(b.ev);
      b.ev = nullptr;
      b.owner = nullptr;
      b.idle = true;
    }
}

IdleScope::IdleScope() : prev(tls_idle) { tls_idle = true; }
IdleScope::~IdleScope() { tls_idle = prev; }

constexpr int SCAN_BS = 256;
constexpr int SCAN_PT = 8;                       // items per thread
constexpr int SCAN_TILE = SCAN_BS * SCAN_PT;

// Block-level exclusive scan; writes the tile total to sums[blockIdx.x].
template <class T>
__global__ void scan_tiles(T* data, int64_t n, int64_t* sums) {
  __shared__ int64_t part[SCAN_BS];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_PT;
  int64_t v[SCAN_PT];
  int64_t acc = 0;
#pragma unroll
  for (int i = 0; i < SCAN_PT; ++i) {
    const int64_t idx = base + i;
    v[i] = idx < n ? (int64_t)data[idx] : 0;
    acc += v[i];
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums
  for (int off = 1; off < SCAN_BS; off <<= 1) {
    int64_t add = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t run = part[threadIdx.x] - acc;         // exclusive prefix of this thread
#pragma unroll
  for (int i = 0; i < SCAN_PT; ++i) {
    const int64_t idx = base + i;
    if (idx < n) data[idx] = (T)run;
    run += v[i];
  }
  if (threadIdx.x == SCAN_BS - 1) sums[blockIdx.x] = part[SCAN_BS - 1];
}

template <class T>
__global__ void scan_add(T* data, int64_t n, const int64_t* sums) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  const int64_t add = sums[blockIdx.x];
  for (int i = threadIdx.x; i < SCAN_TILE; i += SCAN_BS) {
    const int64_t idx = base + i;
    if (idx < n) data[idx] = (T)((int64_t)data[idx] + add);
  }
}

size_t scan_tmp_size(int64_t n) {
  size_t tot = 1;
  while (n > 1) {
    n = (n + SCAN_TILE - 1) / SCAN_TILE;
    tot += (size_t)n + 1;
  }
  return tot + 2;
}

template <class T>
static void scan_rec(T* data, int64_t n, int64_t* tmp, hipStream_t s) {
  if (n <= 0) return;
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  hipLaunchKernelGGL(scan_tiles<T>, dim3((unsigned)nb), dim3(SCAN_BS), 0, s, data, n, tmp);
  GX_HIP(hipGetLastError());
  if (nb > 1) {
    scan_rec<int64_t>(tmp, nb, tmp + nb + 1, s);
    hipLaunchKernelGGL(scan_add<T>, dim3((unsigned)nb), dim3(SCAN_BS), 0, s, data, n, tmp);
    GX_HIP(hipGetLastError());
  }
}

template <class T>
static int64_t scan_impl(T* data, int64_t n, int64_t* tmp, hipStream_t s) {
  if (n <= 0) return 0;
  T last;
  GX_HIP(hipMemcpyAsync(&last, data + n - 1, sizeof(T), hipMemcpyDeviceToHost, s));
  GX_HIP(hipStreamSynchronize(s));
  scan_rec<T>(data, n, tmp, s);
  T lastx;
  GX_HIP(hipMemcpyAsync(&lastx, data + n - 1, sizeof(T), hipMemcpyDeviceToHost, s));
  GX_HIP(hipStreamSynchronize(s));
  return (int64_t)lastx + (int64_t)last;
}

int64_t exclusive_scan(int64_t* data, int64_t n, int64_t* tmp, hipStream_t s) {
  return scan_impl<int64_t>(data, n, tmp, s);
}
int64_t exclusive_scan32(int32_t* data, int64_t n, int64_t* tmp, hipStream_t s) {
  return scan_impl<int32_t>(data, n, tmp, s);
}

}  // namespace gx

extern "C" {

gx_status gx_create(gx_ctx** out, int32_t device, void* hip_stream) {
  if (!out) return GX_EINVAL;
  *out = nullptr;
  gx_ctx* c = nullptr;
  try {
    int ndev = 0;
    GX_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return GX_EINVAL;
    c = new gx_ctx();
    c->device = device;
    GX_HIP(hipSetDevice(device));
    gx::noalloc_scratch_init(device);
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      GX_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
  } catch (const gx::Error& e) {
    delete c;
    return e.code;
  }
  *out = c;
  return GX_OK;
}

void gx_destroy(gx_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  gx::dev_forget(c);                               // before the address can be reused
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  gx::IdleScope idle;                              // its buffers are released unused
  delete c;
}

const char* gx_last_error(const gx_ctx* c) { return c ? c->err.c_str() : "null context"; }

const char* gx_version(void) { return "gx 0.1 (gfx950)"; }

gx_status gx_phase_times(gx_ctx* c, double* ms) {
  if (!c) return GX_EINVAL;
  if (ms)
    for (int i = 0; i < 8; ++i) ms[i] = c->phase_ms[i];
  return GX_OK;
}

}  // extern "C"
