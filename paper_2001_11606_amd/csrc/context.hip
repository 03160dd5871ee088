// Context, error reporting and version of the C ABI.
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "internal.h"

namespace rt {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

ReleaseState& release_state() {
  static thread_local ReleaseState st;
  return st;
}

// Device scratch of the entry point that allocates nothing (rt_solve_noalloc):
// one array per GPU, in the code object, held until the process ends.  Its
// name is a host-side stand-in for the device array; the device address is
// looked up once per device, with that device current, and kept here.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;
}  // namespace

int scratch_setup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return RT_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    set_error("scratch: hipGetSymbolAddress failed on device %d: %s", device,
              hipGetErrorString(e));
    return RT_E_DEVICE;
  }
  g_scratch_ptr[device] = ptr;
  return RT_OK;
}

void* scratch_base(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  return it == g_scratch_ptr.end() ? nullptr : it->second;
}

namespace {
struct Cached {
  void* p;
  bool idle;           // no queued work uses it
  hipStream_t stream;  // else: the stream whose queued work may use it
};
std::mutex g_pool_mu;
// (device, bytes) -> cached block
std::multimap<std::pair<int, size_t>, Cached> g_pool;
size_t g_pool_total = 0;

// sizes are rounded so that blocks of nearly equal requests are shared
size_t pool_round(size_t b) {
  const size_t g = b >= ((size_t)1 << 20) ? ((size_t)2 << 20) : 256;
  return (b + g - 1) / g * g;
}
}  // namespace

void* pool_get(size_t* bytes, int* device) {
  int d = 0;
  (void)hipGetDevice(&d);
  *device = d;
  const size_t want = pool_round(*bytes);
  const ReleaseState& rs = release_state();
  bool wait = false;
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto best = g_pool.end();
    for (auto it = g_pool.lower_bound({d, want});
         it != g_pool.end() && it->first.first == d && it->first.second <= want + want / 8; ++it) {
      const Cached& c = it->second;
      const bool ready = c.idle || (rs.stream_scopes > 0 && c.stream == rs.stream);
      if (ready) {
        best = it;
        break;
      }
      if (best == g_pool.end()) best = it;   // usable after waiting for the device
    }
    if (best != g_pool.end()) {
      const Cached& c = best->second;
      wait = !(c.idle || (rs.stream_scopes > 0 && c.stream == rs.stream));
      p = c.p;
      *bytes = best->first.second;
      g_pool_total -= best->first.second;
      g_pool.erase(best);
    }
  }
  if (p) {
    if (wait) (void)hipDeviceSynchronize();   // another stream may still use it
#ifdef RT_POOL_POISON
    std::memset(p, 0xBE, *bytes);   // a reused block reads as garbage, like a fresh one
#endif
    return p;
  }
  if (hipMalloc(&p, want) == hipSuccess) {
    *bytes = want;
    return p;
  }
  (void)hipGetLastError();
  pool_trim(d);
  if (hipMalloc(&p, want) == hipSuccess) {
    *bytes = want;
    return p;
  }
  (void)hipGetLastError();
  return nullptr;
}

void pool_put(void* p, size_t bytes, int device, bool idle, hipStream_t stream) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (g_pool_total + bytes <= kPoolCapBytes) {
      g_pool.insert({{device, bytes}, Cached{p, idle, stream}});
      g_pool_total += bytes;
      return;
    }
  }
  (void)hipFree(p);   // synchronises with the device before freeing
}

void pool_trim(int device) {
  std::vector<void*> out;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (auto it = g_pool.begin(); it != g_pool.end();) {
      if (device < 0 || it->first.first == device) {
        out.push_back(it->second.p);
        g_pool_total -= it->first.second;
        it = g_pool.erase(it);
      } else {
        ++it;
      }
    }
  }
  for (void* p : out) (void)hipFree(p);
}

size_t pool_cached_bytes(int device) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  size_t t = 0;
  for (const auto& kv : g_pool)
    if (device < 0 || kv.first.first == device) t += kv.first.second;
  return t;
}

}  // namespace rt

int rt_ctx::sync_read(const void* dev, size_t bytes) {
  RT_CHECK_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, stream));
  RT_CHECK_HIP(hipStreamSynchronize(stream));
  return RT_OK;
}

int rt_ctx::prof_mark(size_t* idx) {
  if (prof_used == prof_ev.size()) {
    // timing only (read after the stream is synchronised): no system-scope
    // fence, whose cache writeback and invalidation would slow the product
    // that follows and inflate the timings
    hipEvent_t e;
    RT_CHECK_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    prof_ev.push_back(e);
  }
  RT_CHECK_HIP(hipEventRecord(prof_ev[prof_used], stream));
  *idx = prof_used++;
  return RT_OK;
}

int rt_ctx::prof_collect(double* seconds, int* calls, int nkinds) {
  for (int k = 0; k < nkinds; ++k) {
    seconds[k] = 0.0;
    calls[k] = 0;
  }
  if (prof_used) RT_CHECK_HIP(hipEventSynchronize(prof_ev[prof_used - 1]));
  for (const Span& s : prof_spans) {
    float ms = 0.f;
    RT_CHECK_HIP(hipEventElapsedTime(&ms, prof_ev[s.a], prof_ev[s.b]));
    if (s.kind >= 0 && s.kind < nkinds) {
      seconds[s.kind] += 1e-3 * ms;
      calls[s.kind] += 1;
    }
  }
  prof_spans.clear();
  prof_used = 0;
  return RT_OK;
}

rt_ctx::~rt_ctx() {
  for (hipEvent_t e : prof_ev) (void)hipEventDestroy(e);
}

extern "C" {

const char* rt_last_error(void) { return rt::g_last_error.c_str(); }

const char* rt_version(void) { return "rt-mi355x 0.1 (gfx950)"; }

int rt_create(rt_ctx** ctx, int device, void* hip_stream) {
  rt::clear_error();
  if (!ctx) {
    rt::set_error("rt_create: ctx is NULL");
    return RT_E_ARG;
  }
  *ctx = nullptr;
  int ndev = 0;
  RT_CHECK_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) {
    rt::set_error("rt_create: device %d out of range (%d devices)", device, ndev);
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(device));
  RT_CHECK(rt::scratch_setup(device));   // the scratch array's address on this device
  rt_ctx* c = new rt_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipHostMalloc((void**)&c->host, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    delete c;
    rt::set_error("rt_create: pinned host allocation failed");
    return RT_E_OOM;
  }
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    rt::set_error("rt_create: hipEventCreate failed");
    rt_destroy(c);
    return RT_E_DEVICE;
  }
  *ctx = c;
  return RT_OK;
}

void rt_destroy(rt_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  if (ctx->host) (void)hipHostFree(ctx->host);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  const int dev = ctx->device;
  delete ctx;
  rt::pool_trim(dev);
}

int rt_release_cached(rt_ctx* ctx, int64_t* freed_bytes) {
  if (!ctx) {
    rt::set_error("rt_release_cached: ctx is NULL");
    return RT_E_ARG;
  }
  RT_CHECK_HIP(hipSetDevice(ctx->device));
  RT_CHECK_HIP(hipDeviceSynchronize());
  const size_t b = rt::pool_cached_bytes(ctx->device);
  rt::pool_trim(ctx->device);
  if (freed_bytes) *freed_bytes = (int64_t)b;
  return RT_OK;
}

int rt_cached_bytes(const rt_ctx* ctx, int64_t* bytes) {
  if (!ctx || !bytes) {
    rt::set_error("rt_cached_bytes: NULL argument");
    return RT_E_ARG;
  }
  *bytes = (int64_t)rt::pool_cached_bytes(ctx->device);
  return RT_OK;
}

int rt_set_stream(rt_ctx* ctx, void* hip_stream) {
  if (!ctx) {
    rt::set_error("rt_set_stream: ctx is NULL");
    return RT_E_ARG;
  }
  ctx->stream = (hipStream_t)hip_stream;
  return RT_OK;
}

int rt_set_profiling(rt_ctx* ctx, int on) {
  if (!ctx) {
    rt::set_error("rt_set_profiling: ctx is NULL");
    return RT_E_ARG;
  }
  ctx->profiling = on != 0;
  return RT_OK;
}

}  // extern "C"
