// CPU emulation of the small HIP subset used by the library's kernels, for
// checking kernel indexing on the host (built with AddressSanitizer by
// tests/cpu_hip/build_cpu.py).  It is test infrastructure, not a back end.
//
// Execution model: blocks run one after another; the threads of a block run
// concurrently on a pool of OS threads, so __syncthreads() is a real barrier
// and __shfl_xor is an exchange through a per-block slot array guarded by
// per-group barriers.  Lanes that a GPU would hold inactive simply do not
// call the shuffle; a kernel that shuffles under group-divergent control flow
// therefore deadlocks here (the launcher aborts after a time limit).  Threads
// that return early drop out of the block barrier.  __shared__ variables are
// function-local statics: shared by the threads of the block that is running.
#pragma once

#include <math.h>

#include <algorithm>
#include <atomic>
#include <barrier>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <semaphore>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) (&(x))
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __builtin_nontemporal_load(p) (*(p))
#define __builtin_nontemporal_store(v, p) (*(p) = (v))
// dynamic LDS: a heap buffer of the launch's byte count (bounds seen by ASan)
#define RT_DYNAMIC_LDS(name) unsigned char* name = cpuhip::g_dyn_lds
#define RT_UNIFORM(x) (x)

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

typedef enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1 } hipError_t;
typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
typedef struct ihipGraph_t* hipGraph_t;
typedef struct ihipGraphExec_t* hipGraphExec_t;
typedef struct ihipGraphNode_t* hipGraphNode_t;
enum hipStreamCaptureMode {
  hipStreamCaptureModeGlobal = 0,
  hipStreamCaptureModeThreadLocal,
  hipStreamCaptureModeRelaxed
};
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost,
                     hipMemcpyDeviceToDevice, hipMemcpyDefault };
#define hipHostMallocDefault 0

namespace cpuhip {

struct ThreadCtx {
  dim3 tid, bid, bdim, gdim;
};
inline thread_local ThreadCtx tctx;
inline unsigned char* g_dyn_lds = nullptr;
// stream capture: launches are recorded while this is set (graphs replay them)
inline std::vector<std::function<void()>>* g_capture = nullptr;

struct BlockState {
  int nthreads = 0;
  std::unique_ptr<std::barrier<>> block_bar;
  // per width (log2 index 0..6) a barrier per group
  std::vector<std::unique_ptr<std::barrier<>>> group_bar[7];
  std::vector<uint64_t> slot;
  void reset(int n) {
    nthreads = n;
    block_bar = std::make_unique<std::barrier<>>(n);
    for (int w = 0; w < 7; ++w) {
      group_bar[w].clear();
      int width = 1 << w;
      int groups = (n + width - 1) / width;
      for (int g = 0; g < groups; ++g) {
        int members = std::min(width, n - g * width);
        group_bar[w].push_back(std::make_unique<std::barrier<>>(members));
      }
    }
    slot.assign(n, 0);
  }
};
inline BlockState& g_block_ref() {
  static BlockState* b = new BlockState;
  return *b;
}
#define g_block g_block_ref()

inline int log2i(int w) {
  int l = 0;
  while ((1 << l) < w) ++l;
  return l;
}

class Pool {
 public:
  // never destroyed: detached workers stay parked until the process exits
  static Pool& get() {
    static Pool* p = new Pool;
    return *p;
  }
  void run_block(int nthreads, const std::function<void(int)>& body) {
    ensure(nthreads);
    body_ = &body;
    remaining_.store(nthreads);
    for (int i = 0; i < nthreads; ++i) workers_[i]->go.release();
    if (!done_.try_acquire_for(std::chrono::seconds(120))) {
      fprintf(stderr, "cpuhip: block did not finish (divergent barrier or shuffle?)\n");
      fflush(stderr);
      abort();
    }
  }

 private:
  struct Worker {
    std::binary_semaphore go{0};
  };
  void ensure(int n) {
    while ((int)workers_.size() < n) {
      const int id = (int)workers_.size();
      workers_.push_back(std::make_unique<Worker>());
      Worker* w = workers_.back().get();
      std::thread([this, id, w] {
        for (;;) {
          w->go.acquire();
          (*body_)(id);
          if (remaining_.fetch_sub(1) == 1) done_.release();
        }
      }).detach();
    }
  }
  std::vector<std::unique_ptr<Worker>> workers_;
  const std::function<void(int)>* body_ = nullptr;
  std::atomic<int> remaining_{0};
  std::binary_semaphore done_{0};
};

template <typename F>
void launch(dim3 grid, dim3 block, F&& f, size_t shmem = 0) {
  const int nt = (int)(block.x * block.y * block.z);
  if (nt <= 0 || nt > 1024) {
    fprintf(stderr, "cpuhip: invalid block size %d\n", nt);
    abort();
  }
  for (unsigned bz = 0; bz < grid.z; ++bz)
    for (unsigned by = 0; by < grid.y; ++by)
      for (unsigned bx = 0; bx < grid.x; ++bx) {
        g_block.reset(nt);
        std::unique_ptr<unsigned char[]> dyn(shmem ? new unsigned char[shmem] : nullptr);
        if (shmem) memset(dyn.get(), 0xBE, shmem);
        g_dyn_lds = dyn.get();
        std::function<void(int)> body = [&](int t) {
          tctx.tid = dim3(t % block.x, (t / block.x) % block.y, t / (block.x * block.y));
          tctx.bid = dim3(bx, by, bz);
          tctx.bdim = block;
          tctx.gdim = grid;
          f();
          // leave every barrier so that the remaining threads can proceed
          g_block.block_bar->arrive_and_drop();
          for (int w = 0; w < 7; ++w) g_block.group_bar[w][t >> w]->arrive_and_drop();
        };
        Pool::get().run_block(nt, body);
      }
}

}  // namespace cpuhip

#define threadIdx (cpuhip::tctx.tid)
#define blockIdx (cpuhip::tctx.bid)
#define blockDim (cpuhip::tctx.bdim)
#define gridDim (cpuhip::tctx.gdim)

inline void __syncthreads() { cpuhip::g_block.block_bar->arrive_and_wait(); }
inline int atomicCAS(int* p, int cmp, int v) {
  std::atomic_ref<int>(*p).compare_exchange_strong(cmp, v);
  return cmp;
}
inline int atomicAdd(int* p, int v) { return std::atomic_ref<int>(*p).fetch_add(v); }
inline int atomicMin(int* p, int v) {
  std::atomic_ref<int> a(*p);
  int cur = a.load();
  while (v < cur && !a.compare_exchange_weak(cur, v)) {
  }
  return cur;
}
inline void __threadfence() {}

template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
  static_assert(sizeof(T) <= 8, "shuffle of more than 8 bytes");
  const int t = (int)threadIdx.x;
  const int lane = t % width;
  const int base = t - lane;
  auto& bar = *cpuhip::g_block.group_bar[cpuhip::log2i(width)][t / width];
  uint64_t bits = 0;
  memcpy(&bits, &v, sizeof(T));
  cpuhip::g_block.slot[t] = bits;
  bar.arrive_and_wait();
  uint64_t got = cpuhip::g_block.slot[base + ((lane ^ mask) % width)];
  bar.arrive_and_wait();
  T r;
  memcpy(&r, &got, sizeof(T));
  return r;
}

// value of lane src of the group of width lanes
template <typename T>
inline T __shfl(T v, int src, int width = 64) {
  static_assert(sizeof(T) <= 8, "shuffle of more than 8 bytes");
  const int t = (int)threadIdx.x;
  const int lane = t % width;
  auto& bar = *cpuhip::g_block.group_bar[cpuhip::log2i(width)][t / width];
  uint64_t bits = 0;
  memcpy(&bits, &v, sizeof(T));
  cpuhip::g_block.slot[t] = bits;
  bar.arrive_and_wait();
  const uint64_t got = cpuhip::g_block.slot[t - lane + (src % width)];
  bar.arrive_and_wait();
  T r;
  memcpy(&r, &got, sizeof(T));
  return r;
}

// value of the lane delta below (own value for the lowest delta lanes)
template <typename T>
inline T __shfl_up(T v, unsigned delta, int width = 64) {
  static_assert(sizeof(T) <= 8, "shuffle of more than 8 bytes");
  const int t = (int)threadIdx.x;
  const int lane = t % width;
  auto& bar = *cpuhip::g_block.group_bar[cpuhip::log2i(width)][t / width];
  uint64_t bits = 0;
  memcpy(&bits, &v, sizeof(T));
  cpuhip::g_block.slot[t] = bits;
  bar.arrive_and_wait();
  const uint64_t got = lane >= (int)delta ? cpuhip::g_block.slot[t - (int)delta] : bits;
  bar.arrive_and_wait();
  T r;
  memcpy(&r, &got, sizeof(T));
  return r;
}

// wave-wide vote: bit l of the result is lane l's predicate (64-lane waves)
inline unsigned long long __ballot(int pred) {
  const int t = (int)threadIdx.x;
  const int base = t - t % 64;
  auto& bar = *cpuhip::g_block.group_bar[6][t / 64];
  cpuhip::g_block.slot[t] = pred ? 1 : 0;
  bar.arrive_and_wait();
  unsigned long long m = 0;
  for (int l = 0; l < 64 && base + l < (int)(blockDim.x * blockDim.y * blockDim.z); ++l)
    if (cpuhip::g_block.slot[base + l]) m |= 1ull << l;
  bar.arrive_and_wait();
  return m;
}
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }

template <typename... KArgs, typename... Args>
inline void hipLaunchKernelGGL(void (*k)(KArgs...), dim3 grid, dim3 block, size_t shmem,
                               hipStream_t, Args... args) {
  // a fresh dynamic-LDS buffer per block, sized exactly as requested
  if (cpuhip::g_capture) {
    cpuhip::g_capture->push_back(
        [=] { cpuhip::launch(grid, block, [&] { k(args...); }, shmem); });
    return;
  }
  cpuhip::launch(grid, block, [&] { k(args...); }, shmem);
}

// ---- runtime API -------------------------------------------------------------
inline hipError_t hipMalloc(void** p, size_t bytes) {
  *p = malloc(bytes ? bytes : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
template <typename T>
inline hipError_t hipMalloc(T** p, size_t bytes) {
  return hipMalloc((void**)p, bytes);
}
inline hipError_t hipFree(void* p) {
  free(p);
  return hipSuccess;
}
inline hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) { return hipMalloc(p, bytes); }
inline hipError_t hipHostFree(void* p) { return hipFree(p); }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  memmove(d, s, n);
  return hipSuccess;
}
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  memset(d, v, n);
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamCreate(hipStream_t* s) {
  *s = (hipStream_t) new int(0);
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) {
  delete (int*)s;
  return hipSuccess;
}
using cpuhip_graph = std::vector<std::function<void()>>;
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) {
  if (cpuhip::g_capture) return hipErrorInvalidValue;
  cpuhip::g_capture = new cpuhip_graph();
  return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  *g = (hipGraph_t)cpuhip::g_capture;
  cpuhip::g_capture = nullptr;
  return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*,
                                      size_t) {
  *e = (hipGraphExec_t) new cpuhip_graph(*(cpuhip_graph*)g);
  return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) {
  delete (cpuhip_graph*)g;
  return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete (cpuhip_graph*)e;
  return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  for (auto& f : *(cpuhip_graph*)e) f();
  return hipSuccess;
}
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "cpuhip error"; }
// a device symbol's address is the host object's own address here
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) {
  *p = const_cast<void*>(sym);
  return hipSuccess;
}
inline hipError_t hipEventCreate(hipEvent_t* e) {
  *e = (hipEvent_t) new double(0);
  return hipSuccess;
}
#define hipEventDisableSystemFence 0x20000000
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete (double*)e;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  *(double*)e = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
  return hipSuccess;
}
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  *ms = (float)(1e3 * (*(double*)b - *(double*)a));
  return hipSuccess;
}
