// CPU emulation of the part of the HIP runtime and device language the library's sources
// use, for running the library's kernels through its own host code on the CPU, under
// AddressSanitizer (tests/test_cpu_emu.py).  Test infrastructure only: "device" memory is
// host memory, copies are synchronous, streams and events do nothing, and a kernel launch runs
// its blocks one after the other with one OS thread per GPU thread.  Barriers: a std::barrier
// per block for __syncthreads and one per wavefront of 64 threads for the wavefront barrier.
// Cross-lane operations (shuffles, the DPP patterns the kernels use, ballot, lane reads) go through a
// per-wavefront exchange: each lane writes its value to its slot, the wavefront passes its
// barrier, each lane reads the slot of its source lane, and the wavefront passes its barrier
// again.  A lane's phases pair with those of the other lanes of its wavefront whatever code
// they run, so lanes of different chains of one wavefront may take different branches, as
// long as every exchange reads a lane of the same chain (all the kernels' do).
#pragma once
#include <barrier>
#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/asan_interface.h>
#endif
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __shared__
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) ((const void *)&(x))

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct emu_idx {
  unsigned x, y, z;
};
inline thread_local emu_idx emu_threadIdx{0, 0, 0}, emu_blockIdx{0, 0, 0}, emu_blockDim{1, 1, 1},
    emu_gridDim{1, 1, 1};
inline thread_local std::barrier<> *emu_bar = nullptr;
inline thread_local std::barrier<> *emu_wbar = nullptr;  // the thread's wavefront barrier
inline thread_local uint64_t *emu_xbuf = nullptr;        // its wavefront's exchange slots [64]
inline thread_local int emu_lane = 0;                    // its lane in the wavefront
inline thread_local int emu_or_gen = 0;
inline int emu_or_acc[2];
#define threadIdx emu_threadIdx
#define blockIdx emu_blockIdx
#define blockDim emu_blockDim
#define gridDim emu_gridDim

[[noreturn]] inline void emu_unreachable(const char *what) {
  std::fprintf(stderr, "cpu emulation: %s reached\n", what);
  std::abort();
}

inline void __syncthreads() { emu_bar->arrive_and_wait(); }
inline int __syncthreads_or(int v) {
  const int g = emu_or_gen++ & 1;
  if (v) __atomic_fetch_or(&emu_or_acc[g], 1, __ATOMIC_SEQ_CST);
  emu_bar->arrive_and_wait();
  const int r = __atomic_load_n(&emu_or_acc[g], __ATOMIC_SEQ_CST);
  if (emu_threadIdx.x == 0) __atomic_store_n(&emu_or_acc[g ^ 1], 0, __ATOMIC_SEQ_CST);
  emu_bar->arrive_and_wait();
  return r;
}
// one exchange phase: write this lane's bits, read lane src's (0..63)
inline uint64_t emu_exchange(uint64_t mine, int src) {
  emu_xbuf[emu_lane] = mine;
  emu_wbar->arrive_and_wait();
  const uint64_t r = emu_xbuf[src & 63];
  emu_wbar->arrive_and_wait();
  return r;
}
template <typename T>
uint64_t emu_bits(T v) {
  static_assert(sizeof(T) <= 8, "exchange of at most 64 bits");
  uint64_t u = 0;
  std::memcpy(&u, &v, sizeof(T));
  return u;
}
template <typename T>
T emu_from_bits(uint64_t u) {
  T v;
  std::memcpy(&v, &u, sizeof(T));
  return v;
}
// HIP's definitions: __shfl reads lane src + the first lane of the caller's width segment;
// __shfl_xor reads lane ^ mask, or the caller's own value if that leaves its segment
template <typename T>
T __shfl(T v, int src, int width = 64) {
  const int index = src + (emu_lane & ~(width - 1));
  return emu_from_bits<T>(emu_exchange(emu_bits(v), index));
}
template <typename T>
T __shfl_xor(T v, int mask, int width = 64) {
  int index = emu_lane ^ mask;
  if (index >= ((emu_lane + width) & ~(width - 1))) index = emu_lane;
  return emu_from_bits<T>(emu_exchange(emu_bits(v), index));
}
inline unsigned long long __ballot(int pred) {
  emu_xbuf[emu_lane] = pred ? 1u : 0u;
  emu_wbar->arrive_and_wait();
  unsigned long long m = 0;
  for (int l = 0; l < 64; ++l) m |= (unsigned long long)(emu_xbuf[l] != 0) << l;
  emu_wbar->arrive_and_wait();
  return m;
}
// DPP moves: quad_perm, row_ror:1..15 (lane i of a row of 16 reads lane i - n), row_newbcast:k;
// every source lane exists for these, so old, the masks and bound_ctrl do not matter
inline int emu_update_dpp(int old, int src, int ctrl, int, int, bool) {
  (void)old;
  int from;
  if (ctrl >= 0 && ctrl <= 0xFF) from = (emu_lane & ~3) | ((ctrl >> (2 * (emu_lane & 3))) & 3);
  else if (ctrl >= 0x121 && ctrl <= 0x12F) from = (emu_lane & ~15) | (((emu_lane & 15) - (ctrl & 15)) & 15);
  else if (ctrl >= 0x150 && ctrl <= 0x15F) from = (emu_lane & ~15) | (ctrl & 15);
  else emu_unreachable("a DPP control the emulation does not model");
  return emu_from_bits<int>(emu_exchange(emu_bits(src), from));
}
#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) emu_update_dpp((old), (src), (ctrl), (rm), (bm), (bc))
// the value of the wavefront's first active lane (the kernels take it where every lane is active)
inline int emu_readfirstlane(int v) { return emu_from_bits<int>(emu_exchange(emu_bits(v), 0)); }
#define __builtin_amdgcn_readfirstlane(v) emu_readfirstlane((v))
// the value of lane L of the wavefront
inline int emu_readlane(int v, int L) { return emu_from_bits<int>(emu_exchange(emu_bits(v), L)); }
#define __builtin_amdgcn_readlane(v, L) emu_readlane((v), (L))
#define __builtin_amdgcn_fence(...) ((void)0)
#define __builtin_amdgcn_wave_barrier() emu_wbar->arrive_and_wait()
inline int __double2loint(double v) {
  long long u;
  std::memcpy(&u, &v, 8);
  return (int)(u & 0xffffffffLL);
}
inline int __double2hiint(double v) {
  long long u;
  std::memcpy(&u, &v, 8);
  return (int)(u >> 32);
}
inline double __hiloint2double(int hi, int lo) {
  const unsigned long long u = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
  double v;
  std::memcpy(&v, &u, 8);
  return v;
}
inline int max(int a, int b) { return a > b ? a : b; }
inline int min(int a, int b) { return a < b ? a : b; }
inline int __ffsll(unsigned long long v) { return __builtin_ffsll((long long)v); }

template <typename T>
T atomicAdd(T *p, T v) {
  if constexpr (std::is_integral<T>::value) {
    return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
  } else {
    T old = __atomic_load_n(p, __ATOMIC_SEQ_CST);
    while (!__atomic_compare_exchange_n(p, &old, old + v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
    }
    return old;
  }
}

// ---- runtime
enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidDevice = 101,
  hipErrorNotSupported = 801,
};
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice,
                     hipMemcpyDefault };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
constexpr unsigned hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipHostMallocDefault = 0;
struct emu_handle {
  int unused;
};
typedef emu_handle *hipStream_t;
typedef emu_handle *hipEvent_t;
typedef emu_handle *hipGraph_t;
typedef emu_handle *hipGraphExec_t;
struct hipDeviceProp_t {
  char gcnArchName[256];
  int multiProcessorCount;
  size_t totalGlobalMem;
};

inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char *hipGetErrorString(hipError_t) { return "cpu emulation error"; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
inline hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
inline hipError_t hipGetDeviceCount(int *n) { *n = 1; return hipSuccess; }
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int) {
  std::memset(p, 0, sizeof *p);
  std::strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-");
  p->multiProcessorCount = 256;
  p->totalGlobalMem = (size_t)288 << 30;
  return hipSuccess;
}
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipMalloc(void **p, size_t n) {
  *p = std::malloc(n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void *p) { std::free(p); return hipSuccess; }
inline hipError_t hipHostMalloc(void **p, size_t n, unsigned) { return hipMalloc(p, n); }
inline hipError_t hipHostFree(void *p) { return hipFree(p); }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
  if (n) std::memcpy(d, s, n);
  return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t = nullptr) {
  return hipMemcpy(d, s, n, k);
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = new emu_handle{0}; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = new emu_handle{0}; return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t = nullptr) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 0.0f; return hipSuccess; }
inline hipError_t hipFuncSetAttribute(const void *, hipFuncAttribute, int) { return hipSuccess; }
inline hipError_t hipGetSymbolAddress(void **p, const void *sym) { *p = const_cast<void *>(sym); return hipSuccess; }
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) { *g = nullptr; return hipErrorNotSupported; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t *, hipGraph_t, void *, char *, size_t) {
  return hipErrorNotSupported;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }

// the kernels' dynamic LDS (each launch's blocks run one at a time, so one array per name);
// declared in the library's namespaces, where the kernels' block-scope declarations find them.
// A launch poisons each array beyond the bytes it asked for, so that AddressSanitizer reports
// an LDS access past the launch's size.
namespace fsmp {
namespace {
constexpr size_t emu_lds_bytes = 160 * 1024;
alignas(16) double vt[emu_lds_bytes / 8];
alignas(16) double smem[emu_lds_bytes / 8];
alignas(16) double lds[emu_lds_bytes / 8];
}  // namespace
}  // namespace fsmp

inline void emu_lds_limit(size_t bytes) {
#if defined(__SANITIZE_ADDRESS__)
  for (double *a : {fsmp::vt, fsmp::smem, fsmp::lds}) {
    __asan_unpoison_memory_region(a, fsmp::emu_lds_bytes);
    if (bytes < fsmp::emu_lds_bytes) __asan_poison_memory_region((char *)a + bytes, fsmp::emu_lds_bytes - bytes);
  }
#else
  (void)bytes;
#endif
}

// a launch: the blocks one after the other, one thread per GPU thread of a block; a thread
// that returns leaves the block's barrier
template <typename... KA, typename... A>
void emu_launch(void (*k)(KA...), dim3 g, dim3 b, size_t lds_bytes, A... args) {
  if (g.y != 1 || g.z != 1 || b.y != 1 || b.z != 1) emu_unreachable("a multi-dimensional launch");
  if (lds_bytes > fsmp::emu_lds_bytes) emu_unreachable("a launch asking for more than 160 KiB of LDS");
  emu_lds_limit(lds_bytes);
  const unsigned n_waves = (b.x + 63) / 64;
  for (unsigned bx = 0; bx < g.x; ++bx) {
    std::barrier<> bar((std::ptrdiff_t)b.x);
    std::vector<std::unique_ptr<std::barrier<>>> wbar;
    std::vector<uint64_t> xbuf(64 * n_waves, 0);
    for (unsigned w = 0; w < n_waves; ++w)
      wbar.emplace_back(new std::barrier<>((std::ptrdiff_t)std::min(64u, b.x - 64 * w)));
    emu_or_acc[0] = emu_or_acc[1] = 0;
    std::vector<std::thread> th;
    th.reserve(b.x);
    for (unsigned t = 0; t < b.x; ++t)
      th.emplace_back([&, t] {
        emu_threadIdx = {t, 0, 0};
        emu_blockIdx = {bx, 0, 0};
        emu_blockDim = {b.x, 1, 1};
        emu_gridDim = {g.x, 1, 1};
        emu_bar = &bar;
        emu_wbar = wbar[t / 64].get();
        emu_xbuf = xbuf.data() + 64 * (t / 64);
        emu_lane = (int)(t % 64);
        emu_or_gen = 0;
        k(args...);
        // a lane that has left reads as 0 in a ballot and no longer holds up its wavefront
        emu_xbuf[emu_lane] = 0;
        emu_wbar->arrive_and_drop();
        bar.arrive_and_drop();
        emu_bar = nullptr;
        emu_wbar = nullptr;
      });
    for (auto &x : th) x.join();
  }
  emu_lds_limit(fsmp::emu_lds_bytes);
}
#define hipLaunchKernelGGL(K, G, B, L, S, ...) emu_launch(K, dim3(G), dim3(B), (size_t)(L), __VA_ARGS__)

