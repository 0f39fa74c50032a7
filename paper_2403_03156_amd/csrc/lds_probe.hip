// lds_probe.hip -- LDS stream bandwidth of the device (the denominator of the chain kernels'
// LDS roofline): every lane of 16-wavefront workgroups reads (or writes) consecutive 16-byte
// words of a 32 KB LDS array, a wavefront's 1 KB per instruction without bank conflicts,
// eight independent accesses in flight per lane; the values read are folded with XOR so
// that no access is dropped.  Bytes moved / kernel time (HIP events), one launch after a
// warm-up launch.  Not part of the sampler: bench.py loads it for its roofline.

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kThreads = 1024;
constexpr int kWords = 2048;  // uint4 words: 32 KB per workgroup (four workgroups per CU)
constexpr int kUnroll = 8;

__global__ void __launch_bounds__(kThreads) lds_read_kernel(int iters, uint32_t *sink) {
  __shared__ uint4 buf[kWords];
  const int t = threadIdx.x;
  for (int i = t; i < kWords; i += kThreads) buf[i] = make_uint4(i, 3 * i, 5 * i, 7 * i);
  __syncthreads();
  uint32_t acc = 0;
  for (int it = 0; it < iters; ++it) {
    const int base = (it * 64 + t) & (kWords - 1);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const uint4 v = buf[(base + u * 256) & (kWords - 1)];
      acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
  }
  if (acc == 0x9E3779B9u) sink[blockIdx.x] = acc;  // keeps the reads; practically never taken
}

__global__ void __launch_bounds__(kThreads) lds_write_kernel(int iters, uint32_t *sink) {
  __shared__ uint4 buf[kWords];
  const int t = threadIdx.x;
  for (int it = 0; it < iters; ++it) {
    const int base = (it * 64 + t) & (kWords - 1);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) buf[(base + u * 256) & (kWords - 1)] = make_uint4(it, t, u, it ^ t);
  }
  __syncthreads();
  const uint4 v = buf[t & (kWords - 1)];
  if ((v.x ^ v.y ^ v.z ^ v.w) == 0x9E3779B9u) sink[blockIdx.x] = v.x;
}

}  // namespace

// Measured LDS bandwidth of `device` in bytes/s (reads, writes); 0 on success, else the
// HIP error code.
extern "C" int lds_probe(int device, int iters, double *read_bps, double *write_bps) {
  hipError_t e = hipSetDevice(device);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return (int)e;
  const int blocks = prop.multiProcessorCount * 4 * 8;
  uint32_t *sink = nullptr;
  e = hipMalloc((void **)&sink, sizeof(uint32_t) * blocks);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const double bytes = (double)blocks * kThreads * iters * kUnroll * 16.0;
  for (int w = 0; w < 2 && e == hipSuccess; ++w) {
    double *out = w == 0 ? read_bps : write_bps;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // a warm-up launch, then the timed one
      e = hipEventRecord(e0, nullptr);
      if (w == 0) hipLaunchKernelGGL(lds_read_kernel, dim3(blocks), dim3(kThreads), 0, nullptr, iters, sink);
      else hipLaunchKernelGGL(lds_write_kernel, dim3(blocks), dim3(kThreads), 0, nullptr, iters, sink);
      if (e == hipSuccess) e = hipGetLastError();
      if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess) *out = bytes / (ms * 1e-3);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (sink) (void)hipFree(sink);
  return (int)e;
}
