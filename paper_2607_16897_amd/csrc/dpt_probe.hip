// Device characterisation for the roofline figures: attainable read
// bandwidth of a buffer that stays in L2 or in the last-level (MALL) cache,
// and attainable FP32 FMA throughput of the vector units as this library
// compiles them (no packed FP32 instructions).
#include <cstdint>

#include "../../include/dptrack.h"
#include "dpt_internal.h"

namespace dpt {
namespace {

// Workgroup w reads slice w % n_slices (slice_f4 float4, a multiple of 256)
// reps times, its threads strided by the workgroup size and starting at a
// workgroup-dependent offset (so that workgroups reading one slice spread over
// the cache channels); the sum only keeps the loads.
__global__ __launch_bounds__(256) void probe_read_kernel(const float4* __restrict__ buf, int64_t slice_f4,
                                                         int n_slices, int reps, float* __restrict__ sink) {
  const float4* s = buf + (int64_t)(blockIdx.x % n_slices) * slice_f4;
  const int64_t off = ((int64_t)blockIdx.x * 7919 * 256) % slice_f4;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int r = 0; r < reps; ++r)
    for (int64_t i = threadIdx.x; i < slice_f4; i += blockDim.x) {
      int64_t j = i + off;
      if (j >= slice_f4) j -= slice_f4;
      const float4 v = s[j];
      acc.x += v.x, acc.y += v.y, acc.z += v.z, acc.w += v.w;
    }
  if (acc.x + acc.y + acc.z + acc.w == 1.2345f) sink[threadIdx.x] = acc.x;  // not taken: the buffer is zero
}

// Eight independent FMA chains per thread.
__global__ __launch_bounds__(256) void probe_fma_kernel(int iters, float a, float b, float* __restrict__ sink) {
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = (float)(threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
  }
  float t = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) t += x[k];
  if (t == 1.2345f) sink[threadIdx.x] = t;
}

int cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return n;
}

// Milliseconds of the second of two launches of `launch` on the null stream
// (no stream of its own: a process that has used more streams than the GPU
// has hardware queues runs its later kernels slower).
template <class F>
int time_ms(F launch, float* ms) {
  const hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = DPT_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = set_error(DPT_E_HIP, "probe: event creation failed");
  } else {
    launch(st);  // warm-up: first touch of the buffer, code load
    if (hipEventRecord(e0, st) != hipSuccess) rc = set_error(DPT_E_HIP, "probe: event record");
    launch(st);
    if (rc == DPT_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipGetLastError() != hipSuccess || hipEventElapsedTime(ms, e0, e1) != hipSuccess))
      rc = set_error(DPT_E_HIP, "probe: launch or timing failed");
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace
}  // namespace dpt

using namespace dpt;

extern "C" {

int dpt_probe_read_bandwidth(int64_t slice_bytes, int32_t n_slices, int32_t reps, double* gbs) {
  if (!gbs || slice_bytes < 4096 || slice_bytes % 4096 || n_slices < 1 || reps < 1 ||
      slice_bytes * n_slices > ((int64_t)1 << 34))
    return set_error(DPT_E_ARG, "probe: slice_bytes a positive multiple of 4096, n_slices, reps >= 1, at most 16 GiB");
  const int n_cu = cus();
  if (n_cu <= 0) return set_error(DPT_E_HIP, "probe: no device");
  void* buf = nullptr;
  float* sink = nullptr;
  if (hipMalloc(&buf, slice_bytes * n_slices) != hipSuccess || hipMalloc(&sink, 256 * sizeof(float)) != hipSuccess) {
    if (buf) (void)hipFree(buf);
    return set_error(DPT_E_OOM, "probe: device allocation failed");
  }
  int rc = DPT_OK;
  if (hipMemset(buf, 0, slice_bytes * n_slices) != hipSuccess) rc = set_error(DPT_E_HIP, "probe: memset");
  const int grid = 8 * n_cu;
  float ms = 0.f;
  if (rc == DPT_OK)
    rc = time_ms(
        [&](hipStream_t st) {
          hipLaunchKernelGGL(probe_read_kernel, dim3(grid), dim3(256), 0, st, (const float4*)buf, slice_bytes / 16,
                             n_slices, reps, sink);
        },
        &ms);
  if (rc == DPT_OK) *gbs = (double)grid * reps * slice_bytes / (ms * 1e-3) / 1e9;
  (void)hipFree(buf);
  (void)hipFree(sink);
  return rc;
}

int dpt_probe_fp32_fma(int32_t iters, double* tflops) {
  if (!tflops || iters < 1) return set_error(DPT_E_ARG, "probe: iters >= 1");
  const int n_cu = cus();
  if (n_cu <= 0) return set_error(DPT_E_HIP, "probe: no device");
  float* sink = nullptr;
  if (hipMalloc(&sink, 256 * sizeof(float)) != hipSuccess) return set_error(DPT_E_OOM, "probe: device allocation");
  const int grid = 8 * n_cu;
  float ms = 0.f;
  const int rc = time_ms(
      [&](hipStream_t st) {
        hipLaunchKernelGGL(probe_fma_kernel, dim3(grid), dim3(256), 0, st, iters, 0.999f, 0.001f, sink);
      },
      &ms);
  if (rc == DPT_OK) *tflops = 2.0 * 8.0 * iters * 256.0 * grid / (ms * 1e-3) / 1e12;
  (void)hipFree(sink);
  return rc;
}

}  // extern "C"
