// qdse_peaks.hip -- the ceilings the rooflines are quoted against, measured
// on the device at hand: a streaming copy (HBM read + write bandwidth) and
// back-to-back matrix-core instructions of the two types the contraction uses
// (v_mfma_f32_16x16x4f32, v_mfma_f64_16x16x4f64), each with independent
// accumulators so that the issue rate, not a dependency, bounds the loop.
#include <vector>

#include <hip/hip_ext.h>

#include "qdse_internal.h"

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_copy(const double4* __restrict__ a,
                                              double4* __restrict__ b, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// Read-only streaming pass: four independent 32-byte loads per thread in
// flight, one sum per workgroup written.
__global__ void __launch_bounds__(256) k_read(const double4* __restrict__ a, long n,
                                              double* __restrict__ out) {
  const long stride = (long)gridDim.x * blockDim.x;
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const double4 v0 = a[i], v1 = a[i + stride], v2 = a[i + 2 * stride], v3 = a[i + 3 * stride];
    s += ((v0.x + v0.y) + (v0.z + v0.w)) + ((v1.x + v1.y) + (v1.z + v1.w)) +
         ((v2.x + v2.y) + (v2.z + v2.w)) + ((v3.x + v3.y) + (v3.z + v3.w));
  }
  for (; i < n; i += stride) {
    const double4 v = a[i];
    s += (v.x + v.y) + (v.z + v.w);
  }
  __shared__ double r[256];
  r[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < 256; ++k) t += r[k];
    out[blockIdx.x] = t;
  }
}

constexpr int kChains = 8;  // independent accumulators per wavefront

__global__ void __launch_bounds__(256) k_mfma32(int iters, float seed, float* out) {
  floatx4 acc[kChains];
  for (int c = 0; c < kChains; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  const float a = seed + threadIdx.x * 1e-7f, b = seed - threadIdx.x * 1e-7f;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  float s = 0.f;
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == 1234.5f) out[blockIdx.x] = s;  // keeps the loop; never true for the seeds used
}

__global__ void __launch_bounds__(256) k_mfma64(int iters, double seed, double* out) {
  doublex4 acc[kChains];
  for (int c = 0; c < kChains; ++c) acc[c] = doublex4{0.0, 0.0, 0.0, 0.0};
  const double a = seed + threadIdx.x * 1e-9, b = seed - threadIdx.x * 1e-9;
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  double s = 0.0;
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == 1234.5) out[blockIdx.x] = s;
}

// Launch-floor probes: a kernel that does nothing, and one that only streams
// `n` doubles (one coalesced pass, one store per workgroup).
__global__ void __launch_bounds__(256) k_empty(double* out) {
  if (threadIdx.x == 1023) out[0] = 1.0;  // never true at 256 threads
}

__global__ void __launch_bounds__(256) k_stream(const double* __restrict__ a, long per,
                                                double* __restrict__ out) {
  const double* p = a + (long)blockIdx.x * per;
  double s = 0.0;
  for (long j = threadIdx.x; j < per; j += blockDim.x) s += p[j];
  __shared__ double r[256];
  r[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 256; ++i) t += r[i];
    out[blockIdx.x] = t;
  }
}

// Average duration in ms of `reps` launches, each timed by events on its own
// dispatch packet (kernel execution only, as the contraction timings are).
template <class F>
int time_packets(hipStream_t st, int reps, F&& launch, double* ms_out) {
  std::vector<hipEvent_t> ev(2 * reps, nullptr);
  int rc = QDSE_OK;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) rc = QDSE_EDEVICE;
  if (!rc) {
    launch(nullptr, nullptr);  // warm-up
    for (int r = 0; r < reps; ++r) launch(ev[2 * r], ev[2 * r + 1]);
    double tot = 0.0;
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) rc = QDSE_EDEVICE;
    for (int r = 0; r < reps && !rc; ++r) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[2 * r], ev[2 * r + 1]) != hipSuccess) rc = QDSE_EDEVICE;
      tot += ms;
    }
    *ms_out = tot / reps;
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  return rc;
}

template <class F>
int time_ms(hipStream_t st, int reps, F&& launch, double* ms_out) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return QDSE_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return QDSE_EDEVICE;
  }
  launch();  // warm-up
  (void)hipEventRecord(e0, st);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, st);
  int rc = QDSE_OK;
  float ms = 0.f;
  if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
    rc = QDSE_EDEVICE;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_out = ms / reps;
  return rc;
}

}  // namespace

extern "C" int qdse_measure_peaks(void* hip_stream, double* copy_gbs, double* mfma32_tflops,
                                  double* mfma64_tflops, double* read_gbs) {
  hipStream_t st = (hipStream_t)hip_stream;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) != hipSuccess) return QDSE_EDEVICE;
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  int rc = QDSE_OK;
  if (read_gbs) {
    // 4 GiB read once per pass: sixteen times the 256 MB Infinity Cache
    const long n4 = (4l << 30) / (long)sizeof(double4);
    const int blocks = ncu * 16;
    double4* a = nullptr;
    double* o = nullptr;
    if (hipMalloc((void**)&a, n4 * sizeof(double4)) != hipSuccess ||
        hipMalloc((void**)&o, (size_t)blocks * sizeof(double)) != hipSuccess) {
      rc = QDSE_ENOMEM;
    } else if (hipMemsetAsync(a, 0, n4 * sizeof(double4), st) != hipSuccess) {
      rc = QDSE_EDEVICE;
    } else {
      double ms = 0.0;
      rc = time_ms(st, 5, [&] {
        hipLaunchKernelGGL(k_read, dim3(blocks), dim3(256), 0, st, (const double4*)a, n4, o);
      }, &ms);
      if (!rc) *read_gbs = (double)n4 * sizeof(double4) / (ms * 1e-3) / 1e9;
    }
    if (a) (void)hipFree(a);
    if (o) (void)hipFree(o);
    if (rc) return rc;
  }
  if (copy_gbs) {
    // 1 GiB each way, larger than the 256 MB Infinity Cache
    const long n4 = (1l << 30) / (long)sizeof(double4);
    double4 *a = nullptr, *b = nullptr;
    if (hipMalloc((void**)&a, n4 * sizeof(double4)) != hipSuccess ||
        hipMalloc((void**)&b, n4 * sizeof(double4)) != hipSuccess) {
      rc = QDSE_ENOMEM;
    } else if (hipMemsetAsync(a, 0, n4 * sizeof(double4), st) != hipSuccess) {
      rc = QDSE_EDEVICE;
    } else {
      double ms = 0.0;
      rc = time_ms(st, 5, [&] {
        hipLaunchKernelGGL(k_copy, dim3(ncu * 16), dim3(256), 0, st, (const double4*)a, b, n4);
      }, &ms);
      if (!rc) *copy_gbs = 2.0 * n4 * sizeof(double4) / (ms * 1e-3) / 1e9;
    }
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (rc) return rc;
  }
  float* o32 = nullptr;
  if (hipMalloc((void**)&o32, 64 * 1024 * sizeof(double)) != hipSuccess) return QDSE_ENOMEM;
  const int iters = 2000, blocks = ncu * 8;  // eight wavefront-groups of four per compute unit
  const double inst = (double)blocks * 4 * iters * kChains;  // wavefront instructions
  if (mfma32_tflops) {
    double ms = 0.0;
    rc = time_ms(st, 3, [&] {
      hipLaunchKernelGGL(k_mfma32, dim3(blocks), dim3(256), 0, st, iters, 0.5f, o32);
    }, &ms);
    if (!rc) *mfma32_tflops = inst * 2.0 * 16 * 16 * 4 / (ms * 1e-3) / 1e12;
  }
  if (!rc && mfma64_tflops) {
    double ms = 0.0;
    rc = time_ms(st, 3, [&] {
      hipLaunchKernelGGL(k_mfma64, dim3(blocks), dim3(256), 0, st, iters, 0.5, (double*)o32);
    }, &ms);
    if (!rc) *mfma64_tflops = inst * 2.0 * 16 * 16 * 4 / (ms * 1e-3) / 1e12;
  }
  (void)hipFree(o32);
  return rc;
}

extern "C" int qdse_measure_launch_floor(void* hip_stream, int workgroups, long long read_bytes,
                                         double* empty_us, double* read_us) {
  if (workgroups < 1 || read_bytes < 0) return QDSE_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  const long per = (long)((read_bytes / (long long)sizeof(double) + workgroups - 1) / workgroups);
  double *a = nullptr, *out = nullptr;
  if (hipMalloc((void**)&out, (size_t)workgroups * sizeof(double)) != hipSuccess) return QDSE_ENOMEM;
  int rc = QDSE_OK;
  if (per > 0 && hipMalloc((void**)&a, (size_t)per * workgroups * sizeof(double)) != hipSuccess)
    rc = QDSE_ENOMEM;
  if (!rc && a && hipMemsetAsync(a, 0, (size_t)per * workgroups * sizeof(double), st) != hipSuccess)
    rc = QDSE_EDEVICE;
  double ms = 0.0;
  if (!rc && empty_us) {
    rc = time_packets(st, 50, [&](hipEvent_t e0, hipEvent_t e1) {
      hipExtLaunchKernelGGL(k_empty, dim3(workgroups), dim3(256), 0, st, e0, e1, 0, out);
    }, &ms);
    if (!rc) *empty_us = ms * 1e3;
  }
  if (!rc && read_us) {
    rc = time_packets(st, 50, [&](hipEvent_t e0, hipEvent_t e1) {
      hipExtLaunchKernelGGL(k_stream, dim3(workgroups), dim3(256), 0, st, e0, e1, 0,
                            (const double*)a, per, out);
    }, &ms);
    if (!rc) *read_us = ms * 1e3;
  }
  (void)hipStreamSynchronize(st);
  if (a) (void)hipFree(a);
  (void)hipFree(out);
  return rc;
}
