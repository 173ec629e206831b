// STREAM-style HBM probe: a read-only kernel and a copy kernel over a
// buffer of the caller's size (16-byte non-temporal loads, one workgroup per
// contiguous chunk), timed with HIP events.  Used to state the per-match kernel's
// bandwidth against what plain streaming reaches on the same GPU.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fastea.h"

namespace {

constexpr int kProbeThreads = 256;

// Each thread keeps kProbeUnroll independent 16-byte loads in flight per
// iteration; consecutive threads read consecutive vectors.
constexpr int kProbeUnroll = 4;
typedef float v4f __attribute__((ext_vector_type(4)));

// Workgroup b reads the contiguous chunk of kProbeThreads * kProbeUnroll
// vectors starting at b * kProbeThreads * kProbeUnroll, every thread issuing
// its kProbeUnroll non-temporal 16-byte loads together (consecutive threads
// read consecutive vectors).  One workgroup per chunk, so the dispatcher
// hands chunks to CUs as they free up: a sweep of shapes on a 1.4 GB stream
// found this the fastest read (a grid-stride loop with a fixed grid read
// ~10% less).  The sum is stored only when it equals -1, which the probe's
// positive data never does, so the loads are kept without a write per
// workgroup.
__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const float4* __restrict__ src, int64_t n,
                                                              float* __restrict__ sink) {
  const v4f* s4 = reinterpret_cast<const v4f*>(src);
  const int64_t base = (int64_t)blockIdx.x * kProbeThreads * kProbeUnroll + threadIdx.x;
  v4f v[kProbeUnroll];
#pragma unroll
  for (int u = 0; u < kProbeUnroll; ++u) {
    const int64_t i = base + (int64_t)u * kProbeThreads;
    v[u] = i < n ? __builtin_nontemporal_load(s4 + i) : (v4f){0.f, 0.f, 0.f, 0.f};
  }
  float acc = 0.f;
#pragma unroll
  for (int u = 0; u < kProbeUnroll; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  if (acc == -1.f) sink[0] = acc;
}

// The same chunks copied: every thread's kProbeUnroll loads, then its stores.
__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const float4* __restrict__ src, int64_t n,
                                                              float4* __restrict__ dst) {
  const v4f* s4 = reinterpret_cast<const v4f*>(src);
  v4f* d4 = reinterpret_cast<v4f*>(dst);
  const int64_t base = (int64_t)blockIdx.x * kProbeThreads * kProbeUnroll + threadIdx.x;
  v4f v[kProbeUnroll];
#pragma unroll
  for (int u = 0; u < kProbeUnroll; ++u) {
    const int64_t i = base + (int64_t)u * kProbeThreads;
    if (i < n) v[u] = __builtin_nontemporal_load(s4 + i);
  }
#pragma unroll
  for (int u = 0; u < kProbeUnroll; ++u) {
    const int64_t i = base + (int64_t)u * kProbeThreads;
    if (i < n) __builtin_nontemporal_store(v[u], d4 + i);
  }
}

__global__ void k_probe_fill(float4* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = make_float4(1.f, 2.f, 3.f, (float)(i & 1023));
}

}  // namespace

extern "C" fea_status fea_hbm_probe(int32_t device, int64_t bytes, int32_t reps, double* read_gbps,
                                    double* copy_gbps) {
  if (bytes < (1 << 20) || reps < 1 || !read_gbps || !copy_gbps) return FEA_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FEA_EINVAL;
  int prev = 0;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(device) != hipSuccess) return FEA_EDEVICE;
  const int64_t n = bytes / 16;
  float4 *a = nullptr, *b = nullptr;
  float* sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  fea_status st = FEA_OK;
  hipDeviceProp_t prop;
  // the fill kernel's grid: 32 workgroups per CU, grid-stride
  const int blocks = (hipGetDeviceProperties(&prop, device) == hipSuccess)
                         ? prop.multiProcessorCount * 32
                         : 8192;
  // the read and copy kernels' grid: one workgroup per chunk
  const int64_t chunk = (int64_t)kProbeThreads * kProbeUnroll;
  const unsigned chunks = (unsigned)((n + chunk - 1) / chunk);
  if (hipMalloc(&a, n * 16) != hipSuccess || hipMalloc(&b, n * 16) != hipSuccess ||
      hipMalloc(&sink, blocks * sizeof(float)) != hipSuccess) {
    st = FEA_ENOMEM;
  } else if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    st = FEA_EDEVICE;
  } else {
    k_probe_fill<<<blocks, kProbeThreads>>>(a, n);
    k_probe_fill<<<blocks, kProbeThreads>>>(b, n);
    double best_r = 0.0, best_c = 0.0;
    for (int r = 0; r < reps + 1 && st == FEA_OK; ++r) {
      float ms = 0.f;
      (void)hipEventRecord(e0, nullptr);
      k_probe_read<<<chunks, kProbeThreads>>>(a, n, sink);
      (void)hipEventRecord(e1, nullptr);
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = FEA_EDEVICE;
        break;
      }
      if (r > 0) best_r = std::max(best_r, (double)n * 16 / (ms * 1e-3) / 1e9);
      (void)hipEventRecord(e0, nullptr);
      k_probe_copy<<<chunks, kProbeThreads>>>(a, n, b);
      (void)hipEventRecord(e1, nullptr);
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = FEA_EDEVICE;
        break;
      }
      if (r > 0) best_c = std::max(best_c, (double)n * 32 / (ms * 1e-3) / 1e9);
    }
    *read_gbps = best_r;
    *copy_gbps = best_c;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  if (sink) (void)hipFree(sink);
  (void)hipSetDevice(prev);
  return st;
}
