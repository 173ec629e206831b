// STREAM-style HBM probe: a read-only kernel (16-byte loads, grid-stride,
// one partial sum per workgroup so the loads are not dead) and a copy
// kernel, timed with HIP events.  Used to state the per-match kernel's
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

__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const float4* __restrict__ src, int64_t n,
                                                              float* __restrict__ sink) {
  float acc = 0.f;
  const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
  int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * stride < n; i += kProbeUnroll * stride) {
    v4f v[kProbeUnroll];
    const v4f* s4 = reinterpret_cast<const v4f*>(src);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = __builtin_nontemporal_load(s4 + i + u * stride);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  for (; i < n; i += stride) {
    const float4 v = src[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  __shared__ float s[kProbeThreads];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kProbeThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) sink[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const float4* __restrict__ src, int64_t n,
                                                              float4* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
  for (int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x; i < n; i += stride) dst[i] = src[i];
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
  // 32 workgroups per CU: fewer leave HBM bandwidth unused (8 per CU read
  // ~6% less on a 1.4 GB stream)
  const int blocks = (hipGetDeviceProperties(&prop, device) == hipSuccess)
                         ? prop.multiProcessorCount * 32
                         : 8192;
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
      k_probe_read<<<blocks, kProbeThreads>>>(a, n, sink);
      (void)hipEventRecord(e1, nullptr);
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = FEA_EDEVICE;
        break;
      }
      if (r > 0) best_r = std::max(best_r, (double)n * 16 / (ms * 1e-3) / 1e9);
      (void)hipEventRecord(e0, nullptr);
      k_probe_copy<<<blocks, kProbeThreads>>>(a, n, b);
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
