// Segmenting on the GPU: validate matches, give each its canonical camera
// pair (i < j, keypoints swapped when needed), stable-sort by pair with an
// LSD radix sort, find the pair runs and gather the structure-of-arrays
// device layout.  This is the data marshalling that precedes the epipolar
// adjustment iterations (FastMap, Experiments: marshalling done on the GPU
// with tensor indexing); here every step is an integer kernel so the result
// is bit-exact and deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "fea_ctx.h"
#include "fea_device.h"

namespace fea {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kScanTile = kScanThreads * kScanPer;
constexpr int kRadixBits = 4;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRsThreads = 256;
constexpr int kRsPer = 8;
constexpr int kRsTile = kRsThreads * kRsPer;

// Exclusive scan of a 256-thread block's values; returns this thread's
// exclusive prefix and writes the block total to *total.
__device__ int block_exclusive_scan(int v, int* total, int* s_w) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int inc = wave_inclusive_scan(v);
  if (lane == 63) s_w[wid] = inc;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / 64; ++w) {
    const int x = s_w[w];
    before += (w < wid) ? x : 0;
    all += x;
  }
  __syncthreads();
  *total = all;
  return before + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_tile(int* __restrict__ data, int64_t n,
                                                             int* __restrict__ tile_sums) {
  __shared__ int s_w[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  int v[kScanPer];
  int sum = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (base + k < n) ? data[base + k] : 0;
    sum += v[k];
  }
  int total;
  int run = block_exclusive_scan(sum, &total, s_w);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) data[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0 && tile_sums) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(int* __restrict__ data, int64_t n,
                                                            const int* __restrict__ offs) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  const int o = offs[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < n) data[base + k] += o;
}

// In-place exclusive scan of n ints; scratch must hold scan_scratch_ints(n).
int64_t scan_scratch_ints(int64_t n) {
  int64_t need = 0;
  while (n > kScanTile) {
    n = (n + kScanTile - 1) / kScanTile;
    need += n;
  }
  return need + 1;
}

hipError_t device_exclusive_scan(int* data, int64_t n, int* scratch, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  if (tiles == 1) {
    k_scan_tile<<<1, kScanThreads, 0, st>>>(data, n, nullptr);
    return hipGetLastError();
  }
  k_scan_tile<<<(unsigned)tiles, kScanThreads, 0, st>>>(data, n, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = device_exclusive_scan(scratch, tiles, scratch + tiles, st);
  if (e != hipSuccess) return e;
  k_scan_add<<<(unsigned)tiles, kScanThreads, 0, st>>>(data, n, scratch);
  return hipGetLastError();
}

// Validation and canonical keys: key = i * N + j with i < j.
__global__ void k_validate(int64_t n, int N, const int32_t* __restrict__ cam1, const int32_t* __restrict__ cam2,
                           const float* __restrict__ x1, const float* __restrict__ y1,
                           const float* __restrict__ x2, const float* __restrict__ y2,
                           uint32_t* __restrict__ keys, int32_t* __restrict__ vals, int* __restrict__ err) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  const int c1 = cam1[m], c2 = cam2[m];
  int bits = 0;
  if (c1 < 0 || c1 >= N || c2 < 0 || c2 >= N)
    bits |= kErrRange;
  else if (c1 == c2)
    bits |= kErrSameCam;
  if (!isfinite(x1[m]) || !isfinite(y1[m]) || !isfinite(x2[m]) || !isfinite(y2[m])) bits |= kErrNonFinite;
  if (bits) atomicOr(err, bits);
  const uint32_t i = (uint32_t)min(max(min(c1, c2), 0), N - 1);
  const uint32_t j = (uint32_t)min(max(max(c1, c2), 0), N - 1);
  keys[m] = i * (uint32_t)N + j;
  vals[m] = (int32_t)m;
}

__global__ __launch_bounds__(kRsThreads) void k_radix_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                           int shift, int n_tiles, int* __restrict__ hist) {
  __shared__ int h[kRadixBins];
  if (threadIdx.x < kRadixBins) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile + (int64_t)threadIdx.x * kRsPer;
#pragma unroll
  for (int k = 0; k < kRsPer; ++k)
    if (base + k < n) atomicAdd(&h[(keys[base + k] >> shift) & (kRadixBins - 1)], 1);
  __syncthreads();
  if (threadIdx.x < kRadixBins) hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one radix pass.  Within a tile, thread t owns the kRsPer
// consecutive keys starting at t*kRsPer; ranks follow (thread, position), so
// equal digits keep their input order.
__global__ __launch_bounds__(kRsThreads) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                              const int32_t* __restrict__ vin,
                                                              uint32_t* __restrict__ kout,
                                                              int32_t* __restrict__ vout, int64_t n, int shift,
                                                              int n_tiles, const int* __restrict__ offs) {
  __shared__ int s_cnt[kRadixBins * kRsThreads];  // digit-major [d][t]
  __shared__ int s_w[kRsThreads / 64];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kRsTile + (int64_t)tid * kRsPer;
  uint32_t key[kRsPer];
  int32_t val[kRsPer];
  int dg[kRsPer];
#pragma unroll
  for (int k = 0; k < kRsPer; ++k) {
    const bool ok = base + k < n;
    key[k] = ok ? kin[base + k] : 0u;
    val[k] = ok ? vin[base + k] : 0;
    dg[k] = ok ? (int)((key[k] >> shift) & (kRadixBins - 1)) : -1;
  }
#pragma unroll
  for (int d = 0; d < kRadixBins; ++d) {
    int c = 0;
#pragma unroll
    for (int k = 0; k < kRsPer; ++k) c += (dg[k] == d);
    s_cnt[d * kRsThreads + tid] = c;
  }
  __syncthreads();
  // exclusive scan of the flattened digit-major array (16 entries per thread)
  int loc[kRadixBins];
  int sum = 0;
#pragma unroll
  for (int k = 0; k < kRadixBins; ++k) {
    loc[k] = s_cnt[tid * kRadixBins + k];
    sum += loc[k];
  }
  int total;
  int run = block_exclusive_scan(sum, &total, s_w);
#pragma unroll
  for (int k = 0; k < kRadixBins; ++k) {
    const int x = loc[k];
    loc[k] = run;
    run += x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRadixBins; ++k) s_cnt[tid * kRadixBins + k] = loc[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRsPer; ++k) {
    if (dg[k] < 0) continue;
    const int d = dg[k];
    int r = 0;
#pragma unroll
    for (int q = 0; q < kRsPer; ++q) r += (q < k) && (dg[q] == d);
    const int local = s_cnt[d * kRsThreads + tid] - s_cnt[d * kRsThreads];
    const int64_t dst = (int64_t)offs[(int64_t)d * n_tiles + blockIdx.x] + local + r;
    kout[dst] = key[k];
    vout[dst] = val[k];
  }
}

__global__ void k_head_flags(const uint32_t* __restrict__ sk, int64_t n, int* __restrict__ flag) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) flag[p] = (p == 0 || sk[p] != sk[p - 1]) ? 1 : 0;
}

__global__ void k_heads(const uint32_t* __restrict__ sk, const int* __restrict__ excl, int64_t n,
                        uint32_t* __restrict__ pair_key, int32_t* __restrict__ seg_start,
                        int32_t* __restrict__ pid, int* __restrict__ n_pairs) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int head = (p == 0 || sk[p] != sk[p - 1]) ? 1 : 0;
  const int id = excl[p] + head - 1;
  pid[p] = id;
  if (head) {
    pair_key[id] = sk[p];
    seg_start[id] = (int32_t)p;
  }
  if (p == n - 1) *n_pairs = id + 1;
}

__global__ void k_gather(int64_t n, const int32_t* __restrict__ sv, const int32_t* __restrict__ pid,
                         const int32_t* __restrict__ seg_start, const int32_t* __restrict__ phys_off,
                         const float* __restrict__ x1, const float* __restrict__ y1,
                         const float* __restrict__ x2, const float* __restrict__ y2,
                         const int32_t* __restrict__ cam1, const int32_t* __restrict__ cam2,
                         float* __restrict__ ox1, float* __restrict__ oy1, float* __restrict__ ox2,
                         float* __restrict__ oy2, int32_t* __restrict__ opos, int32_t* __restrict__ perm,
                         uint8_t* __restrict__ swp) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t m = sv[p];
  const int32_t k = pid[p];
  const int64_t dst = (int64_t)phys_off[k] + (p - seg_start[k]);
  const bool s = cam1[m] > cam2[m];
  const float a = x1[m], b = y1[m], c = x2[m], d = y2[m];
  ox1[dst] = s ? c : a;
  oy1[dst] = s ? d : b;
  ox2[dst] = s ? a : c;
  oy2[dst] = s ? b : d;
  opos[dst] = (int32_t)p;
  perm[p] = m;
  swp[p] = s ? 1 : 0;
}

struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  hipError_t alloc(T** out, size_t count) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) ptrs.push_back(p);
    *out = static_cast<T*>(p);
    return e;
  }
};

#define FEA_TRY(expr)                    \
  do {                                   \
    hipError_t _e = (expr);              \
    if (_e != hipSuccess) return _e;     \
  } while (0)

hipError_t alloc_dbuf(DBuf& b, size_t bytes) {
  if (b.p && b.bytes >= bytes) return hipSuccess;
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
  FEA_TRY(hipMalloc(&b.p, std::max<size_t>(bytes, 16)));
  b.bytes = bytes;
  return hipSuccess;
}

// Export, pass 1: the coordinates of every real slot of the full layout to
// its sorted position (padding slots hold lpos = -1).
__global__ void k_export_coords(int64_t n_slots, const int32_t* __restrict__ lpos, const float* __restrict__ x1,
                                const float* __restrict__ y1, const float* __restrict__ x2,
                                const float* __restrict__ y2, float* __restrict__ ox1, float* __restrict__ oy1,
                                float* __restrict__ ox2, float* __restrict__ oy2) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_slots) return;
  const int32_t q = lpos[s];
  if (q < 0) return;
  ox1[q] = x1[s];
  oy1[q] = y1[s];
  ox2[q] = x2[s];
  oy2[q] = y2[s];
}

// Export, pass 2: one workgroup per pair writes the pair's camera ids
// (offset by cam_base) over its sorted range.
__global__ void k_export_cams(const int64_t* __restrict__ seg_off, const int32_t* __restrict__ pair_i,
                              const int32_t* __restrict__ pair_j, int32_t cam_base, int32_t* __restrict__ c1,
                              int32_t* __restrict__ c2) {
  const int n = blockIdx.x;
  const int32_t a = pair_i[n] + cam_base, b = pair_j[n] + cam_base;
  for (int64_t q = seg_off[n] + threadIdx.x; q < seg_off[n + 1]; q += blockDim.x) {
    c1[q] = a;
    c2[q] = b;
  }
}

}  // namespace

// The loaded matches in sorted order (each canonical, lower camera first),
// into device arrays [n_matches] of the context's device: coordinates as
// loaded, camera ids offset by cam_base.  seg_off_dev: the pair ranges
// [P + 1] on the device (caller-provided scratch).
hipError_t export_sorted(fea_ctx* c, int32_t cam_base, const int64_t* seg_off_dev, float* x1, float* y1,
                         float* x2, float* y2, int32_t* cam1, int32_t* cam2) {
  int64_t slots = 0;
  for (int64_t n = 0; n < c->P; ++n)
    slots += (c->seg_off[n + 1] - c->seg_off[n] + kAlign - 1) / kAlign * kAlign;
  if (slots > 0)
    k_export_coords<<<(unsigned)((slots + 255) / 256), 256, 0, c->stream>>>(
        slots, c->lpos[0].as<int32_t>(), c->lay[0][0].as<float>(), c->lay[0][1].as<float>(),
        c->lay[0][2].as<float>(), c->lay[0][3].as<float>(), x1, y1, x2, y2);
  if (c->P > 0)
    k_export_cams<<<(unsigned)c->P, 256, 0, c->stream>>>(seg_off_dev, c->d_pair_i.as<int32_t>(),
                                                       c->d_pair_j.as<int32_t>(), cam_base, cam1, cam2);
  return hipGetLastError();
}

hipError_t segment_matches(fea_ctx* c, const float* x1, const float* y1, const float* x2, const float* y2,
                           const int32_t* cam1, const int32_t* cam2, int* bad_bits) {
  hipStream_t st = c->stream;
  const int64_t M = c->M;
  const int N = c->N;
  *bad_bits = 0;
  Scratch s;
  uint32_t *k0, *k1, *pair_key;
  int32_t *v0, *v1, *pid, *seg_start, *phys32;
  int *flag, *err, *npairs, *scan_scr;
  FEA_TRY(s.alloc(&k0, M));
  FEA_TRY(s.alloc(&k1, M));
  FEA_TRY(s.alloc(&v0, M));
  FEA_TRY(s.alloc(&v1, M));
  FEA_TRY(s.alloc(&err, 2));
  FEA_TRY(hipMemsetAsync(err, 0, 2 * sizeof(int), st));
  const unsigned g256 = (unsigned)((M + 255) / 256);
  if (M > 0) {
    k_validate<<<g256, 256, 0, st>>>(M, N, cam1, cam2, x1, y1, x2, y2, k0, v0, err);
    FEA_TRY(hipGetLastError());
  }
  int h_err = 0;
  FEA_TRY(hipMemcpyAsync(&h_err, err, sizeof(int), hipMemcpyDeviceToHost, st));
  FEA_TRY(hipStreamSynchronize(st));
  if (h_err) {
    *bad_bits = h_err;
    return hipSuccess;
  }
  // LSD radix sort of (key, input index) by key
  const uint64_t max_key = (uint64_t)N * (uint64_t)N;
  int bits = 1;
  while (bits < 32 && (1ull << bits) < max_key) ++bits;
  const int passes = (bits + kRadixBits - 1) / kRadixBits;
  const int64_t n_tiles = (M + kRsTile - 1) / kRsTile;
  int* hist;
  const int64_t hist_n = kRadixBins * std::max<int64_t>(n_tiles, 1);
  FEA_TRY(s.alloc(&hist, hist_n));
  FEA_TRY(s.alloc(&scan_scr, scan_scratch_ints(std::max<int64_t>(hist_n, M))));
  uint32_t *kin = k0, *kout = k1;
  int32_t *vin = v0, *vout = v1;
  if (M > 0) {
    for (int ps = 0; ps < passes; ++ps) {
      const int shift = ps * kRadixBits;
      k_radix_hist<<<(unsigned)n_tiles, kRsThreads, 0, st>>>(kin, M, shift, (int)n_tiles, hist);
      FEA_TRY(hipGetLastError());
      FEA_TRY(device_exclusive_scan(hist, hist_n, scan_scr, st));
      k_radix_scatter<<<(unsigned)n_tiles, kRsThreads, 0, st>>>(kin, vin, kout, vout, M, shift, (int)n_tiles,
                                                                hist);
      FEA_TRY(hipGetLastError());
      std::swap(kin, kout);
      std::swap(vin, vout);
    }
  }
  // pair runs
  FEA_TRY(s.alloc(&flag, M));
  FEA_TRY(s.alloc(&pid, M));
  FEA_TRY(s.alloc(&pair_key, M));
  FEA_TRY(s.alloc(&seg_start, M));
  npairs = err + 1;
  int h_np = 0;
  if (M > 0) {
    k_head_flags<<<g256, 256, 0, st>>>(kin, M, flag);
    FEA_TRY(hipGetLastError());
    FEA_TRY(device_exclusive_scan(flag, M, scan_scr, st));
    k_heads<<<g256, 256, 0, st>>>(kin, flag, M, pair_key, seg_start, pid, npairs);
    FEA_TRY(hipGetLastError());
    FEA_TRY(hipMemcpyAsync(&h_np, npairs, sizeof(int), hipMemcpyDeviceToHost, st));
    FEA_TRY(hipStreamSynchronize(st));
  }
  const int64_t P = h_np;
  std::vector<uint32_t> h_key(P);
  std::vector<int32_t> h_start(P);
  if (P > 0) {
    FEA_TRY(hipMemcpyAsync(h_key.data(), pair_key, P * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    FEA_TRY(hipMemcpyAsync(h_start.data(), seg_start, P * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FEA_TRY(hipStreamSynchronize(st));
  }
  c->P = P;
  c->pair_i.resize(P);
  c->pair_j.resize(P);
  c->seg_off.resize(P + 1);
  c->phys_off.resize(P);
  c->cur_len.resize(P);
  std::vector<int32_t> h_phys(P);
  int64_t off = 0;
  for (int64_t k = 0; k < P; ++k) {
    c->pair_i[k] = (int32_t)(h_key[k] / (uint32_t)N);
    c->pair_j[k] = (int32_t)(h_key[k] % (uint32_t)N);
    c->seg_off[k] = h_start[k];
    const int64_t len = ((k + 1 < P) ? (int64_t)h_start[k + 1] : M) - h_start[k];
    c->cur_len[k] = len;
    c->phys_off[k] = off;
    h_phys[k] = (int32_t)off;
    off += (len + kAlign - 1) / kAlign * kAlign;
  }
  c->seg_off[P] = M;
  c->layout_len = off;
  c->cur = 0;
  // the full device layout (buffer 0; the filtered rounds use buffers 1, 2)
  const size_t cap = (size_t)std::max<int64_t>(off, 1);
  for (int a = 0; a < 4; ++a) FEA_TRY(alloc_dbuf(c->lay[0][a], cap * sizeof(float)));
  FEA_TRY(alloc_dbuf(c->lpos[0], cap * sizeof(int32_t)));
  FEA_TRY(alloc_dbuf(c->perm, std::max<int64_t>(M, 1) * sizeof(int32_t)));
  FEA_TRY(alloc_dbuf(c->swp, std::max<int64_t>(M, 1)));
  for (int a = 0; a < 4; ++a) FEA_TRY(hipMemsetAsync(c->lay[0][a].p, 0, cap * sizeof(float), st));
  FEA_TRY(hipMemsetAsync(c->lpos[0].p, 0xFF, cap * sizeof(int32_t), st));
  if (M > 0) {
    FEA_TRY(s.alloc(&phys32, P));
    FEA_TRY(hipMemcpyAsync(phys32, h_phys.data(), P * sizeof(int32_t), hipMemcpyHostToDevice, st));
    k_gather<<<g256, 256, 0, st>>>(M, vin, pid, seg_start, phys32, x1, y1, x2, y2, cam1, cam2,
                                   c->lay[0][0].as<float>(), c->lay[0][1].as<float>(), c->lay[0][2].as<float>(),
                                   c->lay[0][3].as<float>(), c->lpos[0].as<int32_t>(), c->perm.as<int32_t>(),
                                   c->swp.as<uint8_t>());
    FEA_TRY(hipGetLastError());
  }
  FEA_TRY(hipStreamSynchronize(st));
  return hipSuccess;
}

}  // namespace fea
