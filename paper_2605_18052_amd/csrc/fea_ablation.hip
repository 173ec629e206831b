// Ablations of the per-match pass: the same residual, IRLS weight and dL/dF
// accumulation at the current poses with one design choice of the library's
// kernel taken back, timed with HIP events so that each choice can be priced
// against the HBM peak on the same data.
//
//   1  pose block built inside every workgroup (wave 0, fp64) and staged in
//      LDS before any wave may start, instead of the per-pair pose table;
//   2  sorted layout, but every match adds its 10 contributions to the
//      pair's sums with global atomics, instead of per-lane sums, a DPP wave
//      reduction and one partial per work item;
//   3  matches in the caller's (unsorted) order: each carries its pair id,
//      gathers the pair's matrices from the pose table and adds with atomics.
//
// Variant 0 is the library's own kernel.  Variants write per-pair sums
// (fp32, atomics: order not fixed); they exist for measurement only.
#include <hip/hip_runtime.h>

#include <vector>

#include "fea_ctx.h"
#include "fea_device.h"

namespace fea {
namespace {

constexpr int kAblThreads = 256;
constexpr int kAblSteps = 2;  // 16-byte loads per thread per array (2048-match items)

__device__ __forceinline__ float v4a(const float4& q, int e) {
  return e == 0 ? q.x : (e == 1 ? q.y : (e == 2 ? q.z : q.w));
}

__device__ __forceinline__ double eps_of(const double* F, double x1, double y1, double x2, double y2) {
  const double l0 = fma(F[0], x1, fma(F[1], y1, F[2]));
  const double l1 = fma(F[3], x1, fma(F[4], y1, F[5]));
  const double l2 = fma(F[6], x1, fma(F[7], y1, F[8]));
  return fma(x2, l0, fma(y2, l1, l2));
}

// The 10 contributions of one match (2 c eps p2 p1^T and c eps^2).
__device__ __forceinline__ void contrib(const double* F, const double* Fh, float inv_z, float delta, float x1,
                                        float y1, float x2, float y2, float cxi, float cyi, float cxj, float cyj,
                                        float out[kPartStride]) {
  const double eps = eps_of(F, x1, y1, x2, y2);
  const double eph = eps_of(Fh, x1, y1, x2, y2);
  const float ef = (float)eps;
  const float c = inv_z * __builtin_amdgcn_rcpf(fmaxf(fabsf((float)eph), delta));
  const float k2 = 2.f * c * ef;
  const float x1c = x1 - cxi, y1c = y1 - cyi, x2c = x2 - cxj, y2c = y2 - cyj;
  const float kx = k2 * x2c, ky = k2 * y2c;
  out[0] = kx * x1c;
  out[1] = kx * y1c;
  out[2] = kx;
  out[3] = ky * x1c;
  out[4] = ky * y1c;
  out[5] = ky;
  out[6] = k2 * x1c;
  out[7] = k2 * y1c;
  out[8] = k2;
  out[9] = c * ef * ef;
}

// Variant 1: the pose block of the item's pair built by wave 0 from the
// camera parameters and staged through LDS; otherwise the library kernel.
__global__ __launch_bounds__(kAblThreads) void k_abl_lds_pose(
    const float4* __restrict__ X1, const float4* __restrict__ Y1, const float4* __restrict__ X2,
    const float4* __restrict__ Y2, const int4* __restrict__ items, const int32_t* __restrict__ pair_i,
    const int32_t* __restrict__ pair_j, const double* __restrict__ R, const double* __restrict__ T,
    const double* __restrict__ Fc, const double* __restrict__ Rh, const double* __restrict__ Th,
    const double* __restrict__ Fh, const double* __restrict__ cx, const double* __restrict__ cy,
    const double* __restrict__ ptab, float delta, float* __restrict__ pair_sum) {
  __shared__ double s_blk[23];
  __shared__ float s_red[kAblThreads / kWave][kPartStride];
  const int tid = threadIdx.x;
  const int4 rec = items[blockIdx.x];
  const int n = rec.x, v0 = rec.y >> 2, cnt = rec.z;
  const int nvec = (cnt + kVec - 1) / kVec;
  float4 qa[kAblSteps], qb[kAblSteps], qc[kAblSteps], qd[kAblSteps];
#pragma unroll
  for (int s = 0; s < kAblSteps; ++s) {
    const int v = s * kAblThreads + tid;
    const bool in = v < nvec;
    qa[s] = in ? X1[v0 + v] : make_float4(0.f, 0.f, 0.f, 0.f);
    qb[s] = in ? Y1[v0 + v] : make_float4(0.f, 0.f, 0.f, 0.f);
    qc[s] = in ? X2[v0 + v] : make_float4(0.f, 0.f, 0.f, 0.f);
    qd[s] = in ? Y2[v0 + v] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  if (tid < kWave) {
    const int i = pair_i[n], j = pair_j[n];
    double F[9], G[9];
    Geo g;
    if (pair_geo(R + 9 * i, T + 3 * i, Fc[i], R + 9 * j, T + 3 * j, Fc[j], g))
      fold_principal_point(g.F, cx[i], cy[i], cx[j], cy[j], F);
    else
      for (int k = 0; k < 9; ++k) F[k] = 0.0;
    if (pair_geo(Rh + 9 * i, Th + 3 * i, Fh[i], Rh + 9 * j, Th + 3 * j, Fh[j], g))
      fold_principal_point(g.F, cx[i], cy[i], cx[j], cy[j], G);
    else
      for (int k = 0; k < 9; ++k) G[k] = 0.0;
    if (tid == 0) {
      for (int k = 0; k < 9; ++k) {
        s_blk[k] = F[k];
        s_blk[9 + k] = G[k];
      }
      s_blk[18] = cx[i];
      s_blk[19] = cy[i];
      s_blk[20] = cx[j];
      s_blk[21] = cy[j];
      s_blk[22] = ptab[(int64_t)n * kPairRow + kRowInvZ];
    }
  }
  __syncthreads();
  double F[9], Fhat[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    F[k] = readfirstlane_f64(s_blk[k]);
    Fhat[k] = readfirstlane_f64(s_blk[9 + k]);
  }
  const float cxi = (float)s_blk[18], cyi = (float)s_blk[19], cxj = (float)s_blk[20], cyj = (float)s_blk[21];
  const float inv_z = (float)s_blk[22];
  float acc[kPartStride];
#pragma unroll
  for (int k = 0; k < kPartStride; ++k) acc[k] = 0.f;
#pragma unroll
  for (int s = 0; s < kAblSteps; ++s)
#pragma unroll
    for (int e = 0; e < kVec; ++e) {
      if ((s * kAblThreads + tid) * kVec + e >= cnt) continue;
      float o[kPartStride];
      contrib(F, Fhat, inv_z, delta, v4a(qa[s], e), v4a(qb[s], e), v4a(qc[s], e), v4a(qd[s], e), cxi, cyi, cxj,
              cyj, o);
#pragma unroll
      for (int k = 0; k < kPartStride; ++k) acc[k] += o[k];
    }
  const int wid = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int k = 0; k < kPartStride; ++k) {
    const float w = wave_sum_f32(acc[k]);
    if (lane == 0) s_red[wid][k] = w;
  }
  __syncthreads();
  if (tid < kPartStride) {
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < kAblThreads / kWave; ++w) sum += s_red[w][tid];
    atomicAdd(&pair_sum[(int64_t)n * kPartStride + tid], sum);
  }
}

// Variant 2: sorted layout and pose table, but per-match global atomics.
__global__ __launch_bounds__(kAblThreads) void k_abl_atomics(
    const float4* __restrict__ X1, const float4* __restrict__ Y1, const float4* __restrict__ X2,
    const float4* __restrict__ Y2, const int4* __restrict__ items, const double* __restrict__ ptab, float delta,
    float* __restrict__ pair_sum) {
  const int tid = threadIdx.x;
  const int4 rec = items[blockIdx.x];
  const int n = rec.x, v0 = rec.y >> 2, cnt = rec.z;
  const int nvec = (cnt + kVec - 1) / kVec;
  const double* row = ptab + (int64_t)n * kPairRow;
  double F[9], Fhat[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    F[k] = row[kRowF + k];
    Fhat[k] = row[kRowFh + k];
  }
  const float cxi = (float)row[kRowCx], cyi = (float)row[kRowCx + 1];
  const float cxj = (float)row[kRowCx + 2], cyj = (float)row[kRowCx + 3];
  const float inv_z = (float)row[kRowInvZ];
  float* dst = pair_sum + (int64_t)n * kPartStride;
  for (int v = tid; v < nvec; v += kAblThreads) {
    const float4 a = X1[v0 + v], b = Y1[v0 + v], c = X2[v0 + v], d = Y2[v0 + v];
#pragma unroll
    for (int e = 0; e < kVec; ++e) {
      if (v * kVec + e >= cnt) continue;
      float o[kPartStride];
      contrib(F, Fhat, inv_z, delta, v4a(a, e), v4a(b, e), v4a(c, e), v4a(d, e), cxi, cyi, cxj, cyj, o);
#pragma unroll
      for (int k = 0; k < kPartStride; ++k) atomicAdd(&dst[k], o[k]);
    }
  }
}

// Variant 3: matches in the caller's order, one per thread, each with its
// pair id; matrices gathered from the pose table; per-match atomics.
__global__ __launch_bounds__(kAblThreads) void k_abl_unsorted(int64_t M, const float* __restrict__ ux1,
                                                              const float* __restrict__ uy1,
                                                              const float* __restrict__ ux2,
                                                              const float* __restrict__ uy2,
                                                              const int32_t* __restrict__ upair,
                                                              const double* __restrict__ ptab, float delta,
                                                              float* __restrict__ pair_sum) {
  const int64_t m = (int64_t)blockIdx.x * kAblThreads + threadIdx.x;
  if (m >= M) return;
  const int n = upair[m];
  if (n < 0) return;  // dropped by the filter
  const double* row = ptab + (int64_t)n * kPairRow;
  double F[9], Fhat[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    F[k] = row[kRowF + k];
    Fhat[k] = row[kRowFh + k];
  }
  float o[kPartStride];
  contrib(F, Fhat, (float)row[kRowInvZ], delta, ux1[m], uy1[m], ux2[m], uy2[m], (float)row[kRowCx],
          (float)row[kRowCx + 1], (float)row[kRowCx + 2], (float)row[kRowCx + 3], o);
  float* dst = pair_sum + (int64_t)n * kPartStride;
#pragma unroll
  for (int k = 0; k < kPartStride; ++k) atomicAdd(&dst[k], o[k]);
}

// Retained matches of the current layout back in the caller's order (the
// keypoints stay in the pair's orientation); -1 marks a dropped match.
__global__ __launch_bounds__(kAblThreads) void k_abl_unsort(
    const float* __restrict__ X1, const float* __restrict__ Y1, const float* __restrict__ X2,
    const float* __restrict__ Y2, const int32_t* __restrict__ lpos, const int4* __restrict__ items,
    const int32_t* __restrict__ perm, float* __restrict__ ux1, float* __restrict__ uy1, float* __restrict__ ux2,
    float* __restrict__ uy2, int32_t* __restrict__ upair) {
  const int4 rec = items[blockIdx.x];
  for (int k = threadIdx.x; k < rec.z; k += kAblThreads) {
    const int slot = rec.y + k;
    const int pos = lpos[slot];
    if (pos < 0) continue;
    const int m = perm[pos];
    ux1[m] = X1[slot];
    uy1[m] = Y1[slot];
    ux2[m] = X2[slot];
    uy2[m] = Y2[slot];
    upair[m] = rec.x;
  }
}

// Per-pair sums of the library kernel's per-item partials (fp32 for the
// comparison with the atomic variants).
__global__ void k_abl_item_to_pair(int32_t P, const int32_t* __restrict__ pair_item_off,
                                   const double* __restrict__ part, float* __restrict__ pair_sum) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)P * kPartStride) return;
  const int n = (int)(t / kPartStride), k = (int)(t % kPartStride);
  double s = 0.0;
  for (int it = pair_item_off[n]; it < pair_item_off[n + 1]; ++it) s += part[(int64_t)it * kPartStride + k];
  pair_sum[t] = (float)s;
}

}  // namespace

// Runs ablation `variant` `reps` times on the current layout and poses (the
// items must have the 2048-match shape); mean kernel milliseconds into *ms
// and the per-pair sums into pair_sum_dev (device, P * 10 floats).
hipError_t run_ablation(fea_ctx* c, int variant, int reps, double* ms, float* pair_sum_dev) {
  if (c->n_items == 0 || reps < 1) return hipErrorInvalidValue;
  const int b = c->cur;
  const int p = c->pcur;
  hipError_t e = launch_pair_pose(c, c->R[p].as<double>(), c->T[p].as<double>(), c->Fc[p].as<double>(), false);
  if (e != hipSuccess) return e;
  DBuf ux1, uy1, ux2, uy2, upair;
  auto release = [&]() {
    DBuf* all[] = {&ux1, &uy1, &ux2, &uy2, &upair};
    for (DBuf* d : all)
      if (d->p) (void)hipFree(d->p);
  };
  if (variant == 3) {
    const size_t M = (size_t)std::max<int64_t>(c->M, 1);
    DBuf* f[] = {&ux1, &uy1, &ux2, &uy2};
    for (DBuf* d : f)
      if ((e = hipMalloc(&d->p, M * sizeof(float))) != hipSuccess) return release(), e;
    if ((e = hipMalloc(&upair.p, M * sizeof(int32_t))) != hipSuccess) return release(), e;
    if ((e = hipMemsetAsync(upair.p, 0xFF, M * sizeof(int32_t), c->stream)) != hipSuccess) return release(), e;
    k_abl_unsort<<<(unsigned)c->n_items, kAblThreads, 0, c->stream>>>(
        c->lay[b][0].as<float>(), c->lay[b][1].as<float>(), c->lay[b][2].as<float>(), c->lay[b][3].as<float>(),
        c->lpos[b].as<int32_t>(), c->item_rec.as<int4>(), c->perm.as<int32_t>(), ux1.as<float>(), uy1.as<float>(),
        ux2.as<float>(), uy2.as<float>(), upair.as<int32_t>());
    if ((e = hipGetLastError()) != hipSuccess) return release(), e;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return release(), e;
  }
  const float delta = (float)c->opt.delta;
  const size_t sum_bytes = (size_t)c->P * kPartStride * sizeof(float);
  float total = 0.f;
  for (int r = 0; r < reps + 1 && e == hipSuccess; ++r) {
    if (variant != 0 && (e = hipMemsetAsync(pair_sum_dev, 0, sum_bytes, c->stream)) != hipSuccess) break;
    if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) break;
    switch (variant) {
      case 0:
        e = launch_resgrad_kernel(c, c->tile_cfg, false, true);
        break;
      case 1:
        k_abl_lds_pose<<<(unsigned)c->n_items, kAblThreads, 0, c->stream>>>(
            c->lay[b][0].as<float4>(), c->lay[b][1].as<float4>(), c->lay[b][2].as<float4>(),
            c->lay[b][3].as<float4>(), c->item_rec.as<int4>(), c->d_pair_i.as<int32_t>(),
            c->d_pair_j.as<int32_t>(), c->R[p].as<double>(), c->T[p].as<double>(), c->Fc[p].as<double>(),
            c->Rh.as<double>(), c->Th.as<double>(), c->Fh.as<double>(), c->d_cx.as<double>(), c->d_cy.as<double>(),
            c->ptab.as<double>(), delta, pair_sum_dev);
        e = hipGetLastError();
        break;
      case 2:
        k_abl_atomics<<<(unsigned)c->n_items, kAblThreads, 0, c->stream>>>(
            c->lay[b][0].as<float4>(), c->lay[b][1].as<float4>(), c->lay[b][2].as<float4>(),
            c->lay[b][3].as<float4>(), c->item_rec.as<int4>(), c->ptab.as<double>(), delta, pair_sum_dev);
        e = hipGetLastError();
        break;
      case 3:
        k_abl_unsorted<<<(unsigned)((c->M + kAblThreads - 1) / kAblThreads), kAblThreads, 0, c->stream>>>(
            c->M, ux1.as<float>(), uy1.as<float>(), ux2.as<float>(), uy2.as<float>(), upair.as<int32_t>(),
            c->ptab.as<double>(), delta, pair_sum_dev);
        e = hipGetLastError();
        break;
      default:
        e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) break;
    if ((e = hipEventRecord(e1, c->stream)) != hipSuccess) break;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) break;
    if (r > 0) total += t;  // the first launch warms up
  }
  if (e == hipSuccess && variant == 0) {
    const int64_t t = c->P * kPartStride;
    k_abl_item_to_pair<<<(unsigned)((t + 255) / 256), 256, 0, c->stream>>>(
        (int32_t)c->P, c->pair_item_off.as<int32_t>(), c->part.as<double>(), pair_sum_dev);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  release();
  if (e == hipSuccess) *ms = total / reps;
  return e;
}

}  // namespace fea
