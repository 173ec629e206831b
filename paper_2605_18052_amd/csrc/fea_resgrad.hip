// The per-match pass of FastMap's epipolar adjustment (Method > Epipolar
// Adjustment, the IRLS-reweighted objective) and the round-start outlier
// filter, for gfx950.
//
// k_resgrad: one workgroup per work item (<= 4096 matches of one camera pair,
// contiguous in the pair-sorted SoA layout).  Every thread issues all of its
// 16-byte loads first; meanwhile wave 0 builds the pair's pose block in fp64
// (F at the current poses and F_hat at the round snapshot, with the principal
// points folded in) and stages it in LDS, from where every wave moves it to
// scalar registers.  Per match: eps = q2^T F q1 and eps_hat in fp64 (the
// residual of an inlier is ~1e-3 of its terms, so fp32 would lose ~4
// digits), weight c = 1/(Z max(|eps_hat|, delta)), then the contribution
// 2 c eps p2 p1^T to dL/dF and c eps^2 to L accumulate per lane in fp32.
// The 10 sums are reduced across each wave with DPP, across the 4 waves in
// LDS, and written as one fp64 partial per item -- no atomics, so the result
// is deterministic.
#include <hip/hip_runtime.h>

#include "fea_ctx.h"
#include "fea_device.h"

namespace fea {
namespace {

__device__ __forceinline__ float v4(const float4& q, int e) {
  return e == 0 ? q.x : (e == 1 ? q.y : (e == 2 ? q.z : q.w));
}

// Pose block of pair n at (R, T, Fc) folded for raw pixel coordinates;
// zero if the centres coincide (that pair then contributes nothing).
__device__ __forceinline__ void pose_block(int i, int j, const double* __restrict__ R,
                                           const double* __restrict__ T, const double* __restrict__ Fc,
                                           const double* __restrict__ cx, const double* __restrict__ cy,
                                           double Fp[9]) {
  Geo g;
  if (pair_geo(R + 9 * i, T + 3 * i, Fc[i], R + 9 * j, T + 3 * j, Fc[j], g)) {
    fold_principal_point(g.F, cx[i], cy[i], cx[j], cy[j], Fp);
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) Fp[k] = 0.0;
  }
}

__device__ __forceinline__ double eval_eps(const double* F, double x1, double y1, double x2, double y2) {
  const double l0 = fma(F[0], x1, fma(F[1], y1, F[2]));
  const double l1 = fma(F[3], x1, fma(F[4], y1, F[5]));
  const double l2 = fma(F[6], x1, fma(F[7], y1, F[8]));
  return fma(x2, l0, fma(y2, l1, l2));
}

template <int THREADS, int STEPS, bool LOSS_ONLY>
__global__ __launch_bounds__(THREADS) void k_resgrad(
    const float4* __restrict__ X1, const float4* __restrict__ Y1, const float4* __restrict__ X2,
    const float4* __restrict__ Y2, const int32_t* __restrict__ item_pair, const int32_t* __restrict__ item_start,
    const int32_t* __restrict__ item_count, const int32_t* __restrict__ pair_i, const int32_t* __restrict__ pair_j,
    const double* __restrict__ R, const double* __restrict__ T, const double* __restrict__ Fc,
    const double* __restrict__ Rh, const double* __restrict__ Th, const double* __restrict__ Fh,
    const double* __restrict__ cx, const double* __restrict__ cy, const int32_t* __restrict__ pair_scene,
    const float* __restrict__ inv_z_scene, float delta, double* __restrict__ part) {
  __shared__ double s_blk[23];
  __shared__ float s_red[THREADS / kWave][kPartStride];
  const int tid = threadIdx.x;
  const int item = blockIdx.x;
  const int n = item_pair[item];
  const int v0 = item_start[item] >> 2;
  const int cnt = item_count[item];
  const int nvec = (cnt + kVec - 1) / kVec;

  float4 qa[STEPS], qb[STEPS], qc[STEPS], qd[STEPS];
#pragma unroll
  for (int s = 0; s < STEPS; ++s) {
    const int v = s * THREADS + tid;
    if (v < nvec) {
      qa[s] = X1[v0 + v];
      qb[s] = Y1[v0 + v];
      qc[s] = X2[v0 + v];
      qd[s] = Y2[v0 + v];
    } else {
      qa[s] = qb[s] = qc[s] = qd[s] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  if (tid < kWave) {
    const int i = pair_i[n], j = pair_j[n];
    double F[9], Fhat[9];
    pose_block(i, j, R, T, Fc, cx, cy, F);
    pose_block(i, j, Rh, Th, Fh, cx, cy, Fhat);
    if (tid == 0) {
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        s_blk[k] = F[k];
        s_blk[9 + k] = Fhat[k];
      }
      s_blk[18] = cx[i];
      s_blk[19] = cy[i];
      s_blk[20] = cx[j];
      s_blk[21] = cy[j];
      s_blk[22] = inv_z_scene[pair_scene[n]];
    }
  }
  __syncthreads();
  double F[9], Fhat[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    F[k] = readfirstlane_f64(s_blk[k]);
    Fhat[k] = readfirstlane_f64(s_blk[9 + k]);
  }
  const float cxi = (float)readfirstlane_f64(s_blk[18]);
  const float cyi = (float)readfirstlane_f64(s_blk[19]);
  const float cxj = (float)readfirstlane_f64(s_blk[20]);
  const float cyj = (float)readfirstlane_f64(s_blk[21]);
  const float inv_z = (float)readfirstlane_f64(s_blk[22]);

  float acc[kPartStride];
#pragma unroll
  for (int k = 0; k < kPartStride; ++k) acc[k] = 0.f;
#pragma unroll
  for (int s = 0; s < STEPS; ++s) {
#pragma unroll
    for (int e = 0; e < kVec; ++e) {
      const int local = (s * THREADS + tid) * kVec + e;
      const float x1 = v4(qa[s], e), y1 = v4(qb[s], e), x2 = v4(qc[s], e), y2 = v4(qd[s], e);
      const double eps = eval_eps(F, x1, y1, x2, y2);
      const double eph = eval_eps(Fhat, x1, y1, x2, y2);
      const float ef = (float)eps;
      const float w = fmaxf(fabsf((float)eph), delta);
      const float c = (local < cnt) ? inv_z * __builtin_amdgcn_rcpf(w) : 0.f;
      if (!LOSS_ONLY) {
        const float k2 = 2.f * c * ef;
        const float x1c = x1 - cxi, y1c = y1 - cyi, x2c = x2 - cxj, y2c = y2 - cyj;
        const float kx = k2 * x2c, ky = k2 * y2c;
        acc[0] = fmaf(kx, x1c, acc[0]);
        acc[1] = fmaf(kx, y1c, acc[1]);
        acc[2] += kx;
        acc[3] = fmaf(ky, x1c, acc[3]);
        acc[4] = fmaf(ky, y1c, acc[4]);
        acc[5] += ky;
        acc[6] = fmaf(k2, x1c, acc[6]);
        acc[7] = fmaf(k2, y1c, acc[7]);
        acc[8] += k2;
      }
      acc[9] = fmaf(c * ef, ef, acc[9]);
    }
  }
  const int wid = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int k = 0; k < kPartStride; ++k) {
    const float w = wave_sum_f32(acc[k]);
    if (lane == 0) s_red[wid][k] = w;
  }
  __syncthreads();
  if (tid < kPartStride) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < THREADS / kWave; ++w) sum += (double)s_red[w][tid];
    part[(int64_t)item * kPartStride + tid] = sum;
  }
}

// Round start, pass 1: how many matches of each item survive the filter
// |eps_hat| < tau (strict; Method > Epipolar Adjustment, outlier filtering).
__global__ __launch_bounds__(kFilterThreads) void k_filter_count(
    const float4* __restrict__ X1, const float4* __restrict__ Y1, const float4* __restrict__ X2,
    const float4* __restrict__ Y2, const int32_t* __restrict__ item_pair, const int32_t* __restrict__ item_start,
    const int32_t* __restrict__ item_count, const int32_t* __restrict__ pair_i, const int32_t* __restrict__ pair_j,
    const double* __restrict__ Rh, const double* __restrict__ Th, const double* __restrict__ Fh,
    const double* __restrict__ cx, const double* __restrict__ cy, const int32_t* __restrict__ pair_scene,
    const double* __restrict__ tau_scene, int32_t* __restrict__ keep) {
  __shared__ double s_blk[10];
  __shared__ int s_cnt;
  const int tid = threadIdx.x, item = blockIdx.x;
  const int n = item_pair[item];
  const int v0 = item_start[item] >> 2;
  const int cnt = item_count[item];
  const int nvec = (cnt + kVec - 1) / kVec;
  if (tid == 0) {
    double Fhat[9];
    pose_block(pair_i[n], pair_j[n], Rh, Th, Fh, cx, cy, Fhat);
#pragma unroll
    for (int k = 0; k < 9; ++k) s_blk[k] = Fhat[k];
    s_blk[9] = tau_scene[pair_scene[n]];
    s_cnt = 0;
  }
  __syncthreads();
  double Fhat[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Fhat[k] = s_blk[k];
  const double tau = s_blk[9];
  int kept = 0;
  for (int v = tid; v < nvec; v += kFilterThreads) {
    const float4 a = X1[v0 + v], b = Y1[v0 + v], c = X2[v0 + v], d = Y2[v0 + v];
#pragma unroll
    for (int e = 0; e < kVec; ++e) {
      const double eph = eval_eps(Fhat, v4(a, e), v4(b, e), v4(c, e), v4(d, e));
      kept += (v * kVec + e < cnt) && (fabs(eph) < tau);
    }
  }
  atomicAdd(&s_cnt, kept);
  __syncthreads();
  if (tid == 0) keep[item] = s_cnt;
}

// Round start, pass 2: stable compaction of the surviving matches into the
// other layout buffer.  base[item] is where the item's first survivor goes.
__global__ __launch_bounds__(kFilterThreads) void k_filter_scatter(
    const float4* __restrict__ X1, const float4* __restrict__ Y1, const float4* __restrict__ X2,
    const float4* __restrict__ Y2, const int4* __restrict__ POS, const int32_t* __restrict__ item_pair,
    const int32_t* __restrict__ item_start, const int32_t* __restrict__ item_count,
    const int32_t* __restrict__ pair_i, const int32_t* __restrict__ pair_j, const double* __restrict__ Rh,
    const double* __restrict__ Th, const double* __restrict__ Fh, const double* __restrict__ cx,
    const double* __restrict__ cy, const int32_t* __restrict__ pair_scene, const double* __restrict__ tau_scene,
    const int32_t* __restrict__ base, float* __restrict__ ox1,
    float* __restrict__ oy1, float* __restrict__ ox2, float* __restrict__ oy2, int32_t* __restrict__ opos) {
  __shared__ double s_blk[10];
  __shared__ int s_w[kFilterThreads / kWave];
  const int tid = threadIdx.x, item = blockIdx.x;
  const int n = item_pair[item];
  const int v0 = item_start[item] >> 2;
  const int cnt = item_count[item];
  const int nvec = (cnt + kVec - 1) / kVec;
  if (tid == 0) {
    double Fhat[9];
    pose_block(pair_i[n], pair_j[n], Rh, Th, Fh, cx, cy, Fhat);
#pragma unroll
    for (int k = 0; k < 9; ++k) s_blk[k] = Fhat[k];
    s_blk[9] = tau_scene[pair_scene[n]];
  }
  __syncthreads();
  double Fhat[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Fhat[k] = s_blk[k];
  const double tau = s_blk[9];
  int run = base[item];
  const int lane = tid & 63, wid = tid >> 6;
  const int rounds = (nvec + kFilterThreads - 1) / kFilterThreads;
  for (int r = 0; r < rounds; ++r) {
    const int v = r * kFilterThreads + tid;
    float4 a = make_float4(0, 0, 0, 0), b = a, c = a, d = a;
    int4 p = make_int4(-1, -1, -1, -1);
    if (v < nvec) {
      a = X1[v0 + v];
      b = Y1[v0 + v];
      c = X2[v0 + v];
      d = Y2[v0 + v];
      p = POS[v0 + v];
    }
    int flags = 0, mine = 0;
#pragma unroll
    for (int e = 0; e < kVec; ++e) {
      const double eph = eval_eps(Fhat, v4(a, e), v4(b, e), v4(c, e), v4(d, e));
      const int k = (v < nvec) && (v * kVec + e < cnt) && (fabs(eph) < tau);
      flags |= k << e;
      mine += k;
    }
    // exclusive scan of `mine` over the block, in thread order
    const int inc = wave_inclusive_scan(mine);
    if (lane == 63) s_w[wid] = inc;
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kFilterThreads / kWave; ++w) {
      before += (w < wid) ? s_w[w] : 0;
      total += s_w[w];
    }
    __syncthreads();
    int dst = run + before + inc - mine;
    const int pe[4] = {p.x, p.y, p.z, p.w};
#pragma unroll
    for (int e = 0; e < kVec; ++e) {
      if (flags & (1 << e)) {
        ox1[dst] = v4(a, e);
        oy1[dst] = v4(b, e);
        ox2[dst] = v4(c, e);
        oy2[dst] = v4(d, e);
        opos[dst] = pe[e];
        ++dst;
      }
    }
    run += total;
  }
}

}  // namespace

template <int THREADS, int STEPS, bool LOSS_ONLY>
hipError_t launch_resgrad_t(fea_ctx* c, const double* R, const double* T, const double* F) {
  const int b = c->cur;
  k_resgrad<THREADS, STEPS, LOSS_ONLY><<<(unsigned)c->n_items, THREADS, 0, c->stream>>>(
      c->lay[b][0].as<float4>(), c->lay[b][1].as<float4>(), c->lay[b][2].as<float4>(), c->lay[b][3].as<float4>(),
      c->item_pair.as<int32_t>(), c->item_start.as<int32_t>(), c->item_count.as<int32_t>(),
      c->d_pair_i.as<int32_t>(), c->d_pair_j.as<int32_t>(), R, T, F, c->Rh.as<double>(), c->Th.as<double>(),
      c->Fh.as<double>(), c->d_cx.as<double>(), c->d_cy.as<double>(), c->d_pair_scene.as<int32_t>(),
      c->d_inv_z.as<float>(), (float)c->opt.delta, c->part.as<double>());
  return hipGetLastError();
}

template <bool LOSS_ONLY>
hipError_t launch_resgrad_sel(fea_ctx* c, int cfg, const double* R, const double* T, const double* F) {
  switch (cfg) {
    case 0: return launch_resgrad_t<256, 4, LOSS_ONLY>(c, R, T, F);
    case 1: return launch_resgrad_t<256, 2, LOSS_ONLY>(c, R, T, F);
    case 2: return launch_resgrad_t<256, 1, LOSS_ONLY>(c, R, T, F);
    case 3: return launch_resgrad_t<128, 8, LOSS_ONLY>(c, R, T, F);
    case 4: return launch_resgrad_t<128, 4, LOSS_ONLY>(c, R, T, F);
    case 5: return launch_resgrad_t<128, 2, LOSS_ONLY>(c, R, T, F);
    case 6: return launch_resgrad_t<512, 2, LOSS_ONLY>(c, R, T, F);
    case 7: return launch_resgrad_t<512, 4, LOSS_ONLY>(c, R, T, F);
  }
  return hipErrorInvalidValue;
}

// Per-match kernel with tile shape `cfg` over the current items at poses
// (R, T, F) (per camera, fp64), weights from the round snapshot.
hipError_t launch_resgrad_at(fea_ctx* c, int cfg, const double* R, const double* T, const double* F,
                             bool loss_only) {
  if (c->n_items == 0) return hipSuccess;
  return loss_only ? launch_resgrad_sel<true>(c, cfg, R, T, F) : launch_resgrad_sel<false>(c, cfg, R, T, F);
}

hipError_t launch_resgrad_cfg(fea_ctx* c, int cfg) {
  return launch_resgrad_at(c, cfg, c->R[c->pcur].as<double>(), c->T[c->pcur].as<double>(),
                           c->Fc[c->pcur].as<double>(), false);
}

hipError_t launch_resgrad(fea_ctx* c) {
  if (c->n_items == 0) return hipSuccess;
  hipEvent_t ev1 = nullptr;
  if (c->timing) {
    while (c->ev_pool.size() < c->ev_used + 2) {
      hipEvent_t e;
      hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) return err;
      c->ev_pool.push_back(e);
    }
    hipError_t err = hipEventRecord(c->ev_pool[c->ev_used], c->stream);
    if (err != hipSuccess) return err;
    ev1 = c->ev_pool[c->ev_used + 1];
    c->ev_used += 2;
  }
  hipError_t err = launch_resgrad_cfg(c, c->tile_cfg);
  if (err == hipSuccess && ev1) err = hipEventRecord(ev1, c->stream);
  return err;
}

hipError_t launch_filter_count(fea_ctx* c) {
  if (c->n_items == 0) return hipSuccess;
  const int b = c->cur;
  k_filter_count<<<(unsigned)c->n_items, kFilterThreads, 0, c->stream>>>(
      c->lay[b][0].as<float4>(), c->lay[b][1].as<float4>(), c->lay[b][2].as<float4>(), c->lay[b][3].as<float4>(),
      c->item_pair.as<int32_t>(), c->item_start.as<int32_t>(), c->item_count.as<int32_t>(),
      c->d_pair_i.as<int32_t>(), c->d_pair_j.as<int32_t>(), c->Rh.as<double>(), c->Th.as<double>(),
      c->Fh.as<double>(), c->d_cx.as<double>(), c->d_cy.as<double>(), c->d_pair_scene.as<int32_t>(),
      c->d_tau.as<double>(), c->item_keep.as<int32_t>());
  return hipGetLastError();
}

hipError_t launch_filter_scatter(fea_ctx* c, int dst) {
  if (c->n_items == 0) return hipSuccess;
  const int b = c->cur;
  k_filter_scatter<<<(unsigned)c->n_items, kFilterThreads, 0, c->stream>>>(
      c->lay[b][0].as<float4>(), c->lay[b][1].as<float4>(), c->lay[b][2].as<float4>(), c->lay[b][3].as<float4>(),
      c->lpos[b].as<int4>(), c->item_pair.as<int32_t>(), c->item_start.as<int32_t>(),
      c->item_count.as<int32_t>(), c->d_pair_i.as<int32_t>(), c->d_pair_j.as<int32_t>(), c->Rh.as<double>(),
      c->Th.as<double>(), c->Fh.as<double>(), c->d_cx.as<double>(), c->d_cy.as<double>(),
      c->d_pair_scene.as<int32_t>(), c->d_tau.as<double>(), c->item_base.as<int32_t>(), c->lay[dst][0].as<float>(), c->lay[dst][1].as<float>(),
      c->lay[dst][2].as<float>(), c->lay[dst][3].as<float>(), c->lpos[dst].as<int32_t>());
  return hipGetLastError();
}

}  // namespace fea
