// Quadratic-form inner loop of FastMap's epipolar adjustment (Method >
// Epipolar Adjustment: with the IRLS weights frozen for a round, the
// objective of pair n is f^T W_n f, f = vec(F) and W_n the weighted sum of
// the outer products of the matches' 9-vectors), for gfx950.
//
// Once per round, k_quad_build streams the retained matches of each work item
// (the same 16 bytes per match as the per-match kernel) and accumulates, per
// lane in fp64, the 45 distinct entries of sum c w w^T with
// w = vec(p2 p1^T) in centred pixel coordinates and c the round's IRLS weight
// (times the learned weight on learned scenes).  The 45 sums are reduced over
// the wave with DPP and over the waves in LDS into one fp64 partial per item;
// k_quad_reduce adds a pair's item partials in item order into W_n.
//
// Every step, the camera kernel evaluates dL/dF = 2 W_n f and the loss
// f^T W_n f of each incident pair at the current poses, so a step is one
// kernel of O(pairs) work instead of a pass over the matches.  The whole form
// is fp64: the loss is a small difference of large terms (an inlier's
// residual is ~1e-3 of its terms).
#include <hip/hip_runtime.h>

#include "fea_ctx.h"
#include "fea_device.h"

namespace fea {
namespace {

constexpr int kQuad = 45;  // distinct entries of a symmetric 9x9 matrix
constexpr int kQuadThreads = 256;

__device__ __forceinline__ float v4q(const float4& q, int e) {
  return e == 0 ? q.x : (e == 1 ? q.y : (e == 2 ? q.z : q.w));
}

__device__ __forceinline__ unsigned short v4w(const ushort4& q, int e) {
  return e == 0 ? q.x : (e == 1 ? q.y : (e == 2 ? q.z : q.w));
}

template <bool WEIGHTED>
__global__ __launch_bounds__(kQuadThreads) void k_quad_build(
    const float4* __restrict__ X1, const float4* __restrict__ Y1, const float4* __restrict__ X2,
    const float4* __restrict__ Y2, const int4* __restrict__ items, const double* __restrict__ ptab,
    const ushort4* __restrict__ Wl, double delta, double* __restrict__ qpart) {
  __shared__ double s_red[kQuadThreads / kWave][kQuad];
  const int tid = threadIdx.x, item = blockIdx.x;
  const int4 rec = items[item];
  const int n = rec.x;
  const int v0 = rec.y >> 2;
  const int cnt = rec.z;
  const int nvec = (cnt + kVec - 1) / kVec;
  const double* row = ptab + (int64_t)n * kPairRow;
  double Fh[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Fh[k] = row[kRowFh + k];
  const double cxi = row[kRowCx + 0], cyi = row[kRowCx + 1];
  const double cxj = row[kRowCx + 2], cyj = row[kRowCx + 3];
  const bool learned = WEIGHTED && row[kRowMode] != 0.0;
  const double inv_z = learned ? row[kRowInvZw] : row[kRowInvZ];

  double acc[kQuad];
#pragma unroll
  for (int k = 0; k < kQuad; ++k) acc[k] = 0.0;
  for (int v = tid; v < nvec; v += kQuadThreads) {
    const float4 a = X1[v0 + v], b = Y1[v0 + v], c = X2[v0 + v], d = Y2[v0 + v];
    ushort4 wq = make_ushort4(0, 0, 0, 0);
    if (WEIGHTED) wq = Wl[v0 + v];
#pragma unroll
    for (int e = 0; e < kVec; ++e) {
      if (v * kVec + e >= cnt) continue;
      const double x1 = v4q(a, e), y1 = v4q(b, e), x2 = v4q(c, e), y2 = v4q(d, e);
      // IRLS weight from the snapshot residual (raw pixel coordinates)
      const double l0 = fma(Fh[0], x1, fma(Fh[1], y1, Fh[2]));
      const double l1 = fma(Fh[3], x1, fma(Fh[4], y1, Fh[5]));
      const double l2 = fma(Fh[6], x1, fma(Fh[7], y1, Fh[8]));
      const double eph = fma(x2, l0, fma(y2, l1, l2));
      double cw = inv_z / fmax(fabs(eph), delta);
      if (learned) cw *= (double)__uint_as_float((uint32_t)v4w(wq, e) << 16);
      const double p1[3] = {x1 - cxi, y1 - cyi, 1.0};
      const double p2[3] = {x2 - cxj, y2 - cyj, 1.0};
      double w[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int s = 0; s < 3; ++s) w[3 * r + s] = p2[r] * p1[s];
      int k = 0;
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        const double cr = cw * w[r];
#pragma unroll
        for (int s = r; s < 9; ++s, ++k) acc[k] = fma(cr, w[s], acc[k]);
      }
    }
  }
  wave_sum_f64_multi<kQuad>(acc);
  const int wid = tid >> 6, lane = tid & 63;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < kQuad; ++k) s_red[wid][k] = acc[k];
  __syncthreads();
  if (tid < kQuad) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kQuadThreads / kWave; ++w) s += s_red[w][tid];
    qpart[(int64_t)item * kQuad + tid] = s;
  }
}

// W_n = sum of the pair's item partials, in item order.
__global__ __launch_bounds__(kQuadThreads) void k_quad_reduce(int32_t P, const int32_t* __restrict__ pair_item_off,
                                                              const double* __restrict__ qpart,
                                                              double* __restrict__ qW) {
  const int64_t t = (int64_t)blockIdx.x * kQuadThreads + threadIdx.x;
  if (t >= (int64_t)P * kQuad) return;
  const int n = (int)(t / kQuad), k = (int)(t % kQuad);
  double s = 0.0;
  for (int it = pair_item_off[n]; it < pair_item_off[n + 1]; ++it) s += qpart[(int64_t)it * kQuad + k];
  qW[t] = s;
}

}  // namespace

// Builds W_n for every pair from the current layout, the round snapshot's
// weights and, on learned scenes, the learned weights.  The pose table's
// per-scene normalisers (1/Z, 1/sum of learned weights) are refreshed first:
// they are set after the round's compaction and inference.
hipError_t launch_quad_build(fea_ctx* c) {
  if (c->P == 0) return hipSuccess;
  hipError_t e = launch_pair_pose(c, c->R[c->pcur].as<double>(), c->T[c->pcur].as<double>(),
                                  c->Fc[c->pcur].as<double>(), false);
  if (e != hipSuccess) return e;
  if (c->n_items > 0) {
    const int b = c->cur;
#define FEA_QUAD_BUILD_ARGS                                                                                 \
  c->lay[b][0].as<float4>(), c->lay[b][1].as<float4>(), c->lay[b][2].as<float4>(), c->lay[b][3].as<float4>(), \
      c->item_rec.as<int4>(), c->ptab.as<double>(), c->wlay.as<ushort4>(), c->opt.delta, c->qpart.as<double>()
    if (c->learned_any)
      k_quad_build<true><<<(unsigned)c->n_items, kQuadThreads, 0, c->stream>>>(FEA_QUAD_BUILD_ARGS);
    else
      k_quad_build<false><<<(unsigned)c->n_items, kQuadThreads, 0, c->stream>>>(FEA_QUAD_BUILD_ARGS);
#undef FEA_QUAD_BUILD_ARGS
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int64_t t = c->P * kQuad;
  k_quad_reduce<<<(unsigned)((t + kQuadThreads - 1) / kQuadThreads), kQuadThreads, 0, c->stream>>>(
      (int32_t)c->P, c->pair_item_off.as<int32_t>(), c->qpart.as<double>(), c->qW.as<double>());
  return hipGetLastError();
}

}  // namespace fea
