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

// One item of the round's pass: the threshold test at the snapshot
// (|eps_hat| < tau, strict) of the matches the mask still holds, the updated
// mask, the item's survivor count (and, with WEIGHTED,
// the sum of the survivors' learned weights), and the 45 sums of
// c' w w^T over the survivors with c' = 1/max(|eps_hat|, delta) times the
// learned weight on learned scenes -- the 1/Z normaliser, known only once
// every item has been counted, is applied when the items are summed into
// W_n.  The next 16-byte vectors are loaded before the current ones are used.
template <bool WEIGHTED>
__global__ __launch_bounds__(kQuadThreads) void k_quad_build(
    const float4* __restrict__ X1, const float4* __restrict__ Y1, const float4* __restrict__ X2,
    const float4* __restrict__ Y2, const int4* __restrict__ items, const double* __restrict__ ptab,
    const ushort4* __restrict__ Wl, uchar4* __restrict__ mask, double delta, double* __restrict__ qpart,
    int32_t* __restrict__ keep, double* __restrict__ wkept) {
  __shared__ double s_red[kQuadThreads / kWave][kQuad + 1];
  __shared__ int s_cnt[kQuadThreads / kWave];
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
  const double tau = row[kRowTau];
  const bool learned = WEIGHTED && row[kRowMode] != 0.0;

  double acc[kQuad];
#pragma unroll
  for (int k = 0; k < kQuad; ++k) acc[k] = 0.0;
  double wsum = 0.0;
  int kept = 0;
  int v = tid;
  float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a, c = a, d = a;
  ushort4 wq = make_ushort4(0, 0, 0, 0);
  uchar4 mq = make_uchar4(0, 0, 0, 0);
  if (v < nvec) {
    a = X1[v0 + v];
    b = Y1[v0 + v];
    c = X2[v0 + v];
    d = Y2[v0 + v];
    if (WEIGHTED) wq = Wl[v0 + v];
    mq = mask[v0 + v];
  }
  for (; v < nvec; v += kQuadThreads) {
    const float4 ca = a, cb = b, cc = c, cd = d;
    const ushort4 cw4 = wq;
    const uchar4 cm = mq;
    const int vn = v + kQuadThreads;
    if (vn < nvec) {
      a = X1[v0 + vn];
      b = Y1[v0 + vn];
      c = X2[v0 + vn];
      d = Y2[v0 + vn];
      if (WEIGHTED) wq = Wl[v0 + vn];
      mq = mask[v0 + vn];
    }
    unsigned char out[kVec] = {0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < kVec; ++e) {
      const double x1 = v4q(ca, e), y1 = v4q(cb, e), x2 = v4q(cc, e), y2 = v4q(cd, e);
      const double l0 = fma(Fh[0], x1, fma(Fh[1], y1, Fh[2]));
      const double l1 = fma(Fh[3], x1, fma(Fh[4], y1, Fh[5]));
      const double l2 = fma(Fh[6], x1, fma(Fh[7], y1, Fh[8]));
      const double eph = fma(x2, l0, fma(y2, l1, l2));
      const unsigned char was = e == 0 ? cm.x : (e == 1 ? cm.y : (e == 2 ? cm.z : cm.w));
      if (!(was && v * kVec + e < cnt && fabs(eph) < tau)) continue;
      out[e] = 1;
      ++kept;
      double cw = 1.0 / fmax(fabs(eph), delta);
      if (learned) {
        const double wl = (double)__uint_as_float((uint32_t)v4w(cw4, e) << 16);
        cw *= wl;
        wsum += wl;
      }
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
    mask[v0 + v] = make_uchar4(out[0], out[1], out[2], out[3]);  // a dropped match stays dropped
  }
  wave_sum_f64_multi<kQuad>(acc);
  wsum = wave_sum_f64(wsum);
  int kw = kept;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) kw += __shfl_xor(kw, m);
  const int wid = tid >> 6, lane = tid & 63;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kQuad; ++k) s_red[wid][k] = acc[k];
    s_red[wid][kQuad] = wsum;
    s_cnt[wid] = kw;
  }
  __syncthreads();
  if (tid <= kQuad) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kQuadThreads / kWave; ++w) s += s_red[w][tid];
    if (tid < kQuad)
      qpart[(int64_t)item * kQuad + tid] = s;
    else if (WEIGHTED)
      wkept[item] = s;
  }
  if (tid == 0) {
    int s = 0;
#pragma unroll
    for (int w = 0; w < kQuadThreads / kWave; ++w) s += s_cnt[w];
    keep[item] = s;
  }
}

// Every valid slot of the layout retained (start of a solve).
__global__ void k_mask_init(int64_t n, const int32_t* __restrict__ lpos, unsigned char* __restrict__ mask) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) mask[s] = lpos[s] >= 0 ? 1 : 0;
}

// slot_pos of dropped slots to -1.
__global__ void k_mask_slots(int64_t n, const unsigned char* __restrict__ mask, int32_t* __restrict__ slot_pos) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n && !mask[s]) slot_pos[s] = -1;
}

// W_n = (1/Z of the pair's scene) * the sum of the pair's item partials in
// item order; 1/Z is the pose table's (learned scenes: 1/sum of weights).
__global__ __launch_bounds__(kQuadThreads) void k_quad_reduce(int32_t P, const int32_t* __restrict__ pair_item_off,
                                                              const double* __restrict__ ptab,
                                                              const double* __restrict__ qpart,
                                                              double* __restrict__ qW) {
  const int64_t t = (int64_t)blockIdx.x * kQuadThreads + threadIdx.x;
  if (t >= (int64_t)P * kQuad) return;
  const int n = (int)(t / kQuad), k = (int)(t % kQuad);
  const double* row = ptab + (int64_t)n * kPairRow;
  const double inv_z = row[kRowMode] != 0.0 ? row[kRowInvZw] : row[kRowInvZ];
  double s = 0.0;
  for (int it = pair_item_off[n]; it < pair_item_off[n + 1]; ++it) s += qpart[(int64_t)it * kQuad + k];
  qW[t] = inv_z * s;
}

}  // namespace

// The round's pass over the full layout's items: threshold test at the
// snapshot (pose table rows: F_hat, tau) of the matches the retained mask
// holds, the mask updated in place, survivor counts into item_keep,
// the learned weights' survivor sums into item_wsum (learned scenes), and the
// unnormalised per-item sums of the quadratic form.
hipError_t launch_quad_build(fea_ctx* c) {
  if (c->n_items == 0) return hipSuccess;
  const int b = c->cur;
#define FEA_QUAD_BUILD_ARGS                                                                                 \
  c->lay[b][0].as<float4>(), c->lay[b][1].as<float4>(), c->lay[b][2].as<float4>(), c->lay[b][3].as<float4>(), \
      c->item_rec.as<int4>(), c->ptab.as<double>(), c->wlay.as<ushort4>(), c->qmask.as<uchar4>(), c->opt.delta,  \
      c->qpart.as<double>(), c->item_keep.as<int32_t>(), c->item_wsum.as<double>()
  if (c->learned_any)
    k_quad_build<true><<<(unsigned)c->n_items, kQuadThreads, 0, c->stream>>>(FEA_QUAD_BUILD_ARGS);
  else
    k_quad_build<false><<<(unsigned)c->n_items, kQuadThreads, 0, c->stream>>>(FEA_QUAD_BUILD_ARGS);
#undef FEA_QUAD_BUILD_ARGS
  return hipGetLastError();
}

hipError_t launch_mask_init(fea_ctx* c) {
  const int64_t n = c->layout_len;
  if (n == 0) return hipSuccess;
  k_mask_init<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(n, c->lpos[0].as<int32_t>(),
                                                                  c->qmask.as<unsigned char>());
  return hipGetLastError();
}

hipError_t launch_mask_slots(fea_ctx* c, int32_t* slot_pos) {
  const int64_t n = c->layout_len;
  if (n == 0) return hipSuccess;
  k_mask_slots<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(n, c->qmask.as<unsigned char>(), slot_pos);
  return hipGetLastError();
}

// W_n of every pair from the item sums of launch_quad_build; the pose
// table's normalisers are refreshed first (they are set after the counts).
hipError_t launch_quad_reduce(fea_ctx* c, const int32_t* pair_item_off_dev) {
  if (c->P == 0) return hipSuccess;
  hipError_t e = launch_pair_pose(c, c->R[c->pcur].as<double>(), c->T[c->pcur].as<double>(),
                                  c->Fc[c->pcur].as<double>(), false);
  if (e != hipSuccess) return e;
  const int64_t t = c->P * kQuad;
  k_quad_reduce<<<(unsigned)((t + kQuadThreads - 1) / kQuadThreads), kQuadThreads, 0, c->stream>>>(
      (int32_t)c->P, pair_item_off_dev, c->ptab.as<double>(), c->qpart.as<double>(), c->qW.as<double>());
  return hipGetLastError();
}

}  // namespace fea
