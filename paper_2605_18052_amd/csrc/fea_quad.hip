// Quadratic-form inner loop of FastMap's epipolar adjustment (Method >
// Epipolar Adjustment: with the IRLS weights frozen for a round, the
// objective of pair n is f^T W_n f, f = vec(F) and W_n the weighted sum of
// the outer products of the matches' 9-vectors), for gfx950.
//
// Once per round, k_quad_build streams the retained matches of each work item
// (the same 16 bytes per match as the per-match kernel) and accumulates, per
// lane in fp64, sum c w w^T with w = vec(p2 p1^T) in centred pixel
// coordinates and c the round's IRLS weight (times the learned weight on
// learned scenes), one wavefront per work item.  With p = (u, v, 1) the
// entry of w w^T at (3a + b, 3a' + b') is (p2_a p2_a') (p1_b p1_b'), and each
// factor takes one of only 6 values (u^2, uv, u, v^2, v, 1), so the kernel
// sums the 6 x 6 products c P2_s P1_t -- 36 multiply-adds per match
// instead of the 45 of the form's distinct entries plus the 18 products
// that build c w.  The 36 sums are reduced over the wave (lane swaps and
// DPP) into one fp64 partial per item; k_quad_reduce adds a pair's item partials
// in item order and spreads the 36 sums over W_n's 45 entries.
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
constexpr int kMono = 36;  // products P2_s P1_t summed per match (6 x 6)
constexpr int kQuadThreads = 256;

// Index (0..5) of the product x_a x_b, a <= b, of a 3-vector's entries.
__host__ __device__ constexpr int sym3(int a, int b) { return a == 0 ? b : (a == 1 ? 2 + b : 5); }

// For entry k of the form's upper triangle (row-major: (0,0), (0,1), ...,
// (0,8), (1,1), ...), the index 6 s + t of its sum: entry (i, j) with
// i = 3a + b, j = 3a' + b' is P2_{sym(a, a')} P1_{sym(b, b')}.
struct MonoTable {
  int of[kQuad];
  constexpr MonoTable() : of() {
    int k = 0;
    for (int i = 0; i < 9; ++i)
      for (int j = i; j < 9; ++j, ++k) {
        const int a = i / 3, b = i % 3, a2 = j / 3, b2 = j % 3;
        const int s = a <= a2 ? sym3(a, a2) : sym3(a2, a);
        const int t = b <= b2 ? sym3(b, b2) : sym3(b2, b);
        of[k] = 6 * s + t;
      }
  }
};
__constant__ constexpr MonoTable kMonoOf{};

// One item of the round's pass per wavefront (kBuildItems items per
// workgroup, no block-level synchronisation): the threshold test at the
// snapshot (|eps_hat| < tau, strict) of the matches the mask still holds,
// the updated mask, the item's survivor count (and, with WEIGHTED, the sum
// of the survivors' learned weights), and the 45 sums of c' w w^T over the
// survivors with c' = 1/max(|eps_hat|, delta) times the learned weight on
// learned scenes -- the 1/Z normaliser, known only once every item has been
// counted, is applied when the items are summed into W_n.  The test is
// branch-free: a dropped match gets c' = 0 and adds exactly zero.  Each lane
// takes one match per trip, so only that match's products are live next to
// the 36 per-lane sums (occupancy 4); the 36 sums are reduced over the wave
// by three reduce-scatters (16, 16 and 4 sums), stored straight from the
// lanes that hold them.  The next match is loaded before the current one is
// used.
constexpr int kBuildItems = kQuadThreads / kWave;

template <bool WEIGHTED>
__global__ __launch_bounds__(kQuadThreads) void k_quad_build(
    int32_t n_items, const float* __restrict__ X1, const float* __restrict__ Y1, const float* __restrict__ X2,
    const float* __restrict__ Y2, const int4* __restrict__ items, const double* __restrict__ ptab,
    const unsigned short* __restrict__ Wl, unsigned char* __restrict__ mask, double delta,
    double* __restrict__ qpart, int32_t* __restrict__ keep, double* __restrict__ wkept,
    const int32_t* __restrict__ pair_scene, const int32_t* __restrict__ scene_done) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int item = __builtin_amdgcn_readfirstlane((int)blockIdx.x * kBuildItems + wid);
  if (item >= n_items) return;  // the whole wave
  const int4 rec = items[item];
  const int n = rec.x;
  // a converged scene keeps its mask, counts and sums from its last round
  if (scene_done != nullptr && scene_done[pair_scene[n]] != 0) return;
  const int64_t s0 = rec.y;  // first slot of the item
  const int cnt = rec.z;
  // every slot of the item's last 16-byte vector is visited, so the padding
  // slots of a pair's run are written as dropped, as in the vector layout
  const int nslot = (cnt + kVec - 1) / kVec * kVec;
  const double* row = ptab + (int64_t)n * kPairRow;
  double Fh[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Fh[k] = row[kRowFh + k];
  const double cxi = row[kRowCx + 0], cyi = row[kRowCx + 1];
  const double cxj = row[kRowCx + 2], cyj = row[kRowCx + 3];
  const double tau = row[kRowTau];
  const bool learned = WEIGHTED && row[kRowMode] != 0.0;

  double acc[kMono];
#pragma unroll
  for (int k = 0; k < kMono; ++k) acc[k] = 0.0;
  double wsum = 0.0;
  int kept = 0;
  // one match per lane per trip (consecutive lanes read consecutive words),
  // so that only one match's products are live next to the 36 sums; the
  // next trip's match is loaded before the current one is used
  const float *__restrict__ x1p = X1 + s0, *__restrict__ y1p = Y1 + s0;
  const float *__restrict__ x2p = X2 + s0, *__restrict__ y2p = Y2 + s0;
  const unsigned short* __restrict__ wp = Wl + s0;
  unsigned char* __restrict__ mp = mask + s0;
  const unsigned ns = (unsigned)nslot;
  unsigned j = lane;
  float x1 = 0.f, y1 = 0.f, x2 = 0.f, y2 = 0.f;
  unsigned short wq = 0;
  unsigned char mq = 0;
  if (j < ns) {
    x1 = x1p[j];
    y1 = y1p[j];
    x2 = x2p[j];
    y2 = y2p[j];
    if (WEIGHTED) wq = wp[j];
    mq = mp[j];
  }
  for (; j < ns; j += kWave) {
    const double dx1 = x1, dy1 = y1, dx2 = x2, dy2 = y2;
    const unsigned short cwq = wq;
    const bool was = mq != 0;
    const unsigned jn = j + kWave;
    if (jn < ns) {
      x1 = x1p[jn];
      y1 = y1p[jn];
      x2 = x2p[jn];
      y2 = y2p[jn];
      if (WEIGHTED) wq = wp[jn];
      mq = mp[jn];
    }
    const double l0 = fma(Fh[0], dx1, fma(Fh[1], dy1, Fh[2]));
    const double l1 = fma(Fh[3], dx1, fma(Fh[4], dy1, Fh[5]));
    const double l2 = fma(Fh[6], dx1, fma(Fh[7], dy1, Fh[8]));
    const double eph = fma(dx2, l0, fma(dy2, l1, l2));
    const bool hold = was && j < (unsigned)cnt && fabs(eph) < tau;
    mp[j] = hold ? 1 : 0;  // a dropped match stays dropped
    kept += hold ? 1 : 0;
    // 1 / max(|eps_hat|, delta): the hardware reciprocal refined by two
    // Newton steps r <- r + r (1 - x r), within an ulp of the quotient
    const double x = fmax(fabs(eph), delta);
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    double cw = hold ? r : 0.0;
    if (learned) {
      // the network writes only the slots of real matches: the weight of a
      // padding slot is never read into the arithmetic (0 * NaN is NaN)
      const double wl = (double)(float)__builtin_bit_cast(_Float16, cwq);
      cw = hold ? cw * wl : 0.0;
      wsum += hold ? wl : 0.0;
    }
    const double u1 = dx1 - cxi, v1 = dy1 - cyi, u2 = dx2 - cxj, v2 = dy2 - cyj;
    const double cu2 = cw * u2, cv2 = cw * v2;
    // sym3 order: u^2, uv, u, v^2, v, 1
    const double P1[6] = {u1 * u1, u1 * v1, u1, v1 * v1, v1, 1.0};
    const double cP2[6] = {cu2 * u2, cu2 * v2, cu2, cv2 * v2, cv2, cw};
#pragma unroll
    for (int s2 = 0; s2 < 6; ++s2)
#pragma unroll
      for (int t = 0; t < 6; ++t) acc[6 * s2 + t] = fma(cP2[s2], P1[t], acc[6 * s2 + t]);
  }
  // the wave is the item: the 36 sums as reduce-scatters of 16, 16 and 4,
  // each stored by the lanes that end up holding it
  double* out = qpart + (int64_t)item * kMono;
  {
    double x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = acc[k];
    wave_scatter_stages_f64<16>(x);
    if ((lane & 3) == 0) out[(lane >> 2) & 15] = x[0];
  }
  {
    double x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = acc[16 + k];
    wave_scatter_stages_f64<16>(x);
    if ((lane & 3) == 0) out[16 + ((lane >> 2) & 15)] = x[0];
  }
  {
    double x[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = acc[32 + k];
    wave_scatter_stages_f64<4>(x);
    if ((lane & 15) == 0) out[32 + ((lane >> 4) & 3)] = x[0];
  }
  int kw = kept;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) kw += __shfl_xor(kw, m);
  if (WEIGHTED) wsum = wave_sum_f64(wsum);
  if (lane == 0) {
    keep[item] = kw;
    if (WEIGHTED) wkept[item] = wsum;
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
// item order, entry k taking sum kMonoOf.of[k]; 1/Z is the pose table's
// (learned scenes: 1/sum of weights).
__global__ __launch_bounds__(kQuadThreads) void k_quad_reduce(int32_t P, const int32_t* __restrict__ pair_item_off,
                                                              const double* __restrict__ ptab,
                                                              const double* __restrict__ qpart,
                                                              double* __restrict__ qW,
                                                              const int32_t* __restrict__ pair_scene,
                                                              const int32_t* __restrict__ scene_done) {
  const int64_t t = (int64_t)blockIdx.x * kQuadThreads + threadIdx.x;
  if (t >= (int64_t)P * kQuad) return;
  const int n = (int)(t / kQuad), k = (int)(t % kQuad);
  if (scene_done != nullptr && scene_done[pair_scene[n]] != 0) return;  // keeps its last round's form
  const double* row = ptab + (int64_t)n * kPairRow;
  const double inv_z = row[kRowMode] != 0.0 ? row[kRowInvZw] : row[kRowInvZ];
  const int mk = kMonoOf.of[k];
  double s = 0.0;
  for (int it = pair_item_off[n]; it < pair_item_off[n + 1]; ++it) s += qpart[(int64_t)it * kMono + mk];
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
  c->lay[b][0].as<float>(), c->lay[b][1].as<float>(), c->lay[b][2].as<float>(), c->lay[b][3].as<float>(),     \
      c->item_rec.as<int4>(), c->ptab.as<double>(), c->wlay.as<unsigned short>(), c->qmask.as<unsigned char>(),  \
      c->opt.delta,                                                                                          \
      c->qpart.as<double>(), c->item_keep.as<int32_t>(), c->item_wsum.as<double>(),                          \
      c->d_pair_scene.as<int32_t>(), c->d_scene_done.as<int32_t>()
  const unsigned blocks = (unsigned)((c->n_items + kBuildItems - 1) / kBuildItems);
  if (c->learned_any)
    k_quad_build<true><<<blocks, kQuadThreads, 0, c->stream>>>((int32_t)c->n_items, FEA_QUAD_BUILD_ARGS);
  else
    k_quad_build<false><<<blocks, kQuadThreads, 0, c->stream>>>((int32_t)c->n_items, FEA_QUAD_BUILD_ARGS);
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
      (int32_t)c->P, pair_item_off_dev, c->ptab.as<double>(), c->qpart.as<double>(), c->qW.as<double>(),
      c->d_pair_scene.as<int32_t>(), c->d_scene_done.as<int32_t>());
  return hipGetLastError();
}

}  // namespace fea
