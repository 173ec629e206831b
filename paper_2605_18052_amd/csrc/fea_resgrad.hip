// The per-match pass of FastMap's epipolar adjustment (Method > Epipolar
// Adjustment, the IRLS-reweighted objective) and the round-start outlier
// filter, for gfx950.
//
// k_pair_pose: one thread per camera pair builds the pair's pose block in
// fp64 -- F at the current poses (every step) and F_hat at the round
// snapshot (once per round), both with the principal points folded in so
// they act on raw pixel coordinates -- into a per-pair row of the pose table,
// with the scene's 1/Z and the pair's principal points.
//
// k_resgrad: one workgroup per work item (<= 8192 matches of one camera pair,
// contiguous in the pair-sorted SoA layout; with the quadratic form the
// layout stays whole and a per-match mask marks the retained matches).  Every thread issues all of its
// 16-byte loads first; the pair's row is read with scalar loads (the item,
// hence the pair, is uniform across the workgroup), so no wave waits on
// another before streaming.  Per match: eps = q2^T F q1 and eps_hat in fp64
// (the residual of an inlier is ~1e-3 of its terms, so fp32 would lose ~4
// digits), weight c = 1/(Z max(|eps_hat|, delta)), then the contribution
// 2 c eps p2 p1^T to dL/dF and c eps^2 to L accumulate per lane in fp32.
// The 10 sums are reduced across each wave (a reduce-scatter of lane swaps
// and DPP), across the waves in LDS, and written as one fp64 partial per
// item -- no atomics, so the result is deterministic.  The loss-only pass
// sums c eps^2 and, in the slot the gradient would use, c eps_hat^2: the
// objective at the current poses and at the round's snapshot in one read.
#include <hip/hip_runtime.h>

#include <hip/hip_ext.h>

#include <algorithm>

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

// Pose block of pair n (i < j) into its row of the pose table: F at
// (R, T, Fc) and the scene's weight normalisers, every step; with SNAP also
// F_hat at the snapshot (Rh, Th, Fh), the principal points and the threshold.
template <bool SNAP>
__global__ __launch_bounds__(kPairThreads) void k_pair_pose(
    int32_t P, const int32_t* __restrict__ pair_i, const int32_t* __restrict__ pair_j,
    const double* __restrict__ R, const double* __restrict__ T, const double* __restrict__ Fc,
    const double* __restrict__ Rh, const double* __restrict__ Th, const double* __restrict__ Fh,
    const double* __restrict__ cx, const double* __restrict__ cy, const int32_t* __restrict__ pair_scene,
    const float* __restrict__ inv_z_scene, const float* __restrict__ inv_zw_scene,
    const int32_t* __restrict__ scene_mode, const double* __restrict__ tau_scene, double* __restrict__ ptab) {
  const int n = blockIdx.x * kPairThreads + threadIdx.x;
  if (n >= P) return;
  const int i = pair_i[n], j = pair_j[n], sc = pair_scene[n];
  double* row = ptab + (int64_t)n * kPairRow;
  double Fp[9];
  pose_block(i, j, R, T, Fc, cx, cy, Fp);
#pragma unroll
  for (int k = 0; k < 9; ++k) row[kRowF + k] = Fp[k];
  row[kRowInvZ] = (double)inv_z_scene[sc];
  row[kRowInvZw] = (double)inv_zw_scene[sc];
  row[kRowMode] = scene_mode[sc] != 0 ? 1.0 : 0.0;
  if (SNAP) {
    pose_block(i, j, Rh, Th, Fh, cx, cy, Fp);
#pragma unroll
    for (int k = 0; k < 9; ++k) row[kRowFh + k] = Fp[k];
    row[kRowCx + 0] = cx[i];
    row[kRowCx + 1] = cy[i];
    row[kRowCx + 2] = cx[j];
    row[kRowCx + 3] = cy[j];
    row[kRowTau] = tau_scene[sc];
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 nt_load(const float4* p) {
  const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

// One work item's coordinates (and learned weights / retained mask) in
// registers: STEPS 16-byte loads per array per thread, issued together.
template <int THREADS, int STEPS, bool WEIGHTED>
struct ItemRegs {
  float4 a[STEPS], b[STEPS], c[STEPS], d[STEPS];
  ushort4 w[WEIGHTED ? STEPS : 1];
  uchar4 m[STEPS];

  __device__ __forceinline__ void load(const float4* __restrict__ X1, const float4* __restrict__ Y1,
                                       const float4* __restrict__ X2, const float4* __restrict__ Y2,
                                       const ushort4* __restrict__ Wl, const uchar4* __restrict__ qmask, int4 rec,
                                       int tid) {
    const int v0 = rec.y >> 2;
    const int nvec = (rec.z + kVec - 1) / kVec;
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
      const int v = s * THREADS + tid;
      m[s] = make_uchar4(1, 1, 1, 1);
      if (v < nvec) {
        // read once per pass: non-temporal, so the stream does not
        // displace cached data
        a[s] = nt_load(X1 + v0 + v);
        b[s] = nt_load(Y1 + v0 + v);
        c[s] = nt_load(X2 + v0 + v);
        d[s] = nt_load(Y2 + v0 + v);
        if (WEIGHTED) w[s] = Wl[v0 + v];
        if (qmask) m[s] = qmask[v0 + v];
      } else {
        a[s] = b[s] = c[s] = d[s] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (WEIGHTED) w[s] = make_ushort4(0, 0, 0, 0);
      }
    }
  }
};

// The residuals, weights and gradient sums of one work item whose data sit
// in q, reduced over the workgroup into its fp64 partial part[item]
// (s_red: the workgroup's reduction buffer, free on entry; one barrier).
template <int THREADS, int STEPS, bool LOSS_ONLY, bool WEIGHTED>
__device__ __forceinline__ void resgrad_item(const ItemRegs<THREADS, STEPS, WEIGHTED>& q, int4 rec, int item,
                                             const double* __restrict__ ptab, float delta,
                                             double* __restrict__ part, float (*s_red)[kPartStride], int tid) {
  const int n = rec.x;
  const int cnt = rec.z;
  const double* row = ptab + (int64_t)n * kPairRow;
  double F[9], Fhat[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    F[k] = row[kRowF + k];
    Fhat[k] = row[kRowFh + k];
  }
  const float cxi = (float)row[kRowCx + 0];
  const float cyi = (float)row[kRowCx + 1];
  const float cxj = (float)row[kRowCx + 2];
  const float cyj = (float)row[kRowCx + 3];
  const bool learned = WEIGHTED && row[kRowMode] != 0.0;
  const float inv_z = (float)(learned ? row[kRowInvZw] : row[kRowInvZ]);

  float acc[kPartStride];
#pragma unroll
  for (int k = 0; k < kPartStride; ++k) acc[k] = 0.f;
#pragma unroll
  for (int s = 0; s < STEPS; ++s) {
#pragma unroll
    for (int e = 0; e < kVec; ++e) {
      const int local = (s * THREADS + tid) * kVec + e;
      const float x1 = v4(q.a[s], e), y1 = v4(q.b[s], e), x2 = v4(q.c[s], e), y2 = v4(q.d[s], e);
      const double eps = eval_eps(F, x1, y1, x2, y2);
      const double eph = eval_eps(Fhat, x1, y1, x2, y2);
      const float ef = (float)eps;
      const float w = fmaxf(fabsf((float)eph), delta);
      float c = inv_z * __builtin_amdgcn_rcpf(w);
      if (WEIGHTED && learned) {
        const unsigned short wb = e == 0 ? q.w[s].x : (e == 1 ? q.w[s].y : (e == 2 ? q.w[s].z : q.w[s].w));
        c *= (float)__builtin_bit_cast(_Float16, wb);
      }
      const unsigned char held = e == 0 ? q.m[s].x : (e == 1 ? q.m[s].y : (e == 2 ? q.m[s].z : q.m[s].w));
      c = (local < cnt && held) ? c : 0.f;  // alignment padding and dropped matches hold no weight
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
      } else {
        // the loss-only pass also sums the loss at the round's snapshot,
        // c eps_hat^2, into slot 8 (unused there otherwise)
        const float ehf = (float)eph;
        acc[8] = fmaf(c * ehf, ehf, acc[8]);
      }
      acc[9] = fmaf(c * ef, ef, acc[9]);
    }
  }
  const int wid = tid >> 6, lane = tid & 63;
  wave_sum_f32_scatter(acc);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kPartStride; ++k) s_red[wid][k] = acc[k];
  }
  __syncthreads();
  if (tid < kPartStride) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < THREADS / kWave; ++w) sum += (double)s_red[w][tid];
    part[(int64_t)item * kPartStride + tid] = sum;
  }
}

// One workgroup per work item.
template <int THREADS, int STEPS, bool LOSS_ONLY, bool WEIGHTED>
__global__ __launch_bounds__(THREADS) void k_resgrad(
    const float4* __restrict__ X1, const float4* __restrict__ Y1, const float4* __restrict__ X2,
    const float4* __restrict__ Y2, const int4* __restrict__ items, const double* __restrict__ ptab, float delta,
    double* __restrict__ part, const ushort4* __restrict__ Wl, const uchar4* __restrict__ qmask,
    int skip_flagged) {
  __shared__ float s_red[THREADS / kWave][kPartStride];
  const int tid = threadIdx.x;
  const int item = blockIdx.x;
  const int4 rec = items[item];
  // a step skips the items of converged scenes (flag in the record's last
  // field); their partials are not read by the update
  if (skip_flagged && rec.w != 0) return;
  ItemRegs<THREADS, STEPS, WEIGHTED> q;
  q.load(X1, Y1, X2, Y2, Wl, qmask, rec, tid);
  resgrad_item<THREADS, STEPS, LOSS_ONLY, WEIGHTED>(q, rec, item, ptab, delta, part, s_red, tid);
}

// A fixed number of workgroups per CU, each walking the items
// blockIdx.x, blockIdx.x + gridDim.x, ...: the next item's record and
// coordinates are loaded before the current item is computed, so every
// workgroup keeps its loads in flight while it computes and no load waits
// on a record.  The reduction buffer alternates between two halves, so one
// barrier per item suffices.  Same partials as k_resgrad, bit for bit.
template <int THREADS, int STEPS, bool LOSS_ONLY, bool WEIGHTED>
__global__ __launch_bounds__(THREADS) void k_resgrad_p(
    const float4* __restrict__ X1, const float4* __restrict__ Y1, const float4* __restrict__ X2,
    const float4* __restrict__ Y2, const int4* __restrict__ items, int32_t n_items,
    const double* __restrict__ ptab, float delta, double* __restrict__ part, const ushort4* __restrict__ Wl,
    const uchar4* __restrict__ qmask, int skip_flagged) {
  __shared__ float s_red[2][THREADS / kWave][kPartStride];
  const int tid = threadIdx.x;
  int item = blockIdx.x;
  if (item >= n_items) return;
  int4 rec = items[item];
  // two items per trip, so that the two register buffers keep fixed roles
  // (indexing one array of them by the trip's parity would put them in
  // scratch memory)
  ItemRegs<THREADS, STEPS, WEIGHTED> q0, q1;
  q0.load(X1, Y1, X2, Y2, Wl, qmask, rec, tid);
  for (;;) {
    int next = item + (int)gridDim.x;
    bool more = next < n_items;
    int4 nrec = more ? items[next] : rec;
    if (more) q1.load(X1, Y1, X2, Y2, Wl, qmask, nrec, tid);
    if (!(skip_flagged && rec.w != 0))
      resgrad_item<THREADS, STEPS, LOSS_ONLY, WEIGHTED>(q0, rec, item, ptab, delta, part, s_red[0], tid);
    if (!more) break;
    item = next;
    rec = nrec;
    next = item + (int)gridDim.x;
    more = next < n_items;
    nrec = more ? items[next] : rec;
    if (more) q0.load(X1, Y1, X2, Y2, Wl, qmask, nrec, tid);
    if (!(skip_flagged && rec.w != 0))
      resgrad_item<THREADS, STEPS, LOSS_ONLY, WEIGHTED>(q1, rec, item, ptab, delta, part, s_red[1], tid);
    if (!more) break;
    item = next;
    rec = nrec;
  }
}

// Whether slot value `pos` (a sorted position, -1 for padding) is set in the
// bit mask over sorted positions.
__device__ __forceinline__ bool mask_bit(const uint32_t* __restrict__ mask, int pos) {
  return pos >= 0 && ((mask[pos >> 5] >> (pos & 31)) & 1u);
}

// Round start, pass 1: how many matches of each item survive -- the filter
// |eps_hat| < tau (strict; Method > Epipolar Adjustment, outlier filtering),
// or, with BY_MASK, membership in a saved retained set (resume from a
// checkpoint).
template <bool BY_MASK>
__global__ __launch_bounds__(kFilterThreads) void k_filter_count(
    const float4* __restrict__ X1, const float4* __restrict__ Y1, const float4* __restrict__ X2,
    const float4* __restrict__ Y2, const int4* __restrict__ POS, const int4* __restrict__ items,
    const double* __restrict__ ptab, const uint32_t* __restrict__ mask, int32_t* __restrict__ keep) {
  __shared__ int s_cnt;
  const int tid = threadIdx.x, item = blockIdx.x;
  const int4 rec = items[item];
  const int n = rec.x;
  const int v0 = rec.y >> 2;
  const int cnt = rec.z;
  const int nvec = (cnt + kVec - 1) / kVec;
  const double* row = ptab + (int64_t)n * kPairRow;
  double Fhat[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Fhat[k] = row[kRowFh + k];
  const double tau = row[kRowTau];
  if (tid == 0) s_cnt = 0;
  __syncthreads();
  int kept = 0;
  for (int v = tid; v < nvec; v += kFilterThreads) {
    if (BY_MASK) {
      const int4 p = POS[v0 + v];
      const int pe[4] = {p.x, p.y, p.z, p.w};
#pragma unroll
      for (int e = 0; e < kVec; ++e) kept += (v * kVec + e < cnt) && mask_bit(mask, pe[e]);
    } else {
      const float4 a = X1[v0 + v], b = Y1[v0 + v], c = X2[v0 + v], d = Y2[v0 + v];
#pragma unroll
      for (int e = 0; e < kVec; ++e) {
        const double eph = eval_eps(Fhat, v4(a, e), v4(b, e), v4(c, e), v4(d, e));
        kept += (v * kVec + e < cnt) && (fabs(eph) < tau);
      }
    }
  }
  atomicAdd(&s_cnt, kept);
  __syncthreads();
  if (tid == 0) keep[item] = s_cnt;
}

// Round start, pass 2: stable compaction of the surviving matches into the
// other layout buffer.  base[item] is where the item's first survivor goes.
template <bool BY_MASK>
__global__ __launch_bounds__(kFilterThreads) void k_filter_scatter(
    const float4* __restrict__ X1, const float4* __restrict__ Y1, const float4* __restrict__ X2,
    const float4* __restrict__ Y2, const int4* __restrict__ POS, const int4* __restrict__ items,
    const double* __restrict__ ptab, const uint32_t* __restrict__ mask, const int2* __restrict__ base,
    float* __restrict__ ox1, float* __restrict__ oy1, float* __restrict__ ox2, float* __restrict__ oy2,
    int32_t* __restrict__ opos) {
  __shared__ int s_w[kFilterThreads / kWave];
  const int tid = threadIdx.x, item = blockIdx.x;
  const int4 rec = items[item];
  const int n = rec.x;
  const int v0 = rec.y >> 2;
  const int cnt = rec.z;
  const int nvec = (cnt + kVec - 1) / kVec;
  const double* row = ptab + (int64_t)n * kPairRow;
  double Fhat[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Fhat[k] = row[kRowFh + k];
  const double tau = row[kRowTau];
  const int2 bp = base[item];  // {first destination slot, aligned end of the pair's run or -1}
  int run = bp.x;
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
    const int pe[4] = {p.x, p.y, p.z, p.w};
    int flags = 0, mine = 0;
#pragma unroll
    for (int e = 0; e < kVec; ++e) {
      bool pass;
      if (BY_MASK) {
        pass = mask_bit(mask, pe[e]);
      } else {
        const double eph = eval_eps(Fhat, v4(a, e), v4(b, e), v4(c, e), v4(d, e));
        pass = fabs(eph) < tau;
      }
      const int k = (v < nvec) && (v * kVec + e < cnt) && pass;
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
  // the pair's last item clears the alignment padding after the survivors
  // (fewer than 32 slots), so the new layout needs no clearing beforehand
  for (int sl = run + tid; sl < bp.y; sl += kFilterThreads) {
    ox1[sl] = 0.f;
    oy1[sl] = 0.f;
    ox2[sl] = 0.f;
    oy2[sl] = 0.f;
    opos[sl] = -1;
  }
}

}  // namespace

hipError_t launch_pair_pose(fea_ctx* c, const double* R, const double* T, const double* F, bool snap) {
  if (c->P == 0) return hipSuccess;
  c->ptab_current = R == c->R[c->pcur].as<double>() && T == c->T[c->pcur].as<double>() &&
                    F == c->Fc[c->pcur].as<double>();
  const unsigned blocks = (unsigned)((c->P + kPairThreads - 1) / kPairThreads);
#define FEA_PAIR_POSE_ARGS                                                                                   \
  (int32_t)c->P, c->d_pair_i.as<int32_t>(), c->d_pair_j.as<int32_t>(), R, T, F, c->Rh.as<double>(),          \
      c->Th.as<double>(), c->Fh.as<double>(), c->d_cx.as<double>(), c->d_cy.as<double>(),                  \
      c->d_pair_scene.as<int32_t>(), c->d_inv_z.as<float>(), c->d_inv_zw.as<float>(),                     \
      c->d_scene_mode.as<int32_t>(), c->d_tau.as<double>(), c->ptab.as<double>()
  if (snap)
    k_pair_pose<true><<<blocks, kPairThreads, 0, c->stream>>>(FEA_PAIR_POSE_ARGS);
  else
    k_pair_pose<false><<<blocks, kPairThreads, 0, c->stream>>>(FEA_PAIR_POSE_ARGS);
#undef FEA_PAIR_POSE_ARGS
  return hipGetLastError();
}

// With ev0/ev1 set the dispatch itself records the two events at the
// kernel's start and end (no separate marker packets around it).
// Workgroups of a persistent per-match kernel that reside on one CU at once
// (the runtime's occupancy for its register and LDS use), looked up once.
template <int THREADS, int STEPS, bool LOSS_ONLY, bool WEIGHTED>
int persistent_per_cu() {
  static const int per_cu = [] {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_resgrad_p<THREADS, STEPS, LOSS_ONLY, WEIGHTED>, THREADS,
                                                     0) != hipSuccess ||
        n < 1)
      n = 1;
    return n;
  }();
  return per_cu;
}

template <int THREADS, int STEPS>
void prepare_persistent() {
  (void)persistent_per_cu<THREADS, STEPS, false, false>();
  (void)persistent_per_cu<THREADS, STEPS, true, false>();
  (void)persistent_per_cu<THREADS, STEPS, false, true>();
  (void)persistent_per_cu<THREADS, STEPS, true, true>();
}

template <int THREADS, int STEPS, bool LOSS_ONLY, bool WEIGHTED>
hipError_t launch_resgrad_t(fea_ctx* c, hipEvent_t ev0, hipEvent_t ev1, int skip, bool persistent) {
  const int b = c->cur;
  const int per_cu = persistent ? persistent_per_cu<THREADS, STEPS, LOSS_ONLY, WEIGHTED>() : 0;
  const dim3 grid((unsigned)(per_cu > 0 ? std::min<int64_t>(c->n_items, (int64_t)per_cu * c->n_cu) : c->n_items)),
      block(THREADS);
  const float4 *x1 = c->lay[b][0].as<float4>(), *y1 = c->lay[b][1].as<float4>(), *x2 = c->lay[b][2].as<float4>(),
               *y2 = c->lay[b][3].as<float4>();
  const int4* items = c->item_rec.as<int4>();
  const double* ptab = c->ptab.as<double>();
  const float delta = (float)c->opt.delta;
  double* part = c->part.as<double>();
  const ushort4* wl = c->wlay.as<ushort4>();
  const uchar4* qm = c->opt.inner_loop == 1 ? c->qmask.as<uchar4>() : nullptr;
  if (per_cu > 0) {
    const int32_t ni = (int32_t)c->n_items;
    if (ev0)
      hipExtLaunchKernelGGL(k_resgrad_p<THREADS, STEPS, LOSS_ONLY, WEIGHTED>, grid, block, 0, c->stream, ev0, ev1,
                            0, x1, y1, x2, y2, items, ni, ptab, delta, part, wl, qm, skip);
    else
      k_resgrad_p<THREADS, STEPS, LOSS_ONLY, WEIGHTED>
          <<<grid, block, 0, c->stream>>>(x1, y1, x2, y2, items, ni, ptab, delta, part, wl, qm, skip);
  } else if (ev0) {
    hipExtLaunchKernelGGL(k_resgrad<THREADS, STEPS, LOSS_ONLY, WEIGHTED>, grid, block, 0, c->stream, ev0, ev1, 0,
                          x1, y1, x2, y2, items, ptab, delta, part, wl, qm, skip);
  } else {
    k_resgrad<THREADS, STEPS, LOSS_ONLY, WEIGHTED><<<grid, block, 0, c->stream>>>(x1, y1, x2, y2, items, ptab,
                                                                                  delta, part, wl, qm, skip);
  }
  return hipGetLastError();
}

template <bool LOSS_ONLY, bool WEIGHTED>
hipError_t launch_resgrad_sel(fea_ctx* c, int cfg, hipEvent_t ev0, hipEvent_t ev1, int skip) {
  // the shapes of kTiles, in order
  switch (cfg) {
    case 0: return launch_resgrad_t<256, 4, LOSS_ONLY, WEIGHTED>(c, ev0, ev1, skip, false);
    case 1: return launch_resgrad_t<256, 2, LOSS_ONLY, WEIGHTED>(c, ev0, ev1, skip, false);
    case 2: return launch_resgrad_t<256, 1, LOSS_ONLY, WEIGHTED>(c, ev0, ev1, skip, false);
    case 3: return launch_resgrad_t<128, 8, LOSS_ONLY, WEIGHTED>(c, ev0, ev1, skip, false);
    case 4: return launch_resgrad_t<128, 4, LOSS_ONLY, WEIGHTED>(c, ev0, ev1, skip, false);
    case 5: return launch_resgrad_t<128, 2, LOSS_ONLY, WEIGHTED>(c, ev0, ev1, skip, false);
    case 6: return launch_resgrad_t<512, 2, LOSS_ONLY, WEIGHTED>(c, ev0, ev1, skip, false);
    case 7: return launch_resgrad_t<512, 4, LOSS_ONLY, WEIGHTED>(c, ev0, ev1, skip, false);
    case 8: return launch_resgrad_t<256, 2, LOSS_ONLY, WEIGHTED>(c, ev0, ev1, skip, true);
    case 9: return launch_resgrad_t<256, 1, LOSS_ONLY, WEIGHTED>(c, ev0, ev1, skip, true);
    case 10: return launch_resgrad_t<128, 2, LOSS_ONLY, WEIGHTED>(c, ev0, ev1, skip, true);
    case 11: return launch_resgrad_t<512, 1, LOSS_ONLY, WEIGHTED>(c, ev0, ev1, skip, true);
    case 12: return launch_resgrad_t<512, 2, LOSS_ONLY, WEIGHTED>(c, ev0, ev1, skip, true);
  }
  static_assert(kNumTiles == 13, "a launch for every work-item shape");
  static_assert(kTiles[8].threads == 256 && kTiles[8].steps == 2 && kTiles[9].threads == 256 &&
                    kTiles[9].steps == 1 && kTiles[10].threads == 128 && kTiles[10].steps == 2 &&
                    kTiles[11].threads == 512 && kTiles[11].steps == 1 && kTiles[12].threads == 512 &&
                    kTiles[12].steps == 2 && kTiles[8].persistent && kTiles[12].persistent && !kTiles[7].persistent,
                "the persistent launches follow the table");
  return hipErrorInvalidValue;
}

// Looks up the occupancy of the persistent launches of shape `cfg` now, so
// that no launch issued under graph capture is the first to ask.
void prepare_resgrad(int cfg) {
  if (cfg < 0 || cfg >= kNumTiles || !kTiles[cfg].persistent) return;
  switch (cfg) {
    case 8: prepare_persistent<256, 2>(); break;
    case 9: prepare_persistent<256, 1>(); break;
    case 10: prepare_persistent<128, 2>(); break;
    case 11: prepare_persistent<512, 1>(); break;
    case 12: prepare_persistent<512, 2>(); break;
  }
}

hipError_t launch_resgrad_timed(fea_ctx* c, int cfg, bool loss_only, bool force_plain, hipEvent_t ev0,
                                hipEvent_t ev1, int skip = 0) {
  if (c->n_items == 0) return hipSuccess;
  const bool w = c->learned_any && !force_plain;
  if (loss_only)
    return w ? launch_resgrad_sel<true, true>(c, cfg, ev0, ev1, skip)
             : launch_resgrad_sel<true, false>(c, cfg, ev0, ev1, skip);
  return w ? launch_resgrad_sel<false, true>(c, cfg, ev0, ev1, skip)
           : launch_resgrad_sel<false, false>(c, cfg, ev0, ev1, skip);
}

// The per-match kernel alone, with tile shape `cfg`, over the current items;
// the pose table must hold F for the poses wanted.
hipError_t launch_resgrad_kernel(fea_ctx* c, int cfg, bool loss_only, bool force_plain) {
  return launch_resgrad_timed(c, cfg, loss_only, force_plain, nullptr, nullptr);
}

// Pose table at poses (R, T, F) (per camera, fp64), then the per-match kernel
// with tile shape `cfg`; weights from the round snapshot.
hipError_t launch_resgrad_at(fea_ctx* c, int cfg, const double* R, const double* T, const double* F,
                             bool loss_only, bool force_plain) {
  if (c->n_items == 0) return hipSuccess;
  hipError_t e = launch_pair_pose(c, R, T, F, false);
  if (e != hipSuccess) return e;
  return launch_resgrad_kernel(c, cfg, loss_only, force_plain);
}

hipError_t launch_resgrad_cfg(fea_ctx* c, int cfg) {
  return launch_resgrad_at(c, cfg, c->R[c->pcur].as<double>(), c->T[c->pcur].as<double>(),
                           c->Fc[c->pcur].as<double>(), false, false);
}

// One per-match pass at the current poses (the pose table must hold them:
// launch_pair_pose wrote it after the previous update); with kernel timing
// on, the dispatch records a pair of HIP events at its start and end.  A
// step (step = true) skips the items of converged scenes.
hipError_t launch_resgrad(fea_ctx* c, bool step) {
  if (c->n_items == 0) return hipSuccess;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (c->timing) {
    while (c->ev_pool.size() < c->ev_used + 2) {
      hipEvent_t e;
      const hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) return err;
      c->ev_pool.push_back(e);
    }
    ev0 = c->ev_pool[c->ev_used];
    ev1 = c->ev_pool[c->ev_used + 1];
    c->ev_used += 2;
  }
  return launch_resgrad_timed(c, c->tile_cfg, false, false, ev0, ev1, step && c->opt.converge_deg > 0 ? 1 : 0);
}

hipError_t launch_filter_count(fea_ctx* c, const uint32_t* mask) {
  if (c->n_items == 0) return hipSuccess;
  const int b = c->cur;
#define FEA_FILTER_COUNT_ARGS                                                                                 \
  c->lay[b][0].as<float4>(), c->lay[b][1].as<float4>(), c->lay[b][2].as<float4>(), c->lay[b][3].as<float4>(), \
      c->lpos[b].as<int4>(), c->item_rec.as<int4>(), c->ptab.as<double>(), mask, c->item_keep.as<int32_t>()
  if (mask)
    k_filter_count<true><<<(unsigned)c->n_items, kFilterThreads, 0, c->stream>>>(FEA_FILTER_COUNT_ARGS);
  else
    k_filter_count<false><<<(unsigned)c->n_items, kFilterThreads, 0, c->stream>>>(FEA_FILTER_COUNT_ARGS);
#undef FEA_FILTER_COUNT_ARGS
  return hipGetLastError();
}

hipError_t launch_filter_scatter(fea_ctx* c, int dst, const uint32_t* mask) {
  if (c->n_items == 0) return hipSuccess;
  const int b = c->cur;
#define FEA_FILTER_SCATTER_ARGS                                                                               \
  c->lay[b][0].as<float4>(), c->lay[b][1].as<float4>(), c->lay[b][2].as<float4>(), c->lay[b][3].as<float4>(), \
      c->lpos[b].as<int4>(), c->item_rec.as<int4>(), c->ptab.as<double>(), mask, c->item_base.as<int2>(),       \
      c->lay[dst][0].as<float>(), c->lay[dst][1].as<float>(), c->lay[dst][2].as<float>(),                    \
      c->lay[dst][3].as<float>(), c->lpos[dst].as<int32_t>()
  if (mask)
    k_filter_scatter<true><<<(unsigned)c->n_items, kFilterThreads, 0, c->stream>>>(FEA_FILTER_SCATTER_ARGS);
  else
    k_filter_scatter<false><<<(unsigned)c->n_items, kFilterThreads, 0, c->stream>>>(FEA_FILTER_SCATTER_ARGS);
#undef FEA_FILTER_SCATTER_ARGS
  return hipGetLastError();
}

}  // namespace fea
