// Global Translation (Method > Global Translation).
//
// Relative translations.  With the global rotations fixed, each pair's unit
// relative translation u is chosen among candidate directions by the mean
// epipolar error of the pair's matches, eps(u) = x~2^T [u]x R_ij x~1.  By the
// scalar triple product eps(u) = u . n with n = (R_ij x~1) x x~2, so a pair
// with M matches and K candidates is the product of an M x 3 and a 3 x K
// matrix followed by |.| and a sum over M: a dense contraction of depth 3.
// It runs on the fp32 matrix cores (v_mfma_f32_16x16x4f32, the fourth depth
// slot zero), |D| accumulated per lane; n is computed once per match into LDS.
// A direction and its opposite score the same; the sign comes from a
// cheirality vote (both triangulated depths positive) over the pair's matches.
//
// Camera centres.  The L1 direction loss of
// Eq. fastmap-global-translation-objective is minimised with Adam, one thread
// per (run, camera) wave: the lanes split the camera's pair terms and a fixed
// wave sum adds them (no atomics: the same order at every step), then the
// Adam step.  Several runs from independent random initial centres
// share each launch; they are aligned (centred, unit mean norm) and merged per
// camera by its mean pair loss (Multiple initializations), then the merged
// centres get a final loop.  Everything here is fp64: the work is O(pairs)
// per step and latency-bound.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fea_device.h"
#include "fea_trans.h"

namespace fea {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRtThreads = 256;
constexpr int kRtLds = kRtItem + 16;              // LDS row stride (floats): rows land 16 banks apart
constexpr int kTaThreads = 256;

// ---- relative translations ---------------------------------------------------

// Per pair: R_ij = R_j R_i^T with the focal lengths and principal points, in
// fp32 for the scoring and fp64 for the vote.
__global__ void k_rt_pairs(int64_t n_pairs, const int32_t* __restrict__ pair_i, const int32_t* __restrict__ pair_j,
                           const double* __restrict__ R, const double* __restrict__ f,
                           const double* __restrict__ cx, const double* __restrict__ cy, float* __restrict__ rowf,
                           double* __restrict__ rowd) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= n_pairs) return;
  const int i = pair_i[n], j = pair_j[n];
  const double* Ri = R + 9 * (int64_t)i;
  const double* Rj = R + 9 * (int64_t)j;
  double row[kRtRow];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      row[3 * a + b] = Rj[3 * a] * Ri[3 * b] + Rj[3 * a + 1] * Ri[3 * b + 1] + Rj[3 * a + 2] * Ri[3 * b + 2];
  row[9] = f[i];
  row[10] = f[j];
  row[11] = cx[i];
  row[12] = cy[i];
  row[13] = cx[j];
  row[14] = cy[j];
  row[15] = 0.0;
  for (int k = 0; k < kRtRow; ++k) {
    rowd[kRtRow * n + k] = row[k];
    rowf[kRtRow * n + k] = (float)row[k];
  }
  rowf[kRtRow * n + 9] = (float)(1.0 / row[9]);
  rowf[kRtRow * n + 10] = (float)(1.0 / row[10]);
}

// Scores of kRtGroup candidates over one work item.  MFMA 16x16x4 (fp32):
// lane l supplies A[l%16][l/16] = component l/16 of match l%16 of the block
// and B[l/16][l%16] = component l/16 of candidate l%16; it receives D[4(l/16)+r][l%16]
// for r = 0..3, i.e. four matches of candidate l%16.  Component 3 is zero.
// With CAP every product enters as min(|d|, tau) (one v_med3_f32 clamp each,
// the absolute value folded into the adds), else as |d| (folded into the adds).
template <bool CAP>
__global__ __launch_bounds__(kRtThreads) void k_rt_score(const int4* __restrict__ items, int n_groups,
                                                         const float* __restrict__ rowf,
                                                         const float* __restrict__ x1, const float* __restrict__ y1,
                                                         const float* __restrict__ x2, const float* __restrict__ y2,
                                                         const float* __restrict__ cand, int kp, float tau,
                                                         float* __restrict__ partial) {
  __shared__ float sn[3][kRtLds];
  const int it = blockIdx.x / n_groups;
  const int grp = blockIdx.x - it * n_groups;
  const int4 rec = items[it];  // {pair, layout start, count, -}
  const float* row = rowf + (int64_t)kRtRow * rec.x;
  float Rm[9];
  for (int k = 0; k < 9; ++k) Rm[k] = row[k];
  const float ifi = row[9], ifj = row[10], cxi = row[11], cyi = row[12], cxj = row[13], cyj = row[14];
  const int cnt = rec.z;
  const int nblk = (cnt + 15) >> 4;
  for (int m = threadIdx.x; m < (nblk << 4); m += kRtThreads) {
    float n0 = 0.f, n1 = 0.f, n2 = 0.f;
    if (m < cnt) {
      const int64_t s = (int64_t)rec.y + m;
      const float a0 = (x1[s] - cxi) * ifi, a1 = (y1[s] - cyi) * ifi;
      const float b0 = (x2[s] - cxj) * ifj, b1 = (y2[s] - cyj) * ifj;
      const float r0 = Rm[0] * a0 + Rm[1] * a1 + Rm[2];
      const float r1 = Rm[3] * a0 + Rm[4] * a1 + Rm[5];
      const float r2 = Rm[6] * a0 + Rm[7] * a1 + Rm[8];
      // n = (R_ij x~1) x x~2 with x~2 = (b0, b1, 1)
      n0 = r1 - r2 * b1;
      n1 = r2 * b0 - r0;
      n2 = r0 * b1 - r1 * b0;
    }
    sn[0][m] = n0;
    sn[1][m] = n1;
    sn[2][m] = n2;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kq = lane >> 4, col = lane & 15;
  const int cbase = grp * kRtGroup + wave * (kRtBlocks * 16);
  float bop[kRtBlocks];
#pragma unroll
  for (int q = 0; q < kRtBlocks; ++q) bop[q] = kq < 3 ? cand[(int64_t)kq * kp + cbase + 16 * q + col] : 0.f;
  float accf[kRtBlocks], acc2[kRtBlocks];
#pragma unroll
  for (int q = 0; q < kRtBlocks; ++q) {
    accf[q] = 0.f;
    acc2[q] = 0.f;
  }
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  const float ntau = -tau;
  // the row of the next block is read while this one's products run (the
  // read past the last block stays inside the LDS row: nblk * 16 < kRtLds)
  const float* srow = sn[kq < 3 ? kq : 0];
  float a_next = srow[col];
  for (int mb = 0; mb < nblk; ++mb) {
    const float a = kq < 3 ? a_next : 0.f;
    a_next = srow[((mb + 1) << 4) + col];
#pragma unroll
    for (int q = 0; q < kRtBlocks; ++q) {
      const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bop[q], zero, 0, 0, 0);
      if constexpr (CAP) {
        // |clamp(e, -tau, tau)| = min(|e|, tau): one v_med3 per product, the
        // absolute value rides on the add as a source modifier (fminf would
        // add a canonicalising max before every min)
        const float c0 = __builtin_amdgcn_fmed3f(d[0], ntau, tau), c1 = __builtin_amdgcn_fmed3f(d[1], ntau, tau);
        const float c2 = __builtin_amdgcn_fmed3f(d[2], ntau, tau), c3 = __builtin_amdgcn_fmed3f(d[3], ntau, tau);
        accf[q] += (__builtin_fabsf(c0) + __builtin_fabsf(c1)) + (__builtin_fabsf(c2) + __builtin_fabsf(c3));
      } else
        accf[q] += (__builtin_fabsf(d[0]) + __builtin_fabsf(d[1])) + (__builtin_fabsf(d[2]) + __builtin_fabsf(d[3]));
    }
    if ((mb & 31) == 31) {  // lane sums of at most 128 terms, then at most 4 of those
#pragma unroll
      for (int q = 0; q < kRtBlocks; ++q) {
        acc2[q] += accf[q];
        accf[q] = 0.f;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kRtBlocks; ++q) {
    double s = (double)acc2[q] + (double)accf[q];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (kq == 0) partial[(int64_t)it * kp + cbase + 16 * q + col] = (float)s;
  }
}

// Depth signs of one match for the translation direction u (camera j frame):
// the depths of the least-squares two-view triangulation
// l2 x~2 = l1 R_ij x~1 + u have the signs of -(a.u)(b.b) + (a.b)(b.u) and
// (a.a)(b.u) - (a.b)(a.u), a = R_ij x~1, b = x~2 (the determinant
// |a x b|^2 is positive unless the rays are parallel).
__device__ int cheirality_vote(const double* row, float fx1, float fy1, float fx2, float fy2, const double u[3],
                               double tau) {
  const double ax = ((double)fx1 - row[11]) / row[9], ay = ((double)fy1 - row[12]) / row[9];
  const double bx = ((double)fx2 - row[13]) / row[10], by = ((double)fy2 - row[14]) / row[10];
  const double a0 = row[0] * ax + row[1] * ay + row[2];
  const double a1 = row[3] * ax + row[4] * ay + row[5];
  const double a2 = row[6] * ax + row[7] * ay + row[8];
  // eps(u) = u . (a x b): only matches the chosen direction explains vote
  const double e = u[0] * (a1 - a2 * by) + u[1] * (a2 * bx - a0) + u[2] * (a0 * by - a1 * bx);
  if (!(fabs(e) < tau)) return 0;
  const double aa = a0 * a0 + a1 * a1 + a2 * a2, bb = bx * bx + by * by + 1.0;
  const double ab = a0 * bx + a1 * by + a2;
  const double au = a0 * u[0] + a1 * u[1] + a2 * u[2], bu = bx * u[0] + by * u[1] + u[2];
  const double det = aa * bb - ab * ab;
  if (!(det > 0.0)) return 0;
  const double l1 = -au * bb + ab * bu, l2 = aa * bu - ab * au;
  if (l1 > 0.0 && l2 > 0.0) return 1;
  if (l1 < 0.0 && l2 < 0.0) return -1;
  return 0;
}

// Per pair: mean score of every candidate (sum of the item partials over the
// pair's match count), the lowest (ties: lower index), then the vote of the
// matches with |eps| < tau at that direction.
__global__ __launch_bounds__(kRtThreads) void k_rt_select(int k_cand, int kp, double tau,
                                                          const int32_t* __restrict__ pair_item_off,
                                                          const int4* __restrict__ items,
                                                          const float* __restrict__ partial,
                                                          const float* __restrict__ cand,
                                                          const double* __restrict__ rowd,
                                                          const float* __restrict__ x1, const float* __restrict__ y1,
                                                          const float* __restrict__ x2, const float* __restrict__ y2,
                                                          float* __restrict__ scores, int32_t* __restrict__ best,
                                                          int32_t* __restrict__ vote, double* __restrict__ t_rel,
                                                          double* __restrict__ score_best) {
  __shared__ double sv[kRtThreads];
  __shared__ int si[kRtThreads];
  const int64_t n = blockIdx.x;
  const int i0 = pair_item_off[n], i1 = pair_item_off[n + 1];
  int64_t cnt = 0;
  for (int it = i0; it < i1; ++it) cnt += items[it].z;
  double bv = 0.0;
  int bk = -1;
  for (int k = threadIdx.x; k < k_cand; k += kRtThreads) {
    double s = 0.0;
    for (int it = i0; it < i1; ++it) s += (double)partial[(int64_t)it * kp + k];
    const double mean = s / (double)cnt;
    if (scores) scores[n * k_cand + k] = (float)mean;
    if (bk < 0 || mean < bv) {
      bv = mean;
      bk = k;
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bk;
  __syncthreads();
  for (int s = kRtThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double v2 = sv[threadIdx.x + s];
      const int k2 = si[threadIdx.x + s];
      const int k1 = si[threadIdx.x];
      if (k2 >= 0 && (k1 < 0 || v2 < sv[threadIdx.x] || (v2 == sv[threadIdx.x] && k2 < k1))) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = k2;
      }
    }
    __syncthreads();
  }
  const int kb = si[0];
  const double vb = sv[0];
  const double u[3] = {(double)cand[kb], (double)cand[kp + kb], (double)cand[2 * kp + kb]};
  const double* row = rowd + (int64_t)kRtRow * n;
  int v = 0;
  for (int it = i0; it < i1; ++it) {
    const int4 rec = items[it];
    for (int m = threadIdx.x; m < rec.z; m += kRtThreads) {
      const int64_t s = (int64_t)rec.y + m;
      v += cheirality_vote(row, x1[s], y1[s], x2[s], y2[s], u, tau);
    }
  }
  __syncthreads();
  si[threadIdx.x] = v;
  __syncthreads();
  for (int s = kRtThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) si[threadIdx.x] += si[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int vs = si[0];
    const double sg = vs >= 0 ? 1.0 : -1.0;
    best[n] = kb;
    vote[n] = vs;
    score_best[n] = vb;
    for (int k = 0; k < 3; ++k) t_rel[3 * n + k] = sg * u[k];
  }
}

// ---- camera centres -------------------------------------------------------------

__device__ __forceinline__ double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// o^{i->j} = -R_j^T t^{i->j} / |t^{i->j}|
__global__ void k_ta_targets(int64_t n_pairs, const int32_t* __restrict__ pair_j, const double* __restrict__ R,
                             const double* __restrict__ t_rel, double* __restrict__ target) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pairs) return;
  const double* t = t_rel + 3 * p;
  const double nt = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  const double u[3] = {t[0] / nt, t[1] / nt, t[2] / nt};
  const double* Rj = R + 9 * (int64_t)pair_j[p];
  for (int k = 0; k < 3; ++k) target[3 * p + k] = -(Rj[k] * u[0] + Rj[3 + k] * u[1] + Rj[6 + k] * u[2]);
}

__global__ void k_ta_counters(TaCounters* ctr, double lr) {
  ctr->lr[0] = ctr->lr[1] = lr;
  ctr->b1t[0] = ctr->b1t[1] = 1.0;
  ctr->b2t[0] = ctr->b2t[1] = 1.0;
}

// One wave per (run, camera): the lanes split the camera's pair terms
// (s - n (n.s)) / |d| with s = sign(n - o^{i->j}) / |P|, added for j and
// subtracted for i; a fixed-order wave sum; lanes 0-2 take the Adam step of
// x, y, z.
__global__ __launch_bounds__(kTaThreads) void k_ta_step(int runs, int n_cams, int64_t n_pairs,
                                                        const int32_t* __restrict__ cam_off,
                                                        const int32_t* __restrict__ cam_ent,
                                                        const int32_t* __restrict__ ent_other,
                                                        const double* __restrict__ target,
                                                        const double* __restrict__ o_in, double* __restrict__ o_out,
                                                        double* __restrict__ m, double* __restrict__ v,
                                                        TaCounters* ctr, int p, double beta1, double beta2,
                                                        double eps, double decay) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (kTaThreads / 64) + (threadIdx.x >> 6);
  const double lr = ctr->lr[p];
  const double b1t = ctr->b1t[p] * beta1, b2t = ctr->b2t[p] * beta2;
  if (w == 0 && lane == 0) {  // the other parity's slot: read by the next step only
    ctr->lr[p ^ 1] = lr * decay;
    ctr->b1t[p ^ 1] = b1t;
    ctr->b2t[p ^ 1] = b2t;
  }
  if (w >= (int64_t)runs * n_cams) return;
  const int r = (int)(w / n_cams), c = (int)(w - (int64_t)r * n_cams);
  const int64_t base = (int64_t)r * n_cams * 3;
  const double* o = o_in + base;
  const double inv_np = 1.0 / (double)n_pairs;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  const double oc0 = o[3 * c], oc1 = o[3 * c + 1], oc2 = o[3 * c + 2];
  // the optimiser state of this camera's coordinate (lanes 0..2), loaded
  // before the pair loop so that it arrives meanwhile
  const int64_t a = base + 3 * c + (lane < 3 ? lane : 0);
  double m_old = 0.0, v_old = 0.0, o_old = 0.0;
  if (lane < 3) {
    m_old = m[a];
    v_old = v[a];
    o_old = o_in[a];
  }
  for (int e = cam_off[c] + lane; e < cam_off[c + 1]; e += 64) {
    // the entry and its other camera load side by side (no pair lookup)
    const int ent = cam_ent[e], oc = ent_other[e];
    const int64_t q = ent >> 1;
    const double x0 = o[3 * oc], x1 = o[3 * oc + 1], x2 = o[3 * oc + 2];
    // d = o_j - o_i; this camera is j of the pair when the entry is odd
    const bool cj = ent & 1;
    const double d0 = cj ? oc0 - x0 : x0 - oc0, d1 = cj ? oc1 - x1 : x1 - oc1, d2 = cj ? oc2 - x2 : x2 - oc2;
    const double nd = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    if (!(nd > 0.0)) continue;
    const double inv = 1.0 / nd;
    const double n0 = d0 * inv, n1 = d1 * inv, n2 = d2 * inv;
    const double s0 = sgn(n0 - target[3 * q]) * inv_np, s1 = sgn(n1 - target[3 * q + 1]) * inv_np,
                 s2 = sgn(n2 - target[3 * q + 2]) * inv_np;
    const double ns = n0 * s0 + n1 * s1 + n2 * s2;
    const double sd = (ent & 1) ? inv : -inv;
    g0 += (s0 - n0 * ns) * sd;
    g1 += (s1 - n1 * ns) * sd;
    g2 += (s2 - n2 * ns) * sd;
  }
  double g[3] = {g0, g1, g2};
  wave_sum_f64_scatter(g);
  if (lane < 3) {
    const double gk = lane == 0 ? g[0] : (lane == 1 ? g[1] : g[2]);
    const double mk = beta1 * m_old + (1.0 - beta1) * gk;
    const double vk = beta2 * v_old + (1.0 - beta2) * gk * gk;
    m[a] = mk;
    v[a] = vk;
    const double mh = mk / (1.0 - b1t), vh = vk / (1.0 - b2t);
    o_out[a] = o_old - lr * mh / (sqrt(vh) + eps);
  }
}

// One workgroup per run: centre at the origin, rescale to unit mean norm.
__global__ __launch_bounds__(kTaThreads) void k_ta_align(int n_cams, double* __restrict__ o_all,
                                                         int32_t* __restrict__ err) {
  __shared__ double red[3][kTaThreads];
  double* o = o_all + (int64_t)blockIdx.x * n_cams * 3;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < n_cams; i += kTaThreads) {
    s0 += o[3 * i];
    s1 += o[3 * i + 1];
    s2 += o[3 * i + 2];
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  red[2][threadIdx.x] = s2;
  __syncthreads();
  for (int s = kTaThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  const double c0 = red[0][0] / n_cams, c1 = red[1][0] / n_cams, c2 = red[2][0] / n_cams;
  __syncthreads();
  double sn = 0.0;
  for (int i = threadIdx.x; i < n_cams; i += kTaThreads) {
    const double d0 = o[3 * i] - c0, d1 = o[3 * i + 1] - c1, d2 = o[3 * i + 2] - c2;
    sn += sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  }
  red[0][threadIdx.x] = sn;
  __syncthreads();
  for (int s = kTaThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[0][threadIdx.x] += red[0][threadIdx.x + s];
    __syncthreads();
  }
  const double scale = red[0][0] / n_cams;
  if (!(scale > 0.0)) {
    if (threadIdx.x == 0) *err = 1;
    return;
  }
  for (int i = threadIdx.x; i < n_cams; i += kTaThreads) {
    o[3 * i] = (o[3 * i] - c0) / scale;
    o[3 * i + 1] = (o[3 * i + 1] - c1) / scale;
    o[3 * i + 2] = (o[3 * i + 2] - c2) / scale;
  }
}

// L1 term of every (run, pair).
__global__ void k_ta_pair_loss(int runs, int n_cams, int64_t n_pairs, const int32_t* __restrict__ pair_i,
                               const int32_t* __restrict__ pair_j, const double* __restrict__ target,
                               const double* __restrict__ o_all, double* __restrict__ pair_loss) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)runs * n_pairs) return;
  const int64_t r = idx / n_pairs, q = idx - r * n_pairs;
  const double* o = o_all + r * n_cams * 3;
  const int i = pair_i[q], j = pair_j[q];
  const double d0 = o[3 * j] - o[3 * i], d1 = o[3 * j + 1] - o[3 * i + 1], d2 = o[3 * j + 2] - o[3 * i + 2];
  const double nd = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  double l = 0.0;
  if (nd > 0.0) {
    l += fabs(d0 / nd - target[3 * q]);
    l += fabs(d1 / nd - target[3 * q + 1]);
    l += fabs(d2 / nd - target[3 * q + 2]);
  }
  pair_loss[idx] = l;
}

// Mean pair loss of every (run, camera), summed in pair order.
__global__ void k_ta_cam_loss(int runs, int n_cams, int64_t n_pairs, const int32_t* __restrict__ cam_off,
                              const int32_t* __restrict__ cam_ent, const double* __restrict__ pair_loss,
                              double* __restrict__ cam_loss) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)runs * n_cams) return;
  const int64_t r = idx / n_cams;
  const int c = (int)(idx - r * n_cams);
  double s = 0.0;
  for (int e = cam_off[c]; e < cam_off[c + 1]; ++e) s += pair_loss[r * n_pairs + (cam_ent[e] >> 1)];
  const int deg = cam_off[c + 1] - cam_off[c];
  cam_loss[idx] = deg ? s / (double)deg : 0.0;
}

// One workgroup per run: L_t = sum of the pair terms / |P|.
__global__ __launch_bounds__(kTaThreads) void k_ta_run_loss(int64_t n_pairs, const double* __restrict__ pair_loss,
                                                            double* __restrict__ run_loss) {
  __shared__ double red[kTaThreads];
  const double* pl = pair_loss + (int64_t)blockIdx.x * n_pairs;
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < n_pairs; q += kTaThreads) s += pl[q];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = kTaThreads / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) run_loss[blockIdx.x] = n_pairs > 0 ? red[0] / (double)n_pairs : 0.0;
}

// Per camera: the run with the lowest mean loss (ties: the lower run).
__global__ void k_ta_merge(int runs, int n_cams, const double* __restrict__ o_runs,
                           const double* __restrict__ cam_loss, double* __restrict__ o_out,
                           int32_t* __restrict__ run_of_cam) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cams) return;
  int b = 0;
  for (int r = 1; r < runs; ++r)
    if (cam_loss[(int64_t)r * n_cams + c] < cam_loss[(int64_t)b * n_cams + c]) b = r;
  run_of_cam[c] = b;
  for (int k = 0; k < 3; ++k) o_out[3 * c + k] = o_runs[((int64_t)b * n_cams + c) * 3 + k];
}

unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

}  // namespace

hipError_t launch_rt_pairs(hipStream_t st, int64_t n_pairs, const int32_t* pair_i, const int32_t* pair_j,
                           const double* R, const double* f, const double* cx, const double* cy, float* rowf,
                           double* rowd) {
  if (n_pairs == 0) return hipSuccess;
  k_rt_pairs<<<blocks_for(n_pairs, 256), 256, 0, st>>>(n_pairs, pair_i, pair_j, R, f, cx, cy, rowf, rowd);
  return hipGetLastError();
}

template <bool CAP>
hipError_t launch_rt_score_t(hipStream_t st, int64_t n_items, int n_groups, const int4* items, const float* rowf,
                             const float* x1, const float* y1, const float* x2, const float* y2, const float* cand,
                             int kp, float tau, float* partial, hipEvent_t ev0, hipEvent_t ev1) {
  const dim3 grid((unsigned)(n_items * n_groups)), block(kRtThreads);
  if (ev0)
    hipExtLaunchKernelGGL(k_rt_score<CAP>, grid, block, 0, st, ev0, ev1, 0, items, n_groups, rowf, x1, y1, x2, y2,
                          cand, kp, tau, partial);
  else
    k_rt_score<CAP><<<grid, block, 0, st>>>(items, n_groups, rowf, x1, y1, x2, y2, cand, kp, tau, partial);
  return hipGetLastError();
}

hipError_t launch_rt_score(hipStream_t st, int64_t n_items, int n_groups, const int4* items, const float* rowf,
                           const float* x1, const float* y1, const float* x2, const float* y2, const float* cand,
                           int kp, double tau, float* partial, hipEvent_t ev0, hipEvent_t ev1) {
  if (n_items == 0) return hipSuccess;
  if (std::isinf(tau))
    return launch_rt_score_t<false>(st, n_items, n_groups, items, rowf, x1, y1, x2, y2, cand, kp, 0.f, partial, ev0,
                                    ev1);
  return launch_rt_score_t<true>(st, n_items, n_groups, items, rowf, x1, y1, x2, y2, cand, kp, (float)tau, partial,
                                 ev0, ev1);
}

hipError_t launch_rt_select(hipStream_t st, int64_t n_pairs, int k, int kp, double tau, const int32_t* pair_item_off,
                            const int4* items, const float* partial, const float* cand, const double* rowd,
                            const float* x1, const float* y1, const float* x2, const float* y2, float* scores,
                            int32_t* best, int32_t* vote, double* t_rel, double* score_best) {
  if (n_pairs == 0) return hipSuccess;
  k_rt_select<<<(unsigned)n_pairs, kRtThreads, 0, st>>>(k, kp, tau, pair_item_off, items, partial, cand, rowd, x1, y1,
                                                        x2, y2, scores, best, vote, t_rel, score_best);
  return hipGetLastError();
}

hipError_t launch_ta_targets(hipStream_t st, int64_t n_pairs, const int32_t* pair_j, const double* R,
                             const double* t_rel, double* target) {
  if (n_pairs == 0) return hipSuccess;
  k_ta_targets<<<blocks_for(n_pairs, 256), 256, 0, st>>>(n_pairs, pair_j, R, t_rel, target);
  return hipGetLastError();
}

hipError_t launch_ta_counters(hipStream_t st, TaCounters* ctr, double lr) {
  k_ta_counters<<<1, 1, 0, st>>>(ctr, lr);
  return hipGetLastError();
}

hipError_t launch_ta_step(hipStream_t st, int runs, int n_cams, int64_t n_pairs, const int32_t* cam_off,
                          const int32_t* cam_ent, const int32_t* ent_other, const double* target, const double* o_in,
                          double* o_out, double* m, double* v, TaCounters* ctr, int parity, double beta1,
                          double beta2, double eps, double decay) {
  k_ta_step<<<blocks_for((int64_t)runs * n_cams, kTaThreads / 64), kTaThreads, 0, st>>>(
      runs, n_cams, n_pairs, cam_off, cam_ent, ent_other, target, o_in, o_out, m, v, ctr, parity, beta1, beta2, eps,
      decay);
  return hipGetLastError();
}

hipError_t launch_ta_align(hipStream_t st, int runs, int n_cams, double* o, int32_t* err) {
  k_ta_align<<<runs, kTaThreads, 0, st>>>(n_cams, o, err);
  return hipGetLastError();
}

hipError_t launch_ta_losses(hipStream_t st, int runs, int n_cams, int64_t n_pairs, const int32_t* cam_off,
                            const int32_t* cam_ent, const int32_t* pair_i, const int32_t* pair_j,
                            const double* target, const double* o, double* pair_loss, double* cam_loss,
                            double* run_loss) {
  if (n_pairs > 0)
    k_ta_pair_loss<<<blocks_for((int64_t)runs * n_pairs, 256), 256, 0, st>>>(runs, n_cams, n_pairs, pair_i, pair_j,
                                                                             target, o, pair_loss);
  if (cam_loss)
    k_ta_cam_loss<<<blocks_for((int64_t)runs * n_cams, 256), 256, 0, st>>>(runs, n_cams, n_pairs, cam_off, cam_ent,
                                                                           pair_loss, cam_loss);
  k_ta_run_loss<<<runs, kTaThreads, 0, st>>>(n_pairs, pair_loss, run_loss);
  return hipGetLastError();
}

hipError_t launch_ta_merge(hipStream_t st, int runs, int n_cams, const double* o_runs, const double* cam_loss,
                           double* o_out, int32_t* run_of_cam) {
  k_ta_merge<<<blocks_for(n_cams, 256), 256, 0, st>>>(runs, n_cams, o_runs, cam_loss, o_out, run_of_cam);
  return hipGetLastError();
}

}  // namespace fea
