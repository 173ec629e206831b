// Focal-length vote (Method > Focal Length Estimation, Eq. fastmap-focal-vote).
//
// A 3x3 matrix is an essential matrix exactly when its two non-zero singular
// values are equal, so a candidate focal length f is scored by
//   v(f) = sum over pairs of exp((1 - s1/s2) / tau),
// s1 >= s2 the two largest singular values of E = K_j^T F K_i with
// K = diag(f, f, 1) in centred pixel coordinates.  Per intrinsics group g the
// group's cameras take the candidate and every other camera keeps its
// group's current focal length; with one group this is the shared-intrinsics
// vote.  One wave per (group, 64 candidates): each lane holds one candidate
// and walks the group's pairs in pair order with the rest of the wave (the
// pair's data is the same for every lane), so every lane works and the sum
// of each candidate is a plain serial one (no atomics).  The singular
// values come from the eigenvalues of the symmetric E^T E in closed form
// (the trigonometric solution of its characteristic cubic), all in fp64:
// the work is tiny (pairs x candidates 3x3 problems) and latency-bound.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fea_focal.h"

namespace fea {
namespace {

constexpr int kFvThreads = 256;

// s1 / s2 of a 3x3 matrix from the eigenvalues e1 >= e2 >= e3 of M = E^T E:
// with q = tr(M)/3 and p^2 = |M - qI|_F^2 / 6, the eigenvalues of
// B = (M - qI)/p are 2 cos(phi + 2 pi k/3) with cos(3 phi) = det(B)/2.
// Infinite when s2 = 0 (rank below 2).
__device__ double sv_ratio(const double E[9]) {
  const double m00 = E[0] * E[0] + E[3] * E[3] + E[6] * E[6];
  const double m11 = E[1] * E[1] + E[4] * E[4] + E[7] * E[7];
  const double m22 = E[2] * E[2] + E[5] * E[5] + E[8] * E[8];
  const double m01 = E[0] * E[1] + E[3] * E[4] + E[6] * E[7];
  const double m02 = E[0] * E[2] + E[3] * E[5] + E[6] * E[8];
  const double m12 = E[1] * E[2] + E[4] * E[5] + E[7] * E[8];
  const double q = (m00 + m11 + m22) / 3.0;
  const double a = m00 - q, b = m11 - q, c = m22 - q;
  const double p2 = (a * a + b * b + c * c + 2.0 * (m01 * m01 + m02 * m02 + m12 * m12)) / 6.0;
  if (!(q > 0.0)) return INFINITY;
  if (!(p2 > 0.0)) return 1.0;  // M = qI: all singular values equal
  const double p = sqrt(p2);
  const double det = a * (b * c - m12 * m12) - m01 * (m01 * c - m12 * m02) + m02 * (m01 * m12 - b * m02);
  double r = det / (2.0 * p2 * p);
  r = r < -1.0 ? -1.0 : (r > 1.0 ? 1.0 : r);
  const double phi = acos(r) / 3.0;
  const double e1 = q + 2.0 * p * cos(phi);
  const double e3 = q + 2.0 * p * cos(phi + 2.0943951023931957);  // + 2 pi / 3
  const double e2 = 3.0 * q - e1 - e3;
  if (!(e2 > 0.0)) return INFINITY;
  return sqrt(e1 / e2);
}

__global__ __launch_bounds__(kFvThreads) void k_fv_vote(int n_groups, int n_cand, const int32_t* __restrict__ grp_off,
                                                        const int32_t* __restrict__ grp_pairs,
                                                        const int32_t* __restrict__ pair_i,
                                                        const int32_t* __restrict__ pair_j,
                                                        const int32_t* __restrict__ group,
                                                        const double* __restrict__ F,
                                                        const double* __restrict__ f_cur,
                                                        const double* __restrict__ cand, double inv_tau,
                                                        double* __restrict__ votes) {
  const int lane = threadIdx.x & 63;
  const int nb = (n_cand + 63) >> 6;
  const int64_t w = (int64_t)blockIdx.x * (kFvThreads / 64) + (threadIdx.x >> 6);
  if (w >= (int64_t)n_groups * nb) return;
  const int g = (int)(w / nb), k = (int)(w - (int64_t)g * nb) * 64 + lane;
  const double f = cand[k < n_cand ? k : n_cand - 1];
  double s = 0.0;
  for (int e = grp_off[g]; e < grp_off[g + 1]; ++e) {  // the pair is the same for the whole wave
    const int p = grp_pairs[e];
    const int i = pair_i[p], j = pair_j[p];
    const int gi = group[i], gj = group[j];
    const double fi = gi == g ? f : f_cur[gi];
    const double fj = gj == g ? f : f_cur[gj];
    const double si[3] = {fi, fi, 1.0}, sj[3] = {fj, fj, 1.0};
    const double* Fp = F + 9 * (int64_t)p;
    double E[9];
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) E[3 * r + cc] = sj[r] * Fp[3 * r + cc] * si[cc];
    s += exp((1.0 - sv_ratio(E)) * inv_tau);
  }
  if (k < n_cand) votes[(int64_t)g * n_cand + k] = s;
}

// Per group: the candidate with the highest vote (ties: the lower index).
__global__ __launch_bounds__(kFvThreads) void k_fv_best(int n_cand, const double* __restrict__ votes,
                                                        const double* __restrict__ cand, double* __restrict__ f_best,
                                                        int32_t* __restrict__ k_best) {
  __shared__ double sv[kFvThreads];
  __shared__ int si[kFvThreads];
  const double* v = votes + (int64_t)blockIdx.x * n_cand;
  double bv = 0.0;
  int bk = -1;
  for (int k = threadIdx.x; k < n_cand; k += kFvThreads)
    if (bk < 0 || v[k] > bv) {
      bv = v[k];
      bk = k;
    }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bk;
  __syncthreads();
  for (int s = kFvThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const int k2 = si[threadIdx.x + s], k1 = si[threadIdx.x];
      const double v2 = sv[threadIdx.x + s];
      if (k2 >= 0 && (k1 < 0 || v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && k2 < k1))) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = k2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    f_best[blockIdx.x] = cand[si[0]];
    k_best[blockIdx.x] = si[0];
  }
}

}  // namespace

hipError_t launch_fv_vote(hipStream_t st, int n_groups, int n_cand, const int32_t* grp_off, const int32_t* grp_pairs,
                          const int32_t* pair_i, const int32_t* pair_j, const int32_t* group, const double* F,
                          const double* f_cur, const double* cand, double tau, double* votes, hipEvent_t ev0,
                          hipEvent_t ev1) {
  const int64_t waves = (int64_t)n_groups * ((n_cand + 63) / 64);
  const dim3 grid((unsigned)((waves + kFvThreads / 64 - 1) / (kFvThreads / 64))), block(kFvThreads);
  if (ev0)
    hipExtLaunchKernelGGL(k_fv_vote, grid, block, 0, st, ev0, ev1, 0, n_groups, n_cand, grp_off, grp_pairs, pair_i,
                          pair_j, group, F, f_cur, cand, 1.0 / tau, votes);
  else
    k_fv_vote<<<grid, block, 0, st>>>(n_groups, n_cand, grp_off, grp_pairs, pair_i, pair_j, group, F, f_cur, cand,
                                      1.0 / tau, votes);
  return hipGetLastError();
}

hipError_t launch_fv_best(hipStream_t st, int n_groups, int n_cand, const double* votes, const double* cand,
                          double* f_best, int32_t* k_best) {
  k_fv_best<<<n_groups, kFvThreads, 0, st>>>(n_cand, votes, cand, f_best, k_best);
  return hipGetLastError();
}

}  // namespace fea
