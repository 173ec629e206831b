// Global rotation (Method > Global Rotation, Eq. fastmap-rotation-objective).
//
// Initialisation (after Martinec and Pajdla, as the paper modifies it): the
// first columns c1 minimise sum |c1_j - R^{i->j} c1_i|^2 over unit-norm
// stacked vectors, i.e. the smallest eigenvector of the 3N x 3N normal matrix
// M; the second columns do the same for M/|P| + B/|I| (B the orthogonality
// penalty diag(c1_i c1_i^T)).  Both by power iteration on sigma I - A with
// sigma just above half of A's Gershgorin bound (so the smallest eigenvalues
// of A dominate): one wave per camera applies A over the camera's pairs
// (no atomics); one workgroup renormalises every 8th step.  Without noise the smallest
// eigenvalue of M has the three columns of the true rotations (times any
// fixed vector) as eigenvectors, a three-dimensional space; any vector in it
// is a valid first column.
//
// Optimisation: Adam on the 6D parameters of the mean geodesic distance
// d(R_j, R^{i->j} R_i) = arccos((tr(R_j^T R^{i->j} R_i) - 1)/2); one wave per
// camera sums its pairs' gradients (rotations rebuilt from the 6D parameters
// per pair), the 6D backward and the Adam step follow.  fp64 throughout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fea_device.h"
#include "fea_rotation.h"

namespace fea {
namespace {

constexpr int kRaThreads = 256;
constexpr int kRaWaves = kRaThreads / 64;

// y_w = s (sigma c_w - wm (M c)_w - wp c1_w (c1_w . c_w)) for camera w, with
// (M c)_w = sum over its pairs of r (as camera j) or -R^T r (as camera i),
// r = c_j - R^{i->j} c_i; s = the last renormalisation's 1/|c| on the step
// right after it, 1 on the others (scale == nullptr).
template <bool PEN>
__global__ __launch_bounds__(kRaThreads) void k_ra_apply(int n_cams, const int32_t* __restrict__ cam_off,
                                                         const int32_t* __restrict__ cam_ent,
                                                         const int32_t* __restrict__ pair_i,
                                                         const int32_t* __restrict__ pair_j,
                                                         const double* __restrict__ Rrel,
                                                         const double* __restrict__ c_in,
                                                         const double* __restrict__ scale,
                                                         const double* __restrict__ c1, double sigma, double wm,
                                                         double wp, double* __restrict__ c_out,
                                                         double* __restrict__ sq) {  // [3 n_cams]: y.y, c.y, c.c
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * kRaWaves + (threadIdx.x >> 6);
  if (w >= n_cams) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int e = cam_off[w] + lane; e < cam_off[w + 1]; e += 64) {
    const int ent = cam_ent[e];
    const int64_t q = ent >> 1;
    const int i = pair_i[q], j = pair_j[q];
    const double* R = Rrel + 9 * q;
    const double ci[3] = {c_in[3 * i], c_in[3 * i + 1], c_in[3 * i + 2]};
    double r[3];
    for (int a = 0; a < 3; ++a) r[a] = c_in[3 * j + a] - (R[3 * a] * ci[0] + R[3 * a + 1] * ci[1] + R[3 * a + 2] * ci[2]);
    if (ent & 1) {
      for (int a = 0; a < 3; ++a) acc[a] += r[a];
    } else {
      for (int a = 0; a < 3; ++a) acc[a] -= R[a] * r[0] + R[3 + a] * r[1] + R[6 + a] * r[2];
    }
  }
  wave_sum_f64_multi(acc);
  if (lane != 0) return;
  const double s = scale ? *scale : 1.0;
  const double cw[3] = {c_in[3 * w], c_in[3 * w + 1], c_in[3 * w + 2]};
  double y[3];
  for (int a = 0; a < 3; ++a) y[a] = s * (sigma * cw[a] - wm * acc[a]);
  if (PEN) {
    const double* u = c1 + 3 * w;
    const double d = u[0] * cw[0] + u[1] * cw[1] + u[2] * cw[2];
    for (int a = 0; a < 3; ++a) y[a] -= s * wp * u[a] * d;
  }
  for (int a = 0; a < 3; ++a) c_out[3 * w + a] = y[a];
  sq[w] = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
  sq[n_cams + w] = cw[0] * y[0] + cw[1] * y[1] + cw[2] * y[2];
  sq[2 * n_cams + w] = cw[0] * cw[0] + cw[1] * cw[1] + cw[2] * cw[2];
}

// scale = 1 / sqrt(sum of y.y) (fixed-order block sums; 0 marks a zero
// vector) and the Rayleigh quotient of A at the step's input c:
// c.Ac / c.c = sigma - (c.y) / (s c.c), y = s (sigma c - A c), s the step's
// input scale; written to rho[0].
__global__ __launch_bounds__(kRaThreads) void k_ra_norm(int n, const double* __restrict__ sq, double sigma,
                                                        double s_in, double* __restrict__ scale,
                                                        double* __restrict__ rho) {
  __shared__ double red[3][kRaThreads];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < n; k += kRaThreads) {
    a += sq[k];
    b += sq[n + k];
    c += sq[2 * n + k];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int o = kRaThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *scale = red[0][0] > 0.0 ? 1.0 / sqrt(red[0][0]) : 0.0;
    if (rho) *rho = red[2][0] > 0.0 ? sigma - red[1][0] / (s_in * red[2][0]) : 0.0;
  }
}

// Per camera: c1 = c/|c|; or, with c1 given, the second column: c minus its
// component along c1, normalised, and the 6D parameters (c1, c2).
__global__ void k_ra_columns(int n_cams, const double* __restrict__ c, const double* __restrict__ c1,
                             double* __restrict__ out, int32_t* __restrict__ err) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n_cams) return;
  double v[3] = {c[3 * w], c[3 * w + 1], c[3 * w + 2]};
  if (c1) {
    const double* u = c1 + 3 * w;
    const double d = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
    for (int a = 0; a < 3; ++a) v[a] -= d * u[a];
  }
  const double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  if (!(n > 0.0)) {
    *err = 1;
    return;
  }
  if (c1) {
    for (int a = 0; a < 3; ++a) {
      out[6 * w + a] = c1[3 * w + a];
      out[6 * w + 3 + a] = v[a] / n;
    }
  } else {
    for (int a = 0; a < 3; ++a) out[3 * w + a] = v[a] / n;
  }
}

// One Adam step on the 6D parameters of every camera.
__global__ __launch_bounds__(kRaThreads) void k_ra_step(int n_cams, int64_t n_pairs, const int32_t* __restrict__ cam_off,
                                                        const int32_t* __restrict__ cam_ent,
                                                        const int32_t* __restrict__ pair_i,
                                                        const int32_t* __restrict__ pair_j,
                                                        const double* __restrict__ Rrel,
                                                        const double* __restrict__ a_in, double* __restrict__ a_out,
                                                        double* __restrict__ m, double* __restrict__ v,
                                                        TaCounters* ctr, int p, double beta1, double beta2,
                                                        double eps, double decay) {
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * kRaWaves + (threadIdx.x >> 6);
  const double lr = ctr->lr[p];
  const double b1t = ctr->b1t[p] * beta1, b2t = ctr->b2t[p] * beta2;
  if (w == 0 && lane == 0) {  // the other parity's slot: read by the next step only
    ctr->lr[p ^ 1] = lr * decay;
    ctr->b1t[p ^ 1] = b1t;
    ctr->b2t[p ^ 1] = b2t;
  }
  if (w >= n_cams) return;
  const double inv_np = 1.0 / (double)n_pairs;
  double G[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int e = cam_off[w] + lane; e < cam_off[w + 1]; e += 64) {
    const int ent = cam_ent[e];
    const int64_t q = ent >> 1;
    const double* R = Rrel + 9 * q;
    double Ri[9], Rj[9], T[9];
    rot6d_forward(a_in + 6 * (int64_t)pair_i[q], Ri);
    rot6d_forward(a_in + 6 * (int64_t)pair_j[q], Rj);
    for (int a = 0; a < 3; ++a)  // T = R^{i->j} R_i, the prediction of R_j
      for (int b = 0; b < 3; ++b) T[3 * a + b] = R[3 * a] * Ri[b] + R[3 * a + 1] * Ri[3 + b] + R[3 * a + 2] * Ri[6 + b];
    double tr = 0.0;
    for (int k = 0; k < 9; ++k) tr += Rj[k] * T[k];
    const double x = 0.5 * (tr - 1.0);
    if (!(fabs(x) < 1.0)) continue;
    const double h = -0.5 * inv_np / sqrt(1.0 - x * x);  // d arccos(x)/d tr, over |P|
    if (ent & 1) {
      for (int k = 0; k < 9; ++k) G[k] += h * T[k];
    } else {  // d tr / d R_i = R^{i->j T} R_j
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) G[3 * a + b] += h * (R[a] * Rj[b] + R[3 + a] * Rj[3 + b] + R[6 + a] * Rj[6 + b]);
    }
  }
  wave_sum_f64_multi(G);
  if (lane >= 6) return;
  double ga[6];
  rot6d_vjp(a_in + 6 * (int64_t)w, G, ga);
  double gk = ga[0];
  for (int k = 1; k < 6; ++k)
    if (lane == k) gk = ga[k];
  const int64_t idx = 6 * (int64_t)w + lane;
  const double mk = beta1 * m[idx] + (1.0 - beta1) * gk;
  const double vk = beta2 * v[idx] + (1.0 - beta2) * gk * gk;
  m[idx] = mk;
  v[idx] = vk;
  a_out[idx] = a_in[idx] - lr * (mk / (1.0 - b1t)) / (sqrt(vk / (1.0 - b2t)) + eps);
}

// Mean geodesic distance over the pairs (argument clamped to [-1, 1]).
__global__ __launch_bounds__(kRaThreads) void k_ra_loss(int64_t n_pairs, const int32_t* __restrict__ pair_i,
                                                        const int32_t* __restrict__ pair_j,
                                                        const double* __restrict__ Rrel,
                                                        const double* __restrict__ a6, double* __restrict__ loss) {
  __shared__ double red[kRaThreads];
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < n_pairs; q += kRaThreads) {
    const double* R = Rrel + 9 * q;
    double Ri[9], Rj[9];
    rot6d_forward(a6 + 6 * (int64_t)pair_i[q], Ri);
    rot6d_forward(a6 + 6 * (int64_t)pair_j[q], Rj);
    double tr = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        tr += Rj[3 * a + b] * (R[3 * a] * Ri[b] + R[3 * a + 1] * Ri[3 + b] + R[3 * a + 2] * Ri[6 + b]);
    double x = 0.5 * (tr - 1.0);
    x = x < -1.0 ? -1.0 : (x > 1.0 ? 1.0 : x);
    s += acos(x);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kRaThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (double)n_pairs;
}

__global__ void k_ra_to_R(int n_cams, const double* __restrict__ a6, double* __restrict__ R) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < n_cams) rot6d_forward(a6 + 6 * (int64_t)w, R + 9 * (int64_t)w);
}

unsigned wave_blocks(int n) { return (unsigned)((n + kRaWaves - 1) / kRaWaves); }

}  // namespace

hipError_t launch_ra_apply(hipStream_t st, int n_cams, const int32_t* cam_off, const int32_t* cam_ent,
                           const int32_t* pair_i, const int32_t* pair_j, const double* Rrel, const double* c_in,
                           const double* scale, const double* c1, double sigma, double wm, double wp, double* c_out,
                           double* sq, double* scale_out, bool renorm, double* rho) {
  if (c1)
    k_ra_apply<true><<<wave_blocks(n_cams), kRaThreads, 0, st>>>(n_cams, cam_off, cam_ent, pair_i, pair_j, Rrel, c_in,
                                                                 scale, c1, sigma, wm, wp, c_out, sq);
  else
    k_ra_apply<false><<<wave_blocks(n_cams), kRaThreads, 0, st>>>(n_cams, cam_off, cam_ent, pair_i, pair_j, Rrel,
                                                                  c_in, scale, nullptr, sigma, wm, wp, c_out, sq);
  // the input scale of a renormalising step is 1 (it never follows one)
  if (renorm) k_ra_norm<<<1, kRaThreads, 0, st>>>(n_cams, sq, sigma, 1.0, scale_out, rho);
  return hipGetLastError();
}

hipError_t launch_ra_columns(hipStream_t st, int n_cams, const double* c, const double* c1, double* out,
                             int32_t* err) {
  k_ra_columns<<<(n_cams + 255) / 256, 256, 0, st>>>(n_cams, c, c1, out, err);
  return hipGetLastError();
}

hipError_t launch_ra_step(hipStream_t st, int n_cams, int64_t n_pairs, const int32_t* cam_off, const int32_t* cam_ent,
                          const int32_t* pair_i, const int32_t* pair_j, const double* Rrel, const double* a_in,
                          double* a_out, double* m, double* v, TaCounters* ctr, int parity, double beta1,
                          double beta2, double eps, double decay) {
  k_ra_step<<<wave_blocks(n_cams), kRaThreads, 0, st>>>(n_cams, n_pairs, cam_off, cam_ent, pair_i, pair_j, Rrel, a_in,
                                                        a_out, m, v, ctr, parity, beta1, beta2, eps, decay);
  return hipGetLastError();
}

hipError_t launch_ra_loss(hipStream_t st, int64_t n_pairs, const int32_t* pair_i, const int32_t* pair_j,
                          const double* Rrel, const double* a6, double* loss) {
  k_ra_loss<<<1, kRaThreads, 0, st>>>(n_pairs, pair_i, pair_j, Rrel, a6, loss);
  return hipGetLastError();
}

hipError_t launch_ra_to_R(hipStream_t st, int n_cams, const double* a6, double* R) {
  k_ra_to_R<<<(n_cams + 255) / 256, 256, 0, st>>>(n_cams, a6, R);
  return hipGetLastError();
}

}  // namespace fea
