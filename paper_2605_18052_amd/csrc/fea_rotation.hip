// Global rotation (Method > Global Rotation, Eq. fastmap-rotation-objective).
//
// Initialisation (after Martinec and Pajdla, as the paper modifies it): the
// first columns c1 minimise sum |c1_j - R^{i->j} c1_i|^2 over unit-norm
// stacked vectors, i.e. the smallest eigenvector of the 3N x 3N normal matrix
// M; the second columns do the same for M/|P| + B/|I| (B the orthogonality
// penalty diag(c1_i c1_i^T)).  Both by the Lanczos method with full
// reorthogonalisation (classical Gram-Schmidt, twice) from the caller's
// start vector, in fp64: one wave per camera applies A over the camera's
// pairs (no atomics), one workgroup per basis vector forms the projections,
// one thread per coordinate subtracts them; the host takes the smallest
// eigenvalue of the small tridiagonal matrix (bisection on Sturm counts)
// every 16 steps, stops once it settles, and the Ritz vector is formed on
// the device.  The Krylov space converges to the bottom of the spectrum in
// about the square root of the steps power iteration needs.  Without noise
// the smallest eigenvalue of M has the three columns of the true rotations
// (times any fixed vector) as eigenvectors, a three-dimensional space; any
// vector in it is a valid first column.
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
// r = c_j - R^{i->j} c_i; s = *scale (1 when scale is null); sq receives the
// per-camera y.y, c.y and c.c.
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
  wave_sum_f64_scatter(acc);
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
  // this camera's parameters and optimiser state (lanes 0..5), loaded
  // before the pair loop so that they arrive meanwhile
  const int64_t idx = 6 * (int64_t)w + (lane < 6 ? lane : 0);
  double a_cur[6], m_old = 0.0, v_old = 0.0;
  for (int k = 0; k < 6; ++k) a_cur[k] = a_in[6 * (int64_t)w + k];
  if (lane < 6) {
    m_old = m[idx];
    v_old = v[idx];
  }
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
  wave_sum_f64_scatter(G);
  if (lane >= 6) return;
  double ga[6];
  rot6d_vjp(a_cur, G, ga);
  double gk = ga[0], ak = a_cur[0];
  for (int k = 1; k < 6; ++k)
    if (lane == k) {
      gk = ga[k];
      ak = a_cur[k];
    }
  const double mk = beta1 * m_old + (1.0 - beta1) * gk;
  const double vk = beta2 * v_old + (1.0 - beta2) * gk * gk;
  m[idx] = mk;
  v[idx] = vk;
  a_out[idx] = ak - lr * (mk / (1.0 - b1t)) / (sqrt(vk / (1.0 - b2t)) + eps);
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

// ---- Lanczos with full reorthogonalisation ---------------------------------
// The basis V is row-major [m][n]: row i is the i-th Lanczos vector in the
// camera-major layout (3 entries per camera).
constexpr int kLzThreads = 256;
constexpr int kLzOrthThreads = 64;  // coordinates per workgroup of k_lz_orth (one per lane)
constexpr int kLzOrthWaves = 16;    // wavefronts per workgroup, each a slice of the basis

// h[i] = V_i . w, one workgroup per basis vector (fixed-order sums).
__global__ __launch_bounds__(kLzThreads) void k_lz_dots(int64_t n, const double* __restrict__ V,
                                                        const double* __restrict__ w, double* __restrict__ h) {
  __shared__ double red[kLzThreads];
  const double* v = V + (int64_t)blockIdx.x * n;
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += kLzThreads) s = fma(v[k], w[k], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kLzThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) h[blockIdx.x] = red[0];
}

// w -= sum over i < m of h[i] V_i.  A workgroup takes 64 coordinates (one
// per lane) and splits the basis over its 16 wavefronts (wavefront q sums
// rows q, q + 16, ...), so a pass over an m x n basis runs on 16 n / 64
// wavefronts instead of n / 64; the 16 partial sums are added in LDS in a
// fixed order.  part[block] = the block's sum of w^2 after the subtraction.
__global__ __launch_bounds__(kLzOrthThreads * kLzOrthWaves) void k_lz_orth(int64_t n, int m,
                                                                          const double* __restrict__ V,
                                                                          const double* __restrict__ h,
                                                                          double* __restrict__ w,
                                                                          double* __restrict__ part) {
  __shared__ double s_acc[kLzOrthWaves][kLzOrthThreads];
  const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int64_t k = (int64_t)blockIdx.x * kLzOrthThreads + lane;
  double acc = 0.0;
  if (k < n)
    for (int i = q; i < m; i += kLzOrthWaves) acc = fma(h[i], V[(int64_t)i * n + k], acc);
  s_acc[q][lane] = acc;
  __syncthreads();
  if (q == 0) {
    double x = 0.0;
    if (k < n) {
      double sub = 0.0;
#pragma unroll
      for (int r = 0; r < kLzOrthWaves; ++r) sub += s_acc[r][lane];
      x = w[k] - sub;
      w[k] = x;
    }
    const double sq = wave_sum_f64(x * x);
    if (lane == 0) part[blockIdx.x] = sq;
  }
}

// beta[j] = |w| (the parts summed in order), alpha[j] = h1[j] + h2[j] (the
// coefficient of V_j over both passes), V_{j+1} = w / beta[j] (zero when
// the Krylov space is exhausted).
__global__ __launch_bounds__(1024) void k_lz_next(int64_t n, int nparts, const double* __restrict__ part,
                                                  const double* __restrict__ h1, const double* __restrict__ h2, int j,
                                                  const double* __restrict__ w, double* __restrict__ vnext,
                                                  double* __restrict__ alpha, double* __restrict__ beta) {
  __shared__ double s_beta;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < nparts; ++q) t += part[q];
    const double b = sqrt(t);
    s_beta = b;
    beta[j] = b;
    alpha[j] = h1[j] + h2[j];
  }
  __syncthreads();
  const double inv = s_beta > 0.0 ? 1.0 / s_beta : 0.0;
  for (int64_t k = threadIdx.x; k < n; k += 1024) vnext[k] = w[k] * inv;
}

// y = sum over i < m of s[i] V_i (the Ritz vector), one thread per coordinate.
__global__ void k_lz_combine(int64_t n, int m, const double* __restrict__ V, const double* __restrict__ s,
                             double* __restrict__ y) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double x = 0.0;
  for (int i = 0; i < m; ++i) x = fma(s[i], V[(int64_t)i * n + k], x);
  y[k] = x;
}

unsigned wave_blocks(int n) { return (unsigned)((n + kRaWaves - 1) / kRaWaves); }

}  // namespace

int lz_orth_blocks(int64_t n) { return (int)((n + kLzOrthThreads - 1) / kLzOrthThreads); }

hipError_t launch_lz_step(hipStream_t st, int n_cams, const int32_t* cam_off, const int32_t* cam_ent,
                          const int32_t* pair_i, const int32_t* pair_j, const double* Rrel, const double* c1, double wm,
                          double wp, double* V, int j, double* w, double* sq, double* h1, double* h2, double* part,
                          double* alpha, double* beta) {
  const int64_t n = (int64_t)3 * n_cams;
  const double* vj = V + (int64_t)j * n;
  // w = A v_j: the operator kernel with sigma = 0 and negated weights
  if (c1)
    k_ra_apply<true><<<wave_blocks(n_cams), kRaThreads, 0, st>>>(n_cams, cam_off, cam_ent, pair_i, pair_j, Rrel, vj,
                                                                 nullptr, c1, 0.0, -wm, -wp, w, sq);
  else
    k_ra_apply<false><<<wave_blocks(n_cams), kRaThreads, 0, st>>>(n_cams, cam_off, cam_ent, pair_i, pair_j, Rrel,
                                                                  vj, nullptr, nullptr, 0.0, -wm, -wp, w, sq);
  const int m = j + 1;
  const int nb = lz_orth_blocks(n);
  k_lz_dots<<<m, kLzThreads, 0, st>>>(n, V, w, h1);
  k_lz_orth<<<nb, kLzOrthThreads * kLzOrthWaves, 0, st>>>(n, m, V, h1, w, part);
  k_lz_dots<<<m, kLzThreads, 0, st>>>(n, V, w, h2);
  k_lz_orth<<<nb, kLzOrthThreads * kLzOrthWaves, 0, st>>>(n, m, V, h2, w, part);
  k_lz_next<<<1, 1024, 0, st>>>(n, nb, part, h1, h2, j, w, V + (int64_t)m * n, alpha, beta);
  return hipGetLastError();
}

hipError_t launch_lz_combine(hipStream_t st, int64_t n, int m, const double* V, const double* s, double* y) {
  k_lz_combine<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, m, V, s, y);
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
