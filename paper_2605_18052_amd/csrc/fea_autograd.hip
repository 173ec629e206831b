// Objective and adjoint at parameters held by the caller (device arrays), for
// use behind an autograd function: the forward builds the poses from the 6D
// rotations, translations and log focal lengths and streams the matches
// (loss only); the backward recomputes the forward and runs the same
// residual/gradient and per-camera adjoint kernels as the solver's own step,
// then the 6D-rotation and log-focal chain rules, scaled by the upstream
// gradient.  No per-match intermediate is stored between the two.
#include <hip/hip_runtime.h>

#include "fea_ctx.h"
#include "fea_device.h"

namespace fea {
namespace {

__global__ void k_params_to_pose(int N, const double* __restrict__ a6, const double* __restrict__ t,
                                 const double* __restrict__ logf, const int32_t* __restrict__ group,
                                 double* __restrict__ R, double* __restrict__ T, double* __restrict__ F) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double a[6], Rc[9];
#pragma unroll
  for (int k = 0; k < 6; ++k) a[k] = a6[6 * c + k];
  rot6d_forward(a, Rc);
#pragma unroll
  for (int k = 0; k < 9; ++k) R[9 * c + k] = Rc[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) T[3 * c + k] = t[3 * c + k];
  F[c] = exp(logf[group[c]]);
}

constexpr int kLossThreads = 1024;

// Loss = sum over work items of their loss partial (fixed order).
__global__ __launch_bounds__(kLossThreads) void k_item_loss(int64_t n_items, const double* __restrict__ part,
                                                            double* __restrict__ out) {
  __shared__ double s_red[kLossThreads / kWave];
  double L = 0.0;
  for (int64_t it = threadIdx.x; it < n_items; it += kLossThreads) L += part[it * kPartStride + 9];
  L = wave_sum_f64(L);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = L;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kLossThreads / kWave; ++w) s += s_red[w];
    out[0] = s;
  }
}

// Threads [0, N): dL/da6 = vjp of the 6D map, dL/dt, scaled by gout.
// Threads [N, N+G): dL/dlog f of each group = sum over its cameras of
// f_c dL/df_c, scaled by gout.
__global__ void k_param_grad(int N, int G, const double* __restrict__ a6, const double* __restrict__ gR,
                             const double* __restrict__ gt_in, const double* __restrict__ gf,
                             const double* __restrict__ F, const int32_t* __restrict__ grp_off,
                             const int32_t* __restrict__ grp_cams, const double* __restrict__ gout,
                             double* __restrict__ ga6, double* __restrict__ gt, double* __restrict__ glogf) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const double s = gout ? gout[0] : 1.0;
  if (k < N) {
    double a[6], g[9], ga[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) a[q] = a6[6 * k + q];
#pragma unroll
    for (int q = 0; q < 9; ++q) g[q] = gR[9 * k + q];
    rot6d_vjp(a, g, ga);
    if (ga6)
#pragma unroll
      for (int q = 0; q < 6; ++q) ga6[6 * k + q] = s * ga[q];
    if (gt)
#pragma unroll
      for (int q = 0; q < 3; ++q) gt[3 * k + q] = s * gt_in[3 * k + q];
  } else if (k < N + G) {
    const int g = k - N;
    double acc = 0.0;
    for (int q = grp_off[g]; q < grp_off[g + 1]; ++q) {
      const int c = grp_cams[q];
      acc += gf[c] * F[c];
    }
    if (glogf) glogf[g] = s * acc;
  }
}

}  // namespace

hipError_t launch_params_to_pose(fea_ctx* c, const double* a6, const double* t, const double* logf) {
  k_params_to_pose<<<(unsigned)((c->N + 255) / 256), 256, 0, c->stream>>>(
      c->N, a6, t, logf, c->d_group.as<int32_t>(), c->Re.as<double>(), c->Te.as<double>(), c->Fe.as<double>());
  return hipGetLastError();
}

hipError_t launch_item_loss(fea_ctx* c, double* loss_out) {
  k_item_loss<<<1, kLossThreads, 0, c->stream>>>(c->n_items, c->part.as<double>(), loss_out);
  return hipGetLastError();
}

hipError_t launch_param_grad(fea_ctx* c, const double* a6, const double* gout, double* ga6, double* gt,
                             double* glogf) {
  const int total = c->N + c->G;
  k_param_grad<<<(unsigned)((total + 255) / 256), 256, 0, c->stream>>>(
      c->N, c->G, a6, c->gR.as<double>(), c->gt.as<double>(), c->gf.as<double>(), c->Fe.as<double>(),
      c->d_grp_off.as<int32_t>(), c->d_grp_cams.as<int32_t>(), gout, ga6, gt, glogf);
  return hipGetLastError();
}

}  // namespace fea
