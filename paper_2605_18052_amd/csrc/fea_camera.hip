// Per-camera epilogue of one epipolar-adjustment step on gfx950.
//
// k_camgrad: one wavefront per camera.  Lanes walk the camera's incident
// pairs (a fixed CSR list), each lane sums the pair's item partials (dL/dF
// and the loss, fixed order), recomputes the pair's pose block in fp64 and
// applies the adjoint of F = D_j [u]x R_j R_i^T D_i to obtain this camera's
// share of dL/dR, dL/dt and dL/df.  The 14 sums are reduced across the wave
// by a fixed butterfly, so the gradient is bit-reproducible.  With
// do_update, lane 0 then takes the Adam step (Kingma & Ba, bias-corrected)
// on the 6D rotation and the translation and writes the next pose.
//
// k_focal_loss: one workgroup; sums the loss over cameras and, per
// intrinsics group, d L/d log f = sum_c f_c dL/df_c and its Adam step.
#include <hip/hip_runtime.h>

#include "fea_ctx.h"
#include "fea_device.h"

namespace fea {
namespace {

__device__ __forceinline__ double adam_step(double& p, double& m, double& v, double g, double lr, double b1,
                                            double b2, double eps, double bc1, double bc2) {
  m = b1 * m + (1.0 - b1) * g;
  v = b2 * v + (1.0 - b2) * g * g;
  p -= lr * (m / bc1) / (sqrt(v / bc2) + eps);
  return p;
}

__global__ __launch_bounds__(256) void k_camgrad(
    int N, const int32_t* __restrict__ cam_off, const int32_t* __restrict__ cam_ent,
    const int32_t* __restrict__ pair_i, const int32_t* __restrict__ pair_j,
    const int32_t* __restrict__ pair_item_off, const double* __restrict__ part, const double* __restrict__ R,
    const double* __restrict__ T, const double* __restrict__ Fc, double* __restrict__ gR_out,
    double* __restrict__ gt_out, double* __restrict__ gf_out, double* __restrict__ loss_cam, int do_update,
    double* __restrict__ a6, double* __restrict__ tp, double* __restrict__ m_a6, double* __restrict__ v_a6,
    double* __restrict__ m_t, double* __restrict__ v_t, double lr_rot, double lr_t, double b1, double b2,
    double eps, double bc1, double bc2, double* __restrict__ Rn, double* __restrict__ Tn) {
  const int cam = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (cam >= N) return;  // uniform per wave
  double gR[9], gt[3], gf = 0.0, L = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) gR[k] = 0.0;
  gt[0] = gt[1] = gt[2] = 0.0;
  const int e_end = cam_off[cam + 1];
  for (int e = cam_off[cam] + lane; e < e_end; e += kWave) {
    const int ent = cam_ent[e];
    const int n = ent >> 1, side = ent & 1;
    double G[kPartStride];
#pragma unroll
    for (int k = 0; k < kPartStride; ++k) G[k] = 0.0;
    for (int it = pair_item_off[n]; it < pair_item_off[n + 1]; ++it) {
#pragma unroll
      for (int k = 0; k < kPartStride; ++k) G[k] += part[(int64_t)it * kPartStride + k];
    }
    const int i = pair_i[n], j = pair_j[n];
    Geo g;
    if (!pair_geo(R + 9 * i, T + 3 * i, Fc[i], R + 9 * j, T + 3 * j, Fc[j], g)) continue;
    pair_adjoint(g, G, R + 9 * i, T + 3 * i, R + 9 * j, Fc[i], Fc[j], side, gR, gt, gf);
    if (side == 0) L += G[9];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) gR[k] = wave_sum_f64(gR[k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) gt[k] = wave_sum_f64(gt[k]);
  gf = wave_sum_f64(gf);
  L = wave_sum_f64(L);
  if (lane != 0) return;
#pragma unroll
  for (int k = 0; k < 9; ++k) gR_out[9 * cam + k] = gR[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) gt_out[3 * cam + k] = gt[k];
  gf_out[cam] = gf;
  loss_cam[cam] = L;
  if (!do_update) return;
  double a[6], ga[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) a[k] = a6[6 * cam + k];
  rot6d_vjp(a, gR, ga);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double m = m_a6[6 * cam + k], v = v_a6[6 * cam + k];
    adam_step(a[k], m, v, ga[k], lr_rot, b1, b2, eps, bc1, bc2);
    m_a6[6 * cam + k] = m;
    v_a6[6 * cam + k] = v;
    a6[6 * cam + k] = a[k];
  }
  double Rnew[9];
  rot6d_forward(a, Rnew);
#pragma unroll
  for (int k = 0; k < 9; ++k) Rn[9 * cam + k] = Rnew[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double p = tp[3 * cam + k], m = m_t[3 * cam + k], v = v_t[3 * cam + k];
    adam_step(p, m, v, gt[k], lr_t, b1, b2, eps, bc1, bc2);
    tp[3 * cam + k] = p;
    m_t[3 * cam + k] = m;
    v_t[3 * cam + k] = v;
    Tn[3 * cam + k] = p;
  }
}

constexpr int kFocalThreads = 1024;

__global__ __launch_bounds__(kFocalThreads) void k_focal_loss(
    int N, int G, const int32_t* __restrict__ grp_off, const int32_t* __restrict__ grp_cams,
    const double* __restrict__ gf, const double* __restrict__ Fc, const double* __restrict__ loss_cam,
    double* __restrict__ loss_out, int do_update, int optimize_focal, double* __restrict__ logf,
    double* __restrict__ m_f, double* __restrict__ v_f, double lr, double b1, double b2, double eps, double bc1,
    double bc2, double* __restrict__ Fn) {
  __shared__ double s_red[kFocalThreads / kWave];
  const int tid = threadIdx.x;
  double L = 0.0;
  for (int c = tid; c < N; c += kFocalThreads) L += loss_cam[c];
  L = wave_sum_f64(L);
  if ((tid & 63) == 0) s_red[tid >> 6] = L;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < kFocalThreads / kWave; ++w) s += s_red[w];
    loss_out[0] = s;
  }
  if (!do_update) return;
  for (int g = tid; g < G; g += kFocalThreads) {
    const int b = grp_off[g], e = grp_off[g + 1];
    double fnew;
    if (optimize_focal) {
      double s = 0.0;
      for (int k = b; k < e; ++k) {
        const int c = grp_cams[k];
        s += gf[c] * Fc[c];
      }
      double p = logf[g], m = m_f[g], v = v_f[g];
      adam_step(p, m, v, s, lr, b1, b2, eps, bc1, bc2);
      logf[g] = p;
      m_f[g] = m;
      v_f[g] = v;
      fnew = exp(p);
    } else {
      fnew = exp(logf[g]);
    }
    for (int k = b; k < e; ++k) Fn[grp_cams[k]] = fnew;
  }
}

}  // namespace

hipError_t launch_camgrad(fea_ctx* c, int do_update, double bc1, double bc2) {
  if (c->N == 0) return hipSuccess;
  const int per_block = 256 / kWave;
  const unsigned blocks = (unsigned)((c->N + per_block - 1) / per_block);
  const int nx = c->pcur ^ 1;
  k_camgrad<<<blocks, 256, 0, c->stream>>>(
      c->N, c->d_cam_off.as<int32_t>(), c->d_cam_ent.as<int32_t>(), c->d_pair_i.as<int32_t>(),
      c->d_pair_j.as<int32_t>(), c->pair_item_off.as<int32_t>(), c->part.as<double>(), c->R[c->pcur].as<double>(),
      c->T[c->pcur].as<double>(), c->Fc[c->pcur].as<double>(), c->gR.as<double>(), c->gt.as<double>(),
      c->gf.as<double>(), c->loss_cam.as<double>(), do_update, c->a6.as<double>(), c->tp.as<double>(),
      c->m_a6.as<double>(), c->v_a6.as<double>(), c->m_t.as<double>(), c->v_t.as<double>(), c->opt.lr_rot,
      c->opt.lr_t, c->opt.beta1, c->opt.beta2, c->opt.adam_eps, bc1, bc2, c->R[nx].as<double>(),
      c->T[nx].as<double>());
  return hipGetLastError();
}

hipError_t launch_focal_loss(fea_ctx* c, int do_update, double bc1, double bc2) {
  const int nx = c->pcur ^ 1;
  k_focal_loss<<<1, kFocalThreads, 0, c->stream>>>(
      c->N, c->G, c->d_grp_off.as<int32_t>(), c->d_grp_cams.as<int32_t>(), c->gf.as<double>(),
      c->Fc[c->pcur].as<double>(), c->loss_cam.as<double>(), c->loss.as<double>(), do_update,
      c->opt.optimize_focal, c->logf.as<double>(), c->m_f.as<double>(), c->v_f.as<double>(), c->opt.lr_logf,
      c->opt.beta1, c->opt.beta2, c->opt.adam_eps, bc1, bc2, c->Fc[nx].as<double>());
  return hipGetLastError();
}

}  // namespace fea
