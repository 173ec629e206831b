// Per-camera epilogue of one epipolar-adjustment step on gfx950.
//
// k_camgrad: one wavefront per camera.  Lanes walk the camera's incident
// pairs (a fixed list of int4 entries {2n+side, first item, end item, other
// camera}, so a lane needs one dependent load before it can fetch everything
// else), sum the pair's item partials (dL/dF and the loss, fixed order),
// recompute the pair's pose block in fp64 and apply the adjoint of
// F = D_j [u]x R_j R_i^T D_i to get this camera's share of dL/dR, dL/dt and
// dL/df.  The 14 sums are reduced across the wave by a fixed butterfly, so
// the gradient is bit-reproducible.  With do_update, lane 0 takes the Adam
// step (Kingma & Ba, bias-corrected) on the 6D rotation and the translation
// and, when every intrinsics group holds one camera, on log f as well.
//
// k_focal_update: Adam on log f for intrinsics groups shared by several
// cameras (dL/dlog f = sum over the group of f_c dL/df_c).
// k_loss_sum: the loss, summed over cameras in a fixed order (run on demand).
#include <hip/hip_runtime.h>

#include "fea_ctx.h"
#include "fea_device.h"

namespace fea {
namespace {

__device__ __forceinline__ void adam_step(double& p, double& m, double& v, double g, double lr, double b1,
                                          double b2, double eps, double bc1, double bc2) {
  m = b1 * m + (1.0 - b1) * g;
  v = b2 * v + (1.0 - b2) * g * g;
  p -= lr * (m / bc1) / (sqrt(v / bc2) + eps);
}

struct AdamArgs {
  double lr_rot, lr_t, lr_f, b1, b2, eps;
};

// Step bookkeeping kept on the device so that a captured multi-step graph
// can be replayed: ctr[p] is the Adam step count and ctr[2+p] the global step
// count before this step, where p is the step's parity (which of the two
// pose buffers is current); the step writes the incremented counts to slot
// p^1 for the next step.  Rotations are logged every log_every global steps.
struct StepCtl {
  long long* ctr;
  int p;
  int log_every, max_log;
  double* logR;
};

__global__ __launch_bounds__(256) void k_camgrad(
    int N, const int32_t* __restrict__ cam_off, const int4* __restrict__ cam_ent,
    const double* __restrict__ part, const double* __restrict__ R, const double* __restrict__ T,
    const double* __restrict__ Fc, double* __restrict__ gR_out, double* __restrict__ gt_out,
    double* __restrict__ gf_out, double* __restrict__ loss_cam, int do_update, int focal_inline,
    int optimize_focal, const int32_t* __restrict__ group, double* __restrict__ a6, double* __restrict__ tp,
    double* __restrict__ logf, double* __restrict__ m_a6, double* __restrict__ v_a6,
    double* __restrict__ m_t, double* __restrict__ v_t, double* __restrict__ m_f, double* __restrict__ v_f,
    AdamArgs ad, StepCtl sc, double* __restrict__ Rn, double* __restrict__ Tn, double* __restrict__ Fn) {
  const int cam = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (cam >= N) return;  // uniform per wave
  double gR[9], gt[3], gf = 0.0, L = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) gR[k] = 0.0;
  gt[0] = gt[1] = gt[2] = 0.0;
  const int e_end = cam_off[cam + 1];
  for (int e = cam_off[cam] + lane; e < e_end; e += kWave) {
    const int4 en = cam_ent[e];
    const int side = en.x & 1;
    const int i = side ? en.w : cam;
    const int j = side ? cam : en.w;
    double G[kPartStride];
#pragma unroll
    for (int k = 0; k < kPartStride; ++k) G[k] = 0.0;
    for (int it = en.y; it < en.z; ++it) {
#pragma unroll
      for (int k = 0; k < kPartStride; ++k) G[k] += part[(int64_t)it * kPartStride + k];
    }
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
  const long long t_adam = sc.ctr[sc.p] + 1;
  const long long t_glob = sc.ctr[2 + sc.p] + 1;
  if (cam == 0) {
    sc.ctr[sc.p ^ 1] = t_adam;
    sc.ctr[2 + (sc.p ^ 1)] = t_glob;
  }
  const double bc1 = 1.0 - pow(ad.b1, (double)t_adam);
  const double bc2 = 1.0 - pow(ad.b2, (double)t_adam);
  double a[6], ga[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) a[k] = a6[6 * cam + k];
  rot6d_vjp(a, gR, ga);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double m = m_a6[6 * cam + k], v = v_a6[6 * cam + k];
    adam_step(a[k], m, v, ga[k], ad.lr_rot, ad.b1, ad.b2, ad.eps, bc1, bc2);
    m_a6[6 * cam + k] = m;
    v_a6[6 * cam + k] = v;
    a6[6 * cam + k] = a[k];
  }
  double Rnew[9];
  rot6d_forward(a, Rnew);
#pragma unroll
  for (int k = 0; k < 9; ++k) Rn[9 * cam + k] = Rnew[k];
  if (sc.log_every > 0 && t_glob % sc.log_every == 0) {
    const long long slot = t_glob / sc.log_every - 1;
    if (slot < sc.max_log)
#pragma unroll
      for (int k = 0; k < 9; ++k) sc.logR[(slot * N + cam) * 9 + k] = Rnew[k];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double p = tp[3 * cam + k], m = m_t[3 * cam + k], v = v_t[3 * cam + k];
    adam_step(p, m, v, gt[k], ad.lr_t, ad.b1, ad.b2, ad.eps, bc1, bc2);
    tp[3 * cam + k] = p;
    m_t[3 * cam + k] = m;
    v_t[3 * cam + k] = v;
    Tn[3 * cam + k] = p;
  }
  if (focal_inline) {
    const int g = group[cam];
    double p = logf[g];
    if (optimize_focal) {
      double m = m_f[g], v = v_f[g];
      adam_step(p, m, v, gf * Fc[cam], ad.lr_f, ad.b1, ad.b2, ad.eps, bc1, bc2);
      logf[g] = p;
      m_f[g] = m;
      v_f[g] = v;
    }
    Fn[cam] = exp(p);
  }
}

constexpr int kFocalThreads = 256;

// One thread per intrinsics group shared by several cameras.
__global__ __launch_bounds__(kFocalThreads) void k_focal_update(
    int G, const int32_t* __restrict__ grp_off, const int32_t* __restrict__ grp_cams,
    const double* __restrict__ gf, const double* __restrict__ Fc, int optimize_focal, double* __restrict__ logf,
    double* __restrict__ m_f, double* __restrict__ v_f, AdamArgs ad, const long long* __restrict__ t_adam_now,
    double* __restrict__ Fn) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const int b = grp_off[g], e = grp_off[g + 1];
  if (b == e) return;
  double p = logf[g];
  if (optimize_focal) {
    double s = 0.0;
    for (int k = b; k < e; ++k) {
      const int c = grp_cams[k];
      s += gf[c] * Fc[c];
    }
    const double t = (double)t_adam_now[0];
    double m = m_f[g], v = v_f[g];
    adam_step(p, m, v, s, ad.lr_f, ad.b1, ad.b2, ad.eps, 1.0 - pow(ad.b1, t), 1.0 - pow(ad.b2, t));
    logf[g] = p;
    m_f[g] = m;
    v_f[g] = v;
  }
  const double fnew = exp(p);
  for (int k = b; k < e; ++k) Fn[grp_cams[k]] = fnew;
}

constexpr int kLossThreads = 1024;

__global__ __launch_bounds__(kLossThreads) void k_loss_sum(int N, const double* __restrict__ loss_cam,
                                                           double* __restrict__ loss_out) {
  __shared__ double s_red[kLossThreads / kWave];
  const int tid = threadIdx.x;
  double L = 0.0;
  for (int c = tid; c < N; c += kLossThreads) L += loss_cam[c];
  L = wave_sum_f64(L);
  if ((tid & 63) == 0) s_red[tid >> 6] = L;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < kLossThreads / kWave; ++w) s += s_red[w];
    loss_out[0] = s;
  }
}

AdamArgs adam_args(const fea_ctx* c) {
  return AdamArgs{c->opt.lr_rot * c->lr_scale, c->opt.lr_t * c->lr_scale, c->opt.lr_logf * c->lr_scale,
                  c->opt.beta1, c->opt.beta2, c->opt.adam_eps};
}

StepCtl step_ctl(fea_ctx* c) {
  return StepCtl{c->counters.as<long long>(), c->pcur, c->opt.log_every, c->opt.max_log, c->logR.as<double>()};
}

}  // namespace

hipError_t launch_camgrad(fea_ctx* c, int do_update) {
  if (c->N == 0) return hipSuccess;
  const int per_block = 256 / kWave;
  const unsigned blocks = (unsigned)((c->N + per_block - 1) / per_block);
  const int nx = c->pcur ^ 1;
  k_camgrad<<<blocks, 256, 0, c->stream>>>(
      c->N, c->d_cam_off.as<int32_t>(), c->d_cam_ent.as<int4>(), c->part.as<double>(), c->R[c->pcur].as<double>(),
      c->T[c->pcur].as<double>(), c->Fc[c->pcur].as<double>(), c->gR.as<double>(), c->gt.as<double>(),
      c->gf.as<double>(), c->loss_cam.as<double>(), do_update, c->all_single ? 1 : 0, c->opt.optimize_focal,
      c->d_group.as<int32_t>(), c->a6.as<double>(), c->tp.as<double>(), c->logf.as<double>(),
      c->m_a6.as<double>(), c->v_a6.as<double>(), c->m_t.as<double>(), c->v_t.as<double>(), c->m_f.as<double>(),
      c->v_f.as<double>(), adam_args(c), step_ctl(c), c->R[nx].as<double>(), c->T[nx].as<double>(),
      c->Fc[nx].as<double>());
  return hipGetLastError();
}

// Gradient only (no update) at the poses (R, T, F).
hipError_t launch_camgrad_at(fea_ctx* c, const double* R, const double* T, const double* F) {
  if (c->N == 0) return hipSuccess;
  const int per_block = 256 / kWave;
  const unsigned blocks = (unsigned)((c->N + per_block - 1) / per_block);
  k_camgrad<<<blocks, 256, 0, c->stream>>>(
      c->N, c->d_cam_off.as<int32_t>(), c->d_cam_ent.as<int4>(), c->part.as<double>(), R, T, F,
      c->gR.as<double>(), c->gt.as<double>(), c->gf.as<double>(), c->loss_cam.as<double>(), 0, 0, 0,
      c->d_group.as<int32_t>(), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
      adam_args(c), step_ctl(c), nullptr, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_focal_update(fea_ctx* c) {
  if (c->G == 0) return hipSuccess;
  const int nx = c->pcur ^ 1;
  k_focal_update<<<(unsigned)((c->G + kFocalThreads - 1) / kFocalThreads), kFocalThreads, 0, c->stream>>>(
      c->G, c->d_grp_off.as<int32_t>(), c->d_grp_cams.as<int32_t>(), c->gf.as<double>(),
      c->Fc[c->pcur].as<double>(), c->opt.optimize_focal, c->logf.as<double>(), c->m_f.as<double>(),
      c->v_f.as<double>(), adam_args(c), c->counters.as<long long>() + (c->pcur ^ 1), c->Fc[nx].as<double>());
  return hipGetLastError();
}

hipError_t launch_loss_sum(fea_ctx* c) {
  k_loss_sum<<<1, kLossThreads, 0, c->stream>>>(c->N, c->loss_cam.as<double>(), c->loss.as<double>());
  return hipGetLastError();
}

}  // namespace fea
