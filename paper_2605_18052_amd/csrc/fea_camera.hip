// Per-camera epilogue of one epipolar-adjustment step on gfx950.
//
// k_camgrad: one wavefront per camera.  Lanes walk the camera's incident
// pairs (a fixed list of int4 entries {2n+side, first item, end item, other
// camera}, so a lane needs one dependent load before it can fetch everything
// else), take the pair's dL/dF -- the sum of its item partials from the
// per-match kernel (fixed order) or, with QUAD, 2 W_n f from the pair's
// quadratic form at the current poses -- recompute the pair's pose block in
// fp64 and apply the adjoint of F = D_j [u]x R_j R_i^T D_i to get this
// camera's share of dL/dR, dL/dt and dL/df.  The 14 sums are reduced across
// the wave with DPP in a fixed order, so the gradient is bit-reproducible.
// With do_update, lanes 0, 1 and 2 take the Adam steps (Kingma & Ba,
// bias-corrected) on the 6D rotation, the translation and, when every
// intrinsics group holds one camera, log f; their optimiser state is loaded
// before the pair loop, and the bias corrections come from running powers
// beta^t kept with the step counters.
//
// k_focal_update: Adam on log f for intrinsics groups shared by several
// cameras (dL/dlog f = sum over the group of f_c dL/df_c).
// k_loss_sum: the loss, summed over cameras in a fixed order (run on demand).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

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

// Base learning rates (scaled on the device by StepCounters::lr_scale).
struct AdamArgs {
  double lr_rot, lr_t, lr_f, b1, b2, eps;
};

// Step bookkeeping kept on the device so that a captured multi-step graph
// can be replayed: slot p of the counters holds the Adam step count, the
// global step count and beta1^t, beta2^t before this step, where p is the
// step's parity (which of the two pose buffers is current); the step writes
// the advanced values to slot p^1 for the next step.  Rotations are logged
// every log_every global steps.
struct StepCtl {
  StepCounters* ctr;
  int p;
  int log_every, max_log;
  double* logR;
};

constexpr int kQuad = 45;  // distinct entries of the symmetric 9x9 W_n

// dL/dF = 2 W f and the loss f^T W f of a pair from its quadratic form.
__device__ __forceinline__ void quad_partials(const double* __restrict__ W, const double F[9],
                                              double G[kPartStride]) {
  double Wf[9];
#pragma unroll
  for (int r = 0; r < 9; ++r) Wf[r] = 0.0;
  int k = 0;
#pragma unroll
  for (int r = 0; r < 9; ++r)
#pragma unroll
    for (int s = r; s < 9; ++s, ++k) {
      const double w = W[k];
      Wf[r] = fma(w, F[s], Wf[r]);
      if (s != r) Wf[s] = fma(w, F[r], Wf[s]);
    }
  double L = 0.0;
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    G[r] = 2.0 * Wf[r];
    L = fma(F[r], Wf[r], L);
  }
  G[9] = L;
}

// The per-camera pass's arguments that stay the same from step to step.
struct CamArgs {
  int N;
  const int32_t* cam_off;
  const int4* cam_ent;
  const double* part;
  const double* qW;
  double *gR_out, *gt_out, *gf_out, *loss_cam;
  int do_update, focal_inline, optimize_focal;
  const int32_t* group;
  double *a6, *tp, *logf, *m_a6, *v_a6, *m_t, *v_t, *m_f, *v_f;
  AdamArgs ad;
  const int32_t* cam_scene;
  const int32_t* scene_done;
};

// The poses a step reads (current parity) and writes (the other one).
struct PosePair {
  const double *R, *T, *Fc;
  double *Rn, *Tn, *Fn;
};

// One camera's share of a step, run by one wavefront (see the file comment).
template <bool QUAD>
__device__ __forceinline__ void camera_pass(const CamArgs& a, const PosePair& pp, const StepCtl sc, const int cam,
                                            const int lane) {
  const int N = a.N;
  const int32_t* __restrict__ cam_off = a.cam_off;
  const int4* __restrict__ cam_ent = a.cam_ent;
  const double* __restrict__ part = a.part;
  const double* __restrict__ qW = a.qW;
  const double* __restrict__ R = pp.R;
  const double* __restrict__ T = pp.T;
  const double* __restrict__ Fc = pp.Fc;
  double* __restrict__ gR_out = a.gR_out;
  double* __restrict__ gt_out = a.gt_out;
  double* __restrict__ gf_out = a.gf_out;
  double* __restrict__ loss_cam = a.loss_cam;
  const int do_update = a.do_update, focal_inline = a.focal_inline, optimize_focal = a.optimize_focal;
  const int32_t* __restrict__ group = a.group;
  double* __restrict__ a6 = a.a6;
  double* __restrict__ tp = a.tp;
  double* __restrict__ logf = a.logf;
  double* __restrict__ m_a6 = a.m_a6;
  double* __restrict__ v_a6 = a.v_a6;
  double* __restrict__ m_t = a.m_t;
  double* __restrict__ v_t = a.v_t;
  double* __restrict__ m_f = a.m_f;
  double* __restrict__ v_f = a.v_f;
  const AdamArgs ad = a.ad;
  double* __restrict__ Rn = pp.Rn;
  double* __restrict__ Tn = pp.Tn;
  double* __restrict__ Fn = pp.Fn;
  const int32_t* __restrict__ cam_scene = a.cam_scene;
  const int32_t* __restrict__ scene_done = a.scene_done;
  // The loads go in the order of their chains, so that the chains overlap:
  // the camera's entry range, its scene, the optimiser state, then the
  // camera's first entries and the scene's stop flag (a stopped scene
  // ignores the rest).
  const int e_end = cam_off[cam + 1];
  int e = cam_off[cam] + lane;
  const bool may_stop = do_update && scene_done != nullptr;
  const int scene = may_stop ? cam_scene[cam] : 0;
  // optimiser state: lane k < 6 owns 6D coordinate k, lanes 6..8 the
  // translation, lane 9 log f (single-camera intrinsics groups); every
  // update lane also needs the whole 6D vector
  const bool upd = do_update && lane < (focal_inline ? 10 : 9);
  double a_cur[6], p_own = 0.0, m_own = 0.0, v_own = 0.0;
  int grp = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) a_cur[k] = 0.0;
  if (upd) {
#pragma unroll
    for (int k = 0; k < 6; ++k) a_cur[k] = a6[6 * cam + k];
    if (lane < 6) {
      p_own = a_cur[lane < 6 ? lane : 0];
      m_own = m_a6[6 * cam + lane];
      v_own = v_a6[6 * cam + lane];
    } else if (lane < 9) {
      p_own = tp[3 * cam + lane - 6];
      m_own = m_t[3 * cam + lane - 6];
      v_own = v_t[3 * cam + lane - 6];
    } else {
      grp = group[cam];
      p_own = logf[grp];
      m_own = m_f[grp];
      v_own = v_f[grp];
    }
  }
  int4 en_next = make_int4(0, 0, 0, 0);
  if (e < e_end) en_next = cam_ent[e];
  const bool stopped = may_stop && scene_done[scene] != 0;
  // the current rotation's Gram-Schmidt frame for the 6D gradient below,
  // formed now so that its square roots and divisions overlap the entries'
  // loads instead of following the wave sums
  const Rot6dFrame frame = rot6d_frame(a_cur);
  if (stopped) {
    // a converged scene takes no step: its poses carry over to the next
    // parity unchanged (the rotation log still records them) and its
    // gradient, loss and optimiser state are left as they are
    const int p = sc.p;
    const long long t_glob = sc.ctr->global_t[p] + 1;
    if (cam == 0 && lane == 0) {
      sc.ctr->adam_t[p ^ 1] = sc.ctr->adam_t[p] + 1;
      sc.ctr->global_t[p ^ 1] = t_glob;
      sc.ctr->b1t[p ^ 1] = sc.ctr->b1t[p] * ad.b1;
      sc.ctr->b2t[p ^ 1] = sc.ctr->b2t[p] * ad.b2;
    }
    if (lane < 9) {
      const double r = R[9 * cam + lane];
      Rn[9 * cam + lane] = r;
      if (sc.log_every > 0 && t_glob % sc.log_every == 0) {
        const long long slot = t_glob / sc.log_every - 1;
        if (slot < sc.max_log) sc.logR[(slot * N + cam) * 9 + lane] = r;
      }
    }
    if (lane < 3) Tn[3 * cam + lane] = T[3 * cam + lane];
    if (lane == 0 && focal_inline) Fn[cam] = Fc[cam];
    return;
  }
  double gR[9], gt[3], gf = 0.0, L = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) gR[k] = 0.0;
  gt[0] = gt[1] = gt[2] = 0.0;
  while (e < e_end) {
    const int4 en = en_next;
    e += kWave;
    if (e < e_end) en_next = cam_ent[e];  // the lane's next entry, in flight meanwhile
    const int side = en.x & 1;
    const int i = side ? en.w : cam;
    const int j = side ? cam : en.w;
    Geo g;
    if (!pair_geo(R + 9 * i, T + 3 * i, Fc[i], R + 9 * j, T + 3 * j, Fc[j], g)) continue;
    double G[kPartStride];
    if (QUAD) {
      quad_partials(qW + (int64_t)(en.x >> 1) * kQuad, g.F, G);
    } else {
#pragma unroll
      for (int k = 0; k < kPartStride; ++k) G[k] = 0.0;
      for (int it = en.y; it < en.z; ++it) {
#pragma unroll
        for (int k = 0; k < kPartStride; ++k) G[k] += part[(int64_t)it * kPartStride + k];
      }
    }
    pair_adjoint(g, G, R + 9 * i, T + 3 * i, R + 9 * j, Fc[i], Fc[j], side, gR, gt, gf);
    if (side == 0) L += G[9];
  }
  double red[14];
#pragma unroll
  for (int k = 0; k < 9; ++k) red[k] = gR[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) red[9 + k] = gt[k];
  red[12] = gf;
  red[13] = L;
  wave_sum_f64_scatter<14>(red);
#pragma unroll
  for (int k = 0; k < 9; ++k) gR[k] = red[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) gt[k] = red[9 + k];
  gf = red[12];
  L = red[13];
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) gR_out[9 * cam + k] = gR[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) gt_out[3 * cam + k] = gt[k];
    gf_out[cam] = gf;
    loss_cam[cam] = L;
  }
  if (upd) {
  const int p = sc.p;
  const long long t_adam = sc.ctr->adam_t[p] + 1;
  const long long t_glob = sc.ctr->global_t[p] + 1;
  const double b1t = sc.ctr->b1t[p] * ad.b1, b2t = sc.ctr->b2t[p] * ad.b2;
  if (cam == 0 && lane == 0) {
    sc.ctr->adam_t[p ^ 1] = t_adam;
    sc.ctr->global_t[p ^ 1] = t_glob;
    sc.ctr->b1t[p ^ 1] = b1t;
    sc.ctr->b2t[p ^ 1] = b2t;
  }
  // every update lane forms the 6D gradient (same instructions, no
  // divergence) and steps its own coordinate
  double ga[6];
  rot6d_vjp(frame, a_cur, gR, ga);
  double g_own, lr;
  if (lane < 6) {
    g_own = ga[0];
#pragma unroll
    for (int k = 1; k < 6; ++k) g_own = (lane == k) ? ga[k] : g_own;
    lr = ad.lr_rot;
  } else if (lane < 9) {
    g_own = (lane == 6) ? gt[0] : ((lane == 7) ? gt[1] : gt[2]);
    lr = ad.lr_t;
  } else {
    g_own = gf * Fc[cam];
    lr = optimize_focal ? ad.lr_f : 0.0;
  }
  lr *= sc.ctr->lr_scale;
  const bool step_own = lane < 9 || optimize_focal;
  if (step_own) adam_step(p_own, m_own, v_own, g_own, lr, ad.b1, ad.b2, ad.eps, 1.0 - b1t, 1.0 - b2t);
  if (lane < 6) {
    a6[6 * cam + lane] = p_own;
    m_a6[6 * cam + lane] = m_own;
    v_a6[6 * cam + lane] = v_own;
  } else if (lane < 9) {
    tp[3 * cam + lane - 6] = p_own;
    m_t[3 * cam + lane - 6] = m_own;
    v_t[3 * cam + lane - 6] = v_own;
    Tn[3 * cam + lane - 6] = p_own;
  } else {
    if (optimize_focal) {
      logf[grp] = p_own;
      m_f[grp] = m_own;
      v_f[grp] = v_own;
    }
    Fn[cam] = exp(p_own);
  }
  // the new rotation from the six updated coordinates (lanes 0..5)
  double a_new[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) a_new[k] = readlane_f64(p_own, k);
  if (lane == 0) {
    double Rnew[9];
    rot6d_forward(a_new, Rnew);
#pragma unroll
    for (int k = 0; k < 9; ++k) Rn[9 * cam + k] = Rnew[k];
    if (sc.log_every > 0 && t_glob % sc.log_every == 0) {
      const long long slot = t_glob / sc.log_every - 1;
      if (slot < sc.max_log)
#pragma unroll
        for (int k = 0; k < 9; ++k) sc.logR[(slot * N + cam) * 9 + k] = Rnew[k];
    }
  }
  }
}


template <bool QUAD>
__global__ __launch_bounds__(256) void k_camgrad(CamArgs a, PosePair pp, StepCtl sc) {
  const int cam = blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
  if (cam >= a.N) return;  // uniform per wave
  camera_pass<QUAD>(a, pp, sc, cam, threadIdx.x & 63);
}

// Both pose buffers: parity p is current, p ^ 1 receives the step's poses.
struct PoseBufs {
  double *R0, *T0, *F0, *R1, *T1, *F1;
  __device__ PosePair at(int p) const {
    return p ? PosePair{R1, T1, F1, R0, T0, F0} : PosePair{R0, T0, F0, R1, T1, F1};
  }
};

// Device-wide wait between two steps of a persistent launch.  Every
// wavefront makes its stores visible at agent scope (all XCDs), one thread
// per workgroup counts the workgroup's arrival on `bar` and waits until the
// count reaches `target` (compared modulo 2^32, so the count never needs
// resetting), then every wavefront acquires at agent scope.  The wait is
// bounded by `limit` wall-clock ticks: past it the workgroup sets *err and
// the caller leaves the kernel, so no wavefront can wait forever (under a
// cooperative launch every workgroup is resident, and none should).
__device__ __forceinline__ bool grid_wait(unsigned* bar, unsigned target, long long limit, int* err) {
  __shared__ int s_ok;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const long long t0 = wall_clock64();
    int ok = 1;
    while ((int)(__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
      __builtin_amdgcn_s_sleep(1);
      if (wall_clock64() - t0 > limit) {
        ok = 0;
        break;
      }
    }
    if (!ok) *err = 1;
    s_ok = ok;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return s_ok != 0;
}

// A round's steps of the quadratic form in one cooperative launch: in every
// step wavefront w takes cameras w, w + W, w + 2W, ... (W wavefronts in the
// grid), and the workgroups wait for each other between steps, since a step
// reads the poses every camera wrote in the one before.  Step s runs at
// parity p0 ^ (s & 1) with the same buffers, step counters and rotation log
// as one k_camgrad<true> launch per step, so the results are the same bits.
__global__ __launch_bounds__(256) void k_quad_steps(CamArgs a, PoseBufs pb, StepCtl sc, int n_steps,
                                                   unsigned* bar, unsigned bar_base, long long limit, int* err) {
  const int per_block = blockDim.x / kWave;
  const int W = gridDim.x * per_block;
  const int wave = blockIdx.x * per_block + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int p0 = sc.p;
  for (int s = 0; s < n_steps; ++s) {
    sc.p = p0 ^ (s & 1);
    const PosePair pp = pb.at(sc.p);
    for (int cam = wave; cam < a.N; cam += W) camera_pass<true>(a, pp, sc, cam, lane);
    if (s + 1 < n_steps && !grid_wait(bar, bar_base + (unsigned)(s + 1) * gridDim.x, limit, err)) return;
  }
}

constexpr int kFocalThreads = 256;
constexpr int kTauThreads = 256;

// One thread per intrinsics group shared by several cameras.
__global__ __launch_bounds__(kFocalThreads) void k_focal_update(
    int G, const int32_t* __restrict__ grp_off, const int32_t* __restrict__ grp_cams,
    const double* __restrict__ gf, const double* __restrict__ Fc, int optimize_focal, double* __restrict__ logf,
    double* __restrict__ m_f, double* __restrict__ v_f, AdamArgs ad, const StepCounters* __restrict__ ctr, int pn,
    double* __restrict__ Fn, const int32_t* __restrict__ cam_scene, const int32_t* __restrict__ scene_done) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const int b = grp_off[g], e = grp_off[g + 1];
  if (b == e) return;
  double p = logf[g];
  // a group lies in one scene; a converged scene's focal length stays
  const bool frozen = scene_done != nullptr && scene_done[cam_scene[grp_cams[b]]] != 0;
  if (optimize_focal && !frozen) {
    double s = 0.0;
    for (int k = b; k < e; ++k) {
      const int c = grp_cams[k];
      s += gf[c] * Fc[c];
    }
    // the camera kernel of this step has advanced the counters to slot pn
    double m = m_f[g], v = v_f[g];
    adam_step(p, m, v, s, ad.lr_f * ctr->lr_scale, ad.b1, ad.b2, ad.eps, 1.0 - ctr->b1t[pn], 1.0 - ctr->b2t[pn]);
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

// Base learning rates; the kernels multiply them by the round's factor held
// in the step counters, so a captured step graph stays valid across rounds.
AdamArgs adam_args(const fea_ctx* c) {
  return AdamArgs{c->opt.lr_rot, c->opt.lr_t, c->opt.lr_logf, c->opt.beta1, c->opt.beta2, c->opt.adam_eps};
}

StepCtl step_ctl(fea_ctx* c) {
  return StepCtl{c->counters.as<StepCounters>(), c->pcur, c->opt.log_every, c->opt.max_log, c->logR.as<double>()};
}

// Round start on the device, one thread per value (the N x 9 rotation
// entries, N x 3 translations, N focal lengths, N x 6 rotation and N x 3
// translation parameters, G log focal lengths), so that no thread walks a
// camera's values one after another: the snapshot history for the learned
// features (r-2 <- r-1 <- r with `shift`; on the first round all three
// become the current poses), the snapshot of the current poses and
// parameters, and with `zero` fresh Adam moments.
__global__ __launch_bounds__(256) void k_round_start(
    int N, int G, int shift, int first, int zero, const double* __restrict__ R, const double* __restrict__ T,
    const double* __restrict__ F, const double* __restrict__ a6, const double* __restrict__ tp,
    const double* __restrict__ logf, double* __restrict__ Rh, double* __restrict__ Th, double* __restrict__ Fh,
    double* __restrict__ Rh1, double* __restrict__ Th1, double* __restrict__ Fh1, double* __restrict__ Rh2,
    double* __restrict__ Th2, double* __restrict__ Fh2, double* __restrict__ a6h, double* __restrict__ tph,
    double* __restrict__ logfh, double* __restrict__ m_a6, double* __restrict__ v_a6, double* __restrict__ m_t,
    double* __restrict__ v_t, double* __restrict__ m_f, double* __restrict__ v_f) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  auto snap = [&](double* h0, double* h1, double* h2, const double* cur, int64_t k) {
    const double now = cur[k];
    if (first) {
      h1[k] = now;
      h2[k] = now;
    } else if (shift) {
      h2[k] = h1[k];
      h1[k] = h0[k];
    }
    h0[k] = now;
  };
  const int64_t n = N;
  if (q < 9 * n) return snap(Rh, Rh1, Rh2, R, q);
  q -= 9 * n;
  if (q < 3 * n) return snap(Th, Th1, Th2, T, q);
  q -= 3 * n;
  if (q < n) return snap(Fh, Fh1, Fh2, F, q);
  q -= n;
  if (q < 6 * n) {
    a6h[q] = a6[q];
    if (zero) m_a6[q] = v_a6[q] = 0.0;
    return;
  }
  q -= 6 * n;
  if (q < 3 * n) {
    tph[q] = tp[q];
    if (zero) m_t[q] = v_t[q] = 0.0;
    return;
  }
  q -= 3 * n;
  if (q < G) {
    logfh[q] = logf[q];
    if (zero) m_f[q] = v_f[q] = 0.0;
  }
}
constexpr int kRoundStartValues = 22;  // per camera: 9 + 3 + 1 + 6 + 3

// Per-scene sums over a scene's contiguous items: 1,024 threads, each
// adding the items tid, tid + 1024, ... in that order (four independent
// loads per trip), then the wave sums and the 16 wave totals in wave order:
// a fixed order, the same for a scene alone or in a batch.
constexpr int kSceneSumThreads = 1024;

// Loss of every scene: the sum of its items' loss partials (a scene's items
// are contiguous, since its cameras are), one workgroup per scene; with
// out_snap, also the sum of a loss-only pass's snapshot losses (slot 8).
__global__ __launch_bounds__(kSceneSumThreads) void k_scene_loss(const int32_t* __restrict__ scene_item_off,
                                                                 const double* __restrict__ part,
                                                                 double* __restrict__ out,
                                                                 double* __restrict__ out_snap) {
  __shared__ double s_red[2][kSceneSumThreads / kWave];
  constexpr int T = kSceneSumThreads;
  const int sc = blockIdx.x, tid = threadIdx.x;
  const int e = scene_item_off[sc + 1];
  const bool snap = out_snap != nullptr;
  double L = 0.0, Ls = 0.0;
  for (int it = scene_item_off[sc] + tid; it < e; it += 4 * T) {
    double x[4], y[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool in = it + r * T < e;
      const double* row = part + (int64_t)(it + r * T) * kPartStride;
      x[r] = in ? row[9] : 0.0;
      y[r] = (in && snap) ? row[8] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      L += x[r];
      Ls += y[r];
    }
  }
  L = wave_sum_f64(L);
  Ls = wave_sum_f64(Ls);
  if ((tid & 63) == 0) {
    s_red[0][tid >> 6] = L;
    s_red[1][tid >> 6] = Ls;
  }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0, ts = 0.0;
    for (int w = 0; w < T / kWave; ++w) {
      t += s_red[0][w];
      ts += s_red[1][w];
    }
    out[sc] = t;
    if (snap) out_snap[sc] = ts;
  }
}

// Snapshot of a round start (parameters and the poses derived from them),
// for the restores below.
struct SnapView {
  const double *a6, *tp, *logf, *R, *T, *F;
};
struct PoseView {
  double *a6, *tp, *logf, *R, *T, *F;
};

// Every camera of a scene (cameras scene_cams[b, e)) gets the snapshot's
// parameters and poses back, the workgroup's threads over the cameras.
__device__ void restore_scene(int b, int e, const int32_t* __restrict__ scene_cams,
                              const int32_t* __restrict__ group, const SnapView& h, const PoseView& p, int nthreads) {
  for (int k = b + (int)threadIdx.x; k < e; k += nthreads) {
    const int c = scene_cams[k];
#pragma unroll
    for (int q = 0; q < 6; ++q) p.a6[6 * c + q] = h.a6[6 * c + q];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      p.tp[3 * c + q] = h.tp[3 * c + q];
      p.T[3 * c + q] = h.T[3 * c + q];
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) p.R[9 * c + q] = h.R[9 * c + q];
    p.F[c] = h.F[c];
    p.logf[group[c]] = h.logf[group[c]];  // the same value from every camera of the group
  }
}

// Non-finite guard at a round boundary, one workgroup per scene: if any of
// the scene's cameras holds a non-finite parameter (6D rotation,
// translation, log focal length of its group), pose (R, t, f) or loss share
// of the last step, every camera of the scene gets the parameters and poses
// of the snapshot the finished round started from (checked finite when it
// was taken) and the scene is stopped: done[s] = -(round + 1), which every
// step kernel honours as it honours a converged scene.  A scene already
// stopped or converged is left alone.
constexpr int kGuardThreads = 1024;

__global__ __launch_bounds__(kGuardThreads) void k_guard(const int32_t* __restrict__ scene_cam_off,
                                                         const int32_t* __restrict__ scene_cams,
                                                         const int32_t* __restrict__ group, SnapView h, PoseView p,
                                                         const double* __restrict__ loss_cam, int32_t round,
                                                         int32_t* __restrict__ done) {
  const int s = blockIdx.x, tid = threadIdx.x;
  if (done[s] != 0) return;  // uniform over the workgroup
  const int b = scene_cam_off[s], e = scene_cam_off[s + 1];
  int bad = 0;
  for (int k = b + tid; k < e; k += kGuardThreads) {
    const int c = scene_cams[k];
    double acc = p.logf[group[c]] + p.F[c] + loss_cam[c];
#pragma unroll
    for (int q = 0; q < 6; ++q) acc += p.a6[6 * c + q];
#pragma unroll
    for (int q = 0; q < 3; ++q) acc += p.tp[3 * c + q] + p.T[3 * c + q];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc += p.R[9 * c + q];
    // a sum of finite values can overflow to inf only if the values are
    // huge, which is as much a failure as a non-finite one
    bad |= !isfinite(acc);
  }
  if (!__syncthreads_or(bad)) return;
  restore_scene(b, e, scene_cams, group, h, p, kGuardThreads);
  if (tid == 0) done[s] = -(round + 1);
}

// The learned-weight judge after a round, on the device: a scene that ran
// the round on learned weights and whose plain IRLS objective (this round's
// plain weights) did not go down from the snapshot (l0) to the round's end
// (l1) -- or is not a number -- gets the snapshot back and plain weights
// from the next round on (ok[s] = 0; fallbacks[s] counts the rejections).
__global__ __launch_bounds__(kGuardThreads) void k_judge(const int32_t* __restrict__ scene_cam_off,
                                                         const int32_t* __restrict__ scene_cams,
                                                         const int32_t* __restrict__ group, SnapView h, PoseView p,
                                                         const int32_t* __restrict__ mode,
                                                         const double* __restrict__ l0,
                                                         const double* __restrict__ l1, int32_t* __restrict__ ok,
                                                         int32_t* __restrict__ fallbacks) {
  const int s = blockIdx.x;
  if (mode[s] == 0 || l1[s] <= l0[s]) return;  // uniform over the workgroup
  restore_scene(scene_cam_off[s], scene_cam_off[s + 1], scene_cams, group, h, p, kGuardThreads);
  if (threadIdx.x == 0) {
    ok[s] = 0;
    fallbacks[s] += 1;
  }
}

// Weighting mode of each scene for the round: learned while enabled and not
// rejected by the judge.
__global__ void k_choose_mode(int S, int enabled, const int32_t* __restrict__ ok, int32_t* __restrict__ mode) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < S) mode[s] = (enabled && ok[s] != 0) ? 1 : 0;
}

// Round start on the device, so that a round needs no host round trip:
// one workgroup per scene sorts its cameras' focal lengths in LDS (bitonic,
// padded with +inf to a power of two), takes the median the host would (the
// middle value, or the mean of the two middle values for an even count; 1
// for a scene without cameras), sets the threshold tau_px / median
// (infinite stays infinite) and shifts the history of medians at the
// snapshots r, r-1, r-2 (all three set at the first round), in fp64 and as
// the fp32 copy the learned features read.
constexpr int kTauSortThreads = 1024;

__global__ __launch_bounds__(kTauSortThreads) void k_scene_tau(int S, const int32_t* __restrict__ scene_cam_off,
                                                               const int32_t* __restrict__ scene_cams,
                                                               const double* __restrict__ Fc, double tau_px,
                                                               int first, double* __restrict__ fbar_hist,
                                                               float* __restrict__ fbar, double* __restrict__ tau) {
  __shared__ double v[kMaxSceneCams];
  const int s = blockIdx.x;
  const int b = scene_cam_off[s], n = scene_cam_off[s + 1] - b;
  int p2 = 1;
  while (p2 < n) p2 <<= 1;
  for (int i = threadIdx.x; i < p2; i += kTauSortThreads) v[i] = i < n ? Fc[scene_cams[b + i]] : INFINITY;
  __syncthreads();
  // stage (k, j) compares the p2 / 2 pairs (i, i + j), i with bit j clear:
  // pair q's i is q with a zero bit inserted at bit j, so every thread
  // takes one pair per stage up to 2,048 cameras
  for (int k = 2; k <= p2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int q = threadIdx.x; q < (p2 >> 1); q += kTauSortThreads) {
        const int i = ((q & ~(j - 1)) << 1) | (q & (j - 1));
        const int l = i | j;
        const double a = v[i], c = v[l];
        if (((i & k) == 0) ? (a > c) : (a < c)) {
          v[i] = c;
          v[l] = a;
        }
      }
      __syncthreads();
    }
  if (threadIdx.x == 0) {
    const double med = n == 0 ? 1.0 : ((n & 1) ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]));
    if (first) {
      for (int k = 0; k < 3; ++k) fbar_hist[k * S + s] = med;
    } else {
      fbar_hist[2 * S + s] = fbar_hist[S + s];
      fbar_hist[S + s] = fbar_hist[s];
      fbar_hist[s] = med;
    }
    for (int k = 0; k < 3; ++k) fbar[k * S + s] = (float)fbar_hist[k * S + s];
    tau[s] = isinf(tau_px) ? tau_px : tau_px / med;
  }
}

// Per-scene convergence test at a round start (before the snapshot is
// replaced): one workgroup per scene takes the mean over its cameras of the
// rotation between the previous round's snapshot and the current poses,
// 2 asin(|R - R_hat|_F / (2 sqrt 2)) (the geodesic angle, written for
// accuracy at small angles), and the mean |log(f / f_hat)|, both in
// degrees (per-thread sums, a fixed-order wave and workgroup sum).  With
// `check` (this round's threshold equals the previous round's) a scene
// still active whose two figures are below tol_deg is marked converged at
// `round` (stored as round + 1).
constexpr int kConvThreads = 256;

__global__ __launch_bounds__(kConvThreads) void k_scene_converge(
    const int32_t* __restrict__ scene_cam_off, const int32_t* __restrict__ scene_cams,
    const double* __restrict__ Rh, const double* __restrict__ Fh, const double* __restrict__ R,
    const double* __restrict__ F, int check, int round, double tol_deg, int32_t* __restrict__ done,
    double* __restrict__ change) {
  __shared__ double s_rot[kConvThreads / kWave], s_foc[kConvThreads / kWave];
  const int s = blockIdx.x, tid = threadIdx.x;
  const int b = scene_cam_off[s], e = scene_cam_off[s + 1];
  double rot = 0.0, foc = 0.0;
  for (int k = b + tid; k < e; k += kConvThreads) {
    const int c = scene_cams[k];
    double d2 = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const double d = R[9 * c + q] - Rh[9 * c + q];
      d2 = fma(d, d, d2);
    }
    const double half = fmin(1.0, sqrt(d2) / (2.0 * 1.4142135623730951));
    rot += 2.0 * asin(half);
    foc += fabs(log(F[c] / Fh[c]));
  }
  rot = wave_sum_f64(rot);
  foc = wave_sum_f64(foc);
  if ((tid & 63) == 0) {
    s_rot[tid >> 6] = rot;
    s_foc[tid >> 6] = foc;
  }
  __syncthreads();
  if (tid == 0) {
    rot = 0.0;
    foc = 0.0;
    for (int w = 0; w < kConvThreads / kWave; ++w) {
      rot += s_rot[w];
      foc += s_foc[w];
    }
    const double to_deg = 57.29577951308232;
    const double n = (double)max(e - b, 1);
    rot = rot / n * to_deg;
    foc = foc / n * to_deg;
    change[s] = rot;
    if (check && done[s] == 0 && rot < tol_deg && foc < tol_deg) done[s] = round + 1;
  }
}

// Each scene's loss from its cameras' shares (the share of a pair sits with
// its lower camera), summed in camera order, into row `round` of the log.
__global__ __launch_bounds__(kConvThreads) void k_scene_loss_log(int S, const int32_t* __restrict__ scene_cam_off,
                                                                 const int32_t* __restrict__ scene_cams,
                                                                 const double* __restrict__ loss_cam, int round,
                                                                 double* __restrict__ log) {
  __shared__ double s_red[kConvThreads / kWave];
  const int s = blockIdx.x, tid = threadIdx.x;
  double L = 0.0;
  for (int k = scene_cam_off[s] + tid; k < scene_cam_off[s + 1]; k += kConvThreads) L += loss_cam[scene_cams[k]];
  L = wave_sum_f64(L);
  if ((tid & 63) == 0) s_red[tid >> 6] = L;
  __syncthreads();
  if (tid == 0) {
    L = 0.0;
    for (int w = 0; w < kConvThreads / kWave; ++w) L += s_red[w];
    log[(int64_t)round * S + s] = L;
  }
}

// Per-scene normalisers of a quadratic-form round on the device (each
// scene's items contiguous): Z_s = survivors (exact, int64) and, on learned
// rounds, Z_w = sum of the survivors' learned weights (in the fixed order of
// the per-scene sums above: deterministic).  Writes
// 1/Z and 1/Z_w as the pose table reads them and Z_s; k_total_z then puts
// the total Z in zs[S].
__global__ __launch_bounds__(kSceneSumThreads) void k_scene_z(const int32_t* __restrict__ scene_item_off,
                                                              const int32_t* __restrict__ keep,
                                                              const double* __restrict__ wsum, int learned,
                                                              int64_t* __restrict__ zs, float* __restrict__ inv_z,
                                                              float* __restrict__ inv_zw,
                                                              const int32_t* __restrict__ scene_done) {
  __shared__ long long s_z[kSceneSumThreads / kWave];
  __shared__ double s_w[kSceneSumThreads / kWave];
  constexpr int T = kSceneSumThreads;
  const int s = blockIdx.x, t = threadIdx.x;
  if (scene_done != nullptr && scene_done[s] != 0) return;  // a converged scene keeps its counts
  const int e = scene_item_off[s + 1];
  long long z = 0;
  double w = 0.0;
  for (int it = scene_item_off[s] + t; it < e; it += 4 * T) {
    int k[4];
    double x[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool in = it + r * T < e;
      k[r] = in ? keep[it + r * T] : 0;
      x[r] = (learned && in) ? wsum[it + r * T] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      z += k[r];
      w += x[r];
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) z += __shfl_xor(z, m);
  w = wave_sum_f64(w);
  if ((t & 63) == 0) {
    s_z[t >> 6] = z;
    s_w[t >> 6] = w;
  }
  __syncthreads();
  if (t == 0) {
    z = 0;
    w = 0.0;
    for (int q = 0; q < T / kWave; ++q) {
      z += s_z[q];
      w += s_w[q];
    }
    zs[s] = z;
    inv_z[s] = z > 0 ? (float)(1.0 / (double)z) : 0.f;
    if (learned) inv_zw[s] = w > 0 ? (float)(1.0 / w) : 0.f;
  }
}

// The total Z after k_scene_z (one thread; S is small).
__global__ void k_total_z(int S, int64_t* __restrict__ zs) {
  long long z = 0;
  for (int s = 0; s < S; ++s) z += zs[s];
  zs[S] = z;
}

}  // namespace

hipError_t launch_scene_loss(fea_ctx* c, double* out, double* out_snap) {
  if (c->S == 0) return hipSuccess;
  k_scene_loss<<<(unsigned)c->S, kSceneSumThreads, 0, c->stream>>>(
      c->d_scene_item_off.as<int32_t>(), c->part.as<double>(), out ? out : c->scene_loss.as<double>(), out_snap);
  return hipGetLastError();
}

hipError_t launch_round_start(fea_ctx* c, bool shift, bool first, bool zero) {
  const int64_t n = (int64_t)kRoundStartValues * c->N + c->G;
  if (n == 0) return hipSuccess;
  const int p = c->pcur;
  k_round_start<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(
      c->N, c->G, shift ? 1 : 0, first ? 1 : 0, zero ? 1 : 0, c->R[p].as<double>(), c->T[p].as<double>(),
      c->Fc[p].as<double>(), c->a6.as<double>(), c->tp.as<double>(), c->logf.as<double>(), c->Rh.as<double>(),
      c->Th.as<double>(), c->Fh.as<double>(), c->Rh1.as<double>(), c->Th1.as<double>(), c->Fh1.as<double>(),
      c->Rh2.as<double>(), c->Th2.as<double>(), c->Fh2.as<double>(), c->a6h.as<double>(), c->tph.as<double>(),
      c->logfh.as<double>(), c->m_a6.as<double>(), c->v_a6.as<double>(), c->m_t.as<double>(), c->v_t.as<double>(),
      c->m_f.as<double>(), c->v_f.as<double>());
  return hipGetLastError();
}

namespace {
CamArgs cam_args(fea_ctx* c, int do_update) {
  CamArgs a;
  a.N = c->N;
  a.cam_off = c->d_cam_off.as<int32_t>();
  a.cam_ent = c->d_cam_ent.as<int4>();
  a.part = c->part.as<double>();
  a.qW = c->qW.as<double>();
  a.gR_out = c->gR.as<double>();
  a.gt_out = c->gt.as<double>();
  a.gf_out = c->gf.as<double>();
  a.loss_cam = c->loss_cam.as<double>();
  a.do_update = do_update;
  a.focal_inline = c->all_single ? 1 : 0;
  a.optimize_focal = c->opt.optimize_focal;
  a.group = c->d_group.as<int32_t>();
  a.a6 = c->a6.as<double>();
  a.tp = c->tp.as<double>();
  a.logf = c->logf.as<double>();
  a.m_a6 = c->m_a6.as<double>();
  a.v_a6 = c->v_a6.as<double>();
  a.m_t = c->m_t.as<double>();
  a.v_t = c->v_t.as<double>();
  a.m_f = c->m_f.as<double>();
  a.v_f = c->v_f.as<double>();
  a.ad = adam_args(c);
  a.cam_scene = c->d_cam_scene.as<int32_t>();
  a.scene_done = c->d_scene_done.as<int32_t>();
  return a;
}
}  // namespace

// quad: dL/dF of each pair from its quadratic form W_n (built for the round)
// instead of the per-match kernel's item partials.
hipError_t launch_camgrad(fea_ctx* c, int do_update, bool quad) {
  if (c->N == 0) return hipSuccess;
  const int per_block = 256 / kWave;
  const unsigned blocks = (unsigned)((c->N + per_block - 1) / per_block);
  const int p = c->pcur, nx = p ^ 1;
  const PosePair pp{c->R[p].as<double>(),  c->T[p].as<double>(),  c->Fc[p].as<double>(),
                    c->R[nx].as<double>(), c->T[nx].as<double>(), c->Fc[nx].as<double>()};
  if (quad)
    k_camgrad<true><<<blocks, 256, 0, c->stream>>>(cam_args(c, do_update), pp, step_ctl(c));
  else
    k_camgrad<false><<<blocks, 256, 0, c->stream>>>(cam_args(c, do_update), pp, step_ctl(c));
  return hipGetLastError();
}

// Gradient only (no update) at the poses (R, T, F), from the item partials.
hipError_t launch_camgrad_at(fea_ctx* c, const double* R, const double* T, const double* F) {
  if (c->N == 0) return hipSuccess;
  const int per_block = 256 / kWave;
  const unsigned blocks = (unsigned)((c->N + per_block - 1) / per_block);
  CamArgs a = cam_args(c, 0);
  a.qW = nullptr;
  a.focal_inline = 0;
  a.optimize_focal = 0;
  a.a6 = a.tp = a.logf = a.m_a6 = a.v_a6 = a.m_t = a.v_t = a.m_f = a.v_f = nullptr;
  a.cam_scene = nullptr;
  a.scene_done = nullptr;
  const PosePair pp{R, T, F, nullptr, nullptr, nullptr};
  k_camgrad<false><<<blocks, 256, 0, c->stream>>>(a, pp, step_ctl(c));
  return hipGetLastError();
}

// Workgroups of k_quad_steps: one wavefront per camera up to as many
// workgroups as reside on the device at once (0 if the kernel cannot run).
int quad_steps_blocks(fea_ctx* c) {
  if (c->quad_steps_cap < 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_quad_steps, 256, 0) != hipSuccess) per_cu = 0;
    (void)hipGetLastError();
    c->quad_steps_cap = per_cu * c->n_cu;
  }
  const int per_block = 256 / kWave;
  return std::min((c->N + per_block - 1) / per_block, c->quad_steps_cap);
}

hipError_t launch_quad_steps(fea_ctx* c, int n_steps, int blocks) {
  if (c->N == 0 || n_steps <= 0) return hipSuccess;
  if (blocks <= 0) return hipErrorInvalidValue;
  CamArgs a = cam_args(c, 1);
  PoseBufs pb{c->R[0].as<double>(), c->T[0].as<double>(), c->Fc[0].as<double>(),
              c->R[1].as<double>(), c->T[1].as<double>(), c->Fc[1].as<double>()};
  StepCtl sc = step_ctl(c);
  unsigned* bar = c->wait_state.as<unsigned>();
  int* err = reinterpret_cast<int*>(bar + 1);
  unsigned base = c->wait_base;
  const long long limit_us = c->opt.wait_limit_us > 0 ? c->opt.wait_limit_us : 500000;
  long long limit = limit_us * (long long)c->wall_clock_khz / 1000;
  void* args[] = {&a, &pb, &sc, &n_steps, &bar, &base, &limit, &err};
  const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_quad_steps), dim3((unsigned)blocks),
                                                  dim3(256), args, 0, c->stream);
  if (e == hipSuccess) c->wait_base += (unsigned)(n_steps - 1) * (unsigned)blocks;
  return e;
}

hipError_t launch_focal_update(fea_ctx* c) {
  if (c->G == 0) return hipSuccess;
  const int nx = c->pcur ^ 1;
  k_focal_update<<<(unsigned)((c->G + kFocalThreads - 1) / kFocalThreads), kFocalThreads, 0, c->stream>>>(
      c->G, c->d_grp_off.as<int32_t>(), c->d_grp_cams.as<int32_t>(), c->gf.as<double>(),
      c->Fc[c->pcur].as<double>(), c->opt.optimize_focal, c->logf.as<double>(), c->m_f.as<double>(),
      c->v_f.as<double>(), adam_args(c), c->counters.as<StepCounters>(), c->pcur ^ 1, c->Fc[nx].as<double>(),
      c->d_cam_scene.as<int32_t>(), c->d_scene_done.as<int32_t>());
  return hipGetLastError();
}

hipError_t launch_loss_sum(fea_ctx* c) {
  k_loss_sum<<<1, kLossThreads, 0, c->stream>>>(c->N, c->loss_cam.as<double>(), c->loss.as<double>());
  return hipGetLastError();
}


hipError_t launch_scene_tau(fea_ctx* c, double tau_px, bool first) {
  if (c->S == 0) return hipSuccess;
  k_scene_tau<<<(unsigned)c->S, kTauSortThreads, 0, c->stream>>>(
      c->S, c->d_scene_cam_off.as<int32_t>(), c->d_scene_cams.as<int32_t>(), c->Fc[c->pcur].as<double>(), tau_px,
      first ? 1 : 0, c->d_fbar_hist.as<double>(), c->d_fbar.as<float>(), c->d_tau.as<double>());
  return hipGetLastError();
}

namespace {
SnapView snap_view(fea_ctx* c) {
  return SnapView{c->a6h.as<double>(), c->tph.as<double>(), c->logfh.as<double>(),
                  c->Rh.as<double>(),  c->Th.as<double>(),  c->Fh.as<double>()};
}
PoseView pose_view(fea_ctx* c) {
  const int p = c->pcur;
  return PoseView{c->a6.as<double>(),   c->tp.as<double>(),   c->logf.as<double>(),
                  c->R[p].as<double>(), c->T[p].as<double>(), c->Fc[p].as<double>()};
}
}  // namespace

hipError_t launch_guard(fea_ctx* c, int32_t round) {
  if (c->S == 0 || c->N == 0) return hipSuccess;
  k_guard<<<(unsigned)c->S, kGuardThreads, 0, c->stream>>>(c->d_scene_cam_off.as<int32_t>(),
                                                           c->d_scene_cams.as<int32_t>(), c->d_group.as<int32_t>(),
                                                           snap_view(c), pose_view(c), c->loss_cam.as<double>(),
                                                           round, c->d_scene_done.as<int32_t>());
  c->ptab_current = false;
  return hipGetLastError();
}

hipError_t launch_judge(fea_ctx* c) {
  if (c->S == 0 || c->N == 0) return hipSuccess;
  k_judge<<<(unsigned)c->S, kGuardThreads, 0, c->stream>>>(
      c->d_scene_cam_off.as<int32_t>(), c->d_scene_cams.as<int32_t>(), c->d_group.as<int32_t>(), snap_view(c),
      pose_view(c), c->d_scene_mode.as<int32_t>(), c->d_judge_l0.as<double>(), c->d_judge_l1.as<double>(),
      c->d_learned_ok.as<int32_t>(), c->d_fallbacks.as<int32_t>());
  c->ptab_current = false;
  return hipGetLastError();
}

hipError_t launch_choose_mode(fea_ctx* c, bool enabled) {
  if (c->S == 0) return hipSuccess;
  k_choose_mode<<<(unsigned)((c->S + 255) / 256), 256, 0, c->stream>>>(
      c->S, enabled ? 1 : 0, c->d_learned_ok.as<int32_t>(), c->d_scene_mode.as<int32_t>());
  return hipGetLastError();
}

hipError_t launch_scene_converge(fea_ctx* c, bool check, int32_t round) {
  if (c->S == 0) return hipSuccess;
  const int p = c->pcur;
  k_scene_converge<<<(unsigned)c->S, kConvThreads, 0, c->stream>>>(
      c->d_scene_cam_off.as<int32_t>(), c->d_scene_cams.as<int32_t>(), c->Rh.as<double>(), c->Fh.as<double>(),
      c->R[p].as<double>(), c->Fc[p].as<double>(), check ? 1 : 0, round, c->opt.converge_deg,
      c->d_scene_done.as<int32_t>(), c->d_scene_change.as<double>());
  return hipGetLastError();
}

hipError_t launch_scene_loss_log(fea_ctx* c, int32_t round) {
  if (c->S == 0) return hipSuccess;
  k_scene_loss_log<<<(unsigned)c->S, kConvThreads, 0, c->stream>>>(
      c->S, c->d_scene_cam_off.as<int32_t>(), c->d_scene_cams.as<int32_t>(), c->loss_cam.as<double>(), round,
      c->d_scene_loss_log.as<double>());
  return hipGetLastError();
}

hipError_t launch_scene_z(fea_ctx* c) {
  if (c->S == 0) return hipSuccess;
  k_scene_z<<<(unsigned)c->S, kSceneSumThreads, 0, c->stream>>>(
      c->d_scene_item_off.as<int32_t>(), c->item_keep.as<int32_t>(), c->item_wsum.as<double>(),
      c->learned_any ? 1 : 0, c->d_scene_z.as<int64_t>(), c->d_inv_z.as<float>(), c->d_inv_zw.as<float>(),
      c->d_scene_done.as<int32_t>());
  k_total_z<<<1, 1, 0, c->stream>>>(c->S, c->d_scene_z.as<int64_t>());
  return hipGetLastError();
}

}  // namespace fea
