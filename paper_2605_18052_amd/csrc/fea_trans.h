// Global Translation stages (Method > Global Translation): the
// relative-translation candidate search and the camera-centre alignment with
// multiple random initialisations.  Kernels and launchers in fea_trans.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fea {

// Candidate search: one scoring workgroup covers one work item (a run of at
// most kRtItem matches of one pair) and kRtGroup candidates (4 waves x
// kRtBlocks blocks of 16 candidates).
constexpr int kRtItem = 2048;
constexpr int kRtBlocks = 16;
constexpr int kRtGroup = 4 * kRtBlocks * 16;
constexpr int kRtRow = 16;  // per-pair row: R_ij (9), 1/f_i, 1/f_j, cx_i, cy_i, cx_j, cy_j, pad

// Adam state shared by all cameras of one alignment phase, one slot per step
// parity: the learning rate of the step and the running powers of the betas.
struct TaCounters {
  double lr[2];
  double b1t[2];
  double b2t[2];
};

hipError_t launch_rt_pairs(hipStream_t st, int64_t n_pairs, const int32_t* pair_i, const int32_t* pair_j,
                           const double* R, const double* f, const double* cx, const double* cy, float* rowf,
                           double* rowd);
hipError_t launch_rt_score(hipStream_t st, int64_t n_items, int n_groups, const int4* items, const float* rowf,
                           const float* x1, const float* y1, const float* x2, const float* y2, const float* cand,
                           int kp, double tau, float* partial, hipEvent_t ev0, hipEvent_t ev1);
hipError_t launch_rt_select(hipStream_t st, int64_t n_pairs, int k, int kp, double tau, const int32_t* pair_item_off,
                            const int4* items, const float* partial, const float* cand, const double* rowd,
                            const float* x1, const float* y1, const float* x2, const float* y2, float* scores,
                            int32_t* best, int32_t* vote, double* t_rel, double* score_best);

hipError_t launch_ta_targets(hipStream_t st, int64_t n_pairs, const int32_t* pair_j, const double* R,
                             const double* t_rel, double* target);
hipError_t launch_ta_counters(hipStream_t st, TaCounters* ctr, double lr);
hipError_t launch_ta_step(hipStream_t st, int runs, int n_cams, int64_t n_pairs, const int32_t* cam_off,
                          const int32_t* cam_ent, const int32_t* ent_other, const double* target, const double* o_in, double* o_out, double* m, double* v,
                          TaCounters* ctr, int parity, double beta1, double beta2, double eps, double decay);
hipError_t launch_ta_align(hipStream_t st, int runs, int n_cams, double* o, int32_t* err);
hipError_t launch_ta_losses(hipStream_t st, int runs, int n_cams, int64_t n_pairs, const int32_t* cam_off,
                            const int32_t* cam_ent, const int32_t* pair_i, const int32_t* pair_j,
                            const double* target, const double* o, double* pair_loss, double* cam_loss,
                            double* run_loss);
hipError_t launch_ta_merge(hipStream_t st, int runs, int n_cams, const double* o_runs, const double* cam_loss,
                           double* o_out, int32_t* run_of_cam);

}  // namespace fea
