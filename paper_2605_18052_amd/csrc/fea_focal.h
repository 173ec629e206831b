// Focal-length vote (Method > Focal Length Estimation): kernels and
// launchers in fea_focal.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fea {

hipError_t launch_fv_vote(hipStream_t st, int n_groups, int n_cand, const int32_t* grp_off, const int32_t* grp_pairs,
                          const int32_t* pair_i, const int32_t* pair_j, const int32_t* group, const double* F,
                          const double* f_cur, const double* cand, double tau, double* votes, hipEvent_t ev0,
                          hipEvent_t ev1);
hipError_t launch_fv_best(hipStream_t st, int n_groups, int n_cand, const double* votes, const double* cand,
                          double* f_best, int32_t* k_best);

}  // namespace fea
