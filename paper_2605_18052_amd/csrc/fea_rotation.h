// Global rotation (Method > Global Rotation): kernels and launchers in
// fea_rotation.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fea_trans.h"  // TaCounters: the Adam step counters

namespace fea {

// One Lanczos step on A = wm M + wp diag(c1 c1^T) (c1 nullable: wp unused):
// w = A V_j orthogonalised twice against V_0..V_j, alpha[j] its coefficient
// on V_j, beta[j] = |w|, V_{j+1} = w / beta[j].  V holds (j+2) * 3 n_cams
// doubles; sq 3 n_cams, h1/h2 j+1, part lz_orth_blocks(3 n_cams) scratch.
hipError_t launch_lz_step(hipStream_t st, int n_cams, const int32_t* cam_off, const int32_t* cam_ent,
                          const int32_t* pair_i, const int32_t* pair_j, const double* Rrel, const double* c1, double wm,
                          double wp, double* V, int j, double* w, double* sq, double* h1, double* h2, double* part,
                          double* alpha, double* beta);
int lz_orth_blocks(int64_t n);
// y = sum over i < m of s[i] V_i.
hipError_t launch_lz_combine(hipStream_t st, int64_t n, int m, const double* V, const double* s, double* y);
hipError_t launch_ra_columns(hipStream_t st, int n_cams, const double* c, const double* c1, double* out,
                             int32_t* err);
hipError_t launch_ra_step(hipStream_t st, int n_cams, int64_t n_pairs, const int32_t* cam_off, const int32_t* cam_ent,
                          const int32_t* pair_i, const int32_t* pair_j, const double* Rrel, const double* a_in,
                          double* a_out, double* m, double* v, TaCounters* ctr, int parity, double beta1,
                          double beta2, double eps, double decay);
hipError_t launch_ra_loss(hipStream_t st, int64_t n_pairs, const int32_t* pair_i, const int32_t* pair_j,
                          const double* Rrel, const double* a6, double* loss);
hipError_t launch_ra_to_R(hipStream_t st, int n_cams, const double* a6, double* R);

}  // namespace fea
