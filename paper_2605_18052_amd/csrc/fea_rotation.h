// Global rotation (Method > Global Rotation): kernels and launchers in
// fea_rotation.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fea_trans.h"  // TaCounters: the Adam step counters

namespace fea {

// One power-iteration step: c_out = s (sigma c_in - wm M c_in - wp P c_in)
// with s = *scale (1 when scale is null: pass it only on the step after a
// renormalisation); with renorm also scale_out = 1/|c_out| and *rho = the
// Rayleigh quotient of A at c_in (sq holds 3 n_cams doubles).  Between
// renormalisations the vector grows by at most sigma per step (the scale
// only keeps it inside the fp64 range; the direction is the result).
hipError_t launch_ra_apply(hipStream_t st, int n_cams, const int32_t* cam_off, const int32_t* cam_ent,
                           const int32_t* pair_i, const int32_t* pair_j, const double* Rrel, const double* c_in,
                           const double* scale, const double* c1, double sigma, double wm, double wp, double* c_out,
                           double* sq, double* scale_out, bool renorm, double* rho);
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
