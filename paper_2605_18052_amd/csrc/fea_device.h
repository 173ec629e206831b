// Device-side building blocks shared by the HIP kernels of libfastea:
// wavefront reductions and scans for gfx950 (64-lane waves, DPP), and the
// fp64 two-view geometry of FastMap's epipolar adjustment (Method >
// Optimization Formulations > Epipolar Adjustment): pose block, its adjoint
// and the 6D rotation representation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fea {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Cross-lane primitives (gfx9 DPP: quad_perm, row_half_mirror, row_mirror).
// ---------------------------------------------------------------------------

__device__ __forceinline__ float dpp_quad_1032(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_quad_2301(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_row_half_mirror(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_row_mirror(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));
}

// Sum of v over all 64 lanes, returned wave-uniform.  Within each row of 16
// lanes the DPP butterfly leaves every lane holding the row sum; the four row
// sums are then read with v_readlane and added in a fixed order.
__device__ __forceinline__ float wave_sum_f32(float v) {
  v += dpp_quad_1032(v);
  v += dpp_quad_2301(v);
  v += dpp_row_half_mirror(v);
  v += dpp_row_mirror(v);
  const float s0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float s1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float s2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float s3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (s0 + s1) + (s2 + s3);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// l <-> l^32 exchange of two fp64 values and their sum: lanes < 32 return
// x(l) + x(l + 32), lanes >= 32 return y(l - 32) + y(l).  v_permlane32_swap
// trades the upper 32 lanes of its first operand with the lower 32 of its
// second.
__device__ __forceinline__ double swap32_add(double x, double y) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

// The same between the rows of 16 lanes: rows 0 and 2 return x summed with
// the next row, rows 1 and 3 return y summed with the previous row
// (v_permlane16_swap trades the odd rows of its first operand with the even
// rows of its second).
__device__ __forceinline__ double swap16_add(double x, double y) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(y), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

// The six stages of the fp64 reduce-scatter below over S = 2^L slots
// (1 <= S <= 16), in place: on return x[0] of a lane holds the wave sum of
// x[k], k the lane's bits 5, 4, 3, 2 (the first L of them) read from the
// top bit down -- for S = 16, k = (lane >> 2) & 15; for S = 4,
// k = (lane >> 4) & 3.
template <int S>
__device__ __forceinline__ void wave_scatter_stages_f64(double (&x)[S]) {
  static_assert(S == 1 || S == 2 || S == 4 || S == 8 || S == 16, "a power of two up to 16");
  const int lane = __lane_id();
  // stage 1: l <-> l^32
  if constexpr (S >= 2) {
#pragma unroll
    for (int k = 0; k < S / 2; ++k) x[k] = swap32_add(x[k], x[k + S / 2]);
  } else {
    x[0] = swap32_add(x[0], x[0]);
  }
  // stage 2: neighbouring rows
  if constexpr (S >= 4) {
#pragma unroll
    for (int k = 0; k < S / 4; ++k) x[k] = swap16_add(x[k], x[k + S / 4]);
  } else {
    x[0] = swap16_add(x[0], x[0]);
  }
  // stage 3: row mirror
  if constexpr (S >= 8) {
    const bool up = (lane & 8) != 0;
#pragma unroll
    for (int k = 0; k < S / 8; ++k) {
      const double keep = up ? x[k + S / 8] : x[k], send = up ? x[k] : x[k + S / 8];
      x[k] = keep + dpp_f64<0x140>(send);
    }
  } else {
    x[0] += dpp_f64<0x140>(x[0]);
  }
  // stage 4: half-row mirror
  if constexpr (S >= 16) {
    const bool up = (lane & 4) != 0;
    const double keep = up ? x[1] : x[0], send = up ? x[0] : x[1];
    x[0] = keep + dpp_f64<0x141>(send);
  } else {
    x[0] += dpp_f64<0x141>(x[0]);
  }
  x[0] += dpp_f64<0x4E>(x[0]);  // quad_perm [2,3,0,1]
  x[0] += dpp_f64<0xB1>(x[0]);  // quad_perm [1,0,3,2]
}

// Wave sums of up to 16 fp64 values, every lane receiving the results, as a
// reduce-scatter over S slots (S the power of two >= NV, the values padded
// with zeros).  Six stages pair the lanes across one bit of the lane index
// each: l <-> l^32 (v_permlane32_swap), neighbouring rows of 16
// (v_permlane16_swap), the row mirror (p <-> 15 - p), the half-row mirror
// (q <-> 7 - q), then the two pairings inside a quad.  While a lane carries
// more than one value a stage halves them -- the lane keeps the half its
// side owns and adds the partner's copy -- and after that every stage is a
// plain butterfly; so 16 sums cost about the exchanges of two single ones.
// With S = 2^L, sum k ends in the lanes whose bits 5, 4, 3, 2 (the first L
// of them) spell k from its top bit down, and is read from there.  The
// order of the additions is fixed, so the sums are reproducible and every
// lane receives the same bits.
template <int NV>
__device__ __forceinline__ void wave_sum_f64_scatter(double (&v)[NV]) {
  static_assert(NV >= 1 && NV <= 16, "1 to 16 values");
  constexpr int S = NV <= 1 ? 1 : NV <= 2 ? 2 : NV <= 4 ? 4 : NV <= 8 ? 8 : 16;
  constexpr int L = S == 1 ? 0 : S == 2 ? 1 : S == 4 ? 2 : S == 8 ? 3 : 4;
  double x[S];
#pragma unroll
  for (int k = 0; k < S; ++k) x[k] = k < NV ? v[k] : 0.0;
  wave_scatter_stages_f64<S>(x);
  constexpr int kBit[4] = {32, 16, 8, 4};
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    int src = 0;
#pragma unroll
    for (int t = 0; t < L; ++t) src += ((k >> (L - 1 - t)) & 1) ? kBit[t] : 0;
    v[k] = readlane_f64(x[0], src);
  }
}

// The fp32 forms of the exchanges above, and the same reduce-scatter for up
// to 16 fp32 values (one lane swap per exchange instead of two).
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float swap32_add(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_add(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
template <int NV>
__device__ __forceinline__ void wave_sum_f32_scatter(float (&v)[NV]) {
  static_assert(NV >= 1 && NV <= 16, "1 to 16 values");
  constexpr int S = NV <= 1 ? 1 : NV <= 2 ? 2 : NV <= 4 ? 4 : NV <= 8 ? 8 : 16;
  constexpr int L = S == 1 ? 0 : S == 2 ? 1 : S == 4 ? 2 : S == 8 ? 3 : 4;
  float x[S];
#pragma unroll
  for (int k = 0; k < S; ++k) x[k] = k < NV ? v[k] : 0.f;
  const int lane = __lane_id();
  if constexpr (S >= 2) {
#pragma unroll
    for (int k = 0; k < S / 2; ++k) x[k] = swap32_add(x[k], x[k + S / 2]);
  } else {
    x[0] = swap32_add(x[0], x[0]);
  }
  if constexpr (S >= 4) {
#pragma unroll
    for (int k = 0; k < S / 4; ++k) x[k] = swap16_add(x[k], x[k + S / 4]);
  } else {
    x[0] = swap16_add(x[0], x[0]);
  }
  if constexpr (S >= 8) {
    const bool up = (lane & 8) != 0;
#pragma unroll
    for (int k = 0; k < S / 8; ++k) {
      const float keep = up ? x[k + S / 8] : x[k], send = up ? x[k] : x[k + S / 8];
      x[k] = keep + dpp_f32<0x140>(send);
    }
  } else {
    x[0] += dpp_f32<0x140>(x[0]);
  }
  if constexpr (S >= 16) {
    const bool up = (lane & 4) != 0;
    const float keep = up ? x[1] : x[0], send = up ? x[0] : x[1];
    x[0] = keep + dpp_f32<0x141>(send);
  } else {
    x[0] += dpp_f32<0x141>(x[0]);
  }
  x[0] += dpp_f32<0x4E>(x[0]);
  x[0] += dpp_f32<0xB1>(x[0]);
  constexpr int kBit[4] = {32, 16, 8, 4};
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    int src = 0;
#pragma unroll
    for (int t = 0; t < L; ++t) src += ((k >> (L - 1 - t)) & 1) ? kBit[t] : 0;
    v[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x[0]), src));
  }
}

// Sum of v over all 64 lanes in fp64 (fixed order, every lane receives the
// same bits).
__device__ __forceinline__ double wave_sum_f64(double v) {
  double a[1] = {v};
  wave_sum_f64_scatter<1>(a);
  return a[0];
}

__device__ __forceinline__ double readfirstlane_f64(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Inclusive prefix sum of an int over the 64 lanes (Hillis-Steele with
// ds_bpermute; used only in once-per-round kernels).
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  const int lane = __lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int o = __builtin_amdgcn_ds_bpermute((lane - d) << 2, v);
    if (lane >= d) v += o;
  }
  return v;
}

// ---------------------------------------------------------------------------
// Two-view geometry in fp64 (row-major 3x3).
// ---------------------------------------------------------------------------

struct Geo {
  double Rij[9];  // R_j R_i^T
  double u[3];    // t_ij / |t_ij|
  double tn;      // |t_ij|
  double F[9];    // D_j [u]x R_ij D_i  (for centred pixel coordinates)
};

// Pose block of pair (i, j): relative rotation and unit translation, the
// essential matrix E = [u]x R_ij and F = D_j E D_i with D = diag(1/f,1/f,1).
// Returns false when the camera centres coincide (t_ij = 0).
__device__ __forceinline__ bool pair_geo(const double* __restrict__ Ri, const double* __restrict__ ti,
                                         double fi, const double* __restrict__ Rj,
                                         const double* __restrict__ tj, double fj, Geo& g) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      g.Rij[3 * r + c] = Rj[3 * r] * Ri[3 * c] + Rj[3 * r + 1] * Ri[3 * c + 1] + Rj[3 * r + 2] * Ri[3 * c + 2];
  double tij[3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
    tij[r] = tj[r] - (g.Rij[3 * r] * ti[0] + g.Rij[3 * r + 1] * ti[1] + g.Rij[3 * r + 2] * ti[2]);
  g.tn = sqrt(tij[0] * tij[0] + tij[1] * tij[1] + tij[2] * tij[2]);
  if (!(g.tn > 0.0)) return false;
  const double inv = 1.0 / g.tn;
  g.u[0] = tij[0] * inv;
  g.u[1] = tij[1] * inv;
  g.u[2] = tij[2] * inv;
  // rows of [u]x R: (u1 R2 - u2 R1, u2 R0 - u0 R2, u0 R1 - u1 R0) with R_k row k
  const double ifi = 1.0 / fi, ifj = 1.0 / fj;
  const double di[3] = {ifi, ifi, 1.0};
  const double dj[3] = {ifj, ifj, 1.0};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double e0 = g.u[1] * g.Rij[6 + c] - g.u[2] * g.Rij[3 + c];
    const double e1 = g.u[2] * g.Rij[c] - g.u[0] * g.Rij[6 + c];
    const double e2 = g.u[0] * g.Rij[3 + c] - g.u[1] * g.Rij[c];
    g.F[c] = dj[0] * e0 * di[c];
    g.F[3 + c] = dj[1] * e1 * di[c];
    g.F[6 + c] = dj[2] * e2 * di[c];
  }
  return true;
}

// F' acting on raw pixel coordinates q = (x, y, 1): F' = T_j^T F T_i with
// T = [[1,0,-cx],[0,1,-cy],[0,0,1]], so q2^T F' q1 = p2^T F p1 for centred p.
__device__ __forceinline__ void fold_principal_point(const double F[9], double cxi, double cyi, double cxj,
                                                     double cyj, double Fp[9]) {
  double A[9];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    A[3 * r] = F[3 * r];
    A[3 * r + 1] = F[3 * r + 1];
    A[3 * r + 2] = F[3 * r + 2] - cxi * F[3 * r] - cyi * F[3 * r + 1];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    Fp[c] = A[c];
    Fp[3 + c] = A[3 + c];
    Fp[6 + c] = A[6 + c] - cxj * A[c] - cyj * A[3 + c];
  }
}

// Adjoint of the pose block: given G = dL/dF for pair (i, j) (F for centred
// coordinates), accumulate dL/dR, dL/dt, dL/df of the camera on `side`
// (0 = i, 1 = j) into gR/gt/gf.  Chain: F = D_j E D_i, E = [u]x R_ij,
// u = t_ij/|t_ij|, t_ij = t_j - R_ij t_i, R_ij = R_j R_i^T.
__device__ __forceinline__ void pair_adjoint(const Geo& g, const double G[9], const double* __restrict__ Ri,
                                             const double* __restrict__ ti, const double* __restrict__ Rj,
                                             double fi, double fj, int side, double gR[9], double gt[3],
                                             double& gf) {
  // focal: F_ab carries 1/f_i in columns 0,1 and 1/f_j in rows 0,1
  if (side == 0) {
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) s += G[3 * a] * g.F[3 * a] + G[3 * a + 1] * g.F[3 * a + 1];
    gf += -s / fi;
  } else {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) s += G[b] * g.F[b] + G[3 + b] * g.F[3 + b];
    gf += -s / fj;
  }
  // H = dL/dE = D_j G D_i
  const double ifi = 1.0 / fi, ifj = 1.0 / fj;
  const double di[3] = {ifi, ifi, 1.0};
  const double dj[3] = {ifj, ifj, 1.0};
  double H[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) H[3 * a + b] = dj[a] * G[3 * a + b] * di[b];
  // dL/d[u]x = H R_ij^T ; its action on u gives g_u
  double M[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      M[3 * a + b] = H[3 * a] * g.Rij[3 * b] + H[3 * a + 1] * g.Rij[3 * b + 1] + H[3 * a + 2] * g.Rij[3 * b + 2];
  const double gu0 = M[7] - M[5], gu1 = M[2] - M[6], gu2 = M[3] - M[1];
  const double ug = g.u[0] * gu0 + g.u[1] * gu1 + g.u[2] * gu2;
  const double inv = 1.0 / g.tn;
  const double gtij[3] = {(gu0 - ug * g.u[0]) * inv, (gu1 - ug * g.u[1]) * inv, (gu2 - ug * g.u[2]) * inv};
  // Q = dL/dR_ij = -[u]x H - gtij ti^T
  double Q[9];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double s0 = g.u[1] * H[6 + c] - g.u[2] * H[3 + c];
    const double s1 = g.u[2] * H[c] - g.u[0] * H[6 + c];
    const double s2 = g.u[0] * H[3 + c] - g.u[1] * H[c];
    Q[c] = -s0 - gtij[0] * ti[c];
    Q[3 + c] = -s1 - gtij[1] * ti[c];
    Q[6 + c] = -s2 - gtij[2] * ti[c];
  }
  if (side == 1) {
    // dL/dt_j = gtij ; dL/dR_j = Q R_i
#pragma unroll
    for (int k = 0; k < 3; ++k) gt[k] += gtij[k];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        gR[3 * a + b] += Q[3 * a] * Ri[b] + Q[3 * a + 1] * Ri[3 + b] + Q[3 * a + 2] * Ri[6 + b];
  } else {
    // dL/dt_i = -R_ij^T gtij ; dL/dR_i = Q^T R_j
#pragma unroll
    for (int k = 0; k < 3; ++k)
      gt[k] -= g.Rij[k] * gtij[0] + g.Rij[3 + k] * gtij[1] + g.Rij[6 + k] * gtij[2];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        gR[3 * a + b] += Q[a] * Rj[b] + Q[3 + a] * Rj[3 + b] + Q[6 + a] * Rj[6 + b];
  }
}

// 6D rotation representation (two Gram-Schmidt columns, the parameterisation
// FastMap uses for global rotations): a = (a1, a2) -> R = [b1 b2 b1 x b2].
__device__ __forceinline__ void rot6d_forward(const double a[6], double R[9]) {
  const double i1 = 1.0 / sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  const double b1[3] = {a[0] * i1, a[1] * i1, a[2] * i1};
  const double d = b1[0] * a[3] + b1[1] * a[4] + b1[2] * a[5];
  const double v[3] = {a[3] - d * b1[0], a[4] - d * b1[1], a[5] - d * b1[2]};
  const double i2 = 1.0 / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const double b2[3] = {v[0] * i2, v[1] * i2, v[2] * i2};
  R[0] = b1[0]; R[3] = b1[1]; R[6] = b1[2];
  R[1] = b2[0]; R[4] = b2[1]; R[7] = b2[2];
  R[2] = b1[1] * b2[2] - b1[2] * b2[1];
  R[5] = b1[2] * b2[0] - b1[0] * b2[2];
  R[8] = b1[0] * b2[1] - b1[1] * b2[0];
}

// The Gram-Schmidt frame of a 6D vector that the map above builds (b1, b2,
// the projection d = b1.a2 and the inverse norms), which its vector-Jacobian
// product reuses; a caller that knows a early can form it ahead of dL/dR.
struct Rot6dFrame {
  double b1[3], b2[3], d, i1, i2;
};

__device__ __forceinline__ Rot6dFrame rot6d_frame(const double a[6]) {
  Rot6dFrame f;
  f.i1 = 1.0 / sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  f.b1[0] = a[0] * f.i1;
  f.b1[1] = a[1] * f.i1;
  f.b1[2] = a[2] * f.i1;
  f.d = f.b1[0] * a[3] + f.b1[1] * a[4] + f.b1[2] * a[5];
  const double v[3] = {a[3] - f.d * f.b1[0], a[4] - f.d * f.b1[1], a[5] - f.d * f.b1[2]};
  f.i2 = 1.0 / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  f.b2[0] = v[0] * f.i2;
  f.b2[1] = v[1] * f.i2;
  f.b2[2] = v[2] * f.i2;
  return f;
}

// Vector-Jacobian product of rot6d_forward at a (frame f = rot6d_frame(a)):
// dL/da from dL/dR.
__device__ __forceinline__ void rot6d_vjp(const Rot6dFrame& f, const double a[6], const double gR[9],
                                          double ga[6]) {
  const double* b1 = f.b1;
  const double* b2 = f.b2;
  // columns of gR
  double g1[3] = {gR[0], gR[3], gR[6]};
  double g2[3] = {gR[1], gR[4], gR[7]};
  const double g3[3] = {gR[2], gR[5], gR[8]};
  // third column is b1 x b2
  g1[0] += b2[1] * g3[2] - b2[2] * g3[1];
  g1[1] += b2[2] * g3[0] - b2[0] * g3[2];
  g1[2] += b2[0] * g3[1] - b2[1] * g3[0];
  g2[0] += g3[1] * b1[2] - g3[2] * b1[1];
  g2[1] += g3[2] * b1[0] - g3[0] * b1[2];
  g2[2] += g3[0] * b1[1] - g3[1] * b1[0];
  // b2 = v/|v|
  const double p2 = b2[0] * g2[0] + b2[1] * g2[1] + b2[2] * g2[2];
  const double gv[3] = {(g2[0] - p2 * b2[0]) * f.i2, (g2[1] - p2 * b2[1]) * f.i2, (g2[2] - p2 * b2[2]) * f.i2};
  // v = a2 - (b1.a2) b1
  const double q = b1[0] * gv[0] + b1[1] * gv[1] + b1[2] * gv[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    ga[3 + k] = gv[k] - q * b1[k];
    g1[k] += -f.d * gv[k] - q * a[3 + k];
  }
  // b1 = a1/|a1|
  const double p1 = b1[0] * g1[0] + b1[1] * g1[1] + b1[2] * g1[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) ga[k] = (g1[k] - p1 * b1[k]) * f.i1;
}

// The same with the frame formed here.
__device__ __forceinline__ void rot6d_vjp(const double a[6], const double gR[9], double ga[6]) {
  rot6d_vjp(rot6d_frame(a), a, gR, ga);
}

}  // namespace fea
