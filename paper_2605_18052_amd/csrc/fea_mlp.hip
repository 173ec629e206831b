// Learned per-match inlier weights for gfx950: an MLP 8 -> 64 -> 64 -> 1
// (ReLU, ReLU, sigmoid) on each match's features (its epipolar residual at
// the last three round snapshots, its keypoints scaled to [-1, 1] and the
// angle between the pair's optical axes).  The weight multiplies the match's
// IRLS weight in the learned solve.
//
// Inference (k_mlp_weights) is a dense contraction, so it runs on the matrix
// cores: each wave takes 32 matches at a time and evaluates
//   H1^T = relu(W1 X^T + b1),  H2^T = relu(W2 H1^T + b2),  y = sigmoid(w3.H2 + b3)
// with fp16 MFMA (fp16 operands, fp32 accumulation; fp16 rather than bf16
// for the 3 extra significand bits at the same matrix-core rate).  The input
// features enter as two fp16 parts, x = hi + lo (hi the rounded feature, lo
// the rounded remainder), through a first layer of contraction depth 16
// whose A operand holds W1 twice: the rounding of the features, which would
// dominate the error of the weight, is gone at no extra matrix-core cost
// (the depth-16 instruction takes as long as the depth-8 one).  Hidden
// activations are rounded to nearest and saturate at fp16's largest finite
// value (the trained network's stay below ~20).  The weight is stored per
// match as fp16.  With the weights as the A operand and the activations as
// the B operand, the accumulator of one layer is already laid out as the B
// operand of the next (lane l holds match l%32 and hidden units
// 8s + 4(l/32) + 0..3 of K-slice s), so no data moves between layers; the
// output layer is one more MFMA chain whose A operand repeats w3 in every
// row, so that every accumulator register of lane l ends up holding the
// logit of match l%32.
//
// Training (k_mlp_fwd_bwd, k_mlp_grad_reduce, k_mlp_adam) runs on the vector
// units in fp32: one thread per sample for the forward and backward passes,
// the weight gradients of a workgroup's 128 samples formed from LDS-staged
// activations, per-workgroup partials summed in a fixed order, then Adam.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fea_ctx.h"
#include "fea_device.h"

namespace fea {
namespace {

typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kNF = kMlpFeat;    // 8
constexpr int kNH = kMlpHidden;  // 64
constexpr int kOffB1 = kNH * kNF;
constexpr int kOffW2 = kOffB1 + kNH;
constexpr int kOffB2 = kOffW2 + kNH * kNH;
constexpr int kOffW3 = kOffB2 + kNH;
constexpr int kOffB3 = kOffW3 + kNH;

__device__ __forceinline__ float sigmoidf_(float z) { return 1.f / (1.f + __expf(-z)); }

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two fp32 values as packed fp16, rounded to nearest (one instruction).
__device__ __forceinline__ unsigned pk_f16(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){a, b}, f16x2));
}

// Accumulator registers first..first+7 as one fp16 B-operand slice of the
// next layer, ReLU applied: per pair one packed conversion, one packed fp16
// min with 65504 (an overflow to infinity saturates at fp16's largest
// finite value) and one packed 16-bit integer max with 0 -- a negative fp16
// has its sign bit set, so as a signed integer it is negative and maps to
// +0, while non-negative values are unchanged.
__device__ __forceinline__ f16x8 relu_slice(const f32x16& acc, int first) {
  u32x4 w;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const f16x2 v = __builtin_elementwise_min(
        __builtin_convertvector((f32x2){acc[first + 2 * k], acc[first + 2 * k + 1]}, f16x2),
        (f16x2){(_Float16)65504.f, (_Float16)65504.f});
    w[k] = __builtin_bit_cast(unsigned, __builtin_elementwise_max(__builtin_bit_cast(s16x2, v), (s16x2)0));
  }
  return __builtin_bit_cast(f16x8, w);
}

__device__ __forceinline__ double eps_at(const double* F, double x1, double y1, double x2, double y2) {
  const double l0 = fma(F[0], x1, fma(F[1], y1, F[2]));
  const double l1 = fma(F[3], x1, fma(F[4], y1, F[5]));
  const double l2 = fma(F[6], x1, fma(F[7], y1, F[8]));
  return fma(x2, l0, fma(y2, l1, l2));
}

// Residual feature: log(1 + |eps| * fbar) / log(257), the residual in pixel
// equivalents, log-compressed so that 256 px maps to 1.  fp32 with the
// hardware log2 (the feature enters the network in fp16): log2(1 + x) /
// log2(257).
__device__ __forceinline__ float res_feature(double e, float fbar) {
  return __log2f(1.f + (float)fabs(e) * fbar) * 0.124912178f;  // 1 / log2(257)
}

struct Snap3 {
  const double *R0, *T0, *F0, *R1, *T1, *F1, *R2, *T2, *F2;
};

__device__ void folded_F(int i, int j, const double* R, const double* T, const double* Fc,
                         const double* cx, const double* cy, double out[9]) {
  Geo g;
  if (pair_geo(R + 9 * i, T + 3 * i, Fc[i], R + 9 * j, T + 3 * j, Fc[j], g))
    fold_principal_point(g.F, cx[i], cy[i], cx[j], cy[j], out);
  else
    for (int k = 0; k < 9; ++k) out[k] = 0.0;
}

// Per-pair row of the feature table: F folded for raw pixels at the round
// snapshots r, r-1, r-2; the angle between the optical axes at r over pi/2;
// 1/cx, 1/cy of both cameras; the scene's median f at the three snapshots.
constexpr int kSnapRow = 40;
constexpr int kSnapAng = 27, kSnapInvC = 28, kSnapFbar = 32;

__global__ __launch_bounds__(kPairThreads) void k_snap3(int32_t P, const int32_t* __restrict__ pair_i,
                                                        const int32_t* __restrict__ pair_j,
                                                        const int32_t* __restrict__ pair_scene, Snap3 sn,
                                                        const double* __restrict__ cx,
                                                        const double* __restrict__ cy,
                                                        const float* __restrict__ fbar, int n_scenes,
                                                        double* __restrict__ stab) {
  const int n = blockIdx.x * kPairThreads + threadIdx.x;
  if (n >= P) return;
  const int i = pair_i[n], j = pair_j[n], sc = pair_scene[n];
  double* row = stab + (int64_t)n * kSnapRow;
  double F[9];
  folded_F(i, j, sn.R0, sn.T0, sn.F0, cx, cy, F);
#pragma unroll
  for (int k = 0; k < 9; ++k) row[k] = F[k];
  folded_F(i, j, sn.R1, sn.T1, sn.F1, cx, cy, F);
#pragma unroll
  for (int k = 0; k < 9; ++k) row[9 + k] = F[k];
  folded_F(i, j, sn.R2, sn.T2, sn.F2, cx, cy, F);
#pragma unroll
  for (int k = 0; k < 9; ++k) row[18 + k] = F[k];
  // optical axes are the third rows of the snapshot rotations
  const double* zi = sn.R0 + 9 * i + 6;
  const double* zj = sn.R0 + 9 * j + 6;
  const double cs = fmin(1.0, fmax(-1.0, zi[0] * zj[0] + zi[1] * zj[1] + zi[2] * zj[2]));
  row[kSnapAng] = acos(cs) / 1.5707963267948966;
  row[kSnapInvC + 0] = 1.0 / cx[i];
  row[kSnapInvC + 1] = 1.0 / cy[i];
  row[kSnapInvC + 2] = 1.0 / cx[j];
  row[kSnapInvC + 3] = 1.0 / cy[j];
  row[kSnapFbar + 0] = fbar[sc];
  row[kSnapFbar + 1] = fbar[n_scenes + sc];
  row[kSnapFbar + 2] = fbar[2 * n_scenes + sc];
}

constexpr int kInferThreads = 256;

// Lanes l < 32 receive lo[] of lane l+32 and lanes l >= 32 receive hi[] of
// lane l-32 (v_permlane32_swap trades the upper half of its first operand
// with the lower half of its second).
__device__ __forceinline__ void swap_half(const u32x4& lo, const u32x4& hi, bool upper, u32x4& dst) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const auto r = __builtin_amdgcn_permlane32_swap(lo[q], hi[q], false, false);
    dst[q] = upper ? r[0] : r[1];
  }
}

// Inference over one work item.  Each wave takes 64 matches per iteration,
// one per lane: the lane computes all 8 features of its match once (the
// residuals in fp64 with the pair's snapshot matrices read by scalar loads)
// and splits them into fp16 parts hi and lo; then lanes l and l^32 trade
// parts so that the two groups of 32 matches are in the B layout of
// v_mfma_f32_32x32x16_f16 (lane l < 32: hi of match l; lane l >= 32: lo of
// match l-32 -- contraction index 8(l/32) + feature).  Layer 2 (K = 64)
// uses the same instruction, whose B operand takes 8 units per lane: with
// the contraction index permuted identically in W2's columns, the layer-1
// accumulator registers of a lane are that operand as they stand.  The next
// iteration's coordinates are loaded before this one is computed.
template <bool STORE_FEAT>
__global__ __launch_bounds__(kInferThreads) void k_mlp_weights(
    const float* __restrict__ X1, const float* __restrict__ Y1, const float* __restrict__ X2,
    const float* __restrict__ Y2, const int4* __restrict__ items, const double* __restrict__ stab,
    const float* __restrict__ params, unsigned short* __restrict__ Wout, double* __restrict__ item_wsum,
    float* __restrict__ feat_out) {
  __shared__ float s_sum[kInferThreads / kWave];
  // layer 2's biases in the accumulator layout, [tile][lane half][register]
  __shared__ __align__(16) float s_b2[2][2][16];
  const int item = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int4 rec = items[item];
  const int n = rec.x, start = rec.y, cnt = rec.z;
  const double* row = stab + (int64_t)n * kSnapRow;
  if (tid < 64) {
    const int t = tid >> 5, hh = (tid >> 4) & 1, r = tid & 15;
    s_b2[t][hh][r] = params[kOffB2 + 32 * t + 8 * (r >> 2) + 4 * hh + (r & 3)];
  }
  // weights in the A layout: row (lane%32) + 32*tile.  Layer 1, k = 8h + q:
  // q < 7 multiplies feature q in both halves (its hi and lo parts); q = 7
  // carries the bias b1 + W1[:,7] * angle (the angle feature is the pair's,
  // constant over the item) as hi in h = 0 and lo in h = 1, times the
  // constant ones of the B operand: the bias needs no register of its own.
  // Layer 2 slice (t2, g) value j <-> hidden-in unit 32 t2 + 16 g + 8 (j/4)
  // + 4 h + j%4
  const int r32 = lane & 31, h = lane >> 5;
  const float ang = (float)row[kSnapAng];
  f16x8 a1[2];
  f16x8 a2[2][4], a3[4];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int orow = r32 + 32 * t;
#pragma unroll
    for (int q = 0; q < kNF - 1; ++q) a1[t][q] = (_Float16)params[orow * kNF + q];
    const float b = fmaf(params[orow * kNF + kNF - 1], ang, params[kOffB1 + orow]);
    const _Float16 bh = (_Float16)b;
    a1[t][kNF - 1] = h ? (_Float16)(b - (float)bh) : bh;
#pragma unroll
    for (int sl = 0; sl < 4; ++sl) {
      const int t2 = sl >> 1, g = sl & 1;
#pragma unroll
      for (int jv = 0; jv < 8; ++jv) {
        const int unit = 32 * t2 + 16 * g + 8 * (jv >> 2) + 4 * h + (jv & 3);
        a2[t][sl][jv] = (_Float16)params[kOffW2 + orow * kNH + unit];
      }
    }
  }
  // output layer: w3 in every row, contraction permuted as for layer 2
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    const int t2 = sl >> 1, g = sl & 1;
#pragma unroll
    for (int jv = 0; jv < 8; ++jv)
      a3[sl][jv] = (_Float16)params[kOffW3 + 32 * t2 + 16 * g + 8 * (jv >> 2) + 4 * h + (jv & 3)];
  }
  const float b3 = params[kOffB3];
  double F0[9], F1[9], F2[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    F0[k] = row[k];
    F1[k] = row[9 + k];
    F2[k] = row[18 + k];
  }
  const float icxi = (float)row[kSnapInvC + 0], icyi = (float)row[kSnapInvC + 1];
  const float icxj = (float)row[kSnapInvC + 2], icyj = (float)row[kSnapInvC + 3];
  const float fb0 = (float)row[kSnapFbar + 0], fb1 = (float)row[kSnapFbar + 1], fb2 = (float)row[kSnapFbar + 2];

  __syncthreads();  // s_b2 written
  constexpr int kStride = kInferThreads;  // matches per iteration of the workgroup
  float wsum = 0.f;
  int m = wid * kWave + lane;
  int idx = start + (m < cnt ? m : 0);
  float x1 = X1[idx], y1 = Y1[idx], x2 = X2[idx], y2 = Y2[idx];
  for (int base = wid * kWave; base < cnt; base += kStride) {
    const bool valid = m < cnt;
    const int cur = idx;
    const float cx1 = x1, cy1 = y1, cx2 = x2, cy2 = y2;
    // prefetch the next iteration's match
    m += kStride;
    idx = start + (m < cnt ? m : 0);
    x1 = X1[idx];
    y1 = Y1[idx];
    x2 = X2[idx];
    y2 = Y2[idx];
    float f[8];
    f[0] = res_feature(eps_at(F0, cx1, cy1, cx2, cy2), fb0);
    f[1] = res_feature(eps_at(F1, cx1, cy1, cx2, cy2), fb1);
    f[2] = res_feature(eps_at(F2, cx1, cy1, cx2, cy2), fb2);
    f[3] = fmaf(cx1, icxi, -1.f);
    f[4] = fmaf(cy1, icyi, -1.f);
    f[5] = fmaf(cx2, icxj, -1.f);
    f[6] = fmaf(cy2, icyj, -1.f);
    f[7] = ang;
    if (STORE_FEAT && valid) {
      float4* fo = reinterpret_cast<float4*>(feat_out + (int64_t)cur * kNF);
      fo[0] = make_float4(f[0], f[1], f[2], f[3]);
      fo[1] = make_float4(f[4], f[5], f[6], f[7]);
    }
    // features 0..6 as fp16 parts x = hi + lo and the one that carries the
    // bias, packed in pairs
    u32x4 fhi, flo;
    f[7] = 1.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f16x2 hv = __builtin_convertvector((f32x2){f[2 * q], f[2 * q + 1]}, f16x2);
      fhi[q] = __builtin_bit_cast(unsigned, hv);
      flo[q] = pk_f16(f[2 * q] - (float)hv[0], q < 3 ? f[2 * q + 1] - (float)hv[1] : 1.f);
    }
    // lanes l and l^32 trade parts: group A = matches of lanes 0..31,
    // group B = lanes 32..63; lanes < 32 supply hi, lanes >= 32 lo
    u32x4 recv;
    swap_half(fhi, flo, h != 0, recv);
    float zg[2];
#pragma unroll
    for (int grp = 0; grp < 2; ++grp) {
      // group A: h=0 own hi, h=1 the partner's lo; group B: h=0 the
      // partner's hi, h=1 own lo
      const u32x4 xv = (grp == 0) ? (h ? recv : fhi) : (h ? flo : recv);
      const f16x8 bx = __builtin_bit_cast(f16x8, xv);
      f32x16 acc1[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) acc1[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a1[t], bx, (f32x16){}, 0, 0, 0);
      f16x8 hb[4];
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) hb[sl] = relu_slice(acc1[sl >> 1], 8 * (sl & 1));
      f32x16 acc2[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        acc2[t] = *reinterpret_cast<const f32x16*>(&s_b2[t][h][0]);
#pragma unroll
        for (int sl = 0; sl < 4; ++sl)
          acc2[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a2[t][sl], hb[sl], acc2[t], 0, 0, 0);
      }
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) hb[sl] = relu_slice(acc2[sl >> 1], 8 * (sl & 1));
      f32x16 acc3 = {};
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) acc3 = __builtin_amdgcn_mfma_f32_32x32x16_f16(a3[sl], hb[sl], acc3, 0, 0, 0);
      zg[grp] = acc3[0];  // every row of the output tile is the logit
    }
    // lane l's own match is in group h
    const float w = sigmoidf_((h ? zg[1] : zg[0]) + b3);
    if (valid) {
      const _Float16 wh = (_Float16)w;
      Wout[cur] = __builtin_bit_cast(unsigned short, wh);
      wsum += (float)wh;  // the weight as stored
    }
  }
  wsum = wave_sum_f32(wsum);
  if (lane == 0) s_sum[wid] = wsum;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < kInferThreads / kWave; ++w) s += (double)s_sum[w];
    item_wsum[item] = s;
  }
}

// ---- training ---------------------------------------------------------------

constexpr int kTrainThreads = 64;

// Sample k of batch b: ((b*B + k) * stride) mod n, a bijection of [0, n) when
// gcd(stride, n) = 1, so an epoch visits every sample once (n, stride < 2^31,
// so the product fits in 64 bits).
__device__ __forceinline__ int64_t sample_index(int64_t b, int64_t k, int64_t B, int64_t stride, int64_t n) {
  const uint64_t pos = (uint64_t)(b * B + k) % (uint64_t)n;
  return (int64_t)((pos * (uint64_t)stride) % (uint64_t)n);
}

// Forward + backward of the BCE loss for one batch chunk of kTrainThreads
// samples (one wave); writes this workgroup's gradient partial (kMlpParams
// floats) and loss partial.  The per-sample gradient is scaled by inv_total
// (1/batch).  W2 is read from global memory (16 KB, cache-resident).
__global__ __launch_bounds__(kTrainThreads) void k_mlp_fwd_bwd(
    const float* __restrict__ feat, const float* __restrict__ target, int64_t n, int64_t batch_begin,
    int64_t batch_size, int64_t stride, int64_t batch_index, const float* __restrict__ params,
    float inv_total, float* __restrict__ gpart, double* __restrict__ lpart) {
  const float* __restrict__ sW2 = params + kOffW2;
  __shared__ float sH1[kTrainThreads][kNH + 1];
  __shared__ float sH2[kTrainThreads][kNH + 1];  // later reused for dL/dh1
  __shared__ float sD2[kTrainThreads][kNH + 1];
  __shared__ float sX[kTrainThreads][kNF];
  __shared__ float sDz[kTrainThreads];
  __shared__ double sL[kTrainThreads / kWave];
  const int tid = threadIdx.x;
  const int64_t local = (int64_t)blockIdx.x * kTrainThreads + tid;
  const bool valid = local < batch_size;
  const int64_t s = valid ? sample_index(batch_index, local, batch_size, stride, n) : 0;
  float x[kNF];
#pragma unroll
  for (int k = 0; k < kNF; ++k) {
    x[k] = valid ? feat[s * kNF + k] : 0.f;
    sX[tid][k] = x[k];
  }
  const float t = valid ? target[s] : 0.f;
  __syncthreads();
  float h1[kNH];
#pragma unroll
  for (int i = 0; i < kNH; ++i) {
    float z = params[kOffB1 + i];
#pragma unroll
    for (int k = 0; k < kNF; ++k) z = fmaf(params[i * kNF + k], x[k], z);
    h1[i] = fmaxf(z, 0.f);
    sH1[tid][i] = h1[i];
  }
  float z3 = params[kOffB3];
  float h2[kNH];
  for (int i = 0; i < kNH; ++i) {
    float z = params[kOffB2 + i];
#pragma unroll
    for (int k = 0; k < kNH; ++k) z = fmaf(sW2[i * kNH + k], h1[k], z);
    h2[i] = fmaxf(z, 0.f);
    sH2[tid][i] = h2[i];
    z3 = fmaf(params[kOffW3 + i], h2[i], z3);
  }
  // stable BCE: max(z,0) - z t + log(1 + exp(-|z|))
  const double li = valid ? (double)(fmaxf(z3, 0.f) - z3 * t + log1pf(__expf(-fabsf(z3)))) : 0.0;
  const float dz = valid ? (sigmoidf_(z3) - t) * inv_total : 0.f;
  sDz[tid] = dz;
  float d2[kNH];
#pragma unroll
  for (int i = 0; i < kNH; ++i) {
    d2[i] = h2[i] > 0.f ? dz * params[kOffW3 + i] : 0.f;
    sD2[tid][i] = d2[i];
  }
  __syncthreads();  // sH2 fully written and read for dw3 below before reuse
  // dw3 and b3 partials need h2 of every sample: one thread per hidden unit
  float gw3 = 0.f, gb3 = 0.f;
  if (tid < kNH)
    for (int q = 0; q < kTrainThreads; ++q) gw3 = fmaf(sDz[q], sH2[q][tid], gw3);
  if (tid == 0)
    for (int q = 0; q < kTrainThreads; ++q) gb3 += sDz[q];
  __syncthreads();
  // dL/dh1 (masked by ReLU) into the sH2 slot
  for (int k = 0; k < kNH; ++k) {
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < kNH; ++i) acc = fmaf(sW2[i * kNH + k], d2[i], acc);
    sH2[tid][k] = h1[k] > 0.f ? acc : 0.f;
  }
  // loss partial
  double lw = wave_sum_f64(li);
  if ((tid & 63) == 0) sL[tid >> 6] = lw;
  __syncthreads();
  float* gp = gpart + (int64_t)blockIdx.x * kMlpParams;
  // dW2[i][k] = sum_q D2[q][i] H1[q][k]
  for (int e = tid; e < kNH * kNH; e += kTrainThreads) {
    const int i = e / kNH, k = e % kNH;
    float acc = 0.f;
    for (int q = 0; q < kTrainThreads; ++q) acc = fmaf(sD2[q][i], sH1[q][k], acc);
    gp[kOffW2 + e] = acc;
  }
  // dW1[i][k] = sum_q D1[q][i] X[q][k]; db1, db2
  for (int e = tid; e < kNH * kNF; e += kTrainThreads) {
    const int i = e / kNF, k = e % kNF;
    float acc = 0.f;
    for (int q = 0; q < kTrainThreads; ++q) acc = fmaf(sH2[q][i], sX[q][k], acc);
    gp[e] = acc;
  }
  if (tid < kNH) {
    float a = 0.f, b = 0.f;
    for (int q = 0; q < kTrainThreads; ++q) {
      a += sH2[q][tid];
      b += sD2[q][tid];
    }
    gp[kOffB1 + tid] = a;
    gp[kOffB2 + tid] = b;
    gp[kOffW3 + tid] = gw3;
  }
  if (tid == 0) {
    gp[kOffB3] = gb3;
    double L = 0.0;
    for (int w = 0; w < kTrainThreads / kWave; ++w) L += sL[w];
    lpart[blockIdx.x] = L;
  }
}

// grad[p] = sum over workgroups of their partial (fixed order); the loss
// sum times `scale` is added to loss_acc[0] (accumulate) or stored there.
__global__ void k_mlp_grad_reduce(int n_parts, const float* __restrict__ gpart, float* __restrict__ grad,
                                  const double* __restrict__ lpart, double* __restrict__ loss_acc, int accumulate,
                                  double scale) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kMlpParams) {
    float s = 0.f;
    for (int w = 0; w < n_parts; ++w) s += gpart[(int64_t)w * kMlpParams + p];
    grad[p] = s;
  }
  if (p == 0) {
    double L = 0.0;
    for (int w = 0; w < n_parts; ++w) L += lpart[w];
    loss_acc[0] = accumulate ? loss_acc[0] + L * scale : L * scale;
  }
}

__global__ void k_mlp_adam(float* __restrict__ params, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ grad, float lr, float b1, float b2, float eps, float bc1,
                           float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  const float g = grad[p];
  const float mm = b1 * m[p] + (1.f - b1) * g;
  const float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  params[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

}  // namespace

hipError_t launch_mlp_weights(fea_ctx* c, const float* params, unsigned short* wout, double* item_wsum,
                              float* feat_out) {
  if (c->n_items == 0) return hipSuccess;
  const int b = c->cur;
  Snap3 sn{c->Rh.as<double>(),  c->Th.as<double>(),  c->Fh.as<double>(),  c->Rh1.as<double>(), c->Th1.as<double>(),
           c->Fh1.as<double>(), c->Rh2.as<double>(), c->Th2.as<double>(), c->Fh2.as<double>()};
  k_snap3<<<(unsigned)((c->P + kPairThreads - 1) / kPairThreads), kPairThreads, 0, c->stream>>>(
      (int32_t)c->P, c->d_pair_i.as<int32_t>(), c->d_pair_j.as<int32_t>(), c->d_pair_scene.as<int32_t>(), sn,
      c->d_cx.as<double>(), c->d_cy.as<double>(), c->d_fbar.as<float>(), c->S, c->stab.as<double>());
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
#define FEA_MLP_ARGS                                                                                       \
  c->lay[b][0].as<float>(), c->lay[b][1].as<float>(), c->lay[b][2].as<float>(), c->lay[b][3].as<float>(), \
      c->item_rec.as<int4>(), c->stab.as<double>(), params, wout, item_wsum
  if (feat_out)
    k_mlp_weights<true><<<(unsigned)c->n_items, kInferThreads, 0, c->stream>>>(FEA_MLP_ARGS, feat_out);
  else
    k_mlp_weights<false><<<(unsigned)c->n_items, kInferThreads, 0, c->stream>>>(FEA_MLP_ARGS, nullptr);
#undef FEA_MLP_ARGS
  return hipGetLastError();
}

// One training step on `batch` samples: gradient (fixed-order reduction of
// per-workgroup partials) then Adam (step index t, 1-based).
hipError_t mlp_train_step(hipStream_t st, const float* feat, const float* target, int64_t n, int64_t batch,
                          int64_t stride, int64_t batch_index, float* params, float* m, float* v,
                          float* gpart, double* lpart, float* grad, double* loss_acc, float lr, int64_t t) {
  const int parts = (int)((batch + kTrainThreads - 1) / kTrainThreads);
  k_mlp_fwd_bwd<<<parts, kTrainThreads, 0, st>>>(feat, target, n, 0, batch, stride, batch_index, params,
                                                 1.f / (float)batch, gpart, lpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_mlp_grad_reduce<<<(kMlpParams + 255) / 256, 256, 0, st>>>(parts, gpart, grad, lpart, loss_acc, 1, 1.0);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.f - powf(b1, (float)t), bc2 = 1.f - powf(b2, (float)t);
  k_mlp_adam<<<(kMlpParams + 255) / 256, 256, 0, st>>>(params, m, v, grad, lr, b1, b2, 1e-8f, bc1, bc2);
  return hipGetLastError();
}

// Gradient only (no update) of the mean BCE over samples [0, n) in order
// (stride 1, one batch): used to check the kernels against the oracle.
hipError_t mlp_grad_once(hipStream_t st, const float* feat, const float* target, int64_t n, const float* params,
                         float* gpart, double* lpart, float* grad, double* loss_acc) {
  const int parts = (int)((n + kTrainThreads - 1) / kTrainThreads);
  k_mlp_fwd_bwd<<<parts, kTrainThreads, 0, st>>>(feat, target, n, 0, n, 1, 0, params, 1.f / (float)n, gpart,
                                                 lpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_mlp_grad_reduce<<<(kMlpParams + 255) / 256, 256, 0, st>>>(parts, gpart, grad, lpart, loss_acc, 1, 1.0);
  return hipGetLastError();
}

int mlp_train_threads() { return kTrainThreads; }

// ---- gradient without allocation ------------------------------------------
// Workspace of fea_mlp_grad_noalloc: the per-workgroup loss partials
// (double [kNoAllocParts]) then the gradient partials (float [kNoAllocParts *
// kMlpParams]), one copy per GPU for the life of the process.  Host code uses
// it only through the device address hipGetSymbolAddress returns for the
// current device (the array's own name is a host-side stand-in).
constexpr int64_t kNoAllocParts = kMlpNoAllocMaxSamples / kTrainThreads;
constexpr size_t kScratchLpartBytes = (size_t)kNoAllocParts * sizeof(double);
constexpr size_t kScratchBytes = kScratchLpartBytes + (size_t)kNoAllocParts * kMlpParams * sizeof(float);
static_assert(kMlpNoAllocMaxSamples % kTrainThreads == 0, "whole workgroups");
static_assert(kScratchLpartBytes % 256 == 0, "gradient partials start 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// The device address of this GPU's workspace (looked up once per device,
// with that device current).
hipError_t mlp_scratch(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
  return hipSuccess;
}

}  // namespace fea

extern "C" fea_status fea_mlp_grad_noalloc(int32_t device, void* hip_stream, const float* feat_dev,
                                           const float* target_dev, int64_t n, const float* params_dev,
                                           float* grad_dev, double* loss_dev) {
  using namespace fea;
  if (!feat_dev || !target_dev || !params_dev || !grad_dev) return FEA_EINVAL;
  if (n < 1 || n > kMlpNoAllocMaxSamples) return FEA_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FEA_EINVAL;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) return FEA_EDEVICE;
  if (prev != device && hipSetDevice(device) != hipSuccess) return FEA_EDEVICE;
  fea_status st = FEA_OK;
  unsigned char* ws = nullptr;
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (mlp_scratch(device, &ws) != hipSuccess) {
    st = FEA_EDEVICE;
  } else {
    double* lpart = reinterpret_cast<double*>(ws);
    float* gpart = reinterpret_cast<float*>(ws + kScratchLpartBytes);
    const int parts = (int)((n + kTrainThreads - 1) / kTrainThreads);
    k_mlp_fwd_bwd<<<parts, kTrainThreads, 0, s>>>(feat_dev, target_dev, n, 0, n, 1, 0, params_dev,
                                                  1.f / (float)n, gpart, lpart);
    if (hipGetLastError() != hipSuccess) st = FEA_EDEVICE;
    if (st == FEA_OK) {
      // loss_dev may be NULL: the loss then goes to the workspace's first slot
      k_mlp_grad_reduce<<<(kMlpParams + 255) / 256, 256, 0, s>>>(parts, gpart, grad_dev, lpart,
                                                                  loss_dev ? loss_dev : lpart, 0, 1.0 / (double)n);
      if (hipGetLastError() != hipSuccess) st = FEA_EDEVICE;
    }
  }
  if (prev != device) (void)hipSetDevice(prev);
  return st;
}
