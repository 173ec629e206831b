// Layout constants shared by libfastea's kernels and its host code: the
// per-match stream, the pose table, the per-item partials, the work-item
// shapes of the per-match kernel, the network's parameters and the device
// step counters.
#pragma once

#include <cstdint>

#include "fastea.h"

namespace fea {

// Device layout of the per-match stream: structure-of-arrays of raw pixel
// coordinates (x1, y1, x2, y2 as fp32), sorted by camera pair, each pair's
// run starting at a multiple of kAlign matches: 128 bytes per array, one
// cache line, so that a work item (a run of at most tile_matches matches of
// one pair, tile_matches a multiple of kAlign) starts on a line and 16-byte
// vector loads stay aligned.  One workgroup of the per-match kernel
// processes one item.
constexpr int kVec = 4;
constexpr int kAlign = 32;
constexpr int kFilterThreads = 256;
constexpr int kPartStride = 10;  // per item: dL/dF (9, centred coords) and the loss

// Pose table: one row of kPairRow doubles per camera pair.  F (current poses)
// and F_hat (round snapshot) are the pair's epipolar matrices folded for raw
// pixel coordinates; then the scene's 1/Z for plain and learned weights, the
// learned flag, the principal points (cx_i, cy_i, cx_j, cy_j) and tau.
constexpr int kRowF = 0, kRowFh = 9, kRowInvZ = 18, kRowInvZw = 19, kRowMode = 20, kRowCx = 21,
              kRowTau = 25;
constexpr int kPairRow = 32;
constexpr int kPairThreads = 256;
// Scenes up to this many cameras take the device round start (median of
// their focal lengths sorted in LDS); larger ones the host path.
constexpr int kMaxSceneCams = 8192;

// Work-item shapes of the per-match kernel: threads per workgroup and 16-byte
// loads per thread per array (matches per item = threads * 4 * steps), and
// whether the launch is persistent: as many workgroups per CU as can reside
// at once, each walking the items with the next item's loads in flight,
// instead of one workgroup per item.
struct TileCfg {
  int threads, steps;
  bool persistent;
};
constexpr TileCfg kTiles[] = {{256, 4, false}, {256, 2, false}, {256, 1, false}, {128, 8, false},
                              {128, 4, false}, {128, 2, false}, {512, 2, false}, {512, 4, false},
                              {256, 2, true},  {256, 1, true},  {128, 2, true},  {512, 1, true},
                              {512, 2, true}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);
constexpr int kGraphSteps = 10;  // steps per captured graph (even: the pose parity is preserved)

// Learned inlier weights: MLP 8 -> 64 -> 64 -> 1, parameters packed as
// W1 [64*8], b1 [64], W2 [64*64], b2 [64], w3 [64], b3.
constexpr int kMlpFeat = 8;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = kMlpHidden * kMlpFeat + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpHidden + 1;
// Largest sample count of fea_mlp_grad_noalloc (its workspace holds one
// gradient partial per 64 samples: 1,024 x 4,801 floats, about 19.7 MB).
constexpr int64_t kMlpNoAllocMaxSamples = FEA_MLP_NOALLOC_MAX_SAMPLES;
constexpr int tile_matches_of(int cfg) { return kTiles[cfg].threads * kVec * kTiles[cfg].steps; }

// Device-side step counters, one slot per pose parity p (see the camera
// kernel): Adam steps since the moments were zeroed, global steps, and the
// running powers beta1^t, beta2^t of the bias corrections.
struct StepCounters {
  long long adam_t[2];
  long long global_t[2];
  double b1t[2];
  double b2t[2];
  double lr_scale;  // learning-rate factor of the round (lr_decay^round)
};

}  // namespace fea
