// Host-side context of libfastea and the launchers of its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fastea.h"

namespace fea {

// Device layout of the per-match stream: structure-of-arrays of raw pixel
// coordinates (x1, y1, x2, y2 as fp32), sorted by camera pair, each pair's
// run starting at a multiple of kAlign matches so that 16-byte vector loads
// stay aligned.  A work item is a run of at most tile_matches matches of one
// pair; one workgroup of the per-match kernel processes one item.
constexpr int kVec = 4;
constexpr int kAlign = 4;
constexpr int kFilterThreads = 256;
constexpr int kPartStride = 10;  // per item: dL/dF (9, centred coords) and the loss

// Work-item shapes of the per-match kernel: threads per workgroup and 16-byte
// loads per thread per array; matches per item = threads * 4 * steps.
struct TileCfg {
  int threads, steps;
};
constexpr TileCfg kTiles[] = {{256, 4}, {256, 2}, {256, 1}, {128, 8},
                              {128, 4}, {128, 2}, {512, 2}, {512, 4}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);
constexpr int kGraphSteps = 10;  // steps per captured graph (even: the pose parity is preserved)
constexpr int tile_matches_of(int cfg) { return kTiles[cfg].threads * kVec * kTiles[cfg].steps; }

// Thin owner of one device allocation.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

// Error bits raised by the validation kernel.
enum : int { kErrSameCam = 1, kErrRange = 2, kErrNonFinite = 4 };

}  // namespace fea

struct fea_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  fea_options opt{};
  std::string err;

  // intrinsics (host)
  bool have_intr = false;
  int32_t N = 0, G = 0;
  std::vector<double> f_in, cx, cy;
  std::vector<int32_t> group, grp_off, grp_cams;

  // matches
  bool have_matches = false;
  int64_t M = 0;
  int64_t P = 0;
  std::vector<int32_t> pair_i, pair_j;  // lexicographic pair table
  std::vector<int64_t> seg_off;         // full sorted ranges [P+1]
  std::vector<int32_t> cam_off, cam_ent;  // camera -> (pair*2 + side)
  std::vector<int64_t> phys_off, cur_len;  // current layout per pair
  int64_t layout_len = 0;                  // current layout length (matches)
  int cur = 0;                             // which layout buffer is live (0 = full)

  // items of the current layout
  int64_t n_items = 0;
  std::vector<int32_t> h_item_pair, h_item_start, h_item_count, h_pair_item_off;
  int tile_cfg = 0;        // index into kTiles
  bool tile_tuned = false; // tile_cfg chosen for this set of matches
  std::vector<int32_t> h_cam_ent4;  // per camera entry: {2n+side, item_begin, item_end, other}

  // scenes: a partition of the cameras into independent problems solved
  // together (each with its own gauge, Z, threshold and loss)
  int32_t S = 1;
  std::vector<int32_t> cam_scene;   // [N]
  std::vector<int32_t> pair_scene;  // [P]
  std::vector<int64_t> Zs;          // retained matches per scene
  std::vector<double> taus;         // threshold per scene, normalised units

  // poses
  bool have_poses = false;
  int pcur = 0;
  std::vector<double> gauge_c;  // [3S] applied gauge centre per scene
  std::vector<double> gauge_s;  // [S] applied gauge scale per scene

  // round state
  int round = -1;
  int step = 0;
  int64_t adam_t = 0;      // Adam step count since the moments were last zeroed
  double lr_scale = 1.0;   // lr_decay^round
  bool all_single = true;  // every intrinsics group has one camera
  int64_t Z = 0;
  double tau = 0.0;
  int64_t global_step = 0;
  int32_t n_logged = 0;

  // device buffers
  fea::DBuf lay[3][4];   // x1, y1, x2, y2 (fp32): [0] full layout, [1]/[2] filtered (ping-pong)
  fea::DBuf lpos[3];     // int32: sorted position of each layout entry (-1 = padding)
  fea::DBuf perm;        // int32 [M] input index of each sorted position
  fea::DBuf swp;         // uint8 [M]
  fea::DBuf item_pair, item_start, item_count, pair_item_off, item_keep, item_base;
  fea::DBuf part;        // double [n_items * kPartStride]
  fea::DBuf d_pair_i, d_pair_j, d_cam_off, d_cam_ent, d_group, d_grp_off, d_grp_cams;
  fea::DBuf d_cx, d_cy;
  fea::DBuf d_pair_scene, d_inv_z, d_tau;  // int32 [P], float [S], double [S]
  fea::DBuf a6, tp, logf, m_a6, v_a6, m_t, v_t, m_f, v_f;
  fea::DBuf R[2], T[2], Fc[2];  // derived current/next R (N*9), t (N*3), f (N)
  fea::DBuf Rh, Th, Fh;         // round snapshot
  fea::DBuf gR, gt, gf, loss_cam, loss;
  fea::DBuf logR;
  fea::DBuf errflag;
  fea::DBuf Re, Te, Fe;  // poses built from caller-given parameters
  fea::DBuf counters;    // int64 [4]: Adam step count and global step count, two parities

  // captured step graph (kGraphSteps steps of the current round)
  hipGraphExec_t graph = nullptr;
  int graph_pcur = -1;

  // kernel timing (HIP events around each per-match pass)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
};

namespace fea {

// --- segmenting (fea_segment.hip) ---
// Validates matches, builds canonical pair keys, stable-sorts by key and
// writes the sorted pair table.  Returns hipSuccess or an error; sets
// *bad_bits to the validation error bits.
hipError_t segment_matches(fea_ctx* c, const float* x1, const float* y1, const float* x2, const float* y2,
                           const int32_t* cam1, const int32_t* cam2, int* bad_bits);

// --- per-match pass (fea_resgrad.hip) ---
hipError_t launch_resgrad(fea_ctx* c);
hipError_t launch_resgrad_cfg(fea_ctx* c, int cfg);
hipError_t launch_resgrad_at(fea_ctx* c, int cfg, const double* R, const double* T, const double* F,
                             bool loss_only);
hipError_t launch_filter_count(fea_ctx* c);
hipError_t launch_filter_scatter(fea_ctx* c, int dst);

// --- per-camera epilogue (fea_camera.hip) ---
hipError_t launch_camgrad(fea_ctx* c, int do_update);
hipError_t launch_focal_update(fea_ctx* c);
hipError_t launch_loss_sum(fea_ctx* c);
hipError_t launch_camgrad_at(fea_ctx* c, const double* R, const double* T, const double* F);

// --- parameters given as device arrays (fea_autograd.hip) ---
hipError_t launch_params_to_pose(fea_ctx* c, const double* a6, const double* t, const double* logf);
hipError_t launch_item_loss(fea_ctx* c, double* loss_out);
hipError_t launch_param_grad(fea_ctx* c, const double* a6, const double* gout, double* ga6, double* gt,
                             double* glogf);

}  // namespace fea
