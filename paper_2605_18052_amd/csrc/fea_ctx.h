// Host-side context of libfastea and the launchers of its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "fastea.h"
#include "fea_layout.h"

namespace fea {

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
  int n_cu = 256;                         // compute units of the device (persistent launches)
  int quad_steps_cap = -1;                // resident workgroups of k_quad_steps (-1: not asked yet)
  fea::DBuf wait_state;                   // uint32 [2]: arrival count of the device-wide waits, error flag
  unsigned wait_base = 0;                 // arrivals counted so far (the next launch's base)
  int last_quad_blocks = 0;               // workgroups of the last k_quad_steps launch
  int wall_clock_khz = 100000;            // rate of the device's wall clock (wall_clock64)
  std::vector<float> tune_ms;             // the autotuner's mean time per shape of kTiles (last tuning)
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
  std::vector<int32_t> h_item_rec;  // per item {pair, start, count, 0}
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
  std::vector<float> inv_zw_h;      // 1 / sum of retained learned weights per scene

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
  fea::DBuf pair_item_off, item_keep, item_base;
  fea::DBuf item_rec;  // int4 per item: {pair, start, count, 0}
  fea::DBuf d_scene_item_off;  // int32 [S+1]: items of each scene (contiguous)
  fea::DBuf scene_loss;        // double [S]
  bool scene_items_contiguous = true;  // each scene's items form one range
  fea::DBuf part;        // double [n_items * kPartStride]
  fea::DBuf d_pair_i, d_pair_j, d_cam_off, d_cam_ent, d_group, d_grp_off, d_grp_cams;
  fea::DBuf d_cx, d_cy;
  fea::DBuf d_pair_scene, d_inv_z, d_tau;  // int32 [P], float [S], double [S]
  fea::DBuf ptab;  // double [P * kPairRow], the pose table
  bool ptab_current = false;  // the pose table's F is that of the current poses
  fea::DBuf stab;  // double [P * 40]: per-pair rows for the learned features
  fea::DBuf qpart;           // double [n_items * 36]: per-item sums of c P2_s P1_t (quadratic form)
  fea::DBuf qW;              // double [P * 45]: W_n of every pair for the round
  fea::DBuf qmask;           // uint8 [full layout]: retained (the quadratic form keeps the full layout)
  fea::DBuf a6, tp, logf, m_a6, v_a6, m_t, v_t, m_f, v_f;
  fea::DBuf R[2], T[2], Fc[2];  // derived current/next R (N*9), t (N*3), f (N)
  fea::DBuf Rh, Th, Fh;         // round snapshot
  fea::DBuf gR, gt, gf, loss_cam, loss;
  fea::DBuf logR;
  fea::DBuf errflag;
  fea::DBuf Re, Te, Fe;  // poses built from caller-given parameters
  fea::DBuf counters;    // int64 [4]: Adam step count and global step count, two parities

  // learned weights
  fea::DBuf Rh1, Th1, Fh1, Rh2, Th2, Fh2;  // snapshots of the two previous rounds
  fea::DBuf d_fbar;                       // float [3*S]: median f per scene at the 3 snapshots
  fea::DBuf d_fbar_hist;                  // double [3*S]: the same medians in fp64 (device round start)
  fea::DBuf d_scene_cam_off, d_scene_cams;  // int32 [S+1], [N]: cameras of each scene
  fea::DBuf d_scene_z;                    // int64 [S+1]: survivors per scene, total last (quadratic form)
  int32_t max_scene_cams = 0;             // largest scene, in cameras
  bool host_tau_stale = false;            // taus, tau, fbar_hist live on the device until read back
  bool host_z_stale = false;              // Zs, Z live on the device until read back
  int64_t* inl_log = nullptr;             // pinned host: Z of each solver round (64)
  fea::DBuf mlp;                          // float [kMlpParams]
  fea::DBuf wlay;                         // fp16 [layout] learned weight of each layout slot
  fea::DBuf item_wsum;                    // double [n_items]
  fea::DBuf d_inv_zw;                     // float [S]: 1 / sum of learned weights per scene
  fea::DBuf d_scene_mode;                 // int32 [S]: 1 = learned weights this round, 0 = plain
  fea::DBuf a6h, tph, logfh;              // parameters at the round snapshot (judge fallback)
  fea::DBuf d_learned_ok;                 // int32 [S]: 0 once the judge rejected the scene's learned weights
  fea::DBuf d_fallbacks;                  // int32 [S]: the judge's rejections per scene
  fea::DBuf d_judge_l0, d_judge_l1;       // double [S]: plain objective at a learned round's start and end
  bool judge_written = false;             // d_judge_l0/l1 hold a judge pass of the current scenes
  int32_t fallbacks_base = 0;             // rejections restored from a checkpoint (added to d_fallbacks)
  hipEvent_t judge_ev = nullptr;          // recorded after the judge's flags are copied to judge_ok_h
  int32_t* judge_ok_h = nullptr;          // pinned [S]: d_learned_ok as of the last judge
  int32_t judge_ok_cap = 0;               // capacity of judge_ok_h
  bool judge_pending = false;             // judge_ok_h not yet read since judge_ev was recorded

  // per-scene early exit (options.converge_deg > 0)
  fea::DBuf d_cam_scene;                  // int32 [N]: scene of each camera
  fea::DBuf d_scene_done;                 // int32 [S]: 0 active, r + 1 once converged at round r,
                                          // -(r + 1) once stopped by the non-finite guard at round r
  fea::DBuf d_scene_change;               // double [S]: largest camera rotation over the last round, degrees
  std::vector<int32_t> scene_done_h;      // host copy of d_scene_done (read at every round start)
  int32_t n_done = 0;                     // converged or stopped scenes (read at round starts with converge_deg)
  int32_t n_nonfinite = 0;                // scenes the non-finite guard had stopped at the last check
  double prev_tau_px = -1.0;              // threshold of the previous round, pixels (-1: none yet)
  fea::DBuf d_scene_loss_log;             // double [64 * S]: each scene's loss at the end of each round
  fea::DBuf d_scene_z_log;                // int64 [64 * S]: each scene's retained matches in each round
  bool have_mlp = false;
  bool learned_any = false;               // some scene uses learned weights this round
  std::vector<int32_t> scene_mode;        // host copy of d_scene_mode
  std::vector<int32_t> scene_learned_ok;  // 0 once the judge rejected a scene's learned round
  int32_t fallbacks = 0;                  // rejected learned rounds (all scenes)
  std::vector<double> fbar_hist;          // [3*S] median f per scene, snapshots r, r-1, r-2

  // captured step graph (kGraphSteps steps of the current round)
  hipGraphExec_t graph = nullptr;
  int graph_pcur = -1;
  uint64_t graph_gen = 0;  // device-buffer generation the graph was captured at

  // pinned staging ring for small host-to-device copies
  void* stage = nullptr;
  size_t stage_used = 0;
  double* loss_log = nullptr;  // pinned host: loss at the end of each solver round (64)

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
hipError_t export_sorted(fea_ctx* c, int32_t cam_base, const int64_t* seg_off_dev, float* x1, float* y1,
                         float* x2, float* y2, int32_t* cam1, int32_t* cam2);

// --- per-match pass (fea_resgrad.hip) ---
hipError_t launch_pair_pose(fea_ctx* c, const double* R, const double* T, const double* F, bool snap);
hipError_t launch_resgrad_kernel(fea_ctx* c, int cfg, bool loss_only, bool force_plain);
void prepare_resgrad(int cfg);
hipError_t launch_resgrad(fea_ctx* c, bool step = false);
hipError_t launch_resgrad_cfg(fea_ctx* c, int cfg);
hipError_t launch_resgrad_at(fea_ctx* c, int cfg, const double* R, const double* T, const double* F,
                             bool loss_only, bool force_plain);
hipError_t launch_filter_count(fea_ctx* c, const uint32_t* mask);
hipError_t launch_filter_scatter(fea_ctx* c, int dst, const uint32_t* mask);

// --- per-camera epilogue (fea_camera.hip) ---
hipError_t launch_camgrad(fea_ctx* c, int do_update, bool quad);
hipError_t launch_quad_build(fea_ctx* c);
hipError_t launch_mask_init(fea_ctx* c);
hipError_t launch_mask_slots(fea_ctx* c, int32_t* slot_pos);
hipError_t launch_quad_reduce(fea_ctx* c, const int32_t* pair_item_off_dev);
hipError_t launch_focal_update(fea_ctx* c);
hipError_t launch_loss_sum(fea_ctx* c);
hipError_t launch_judge(fea_ctx* c);
hipError_t launch_choose_mode(fea_ctx* c, bool enabled);
hipError_t launch_round_start(fea_ctx* c, bool shift, bool first, bool zero);
hipError_t launch_scene_tau(fea_ctx* c, double tau_px, bool first);
hipError_t launch_scene_z(fea_ctx* c);
hipError_t launch_scene_loss(fea_ctx* c, double* out = nullptr, double* out_snap = nullptr);
hipError_t launch_scene_converge(fea_ctx* c, bool check, int32_t round);
hipError_t launch_guard(fea_ctx* c, int32_t round);
hipError_t launch_scene_loss_log(fea_ctx* c, int32_t round);
hipError_t run_ablation(fea_ctx* c, int variant, int reps, double* ms, float* pair_sum_dev);
hipError_t launch_camgrad_at(fea_ctx* c, const double* R, const double* T, const double* F);
int quad_steps_blocks(fea_ctx* c);
hipError_t launch_quad_steps(fea_ctx* c, int n_steps, int blocks);

// --- parameters given as device arrays (fea_autograd.hip) ---
hipError_t launch_params_to_pose(fea_ctx* c, const double* a6, const double* t, const double* logf);
hipError_t launch_item_loss(fea_ctx* c, double* loss_out);
hipError_t launch_param_grad(fea_ctx* c, const double* a6, const double* gout, double* ga6, double* gt,
                             double* glogf);

// --- learned weights (fea_mlp.hip) ---
hipError_t launch_mlp_weights(fea_ctx* c, const float* params, unsigned short* wout, double* item_wsum,
                              float* feat_out);
hipError_t mlp_train_step(hipStream_t st, const float* feat, const float* target, int64_t n, int64_t batch,
                          int64_t stride, int64_t batch_index, float* params, float* m, float* v, float* gpart,
                          double* lpart, float* grad, double* loss_acc, float lr, int64_t t);
hipError_t mlp_grad_once(hipStream_t st, const float* feat, const float* target, int64_t n, const float* params,
                         float* gpart, double* lpart, float* grad, double* loss_acc);
int mlp_train_threads();

}  // namespace fea
