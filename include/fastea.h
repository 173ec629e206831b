/*
 * fastea -- MI355X (gfx950) epipolar adjustment for FastMap-style
 * structure from motion.  C ABI.
 *
 * The library refines world-to-camera camera poses (R_i, t_i) and focal
 * lengths f_i by minimising the IRLS-reweighted epipolar objective of the
 * FastMap chapter (Method > Optimization Formulations > Epipolar Adjustment,
 * Eq. fastmap-epipolar-objective and the re-weighted objective after
 * Eq. fastmap-epipolar-objective-l2), over millions of keypoint matches on
 * one GPU.  For a pair of cameras i < j:
 *     R_ij = R_j R_i^T,  t_ij = t_j - R_ij t_i,  u = t_ij / |t_ij|,
 *     E = [u]x R_ij,  F = D_j E D_i,  D_k = diag(1/f_k, 1/f_k, 1),
 * and a match with centred pixel coordinates p1 = (x1-cx_i, y1-cy_i, 1) in
 * camera i and p2 in camera j has residual eps = p2^T F p1 (the epipolar
 * error in normalised homogeneous coordinates).  Each IRLS round freezes the
 * poses (snapshot), drops matches with |eps_hat| >= tau (threshold schedule
 * decreasing to a minimum), and minimises
 *     L = (1/Z) sum_m eps_m^2 / max(|eps_hat_m|, delta)
 * over the Z retained matches with Adam steps (rotations in the 6D
 * representation, focal lengths as log f per intrinsics group).
 *
 * Conventions
 *   - Every function returns a fea_status (0 = success, < 0 = error) and
 *     never aborts or throws; fea_last_error() describes the last failure.
 *   - Arrays are row-major; R is 3x3 world-to-camera; t is 3.
 *   - Host pointers are read (or written) during the call only; the caller
 *     keeps ownership.  Device pointers ("_dev") are borrowed for the call and
 *     must be device memory of the context's GPU.
 *   - A context is not thread-safe; separate contexts are independent.
 *     All device work is issued on the context's HIP stream.
 *   - Call order: fea_create -> fea_load_intrinsics -> fea_load_matches* ->
 *     fea_init_poses -> (fea_epipolar_adjust | fea_begin_round/fea_step ...)
 *     -> fea_get_poses.  Out-of-order calls return FEA_ESTATE.
 */
#ifndef FASTEA_H
#define FASTEA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FEA_VERSION 100 /* 0.1.0 */

typedef struct fea_ctx fea_ctx;

typedef enum {
  FEA_OK = 0,
  FEA_EINVAL = -1,       /* bad argument (null pointer, size, id out of range) */
  FEA_ENOMEM = -2,       /* device or host allocation failed */
  FEA_EDEVICE = -3,      /* HIP runtime error */
  FEA_ESTATE = -4,       /* call out of order */
  FEA_EDEGENERATE = -5,  /* a camera pair with coincident centres (t_ij = 0) */
  FEA_ENONFINITE = -6    /* non-finite input coordinates, poses or focals */
} fea_status;

/* Solver options.  The paper fixes none of these constants; the defaults
 * (fea_default_options) are this library's documented choices. */
typedef struct {
  int32_t rounds;          /* IRLS rounds (default 20) */
  int32_t iters_per_round; /* Adam steps per round (default 50) */
  double tau_px_init;      /* round-0 filter threshold in pixels (128) */
  double tau_px_min;       /* threshold floor in pixels (4) */
  double tau_decay;        /* threshold factor per round (0.5) */
  double delta;            /* weight floor: 1/max(|eps_hat|, delta), normalised units (1e-4) */
  double lr_rot;           /* Adam learning rate of the 6D rotation parameters (3e-3) */
  double lr_t;             /* ... of translations, in the normalised gauge (4e-2) */
  double lr_logf;          /* ... of log focal length per intrinsics group (1e-3) */
  double beta1, beta2;     /* Adam moment decay (0.9, 0.999) */
  double adam_eps;         /* Adam epsilon (1e-12) */
  int32_t optimize_focal;  /* 1: refine focal lengths (default), 0: keep them fixed */
  int32_t gauge_normalize; /* 1: before solving, move camera centres to mean 0
                              and median matched-pair baseline 1 (default);
                              poses are returned in the caller's frame */
  int32_t log_every;       /* >0: keep the rotations every log_every steps (0) */
  int32_t max_log;         /* capacity of that log, in snapshots (0) */
  double lr_decay;         /* learning rates of round r are lr * lr_decay^r (0.9) */
  int32_t reset_moments;   /* 1: zero the Adam moments at every round start (1) */
  int32_t tile_matches;    /* matches per work item of the per-match kernel:
                              1024, 2048, 4096 or 8192; 0 = pick by timing the
                              candidates at the first round, or reuse the pick
                              made earlier in this process for a problem of
                              the same size class; 8192 with inner_loop = 1
                              (0) */
  int32_t use_graphs;      /* 1: issue runs of steps as captured HIP graphs (1) */
  int32_t weight_mode;     /* 0: plain IRLS weights (default); 1: learned
                              inlier weights (fea_set_mlp) judged by the plain
                              objective each round, plain weights as fallback */
  int32_t inner_loop;      /* 0: every step streams the retained matches
                              (per-match residual and gradient, default);
                              1: the weighted quadratic form of each pair,
                              f^T W_n f with W_n summed over its matches once
                              per round, so that a step costs O(pairs) */
  int32_t tile_persistent; /* with tile_matches 1024, 2048 or 4096: 1 takes
                              the persistent launch of that item size (as
                              many workgroups per CU as reside at once, each
                              walking the items with the next item's loads
                              in flight), 0 one workgroup per item (0) */
  int32_t persistent_steps; /* with inner_loop = 1 and every intrinsics
                              group a single camera: 1 runs each call's
                              steps in one cooperative launch (every
                              wavefront takes cameras of each step in turn,
                              and the workgroups wait for each other between
                              steps; the same results as one launch per
                              step), 0 one launch per step (0: on this
                              device the wait between steps costs more
                              than a launch) */
  int32_t wait_limit_us;   /* bound of one device-wide wait between the
                              steps of a persistent launch, microseconds
                              (0: 500,000); a wait that runs past it ends
                              the launch, and the next round boundary
                              reports FEA_EDEVICE (0) */
  double converge_deg;     /* per-scene early exit (0 = off, default): at the
                              start of a round whose threshold equals the
                              previous round's (the schedule at its floor), a
                              scene whose cameras rotated by less than
                              converge_deg degrees on average over the
                              previous round (geodesic distance), and whose
                              mean |log f| change is below
                              converge_deg * pi/180, is
                              converged: it takes no further steps and its
                              poses and optimiser state stay as they are;
                              the solve ends once every scene has converged */
} fea_options;

/* What fea_epipolar_adjust did. */
typedef struct {
  int32_t rounds_run;
  int32_t iters_run;
  int64_t inliers_per_round[64]; /* Z of each round (first 64 rounds) */
  double loss_per_round[64];     /* loss at the last step of each round */
  double ms_total;               /* wall time of the call, milliseconds */
  int32_t n_logged;              /* pose snapshots kept (log_every > 0) */
  int32_t fallbacks;             /* learned rounds rejected by the judge (all scenes) */
  int32_t scenes_converged;      /* scenes the early exit stopped (converge_deg > 0) */
  int32_t scenes_nonfinite;      /* scenes the non-finite guard stopped (see fea_epipolar_adjust) */
  int32_t reserved[4];
} fea_report;

/* Sizes and state of a context. */
typedef struct {
  int32_t n_cams;
  int32_t n_groups;      /* intrinsics groups */
  int64_t n_matches;     /* loaded matches */
  int64_t n_pairs;       /* distinct camera pairs among them */
  int64_t n_retained;    /* matches kept by the current round (Z) */
  int64_t n_items;       /* work items of the per-match pass */
  int64_t layout_matches;/* matches in the device layout incl. alignment padding */
  int32_t round;         /* current round index, -1 before the first */
  int32_t step;          /* Adam steps taken in the current round */
  double gauge_center[3];/* applied gauge: centre' = (centre - gauge_center)/gauge_scale */
  double gauge_scale;
  double tau;            /* current threshold, normalised units */
  int32_t tile_matches;  /* matches per work item of the per-match kernel */
  int32_t tile_threads;  /* threads per workgroup of the per-match kernel */
  int32_t n_scenes;      /* independent scenes in the context (fea_set_scenes) */
  int32_t tile_persistent; /* 0: one workgroup per work item; 1: as many
                              workgroups per CU as reside at once, each
                              walking the items with the next item's loads
                              in flight */
  int32_t quad_steps_blocks; /* workgroups of the last persistent launch of
                              the quadratic form's steps (0: none, the steps
                              ran one launch each) */
  int32_t reserved[3];
} fea_info;

/* Library version (FEA_VERSION of the build). */
int32_t fea_version(void);

/* Human-readable name of a status code (static string). */
const char *fea_status_string(fea_status s);

/* Checks options without a context or a GPU: FEA_OK when fea_create and
 * fea_set_options would accept them, else FEA_EINVAL with the reason written
 * to why (NUL-terminated, at most why_len bytes; why may be NULL).  Besides
 * the ranges documented at each field, learned weights (weight_mode = 1)
 * with the quadratic form (inner_loop = 1) accept tile_matches 0 or 8192
 * only. */
fea_status fea_check_options(const fea_options *opt, char *why, size_t why_len);

/* Fills *out with the default options.  FEA_EINVAL if out is NULL. */
fea_status fea_default_options(fea_options *out);

/* Creates a context on GPU `device` (HIP device index).  opt may be NULL
 * (defaults).  hip_stream: a hipStream_t to issue all work on, or NULL for a
 * stream owned by the context (created at default priority).  On success
 * *out receives the context; release it with fea_destroy. */
fea_status fea_create(fea_ctx **out, int32_t device, const fea_options *opt,
                      void *hip_stream);

/* Releases every resource of the context (NULL is a no-op). */
void fea_destroy(fea_ctx *ctx);

/* Message of the last failed call on this context ("" if none). */
const char *fea_last_error(const fea_ctx *ctx);

/* Replaces the solver options (allowed at any time before fea_epipolar_adjust
 * or fea_begin_round; takes effect from the next round). */
fea_status fea_set_options(fea_ctx *ctx, const fea_options *opt);

/* Camera intrinsics (Method > Intrinsics Estimation: principal point fixed at
 * the image centre, a few physical cameras with shared intrinsics).
 * f, cx, cy: host arrays [n_cams] in pixels, f > 0 and finite.  intr_group:
 * host array [n_cams] of group ids in [0, n_cams), or NULL for one group per
 * camera; cameras of one group share one focal length (initialised to the
 * geometric mean of their f).  Resets any loaded matches and poses. */
fea_status fea_load_intrinsics(fea_ctx *ctx, int32_t n_cams, const double *f,
                               const double *cx, const double *cy, const int32_t *intr_group);

/* Batching: partition the cameras into n_scenes independent scenes solved
 * together (one launch of each kernel covers every scene).  cam_scene: host
 * array [n_cams] of scene ids in [0, n_scenes).  Each scene keeps its own
 * gauge, retained-match count Z, threshold (over its own median focal
 * length) and loss, so the result equals solving the scenes one by one.
 * Call after fea_load_intrinsics and before fea_load_matches; matches must
 * not link two scenes and an intrinsics group must not span scenes
 * (FEA_EINVAL).  The default is one scene. */
fea_status fea_set_scenes(fea_ctx *ctx, int32_t n_scenes, const int32_t *cam_scene);

/* Per-scene state (host arrays [n_scenes], [n_scenes], [3*n_scenes],
 * [n_scenes], [n_scenes]; any may be NULL): loss at the last evaluated step,
 * retained matches of the current round, the applied gauge, and whether the
 * scene still uses learned weights (0 once the judge fell back). */
fea_status fea_get_scene_stats(fea_ctx *ctx, double *loss, int64_t *retained,
                               double *gauge_center, double *gauge_scale, int32_t *learned);

/* The two values the learned-weight judge compared at the end of the last
 * learned round (Method > Epipolar Adjustment, the IRLS objective with the
 * round's plain weights): per scene, host arrays [n_scenes] (either may be
 * NULL), the objective at the round's snapshot poses and at the poses the
 * round ended with, before any restore.  Both come from one pass over the
 * matches.  Zeros before the first learned round.  Synchronises the
 * context's stream. */
fea_status fea_get_judge_losses(fea_ctx *ctx, double *loss_snapshot, double *loss_end);

/* Per-scene convergence (options.converge_deg): converged_round [n_scenes]
 * receives the round at whose start each scene was found converged (it took
 * no steps from that round on), or -1; change_deg [n_scenes] the mean
 * rotation of the scene's cameras over the last completed round, in
 * degrees, as measured at the latest round start (measured only with
 * converge_deg > 0; 0 before the second round).  Host arrays; either may be
 * NULL. */
fea_status fea_get_scene_convergence(fea_ctx *ctx, int32_t *converged_round, double *change_deg);

/* Scenes stopped by the non-finite guard (see fea_epipolar_adjust):
 * stopped_round [n_scenes] (host, not NULL) receives the round at whose start
 * the scene was found non-finite (options.rounds or the rounds run if at the
 * end of the solve), or -1.  Its poses are those of the snapshot taken at
 * the start of the round before. */
fea_status fea_get_scene_nonfinite(fea_ctx *ctx, int32_t *stopped_round);

/* Keypoint matches (Method > Epipolar Adjustment: point pairs Q_n of the
 * image pairs P).  Match m relates pixel (x1[m], y1[m]) of camera cam1[m] to
 * (x2[m], y2[m]) of camera cam2[m].  Host arrays of length n, copied.
 * Errors: FEA_EINVAL if cam1 == cam2 or an id is outside [0, n_cams) or
 * n >= 2^31; FEA_ENONFINITE for a non-finite coordinate.  n = 0 is valid.
 * The library canonicalises every match to cam1 < cam2 (swapping its
 * keypoints) and sorts them by camera pair on the GPU (stable). */
fea_status fea_load_matches(fea_ctx *ctx, int64_t n, const float *x1, const float *y1,
                            const float *x2, const float *y2, const int32_t *cam1,
                            const int32_t *cam2);

/* Same as fea_load_matches, with device arrays (borrowed during the call). */
fea_status fea_load_matches_device(fea_ctx *ctx, int64_t n, const float *x1_dev,
                                   const float *y1_dev, const float *x2_dev,
                                   const float *y2_dev, const int32_t *cam1_dev,
                                   const int32_t *cam2_dev);

/* Initial poses (Method > Optimization Formulations > Epipolar Adjustment:
 * the adjustment starts from the global rotations and translations of the
 * earlier stages and optimises world-to-camera poses): R [n_cams*9]
 * row-major world-to-camera rotations, t [n_cams*3]; host arrays.  Rotations must be proper (det > 0) and finite.
 * Applies the gauge normalisation if enabled and resets the round state.
 * FEA_EDEGENERATE if two matched cameras share a centre. */
fea_status fea_init_poses(fea_ctx *ctx, const double *R, const double *t);

/* Replaces the current poses (caller's frame, host arrays: R [n_cams*9],
 * t [n_cams*3], f [n_cams] or NULL to keep the focal lengths) without
 * touching the round: the snapshot, the retained matches and the Adam moments
 * stay as they are.  Used to evaluate the objective at arbitrary poses and by
 * optimisers that run outside the library.  Requires fea_init_poses. */
fea_status fea_set_poses(fea_ctx *ctx, const double *R, const double *t, const double *f);

/* Starts an IRLS round (re-weighting rounds and outlier filtering of the
 * Epipolar Adjustment paragraph): freezes the current poses as the snapshot,
 * drops matches with |eps_hat| >= tau_px / median(f) (tau_px in pixels; pass
 * INFINITY to keep all), and resets the Adam moments.  Dropped matches stay
 * dropped for the rest of the solve. */
fea_status fea_begin_round(fea_ctx *ctx, double tau_px);

/* One pass of the residual, IRLS weight and gradient at the current poses,
 * with the current round's weights (no parameter update), by the inner loop
 * the options select (per match, or the pairs' quadratic forms).  The
 * objective is the re-weighted one that follows
 * Eq. fastmap-epipolar-objective-l2 (the L1 objective of
 * Eq. fastmap-epipolar-objective approximated by squared residuals over the
 * snapshot's |eps_hat|), with Z the round's retained matches and
 * 1/max(|eps_hat|, delta) as the weight; the gradient is the one the fused
 * kernel of Method > Kernel Fusion computes, taken per match.  Outputs are
 * device arrays, caller-allocated, any of which may be NULL:
 *   loss_dev [1]; gR_dev [n_cams*9] dL/dR (R as an unconstrained 3x3);
 *   gt_dev [n_cams*3] dL/dt; gf_dev [n_cams] dL/df.
 * Derivatives are taken in the gauge the context works in (fea_info). */
fea_status fea_residual_grad(fea_ctx *ctx, double *loss_dev, double *gR_dev, double *gt_dev,
                             double *gf_dev);

/* Autograd support (parameters held by the caller as device arrays, in the
 * context's gauge; see fea_info).  Parameters: a6 [n_cams*6] the 6D rotation
 * parameters (first two columns of R, unnormalised), t [n_cams*3], logf
 * [n_groups] log focal length per intrinsics group.  The objective uses the
 * current round's snapshot and retained matches; the context's own poses
 * and optimiser state are not touched.  All results are written on the
 * context's stream.
 *
 * fea_get_params_dev: the context's current parameters into such arrays
 * (any pointer may be NULL). */
fea_status fea_get_params_dev(fea_ctx *ctx, double *a6_dev, double *t_dev, double *logf_dev);

/* fea_set_params_dev: replaces the context's current parameters with such
 * arrays (device pointers, read on the context's stream before the call's
 * work completes; none may be NULL) and derives the poses from them, e.g.
 * after a caller's own optimiser step.  The Adam moments and the round's
 * snapshot are kept.  The values are not inspected on the host: a
 * non-finite value is caught by the non-finite guard at the next round
 * boundary (fea_begin_round, fea_epipolar_adjust).  FEA_ESTATE before
 * fea_init_poses. */
fea_status fea_set_params_dev(fea_ctx *ctx, const double *a6_dev, const double *t_dev, const double *logf_dev);

/* Forward: loss_dev [1] = L(a6, t, logf), the round's re-weighted epipolar
 * objective (the IRLS form after Eq. fastmap-epipolar-objective-l2) at the
 * caller's parameters. */
fea_status fea_loss_dev(fea_ctx *ctx, const double *a6_dev, const double *t_dev,
                        const double *logf_dev, double *loss_dev);

/* Backward of the same objective (Method > Kernel Fusion: forward and
 * backward fused, here as a hand-written adjoint with the forward recomputed
 * and no per-match state kept):
 * ga6_dev [n_cams*6], gt_dev [n_cams*3], glogf_dev [n_groups] receive
 * gout * dL/d(parameter), gout_dev [1] the upstream gradient (NULL = 1).
 * Output pointers may be NULL. */
fea_status fea_adjoint_dev(fea_ctx *ctx, const double *a6_dev, const double *t_dev,
                           const double *logf_dev, const double *gout_dev, double *ga6_dev,
                           double *gt_dev, double *glogf_dev);

/* ---- Learned inlier weights ------------------------------------------
 * An MLP 8 -> 64 -> 64 -> 1 (ReLU, ReLU, sigmoid) maps each retained match's
 * features to a weight in (0, 1) that multiplies its IRLS weight; the
 * network runs once per round (matrix cores, fp16 activations and weights,
 * fp32 accumulation; the features enter as two fp16 parts; the weight is
 * kept per match as fp16).  Features:
 * the match's residual at the last three round snapshots as
 * log(1 + |eps| * median f) / log(257), its keypoints scaled to [-1, 1] by
 * each camera's principal point (x/cx - 1, ...; the keypoint in the camera
 * with the lower index first), and the angle between the
 * pair's optical axes over pi/2.  Parameters: FEA_MLP_PARAMS floats packed
 * as W1 [64*8], b1 [64], W2 [64*64], b2 [64], w3 [64], b3 (row-major).
 * With options.weight_mode = 1, fea_epipolar_adjust uses the learned weights
 * and judges every round with the plain objective: a scene whose plain
 * objective did not decrease over the round is restored to the round's
 * snapshot and continues with plain weights. */
#define FEA_MLP_FEATURES 8
#define FEA_MLP_PARAMS 4801

/* Loads the network parameters (host array [FEA_MLP_PARAMS]).  Returns
 * FEA_ENONFINITE for a non-finite parameter and FEA_EINVAL for a weight of
 * W1, W2 or w3 beyond fp16's largest finite value, 65504 (inference takes
 * the weights as fp16; the biases stay fp32).  The hidden activations are
 * also taken as fp16: networks whose activations exceed that range on the
 * bounded features are outside what the inference supports. */
fea_status fea_set_mlp(fea_ctx *ctx, const float *params);

/* Features of the current round's layout (after fea_begin_round):
 * feat_dev [layout_matches*8] and slot_pos_dev [layout_matches] (device,
 * caller-allocated; fea_info.layout_matches), slot_pos = sorted position of
 * the match in each layout slot or -1 for alignment padding. */
fea_status fea_mlp_features_dev(fea_ctx *ctx, float *feat_dev, int32_t *slot_pos_dev);

/* Learned weight of every match in input order for the current round (host
 * [n_matches]; 0 for matches the filter dropped; 1 when not learned). */
fea_status fea_get_learned_weights(fea_ctx *ctx, float *w);

/* Trains the network on GPU `device` with the library's forward/backward
 * kernels: mean binary cross-entropy of n samples (feat_dev [n*8],
 * target_dev [n] in [0,1], device arrays), Adam (beta 0.9/0.999, eps 1e-8,
 * learning rate lr), `epochs` passes in batches of `batch` samples in an
 * order drawn from `seed`; params_dev [FEA_MLP_PARAMS] is updated in place;
 * loss_per_epoch (host [epochs], nullable) receives the mean loss. */
fea_status fea_mlp_train(int32_t device, const float *feat_dev, const float *target_dev, int64_t n,
                         int32_t epochs, int32_t batch, double lr, uint64_t seed, float *params_dev,
                         double *loss_per_epoch);

/* Mean BCE loss and its gradient over samples [0, n) (device arrays;
 * grad_dev [FEA_MLP_PARAMS]); loss written to *loss (host). */
fea_status fea_mlp_grad(int32_t device, const float *feat_dev, const float *target_dev, int64_t n,
                        const float *params_dev, float *grad_dev, double *loss);

/* fea_mlp_grad without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving or training loops,
 * harnesses that forbid hipMalloc): the same kernels, with the per-workgroup
 * partials in a fixed workspace the library holds on each GPU it runs on
 * (about 19.7 MB, kept until the process ends).  Queued on hip_stream
 * (a hipStream_t; NULL = the null stream) on GPU `device`, which becomes
 * current for the call only; nothing is allocated, freed or waited for.
 * n in [1, FEA_MLP_NOALLOC_MAX_SAMPLES]; grad_dev [FEA_MLP_PARAMS] receives
 * the gradient of the mean BCE loss and loss_dev [1] (device, nullable) the
 * mean loss.  Calls that overlap on one GPU share the workspace and race:
 * order them on one stream.  FEA_EINVAL for a NULL array, n outside the
 * range or an unknown device; FEA_EDEVICE if a launch fails. */
#define FEA_MLP_NOALLOC_MAX_SAMPLES 65536
fea_status fea_mlp_grad_noalloc(int32_t device, void *hip_stream, const float *feat_dev,
                                const float *target_dev, int64_t n, const float *params_dev,
                                float *grad_dev, double *loss_dev);

/* n_steps first-order steps of the current round (Method > First-order
 * Optimization; Adam as the optimiser the paper cites), each a residual,
 * weight and gradient pass over the round's objective, the per-camera chain
 * rule through the 6D rotation (Method > Optimization Formulations > Global
 * Rotation) and log f, and the update.  Needs a round (FEA_ESTATE). */
fea_status fea_step(fea_ctx *ctx, int32_t n_steps);

/* The whole solve (Method > Optimization Formulations > Epipolar
 * Adjustment: the weights are recomputed and another optimisation loop run
 * after each round, with outliers filtered by a threshold that starts large
 * and decreases to a minimum; focal lengths folded into the essential
 * matrices): options.rounds rounds of fea_begin_round with the threshold
 * schedule max(tau_px_init * tau_decay^r, tau_px_min), each followed by
 * options.iters_per_round steps.  out may be NULL.
 * Non-finite guard: at every round boundary (and once more after the last
 * round) each scene's parameters, poses and last-step loss are checked on
 * the device; a scene holding a non-finite value gets back the parameters
 * and poses of the snapshot its last round started from (the last values
 * found finite) and takes no further steps, while the other scenes go on.
 * The call then returns FEA_ENONFINITE after filling out (scenes_nonfinite
 * counts such scenes; fea_get_scene_nonfinite names them).  fea_begin_round
 * runs the same check and returns FEA_ENONFINITE when it stops a scene. */
fea_status fea_epipolar_adjust(fea_ctx *ctx, fea_report *out);

/* Batched solve of independent problems (the batching of Method > Kernel
 * Fusion's launch-bound small scenes, Table fastmap-kernel_fusion: every
 * kernel launch covers all scenes): scenes [n_scenes] are contexts that
 * each hold one scene (fea_set_scenes not used) with intrinsics, matches and
 * initial poses loaded, all on one device; each is solved as
 * fea_epipolar_adjust would solve it alone, with options opt (NULL = the
 * first context's options; learned weights take the first context's
 * network), the scenes' early exit included.  The library builds one
 * working context holding every scene (the matches are exported in sorted
 * order on the device and segmented again: O(total matches) of set-up work
 * and device memory), solves it, and frees it.  Afterwards each context
 * holds its solved poses as if fea_init_poses and fea_set_poses had been
 * called with them (round state reset).  out [n_scenes] (nullable) receives
 * each scene's report: its rounds (up to its convergence round), steps,
 * per-round loss and retained matches of that scene, fallbacks 1 if the judge
 * rejected its learned weights, scenes_converged 1 if it converged,
 * scenes_nonfinite 1 if the non-finite guard stopped it, and ms_total the
 * batched solve's wall time (set-up excluded).  If the guard stopped a
 * scene the results are still written back and the call returns
 * FEA_ENONFINITE.  Errors:
 * FEA_EINVAL for n_scenes < 1, a NULL or repeated context, contexts on
 * several devices or holding several scenes, more than 65535 cameras or 2^31
 * matches in all, invalid options; FEA_ESTATE for a context without poses
 * (or learned weights without a network); the message goes to the first
 * context.  On an error the contexts keep their state unless the write-back
 * of results had begun. */
fea_status fea_batch_solve(int32_t n_scenes, fea_ctx *const *scenes, const fea_options *opt, fea_report *out);

/* Current poses in the caller's frame: R [n_cams*9], t [n_cams*3], f
 * [n_cams] (host arrays, caller-allocated; any may be NULL). */
fea_status fea_get_poses(fea_ctx *ctx, double *R, double *t, double *f);

/* The segmentation of the loaded matches (host arrays, caller-allocated,
 * any may be NULL): perm [n_matches] input index of the match at each sorted
 * position; swapped [n_matches] 1 if that match was re-oriented;
 * pair_cams [2*n_pairs] (i, j) of each pair in lexicographic order;
 * seg_off [n_pairs+1] sorted range of each pair. */
fea_status fea_get_segments(fea_ctx *ctx, int32_t *perm, uint8_t *swapped,
                            int32_t *pair_cams, int64_t *seg_off);

/* Which matches the current round retains (host array [n_matches], indexed
 * by input order; 1 = retained).  n_retained may be NULL. */
fea_status fea_get_mask(fea_ctx *ctx, uint8_t *mask, int64_t *n_retained);

/* ---- Ablations (measurement) -------------------------------------------
 * One per-match pass at the current poses and round weights with one design
 * choice of the library's kernel taken back, for pricing that choice against
 * HBM peak on the same data: 0 = the library's kernel (pair pose table read
 * with scalar loads, per-lane sums, DPP wave reduction, one partial per work
 * item); 1 = pose block built in every workgroup and staged in LDS (needs
 * options.tile_matches = 2048); 2 = per-match global atomics into per-pair
 * sums; 3 = matches in the caller's order with a pair id each and per-match
 * atomics.  Runs reps + 1 launches (the first untimed) and writes the mean
 * kernel time (HIP events, ms) to *ms_per_pass and, if pair_sums is not
 * NULL, the per-pair sums (host [n_pairs*10] fp32: dL/dF for centred
 * coordinates and the loss, plain weights).  Variant 3 allocates and frees
 * ~20 bytes per match of scratch.  Needs a round (FEA_ESTATE). */
fea_status fea_ablation(fea_ctx *ctx, int32_t variant, int32_t reps, double *ms_per_pass, float *pair_sums);

/* ---- Checkpoint / resume ----------------------------------------------
 * The solver state between calls, as an opaque byte string: parameters
 * (6D rotations, translations, log f), Adam moments and step counts, the
 * round snapshot and the two before it (learned features), round and step
 * indices, per-scene thresholds, gauges and weighting modes, the options,
 * the pairs' quadratic forms of the round, and the retained matches of the
 * round as one bit per sorted position.
 * fea_get_state: with buf == NULL writes the required size to *len; else
 * *len must be at least that size (FEA_EINVAL otherwise, with the size
 * written back) and the state is copied to the caller's host buffer.
 * Needs initialised poses (FEA_ESTATE).
 * fea_set_state: restores a state into a context that loaded the same
 * intrinsics groups, scenes and matches in the same order (checked by sizes
 * and a hash of the pair table, segments and sorted order: FEA_EINVAL
 * otherwise); for a state taken on learned weights the same network must be
 * loaded first (FEA_ESTATE).  The next steps then reproduce bit for bit the
 * steps the saved context would have taken.  The buffer is only read. */
fea_status fea_get_state(fea_ctx *ctx, void *buf, size_t *len);
fea_status fea_set_state(fea_ctx *ctx, const void *buf, size_t len);

/* Sizes and state. */
fea_status fea_get_info(fea_ctx *ctx, fea_info *out);

/* The autotuner's last tuning on this context: ms [cap] receives the mean
 * time of one per-match pass for each candidate work-item shape (13 shapes:
 * 1024 to 8192 matches per item, 128 to 512 threads, one workgroup per item
 * or persistent workgroups); *n the number of shapes timed (0 if the shape
 * was given or reused).  The pick is the first shape, in that order, within
 * 3% of the fastest. */
fea_status fea_get_tile_timings(fea_ctx *ctx, float *ms, int32_t cap, int32_t *n);

/* Blocks until all work issued on the context's stream has finished. */
fea_status fea_synchronize(fea_ctx *ctx);

/* The HIP stream (hipStream_t) every call on this context issues its work on:
 * the one given to fea_create, or the context's own.  Callers that produce or
 * consume the *_dev arrays on another stream order the two with events on
 * this handle instead of synchronising the host.  The context keeps
 * ownership; the handle is valid until fea_destroy.  FEA_EINVAL if either
 * pointer is NULL. */
fea_status fea_get_stream(fea_ctx *ctx, void **stream);

/* STREAM-style HBM probe on GPU `device`: a read-only kernel and a copy
 * kernel over `bytes` bytes (rounded down to 16-byte vectors), best of
 * `reps` timed launches each.  Writes the achieved read and copy bandwidth
 * (copy counts read + write bytes) in GB/s.  Allocates and frees its own
 * buffers. */
fea_status fea_hbm_probe(int32_t device, int64_t bytes, int32_t reps, double *read_gbps,
                         double *copy_gbps);

/* Kernel timing for measurement.  While enabled, every launch of the
 * per-match residual/gradient kernel records a pair of HIP events at its
 * own start and end on the context's stream (steps run without graph
 * replay meanwhile).  fea_set_kernel_timing(ctx, 1) clears earlier records;
 * fea_get_kernel_timing synchronises the stream and returns the summed
 * event time (ms) and the number of timed launches.  fea_get_kernel_times
 * writes the first min(cap, launches) per-launch durations (ms, launch
 * order) into the caller's host array `ms` (NULL with cap 0 only counts)
 * and the number of timed launches into *n. */
fea_status fea_set_kernel_timing(fea_ctx *ctx, int32_t enable);
fea_status fea_get_kernel_timing(fea_ctx *ctx, double *resgrad_ms, int64_t *resgrad_launches);
fea_status fea_get_kernel_times(fea_ctx *ctx, float *ms, int64_t cap, int64_t *n);

/* Rotation log kept by fea_epipolar_adjust when options.log_every > 0:
 * R_log [max_log * n_cams * 9] host, in the caller's frame; *n_logged
 * receives the count.  Entry k holds the rotations after step
 * (k+1)*log_every, counting steps across rounds. */
fea_status fea_get_rotation_log(fea_ctx *ctx, double *R_log, int32_t *n_logged);

/* ---- Global rotation (Method > Global Rotation) --------------------------
 * Eq. fastmap-rotation-objective: world-to-camera rotations R_i minimising
 *   L_R = (1/|P|) sum over pairs of d(R_j, R^{i->j} R_i),
 * d(R, R') = arccos((tr(R^T R') - 1)/2) (argument clamped to [-1, 1]), by
 * Adam on the 6D parameterisation (bias-corrected; the learning rate of step
 * k of T is lr * lr_end_frac^(k/T); the arccos derivative is taken where its
 * argument is strictly inside (-1, 1), zero elsewhere).  Initialisation
 * (after Martinec and Pajdla, as the paper modifies it): the first columns
 * minimise sum |c_j - R^{i->j} c_i|^2 over unit-norm stacked vectors, the
 * second columns the same over |P| plus sum (c1_i . c2_i)^2 / |I|, each the
 * Ritz vector of the smallest eigenvalue of the problem's 3N x 3N normal
 * matrix by the Lanczos method with full reorthogonalisation from the
 * caller's random start vectors v0 (until the smallest Ritz value changes
 * by less than 3e-5 of itself over 16 steps; restarted from the Ritz vector
 * every 256 steps; at most init_iters products with the matrix)
 * [2 * n_cams * 3] (any vector in the near-null space of the first problem
 * is a valid first column: the rotations are fixed up to one global
 * rotation), normalised per camera, the second made orthogonal to the
 * first; the third column is their cross product.  With a6_init
 * [n_cams * 6] (nullable) the initialisation is skipped and the
 * optimisation starts there.  Inputs (host, copied): pair_i, pair_j
 * [n_pairs] (cameras in [0, n_cams), i != j), R_rel [n_pairs*9] row-major
 * with R_j ~ R_rel R_i.  Outputs (host): R_out [n_cams*9], R_init [n_cams*9]
 * (nullable: the rotations the optimisation starts from), loss [2]
 * (nullable: L_R at the start and the end), ms (nullable: device time of the
 * call, HIP events).  FEA_EINVAL for invalid sizes, pairs or options;
 * FEA_ENONFINITE for non-finite input; FEA_EDEGENERATE if a camera's column
 * vanishes in the initialisation (a camera without pairs).  Device scratch of
 * O(n_pairs + 257 * 3 n_cams) doubles is allocated and freed by the call. */
typedef struct {
  int32_t init_iters; /* at most this many Lanczos steps per column (default 200000) */
  int32_t iters;      /* Adam steps (1000) */
  double lr;          /* first learning rate (1e-2) */
  double lr_end_frac; /* last over first learning rate (1e-2) */
  double beta1, beta2, adam_eps; /* 0.9, 0.999, 1e-12 */
} fea_ra_options;

fea_status fea_ra_default_options(fea_ra_options *out);
fea_status fea_rotation_averaging(fea_ctx *ctx, int32_t n_cams, int64_t n_pairs, const int32_t *pair_i,
                                  const int32_t *pair_j, const double *R_rel, const double *v0,
                                  const double *a6_init, const fea_ra_options *opt, double *R_out,
                                  double *R_init, double *loss, float *ms);

/* ---- Focal-length vote (Method > Focal Length Estimation) ---------------
 * Eq. fastmap-focal-vote: a 3x3 matrix is essential exactly when its two
 * non-zero singular values are equal, so a candidate focal length f scores
 *   v(f) = sum over pairs of exp((1 - s1/s2) / tau),
 * s1 >= s2 the two largest singular values of E = K_j^T F K_i with
 * K = diag(f, f, 1) in centred pixel coordinates.  Per intrinsics group g
 * (group [n_cams], NULL = one group for every camera, the paper's shared
 * intrinsics): the pairs with a camera in g vote; g's cameras take the
 * candidate, every other camera keeps its group's f_cur (one sweep of
 * per-camera votes when every camera is its own group).  The best candidate
 * per group has the highest vote (ties: the lower index).  Inputs (host,
 * copied): pair_i, pair_j [n_pairs] (cameras in [0, n_cams), i != j),
 * F [n_pairs*9] row-major with p_j^T F p_i = 0 for centred pixel coordinates
 * p = (x - cx, y - cy, 1) (any scale or sign), f_cur [n_groups] (required
 * with more than one group), cand_f [n_cand] > 0, tau > 0.  Outputs (host):
 * f_best [n_groups], k_best [n_groups] (nullable), votes
 * [n_groups*n_cand] (nullable), ms (nullable: the vote kernel's HIP-event
 * time).  fp64 throughout; the singular-value ratio comes from the closed-form
 * eigenvalues of E^T E, which fix it to ~1.5e-8 near equal values.  The
 * context only supplies device, stream and error message.  FEA_EINVAL for
 * invalid sizes, pairs, groups or values; FEA_ENONFINITE for a non-finite F. */
fea_status fea_focal_vote(fea_ctx *ctx, int32_t n_cams, int64_t n_pairs, const int32_t *pair_i,
                          const int32_t *pair_j, const double *F, const int32_t *group, const double *f_cur,
                          int32_t n_cand, const double *cand_f, double tau, double *f_best, int32_t *k_best,
                          double *votes, float *ms);

/* ---- Global Translation (the stages before epipolar adjustment) ---------
 * Relative translations (Method > Global Translation > Relative
 * translation): with the global rotations fixed, every image pair of the
 * loaded matches gets a unit relative translation chosen among candidate
 * directions by its mean epipolar error.  For pair n = (i, j) (the pair order
 * of fea_get_segments) and candidate u:
 *   score(u) = mean over the pair's matches of |x~2^T [u]x R_ij x~1|,
 * x~ = ((x - cx)/f, (y - cy)/f, 1), R_ij = R_j R_i^T: the epipolar-adjustment
 * residual with the relative translation set to u.  With a finite tau_px
 * every match's term is capped, min(|eps|, tau) with tau = tau_px / median f:
 * the paper scores two-view inliers, and the cap keeps outliers among the
 * matches from steering the choice (tau_px = INFINITY: the plain mean).  The
 * lowest score wins (ties: the lower candidate index).  A direction and its
 * opposite score the same, so the sign is decided by cheirality: each match
 * with |eps| < tau at the chosen direction votes +1 when both depths of its
 * least-squares two-view triangulation with translation u are positive, -1
 * when both are negative, 0 otherwise; the result is u for a vote sum >= 0,
 * else -u.  Scores are fp32 on the matrix cores; the vote is fp64.  Inputs
 * (host, copied): R [n_cams*9] world-to-camera rotations, f [n_cams] focal
 * lengths (NULL = the loaded intrinsics), tau_px > 0, cand [n_cand*3] unit
 * vectors (one hemisphere suffices).  Outputs (host, caller-allocated,
 * n_pairs = fea_get_info's n_pairs): t_rel [n_pairs*3], best [n_pairs]
 * (nullable), vote [n_pairs] (nullable), score_best [n_pairs] (nullable),
 * scores [n_pairs*n_cand] (nullable: every candidate's mean score),
 * score_ms (nullable: duration of the scoring kernel, HIP events).
 * Requires loaded matches (FEA_ESTATE otherwise); FEA_EINVAL for
 * n_cand outside [1, 2^22], candidates that are not unit vectors (1e-6) or
 * focal lengths <= 0 or tau_px <= 0; FEA_ENONFINITE for non-finite input.  Device scratch
 * (n_cand rounded up to 1024, times the number of 2048-match work items, in
 * fp32) is allocated and freed by the call. */
fea_status fea_relative_translations(fea_ctx *ctx, const double *R, const double *f, double tau_px, int32_t n_cand,
                                     const double *cand, double *t_rel, int32_t *best, int32_t *vote,
                                     double *score_best, float *scores, float *score_ms);

/* Camera centres (Eq. fastmap-global-translation-objective, Multiple
 * initializations): targets o^{i->j} = -R_j^T t^{i->j} / |t^{i->j}|; the loss
 *   L_t = (1/|P|) sum over pairs of | (o_j - o_i)/|o_j - o_i| - o^{i->j} |_1
 * over the centres o is minimised with Adam (bias-corrected; the learning
 * rate of step k of a phase of T steps is lr * lr_end_frac^(k/T); sign(0) = 0;
 * a pair whose two centres coincide contributes nothing), n_runs times side by
 * side from the caller's initial centres o_init [n_runs*n_cams*3] (the random
 * numbers of the method are inputs).  Each run's result is centred at the
 * origin and scaled to unit mean norm; each camera then takes its centre from
 * the run with the lowest mean loss over that camera's pairs (ties: the lower
 * run; a camera without pairs scores 0); the merged centres are optimised
 * iters_final more steps from lr_final and aligned again.  Pairs are given
 * explicitly (pair_i, pair_j [n_pairs], cameras in [0, n_cams), i != j;
 * t_rel [n_pairs*3] in camera j's frame, any non-zero length; R
 * [n_cams*9]); the context only supplies device, stream and error message
 * (no intrinsics or matches needed).  Outputs (host): o_out [n_cams*3]
 * (aligned), run_of_cam [n_cams], run_loss [n_runs], final_loss, run_o
 * [n_runs*n_cams*3] (aligned run results), cam_loss [n_runs*n_cams], ms
 * (device time of the whole call, HIP events); all but o_out nullable.
 * FEA_EINVAL for invalid sizes, pairs or options (n_runs in [1, 64]),
 * FEA_ENONFINITE for non-finite input, FEA_EDEGENERATE for a zero relative
 * translation or a run whose centres all coincide.  Device scratch of
 * O(n_runs * (n_cams + n_pairs)) is allocated and freed by the call. */
typedef struct {
  int32_t iters_run;   /* Adam steps of every run (default 1500) */
  int32_t iters_final; /* Adam steps on the merged centres (500) */
  double lr;           /* first learning rate of a run (2e-2) */
  double lr_final;     /* first learning rate of the final loop (2e-3) */
  double lr_end_frac;  /* learning rate at the end of a phase / at its start (1e-3) */
  double beta1, beta2, adam_eps; /* 0.9, 0.999, 1e-12 */
} fea_ta_options;

fea_status fea_ta_default_options(fea_ta_options *out);
fea_status fea_translation_align(fea_ctx *ctx, int32_t n_cams, int64_t n_pairs, const int32_t *pair_i,
                                 const int32_t *pair_j, const double *R, const double *t_rel, int32_t n_runs,
                                 const double *o_init, const fea_ta_options *opt, double *o_out,
                                 int32_t *run_of_cam, double *run_loss, double *final_loss, double *run_o,
                                 double *cam_loss, float *ms);

#ifdef __cplusplus
}
#endif
#endif /* FASTEA_H */
