/*
 * FP64 CPU oracle for FastMap's epipolar adjustment (EA).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct
 * implementation of what the GPU library computes, written from the paper
 * (FastMap chapter: Method > Optimization Formulations > Epipolar Adjustment,
 * Eq. fastmap-epipolar-objective and the IRLS objective that follows it).  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no source with the HIP library.
 *
 * Conventions (all arrays row-major, all arithmetic double precision):
 *   - world-to-camera poses: X_cam = R X + t; R is 3x3 row-major, t is 3.
 *   - a match (x1,y1) in camera cam1 <-> (x2,y2) in camera cam2, pixel
 *     coordinates; principal point (cx, cy) per camera (the image centre).
 *   - for a pair i<j: R_ij = R_j R_i^T, t_ij = t_j - R_ij t_i,
 *     u = t_ij / |t_ij|, E = [u]x R_ij, F = D_j E D_i with
 *     D_k = diag(1/f_k, 1/f_k, 1); residual eps = p2^T F p1 with
 *     p = (x - cx, y - cy, 1), i.e. eps = x~2^T E x~1 in normalised
 *     homogeneous coordinates.
 *
 * Readings of the paper taken here where it is silent or inconsistent
 * (listed again in the design notes):
 *   - the relative translation enters E as a unit vector;
 *   - the IRLS weight of a match is 1 / (Z * max(|eps_hat|, delta)) where
 *     eps_hat is the residual at the poses frozen at the start of the round
 *     and Z is the number of matches still retained;
 *   - the filter keeps a match while |eps_hat| < tau (strict), and once a
 *     match is dropped it stays dropped;
 *   - the per-match weighted-L2 sum is used (factor 1, not 2);
 *   - rotations are optimised in the 6D (two-column Gram-Schmidt)
 *     representation, focal lengths as log f per intrinsics group,
 *     translations directly; the optimiser is Adam with bias correction,
 *     its moments reset at the start of every IRLS round (optionally kept),
 *     its learning rates optionally decayed per round.
 */
#ifndef FEA_ORACLE_H
#define FEA_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int64_t n_matches;
  int32_t n_cams;
  const float *x1, *y1, *x2, *y2;
  const int32_t *cam1, *cam2;
  const double *cx, *cy; /* [n_cams] */
} orc_problem;

typedef struct {
  int32_t rounds;          /* IRLS rounds */
  int32_t iters_per_round; /* Adam steps per round */
  double tau_px_init;      /* filter threshold of round 0, pixels */
  double tau_px_min;       /* floor of the threshold schedule, pixels */
  double tau_decay;        /* threshold multiplier per round */
  double delta;            /* floor of |eps_hat| in the weight, normalised units */
  double lr_rot, lr_t, lr_logf;
  double beta1, beta2, adam_eps;
  int32_t optimize_focal;
  int32_t gauge_normalize; /* 0 none, 1 centre + median-baseline scale at start */
  double lr_decay;         /* learning rates of round r: lr * lr_decay^r */
  int32_t reset_moments;   /* 1: Adam moments (and step count) restart every round */
  double converge_deg;     /* early exit, 0 = off: the solve stops at the start of a
                              round whose threshold equals the previous round's when
                              the cameras' mean rotation over that round (geodesic
                              distance) is below converge_deg degrees and their mean
                              |log f change| below converge_deg pi/180; the rounds
                              not run report loss NaN and inliers -1 */
} orc_options;

void orc_default_options(orc_options *o);

/* Canonical pairs and stable ordering (Method > Epipolar Adjustment: the
 * pair set P = {(i_n, j_n)} and per-pair point sets Q_n).  Each match is
 * re-oriented so that cam1 < cam2 (swapping its keypoints), pairs get ids in
 * lexicographic (i, j) order, and matches are ordered by pair id keeping their
 * input order within a pair.  Outputs (caller-allocated, worst case n):
 * perm[p] = input index of the match at sorted position p; swapped[p] = 1 if
 * that match was re-oriented; pair_cams[2*k..2*k+1] = (i, j) of pair k;
 * seg_off[k]..seg_off[k+1] = its sorted range.  Returns 0, or -1 if some
 * match has cam1 == cam2 or a camera id out of [0, n_cams). */
int orc_segment(int64_t n, int32_t n_cams, const int32_t *cam1, const int32_t *cam2,
                int32_t *perm, uint8_t *swapped, int32_t *pair_cams, int64_t *seg_off,
                int64_t *n_pairs);

/* 6D rotation representation (Zhou et al., cited for global rotation):
 * a6 = (a1, a2) are the unnormalised first two columns. */
void orc_rot6d_to_R(const double a6[6], double R[9]);
void orc_R_to_rot6d(const double R[9], double a6[6]);
void orc_rot6d_backward(const double a6[6], const double gR[9], double ga6[6]);

/* Fundamental matrix of pair (i, j) from global poses and focal lengths
 * (Eq. fastmap-epipolar-objective with focal lengths folded in, as the
 * paragraph after the IRLS objective describes).  Returns -1 if t_ij = 0. */
int orc_pair_F(const double Ri[9], const double ti[3], double fi, const double Rj[9],
               const double tj[3], double fj, double F[9]);

/* Epipolar residual of every match at poses (R, t, f) (input order). */
int orc_residuals(const orc_problem *pb, const double *R, const double *t, const double *f,
                  double *eps);

/* One filtering step (Method > Epipolar Adjustment, outlier filtering):
 * mask[m] &= |eps_hat_m| < tau at the snapshot poses. Returns Z = sum mask. */
int64_t orc_update_mask(const orc_problem *pb, const double *Rh, const double *th,
                        const double *fh, double tau, uint8_t *mask);

/* IRLS loss and its gradient with respect to every camera's R (9, treated as
 * an unconstrained 3x3 matrix), t (3) and f (1):
 *   L = sum_m mask_m * eps_m^2 / (Z * max(|eps_hat_m|, delta)),
 * eps at (R,t,f), eps_hat at the snapshot (Rh,th,fh), Z = sum mask.
 * Returns 0, -1 on bad input, -2 on a degenerate pair (t_ij = 0). */
int orc_loss_grad(const orc_problem *pb, const double *R, const double *t, const double *f,
                  const double *Rh, const double *th, const double *fh, const uint8_t *mask,
                  double delta, double *loss, double *gR, double *gt, double *gf);

/* As orc_loss_grad with a non-negative weight per match (input order): the
 * IRLS factor of match m is weight[m] / (Z_w max(|eps_hat|, delta)) with Z_w
 * the sum of the retained matches' weights -- the learned inlier weight in
 * place of the 0/1 retained mask.  Returns -3 for a negative or NaN weight. */
int orc_loss_grad_weighted(const orc_problem *pb, const double *R, const double *t,
                           const double *f, const double *Rh, const double *th,
                           const double *fh, const uint8_t *mask, const double *weight,
                           double delta, double *loss, double *gR, double *gt, double *gf);

/* One Adam step (Kingma & Ba, cited as the adaptive first-order optimiser)
 * on n parameters; step is the 1-based step index. */
void orc_adam(int64_t n, double *p, double *m, double *v, const double *g, int64_t step,
              double lr, double beta1, double beta2, double eps);

/* Move camera centres to mean 0 and rescale them so that the median distance
 * between the centres of the matched pairs is 1 (a similarity; the loss is
 * invariant to it).  Writes the applied centre and scale. */
void orc_gauge_normalize(int32_t n, const double *R, double *t, int64_t n_pairs,
                         const int32_t *pair_cams, double *center, double *scale);

/* The whole EA loop: rounds of (snapshot, filter, reset Adam, K Adam steps).
 * In: initial R, t, f and intrinsics groups (intr_group may be NULL: one per
 * camera).  Out: final R, t, f in the caller's frame; loss_per_round[rounds]
 * (loss at the last step of each round); inliers[rounds] (Z per round);
 * optional pose log every log_every steps (log_R: n_log x n_cams x 9). */
int orc_epipolar_adjust(const orc_problem *pb, const orc_options *opt, const double *R0,
                        const double *t0, const double *f0, const int32_t *intr_group,
                        double *R, double *t, double *f, double *loss_per_round,
                        int64_t *inliers, int32_t log_every, int32_t max_log, double *log_R,
                        int32_t *n_logged, uint8_t *mask_out);

/* ---- learned inlier weights ---------------------------------------------
 * A multilayer perceptron 8 -> 64 -> 64 -> 1 (ReLU, ReLU, sigmoid) maps the
 * features of a match to a weight in (0, 1) that multiplies its IRLS weight.
 * Parameters (row-major): W1 [64*8], b1 [64], W2 [64*64], b2 [64], w3 [64],
 * b3 [1], packed in that order into one array of ORC_MLP_NPARAM doubles.
 *
 * Features of match m at round r (ORC_MLP_NFEAT = 8):
 *   0..2  g(|eps_hat|) at the snapshots of rounds r, r-1, r-2 (the earliest
 *         available snapshot repeats for r < 2), with
 *         g(e) = log(1 + e * fbar) / log(1 + 256), fbar the median focal
 *         length of the snapshot, i.e. the residual in pixel-equivalents,
 *         log-compressed so 256 px maps to 1;
 *   3..6  keypoints scaled to [-1, 1]: x1/cx1 - 1, y1/cy1 - 1, x2/cx2 - 1,
 *         y2/cy2 - 1 (cx = W/2, cy = H/2 of each keypoint's camera);
 *   7     angle between the optical axes of the two cameras at snapshot r,
 *         divided by pi/2. */
#define ORC_MLP_NFEAT 8
#define ORC_MLP_HIDDEN 64
#define ORC_MLP_NPARAM (64 * 8 + 64 + 64 * 64 + 64 + 64 + 1)

/* Features of every match (input order) given the snapshot poses of the last
 * three rounds (R0/t0/f0 = round r, R1.. = r-1, R2.. = r-2).  Keypoint
 * features follow the pair's orientation (lower camera index first), so a
 * match and its swapped copy have the same features. */
int orc_mlp_features(const orc_problem *pb, const double *R0, const double *t0, const double *f0,
                     const double *R1, const double *t1, const double *f1, const double *R2,
                     const double *t2, const double *f2, double *feat);

/* Forward pass: y[m] = MLP(feat[m]) for n rows of ORC_MLP_NFEAT. */
void orc_mlp_forward(int64_t n, const double *feat, const double *params, double *y);

/* Mean binary cross-entropy against targets in [0, 1] and its gradient with
 * respect to the packed parameters. */
double orc_mlp_bce_grad(int64_t n, const double *feat, const double *target, const double *params,
                        double *grad);

/* ---- Global Translation: relative translations ---------------------------
 * Method > Global Translation > Relative translation: with the global
 * rotations fixed, each pair's unit relative translation is re-estimated by
 * scoring candidate directions on the unit sphere by their mean epipolar
 * error and keeping the best.  For every canonical pair (i < j, in the
 * lexicographic order of orc_segment) and candidate u (cand[3k..3k+2]):
 *   score(u) = mean over the pair's matches of min(|x~2^T [u]x R_ij x~1|, tau),
 * x~ = ((x - cx)/f, (y - cy)/f, 1), R_ij = R_j R_i^T (the EA residual with the
 * relative translation set to u).  tau = INFINITY is the paper's plain mean;
 * a finite tau (normalised units, reading: the paper scores two-view inliers,
 * and the truncation keeps the outliers among the matches from steering the
 * choice) caps each match's term.  best = the lowest score (ties: the lower
 * index).  The score does not change under u -> -u, so the sign is taken by
 * cheirality (reading; the paper does not say): every match with
 * |eps(u)| < tau votes +1 when both depths of its two-view triangulation
 * with t_ij = u are positive, -1 when both are negative, 0 otherwise;
 * t_rel = u if the vote sum is >= 0, else -u.  Outputs, caller-allocated for
 * P pairs (P <= n_matches):
 * pair_cams [2P], scores [P * n_cand] (nullable), best [P], t_rel [3P],
 * vote [P].  Returns 0, or -1 for invalid matches or n_cand < 1. */
int orc_rel_trans(const orc_problem *pb, const double *R, const double *f, int32_t n_cand,
                  const double *cand, double tau, int64_t *n_pairs, int32_t *pair_cams,
                  double *scores, int32_t *best, double *t_rel, int64_t *vote);

/* ---- Global Translation: camera centres ------------------------------------
 * Eq. fastmap-global-translation-objective and the text around it: targets
 * o^{i->j} = -R_j^T t^{i->j} (t^{i->j} normalised to unit length); the loss
 *   L_t = (1/|P|) sum_{(i,j)} | (o_j - o_i)/|o_j - o_i| - o^{i->j} |_1
 * over the camera centres o; its gradient uses sign(0) = 0 and a pair whose
 * two centres coincide contributes nothing. */
int orc_ta_targets(int32_t n_cams, int64_t n_pairs, const int32_t *pair_i,
                   const int32_t *pair_j, const double *R, const double *t_rel, double *target);
double orc_ta_loss_grad(int32_t n_cams, int64_t n_pairs, const int32_t *pair_i,
                        const int32_t *pair_j, const double *target, const double *o,
                        double *grad, double *pair_loss);

/* Multiple initialisations and merge (Global Translation > Multiple
 * initializations): each run optimises the centres from its own initial
 * values with Adam (readings: Adam with bias correction; the learning rate of
 * step k of a run of T steps is lr * lr_end_frac^(k/T)); each run's result is
 * centred at the origin and rescaled to unit mean norm; every camera takes its
 * centre from the run with the lowest mean loss over that camera's pairs
 * (ties: the lower run; a camera without pairs scores 0); the merged centres
 * are optimised iters_final more steps from lr_final and aligned again.
 * o_init [n_runs * N * 3]; outputs o_out [N*3], run_o [n_runs*N*3] (aligned
 * run results, nullable), cam_loss [n_runs*N] (nullable), run_of_cam [N],
 * run_loss [n_runs] (nullable), final_loss (nullable). */
typedef struct {
  int32_t iters_run, iters_final;
  double lr, lr_final, lr_end_frac;
  double beta1, beta2, adam_eps;
} orc_ta_options;
void orc_ta_default_options(orc_ta_options *o);
int orc_ta_solve(int32_t n_cams, int64_t n_pairs, const int32_t *pair_i, const int32_t *pair_j,
                 const double *target, int32_t n_runs, const double *o_init,
                 const orc_ta_options *opt, double *o_out, double *run_o, double *cam_loss,
                 int32_t *run_of_cam, double *run_loss, double *final_loss);

/* Number of OpenMP threads the oracle would use (1 without OpenMP). */
int orc_num_threads(void);
void orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
