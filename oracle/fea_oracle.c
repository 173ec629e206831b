/*
 * FP64 CPU oracle for FastMap epipolar adjustment -- TEST INFRASTRUCTURE ONLY.
 * See fea_oracle.h for the conventions and the readings of the paper.
 * Every function is written for clarity: straight loops in double precision,
 * no blocking, no fusion, no reordering beyond what the definitions state.
 */
#include "fea_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads for the following parallel regions (per-pair partial sums are
   added in a fixed order, so results do not depend on it). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

void orc_default_options(orc_options *o) {
  o->rounds = 20;
  o->iters_per_round = 50;
  o->tau_px_init = 128.0;
  o->tau_px_min = 4.0;
  o->tau_decay = 0.5;
  o->delta = 1e-4;
  o->lr_rot = 3e-3;
  o->lr_t = 4e-2;
  o->lr_logf = 1e-3;
  o->beta1 = 0.9;
  o->beta2 = 0.999;
  o->adam_eps = 1e-12;
  o->optimize_focal = 1;
  o->gauge_normalize = 1;
  o->lr_decay = 0.9;
  o->reset_moments = 1;
  o->converge_deg = 0.0;
}

/* ---- small 3x3 helpers (row-major) ------------------------------------ */

static void mat_mul(const double A[9], const double B[9], double C[9]) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[r * 3 + k] * B[k * 3 + c];
      C[r * 3 + c] = s;
    }
}

static void mat_mul_bt(const double A[9], const double B[9], double C[9]) { /* A B^T */
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[r * 3 + k] * B[c * 3 + k];
      C[r * 3 + c] = s;
    }
}

static void mat_mul_at(const double A[9], const double B[9], double C[9]) { /* A^T B */
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[k * 3 + r] * B[k * 3 + c];
      C[r * 3 + c] = s;
    }
}

static void mat_vec(const double A[9], const double x[3], double y[3]) {
  for (int r = 0; r < 3; ++r) y[r] = A[r * 3] * x[0] + A[r * 3 + 1] * x[1] + A[r * 3 + 2] * x[2];
}

static void mat_t_vec(const double A[9], const double x[3], double y[3]) {
  for (int r = 0; r < 3; ++r) y[r] = A[r] * x[0] + A[3 + r] * x[1] + A[6 + r] * x[2];
}

static void skew(const double u[3], double S[9]) { /* S x = u cross x */
  S[0] = 0.0;   S[1] = -u[2]; S[2] = u[1];
  S[3] = u[2];  S[4] = 0.0;   S[5] = -u[0];
  S[6] = -u[1]; S[7] = u[0];  S[8] = 0.0;
}

static void cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* ---- segmenting --------------------------------------------------------- */

typedef struct {
  int64_t key; /* i * n_cams + j with i < j */
  int64_t idx; /* input position: the tie-break that makes the sort stable */
} seg_item;

static int seg_cmp(const void *a, const void *b) {
  const seg_item *x = (const seg_item *)a, *y = (const seg_item *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;
  return 0;
}

int orc_segment(int64_t n, int32_t n_cams, const int32_t *cam1, const int32_t *cam2,
                int32_t *perm, uint8_t *swapped, int32_t *pair_cams, int64_t *seg_off,
                int64_t *n_pairs) {
  for (int64_t m = 0; m < n; ++m) {
    if (cam1[m] < 0 || cam1[m] >= n_cams || cam2[m] < 0 || cam2[m] >= n_cams) return -1;
    if (cam1[m] == cam2[m]) return -1;
  }
  seg_item *it = (seg_item *)malloc(sizeof(seg_item) * (size_t)(n > 0 ? n : 1));
  if (!it) return -1;
  for (int64_t m = 0; m < n; ++m) {
    int64_t i = cam1[m] < cam2[m] ? cam1[m] : cam2[m];
    int64_t j = cam1[m] < cam2[m] ? cam2[m] : cam1[m];
    it[m].key = i * (int64_t)n_cams + j;
    it[m].idx = m;
  }
  qsort(it, (size_t)n, sizeof(seg_item), seg_cmp);
  int64_t np = 0;
  for (int64_t p = 0; p < n; ++p) {
    int64_t m = it[p].idx;
    perm[p] = (int32_t)m;
    swapped[p] = (uint8_t)(cam1[m] > cam2[m]);
    if (p == 0 || it[p].key != it[p - 1].key) {
      pair_cams[2 * np] = (int32_t)(it[p].key / n_cams);
      pair_cams[2 * np + 1] = (int32_t)(it[p].key % n_cams);
      seg_off[np] = p;
      ++np;
    }
  }
  seg_off[np] = n;
  *n_pairs = np;
  free(it);
  return 0;
}

/* ---- 6D rotation representation ---------------------------------------- */

void orc_rot6d_to_R(const double a6[6], double R[9]) {
  const double *a1 = a6, *a2 = a6 + 3;
  double b1[3], b2[3], b3[3], v[3];
  double n1 = sqrt(dot3(a1, a1));
  for (int k = 0; k < 3; ++k) b1[k] = a1[k] / n1;
  double d = dot3(b1, a2);
  for (int k = 0; k < 3; ++k) v[k] = a2[k] - d * b1[k];
  double n2 = sqrt(dot3(v, v));
  for (int k = 0; k < 3; ++k) b2[k] = v[k] / n2;
  cross(b1, b2, b3);
  for (int r = 0; r < 3; ++r) {
    R[r * 3 + 0] = b1[r];
    R[r * 3 + 1] = b2[r];
    R[r * 3 + 2] = b3[r];
  }
}

void orc_R_to_rot6d(const double R[9], double a6[6]) {
  for (int r = 0; r < 3; ++r) {
    a6[r] = R[r * 3 + 0];
    a6[3 + r] = R[r * 3 + 1];
  }
}

void orc_rot6d_backward(const double a6[6], const double gR[9], double ga6[6]) {
  const double *a1 = a6, *a2 = a6 + 3;
  double b1[3], b2[3], v[3];
  double n1 = sqrt(dot3(a1, a1));
  for (int k = 0; k < 3; ++k) b1[k] = a1[k] / n1;
  double d = dot3(b1, a2);
  for (int k = 0; k < 3; ++k) v[k] = a2[k] - d * b1[k];
  double n2 = sqrt(dot3(v, v));
  for (int k = 0; k < 3; ++k) b2[k] = v[k] / n2;
  double gb1[3], gb2[3], gb3[3], tmp[3];
  for (int r = 0; r < 3; ++r) {
    gb1[r] = gR[r * 3 + 0];
    gb2[r] = gR[r * 3 + 1];
    gb3[r] = gR[r * 3 + 2];
  }
  /* b3 = b1 x b2 */
  cross(b2, gb3, tmp);
  for (int k = 0; k < 3; ++k) gb1[k] += tmp[k];
  cross(gb3, b1, tmp);
  for (int k = 0; k < 3; ++k) gb2[k] += tmp[k];
  /* b2 = v / |v|, v = a2 - (b1 . a2) b1 */
  double gv[3], s = dot3(b2, gb2);
  for (int k = 0; k < 3; ++k) gv[k] = (gb2[k] - s * b2[k]) / n2;
  double b1gv = dot3(b1, gv);
  for (int k = 0; k < 3; ++k) {
    ga6[3 + k] = gv[k] - b1gv * b1[k];
    gb1[k] += -d * gv[k] - b1gv * a2[k];
  }
  /* b1 = a1 / |a1| */
  double s1 = dot3(b1, gb1);
  for (int k = 0; k < 3; ++k) ga6[k] = (gb1[k] - s1 * b1[k]) / n1;
}

/* ---- pair geometry -------------------------------------------------------- */

typedef struct {
  double Rij[9], tij[3], u[3], tnorm, E[9], F[9];
} pair_geom;

/* R_ij = R_j R_i^T, t_ij = t_j - R_ij t_i, u = t_ij/|t_ij|, E = [u]x R_ij,
 * F = D_j E D_i (Eq. fastmap-epipolar-objective, focal lengths folded in). */
static int pair_geometry(const double Ri[9], const double ti[3], double fi, const double Rj[9],
                         const double tj[3], double fj, pair_geom *g) {
  mat_mul_bt(Rj, Ri, g->Rij);
  double Rt[3];
  mat_vec(g->Rij, ti, Rt);
  for (int k = 0; k < 3; ++k) g->tij[k] = tj[k] - Rt[k];
  g->tnorm = sqrt(dot3(g->tij, g->tij));
  if (!(g->tnorm > 0.0)) return -1;
  for (int k = 0; k < 3; ++k) g->u[k] = g->tij[k] / g->tnorm;
  double S[9];
  skew(g->u, S);
  mat_mul(S, g->Rij, g->E);
  double di[3] = {1.0 / fi, 1.0 / fi, 1.0};
  double dj[3] = {1.0 / fj, 1.0 / fj, 1.0};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) g->F[a * 3 + b] = dj[a] * g->E[a * 3 + b] * di[b];
  return 0;
}

int orc_pair_F(const double Ri[9], const double ti[3], double fi, const double Rj[9],
               const double tj[3], double fj, double F[9]) {
  pair_geom g;
  if (pair_geometry(Ri, ti, fi, Rj, tj, fj, &g)) return -1;
  memcpy(F, g.F, sizeof(g.F));
  return 0;
}

/* Residual of one match whose keypoint p1 lies in camera i and p2 in camera
 * j: eps = p2^T F p1. */
static double match_residual(const double F[9], double p1x, double p1y, double p2x,
                             double p2y) {
  double p1[3] = {p1x, p1y, 1.0}, p2[3] = {p2x, p2y, 1.0}, Fp1[3];
  mat_vec(F, p1, Fp1);
  return dot3(p2, Fp1);
}

/* Canonical orientation of match m: returns camera ids i < j and the centred
 * keypoints of i (a) and j (b). */
static void canonical_match(const orc_problem *pb, int64_t m, int32_t *i, int32_t *j,
                            double *ax, double *ay, double *bx, double *by) {
  int32_t c1 = pb->cam1[m], c2 = pb->cam2[m];
  double x1 = (double)pb->x1[m] - pb->cx[c1], y1 = (double)pb->y1[m] - pb->cy[c1];
  double x2 = (double)pb->x2[m] - pb->cx[c2], y2 = (double)pb->y2[m] - pb->cy[c2];
  if (c1 < c2) {
    *i = c1; *j = c2; *ax = x1; *ay = y1; *bx = x2; *by = y2;
  } else {
    *i = c2; *j = c1; *ax = x2; *ay = y2; *bx = x1; *by = y1;
  }
}

static int check_problem(const orc_problem *pb) {
  for (int64_t m = 0; m < pb->n_matches; ++m) {
    int32_t c1 = pb->cam1[m], c2 = pb->cam2[m];
    if (c1 < 0 || c2 < 0 || c1 >= pb->n_cams || c2 >= pb->n_cams || c1 == c2) return -1;
  }
  return 0;
}

int orc_residuals(const orc_problem *pb, const double *R, const double *t, const double *f,
                  double *eps) {
  if (check_problem(pb)) return -1;
  for (int64_t m = 0; m < pb->n_matches; ++m) {
    int32_t i, j;
    double ax, ay, bx, by;
    canonical_match(pb, m, &i, &j, &ax, &ay, &bx, &by);
    pair_geom g;
    if (pair_geometry(R + 9 * i, t + 3 * i, f[i], R + 9 * j, t + 3 * j, f[j], &g)) return -2;
    eps[m] = match_residual(g.F, ax, ay, bx, by);
  }
  return 0;
}

int64_t orc_update_mask(const orc_problem *pb, const double *Rh, const double *th,
                        const double *fh, double tau, uint8_t *mask) {
  double *eps = (double *)malloc(sizeof(double) * (size_t)(pb->n_matches > 0 ? pb->n_matches : 1));
  if (!eps) return -1;
  if (orc_residuals(pb, Rh, th, fh, eps)) {
    free(eps);
    return -1;
  }
  int64_t Z = 0;
  for (int64_t m = 0; m < pb->n_matches; ++m) {
    mask[m] = (uint8_t)(mask[m] && fabs(eps[m]) < tau);
    Z += mask[m];
  }
  free(eps);
  return Z;
}

/* ---- loss and gradient -------------------------------------------------- */

typedef struct {
  int64_t n_pairs;
  int32_t *perm;
  uint8_t *swapped;
  int32_t *pair_cams;
  int64_t *seg_off;
} seg_result;

static int segment_problem(const orc_problem *pb, seg_result *s) {
  size_t n = (size_t)(pb->n_matches > 0 ? pb->n_matches : 1);
  s->perm = (int32_t *)malloc(sizeof(int32_t) * n);
  s->swapped = (uint8_t *)malloc(n);
  s->pair_cams = (int32_t *)malloc(sizeof(int32_t) * 2 * n);
  s->seg_off = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
  if (!s->perm || !s->swapped || !s->pair_cams || !s->seg_off) return -1;
  return orc_segment(pb->n_matches, pb->n_cams, pb->cam1, pb->cam2, s->perm, s->swapped,
                     s->pair_cams, s->seg_off, &s->n_pairs);
}

static void free_segments(seg_result *s) {
  free(s->perm);
  free(s->swapped);
  free(s->pair_cams);
  free(s->seg_off);
}

/* Gradient of the IRLS objective given an existing segmentation.
 * Per pair n: G_n = sum_m 2 c_m eps_m p2 p1^T (dL/dF), L_n = sum_m c_m eps_m^2;
 * then the chain rule through F = D_j E D_i, E = [u]x R_ij, u = t_ij/|t_ij|,
 * t_ij = t_j - R_ij t_i, R_ij = R_j R_i^T to the per-camera R, t and f. */
/* With weight == NULL every retained match counts once and Z is their
 * number; otherwise match m counts weight[m] and Z is the sum of the
 * retained matches' weights (the learned inlier weight taking the place of
 * the 0/1 mask, the IRLS factor kept). */
static int loss_grad_seg(const orc_problem *pb, const seg_result *s, const double *R,
                         const double *t, const double *f, const double *Rh,
                         const double *th, const double *fh, const uint8_t *mask,
                         const double *weight, double delta, double *loss, double *gR,
                         double *gt, double *gf) {
  int32_t N = pb->n_cams;
  memset(gR, 0, sizeof(double) * 9 * (size_t)N);
  memset(gt, 0, sizeof(double) * 3 * (size_t)N);
  memset(gf, 0, sizeof(double) * (size_t)N);
  *loss = 0.0;
  double Z = 0.0;
  for (int64_t m = 0; m < pb->n_matches; ++m)
    if (mask[m]) Z += weight ? weight[m] : 1.0;
  if (!(Z > 0.0) || s->n_pairs == 0) return 0;
  int64_t P = s->n_pairs;
  double *G = (double *)calloc((size_t)P * 9, sizeof(double));
  double *L = (double *)calloc((size_t)P, sizeof(double));
  int *bad = (int *)calloc((size_t)P, sizeof(int));
  if (!G || !L || !bad) {
    free(G); free(L); free(bad);
    return -1;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t n = 0; n < P; ++n) {
    int32_t i = s->pair_cams[2 * n], j = s->pair_cams[2 * n + 1];
    pair_geom g, gh;
    if (pair_geometry(R + 9 * i, t + 3 * i, f[i], R + 9 * j, t + 3 * j, f[j], &g) ||
        pair_geometry(Rh + 9 * i, th + 3 * i, fh[i], Rh + 9 * j, th + 3 * j, fh[j], &gh)) {
      bad[n] = 1;
      continue;
    }
    for (int64_t p = s->seg_off[n]; p < s->seg_off[n + 1]; ++p) {
      int64_t m = s->perm[p];
      if (!mask[m]) continue;
      int32_t ci, cj;
      double ax, ay, bx, by;
      canonical_match(pb, m, &ci, &cj, &ax, &ay, &bx, &by);
      double e = match_residual(g.F, ax, ay, bx, by);
      double eh = match_residual(gh.F, ax, ay, bx, by);
      double c = (weight ? weight[m] : 1.0) / (Z * fmax(fabs(eh), delta));
      double p1[3] = {ax, ay, 1.0}, p2[3] = {bx, by, 1.0};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) G[9 * n + a * 3 + b] += 2.0 * c * e * p2[a] * p1[b];
      L[n] += c * e * e;
    }
  }
  for (int64_t n = 0; n < P; ++n)
    if (bad[n]) {
      free(G); free(L); free(bad);
      return -2;
    }
  for (int64_t n = 0; n < P; ++n) {
    int32_t i = s->pair_cams[2 * n], j = s->pair_cams[2 * n + 1];
    pair_geom g;
    pair_geometry(R + 9 * i, t + 3 * i, f[i], R + 9 * j, t + 3 * j, f[j], &g);
    const double *Gn = G + 9 * n;
    *loss += L[n];
    /* focal lengths: F_ab = dj_a E_ab di_b, d(1/f)/df = -1/f^2 */
    double si = 0.0, sj = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 2; ++b) si += Gn[a * 3 + b] * g.F[a * 3 + b];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 3; ++b) sj += Gn[a * 3 + b] * g.F[a * 3 + b];
    gf[i] += -si / f[i];
    gf[j] += -sj / f[j];
    /* dL/dE = H = D_j G D_i */
    double H[9];
    double di[3] = {1.0 / f[i], 1.0 / f[i], 1.0}, dj[3] = {1.0 / f[j], 1.0 / f[j], 1.0};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) H[a * 3 + b] = dj[a] * Gn[a * 3 + b] * di[b];
    /* E = S R_ij with S = [u]x: dL/dS = H R_ij^T, dL/dR_ij (via E) = S^T H */
    double M[9];
    mat_mul_bt(H, g.Rij, M);
    double gu[3] = {M[7] - M[5], M[2] - M[6], M[3] - M[1]};
    /* u = t_ij/|t_ij| */
    double ugu = dot3(g.u, gu), gtij[3];
    for (int k = 0; k < 3; ++k) gtij[k] = (gu[k] - ugu * g.u[k]) / g.tnorm;
    /* t_ij = t_j - R_ij t_i */
    double RtG[3];
    mat_t_vec(g.Rij, gtij, RtG);
    for (int k = 0; k < 3; ++k) {
      gt[3 * j + k] += gtij[k];
      gt[3 * i + k] -= RtG[k];
    }
    double S[9], Q[9];
    skew(g.u, S);
    mat_mul_at(S, H, Q); /* S^T H */
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Q[a * 3 + b] -= gtij[a] * t[3 * i + b];
    /* R_ij = R_j R_i^T: dL/dR_j = Q R_i, dL/dR_i = Q^T R_j */
    double gRj[9], gRi[9];
    mat_mul(Q, R + 9 * i, gRj);
    mat_mul_at(Q, R + 9 * j, gRi);
    for (int k = 0; k < 9; ++k) {
      gR[9 * j + k] += gRj[k];
      gR[9 * i + k] += gRi[k];
    }
  }
  free(G);
  free(L);
  free(bad);
  return 0;
}

int orc_loss_grad(const orc_problem *pb, const double *R, const double *t, const double *f,
                  const double *Rh, const double *th, const double *fh, const uint8_t *mask,
                  double delta, double *loss, double *gR, double *gt, double *gf) {
  if (check_problem(pb)) return -1;
  seg_result s;
  memset(&s, 0, sizeof(s));
  if (segment_problem(pb, &s)) {
    free_segments(&s);
    return -1;
  }
  int rc = loss_grad_seg(pb, &s, R, t, f, Rh, th, fh, mask, NULL, delta, loss, gR, gt, gf);
  free_segments(&s);
  return rc;
}

int orc_loss_grad_weighted(const orc_problem *pb, const double *R, const double *t,
                           const double *f, const double *Rh, const double *th,
                           const double *fh, const uint8_t *mask, const double *weight,
                           double delta, double *loss, double *gR, double *gt, double *gf) {
  if (check_problem(pb)) return -1;
  for (int64_t m = 0; m < pb->n_matches; ++m)
    if (!(weight[m] >= 0.0)) return -3;
  seg_result s;
  memset(&s, 0, sizeof(s));
  if (segment_problem(pb, &s)) {
    free_segments(&s);
    return -1;
  }
  int rc = loss_grad_seg(pb, &s, R, t, f, Rh, th, fh, mask, weight, delta, loss, gR, gt, gf);
  free_segments(&s);
  return rc;
}

/* ---- optimiser ---------------------------------------------------------- */

void orc_adam(int64_t n, double *p, double *m, double *v, const double *g, int64_t step,
              double lr, double beta1, double beta2, double eps) {
  double bc1 = 1.0 - pow(beta1, (double)step);
  double bc2 = 1.0 - pow(beta2, (double)step);
  for (int64_t k = 0; k < n; ++k) {
    m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
    v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
    double mh = m[k] / bc1, vh = v[k] / bc2;
    p[k] -= lr * mh / (sqrt(vh) + eps);
  }
}

static double median_of(const double *x, int64_t n);

void orc_gauge_normalize(int32_t n, const double *R, double *t, int64_t n_pairs,
                         const int32_t *pair_cams, double *center, double *scale) {
  double *o = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  double mean[3] = {0.0, 0.0, 0.0};
  for (int32_t c = 0; c < n; ++c) {
    mat_t_vec(R + 9 * c, t + 3 * c, o + 3 * c);
    for (int k = 0; k < 3; ++k) {
      o[3 * c + k] = -o[3 * c + k];
      mean[k] += o[3 * c + k] / n;
    }
  }
  /* scale: median distance between the centres of the matched pairs */
  double s = 0.0;
  if (n_pairs > 0) {
    double *base = (double *)malloc(sizeof(double) * (size_t)n_pairs);
    for (int64_t k = 0; k < n_pairs; ++k) {
      const double *oi = o + 3 * pair_cams[2 * k], *oj = o + 3 * pair_cams[2 * k + 1];
      double d[3] = {oj[0] - oi[0], oj[1] - oi[1], oj[2] - oi[2]};
      base[k] = sqrt(dot3(d, d));
    }
    s = median_of(base, n_pairs);
    free(base);
  }
  if (!(s > 0.0)) s = 1.0;
  for (int32_t c = 0; c < n; ++c) {
    double on[3];
    for (int k = 0; k < 3; ++k) on[k] = (o[3 * c + k] - mean[k]) / s;
    mat_vec(R + 9 * c, on, t + 3 * c);
    for (int k = 0; k < 3; ++k) t[3 * c + k] = -t[3 * c + k];
  }
  for (int k = 0; k < 3; ++k) center[k] = mean[k];
  *scale = s;
  free(o);
}

static int dbl_cmp(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

static double median_of(const double *x, int64_t n) {
  double *y = (double *)malloc(sizeof(double) * (size_t)n);
  memcpy(y, x, sizeof(double) * (size_t)n);
  qsort(y, (size_t)n, sizeof(double), dbl_cmp);
  {
  }
  double med = (n % 2) ? y[n / 2] : 0.5 * (y[n / 2 - 1] + y[n / 2]);
  free(y);
  return med;
}

int orc_epipolar_adjust(const orc_problem *pb, const orc_options *opt, const double *R0,
                        const double *t0, const double *f0, const int32_t *intr_group,
                        double *R, double *t, double *f, double *loss_per_round,
                        int64_t *inliers, int32_t log_every, int32_t max_log, double *log_R,
                        int32_t *n_logged, uint8_t *mask_out) {
  if (check_problem(pb)) return -1;
  int32_t N = pb->n_cams;
  int64_t M = pb->n_matches;
  for (int32_t c = 0; c < N; ++c)
    if (!(f0[c] > 0.0)) return -1;
  int32_t G = 0;
  for (int32_t c = 0; c < N; ++c) {
    int32_t g = intr_group ? intr_group[c] : c;
    if (g < 0 || g >= N) return -1;
    if (g + 1 > G) G = g + 1;
  }
  seg_result s;
  memset(&s, 0, sizeof(s));
  if (segment_problem(pb, &s)) {
    free_segments(&s);
    return -1;
  }
  double *a6 = (double *)malloc(sizeof(double) * 6 * (size_t)N);
  double *logf = (double *)calloc((size_t)G, sizeof(double));
  int32_t *gcount = (int32_t *)calloc((size_t)G, sizeof(int32_t));
  double *Rh = (double *)malloc(sizeof(double) * 9 * (size_t)N);
  double *thh = (double *)malloc(sizeof(double) * 3 * (size_t)N);
  double *fh = (double *)malloc(sizeof(double) * (size_t)N);
  double *gR = (double *)malloc(sizeof(double) * 9 * (size_t)N);
  double *gt = (double *)malloc(sizeof(double) * 3 * (size_t)N);
  double *gf = (double *)malloc(sizeof(double) * (size_t)N);
  double *ga6 = (double *)malloc(sizeof(double) * 6 * (size_t)N);
  double *glogf = (double *)malloc(sizeof(double) * (size_t)G);
  double *m_a6 = (double *)malloc(sizeof(double) * 6 * (size_t)N);
  double *v_a6 = (double *)malloc(sizeof(double) * 6 * (size_t)N);
  double *m_t = (double *)malloc(sizeof(double) * 3 * (size_t)N);
  double *v_t = (double *)malloc(sizeof(double) * 3 * (size_t)N);
  double *m_f = (double *)malloc(sizeof(double) * (size_t)G);
  double *v_f = (double *)malloc(sizeof(double) * (size_t)G);
  uint8_t *mask = (uint8_t *)malloc((size_t)(M > 0 ? M : 1));
  double *eps = (double *)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
  int rc = 0;

  /* parameters: 6D rotation, translation, log focal per group */
  memcpy(t, t0, sizeof(double) * 3 * (size_t)N);
  for (int32_t c = 0; c < N; ++c) {
    orc_R_to_rot6d(R0 + 9 * c, a6 + 6 * c);
    orc_rot6d_to_R(a6 + 6 * c, R + 9 * c);
    int32_t g = intr_group ? intr_group[c] : c;
    logf[g] += log(f0[c]);
    gcount[g] += 1;
  }
  for (int32_t g = 0; g < G; ++g)
    if (gcount[g] > 0) logf[g] /= gcount[g];
  for (int32_t c = 0; c < N; ++c) f[c] = exp(logf[intr_group ? intr_group[c] : c]);
  double g_center[3] = {0.0, 0.0, 0.0}, g_scale = 1.0;
  if (opt->gauge_normalize)
    orc_gauge_normalize(N, R, t, s.n_pairs, s.pair_cams, g_center, &g_scale);
  for (int64_t m = 0; m < M; ++m) mask[m] = 1;
  int32_t nlog = 0;
  int64_t it_global = 0;
  int64_t adam_step = 0;

  for (int32_t r = 0; r < opt->rounds; ++r) {
    loss_per_round[r] = NAN;
    inliers[r] = -1;
  }
  double prev_tau_px = -1.0;
  for (int32_t r = 0; r < opt->rounds && rc == 0; ++r) {
    double tau_px = opt->tau_px_init * pow(opt->tau_decay, (double)r);
    if (tau_px < opt->tau_px_min) tau_px = opt->tau_px_min;
    if (opt->converge_deg > 0.0 && r > 0 && tau_px == prev_tau_px) {
      /* early exit (a batching addition; the paper runs a fixed schedule):
       * Rh, fh still hold the previous round's snapshot */
      double mean_rot = 0.0, mean_f = 0.0;
      for (int32_t c = 0; c < N; ++c) {
        double tr = 0.0;
        for (int k = 0; k < 9; ++k) tr += Rh[9 * c + k] * R[9 * c + k]; /* tr(Rh^T R) */
        double ca = 0.5 * (tr - 1.0);
        if (ca > 1.0) ca = 1.0;
        if (ca < -1.0) ca = -1.0;
        mean_rot += acos(ca) / N;
        mean_f += fabs(log(f[c] / fh[c])) / N;
      }
      const double to_deg = 57.29577951308232; /* 180 / pi */
      if (mean_rot * to_deg < opt->converge_deg && mean_f * to_deg < opt->converge_deg) break;
    }
    prev_tau_px = tau_px;
    /* snapshot and filter (Method > Epipolar Adjustment, re-weighting rounds) */
    memcpy(Rh, R, sizeof(double) * 9 * (size_t)N);
    memcpy(thh, t, sizeof(double) * 3 * (size_t)N);
    memcpy(fh, f, sizeof(double) * (size_t)N);
    double tau = tau_px / median_of(fh, N);
    if (orc_residuals(pb, Rh, thh, fh, eps)) {
      rc = -2;
      break;
    }
    int64_t Z = 0;
    for (int64_t m = 0; m < M; ++m) {
      mask[m] = (uint8_t)(mask[m] && fabs(eps[m]) < tau);
      Z += mask[m];
    }
    inliers[r] = Z;
    if (opt->reset_moments || r == 0) {
      memset(m_a6, 0, sizeof(double) * 6 * (size_t)N);
      memset(v_a6, 0, sizeof(double) * 6 * (size_t)N);
      memset(m_t, 0, sizeof(double) * 3 * (size_t)N);
      memset(v_t, 0, sizeof(double) * 3 * (size_t)N);
      memset(m_f, 0, sizeof(double) * (size_t)G);
      memset(v_f, 0, sizeof(double) * (size_t)G);
      adam_step = 0;
    }
    const double lr_scale = pow(opt->lr_decay, (double)r);
    double loss = 0.0;
    for (int32_t k = 0; k < opt->iters_per_round; ++k) {
      rc = loss_grad_seg(pb, &s, R, t, f, Rh, thh, fh, mask, NULL, opt->delta, &loss, gR, gt, gf);
      if (rc) break;
      for (int32_t c = 0; c < N; ++c) orc_rot6d_backward(a6 + 6 * c, gR + 9 * c, ga6 + 6 * c);
      memset(glogf, 0, sizeof(double) * (size_t)G);
      for (int32_t c = 0; c < N; ++c) glogf[intr_group ? intr_group[c] : c] += gf[c] * f[c];
      int64_t step = ++adam_step;
      orc_adam(6 * (int64_t)N, a6, m_a6, v_a6, ga6, step, opt->lr_rot * lr_scale, opt->beta1,
               opt->beta2, opt->adam_eps);
      orc_adam(3 * (int64_t)N, t, m_t, v_t, gt, step, opt->lr_t * lr_scale, opt->beta1,
               opt->beta2, opt->adam_eps);
      if (opt->optimize_focal)
        orc_adam(G, logf, m_f, v_f, glogf, step, opt->lr_logf * lr_scale, opt->beta1,
                 opt->beta2, opt->adam_eps);
      for (int32_t c = 0; c < N; ++c) {
        orc_rot6d_to_R(a6 + 6 * c, R + 9 * c);
        f[c] = exp(logf[intr_group ? intr_group[c] : c]);
      }
      ++it_global;
      if (log_R && log_every > 0 && (it_global % log_every) == 0 && nlog < max_log) {
        memcpy(log_R + (size_t)nlog * 9 * N, R, sizeof(double) * 9 * (size_t)N);
        ++nlog;
      }
    }
    loss_per_round[r] = loss;
  }
  if (n_logged) *n_logged = nlog;
  if (mask_out) memcpy(mask_out, mask, (size_t)M);
  /* back to the caller's frame: centre o = scale * o' + center */
  if (opt->gauge_normalize) {
    for (int32_t c = 0; c < N; ++c) {
      double o[3], on[3];
      mat_t_vec(R + 9 * c, t + 3 * c, o);
      for (int k = 0; k < 3; ++k) on[k] = -o[k] * g_scale + g_center[k];
      mat_vec(R + 9 * c, on, t + 3 * c);
      for (int k = 0; k < 3; ++k) t[3 * c + k] = -t[3 * c + k];
    }
  }
  free(a6); free(logf); free(gcount); free(Rh); free(thh); free(fh); free(gR); free(gt);
  free(gf); free(ga6); free(glogf); free(m_a6); free(v_a6); free(m_t); free(v_t);
  free(m_f); free(v_f); free(mask); free(eps);
  free_segments(&s);
  return rc;
}

/* ---- learned inlier weights (see fea_oracle.h) ------------------------- */

static double feature_residual(double e, double fbar) {
  return log(1.0 + fabs(e) * fbar) / log(1.0 + 256.0);
}

int orc_mlp_features(const orc_problem *pb, const double *R0, const double *t0, const double *f0,
                     const double *R1, const double *t1, const double *f1, const double *R2,
                     const double *t2, const double *f2, double *feat) {
  int64_t M = pb->n_matches;
  int32_t N = pb->n_cams;
  const double *Rs[3] = {R0, R1, R2}, *ts[3] = {t0, t1, t2}, *fs[3] = {f0, f1, f2};
  double *eps = (double *)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
  if (!eps) return -1;
  for (int k = 0; k < 3; ++k) {
    if (orc_residuals(pb, Rs[k], ts[k], fs[k], eps)) {
      free(eps);
      return -1;
    }
    double fbar = median_of(fs[k], N);
    for (int64_t m = 0; m < M; ++m) feat[ORC_MLP_NFEAT * m + k] = feature_residual(eps[m], fbar);
  }
  free(eps);
  for (int64_t m = 0; m < M; ++m) {
    /* keypoints in the pair's own orientation: the camera with the lower
     * index first, as the pair n = (i, j), i < j, is defined */
    int32_t c1 = pb->cam1[m], c2 = pb->cam2[m];
    double u1 = pb->x1[m], v1 = pb->y1[m], u2 = pb->x2[m], v2 = pb->y2[m];
    if (c1 > c2) {
      int32_t tc = c1;
      c1 = c2;
      c2 = tc;
      double tu = u1, tv = v1;
      u1 = u2;
      v1 = v2;
      u2 = tu;
      v2 = tv;
    }
    double *x = feat + ORC_MLP_NFEAT * m;
    x[3] = u1 / pb->cx[c1] - 1.0;
    x[4] = v1 / pb->cy[c1] - 1.0;
    x[5] = u2 / pb->cx[c2] - 1.0;
    x[6] = v2 / pb->cy[c2] - 1.0;
    /* optical axis of camera c in world coordinates: third row of R_c */
    const double *za = R0 + 9 * c1 + 6, *zb = R0 + 9 * c2 + 6;
    double cosang = dot3(za, zb);
    if (cosang > 1.0) cosang = 1.0;
    if (cosang < -1.0) cosang = -1.0;
    x[7] = acos(cosang) / (0.5 * 3.14159265358979323846);
  }
  return 0;
}

typedef struct {
  const double *W1, *b1, *W2, *b2, *w3, *b3;
} mlp_view;

static mlp_view mlp_unpack(const double *p) {
  mlp_view v;
  v.W1 = p;
  v.b1 = v.W1 + ORC_MLP_HIDDEN * ORC_MLP_NFEAT;
  v.W2 = v.b1 + ORC_MLP_HIDDEN;
  v.b2 = v.W2 + ORC_MLP_HIDDEN * ORC_MLP_HIDDEN;
  v.w3 = v.b2 + ORC_MLP_HIDDEN;
  v.b3 = v.w3 + ORC_MLP_HIDDEN;
  return v;
}

/* One sample: hidden activations and output logit. */
static double mlp_sample(const mlp_view *v, const double *x, double *h1, double *h2) {
  for (int i = 0; i < ORC_MLP_HIDDEN; ++i) {
    double z = v->b1[i];
    for (int k = 0; k < ORC_MLP_NFEAT; ++k) z += v->W1[ORC_MLP_NFEAT * i + k] * x[k];
    h1[i] = z > 0.0 ? z : 0.0;
  }
  for (int i = 0; i < ORC_MLP_HIDDEN; ++i) {
    double z = v->b2[i];
    for (int k = 0; k < ORC_MLP_HIDDEN; ++k) z += v->W2[ORC_MLP_HIDDEN * i + k] * h1[k];
    h2[i] = z > 0.0 ? z : 0.0;
  }
  double z3 = v->b3[0];
  for (int k = 0; k < ORC_MLP_HIDDEN; ++k) z3 += v->w3[k] * h2[k];
  return z3;
}

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }

void orc_mlp_forward(int64_t n, const double *feat, const double *params, double *y) {
  mlp_view v = mlp_unpack(params);
  double h1[ORC_MLP_HIDDEN], h2[ORC_MLP_HIDDEN];
  for (int64_t m = 0; m < n; ++m) y[m] = sigmoid(mlp_sample(&v, feat + ORC_MLP_NFEAT * m, h1, h2));
}

double orc_mlp_bce_grad(int64_t n, const double *feat, const double *target, const double *params,
                        double *grad) {
  mlp_view v = mlp_unpack(params);
  memset(grad, 0, sizeof(double) * ORC_MLP_NPARAM);
  double *gW1 = grad, *gb1 = gW1 + ORC_MLP_HIDDEN * ORC_MLP_NFEAT, *gW2 = gb1 + ORC_MLP_HIDDEN;
  double *gb2 = gW2 + ORC_MLP_HIDDEN * ORC_MLP_HIDDEN, *gw3 = gb2 + ORC_MLP_HIDDEN,
         *gb3 = gw3 + ORC_MLP_HIDDEN;
  double h1[ORC_MLP_HIDDEN], h2[ORC_MLP_HIDDEN], d2[ORC_MLP_HIDDEN], d1[ORC_MLP_HIDDEN];
  double loss = 0.0;
  for (int64_t m = 0; m < n; ++m) {
    const double *x = feat + ORC_MLP_NFEAT * m;
    double z3 = mlp_sample(&v, x, h1, h2);
    double t = target[m];
    /* BCE of sigmoid(z) written stably: max(z,0) - z t + log(1 + exp(-|z|)) */
    loss += (z3 > 0 ? z3 : 0.0) - z3 * t + log1p(exp(-fabs(z3)));
    double dz3 = (sigmoid(z3) - t) / (double)n;
    gb3[0] += dz3;
    for (int k = 0; k < ORC_MLP_HIDDEN; ++k) {
      gw3[k] += dz3 * h2[k];
      d2[k] = h2[k] > 0.0 ? dz3 * v.w3[k] : 0.0;
    }
    for (int i = 0; i < ORC_MLP_HIDDEN; ++i) {
      gb2[i] += d2[i];
      for (int k = 0; k < ORC_MLP_HIDDEN; ++k) gW2[ORC_MLP_HIDDEN * i + k] += d2[i] * h1[k];
    }
    for (int k = 0; k < ORC_MLP_HIDDEN; ++k) {
      double s = 0.0;
      for (int i = 0; i < ORC_MLP_HIDDEN; ++i) s += v.W2[ORC_MLP_HIDDEN * i + k] * d2[i];
      d1[k] = h1[k] > 0.0 ? s : 0.0;
    }
    for (int i = 0; i < ORC_MLP_HIDDEN; ++i) {
      gb1[i] += d1[i];
      for (int k = 0; k < ORC_MLP_NFEAT; ++k) gW1[ORC_MLP_NFEAT * i + k] += d1[i] * x[k];
    }
  }
  return loss / (double)(n > 0 ? n : 1);
}

/* ---- relative translations (Global Translation > Relative translation) --- */

/* Depth signs of the two-view triangulation of one match for a relative
 * translation t (camera j frame): the depths (l1, l2) minimising
 * |l1 a - l2 b + t|^2 with a = R_ij x~1, b = x~2 solve the 2x2 normal
 * equations [a.a, -a.b; -a.b, b.b] (l1, l2) = (-a.t, b.t).  Returns +1 when
 * both depths are positive, -1 when both are negative, 0 otherwise (also
 * when the rays are parallel and the depths undefined). */
static int cheirality_vote(const double a[3], const double b[3], const double t[3]) {
  const double aa = dot3(a, a), bb = dot3(b, b), ab = dot3(a, b);
  const double at = dot3(a, t), bt = dot3(b, t);
  const double det = aa * bb - ab * ab;
  if (!(det > 0.0)) return 0;
  const double l1 = (-at * bb + ab * bt) / det;
  const double l2 = (aa * bt - ab * at) / det;
  if (l1 > 0.0 && l2 > 0.0) return 1;
  if (l1 < 0.0 && l2 < 0.0) return -1;
  return 0;
}

int orc_rel_trans(const orc_problem *pb, const double *R, const double *f, int32_t n_cand,
                  const double *cand, double tau, int64_t *n_pairs_out, int32_t *pair_cams,
                  double *scores, int32_t *best, double *t_rel, int64_t *vote) {
  if (check_problem(pb) || n_cand < 1) return -1;
  seg_result s;
  if (segment_problem(pb, &s)) {
    free_segments(&s);
    return -1;
  }
  const int64_t P = s.n_pairs;
  *n_pairs_out = P;
  int rc = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t n = 0; n < P; ++n) {
    const int32_t i = s.pair_cams[2 * n], j = s.pair_cams[2 * n + 1];
    pair_cams[2 * n] = i;
    pair_cams[2 * n + 1] = j;
    double Rij[9];
    mat_mul_bt(R + 9 * j, R + 9 * i, Rij);
    const int64_t b0 = s.seg_off[n], b1 = s.seg_off[n + 1];
    double best_score = 0.0;
    int32_t best_k = -1;
    for (int32_t k = 0; k < n_cand; ++k) {
      /* E = [u]x R_ij for the candidate direction u; eps = x~2^T E x~1 */
      double S[9], E[9];
      skew(cand + 3 * k, S);
      mat_mul(S, Rij, E);
      double sum = 0.0;
      for (int64_t p = b0; p < b1; ++p) {
        int32_t ci, cj;
        double ax, ay, bx, by;
        canonical_match(pb, s.perm[p], &ci, &cj, &ax, &ay, &bx, &by);
        const double x1[3] = {ax / f[i], ay / f[i], 1.0}, x2[3] = {bx / f[j], by / f[j], 1.0};
        double Ex1[3];
        mat_vec(E, x1, Ex1);
        const double e = fabs(dot3(x2, Ex1));
        sum += e < tau ? e : tau;
      }
      const double mean = sum / (double)(b1 - b0);
      if (scores) scores[n * n_cand + k] = mean;
      if (best_k < 0 || mean < best_score) {
        best_score = mean;
        best_k = k;
      }
    }
    best[n] = best_k;
    const double *u = cand + 3 * best_k;
    double S[9], E[9];
    skew(u, S);
    mat_mul(S, Rij, E);
    int64_t v = 0;
    for (int64_t p = b0; p < b1; ++p) {
      int32_t ci, cj;
      double ax, ay, bx, by;
      canonical_match(pb, s.perm[p], &ci, &cj, &ax, &ay, &bx, &by);
      const double x1[3] = {ax / f[i], ay / f[i], 1.0}, x2[3] = {bx / f[j], by / f[j], 1.0};
      double a[3], Ex1[3];
      mat_vec(E, x1, Ex1);
      if (!(fabs(dot3(x2, Ex1)) < tau)) continue; /* only matches the chosen direction explains */
      mat_vec(Rij, x1, a);
      v += cheirality_vote(a, x2, u);
    }
    vote[n] = v;
    const double sg = v >= 0 ? 1.0 : -1.0;
    for (int k = 0; k < 3; ++k) t_rel[3 * n + k] = sg * u[k];
  }
  free_segments(&s);
  return rc;
}

/* ---- global translation alignment (Global Translation) ------------------ */

int orc_ta_targets(int32_t n_cams, int64_t n_pairs, const int32_t *pair_i,
                   const int32_t *pair_j, const double *R, const double *t_rel, double *target) {
  for (int64_t p = 0; p < n_pairs; ++p) {
    const int32_t i = pair_i[p], j = pair_j[p];
    if (i < 0 || j < 0 || i >= n_cams || j >= n_cams || i == j) return -1;
    const double nt = sqrt(dot3(t_rel + 3 * p, t_rel + 3 * p));
    if (!(nt > 0.0)) return -2;
    double u[3] = {t_rel[3 * p] / nt, t_rel[3 * p + 1] / nt, t_rel[3 * p + 2] / nt}, o[3];
    mat_t_vec(R + 9 * j, u, o); /* R_j^T u */
    for (int k = 0; k < 3; ++k) target[3 * p + k] = -o[k];
  }
  return 0;
}

static double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

double orc_ta_loss_grad(int32_t n_cams, int64_t n_pairs, const int32_t *pair_i,
                        const int32_t *pair_j, const double *target, const double *o,
                        double *grad, double *pair_loss) {
  if (grad)
    for (int64_t k = 0; k < 3 * (int64_t)n_cams; ++k) grad[k] = 0.0;
  double L = 0.0;
  for (int64_t p = 0; p < n_pairs; ++p) {
    const int32_t i = pair_i[p], j = pair_j[p];
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = o[3 * j + k] - o[3 * i + k];
    const double nd = sqrt(dot3(d, d));
    double lp = 0.0;
    if (nd > 0.0) {
      double n[3], r[3], s[3];
      for (int k = 0; k < 3; ++k) {
        n[k] = d[k] / nd;
        r[k] = n[k] - target[3 * p + k];
        lp += fabs(r[k]);
        s[k] = sgn(r[k]) / (double)n_pairs; /* dL/dn */
      }
      if (grad) {
        /* n = d/|d|: dn/dd = (I - n n^T)/|d| */
        const double ns = dot3(n, s);
        for (int k = 0; k < 3; ++k) {
          const double gd = (s[k] - n[k] * ns) / nd;
          grad[3 * j + k] += gd;
          grad[3 * i + k] -= gd;
        }
      }
    }
    if (pair_loss) pair_loss[p] = lp;
    L += lp;
  }
  return n_pairs > 0 ? L / (double)n_pairs : 0.0;
}

/* Centre at the origin and rescale to unit mean norm (the alignment of the
 * multiple-initialisation merge). */
static int ta_align(int32_t N, double *o) {
  double c[3] = {0, 0, 0};
  for (int32_t i = 0; i < N; ++i)
    for (int k = 0; k < 3; ++k) c[k] += o[3 * i + k];
  for (int k = 0; k < 3; ++k) c[k] /= (double)N;
  double s = 0.0;
  for (int32_t i = 0; i < N; ++i) {
    double d[3] = {o[3 * i] - c[0], o[3 * i + 1] - c[1], o[3 * i + 2] - c[2]};
    s += sqrt(dot3(d, d));
  }
  s /= (double)N;
  if (!(s > 0.0)) return -1;
  for (int32_t i = 0; i < N; ++i)
    for (int k = 0; k < 3; ++k) o[3 * i + k] = (o[3 * i + k] - c[k]) / s;
  return 0;
}

/* Adam on the camera centres: iters steps, learning rate decayed
 * geometrically from lr to lr * end_frac over the run (step k uses
 * lr * end_frac^(k / iters)). */
static void ta_adam_run(int32_t N, int64_t P, const int32_t *pi, const int32_t *pj,
                        const double *target, double *o, int32_t iters, double lr,
                        const orc_ta_options *opt) {
  const size_t n3 = 3 * (size_t)N;
  double *g = (double *)calloc(n3, sizeof(double));
  double *m = (double *)calloc(n3, sizeof(double));
  double *v = (double *)calloc(n3, sizeof(double));
  for (int32_t k = 0; k < iters; ++k) {
    orc_ta_loss_grad(N, P, pi, pj, target, o, g, NULL);
    const double lr_k = lr * pow(opt->lr_end_frac, (double)k / (double)iters);
    orc_adam((int64_t)n3, o, m, v, g, k + 1, lr_k, opt->beta1, opt->beta2, opt->adam_eps);
  }
  free(g);
  free(m);
  free(v);
}

void orc_ta_default_options(orc_ta_options *o) {
  o->iters_run = 1500;
  o->iters_final = 500;
  o->lr = 2e-2;
  o->lr_final = 2e-3;
  o->lr_end_frac = 1e-3;
  o->beta1 = 0.9;
  o->beta2 = 0.999;
  o->adam_eps = 1e-12;
}

int orc_ta_solve(int32_t N, int64_t P, const int32_t *pi, const int32_t *pj, const double *target,
                 int32_t n_runs, const double *o_init, const orc_ta_options *opt, double *o_out,
                 double *run_o, double *cam_loss, int32_t *run_of_cam, double *run_loss,
                 double *final_loss) {
  if (N < 1 || n_runs < 1) return -1;
  const size_t n3 = 3 * (size_t)N;
  double *ro = (double *)malloc(sizeof(double) * n3 * (size_t)n_runs);
  double *cl = (double *)calloc((size_t)N * (size_t)n_runs, sizeof(double));
  double *pl = (double *)malloc(sizeof(double) * (size_t)(P > 0 ? P : 1));
  int32_t *deg = (int32_t *)calloc((size_t)N, sizeof(int32_t));
  int rc = 0;
  for (int64_t p = 0; p < P; ++p) {
    deg[pi[p]]++;
    deg[pj[p]]++;
  }
  for (int32_t r = 0; r < n_runs && !rc; ++r) {
    double *o = ro + n3 * (size_t)r;
    memcpy(o, o_init + n3 * (size_t)r, sizeof(double) * n3);
    ta_adam_run(N, P, pi, pj, target, o, opt->iters_run, opt->lr, opt);
    if (ta_align(N, o)) rc = -2;
    const double L = orc_ta_loss_grad(N, P, pi, pj, target, o, NULL, pl);
    if (run_loss) run_loss[r] = L;
    /* mean loss of each camera over its pairs */
    double *c = cl + (size_t)N * (size_t)r;
    for (int64_t p = 0; p < P; ++p) {
      c[pi[p]] += pl[p];
      c[pj[p]] += pl[p];
    }
    for (int32_t i = 0; i < N; ++i) c[i] = deg[i] ? c[i] / (double)deg[i] : 0.0;
  }
  if (!rc) {
    for (int32_t i = 0; i < N; ++i) {
      int32_t b = 0;
      for (int32_t r = 1; r < n_runs; ++r)
        if (cl[(size_t)N * r + i] < cl[(size_t)N * b + i]) b = r;
      run_of_cam[i] = b;
      for (int k = 0; k < 3; ++k) o_out[3 * i + k] = ro[n3 * (size_t)b + 3 * i + k];
    }
    ta_adam_run(N, P, pi, pj, target, o_out, opt->iters_final, opt->lr_final, opt);
    if (ta_align(N, o_out)) rc = -2;
    const double L = orc_ta_loss_grad(N, P, pi, pj, target, o_out, NULL, NULL);
    if (final_loss) *final_loss = L;
  }
  if (run_o) memcpy(run_o, ro, sizeof(double) * n3 * (size_t)n_runs);
  if (cam_loss) memcpy(cam_loss, cl, sizeof(double) * (size_t)N * (size_t)n_runs);
  free(ro);
  free(cl);
  free(pl);
  free(deg);
  return rc;
}
