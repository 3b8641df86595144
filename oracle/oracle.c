/* CPU oracle for SciFi Seeding + VELO-SciFi Matching (FP64).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.
 *
 * It follows the paper's steps in the paper's order, one plain loop per step:
 *   Sec. 3.3   XZ seeding: T1 x T3 doublets in the window of eq. tolHp shifted
 *              by eq. alphacorr, third hit in T2 around the prediction of
 *              Delta x2 = k3 c_x, extension to the remaining x-layers (1 mm),
 *              least-squares fit of eq. trackequation with d_ratio fixed;
 *   Sec. 3.3.4 O(n) clone killing with the score of eq. seed_clone_score;
 *   Sec. 3.4   iterative UV seeding (2 mm, t_y averaging, y-z line fit);
 *   Sec. 4     Matching: kink plane of eq. z_match (Table 1), y plane at
 *              10 m, preselection, chi2_match, final clone removal.
 * Where the paper is silent the documented reading is taken; each is marked
 * READING below.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

/* Layer roles (Sec. 1: x-u-v-x per station). */
static const int X_LAYERS[6] = {0, 3, 4, 7, 8, 11};
static const int UV_LAYERS[6] = {1, 2, 5, 6, 9, 10};
/* READING: iteration 0 starts from the first x-layer of each station,
 * iteration 1 from the last one (disjoint sets, Sec. 3.3). Order T1, T2, T3.
 * The optional third iteration (after the clean-up) uses iteration 0's
 * layers. */
static const int INIT_LAYERS[3][3] = {{0, 4, 8}, {3, 7, 11}, {0, 4, 8}};
static const int EXT_LAYERS[3][3] = {{3, 7, 11}, {0, 4, 8}, {3, 7, 11}};

void orc_default_geom(orc_geom *g) {
  static const double z[ORC_NL] = {7826.0, 7896.0, 7966.0, 8036.0, 8527.5, 8597.5,
                                   8667.5, 8737.5, 9229.0, 9299.0, 9369.0, 9439.0};
  const double t5 = tan(5.0 * M_PI / 180.0);
  for (int l = 0; l < ORC_NL; ++l) {
    g->z[l] = z[l];
    int kind = l % 4; /* x u v x */
    g->tan_a[l] = kind == 1 ? t5 : (kind == 2 ? -t5 : 0.0);
  }
  g->z_ref = 8525.0; /* Sec. 3.1 */
  /* READING: UT layer positions and stereo angles (the paper gives none) */
  static const double uz[ORC_NUT] = {2327.5, 2372.5, 2597.5, 2642.5};
  for (int i = 0; i < ORC_NUT; ++i) {
    g->ut_z[i] = uz[i];
    g->ut_tan[i] = (i == 1) ? t5 : (i == 2 ? -t5 : 0.0);
  }
}

void orc_default_params(orc_params *p) {
  memset(p, 0, sizeof(*p));
  p->p_min = 3000.0;          /* Sec. 3.2: p_min > 3 GeV/c, in MeV */
  p->invp_a = 1.6322e-7;      /* eq. invp; READING: per MeV/c (see DESIGN) */
  p->invp_b = -5.0217e-12;
  p->alpha0 = 2.180e6;        /* eq. alphacorr */
  p->alpha1 = -1073.0;
  p->d_ratio = -3.0e-4;       /* READING: value not printed */
  p->kappa_c = 3.0e-3;        /* READING: third-hit band centre */
  p->t2_tol0 = 0.5;           /* READING: third-hit band width */
  p->t2_tol1 = 0.5;
  p->ext_tol = 1.0;           /* Sec. 3.2: 1 mm */
  p->min_x_hits = 5;          /* Sec. 3.2: at least 5 of 6 x-layers */
  p->sigma_x = 0.07;          /* READING: hit resolution */
  p->chi2x_max = 6.0;         /* READING: "bad chi2" */
  p->uv_tol = 2.0;            /* Sec. 3.4: 2 mm */
  p->y_max = 2500.0;          /* READING: selection window = the half's y range */
  p->min_uv_hits = 4;         /* READING */
  p->chi2y_max = 6.0;         /* READING */
  p->zm[0] = 5287.6;          /* Table 1 */
  p->zm[1] = -7.98878;
  p->zm[2] = 317.683;
  p->zm[3] = 0.0119379;
  p->zm[4] = -1418.42;
  p->z_ymatch = 10000.0;      /* Sec. 4: y matched at 10 m */
  p->z_state = 9439.0;        /* READING: SciFi state at the last layer */
  p->max_dx = 20.0;           /* Sec. 4.2 preselection */
  p->max_dy = 150.0;
  p->max_dtx = 1.5;
  p->max_dty = 0.02;
  p->tolx_scale = 4.0 / 5.0;  /* Sec. 4.2 tolerances */
  p->tolx_a = 10.12;
  p->tolx_b = 101.0;
  p->toly_scale = 1.0 / 5.0;
  p->toly_a = 1.59;
  p->toly_b = 212.1;
  p->tol_tx = 0.5;
  p->tol_ty = 1.0 / 937.5;
  p->chi2m_max = 2.0;
  p->polarity = 1.0;
  p->uv_mode = 0;             /* Sec. 3.4: the iterative search is the default */
  p->hough_bins = 64;         /* READING: the Hough variant's binning is not printed */
  p->hough_best = 8;          /* Sec. 3.4: up to eight best bins */
  p->hough_fine = 4;          /* READING: "several finer bins" */
  p->hough_min = 2;           /* READING */
  p->final_sel = 0;           /* READING: no network weights are published */
  p->ghost_cut = 0.8;         /* Sec. 4.4: ghost probability < 0.8 */
  p->clone_gap = 0.05;        /* Sec. 4.4: clone if at least 0.05 higher */
  p->third_iter = 0;          /* Sec. 3: the HLT1 form runs two iterations */
  p->p_min3 = 1500.0;         /* READING: the third iteration's windows open for 1.5 GeV/c */
  p->ut_mode = 0;             /* Sec. 4.3: UT hits are optional */
  p->ut_min_hits = 3;         /* Sec. 4.3: more than two UT hits */
  p->a_gamma = 7.707063e-11;  /* Table 1 */
  p->b_gamma = -7.817364e-3;
  /* Table 2, layers UTaX, UTaU, UTbV, UTbX; no loose window is printed for
   * UTbX and no tight one for UTaX (hi = 0) */
  static const double la[ORC_NUT] = {0.8333, 0.8333, 1.3333, 0.0};
  static const double lb[ORC_NUT] = {3.3333, 3.3333, 3.3333, 0.0};
  static const double llo[ORC_NUT] = {1.2, 1.2, 1.5, 0.0};
  static const double lhi[ORC_NUT] = {8.5, 8.5, 9.5, 0.0};
  static const double ta[ORC_NUT] = {0.0, 0.2, 0.4, 0.4};
  static const double tb[ORC_NUT] = {0.0, 0.6, 1.2, 1.2};
  static const double tlo[ORC_NUT] = {0.0, 0.5, 1.0, 1.0};
  static const double thi[ORC_NUT] = {0.0, 2.0, 4.0, 4.0};
  for (int i = 0; i < ORC_NUT; ++i) {
    p->ut_loose_a[i] = la[i]; p->ut_loose_b[i] = lb[i];
    p->ut_loose_lo[i] = llo[i]; p->ut_loose_hi[i] = lhi[i];
    p->ut_tight_a[i] = ta[i]; p->ut_tight_b[i] = tb[i];
    p->ut_tight_lo[i] = tlo[i]; p->ut_tight_hi[i] = thi[i];
  }
}

/* ---------------------------------------------------------- helpers ----- */

/* g(u) = u^2 (1 + d_ratio u): the non-linear part of eq. trackequation. */
static double gfun(double u, double d) { return u * u * (1.0 + d * u); }

/* x(z) of eq. trackequation. */
static double xmodel(double a, double b, double c, double z, double zref, double d) {
  double u = z - zref;
  return a + b * u + c * gfun(u, d);
}

/* First index i in [lo, hi) with x[i] >= v (x sorted ascending), else hi. */
static int first_at_least(const float *x, int lo, int hi, double v) {
  while (lo < hi) {
    int mid = lo + (hi - lo) / 2;
    if ((double)x[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

/* Closest hit to `pred` among hits of [lo, hi) inside [pred - tol, pred + tol].
 * READING: distances closer than ORC_TIE_MM are a tie, won by the lower
 * position (a prediction midway between two hits, as a mean t_y of two hits of
 * one layer gives, is a tie that rounding alone would otherwise break); the
 * hits are visited in ascending position and a later hit replaces the current
 * one only if it is closer by more than ORC_TIE_MM.  Returns -1 if none. */
#define ORC_TIE_MM 1e-6
static int closest_in_window(const float *x, int lo, int hi, double pred, double tol) {
  int best = -1;
  double bestd = 0.0;
  for (int i = first_at_least(x, lo, hi, pred - tol); i < hi && (double)x[i] <= pred + tol; ++i) {
    double d = fabs((double)x[i] - pred);
    if (best < 0 || d < bestd - ORC_TIE_MM) { best = i; bestd = d; }
  }
  return best;
}

/* Off in a worker of an orc_run call made with log_margins = 0: the margin
 * bookkeeping that costs a rescan or a pass of its own is then skipped. */
static _Thread_local int g_nolog = 0;

/* Margin of a closest-hit decision (see ORC_NEAR in oracle.h): with a hit
 * chosen, the smaller of (tol - d)/tol and (d_other - d)/tol over the other
 * hits in the window; with none, (d - tol)/tol of the nearest hit outside.
 * INFINITY when the zone is empty. */
static double closest_margin(const float *x, int lo, int hi, double pred, double tol, int best) {
  double m = INFINITY;
  if (best >= 0) {
    const double d1 = fabs((double)x[best] - pred);
    m = (tol - d1) / tol;
    for (int i = first_at_least(x, lo, hi, pred - tol); i < hi && (double)x[i] <= pred + tol; ++i) {
      if (i == best) continue;
      const double r = fabs(fabs((double)x[i] - pred) - d1) / tol;
      if (r < m) m = r;
    }
  } else {
    const int j = first_at_least(x, lo, hi, pred);
    if (j < hi) m = fmin(m, ((double)x[j] - pred - tol) / tol);
    if (j > lo) m = fmin(m, (pred - (double)x[j - 1] - tol) / tol);
  }
  return fabs(m);
}

/* Margin of a cut q < cut (or |q| <= cut for a window), either way. */
static double cut_margin(double q, double cut) { return fabs(cut - q) / fabs(cut); }

/* Solve the 3x3 system A p = r by Gaussian elimination with partial pivoting. */
static int solve3(double A[3][3], double r[3], double p[3]) {
  for (int k = 0; k < 3; ++k) {
    int piv = k;
    for (int i = k + 1; i < 3; ++i) if (fabs(A[i][k]) > fabs(A[piv][k])) piv = i;
    if (A[piv][k] == 0.0) return -1;
    if (piv != k) {
      for (int j = 0; j < 3; ++j) { double t = A[k][j]; A[k][j] = A[piv][j]; A[piv][j] = t; }
      double t = r[k]; r[k] = r[piv]; r[piv] = t;
    }
    for (int i = k + 1; i < 3; ++i) {
      double f = A[i][k] / A[k][k];
      for (int j = k; j < 3; ++j) A[i][j] -= f * A[k][j];
      r[i] -= f * r[k];
    }
  }
  for (int k = 2; k >= 0; --k) {
    double s = r[k];
    for (int j = k + 1; j < 3; ++j) s -= A[k][j] * p[j];
    p[k] = s / A[k][k];
  }
  return 0;
}

/* Least-squares fit of eq. trackequation, x = a + b u + c g(u), u = z - z_ref,
 * d_ratio fixed, equal weights (Sec. 3.2 last step).  The normal equations are
 * written for the scaled basis [1, u/S, g(u)/S^2] (S = 1 m) so that they are
 * well conditioned; the parameters are unscaled on return. */
static int fit_xz(const double *z, const double *x, int n, double zref, double d,
                  double *a, double *b, double *c) {
  const double S = 1000.0;
  double A[3][3] = {{0}}, r[3] = {0}, q[3];
  for (int i = 0; i < n; ++i) {
    double u = z[i] - zref;
    double f[3] = {1.0, u / S, gfun(u, d) / (S * S)};
    for (int j = 0; j < 3; ++j) {
      r[j] += f[j] * x[i];
      for (int k = 0; k < 3; ++k) A[j][k] += f[j] * f[k];
    }
  }
  if (solve3(A, r, q)) return -1;
  *a = q[0];
  *b = q[1] / S;
  *c = q[2] / (S * S);
  return 0;
}

/* Weighted least-squares straight line y = y0 + t (z - z_ref) (Sec. 3.4). */
static void fit_line(const double *z, const double *y, const double *w, int n, double zref,
                     double *y0, double *t) {
  double s0 = 0, s1 = 0, s2 = 0, r0 = 0, r1 = 0;
  for (int i = 0; i < n; ++i) {
    double u = z[i] - zref;
    s0 += w[i]; s1 += w[i] * u; s2 += w[i] * u * u;
    r0 += w[i] * y[i]; r1 += w[i] * u * y[i];
  }
  double det = s0 * s2 - s1 * s1;
  *y0 = (r0 * s2 - r1 * s1) / det;
  *t = (s0 * r1 - s1 * r0) / det;
}

/* ------------------------------------------------------ XZ seeding ------ */

/* Window constants of one iteration, from the nominal z of its T1 and T3
 * layers: out[0] = Delta x3^max of eq. tolHp (the T3 half-width for tracks
 * above p_min), out[1] = alpha_corr of eq. alphacorr (the window-centre
 * shift, READING: in mm). */
static void window_constants(const orc_geom *g, const orc_params *P, int it, double out[2]) {
  const double z1 = g->z[INIT_LAYERS[it][0]], z3 = g->z[INIT_LAYERS[it][2]];
  const double a = P->invp_a, b = P->invp_b;
  const double pm = it == 2 ? P->p_min3 : P->p_min;
  out[0] = (z3 - z1) / (2.0 * z1 * b) * (-a + sqrt(a * a + 4.0 * b / pm));
  const double k = z1 / (z3 - z1);
  out[1] = P->alpha0 / (k * (pm - P->alpha1));
}

/* Geometric factor of the third hit (Sec. 3.3.3), READING: the exact one of
 * eq. trackequation: the deviation of the T2 hit from the T1-T3 chord is
 * K3 * c_x with K3 = g(zb2) - g(zb1) - (z2 - z1)/(z3 - z1) (g(zb3) - g(zb1)). */
static double k3_factor(double z1, double z2, double z3, double zr, double d) {
  return gfun(z2 - zr, d) - gfun(z1 - zr, d) -
         (z2 - z1) / (z3 - z1) * (gfun(z3 - zr, d) - gfun(z1 - zr, d));
}

void orc_window_constants(const orc_geom *g, const orc_params *p, int it, double out[3]) {
  window_constants(g, p, it, out);
  out[2] = k3_factor(g->z[INIT_LAYERS[it][0]], g->z[INIT_LAYERS[it][1]],
                     g->z[INIT_LAYERS[it][2]], g->z_ref, p->d_ratio);
}

typedef struct { void *p; int n, cap; size_t sz; } dyn;
static void *dyn_push(dyn *v) {
  if (v->n == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 64;
    v->p = realloc(v->p, (size_t)v->cap * v->sz);
  }
  return (char *)v->p + (size_t)(v->n++) * v->sz;
}

/* One iteration of the XZ seeding of one half of one event (Sec. 3.2, 3.3).
 * Appends every three-hit combination, with the outcome of its extension and
 * fit, to `out`, in the order (T1 hit, T3 hit, T2 hit). */
static void xz_iteration(const orc_geom *g, const orc_params *P, const int32_t *off,
                         const float *X, const float *Z, int half, int it, dyn *out) {
  const int L1 = INIT_LAYERS[it][0], L2 = INIT_LAYERS[it][1], L3 = INIT_LAYERS[it][2];
  const double z2 = g->z[L2], z3 = g->z[L3], zr = g->z_ref, d = P->d_ratio;
  const double a = P->invp_a, b = P->invp_b;
  double wc[2];
  window_constants(g, P, it, wc);
  const double dx3max = wc[0], alpha_corr = wc[1];
  const int logm = !g_nolog;
  const int b1 = off[half * 12 + L1], e1 = off[half * 12 + L1 + 1];
  const int b2 = off[half * 12 + L2], e2 = off[half * 12 + L2 + 1];
  const int b3 = off[half * 12 + L3], e3 = off[half * 12 + L3 + 1];

  for (int i1 = b1; i1 < e1; ++i1) {
    const double x1 = X[i1], zh1 = Z[i1];
    /* Two-hit window around the straight line from the origin through the T1
     * hit, x3_inf = x1 z3 / z1, shifted by alpha_corr (Sec. 3.3.2). */
    const double centre = (z3 + alpha_corr) / zh1 * x1;
    const double lo3 = centre - dx3max, hi3 = centre + dx3max;
    for (int i3 = first_at_least(X, b3, e3, lo3); i3 < e3 && (double)X[i3] <= hi3; ++i3) {
      const double x3 = X[i3], zh3 = Z[i3];
      /* Back-propagated x0 and the momentum estimate of eq. invp. */
      const double t13 = (x3 - x1) / (zh3 - zh1);
      const double x0 = x1 - zh1 * t13;
      const double invp = a * fabs(x0) + b * x0 * x0;
      /* Third-hit window (Sec. 3.3.3): Delta x2 = K3 c_x with K3 the exact
       * geometric factor of eq. trackequation; c_x predicted from 1/p with
       * the sign s = sign(x0) removed (READING: band centre kappa_c/p). */
      const double s = x0 >= 0.0 ? 1.0 : -1.0;
      const double c_pred = -s * P->kappa_c * invp;
      const double K3 = k3_factor(zh1, z2, zh3, zr, d);
      const double pred2 = x1 + (z2 - zh1) * t13 + K3 * c_pred;
      const double tol2 = P->t2_tol0 + P->t2_tol1 * fabs(K3 * c_pred);
      for (int i2 = first_at_least(X, b2, e2, pred2 - tol2); i2 < e2 && (double)X[i2] <= pred2 + tol2; ++i2) {
        orc_cand *cd = (orc_cand *)dyn_push(out);
        memset(cd, 0, sizeof(*cd));
        cd->half = half;
        cd->it = it;
        /* the two windows that admitted this combination */
        cd->margin = fmin(cut_margin(fabs(x3 - centre), dx3max),
                          cut_margin(fabs((double)X[i2] - pred2), tol2));
        for (int l = 0; l < ORC_NL; ++l) cd->pos[l] = -1;
        cd->pos[L1] = i1; cd->pos[L2] = i2; cd->pos[L3] = i3;
        /* Track model through the three hits (exact 3-point solve). */
        const double x2 = X[i2], zh2 = Z[i2];
        double zz[6], xx[6];
        zz[0] = zh1; zz[1] = zh2; zz[2] = zh3;
        xx[0] = x1; xx[1] = x2; xx[2] = x3;
        double pa, pb, pc;
        if (fit_xz(zz, xx, 3, zr, d, &pa, &pb, &pc)) { cd->status = 1; continue; }
        /* Extension to the three remaining x-layers: closest hit within
         * ext_tol of the model at the layer (Sec. 3.2). */
        int n = 3;
        for (int j = 0; j < 3; ++j) {
          const int L = EXT_LAYERS[it][j];
          const int lo = off[half * 12 + L], hi = off[half * 12 + L + 1];
          const double pe = xmodel(pa, pb, pc, g->z[L], zr, d);
          const int h = closest_in_window(X, lo, hi, pe, P->ext_tol);
          if (logm) cd->margin = fmin(cd->margin, closest_margin(X, lo, hi, pe, P->ext_tol, h));
          if (h >= 0) { cd->pos[L] = h; ++n; }
        }
        cd->n = n;
        if (n < P->min_x_hits) { cd->status = 1; continue; }
        /* Least-squares fit over all x hits in layer order. */
        int m = 0;
        for (int j = 0; j < 6; ++j) {
          const int h = cd->pos[X_LAYERS[j]];
          if (h >= 0) { zz[m] = Z[h]; xx[m] = X[h]; ++m; }
        }
        if (fit_xz(zz, xx, m, zr, d, &pa, &pb, &pc)) { cd->status = 2; continue; }
        double chi2 = 0.0;
        for (int j = 0; j < m; ++j) {
          const double r = (xx[j] - xmodel(pa, pb, pc, zz[j], zr, d)) / P->sigma_x;
          chi2 += r * r;
        }
        chi2 /= (double)(m - 3);
        cd->a = pa; cd->b = pb; cd->c = pc; cd->chi2 = chi2;
        /* eq. seed_clone_score, READING: |c_x| so that the score is >= 0. */
        cd->score = (m == 6 ? 1.0 : 10.0) * (1000.0 * chi2 + fabs(pc));
        cd->status = chi2 < P->chi2x_max ? 0 : 2;
        cd->margin = fmin(cd->margin, cut_margin(chi2, P->chi2x_max));
      }
    }
  }
}

int orc_xz_candidates(const orc_geom *g, const orc_params *p, const int32_t *zone_off,
                      const float *x, const float *z, int half, int it,
                      orc_cand *out, int cap) {
  dyn v = {NULL, 0, 0, sizeof(orc_cand)};
  xz_iteration(g, p, zone_off, x, z, half, it, &v);
  int n = v.n;
  if (out) memcpy(out, v.p, sizeof(orc_cand) * (size_t)(n < cap ? n : cap));
  free(v.p);
  return n;
}

/* ---------------------------------------------------- clone killing ----- */

/* O(n) clone killing of Sec. 3.3.4 over the candidates of one half (both
 * iterations).  Pass 1: every hit keeps the lowest score of the tracks that use
 * it.  Pass 2: a track keeps the hits that still carry its own score, and
 * survives with >= 3 of them, or >= 2 if it has 6 hits.  Then the repeated
 * tracks of the two iterations (identical x-hit sets, Sec. 3) are removed,
 * keeping the first iteration's copy.  n_pos bounds the hit positions used. */
/* Vote margin of every candidate: over its hits, the relative gap between
 * its score and the lowest score of the other candidates on that hit whose
 * x-hit set differs (identical sets carry identical scores by construction),
 * and the x-z margin of every such candidate with a score no higher than its
 * own (whether that rival takes part in the vote can change who owns the
 * hit).  The first n_vote candidates are the voters; the rest are near
 * misses of the fit, rivals only. */
static void vote_margins(const orc_cand *c, int n, int n_vote, int n_pos, const double *xzm,
                         double *vm) {
  if (g_nolog) {
    for (int i = 0; i < n_vote; ++i) vm[i] = INFINITY;
    return;
  }
  int *cnt = (int *)calloc((size_t)(n_pos + 1), sizeof(int));
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < ORC_NL; ++l)
      if (c[i].pos[l] >= 0) ++cnt[c[i].pos[l] + 1];
  for (int h = 0; h < n_pos; ++h) cnt[h + 1] += cnt[h];
  int *fill = (int *)malloc(sizeof(int) * (size_t)(n_pos > 0 ? n_pos : 1));
  int *lst = (int *)malloc(sizeof(int) * (size_t)(cnt[n_pos] > 0 ? cnt[n_pos] : 1));
  for (int h = 0; h < n_pos; ++h) fill[h] = cnt[h];
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < ORC_NL; ++l)
      if (c[i].pos[l] >= 0) lst[fill[c[i].pos[l]]++] = i;
  for (int i = 0; i < n_vote; ++i) {
    double m = INFINITY;
    const double scale = c[i].score > 0.0 ? c[i].score : 1e-300;
    for (int l = 0; l < ORC_NL; ++l) {
      const int h = c[i].pos[l];
      if (h < 0) continue;
      double lo = INFINITY;
      for (int k = cnt[h]; k < cnt[h + 1]; ++k) {
        const int j = lst[k];
        if (j == i || memcmp(c[i].pos, c[j].pos, sizeof(c[i].pos)) == 0) continue;
        if (j < n_vote && c[j].score < lo) lo = c[j].score;
        if (c[j].score <= c[i].score) m = fmin(m, xzm[j]);
      }
      if (lo < INFINITY) m = fmin(m, fabs(c[i].score - lo) / scale);
    }
    vm[i] = m;
  }
  free(cnt); free(fill); free(lst);
}

void orc_clone_vote(const orc_cand *c, int n, int n_pos, int32_t *keep) {
  double *T = (double *)malloc(sizeof(double) * (size_t)(n_pos > 0 ? n_pos : 1));
  for (int i = 0; i < n_pos; ++i) T[i] = INFINITY;
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < ORC_NL; ++l) {
      const int h = c[i].pos[l];
      if (h >= 0 && c[i].score < T[h]) T[h] = c[i].score;
    }
  for (int i = 0; i < n; ++i) {
    int own = 0;
    for (int l = 0; l < ORC_NL; ++l) {
      const int h = c[i].pos[l];
      if (h >= 0 && T[h] == c[i].score) ++own;
    }
    keep[i] = own >= 3 || (own >= 2 && c[i].n == 6);
  }
  for (int i = 0; i < n; ++i) {
    if (!keep[i] || c[i].it == 0) continue;
    for (int j = 0; j < n; ++j) {
      if (!keep[j] || c[j].it != 0) continue;
      if (memcmp(c[i].pos, c[j].pos, sizeof(c[i].pos)) == 0) { keep[i] = 0; break; }
    }
  }
  free(T);
}

/* -------------------------------------------------------- UV seeding ---- */

/* Iterative UV seeding of Sec. 3.4 for one x-z track.  Two passes, from the
 * u-layer then the v-layer of T1 (READING), each trying every hit of the
 * initial layer whose y lies in the half; t_y from the origin, then the
 * closest hit within uv_tol in each of the five other stereo layers in
 * ascending z, averaging t_y after each found hit.  Each combination gets a
 * weighted y-z line fit; the best has most hits, then lowest chi2_y, then the
 * earlier (pass, initial hit).  Returns 1 and fills `out` if a seed is made. */
/* One UV combination as the margin log sees it. */
typedef struct { int n, pos[ORC_NL]; double chi2, m; int valid; } uv_try;

/* Near miss of kind k for the x-z track `cd` with stereo hits spos (NULL: x
 * hits only). */
static void push_near(dyn *near, int event, int kind, int velo, const orc_cand *cd,
                      const int *spos, const int32_t *ID, double m) {
  if (g_nolog) return;
  orc_near *r = (orc_near *)dyn_push(near);
  memset(r, 0, sizeof(*r));
  r->event = event; r->kind = kind; r->velo_idx = velo; r->it = cd->it; r->margin = m;
  for (int l = 0; l < ORC_NL; ++l) {
    const int h = spos && spos[l] >= 0 ? spos[l] : cd->pos[l];
    r->id[l] = h >= 0 ? ID[h] : -1;
  }
}

static int uv_iterative(const orc_geom *g, const orc_params *P, const int32_t *off,
                        const float *X, const float *Z, const int32_t *ID, const orc_cand *cd,
                        orc_seed *out, dyn *near, int event) {
  const int half = cd->half;
  const double zr = g->z_ref, d = P->d_ratio;
  const double ylo = half == 0 ? 0.0 : -P->y_max, yhi = half == 0 ? P->y_max : 0.0;
  int best_n = 0, best_k = -1;
  double best_chi2 = 0.0, best_y0 = 0.0, best_ty = 0.0;
  int best_pos[ORC_NL];
  dyn tries = {NULL, 0, 0, sizeof(uv_try)};
  const int logm = !g_nolog;
  for (int pass = 0; pass < 2; ++pass) {
    const int L0 = pass == 0 ? 1 : 2;
    const double t0 = g->tan_a[L0];
    const double xp = xmodel(cd->a, cd->b, cd->c, g->z[L0], zr, d);
    const double e1 = xp - yhi * t0, e2 = xp - ylo * t0;
    const double lo = e1 < e2 ? e1 : e2, hi = e1 < e2 ? e2 : e1;
    const int b0 = off[half * 12 + L0], en0 = off[half * 12 + L0 + 1];
    for (int h0 = first_at_least(X, b0, en0, lo); h0 < en0 && (double)X[h0] <= hi; ++h0) {
      double zs[6], ys[6], ws[6];
      int pos[ORC_NL];
      for (int l = 0; l < ORC_NL; ++l) pos[l] = -1;
      int n = 0;
      const double zh0 = Z[h0];
      const double y0h = (xmodel(cd->a, cd->b, cd->c, zh0, zr, d) - X[h0]) / t0;
      double ty = y0h / zh0;
      pos[L0] = h0;
      /* margin: the initial hit's y inside the half's range at the layer */
      const double yw = (xp - X[h0]) / t0;
      double mc = fmin(fabs(yw - ylo), fabs(yhi - yw)) / P->y_max;
      zs[n] = zh0; ys[n] = y0h; ws[n] = t0 * t0 / (P->sigma_x * P->sigma_x); ++n;
      for (int j = 0; j < 6; ++j) {
        const int L = UV_LAYERS[j];
        if (L == L0) continue;
        const double zl = g->z[L], tl = g->tan_a[L];
        const double pred = xmodel(cd->a, cd->b, cd->c, zl, zr, d) - ty * zl * tl;
        const int zlo = off[half * 12 + L], zhi = off[half * 12 + L + 1];
        const int h = closest_in_window(X, zlo, zhi, pred, P->uv_tol);
        if (logm) mc = fmin(mc, closest_margin(X, zlo, zhi, pred, P->uv_tol, h));
        if (h < 0) continue;
        const double zh = Z[h];
        const double yl = (xmodel(cd->a, cd->b, cd->c, zh, zr, d) - X[h]) / tl;
        ty = 0.5 * (ty + yl / zh);
        pos[L] = h;
        zs[n] = zh; ys[n] = yl; ws[n] = tl * tl / (P->sigma_x * P->sigma_x); ++n;
      }
      uv_try scratch_try, *tr = logm ? (uv_try *)dyn_push(&tries) : &scratch_try;
      tr->n = n; tr->valid = 0; tr->chi2 = INFINITY; tr->m = mc;
      memcpy(tr->pos, pos, sizeof(pos));
      if (n < P->min_uv_hits) continue;
      double fy0, fty;
      fit_line(zs, ys, ws, n, zr, &fy0, &fty);
      double chi2 = 0.0;
      for (int i = 0; i < n; ++i) {
        const double r = ys[i] - (fy0 + fty * (zs[i] - zr));
        chi2 += ws[i] * r * r;
      }
      chi2 /= (double)(n - 2);
      tr->chi2 = chi2;
      tr->m = fmin(mc, cut_margin(chi2, P->chi2y_max));
      if (!(chi2 < P->chi2y_max)) continue;
      tr->valid = 1;
      if (n > best_n || (n == best_n && chi2 < best_chi2)) {
        best_n = n; best_chi2 = chi2; best_y0 = fy0; best_ty = fty;
        memcpy(best_pos, pos, sizeof(pos));
        best_k = tries.n - 1;
      }
    }
  }
  double seed_m = cd->margin;
  if (logm) {
    /* the chosen combination's own decisions, its lead over the runners-up
     * with as many hits, and every other combination that came near */
    const uv_try *T = (const uv_try *)tries.p;
    const double scale = fmax(best_chi2, 1e-3 * P->chi2y_max);
    if (best_k >= 0) seed_m = fmin(seed_m, T[best_k].m);
    for (int k = 0; k < tries.n; ++k) {
      /* the chosen hit set reached again from another initial hit is the
       * same seed, not a rival */
      if (k == best_k || (best_k >= 0 && memcmp(T[k].pos, T[best_k].pos, sizeof(T[k].pos)) == 0))
        continue;
      /* any other combination may win once one of its own decisions goes
       * the other way (a changed hit moves the t_y average and with it the
       * later layers' hits), or once its chi2 passes the chosen one's */
      double m = T[k].m;
      if (best_k >= 0 && T[k].valid && T[k].n == best_n)
        m = fmin(m, fabs(T[k].chi2 - best_chi2) / scale);
      seed_m = fmin(seed_m, m);
      if (near && m < ORC_NEAR) push_near(near, event, 3, -1, cd, T[k].pos, ID, fmin(m, cd->margin));
    }
    free(tries.p);
  }
  if (best_n == 0) return 0;
  memset(out, 0, sizeof(*out));
  out->a = cd->a; out->b = cd->b; out->c = cd->c;
  out->y0 = best_y0; out->ty = best_ty;
  out->chi2x = cd->chi2; out->chi2y = best_chi2; out->score = cd->score;
  out->nx = cd->n; out->nuv = best_n; out->half = cd->half; out->it = cd->it;
  for (int l = 0; l < ORC_NL; ++l) {
    const int h = (g->tan_a[l] == 0.0) ? cd->pos[l] : best_pos[l];
    out->pos[l] = h;
    out->id[l] = h >= 0 ? ID[h] : -1;
  }
  out->margin = seed_m;
  return 1;
}


/* One stereo-hit combination for a given t_y hypothesis, as the Hough
 * variant builds it: the closest hit within uv_tol in each stereo layer,
 * then the weighted y-z line fit.  Returns the hit count (0 if rejected). */
static int uv_attach(const orc_geom *g, const orc_params *P, const int32_t *off, const float *X,
                     const float *Z, const orc_cand *cd, double ty, int pos[ORC_NL],
                     double *chi2_out, double *y0_out, double *ty_out) {
  const double zr = g->z_ref, d = P->d_ratio;
  double zs[6], ys[6], ws[6];
  int n = 0;
  for (int l = 0; l < ORC_NL; ++l) pos[l] = -1;
  for (int j = 0; j < 6; ++j) {
    const int L = UV_LAYERS[j];
    const double zl = g->z[L], tl = g->tan_a[L];
    const double pred = xmodel(cd->a, cd->b, cd->c, zl, zr, d) - ty * zl * tl;
    const int h = closest_in_window(X, off[cd->half * 12 + L], off[cd->half * 12 + L + 1], pred, P->uv_tol);
    if (h < 0) continue;
    pos[L] = h;
    zs[n] = Z[h];
    ys[n] = (xmodel(cd->a, cd->b, cd->c, Z[h], zr, d) - X[h]) / tl;
    ws[n] = tl * tl / (P->sigma_x * P->sigma_x);
    ++n;
  }
  if (n < P->min_uv_hits) return 0;
  double fy0, fty;
  fit_line(zs, ys, ws, n, zr, &fy0, &fty);
  double chi2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = ys[i] - (fy0 + fty * (zs[i] - zr));
    chi2 += ws[i] * r * r;
  }
  chi2 /= (double)(n - 2);
  if (!(chi2 < P->chi2y_max)) return 0;
  *chi2_out = chi2; *y0_out = fy0; *ty_out = fty;
  return n;
}

/* Hough-cluster UV seeding (Sec. 3.4, second variant).  Every stereo hit
 * whose y lies in the half gives t_y = y / z; the t_y values fill a coarse
 * histogram over the half's range; the most populated bins (up to
 * hough_best, ties to the lower bin) are each split into hough_fine finer
 * bins, and the mean t_y of each non-empty fine bin is a hypothesis for which
 * the closest hit within uv_tol is attached in every stereo layer.  The best
 * combination is chosen as in the iterative variant: most hits, then lowest
 * chi2_y, then the earlier hypothesis. */
static int uv_hough(const orc_geom *g, const orc_params *P, const int32_t *off, const float *X,
                    const float *Z, const int32_t *ID, const orc_cand *cd, orc_seed *out) {
  const int half = cd->half, NB = P->hough_bins, NF = P->hough_fine;
  const double zr = g->z_ref, d = P->d_ratio;
  double zmin = 1e300;
  for (int j = 0; j < 6; ++j) zmin = g->z[UV_LAYERS[j]] < zmin ? g->z[UV_LAYERS[j]] : zmin;
  const double lo = half == 0 ? 0.0 : -P->y_max / zmin;
  const double hi = half == 0 ? P->y_max / zmin : 0.0;
  const double w = (hi - lo) / NB;
  const double ylo = half == 0 ? 0.0 : -P->y_max, yhi = half == 0 ? P->y_max : 0.0;
  /* entries: t_y of every stereo hit with y inside the half */
  int cap = 64, n = 0;
  double *tys = (double *)malloc(sizeof(double) * (size_t)cap);
  for (int j = 0; j < 6; ++j) {
    const int L = UV_LAYERS[j];
    for (int h = off[half * 12 + L]; h < off[half * 12 + L + 1]; ++h) {
      const double y = (xmodel(cd->a, cd->b, cd->c, Z[h], zr, d) - X[h]) / g->tan_a[L];
      if (!(y >= ylo && y <= yhi)) continue;
      if (n == cap) { cap *= 2; tys = (double *)realloc(tys, sizeof(double) * (size_t)cap); }
      tys[n++] = y / Z[h];
    }
  }
  int *cnt = (int *)calloc((size_t)NB, sizeof(int));
  for (int i = 0; i < n; ++i) {
    int b = (int)floor((tys[i] - lo) / w);
    b = b < 0 ? 0 : (b >= NB ? NB - 1 : b);
    cnt[b]++;
  }
  int best_n = 0, bpos[ORC_NL];
  double best_chi2 = 0.0, best_y0 = 0.0, best_ty = 0.0;
  int *used = (int *)calloc((size_t)NB, sizeof(int));
  for (int r = 0; r < P->hough_best; ++r) {
    int bb = -1;
    for (int b = 0; b < NB; ++b)
      if (!used[b] && cnt[b] >= P->hough_min && (bb < 0 || cnt[b] > cnt[bb])) bb = b;
    if (bb < 0) break;
    used[bb] = 1;
    const double blo = lo + bb * w, fw = w / NF;
    for (int f = 0; f < NF; ++f) {
      double sum = 0.0;
      int m = 0;
      for (int i = 0; i < n; ++i) {
        int b = (int)floor((tys[i] - lo) / w);
        b = b < 0 ? 0 : (b >= NB ? NB - 1 : b);
        if (b != bb) continue;
        int fi = (int)floor((tys[i] - blo) / fw);
        fi = fi < 0 ? 0 : (fi >= NF ? NF - 1 : fi);
        if (fi != f) continue;
        sum += tys[i];
        ++m;
      }
      if (m == 0) continue;
      int pos[ORC_NL];
      double chi2 = 0.0, y0 = 0.0, ty = 0.0;
      const int k = uv_attach(g, P, off, X, Z, cd, sum / m, pos, &chi2, &y0, &ty);
      if (k > best_n || (k > 0 && k == best_n && chi2 < best_chi2)) {
        best_n = k; best_chi2 = chi2; best_y0 = y0; best_ty = ty;
        memcpy(bpos, pos, sizeof(pos));
      }
    }
  }
  free(tys); free(cnt); free(used);
  if (best_n == 0) return 0;
  memset(out, 0, sizeof(*out));
  out->a = cd->a; out->b = cd->b; out->c = cd->c;
  out->y0 = best_y0; out->ty = best_ty;
  out->chi2x = cd->chi2; out->chi2y = best_chi2; out->score = cd->score;
  out->nx = cd->n; out->nuv = best_n; out->half = cd->half; out->it = cd->it;
  for (int l = 0; l < ORC_NL; ++l) {
    const int h = (g->tan_a[l] == 0.0) ? cd->pos[l] : bpos[l];
    out->pos[l] = h;
    out->id[l] = h >= 0 ? ID[h] : -1;
  }
  out->margin = cd->margin;   /* the Hough bin decisions are not logged */
  return 1;
}

int orc_uv(const orc_geom *g, const orc_params *P, const int32_t *off, const float *X,
           const float *Z, const int32_t *ID, const orc_cand *cd, orc_seed *out) {
  return P->uv_mode == 1 ? uv_hough(g, P, off, X, Z, ID, cd, out)
                         : uv_iterative(g, P, off, X, Z, ID, cd, out, NULL, 0);
}

/* ---------------------------------------------------------- Matching ---- */

typedef struct {
  double chi2, zm, dx, dy, dtx, dty, qop;
  int ok;
  double m;   /* accepted: smallest margin of its cuts; rejected: margin to acceptance */
  int n_ut;
  int32_t ut_id[ORC_NUT];
} pair_eval;

/* One event's UT hits: layer offsets [5] into x and id (NULL off: none). */
typedef struct {
  const int32_t *off;
  const float *x;
  const int32_t *id;
} ut_event;

/* UT hit search of one pair (Sec. 4.3).  gamma_x starts from eq.
 * gamma_parametrisation with the pair's q/p.  Layer by layer, the VELO state
 * is extrapolated with eq. velo_ut_extrapolation (z_ref: the state's z) and
 * compared in the layer's measured coordinate x - y tan(alpha).  Until a hit
 * is found, the loose window of the layer is searched (layers without one are
 * passed over); the closest hit inside is attached, and gamma_x is refitted
 * so that the trajectory goes through it (READING: the text does not say how
 * several hits in the window refine gamma_x; the closest one is used).  In
 * every later layer the closest hit inside the tight window is attached.
 * Windows are inclusive, ties as for SciFi hits.  Returns the number of hits
 * attached; *margin: the smallest closest-hit margin of the layers searched. */
double orc_ut_window(const orc_params *P, int layer, int tight, double qop) {
  const double a = tight ? P->ut_tight_a[layer] : P->ut_loose_a[layer];
  const double b = tight ? P->ut_tight_b[layer] : P->ut_loose_b[layer];
  const double lo = tight ? P->ut_tight_lo[layer] : P->ut_loose_lo[layer];
  const double hi = tight ? P->ut_tight_hi[layer] : P->ut_loose_hi[layer];
  if (!(hi > 0.0)) return 0.0;
  return fmin(fmax(a + b * 1000.0 * fabs(qop), lo), hi);   /* B / p, p in GeV/c */
}

static int ut_search(const orc_geom *g, const orc_params *P, const ut_event *ut, double xv,
                     double yv, double zv, double txv, double tyv, double qop,
                     int32_t ids[ORC_NUT], double *margin) {
  double gam = P->a_gamma + P->b_gamma * qop;
  int loose = 1, n = 0;
  double m = INFINITY;
  for (int i = 0; i < ORC_NUT; ++i) ids[i] = -1;
  if (!ut->off) { *margin = m; return 0; }
  for (int i = 0; i < ORC_NUT; ++i) {
    const double w = orc_ut_window(P, i, !loose, qop);
    if (!(w > 0.0)) continue;
    const double dz = g->ut_z[i] - zv;
    const double yp = yv + tyv * dz;
    const double mp = xv + txv * dz + gam * dz * dz - yp * g->ut_tan[i];
    const int h = closest_in_window(ut->x, ut->off[i], ut->off[i + 1], mp, w);
    if (!g_nolog) m = fmin(m, closest_margin(ut->x, ut->off[i], ut->off[i + 1], mp, w, h));
    if (h < 0) continue;
    ids[i] = ut->id[h];
    ++n;
    if (loose) {
      const double xh = (double)ut->x[h] + yp * g->ut_tan[i];
      gam = (xh - xv - txv * dz) / (dz * dz);
      loose = 0;
    }
  }
  *margin = m;
  return n;
}

/* A pair that passed the chi2_match cut also needs its UT hits (ut_mode 1):
 * with fewer than ut_min_hits it leaves the candidates. */
static void apply_ut(const orc_geom *g, const orc_params *P, const ut_event *ut, double xv,
                     double yv, double zv, double txv, double tyv, pair_eval *r) {
  r->n_ut = 0;
  for (int i = 0; i < ORC_NUT; ++i) r->ut_id[i] = -1;
  if (!r->ok || P->ut_mode != 1) return;
  double m;
  r->n_ut = ut_search(g, P, ut, xv, yv, zv, txv, tyv, r->qop, r->ut_id, &m);
  if (r->n_ut < P->ut_min_hits) {
    r->ok = 0;
    r->m = m;
  } else {
    r->m = fmin(r->m, m);
  }
}

/* One VELO-seed combination (Sec. 4.1, 4.2). */
static pair_eval eval_pair(const orc_params *P, const orc_geom *g, const orc_seed *s,
                           double xv, double yv, double zv, double txv, double tyv, int logm) {
  pair_eval r;
  memset(&r, 0, sizeof(r));
  const double zr = g->z_ref, d = P->d_ratio, zs = P->z_state;
  /* SciFi state at z_s: position and slope of eq. trackequation. */
  const double us = zs - zr;
  const double xs = xmodel(s->a, s->b, s->c, zs, zr, d);
  const double txs = s->b + s->c * (2.0 * us + 3.0 * d * us * us);
  const double dtx = txs - txv;
  /* eq. z_match: z of the kink. */
  const double zm = P->zm[0] + P->zm[1] * fabs(dtx) + P->zm[2] * dtx * dtx +
                    P->zm[3] * fabs(xs) + P->zm[4] * txv * txv;
  const double dx = (xs + (zm - zs) * txs) - (xv + (zm - zv) * txv);
  /* y: straight lines compared at z_y_match. */
  const double dy = (s->y0 + s->ty * (P->z_ymatch - zr)) - (yv + tyv * (P->z_ymatch - zv));
  const double dty = s->ty - tyv;
  r.zm = zm; r.dx = dx; r.dy = dy; r.dtx = dtx; r.dty = dty;
  /* preselection margins: accepted, the tightest cut; rejected, the cut
   * furthest from letting it through */
  const double dev[4] = {fabs(dx), fabs(dy), fabs(dtx), fabs(dty)};
  const double cut[4] = {P->max_dx, P->max_dy, P->max_dtx, P->max_dty};
  double m_in = INFINITY, m_out = 0.0;
  int pass = 1;
  for (int k = 0; k < 4; ++k) {
    if (dev[k] < cut[k]) {
      if (logm) m_in = fmin(m_in, cut_margin(dev[k], cut[k]));
    } else {
      pass = 0;
      if (logm) m_out = fmax(m_out, cut_margin(dev[k], cut[k]));
    }
  }
  r.m = pass ? m_in : m_out;
  if (!pass) return r;
  const double tolx = P->tolx_scale * (P->tolx_a * P->tolx_a + P->tolx_b * P->tolx_b * dtx * dtx);
  const double rho = txv * txv + tyv * tyv;
  const double toly = P->toly_scale * (P->toly_a * P->toly_a + P->toly_b * P->toly_b * rho);
  const double chi2 = dx * dx / tolx + dy * dy / toly + dtx * dtx / P->tol_tx + dty * dty / P->tol_ty;
  r.chi2 = chi2;
  if (!(chi2 < P->chi2m_max)) { r.m = cut_margin(chi2, P->chi2m_max); return r; }
  r.m = fmin(r.m, cut_margin(chi2, P->chi2m_max));
  /* Momentum from the kick (READING): eq. invp evaluated on the distance at
   * z = 0 between the SciFi and VELO straight lines. */
  const double x0 = (xs - zs * txs) - (xv - zv * txv);
  const double invp = P->invp_a * fabs(x0) + P->invp_b * x0 * x0;
  const double q = -(x0 >= 0.0 ? 1.0 : -1.0) * P->polarity;
  r.qop = q * invp;
  r.ok = 1;
  return r;
}

/* The network's eight inputs for one surviving pair (Sec. 4.4).  eta of the
 * VELO state from its slopes: eta = -ln tan(theta / 2) = asinh(1 / tan theta),
 * tan theta = sqrt(tx^2 + ty^2) (floored at 1e-9); the SciFi hit count is the
 * seed's hits on x and stereo layers. */
static void nn_inputs(const pair_eval *r, const orc_seed *s, double txv, double tyv,
                      double f[ORC_NN_IN]) {
  f[0] = r->zm;
  f[1] = r->dx;
  f[2] = r->dy;
  f[3] = r->dtx;
  f[4] = r->dty;
  f[5] = r->chi2;
  f[6] = asinh(1.0 / fmax(sqrt(txv * txv + tyv * tyv), 1e-9));
  f[7] = (double)(s->nx + s->nuv);
}

/* Ghost probability (Sec. 4.4): standardised inputs, one hidden layer of
 * rectified units, logistic output. */
double orc_ghost_prob(const orc_params *P, const double f[ORC_NN_IN]) {
  const orc_ghost_nn *n = &P->ghost_nn;
  double x[ORC_NN_IN];
  for (int i = 0; i < ORC_NN_IN; ++i) x[i] = (f[i] - n->mean[i]) / n->scale[i];
  double out = n->b2;
  for (int j = 0; j < ORC_NN_HID; ++j) {
    double h = n->b1[j];
    for (int i = 0; i < ORC_NN_IN; ++i) h += n->w1[j][i] * x[i];
    out += n->w2[j] * (h > 0.0 ? h : 0.0);
  }
  return 1.0 / (1.0 + exp(-out));
}

int orc_match_pairs(const orc_geom *g, const orc_params *P, const orc_seed *seeds, int ns,
                    int nv, const float *vx, const float *vy, const float *vz,
                    const float *vtx, const float *vty, const int32_t *ut_off,
                    const float *ut_x, const int32_t *ut_id, orc_pair *out, int cap) {
  const ut_event ut = {ut_off, ut_x, ut_id};
  int n = 0;
  for (int v = 0; v < nv; ++v)
    for (int s = 0; s < ns; ++s) {
      pair_eval r = eval_pair(P, g, &seeds[s], vx[v], vy[v], vz[v], vtx[v], vty[v], 0);
      apply_ut(g, P, &ut, vx[v], vy[v], vz[v], vtx[v], vty[v], &r);
      if (!r.ok) continue;
      if (n < cap) {
        orc_pair *q = &out[n];
        q->velo_idx = v;
        q->seed_idx = s;
        nn_inputs(&r, &seeds[s], vtx[v], vty[v], q->f);
        q->gp = P->final_sel == 1 ? orc_ghost_prob(P, q->f) : -1.0;
      }
      ++n;
    }
  return n;
}

/* Margin of one rival's part in the network form of the final selection: a
 * rival t2 (another survivor on the same VELO state or seed) makes t a clone
 * when t2 is retained (gp2 < cut) and gp - gp2 >= gap.  The distance of that
 * verdict from flipping, in units of probability (the scale of both the cut
 * and the gap, which is itself a difference of probabilities): with both
 * conditions true either flip ends it, with both false both must flip, else
 * the failing one must. */
static double rival_flip(double gp, double gp2, double cut, double gap) {
  const double mc = fabs(gp2 - cut), mg = fabs((gp - gp2) - gap);
  const int ret = gp2 < cut, far = (gp - gp2) >= gap;
  if (ret && far) return fmin(mc, mg);
  if (!ret && !far) return fmax(mc, mg);
  return ret ? mg : mc;
}

/* All VELO x seed combinations of one event.  final_sel 0: a combination is
 * kept when its chi2_match is the smallest both among the survivors sharing
 * its seed and among those sharing its VELO track (READING of the final clone
 * removal of Sec. 4.4, with chi2_match in place of the ghost probability).
 * final_sel 1: the ghost network and the clone rule of Sec. 4.4. */
static int match_event(const orc_geom *g, const orc_params *P, const orc_seed *seeds, int ns,
                       int nv, const float *vx, const float *vy, const float *vz,
                       const float *vtx, const float *vty, const int32_t *vid,
                       const ut_event *ut, orc_long *out, int cap, dyn *near, int event);

int orc_match(const orc_geom *g, const orc_params *P, const orc_seed *seeds, int ns, int nv,
              const float *vx, const float *vy, const float *vz, const float *vtx,
              const float *vty, const int32_t *vid, const int32_t *ut_off, const float *ut_x,
              const int32_t *ut_id, orc_long *out, int cap) {
  const ut_event ut = {ut_off, ut_x, ut_id};
  return match_event(g, P, seeds, ns, nv, vx, vy, vz, vtx, vty, vid, &ut, out, cap, NULL, 0);
}

/* The network form of the final selection (Sec. 4.4): every surviving pair's
 * ghost probability; pairs below ghost_cut are retained; a retained pair is
 * dropped as a clone when a retained pair on its VELO state or on its seed has
 * a ghost probability lower by clone_gap or more. */
static int match_event_nn(const orc_geom *g, const orc_params *P, const orc_seed *seeds,
                          int ns, int nv, const float *vx, const float *vy, const float *vz,
                          const float *vtx, const float *vty, const int32_t *vid,
                          const ut_event *ut, orc_long *out, int cap, dyn *near, int event) {
  const int logm = !g_nolog;
  const double cut = P->ghost_cut, gap = P->clone_gap;
  const size_t np = (size_t)ns * (size_t)nv;
  pair_eval *pe = (pair_eval *)malloc(sizeof(pair_eval) * np);
  double *gp = (double *)malloc(sizeof(double) * np);
  double *min_v = (double *)malloc(sizeof(double) * (size_t)nv);
  double *min_s = (double *)malloc(sizeof(double) * (size_t)ns);
  for (int v = 0; v < nv; ++v) min_v[v] = INFINITY;
  for (int s = 0; s < ns; ++s) min_s[s] = INFINITY;
  for (int v = 0; v < nv; ++v)
    for (int s = 0; s < ns; ++s) {
      const size_t k = (size_t)v * ns + s;
      pe[k] = eval_pair(P, g, &seeds[s], vx[v], vy[v], vz[v], vtx[v], vty[v], logm);
      apply_ut(g, P, ut, vx[v], vy[v], vz[v], vtx[v], vty[v], &pe[k]);
      gp[k] = INFINITY;
      if (!pe[k].ok) continue;
      double f[ORC_NN_IN];
      nn_inputs(&pe[k], &seeds[s], vtx[v], vty[v], f);
      gp[k] = orc_ghost_prob(P, f);
      if (gp[k] < cut) {
        if (gp[k] < min_v[v]) min_v[v] = gp[k];
        if (gp[k] < min_s[s]) min_s[s] = gp[k];
      }
    }
  int n = 0;
  for (int v = 0; v < nv; ++v)
    for (int s = 0; s < ns; ++s) {
      const size_t k = (size_t)v * ns + s;
      const pair_eval *r = &pe[k];
      const double q = gp[k];
      const int kept = r->ok && q < cut && q - min_v[v] < gap && q - min_s[s] < gap;
      /* margin: the cut itself, then every rival on the same VELO state or
       * seed (kept: the closest flip; a clone: the clone-making rivals must
       * all flip) */
      double m = r->m;
      if (r->ok && logm) {
        const double mcut = fabs(q - cut);
        if (q >= cut) {
          m = mcut;
        } else {
          double lo = INFINITY, hi = 0.0;
          for (int pass = 0; pass < 2; ++pass) {
            const int n2 = pass ? nv : ns;
            for (int o = 0; o < n2; ++o) {
              const size_t k2 = pass ? (size_t)o * ns + s : (size_t)v * ns + o;
              if (k2 == k || !pe[k2].ok) continue;
              const double f2 = rival_flip(q, gp[k2], cut, gap);
              lo = fmin(lo, f2);
              if (gp[k2] < cut && q - gp[k2] >= gap) hi = fmax(hi, f2);
            }
          }
          m = kept ? fmin(mcut, lo) : hi;
        }
      }
      if (!kept) {
        if (near && logm && m < ORC_NEAR) {
          orc_near *nq = (orc_near *)dyn_push(near);
          memset(nq, 0, sizeof(*nq));
          nq->event = event; nq->kind = 4; nq->velo_idx = v; nq->it = seeds[s].it;
          nq->margin = m;
          memcpy(nq->id, seeds[s].id, sizeof(nq->id));
        }
        continue;
      }
      if (n < cap) {
        orc_long *L = &out[n];
        L->velo_idx = v; L->velo_id = vid[v]; L->seed_idx = s; L->n_ut = r->n_ut;
        memcpy(L->ut_id, r->ut_id, sizeof(L->ut_id));
        L->qop = r->qop; L->chi2 = r->chi2; L->zm = r->zm;
        L->dx = r->dx; L->dy = r->dy; L->dtx = r->dtx; L->dty = r->dty;
        L->gp = q;
        L->margin = fmin(fmin(seeds[s].margin, r->m), m);
      }
      ++n;
    }
  free(pe); free(gp); free(min_v); free(min_s);
  return n;
}

static int match_event(const orc_geom *g, const orc_params *P, const orc_seed *seeds, int ns,
                       int nv, const float *vx, const float *vy, const float *vz,
                       const float *vtx, const float *vty, const int32_t *vid,
                       const ut_event *ut, orc_long *out, int cap, dyn *near, int event) {
  if (ns == 0 || nv == 0) return 0;
  if (P->final_sel == 1)
    return match_event_nn(g, P, seeds, ns, nv, vx, vy, vz, vtx, vty, vid, ut, out, cap, near,
                          event);
  const int logm = !g_nolog;
  pair_eval *pe = (pair_eval *)malloc(sizeof(pair_eval) * (size_t)ns * (size_t)nv);
  double *best_v = (double *)malloc(sizeof(double) * (size_t)nv);
  double *best_s = (double *)malloc(sizeof(double) * (size_t)ns);
  for (int v = 0; v < nv; ++v) best_v[v] = INFINITY;
  for (int s = 0; s < ns; ++s) best_s[s] = INFINITY;
  for (int v = 0; v < nv; ++v)
    for (int s = 0; s < ns; ++s) {
      pair_eval r = eval_pair(P, g, &seeds[s], vx[v], vy[v], vz[v], vtx[v], vty[v], logm);
      apply_ut(g, P, ut, vx[v], vy[v], vz[v], vtx[v], vty[v], &r);
      pe[(size_t)v * ns + s] = r;
      if (r.ok) {
        if (r.chi2 < best_v[v]) best_v[v] = r.chi2;
        if (r.chi2 < best_s[s]) best_s[s] = r.chi2;
      }
    }
  /* the lead of a pair over the other survivors of its row and its column */
  const double floor_m = 1e-3 * P->chi2m_max;
  double *sec_v = (double *)malloc(sizeof(double) * (size_t)nv);
  double *sec_s = (double *)malloc(sizeof(double) * (size_t)ns);
  for (int v = 0; v < nv; ++v) sec_v[v] = INFINITY;
  for (int s = 0; s < ns; ++s) sec_s[s] = INFINITY;
  /* second lowest of each row and column: the lowest once one copy of the
   * best is set aside (an exact tie gives a lead of 0) */
  for (int v = 0; v < nv && logm; ++v) {
    int seen = 0;
    for (int s = 0; s < ns; ++s) {
      const pair_eval *r = &pe[(size_t)v * ns + s];
      if (!r->ok) continue;
      if (r->chi2 == best_v[v] && !seen) { seen = 1; continue; }
      sec_v[v] = fmin(sec_v[v], r->chi2);
    }
  }
  for (int s = 0; s < ns && logm; ++s) {
    int seen = 0;
    for (int v = 0; v < nv; ++v) {
      const pair_eval *r = &pe[(size_t)v * ns + s];
      if (!r->ok) continue;
      if (r->chi2 == best_s[s] && !seen) { seen = 1; continue; }
      sec_s[s] = fmin(sec_s[s], r->chi2);
    }
  }
  int n = 0;
  for (int v = 0; v < nv; ++v)
    for (int s = 0; s < ns; ++s) {
      const pair_eval *r = &pe[(size_t)v * ns + s];
      const int kept = r->ok && r->chi2 == best_v[v] && r->chi2 == best_s[s];
      if (!kept) {
        if (!near) continue;
        double m = r->m;   /* rejected by a cut: its margin to acceptance */
        if (r->ok) {       /* survived the cuts, lost the best choice */
          const double sc = fmax(r->chi2, floor_m);
          m = fmax(r->chi2 > best_v[v] ? (r->chi2 - best_v[v]) / sc : 0.0,
                   r->chi2 > best_s[s] ? (r->chi2 - best_s[s]) / sc : 0.0);
        }
        if (m < ORC_NEAR && logm) {
          orc_near *q = (orc_near *)dyn_push(near);
          memset(q, 0, sizeof(*q));
          q->event = event; q->kind = 4; q->velo_idx = v; q->it = seeds[s].it; q->margin = m;
          memcpy(q->id, seeds[s].id, sizeof(q->id));
        }
        continue;
      }
      if (n < cap) {
        orc_long *L = &out[n];
        L->velo_idx = v; L->velo_id = vid[v]; L->seed_idx = s; L->n_ut = r->n_ut;
        memcpy(L->ut_id, r->ut_id, sizeof(L->ut_id));
        L->qop = r->qop; L->chi2 = r->chi2; L->zm = r->zm;
        L->dx = r->dx; L->dy = r->dy; L->dtx = r->dtx; L->dty = r->dty;
        L->gp = -1.0;
        const double sc = fmax(r->chi2, floor_m);
        L->margin = fmin(fmin(seeds[s].margin, r->m),
                         fmin((sec_v[v] - r->chi2) / sc, (sec_s[s] - r->chi2) / sc));
      }
      ++n;
    }
  free(pe); free(best_v); free(best_s); free(sec_v); free(sec_s);
  return n;
}

/* ------------------------------------------------------- whole event ---- */

typedef struct { dyn seeds, longs, near; } ev_out;

/* Seeding of one event half with the x-z iterations it0..it1 (Sec. 3.3):
 * candidates, the clone vote over all of them (which also drops a repeated
 * iteration-1 track), UV seeding of the survivors; seeds are appended to
 * o->seeds. */
static void seed_half(const orc_geom *g, const orc_params *P, const int32_t *off, const float *X,
                      const float *Z, const int32_t *ID, int half, int it0, int it1, int event,
                      ev_out *o) {
  const int n_pos = off[24];
  dyn c = {NULL, 0, 0, sizeof(orc_cand)};
  for (int it = it0; it <= it1; ++it) xz_iteration(g, P, off, X, Z, half, it, &c);
  /* the clone vote sees the candidates that passed the fit; those the fit
   * or the x-hit count rejected by a narrow margin are near misses, and
   * the fit's near misses are also rivals in the vote margins */
  const orc_cand *all = (const orc_cand *)c.p;
  orc_cand *rv = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)(c.n > 0 ? c.n : 1));
  double *xzm = (double *)malloc(sizeof(double) * (size_t)(c.n > 0 ? c.n : 1));
  int m = 0, nr;
  for (int i = 0; i < c.n; ++i)
    if (all[i].status == 0) { rv[m] = all[i]; xzm[m] = all[i].margin; ++m; }
  nr = m;
  for (int i = 0; i < c.n; ++i) {
    if (all[i].status == 0 || !(all[i].margin < ORC_NEAR)) continue;
    push_near(&o->near, event, 1, -1, &all[i], NULL, ID, all[i].margin);
    if (all[i].status == 2) { rv[nr] = all[i]; xzm[nr] = all[i].margin; ++nr; }
  }
  orc_cand *cs = rv;   /* the voters: rv[0, m) */
  int32_t *keep = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
  double *vm = (double *)malloc(sizeof(double) * (size_t)(nr > 0 ? nr : 1));
  orc_clone_vote(cs, m, n_pos, keep);
  vote_margins(rv, nr, m, n_pos, xzm, vm);
  for (int i = 0; i < m; ++i) {
    cs[i].margin = fmin(cs[i].margin, vm[i]);
    if (!keep[i]) {
      if (cs[i].margin < ORC_NEAR) push_near(&o->near, event, 2, -1, &cs[i], NULL, ID, cs[i].margin);
      continue;
    }
    orc_seed sd;
    const int made = P->uv_mode == 1 ? orc_uv(g, P, off, X, Z, ID, &cs[i], &sd)
                                     : uv_iterative(g, P, off, X, Z, ID, &cs[i], &sd, &o->near, event);
    if (made) *(orc_seed *)dyn_push(&o->seeds) = sd;
  }
  free(keep);
  free(vm);
  free(xzm);
  free(rv);
  free(c.p);
}

static void run_event(const orc_geom *g, const orc_params *P, const int32_t *off,
                      const float *X, const float *Z, const int32_t *ID, int nv,
                      const float *vx, const float *vy, const float *vz, const float *vtx,
                      const float *vty, const int32_t *vid, const ut_event *ut, int event,
                      ev_out *o) {
  o->seeds = (dyn){NULL, 0, 0, sizeof(orc_seed)};
  o->longs = (dyn){NULL, 0, 0, sizeof(orc_long)};
  o->near = (dyn){NULL, 0, 0, sizeof(orc_near)};
  const int n_pos = off[24];
  for (int half = 0; half < 2; ++half) seed_half(g, P, off, X, Z, ID, half, 0, 1, event, o);
  if (P->third_iter == 1) {
    /* Clean-up (Sec. 3): the hits of every seed found so far leave the
     * event; the third iteration runs on what is left, in arrays of their
     * own (zones and x order kept), and its seeds' positions are mapped back
     * to the event's. */
    const int ns1 = o->seeds.n;
    char *used = (char *)calloc((size_t)(n_pos > 0 ? n_pos : 1), 1);
    for (int i = 0; i < ns1; ++i) {
      const orc_seed *sd = &((const orc_seed *)o->seeds.p)[i];
      for (int l = 0; l < ORC_NL; ++l)
        if (sd->pos[l] >= 0) used[sd->pos[l]] = 1;
    }
    float *X2 = (float *)malloc(sizeof(float) * (size_t)(n_pos > 0 ? n_pos : 1));
    float *Z2 = (float *)malloc(sizeof(float) * (size_t)(n_pos > 0 ? n_pos : 1));
    int32_t *ID2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_pos > 0 ? n_pos : 1));
    int32_t *from = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_pos > 0 ? n_pos : 1));
    int32_t off2[25];
    int k = 0;
    for (int zn = 0; zn < 24; ++zn) {
      off2[zn] = k;
      for (int i = off[zn]; i < off[zn + 1]; ++i)
        if (!used[i]) { X2[k] = X[i]; Z2[k] = Z[i]; ID2[k] = ID[i]; from[k] = i; ++k; }
    }
    off2[24] = k;
    for (int half = 0; half < 2; ++half) seed_half(g, P, off2, X2, Z2, ID2, half, 2, 2, event, o);
    for (int i = ns1; i < o->seeds.n; ++i) {
      orc_seed *sd = &((orc_seed *)o->seeds.p)[i];
      for (int l = 0; l < ORC_NL; ++l)
        if (sd->pos[l] >= 0) sd->pos[l] = from[sd->pos[l]];
    }
    free(used); free(X2); free(Z2); free(ID2); free(from);
  }
  const int ns = o->seeds.n;
  if (ns > 0 && nv > 0) {
    /* a pair count above cap only sizes the second call; near misses are
     * taken in the call whose results are kept */
    int cap = ns < nv ? ns : nv;
    cap = cap * 4 + 16;
    orc_long *tmp = (orc_long *)malloc(sizeof(orc_long) * (size_t)cap);
    const int near0 = o->near.n;
    int n = match_event(g, P, (orc_seed *)o->seeds.p, ns, nv, vx, vy, vz, vtx, vty, vid, ut,
                        tmp, cap, &o->near, event);
    if (n > cap) {
      free(tmp);
      o->near.n = near0;
      tmp = (orc_long *)malloc(sizeof(orc_long) * (size_t)n);
      match_event(g, P, (orc_seed *)o->seeds.p, ns, nv, vx, vy, vz, vtx, vty, vid, ut, tmp, n,
                  &o->near, event);
    }
    for (int i = 0; i < n; ++i) *(orc_long *)dyn_push(&o->longs) = tmp[i];
    free(tmp);
  }
}

typedef struct {
  const orc_geom *g;
  const orc_params *P;
  int n_events;
  const int32_t *zone_off;
  const float *hx, *hz;
  const int32_t *hid;
  const int32_t *velo_off;
  const float *vx, *vy, *vz, *vtx, *vty;
  const int32_t *vid;
  const int32_t *ut_off;
  const float *ut_x;
  const int32_t *ut_id;
  ev_out *outs;
  int next;
  int log_margins;
  pthread_mutex_t mu;
} job;

static void *worker(void *arg) {
  job *J = (job *)arg;
  g_nolog = !J->log_margins;
  for (;;) {
    pthread_mutex_lock(&J->mu);
    int e = J->next++;
    pthread_mutex_unlock(&J->mu);
    if (e >= J->n_events) break;
    int32_t off[25];
    const int base = J->zone_off[e * 24];
    for (int k = 0; k <= 24; ++k) off[k] = J->zone_off[e * 24 + k] - base;
    const int v0 = J->velo_off[e], nv = J->velo_off[e + 1] - v0;
    const ut_event ut = {J->ut_off ? J->ut_off + (size_t)e * ORC_NUT : NULL, J->ut_x, J->ut_id};
    run_event(J->g, J->P, off, J->hx + base, J->hz + base, J->hid + base, nv,
              J->vx + v0, J->vy + v0, J->vz + v0, J->vtx + v0, J->vty + v0, J->vid + v0,
              &ut, e, &J->outs[e]);
  }
  return NULL;
}

int orc_run(const orc_geom *g, const orc_params *p, int n_events, const int32_t *zone_off,
            const float *hx, const float *hz, const int32_t *hid, const int32_t *velo_off,
            const float *vx, const float *vy, const float *vz, const float *vtx,
            const float *vty, const int32_t *vid, const int32_t *ut_off, const float *ut_x,
            const int32_t *ut_id, int n_threads, int log_margins, orc_result *res) {
  memset(res, 0, sizeof(*res));
  if (n_events < 0) return -1;
  job J = {g, p, n_events, zone_off, hx, hz, hid, velo_off, vx, vy, vz, vtx, vty, vid,
           ut_off, ut_x, ut_id, NULL, 0, log_margins, PTHREAD_MUTEX_INITIALIZER};
  J.outs = (ev_out *)calloc((size_t)(n_events > 0 ? n_events : 1), sizeof(ev_out));
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  pthread_t th[256];
  for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, worker, &J);
  for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
  int64_t ns = 0, nl = 0, nn = 0;
  for (int e = 0; e < n_events; ++e) {
    ns += J.outs[e].seeds.n; nl += J.outs[e].longs.n; nn += J.outs[e].near.n;
  }
  res->n_near = nn;
  res->near = (orc_near *)malloc(sizeof(orc_near) * (size_t)(nn > 0 ? nn : 1));
  int64_t in = 0;
  for (int e = 0; e < n_events; ++e) {
    if (J.outs[e].near.n)
      memcpy(res->near + in, J.outs[e].near.p, sizeof(orc_near) * (size_t)J.outs[e].near.n);
    in += J.outs[e].near.n;
    free(J.outs[e].near.p);
  }
  res->n_seeds = ns;
  res->n_longs = nl;
  res->seed_off = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_events + 1));
  res->long_off = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_events + 1));
  res->seeds = (orc_seed *)malloc(sizeof(orc_seed) * (size_t)(ns > 0 ? ns : 1));
  res->longs = (orc_long *)malloc(sizeof(orc_long) * (size_t)(nl > 0 ? nl : 1));
  int64_t is = 0, il = 0;
  for (int e = 0; e < n_events; ++e) {
    res->seed_off[e] = (int32_t)is;
    res->long_off[e] = (int32_t)il;
    if (J.outs[e].seeds.n)
      memcpy(res->seeds + is, J.outs[e].seeds.p, sizeof(orc_seed) * (size_t)J.outs[e].seeds.n);
    if (J.outs[e].longs.n)
      memcpy(res->longs + il, J.outs[e].longs.p, sizeof(orc_long) * (size_t)J.outs[e].longs.n);
    is += J.outs[e].seeds.n;
    il += J.outs[e].longs.n;
    free(J.outs[e].seeds.p);
    free(J.outs[e].longs.p);
  }
  res->seed_off[n_events] = (int32_t)is;
  res->long_off[n_events] = (int32_t)il;
  free(J.outs);
  return 0;
}

void orc_free(orc_result *res) {
  free(res->seed_off); free(res->seeds); free(res->long_off); free(res->longs); free(res->near);
  memset(res, 0, sizeof(*res));
}
