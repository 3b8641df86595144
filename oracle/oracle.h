/* CPU oracle for SciFi Seeding + VELO-SciFi Matching, in FP64.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library under paper_2606_14480_amd/) never links, imports or calls it,
 * and shares no header, helper or constant table with it.
 *
 * Every float input is widened exactly to double; every quantity is then
 * computed in double.  Layout of the inputs is the same as the product's
 * batch: hits grouped in zones zone = (event*2 + half)*12 + layer, x-sorted
 * inside each zone.
 */
#ifndef SM_ORACLE_H
#define SM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NL 12
#define ORC_NUT 4
#define ORC_NN_IN 8
#define ORC_NN_HID 32

/* Ghost-probability network of the final selection (Sec. 4.4): inputs
 * z_match, dx, dy, dtx, dty, chi2_match, eta of the VELO state and the
 * seed's SciFi hit count (in that order), each standardised as
 * (x - mean) / scale; one hidden layer of ORC_NN_HID rectified units; a
 * logistic output (READING: the paper gives the layer sizes only). */
typedef struct {
  double mean[ORC_NN_IN], scale[ORC_NN_IN];
  double w1[ORC_NN_HID][ORC_NN_IN], b1[ORC_NN_HID];
  double w2[ORC_NN_HID], b2;
} orc_ghost_nn;

typedef struct {
  double z[ORC_NL];      /* nominal layer z [mm] */
  double tan_a[ORC_NL];  /* tan of the stereo angle (0 for x-layers) */
  double z_ref;          /* eq. trackequation reference point */
  /* UT layers UTaX, UTaU, UTbV, UTbX (Sec. 4.3; positions are a reading) */
  double ut_z[ORC_NUT], ut_tan[ORC_NUT];
} orc_geom;

typedef struct {
  /* XZ seeding (Sec. 3.2, 3.3) */
  double p_min;            /* MeV */
  double invp_a, invp_b;   /* eq. invp */
  double alpha0, alpha1;   /* eq. alphacorr */
  double d_ratio;          /* eq. trackequation */
  double kappa_c;          /* c_x per unit 1/p, for the third-hit window */
  double t2_tol0, t2_tol1; /* third-hit window tol0 + tol1*|K3 c_pred| */
  double ext_tol;          /* x-layer extension window */
  int32_t min_x_hits;
  int32_t pad0;
  double sigma_x;          /* hit resolution */
  double chi2x_max;        /* reduced chi2 cut of the x-z fit */
  /* UV seeding (Sec. 3.4) */
  double uv_tol, y_max;
  int32_t min_uv_hits;
  int32_t pad1;
  double chi2y_max;
  /* Matching (Sec. 4) */
  double zm[5];            /* A_x .. E_x of eq. z_match */
  double z_ymatch, z_state;
  double max_dx, max_dy, max_dtx, max_dty;
  double tolx_scale, tolx_a, tolx_b;
  double toly_scale, toly_a, toly_b;
  double tol_tx, tol_ty;
  double chi2m_max;
  double polarity;
  /* UV variant (Sec. 3.4): 0 iterative (default), 1 Hough clusters */
  int32_t uv_mode;
  int32_t hough_bins;  /* coarse t_y bins over the half's range */
  int32_t hough_best;  /* most populated coarse bins kept */
  int32_t hough_fine;  /* fine bins per kept coarse bin */
  int32_t hough_min;   /* entries a coarse bin needs to be kept */
  int32_t pad2;
  /* Final selection (Sec. 4.4).  final_sel 0: a surviving pair is kept when
   * its chi2_match is the lowest among the survivors on its seed and among
   * those on its VELO state (READING, used without a ghost network).
   * final_sel 1: pairs with ghost probability < ghost_cut are retained; a
   * retained track is a clone, and dropped, when another retained track on
   * its VELO state or on its seed has a ghost probability at least clone_gap
   * lower. */
  int32_t final_sel;
  int32_t pad3;
  double ghost_cut, clone_gap;
  orc_ghost_nn ghost_nn;
  /* UT hit search (Sec. 4.3).  ut_mode 0: off; 1: every pair that passed the
   * preselection and the chi2_match cut is extrapolated to the UT layers
   * with gamma_x = a_gamma + b_gamma q/p (eq. gamma_parametrisation), takes
   * the closest hit in a loose window until one is found (which then fixes
   * gamma_x), then the closest hit in a tight window in each later layer;
   * pairs with fewer than ut_min_hits UT hits leave the candidates before
   * the final selection.  Windows (Table 2): min(max(A + B/p, lo), hi), p in
   * GeV/c; hi = 0 marks a layer without that window. */
  int32_t ut_mode, ut_min_hits;
  double a_gamma, b_gamma;
  double ut_loose_a[ORC_NUT], ut_loose_b[ORC_NUT], ut_loose_lo[ORC_NUT], ut_loose_hi[ORC_NUT];
  double ut_tight_a[ORC_NUT], ut_tight_b[ORC_NUT], ut_tight_lo[ORC_NUT], ut_tight_hi[ORC_NUT];
  /* Third x-z iteration with clean-up (Sec. 3: the HLT2 form cleans the
   * environment between iterations and opens wider windows for lower
   * momenta; the HLT1 form runs two).  third_iter 1: after iterations 0 and
   * 1, every hit on one of their seeds is removed from its event half, and
   * iteration 2 runs on the rest: iteration 0's layers, windows opened for
   * p_min3, its own clone vote, UV search and best choice; its seeds carry
   * it = 2 and join the others before Matching. */
  int32_t third_iter;
  int32_t pad4;
  double p_min3;           /* MeV */
} orc_params;

/* Margins.  Every decision that shapes an output is logged with its
 * relative distance from going the other way: |q - cut| / cut for a window
 * or a cut (for the ghost-probability cut and clone gap of the network form,
 * the distance in units of probability), (second - best) / scale for a closest-hit choice (scale: the
 * window) or a best-candidate choice (scale: the larger of the best value and
 * 1e-3 of the cut), and the relative score gap to the nearest other score on
 * a shared hit for the clone vote.  A kept track carries the smallest margin
 * of its decisions; a rejection that came within ORC_NEAR of going the other
 * way is listed as a near miss (orc_near). */
#define ORC_NEAR 1e-3

/* One three-hit combination and what became of it. */
typedef struct {
  int32_t half, it, status; /* status 0: passed the fit cut; 1: < min_x_hits; 2: chi2 cut */
  int32_t n;                /* number of x hits */
  int32_t pos[ORC_NL];      /* event-relative hit positions by layer, -1 if none */
  double a, b, c, chi2, score;
  double margin;            /* smallest margin of its x-z decisions (and, once voted, the vote) */
} orc_cand;

typedef struct {
  double a, b, c, y0, ty, chi2x, chi2y, score;
  int32_t nx, nuv, half, it;
  int32_t pos[ORC_NL];
  int32_t id[ORC_NL];
  double margin;            /* smallest margin of every decision that made this seed */
} orc_seed;

typedef struct {
  int32_t velo_idx, velo_id, seed_idx, n_ut;
  int32_t ut_id[ORC_NUT];   /* UT hit id per layer, -1 where none (ut_mode 1) */
  double qop, chi2, zm, dx, dy, dtx, dty;
  double gp;                /* ghost probability (final_sel 1), else -1 */
  double margin;            /* smallest margin of its seed's and its matching decisions */
} orc_long;

/* A VELO-seed pair that passed the preselection and the chi2_match cut, with
 * the network's inputs (unstandardised) and, for final_sel 1, its ghost
 * probability (else -1). */
typedef struct {
  int32_t velo_idx, seed_idx;
  double f[ORC_NN_IN];
  double gp;
} orc_pair;

/* A near miss: a track or pair that a decision within ORC_NEAR of its
 * threshold rejected.  kind: 1 an x-z candidate (fit or x-hit count), 2 an
 * x-z track killed by the clone vote, 3 a stereo-hit combination not chosen
 * or cut, 4 a VELO-seed pair rejected or not the best.  id holds the hit ids
 * by layer (-1 where none; only x layers for kinds 1 and 2); velo_idx is the
 * VELO state of a kind-4 pair (-1 otherwise); it the x-z iteration that
 * found the track. */
typedef struct {
  int32_t event, kind, velo_idx, it;   /* it: x-z iteration of the track */
  int32_t id[ORC_NL];
  double margin;
} orc_near;

typedef struct {
  int64_t n_seeds, n_longs;
  int32_t *seed_off;   /* [n_events + 1] */
  orc_seed *seeds;
  int32_t *long_off;   /* [n_events + 1] */
  orc_long *longs;
  int64_t n_near;
  orc_near *near;      /* near misses of every event, by event */
} orc_result;

void orc_default_geom(orc_geom *g);
void orc_default_params(orc_params *p);

/* out[0] = Delta x3^max, out[1] = alpha_corr, out[2] = K3 of iteration `it`
 * (0, 1, or 2: the third iteration's layers and p_min3) at the nominal layer
 * z. */
void orc_window_constants(const orc_geom *g, const orc_params *p, int it, double out[3]);

/* Stage entry points on ONE event (event-local zone offsets [25], hits). */
int orc_xz_candidates(const orc_geom *g, const orc_params *p, const int32_t *zone_off,
                      const float *x, const float *z, int half, int it,
                      orc_cand *out, int cap);
void orc_clone_vote(const orc_cand *c, int n, int n_pos, int32_t *keep);
int orc_uv(const orc_geom *g, const orc_params *p, const int32_t *zone_off,
           const float *x, const float *z, const int32_t *id, const orc_cand *cand,
           orc_seed *out);
/* ut_off: the event's UT layer offsets [5] into ut_x / ut_id (NULL: none) */
int orc_match(const orc_geom *g, const orc_params *p, const orc_seed *seeds, int ns,
              int nv, const float *vx, const float *vy, const float *vz,
              const float *vtx, const float *vty, const int32_t *vid,
              const int32_t *ut_off, const float *ut_x, const int32_t *ut_id,
              orc_long *out, int cap);
/* The pairs of one event that survive the preselection and the chi2_match
 * cut (the candidates of the final selection), VELO-major; returns their
 * count, writing at most cap. */
int orc_match_pairs(const orc_geom *g, const orc_params *p, const orc_seed *seeds, int ns,
                    int nv, const float *vx, const float *vy, const float *vz,
                    const float *vtx, const float *vty, const int32_t *ut_off,
                    const float *ut_x, const int32_t *ut_id, orc_pair *out, int cap);
/* Half-width of the UT search window (Table 2) of layer 0..3 for a track of
 * this q/p (1/MeV), loose (tight = 0) or tight; 0 where Table 2 gives none. */
double orc_ut_window(const orc_params *p, int layer, int tight, double qop);
/* The network's ghost probability for one input vector (unstandardised). */
double orc_ghost_prob(const orc_params *p, const double f[ORC_NN_IN]);

/* Whole batch; returns 0 on success.  Results are malloc'd; free with
 * orc_free.  log_margins = 0 skips the margin bookkeeping that costs time of
 * its own (closest-hit rescans, vote margins, near misses): the tracks are
 * the same, their margins are then only partly filled and no near misses are
 * listed (for timing the method alone). */
/* ut_off [n_events*4 + 1], ut_x, ut_id: the UT hits (NULL: none; then a
 * ut_mode 1 run finds no UT hits). */
int orc_run(const orc_geom *g, const orc_params *p, int n_events, const int32_t *zone_off,
            const float *hx, const float *hz, const int32_t *hid, const int32_t *velo_off,
            const float *vx, const float *vy, const float *vz, const float *vtx,
            const float *vty, const int32_t *vid, const int32_t *ut_off, const float *ut_x,
            const int32_t *ut_id, int n_threads, int log_margins, orc_result *res);
void orc_free(orc_result *res);

#ifdef __cplusplus
}
#endif
#endif
