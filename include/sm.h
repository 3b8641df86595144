/* sm.h — C-ABI of the MI355X SciFi Seeding + VELO-SciFi Matching library.
 *
 * The calls follow the paper's problem statement: SciFi hits and VELO track
 * states go in, T-tracks ("seeds", Sec. 3, output of the UV step of Sec. 3.4)
 * and Long tracks (Sec. 4, output of the final selection of Sec. 4.4) come
 * out.  All compute runs in HIP kernels for gfx950; this header has no torch
 * or HIP types.
 *
 * Conventions shared by every call
 *  - Pointers inside sm_batch / sm_out are DEVICE pointers on the context's
 *    device, owned by the caller, and must stay valid until the call (or, for
 *    sm_submit, the matching sm_poll) returns SM_OK or an error.  Inputs are
 *    never written.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *  - Every call returns an sm_status; nothing aborts the process.  When an
 *    output buffer is too small the call returns SM_ERR_CAPACITY, fills
 *    sm_out.n_seeds / n_longs with the sizes needed, and the content of the
 *    output arrays is unspecified; nothing is truncated silently.  Internal
 *    scratch that proves too small is grown and the batch re-run inside the
 *    call.
 *  - Results are deterministic: the same batch gives bit-identical outputs
 *    whatever the batch composition, launch form or grid shape.
 */
#ifndef SM_H
#define SM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SM_N_LAYERS 12
#define SM_ZONES_PER_EVENT 24
#define SM_N_UT 4   /* UT layers UTaX, UTaU, UTbV, UTbX */

typedef enum {
  SM_OK = 0,
  SM_ERR_INVALID = -1,   /* bad argument or malformed batch */
  SM_ERR_UNSORTED = -2,  /* hits not x-sorted inside a zone (validate mode) */
  SM_ERR_CAPACITY = -3,  /* an output buffer is too small; sizes in sm_out */
  SM_ERR_OOM = -4,       /* device allocation failed */
  SM_ERR_DEVICE = -5,    /* a HIP runtime call failed */
  SM_ERR_BUSY = -6,      /* sm_submit: every serving slot is in use */
  SM_ERR_NOT_READY = -7, /* sm_poll: the batch is still running */
  SM_ERR_LIMIT = -8      /* an event exceeds the library's hard per-event limit */
} sm_status;

typedef struct sm_ctx sm_ctx; /* opaque, library-owned */

/* Detector description (Sec. 1): nominal z of the 12 SciFi layers (3
 * stations x {x, u, v, x}), tan of each layer's stereo angle (0 for x-layers,
 * +-tan 5 deg for u/v) and the reference z of eq. trackequation. */
typedef struct {
  double z[SM_N_LAYERS];
  double tan_stereo[SM_N_LAYERS];
  double z_ref;
  /* UT (Sec. 4.3): z of the four layers and tan of their stereo angles (a
   * stereo hit measures x - y tan(alpha)); the paper prints neither, the
   * defaults are 2327.5, 2372.5, 2597.5, 2642.5 mm and 0, +tan 5, -tan 5, 0 */
  double ut_z[SM_N_UT];
  double ut_tan[SM_N_UT];
} sm_geometry;

/* Ghost-probability network of the final selection (Sec. 4.4).  Inputs, in
 * this order: z_match (eq. z_match), dx, dy, dtx, dty, chi2_match, eta of the
 * VELO state (asinh(1 / sqrt(tx^2 + ty^2)), the slope floored at 1e-9) and the
 * seed's SciFi hit count (n_x + n_uv); each is standardised as
 * (x - mean[i]) / scale[i].  One hidden layer of SM_NN_HIDDEN rectified units
 * (h_j = max(0, b1[j] + sum_i w1[j][i] x_i)), a logistic output
 * (1 / (1 + exp(-(b2 + sum_j w2[j] h_j)))).  Evaluated in FP64.  The paper
 * gives the inputs and layer sizes only; the package's ghost_nn.json holds
 * weights trained on the synthetic generator's truth. */
#define SM_NN_INPUTS 8
#define SM_NN_HIDDEN 32
typedef struct {
  double mean[SM_NN_INPUTS], scale[SM_NN_INPUTS];  /* scale must be non-zero */
  double w1[SM_NN_HIDDEN][SM_NN_INPUTS], b1[SM_NN_HIDDEN];
  double w2[SM_NN_HIDDEN], b2;
} sm_ghost_nn;

/* Every constant of the method.  sm_default_params() fills the paper's values
 * and the documented readings where the paper gives none. */
typedef struct {
  /* XZ seeding, Sec. 3.2-3.3 */
  double p_min;            /* MeV/c, minimum momentum the windows are opened for */
  double invp_a, invp_b;   /* eq. invp, per MeV/c per mm and per mm^2 */
  double alpha0, alpha1;   /* eq. alphacorr */
  double d_ratio;          /* eq. trackequation cubic term, 1/mm */
  double kappa_c;          /* third-hit window centre: c_x = kappa_c / p */
  double t2_tol0, t2_tol1; /* third-hit half-width tol0 + tol1 |K3 c_pred| (mm) */
  double ext_tol;          /* x-layer extension window (mm), Sec. 3.2 */
  int32_t min_x_hits;      /* Sec. 3.2 */
  int32_t pad0;
  double sigma_x;          /* hit resolution used in both chi2 (mm) */
  double chi2x_max;        /* reduced chi2 cut of the x-z fit */
  /* UV seeding, Sec. 3.4 */
  double uv_tol;           /* mm */
  double y_max;            /* |y| range of a detector half (mm) */
  int32_t min_uv_hits;
  int32_t pad1;
  double chi2y_max;        /* reduced chi2 cut of the y-z fit */
  /* Matching, Sec. 4 */
  double zm[5];            /* A_x, B_x, C_x, D_x, E_x of eq. z_match (Table 1) */
  double z_ymatch;         /* z of the y matching plane (mm) */
  double z_state;          /* z of the SciFi state used for matching (mm) */
  double max_dx, max_dy, max_dtx, max_dty;   /* preselection, Sec. 4.2 */
  double tolx_scale, tolx_a, tolx_b;         /* tol_x = s (a^2 + b^2 dtx^2) */
  double toly_scale, toly_a, toly_b;         /* tol_y = s (a^2 + b^2 rho) */
  double tol_tx, tol_ty;
  double chi2m_max;        /* chi2_match cut */
  double polarity;         /* +1 or -1, magnet polarity */
  /* UV seeding variant, Sec. 3.4: 0 the iterative search, 1 the Hough-cluster
   * search.  The Hough search histograms t_y = y/z of every stereo hit whose
   * y lies in the half, over [0, y_max/z_min] (upper half) or
   * [-y_max/z_min, 0] (lower half), z_min the lowest nominal stereo-layer z;
   * keeps the hough_best most populated bins holding at least hough_min
   * entries (ties to the lower bin), splits each into hough_fine bins and
   * tries the mean t_y of every non-empty fine bin as a hypothesis.
   * uv_mode 1 is currently refused by sm_create (SM_ERR_INVALID): its kernel
   * is switched off until a memory fault seen once in it is explained. */
  int32_t uv_mode;
  int32_t hough_bins;      /* 1..128 */
  int32_t hough_best;      /* >= 1, hough_best * hough_fine <= 64 */
  int32_t hough_fine;      /* >= 1 */
  int32_t hough_min;       /* >= 1 */
  int32_t pad2;
  /* Final selection of Matching, Sec. 4.4.  final_sel 0 (default): a pair
   * that passed the preselection and the chi2_match cut is kept when its
   * chi2_match is the lowest among such pairs on its seed and among those on
   * its VELO state (the reading used without network weights).  final_sel 1:
   * pairs whose ghost probability (ghost_nn) is below ghost_cut are
   * retained; a retained track is a clone, and dropped, when another retained
   * track on its VELO state or on its seed has a ghost probability lower by
   * clone_gap or more.  Any other value: SM_ERR_INVALID. */
  int32_t final_sel;
  int32_t pad3;
  double ghost_cut;        /* 0.8 */
  double clone_gap;        /* 0.05 */
  sm_ghost_nn ghost_nn;    /* read when final_sel = 1 */
  /* UT hit search, Sec. 4.3.  ut_mode 0 (default): off.  ut_mode 1: every
   * pair that passed the preselection and the chi2_match cut is extrapolated
   * from its VELO state with eq. velo_ut_extrapolation, gamma_x = a_gamma +
   * b_gamma q/p (eq. gamma_parametrisation; q/p of the pair, 1/MeV).  Layer
   * by layer it takes the closest hit in the loose window until one is
   * found, which refits gamma_x so that the parabola passes through it, then
   * the closest hit in the tight window of each later layer.  A pair with
   * fewer than ut_min_hits UT hits leaves the candidates before the final
   * selection.  Windows (Table 2): min(max(a + b / p, lo), hi), p in GeV/c,
   * per layer; hi = 0 marks a layer without that window.  The batch must then
   * carry UT hits (sm_batch.ut_off non-NULL), else SM_ERR_INVALID. */
  int32_t ut_mode;
  int32_t ut_min_hits;     /* 3 ("more than two"), 1..4 */
  double a_gamma, b_gamma; /* Table 1: 7.707063e-11, -7.817364e-3 */
  double ut_loose_a[SM_N_UT], ut_loose_b[SM_N_UT], ut_loose_lo[SM_N_UT], ut_loose_hi[SM_N_UT];
  double ut_tight_a[SM_N_UT], ut_tight_b[SM_N_UT], ut_tight_lo[SM_N_UT], ut_tight_hi[SM_N_UT];
  /* Third x-z iteration with clean-up (Sec. 3: the HLT2 form finds high
   * momenta first, cleans the environment and searches again with wider
   * windows for lower momenta; the HLT1 form runs two iterations).
   * third_iter 0 (default): two iterations.  third_iter 1: after iterations
   * 0 and 1 of the whole batch, every hit on one of their seeds is removed,
   * and iteration 2 runs on the hits left: iteration 0's layers, windows
   * opened for p_min3, its own clone vote, UV search and best choice.  Its
   * seeds (iter = 2) follow the event's other seeds and join Matching.  Only
   * the batched calls (sm_run, sm_submit, sm_profile) run it: sm_run_plain
   * and sm_run_noalloc return SM_ERR_INVALID. */
  int32_t third_iter;
  int32_t pad4;
  double p_min3;           /* MeV/c, default 1500 */
} sm_params;

/* Library resources; zero fields take defaults. */
typedef struct {
  int32_t device;          /* HIP device ordinal */
  int32_t n_slots;         /* concurrent serving slots (sm_submit), default 2 */
  int32_t seed_wgs;        /* persistent workgroups of the seeding kernel (0: auto);
                              otherwise at least 2 (the per-event form runs one
                              workgroup per detector half), else sm_create
                              returns SM_ERR_INVALID */
  int32_t match_wgs;       /* where batched Matching runs.  0: chosen per batch: a
                              matching kernel of seed_wgs workgroups after the
                              seeding kernels, or, when the batch has items for
                              the big-item form, inside the seeding kernel (the
                              workgroup completing an event matches it); > 0:
                              always the matching kernel, with this many
                              workgroups (at most seed_wgs); < 0: always inside
                              the seeding kernel.  Outputs are identical. */
  int32_t lds_hits;        /* per-workgroup LDS hit budget (0: auto) */
  int32_t validate;        /* 1: check offsets and x-sorting before each batch */
  int64_t mem_budget;      /* bytes of device memory the context may hold (0: no cap) */
} sm_config;

/* One batch of events.  Hits of event e, detector half h (0: y > 0,
 * 1: y < 0) and layer l form zone k = (e*2 + h)*12 + l and occupy
 * [zone_off[k], zone_off[k+1]) of the hit arrays, x-sorted ascending.
 * VELO end-states of event e occupy [velo_off[e], velo_off[e+1]). */
typedef struct {
  int32_t n_events;
  int32_t pad;
  int64_t n_hits;          /* = zone_off[n_events*24] (host-side size of the hit arrays) */
  int64_t n_velo;          /* = velo_off[n_events] (host-side size of the VELO arrays) */
  const int32_t *zone_off; /* [n_events*24 + 1], non-decreasing, zone_off[0] = 0 */
  const float *hit_x;      /* measured x (mm); local coordinate for u/v layers */
  const float *hit_z;      /* z of the hit (mm) */
  const int32_t *hit_id;   /* caller's id, reported back in seeds */
  const int32_t *velo_off; /* [n_events + 1] */
  const float *velo_x, *velo_y, *velo_z, *velo_tx, *velo_ty;
  const int32_t *velo_id;
  /* UT hits (Sec. 4.3), read only with ut_mode 1; NULL when there are none.
   * Hits of event e, layer l (0..3: UTaX, UTaU, UTbV, UTbX) occupy
   * [ut_off[e*4 + l], ut_off[e*4 + l + 1]), x-sorted ascending; ut_x is the
   * measured coordinate (x - y tan(alpha) on stereo layers). */
  int64_t n_ut;            /* = ut_off[n_events*4] */
  const int32_t *ut_off;   /* [n_events*4 + 1], non-decreasing, ut_off[0] = 0 */
  const float *ut_x;
  const int32_t *ut_id;    /* caller's id, reported back in long tracks */
} sm_batch;

/* A T-track (Sec. 3): x(z) = ax + bx u + cx u^2 (1 + d_ratio u) and
 * y(z) = y0 + ty u with u = z - z_ref. */
typedef struct {
  float ax, bx, cx;
  float y0, ty;
  float chi2_x, chi2_y;   /* reduced */
  float score;            /* eq. seed_clone_score, rounded to float */
  int32_t n_x, n_uv;      /* hits on x and on stereo layers */
  int32_t half, iter;     /* detector half and XZ iteration that found it */
  int32_t hits[SM_N_LAYERS]; /* hit_id per layer, -1 where none */
} sm_seed;                /* 96 bytes */

/* A Long track (Sec. 4): one VELO state joined with one seed. */
typedef struct {
  int32_t velo_idx;       /* index of the VELO state inside its event */
  int32_t seed_idx;       /* index of the seed inside its event's seed list */
  int32_t velo_id;
  float qop;              /* q/p from the magnet kick, 1/MeV */
  float chi2;             /* chi2_match */
  float z_match;          /* eq. z_match */
  float dx, dy, dtx, dty; /* matching residuals */
  float ghost_prob;       /* final_sel 1: the network's ghost probability; else -1 */
  int32_t n_ut;           /* ut_mode 1: UT hits attached; else 0 */
  int32_t ut_hits[SM_N_UT]; /* their ut_id per layer, -1 where none */
} sm_long;                /* 64 bytes */

/* Outputs, caller-allocated on the device.  Seeds of event e are
 * seeds[seed_off[e] .. seed_off[e+1]) in canonical order (half, iteration,
 * then the positions of the T1, T3 and T2 hits); long tracks of event e are
 * longs[long_off[e] .. long_off[e+1]) ordered by (velo_idx, seed_idx). */
typedef struct {
  int64_t seed_cap, long_cap; /* capacity of seeds[] and longs[] */
  int32_t *seed_off;          /* [n_events + 1] */
  sm_seed *seeds;
  int32_t *long_off;          /* [n_events + 1] */
  sm_long *longs;
  int64_t n_seeds, n_longs;   /* written by the library (host fields) */
} sm_out;

/* Defaults: the geometry of the synthetic detector and the paper's
 * constants (Sec. 3.3.1 eq. invp, eq. alphacorr, Table 1, Sec. 4.2) plus
 * the readings for the values the paper does not print. */
void sm_default_geometry(sm_geometry *g);
void sm_default_params(sm_params *p);

/* Creates a context on cfg->device (NULL cfg: all defaults).  Allocates the
 * scratch, serving slots and streams it owns (the hits stay resident in
 * device memory across the steps of a batch, Sec. 5.2).  SM_ERR_OOM if the
 * device memory or cfg->mem_budget is too small. */
sm_status sm_create(const sm_geometry *g, const sm_params *p, const sm_config *cfg,
                    sm_ctx **out);

/* Seeding (Sec. 3) + Matching (Sec. 4) of a whole batch: events processed
 * together, as the batches of about a thousand events of Sec. 5.3, here as
 * ONE persistent launch per kernel, replayed from a captured HIP graph, with
 * workgroups pulling (event, half) items longest-first from a device work
 * queue.  Blocks until done (stream-ordered after prior work on `stream`). */
sm_status sm_run(sm_ctx *ctx, const sm_batch *batch, sm_out *out, void *stream);

/* The same computation launched as one kernel sequence per event (the plain
 * form: Sec. 5.3's event-level parallelism left out, thread-level kept);
 * bit-identical results to sm_run.  Blocks until done. */
sm_status sm_run_plain(sm_ctx *ctx, const sm_batch *batch, sm_out *out, void *stream);

/* Serving: starts the batch on a free slot (its own stream) and returns at
 * once with a ticket; SM_ERR_BUSY if no slot is free.  batch and out must stay
 * valid until sm_poll reports completion.  Batches on different slots run on
 * the device at the same time (continuous batching of arriving batches; the
 * paper's trigger feeds its cards batches of events, Sec. 5.3, and states no
 * serving loop). */
sm_status sm_submit(sm_ctx *ctx, const sm_batch *batch, sm_out *out, int64_t *ticket);

/* SM_OK once the ticket's batch is done (out->n_seeds / n_longs filled),
 * SM_ERR_NOT_READY while it runs (wait = 0), or its error.  wait != 0 blocks.
 * A ticket is reported complete exactly once; the slot is then free. */
sm_status sm_poll(sm_ctx *ctx, int64_t ticket, int wait);

/* Per-kernel device time of one batched run, from HIP events recorded on
 * `stream` between the kernels (milliseconds): counters and item order,
 * with the big-item form when one launch does both (then seed_big is 0);
 * the big-item seeding form; the main seeding form built without the
 * matching code (seed) and the one with it (seed_fused), of which only the
 * one that fits the batch is launched (the other's interval is empty); the
 * matching kernel (not launched when Matching runs inside seeding; for
 * batches of up to 4096 events it also writes the seeds to the caller's
 * buffers); the offset scans and the copy of the rest to the caller's
 * buffers; and the whole sequence. */
typedef struct {
  float prepare, seed_big, seed, seed_fused, match, copy, total;
} sm_kernel_times;

/* Tracing: runs the batched form once as plain stream launches (no graph)
 * with an event between kernels and fills `t`.  Results are identical to
 * sm_run.  Blocks until done. */
sm_status sm_profile(sm_ctx *ctx, const sm_batch *batch, sm_out *out, void *stream,
                     sm_kernel_times *t);

/* For callers that cannot allocate device memory (code that runs while a HIP
 * graph is being captured, tight serving loops, harnesses that forbid
 * hipMalloc): the batched computation of sm_run, with outputs bit-identical
 * to sm_run's, run without any allocation.  The call itself makes no device
 * or host allocation and captures no graph: it launches the kernels directly
 * on `stream` and blocks until they are done.
 *
 * Its scratch is one static device array of SM_NOALLOC_SCRATCH_BYTES on each
 * GPU, set up by the first sm_create on that GPU and held until the process
 * ends.  That array is shared by every call on the GPU, from any context or
 * thread: calls that overlap on one GPU race and their outputs are undefined.
 * Each call clears what must start at zero; the array otherwise keeps the
 * last call's contents.  The persistent grid is fixed at
 * SM_NOALLOC_WORKGROUPS workgroups and the big-item form is not used.
 *
 * Limits: n_events <= SM_NOALLOC_MAX_EVENTS and n_velo <= SM_NOALLOC_MAX_VELO,
 * else SM_ERR_LIMIT before any launch.  The per-workgroup scratch (triplets,
 * candidates, UV combinations, matching state) and the seed pool have fixed
 * sizes that the call cannot grow as sm_run does.  A batch that needs more
 * (items denser than those of the uneven workload, such as the stress
 * workload's largest) also returns SM_ERR_LIMIT, and its outputs are then
 * undefined; sm_run handles such batches.  Output capacity behaves
 * as in sm_run (SM_ERR_CAPACITY with the sizes needed). */
#define SM_NOALLOC_MAX_EVENTS 1024
#define SM_NOALLOC_MAX_VELO 262144
#define SM_NOALLOC_WORKGROUPS 128
#define SM_NOALLOC_SCRATCH_BYTES (128ull << 20) /* upper bound; the array takes less */
sm_status sm_run_noalloc(sm_ctx *ctx, const sm_batch *batch, sm_out *out, void *stream);

/* A launch shape of the batched form for one class of batches: the
 * persistent grid of the main seeding form and the hits per workgroup that
 * are staged in LDS (larger items read their hits from global memory).  The
 * paper sizes its blocks from measured occupancy (Sec. 5.3); here an
 * autotuner measures the shapes on the device and hands the best one per
 * batch class to sm_set_shapes. */
typedef struct {
  int32_t max_mean_item_hits; /* the class: batches whose mean (event, half) hit count */
  int32_t max_events;         /*   is at most this, with at most this many events */
  int32_t seed_wgs;           /* workgroups of the main seeding form, >= 2 */
  int32_t lds_hits;           /* 256..6144, a multiple of 256 */
} sm_shape;

/* Replaces the context's table of launch shapes (copied; n = 0 clears it).
 * Each batched call (sm_run, sm_submit, sm_profile) takes the first entry
 * whose class holds its batch; a batch with more events than every class of
 * its item size takes the entry of the smallest such item size with the
 * most events; else the built-in choice (sm_config's seed_wgs and lds_hits,
 * else four workgroups per CU and 1.5x the mean item size).  Per-workgroup scratch for the largest grid of the table is
 * allocated here: SM_ERR_OOM if it does not fit, SM_ERR_BUSY while a serving
 * slot is in use, SM_ERR_INVALID for an entry out of range.  Outputs do not
 * depend on the shape. */
sm_status sm_set_shapes(sm_ctx *ctx, const sm_shape *shapes, int32_t n);

/* The launch shape a batched call would use for this batch (host-side: reads
 * only batch->n_events and batch->n_hits).  max_mean_item_hits and
 * max_events are set to the class bounds of the table entry taken, or to 0
 * for the built-in choice. */
sm_status sm_launch_shape(const sm_ctx *ctx, const sm_batch *batch, sm_shape *shape);

/* Device bytes a batch with these totals needs in a serving slot (used for
 * admission by free memory). */
int64_t sm_batch_bytes(const sm_ctx *ctx, int32_t n_events, int64_t n_hits, int64_t n_velo);

sm_status sm_destroy(sm_ctx *ctx);
const char *sm_status_str(sm_status s);

#ifdef __cplusplus
}
#endif
#endif
