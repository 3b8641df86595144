// Device side of the Seeding + Matching library (gfx950, wave64).
//
// Kernels, in launch order for one batch:
//   k_seed<0, 1024>  workgroup 0 prepares the batch (counters, per-event
//              hand-off counts, the longest-first order of the (event, half)
//              items, the big-form cut) and releases the other workgroups;
//              then the big-item form: 1024-thread workgroups over the
//              largest items (separate k_prepare with input validation)
//   k_seed<0, 256, false> / <0, 256, true>  the main form, persistent: each
//              workgroup pulls items from the queue and runs XZ seeding (both
//              iterations), the clone vote and UV seeding of one detector
//              half of one event, hits staged in LDS; built without and with
//              the matching code, the one that does not fit the batch returns
//              at once; with it, the workgroup that completes an event's
//              second half matches it
//   k_match    Matching of every event after all seeding (when the batch is
//              matched outside seeding)
//   k_copy     per-event offsets (scans) and the seeds and long tracks from
//              the pools to the caller's CSR
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sm.h"

namespace smk {

constexpr int kNL = 12;
constexpr int kSeedWG = 256;        // threads of the seeding workgroup (4 waves)
constexpr int kCandLds = 256;       // x-z candidates whose vote records live in LDS
constexpr int kXtabLds = 1024;      // x hits of an item with an LDS clone-vote entry
constexpr int kSeedLds = 256;       // seeds per item ranked from LDS keys
constexpr int kMsLds = 384;         // seeds per event whose matching state lives in LDS
constexpr int kVflat = 256;         // VELO states per event for the flattened pair search
constexpr int kPvLds = 2048;        // flattened pairs whose VELO state is looked up in LDS
constexpr int kVsLds = 512;         // VELO states per event with LDS best-chi2 entries
constexpr int kSurvLds = 512;       // matching survivors kept in LDS
constexpr int kUtLds = 3 * kMsLds;  // UT hits per event staged in LDS (UT search), in the
                                    // six per-seed prefilter arrays of the matching state
constexpr int kPosBits = 21;        // item-relative hit positions < 2^21
constexpr int kPoolPerItem = 128;   // seed-pool slots of each item (more: the overflow area)
constexpr int kMaxItemHits = 1 << kPosBits;
constexpr int kHoughBins = 128;     // largest coarse t_y histogram
constexpr int kBigWG = 1024;        // threads of the big-item workgroup (16 wave64)
constexpr int kBigBucket = 12;      // items with >= 2^12 - 1 hits are big
constexpr unsigned kPrepSpin = 1u << 22;  // polls of the preparation flag before giving up
constexpr double kTieMm = 1e-6;     // closest-hit distances this close are a tie

// status flags (Counters::flags)
enum : unsigned {
  F_TRIP = 1u << 0,      // triplet scratch too small
  F_CAND = 1u << 1,      // candidate scratch too small
  F_TBL = 1u << 2,       // clone table scratch too small
  F_SST = 1u << 3,       // per-item seed staging too small
  F_POOL = 1u << 4,      // seed pool too small
  F_LPOOL = 1u << 5,     // long-track pool too small
  F_MS = 1u << 6,        // per-event matching scratch too small (seeds)
  F_VS = 1u << 7,        // per-event matching scratch too small (VELO)
  F_SURV = 1u << 8,      // matching survivor list too small
  F_OUT_SEED = 1u << 9,  // caller's seed buffer too small
  F_OUT_LONG = 1u << 10, // caller's long buffer too small
  F_LIMIT = 1u << 11,    // an item has >= 2^21 hits
  F_INVALID = 1u << 12,  // malformed offsets
  F_UNSORTED = 1u << 13, // hits not sorted in a zone
  F_COMBO = 1u << 14,    // UV combination scratch too small
};

struct Counters {
  unsigned seed_queue, match_queue;
  unsigned flags, fuse;           // fuse: matching inside the seeding kernel (else k_match)
  unsigned long long pool_top, lpool_top;
  unsigned need_trip, need_cand, need_tbl, need_sst;
  unsigned need_ms, need_vs, need_surv, need_combo;
  long long total_seeds, total_longs;
  unsigned big_queue, n_big;     // big-item queue: order positions [0, n_big)
  unsigned prep_ready;           // 1 + n_big once the batch is prepared (big form with
                                 // preparation); 0 again after the batch's last kernel
  unsigned stall;                // a wait for the preparation gave up (sticky until the
                                 // host clears the counters)
  unsigned need_big[8];          // needs of the big-item scratch, same order as need_trip..
};

// Everything a batch needs that changes from call to call; lives in device
// memory so a captured graph can be replayed for any batch.
struct Desc {
  sm_batch b;
  sm_seed *seeds;
  sm_long *longs;
  int32_t *seed_off;
  int32_t *long_off;
  long long seed_cap, long_cap;
  int n_events, n_items;
  int grid;   // workgroups of this batch's main seeding form (0: the context's)
  int fuse;   // 1: matching inside the seeding kernel; 0: in k_match (chosen by the host)
  // third x-z iteration: 0 none; 1 the first two iterations, which mark the
  // hits of their seeds with `serial`; 2 the third iteration on the cleaned
  // batch (b then holds the hits left)
  int pass;
  unsigned serial;
  // 1: the matching kernel writes each event's seeds and seed offset (its
  // first seed follows every earlier event's: their counts are known once
  // seeding is done) and the copy kernel only the long tracks and totals
  int mseeds, pad5;
};

// Parameters in the precision each kernel uses.
struct DevParams {
  float zf[kNL];
  double zd[kNL], tand[kNL], inv_tand[kNL];
  // per layer at its nominal z: u = z - z_ref, g(u) of eq. trackequation,
  // z tan(alpha) and 1/z (the UV search evaluates these for every hypothesis)
  double uz[kNL], gz[kNL], ztan[kNL], inv_z[kNL];
  double zref, d;
  float zreff, df;
  // XZ, FP32 search; index 2: the third iteration (iteration 0's layers, its
  // own momentum floor)
  float dx3f[3], alphaf[3];
  float invp_af, invp_bf, kappa_cf, t2_tol0f, t2_tol1f;
  // XZ, FP64 extension + fit
  double ext_tol, inv_sigma2, chi2x_max;
  int min_x_hits, min_uv_hits;
  // UV
  double uv_tol, y_max, chi2y_max;
  // Matching
  double zm[5], z_ymatch, z_state;
  double max_dx, max_dy, max_dtx, max_dty;
  double tolx_scale, tolx_a, tolx_b, toly_scale, toly_a, toly_b, tol_tx, tol_ty;
  double chi2m_max, polarity, invp_a, invp_b;
  float pre_dx, pre_dy, pre_dtx, pre_dty;  // FP32 prefilter, slightly wider
  float zmf[5], z_ymatchf, z_statef;
  // Hough-cluster UV variant
  int uv_mode, hough_bins, hough_best, hough_fine, hough_min;
  // scheduling: main-form workgroups and the item latency model (us, n = hits)
  int main_slots, big_slots;   // big_slots 0: no big-item form
  int match_mode;   // 0: automatic, 1: matching kernel, -1: matching inside the seeding kernel
  float lat_a, lat_b, big_speedup;
  double hough_lo[2], hough_hi[2];
  // final selection (Sec. 4.4): 0 lowest chi2 of seed and VELO state, 1 the
  // ghost network (weights as in sm_ghost_nn) and the clone rule
  int final_sel;
  double ghost_cut, clone_gap;
  double nn_mean[SM_NN_INPUTS], nn_scale[SM_NN_INPUTS];
  double nn_w1[SM_NN_HIDDEN][SM_NN_INPUTS], nn_b1[SM_NN_HIDDEN], nn_w2[SM_NN_HIDDEN], nn_b2;
  // UT hit search (Sec. 4.3): layer z and stereo tan, gamma_x constants, and
  // the windows of Table 2 by kind (0 loose, 1 tight) and layer
  int ut_mode, ut_min_hits;
  double ut_z[SM_N_UT], ut_tan[SM_N_UT], a_gamma, b_gamma;
  double ut_a[2][SM_N_UT], ut_b[2][SM_N_UT], ut_lo[2][SM_N_UT], ut_hi[2][SM_N_UT];
};

// An x-z candidate (Sec. 3.2) in per-workgroup scratch.
struct Cand {
  double a, b, c, chi2;
  unsigned long long score;  // bits of the non-negative FP64 score
  unsigned long long key;    // (iteration, T1, T3, T2 positions)
  int32_t pos[6];            // x-layer hits (item-relative), -1 if none
  int32_t n, it;
};

struct SeedStage {
  sm_seed s;
  unsigned long long key;
};

// Per-seed state for Matching (Sec. 4.1).
struct MState {
  double xs, txs, y_m, ty, x0s;
  float xsf, txsf, y_mf, tyf;
};

struct Surv {
  int v, s;
  double chi2;
};

// One (track, initial stereo hit) combination of the UV search.
struct Combo {
  double chi2, y0, ty;
  int c, n, tb, pad;
  int pos[6];
};

// One position of the longest-first item order: the item and its zone
// offsets in the batch, read by the workgroup that takes the position in one
// round trip.
struct ItemRec {
  int item;
  int zabs[kNL + 1];
  int pad[2];
};

// Library-owned scratch of one slot.
struct Scratch {
  unsigned long long *trip;  // [seed_wgs][trip_cap]
  Cand *cand;                // [seed_wgs][cand_cap]
  unsigned long long *tbl;   // [seed_wgs][tbl_cap]
  SeedStage *sst;            // [seed_wgs][sst_cap]
  Combo *combo;              // [seed_wgs][combo_cap]
  unsigned long long *cscore, *bestchi;  // [seed_wgs][cand_cap], items with many candidates
  int *cinfo, *bestn, *bestidx;          // [seed_wgs][cand_cap]
  int trip_cap, cand_cap, tbl_cap, sst_cap, combo_cap, pad2;
  ItemRec *item_rec;                       // [items_cap]
  int *item_cnt, *item_base;               // [items_cap]
  int *ev_lcnt, *ev_lbase, *ev_done;       // [events_cap]
  sm_seed *pool;              // kPoolPerItem slots per item of the batch, then the
                              // overflow area from pool_static (filled by pool_top)
  long long pool_static;
  sm_long *lpool;
  long long pool_cap, lpool_cap;
  MState *ms;                 // [seed_wgs][ms_cap]
  float *mf;                  // [seed_wgs][6 * ms_cap], events with many seeds
  unsigned long long *best_s; // [seed_wgs][ms_cap]
  unsigned long long *best_v; // [seed_wgs][vs_cap]
  Surv *surv;                 // [seed_wgs][2 * surv_cap]
  int ms_cap, vs_cap, surv_cap, pad;
  Counters *cnt;
  unsigned *need;             // 8 overflow needs of this scratch (trip, cand, tbl, sst,
                              // ms, vs, surv, combo), inside *cnt
  uint32_t *used;             // third iteration: per hit of the batch, the serial of the
                              // last batch whose first two iterations used it
  int *item_cnt3, *item_base3;  // third iteration: its seeds per item, in pool3 (read by
  sm_seed *pool3;               // Matching and the copy beside the first two's)
};

// The third x-z iteration's batch-sized arrays: the cleaned batch, and its
// seeds, which Matching and the copy read beside the first two iterations'.
struct Third {
  int *zcnt;                  // [zones] hits left per zone
  int32_t *zone_off;          // [zones + 1] the cleaned batch's zone offsets
  float *hx, *hz;             // [hits] the hits left, zone by zone, x order kept
  int32_t *hid;
  int *item_cnt, *item_base;  // [items] third-iteration seeds per item, in pool
  sm_seed *pool;
  Counters *cnt;              // the third pass's counters
};

// Per-slot kernel context in device memory: kernels read scratch pointers and
// parameters through one pointer, so no argument has to stay in registers.
// A slot's links between its pinned host memory and the batched sequence:
// the preparing launch gets the batch descriptor in pinned host memory as
// its D and writes the device copy that every later launch reads; the copy
// kernel's workgroup that writes the totals also writes the counters back to
// pinned host memory.  Null pointers: the host moves these itself.
struct Link {
  Desc *desc;             // device descriptor written by the preparing launch
  Counters *hcnt;         // pinned host copy of the counters
  const Counters *cnt3;   // third iteration's counters (device), when on
  Counters *hcnt3;        // their pinned host copy
};

struct KCtx {
  Scratch S;   // main form: per-workgroup arrays for seed_wgs workgroups
  Scratch SB;  // big-item form: own per-workgroup arrays, shared pools and counters
  DevParams P;
  Third T;     // third iteration (null pointers when off)
  Link L;
};

}  // namespace smk

// Dynamic LDS bytes of k_seed for a given LDS hit capacity.
// dynamic LDS of a seeding form; sel: the matching variant it carries (bit 0
// the ghost network, bit 1 the UT search, whose hits are staged after the
// matching state)
size_t smk_seed_lds_bytes(int lds_hits, int sel = 0);
size_t smk_seed_big_lds_bytes(int lds_hits, int sel = 0);

extern "C" {
// Launchers (sm_device.hip); each returns the hipError_t of its launch.
int smk_launch_prepare(const smk::Desc *d, const smk::KCtx *k, int plain, hipStream_t st);
// sel: the matching variant (bit 0: the network form of the final selection,
// final_sel 1; bit 1: the UT search, ut_mode 1), one instantiation each
int smk_launch_seed(const smk::Desc *d, const smk::KCtx *k, int item_begin, int item_count,
                    int use_queue, int grid, int lds_hits, int plain, int uv_mode, int sel,
                    hipStream_t st);
// the main form without the matching code, for batches matched by k_match
int smk_launch_seed_nomatch(const smk::Desc *d, const smk::KCtx *k, int grid, int lds_hits,
                            hipStream_t st);
int smk_launch_seed_big(const smk::Desc *d, const smk::KCtx *k, int grid, int lds_hits, int prep,
                        int sel, hipStream_t st);
int smk_launch_match(const smk::Desc *d, const smk::KCtx *k, int grid, int sel, hipStream_t st);
int smk_seed_big_lds_limit(int bytes);
int smk_seed_lds_limit(int bytes);   // dynamic LDS allowed to the main seeding forms
int smk_seed_big_static_lds();   // static LDS of the big form (its dynamic LDS comes on top)
int smk_launch_copy(const smk::Desc *d, const smk::KCtx *k, int grid, hipStream_t st);
int smk_launch_validate(const smk::Desc *d, const smk::KCtx *k, int grid, hipStream_t st);
int smk_launch_plain_totals(const smk::Desc *d, const smk::KCtx *k, hipStream_t st);
int smk_launch_zero(void *p, int n_words, hipStream_t st);   // clears n_words 32-bit words
// the third iteration's clean-up: the hits the first two iterations left, as
// a batch of their own (three launches: counts per zone, offsets, copy)
int smk_launch_clean(const smk::Desc *d, const smk::KCtx *k, int grid, hipStream_t st);
}
