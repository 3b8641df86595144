// Host side of the C-ABI declared in include/sm.h: contexts, serving slots,
// scratch sizing and growth, the captured graph of the batched form and the
// per-event launch loop of the plain form.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <cstdint>
#include <vector>

#include "sm.h"
#include "sm_device.h"


namespace {

using smk::Counters;
using smk::Desc;
using smk::DevParams;
using smk::Scratch;

// Per-workgroup scratch of a slot.  Grown (doubled past the need) when a
// batch reports that one of them was too small; the batch is then re-run.
struct Caps {
  int trip = 8192, cand = 2048, tbl = 8192, sst = 1024, combo = 2048;
  int ms = 1024, vs = 1024, surv = 2048;
  int items = 0, events = 0;
  long long pool = 0, lpool = 0;
  long long hits = 0, pool3 = 0;   // third iteration: the cleaned batch, its pool's overflow
};

struct Slot {
  hipStream_t stream = nullptr;
  Desc *d_desc = nullptr;
  Desc *h_desc = nullptr;     // pinned
  smk::KCtx *d_kctx = nullptr;  // scratch pointers + parameters, device copy
  Counters *h_cnt = nullptr;  // pinned
  // third iteration: its pass's descriptor (the cleaned batch), context and
  // counters
  Desc *d_desc3 = nullptr;
  Desc *h_desc3 = nullptr;    // pinned
  smk::KCtx *d_kctx3 = nullptr;
  Counters *h_cnt3 = nullptr; // pinned
  smk::Third T{};
  Scratch S{};
  Scratch SB{};     // big-item form
  Caps caps;
  Caps caps_big;
  // captured batched sequence, one per LDS hit capacity used so far; kernel
  // arguments are the slot's fixed descriptor and context pointers, so a
  // graph stays valid when scratch is reallocated
  struct Captured {
    int lds_hits, grid, fuse;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<Captured> graphs;
  int lds_hits = 2048;  // LDS hit capacity of the seeding workgroup for this batch
  int grid = 0;         // workgroups of the main seeding form for this batch
  int fuse = 0;         // this batch is matched inside the seeding kernel
  hipEvent_t done = nullptr;
  // serving state
  bool busy = false;
  int64_t ticket = -1;
  sm_batch batch{};
  sm_out *out = nullptr;
  int tries = 0;
  std::vector<void *> allocs;
};

}  // namespace

struct sm_ctx {
  int device = 0;
  unsigned serial = 0;   // batches run (the third iteration's hit marks)
  sm_geometry g{};
  sm_params p{};
  sm_config cfg{};
  DevParams dp{};
  int seed_wgs = 0;   // workgroups with per-workgroup scratch: the largest grid in use
  int base_wgs = 0;   // grid of the built-in launch shape
  std::vector<sm_shape> shapes;   // launch shapes by batch class (sm_set_shapes)
  size_t lds_limit = 65536;       // dynamic LDS the main seeding forms may take
  int big_wgs = 0, lds_big = 0;  // big-item form: workgroups (one per CU) and LDS hits
  std::vector<Slot> slots;  // slots[0]: blocking calls; 1..: serving
  int64_t next_ticket = 1;
  std::mutex mu;
  int64_t bytes = 0;
  // allocation-free form: pinned host copies of its kernel context (scratch
  // pointers into the device's static array), descriptor and counters
  smk::KCtx *na_kctx = nullptr;
  Desc *na_desc = nullptr;
  Counters *na_cnt = nullptr;
};

namespace {

sm_status hip_status(hipError_t e) { return e == hipSuccess ? SM_OK : SM_ERR_DEVICE; }

DevParams make_params(const sm_geometry &g, const sm_params &p) {
  DevParams d{};
  for (int l = 0; l < smk::kNL; ++l) {
    d.zf[l] = (float)g.z[l];
    d.zd[l] = g.z[l];
    d.tand[l] = g.tan_stereo[l];
    d.inv_tand[l] = g.tan_stereo[l] != 0.0 ? 1.0 / g.tan_stereo[l] : 0.0;
    const double u = g.z[l] - g.z_ref;
    d.uz[l] = u;
    d.gz[l] = u * u * (1.0 + p.d_ratio * u);
    d.ztan[l] = g.z[l] * g.tan_stereo[l];
    d.inv_z[l] = 1.0 / g.z[l];
  }
  d.zref = g.z_ref;
  d.d = p.d_ratio;
  d.zreff = (float)g.z_ref;
  d.df = (float)p.d_ratio;
  // per-iteration window constants: eq. tolHp and eq. alphacorr at the
  // nominal z of the iteration's T1 and T3 layers; index 2: the third
  // iteration (iteration 0's layers, momentum floor p_min3)
  const int l1[3] = {0, 3, 0}, l3[3] = {8, 11, 8};
  for (int it = 0; it < 3; ++it) {
    const double z1 = g.z[l1[it]], z3 = g.z[l3[it]];
    const double a = p.invp_a, b = p.invp_b;
    const double pm = it == 2 ? p.p_min3 : p.p_min;
    const double disc = a * a + 4.0 * b / pm;
    const double x0max = disc >= 0.0 && pm > 0.0 ? (-a + std::sqrt(disc)) / (2.0 * b) : 0.0;
    d.dx3f[it] = (float)((z3 - z1) / z1 * x0max);
    d.alphaf[it] = (float)(p.alpha0 / ((z1 / (z3 - z1)) * (pm - p.alpha1)));
  }
  d.invp_af = (float)p.invp_a;
  d.invp_bf = (float)p.invp_b;
  d.kappa_cf = (float)p.kappa_c;
  d.t2_tol0f = (float)p.t2_tol0;
  d.t2_tol1f = (float)p.t2_tol1;
  d.ext_tol = p.ext_tol;
  d.inv_sigma2 = 1.0 / (p.sigma_x * p.sigma_x);
  d.chi2x_max = p.chi2x_max;
  d.min_x_hits = p.min_x_hits;
  d.min_uv_hits = p.min_uv_hits;
  d.uv_tol = p.uv_tol;
  d.y_max = p.y_max;
  d.chi2y_max = p.chi2y_max;
  for (int i = 0; i < 5; ++i) {
    d.zm[i] = p.zm[i];
    d.zmf[i] = (float)p.zm[i];
  }
  d.z_ymatch = p.z_ymatch;
  d.z_state = p.z_state;
  d.z_ymatchf = (float)p.z_ymatch;
  d.z_statef = (float)p.z_state;
  d.max_dx = p.max_dx; d.max_dy = p.max_dy; d.max_dtx = p.max_dtx; d.max_dty = p.max_dty;
  d.tolx_scale = p.tolx_scale; d.tolx_a = p.tolx_a; d.tolx_b = p.tolx_b;
  d.toly_scale = p.toly_scale; d.toly_a = p.toly_a; d.toly_b = p.toly_b;
  d.tol_tx = p.tol_tx; d.tol_ty = p.tol_ty;
  d.chi2m_max = p.chi2m_max;
  d.polarity = p.polarity;
  // Hough-cluster UV: t_y range of each half from the lowest nominal stereo z
  d.uv_mode = p.uv_mode;
  d.hough_bins = p.hough_bins;
  d.hough_best = p.hough_best;
  d.hough_fine = p.hough_fine;
  d.hough_min = p.hough_min;
  d.final_sel = p.final_sel;
  d.ghost_cut = p.ghost_cut;
  d.clone_gap = p.clone_gap;
  for (int i = 0; i < SM_NN_INPUTS; ++i) {
    d.nn_mean[i] = p.ghost_nn.mean[i];
    d.nn_scale[i] = p.ghost_nn.scale[i];
  }
  for (int j = 0; j < SM_NN_HIDDEN; ++j) {
    for (int i = 0; i < SM_NN_INPUTS; ++i) d.nn_w1[j][i] = p.ghost_nn.w1[j][i];
    d.nn_b1[j] = p.ghost_nn.b1[j];
    d.nn_w2[j] = p.ghost_nn.w2[j];
  }
  d.nn_b2 = p.ghost_nn.b2;
  d.ut_mode = p.ut_mode;
  d.ut_min_hits = p.ut_min_hits;
  d.a_gamma = p.a_gamma;
  d.b_gamma = p.b_gamma;
  for (int i = 0; i < SM_N_UT; ++i) {
    d.ut_z[i] = g.ut_z[i];
    d.ut_tan[i] = g.ut_tan[i];
    d.ut_a[0][i] = p.ut_loose_a[i]; d.ut_b[0][i] = p.ut_loose_b[i];
    d.ut_lo[0][i] = p.ut_loose_lo[i]; d.ut_hi[0][i] = p.ut_loose_hi[i];
    d.ut_a[1][i] = p.ut_tight_a[i]; d.ut_b[1][i] = p.ut_tight_b[i];
    d.ut_lo[1][i] = p.ut_tight_lo[i]; d.ut_hi[1][i] = p.ut_tight_hi[i];
  }
  double zmin = 1e300;
  for (int l = 0; l < smk::kNL; ++l)
    if (g.tan_stereo[l] != 0.0) zmin = std::min(zmin, g.z[l]);
  d.hough_lo[0] = 0.0;
  d.hough_hi[0] = p.y_max / zmin;
  d.hough_lo[1] = -p.y_max / zmin;
  d.hough_hi[1] = 0.0;
  d.invp_a = p.invp_a;
  d.invp_b = p.invp_b;
  // FP32 prefilter of the matching preselection: wider than the FP64 cut by
  // more than the FP32 rounding of the quantities, so it never rejects a pair
  // the FP64 test would keep.
  d.pre_dx = (float)(p.max_dx * (1.0 + 1e-4) + 0.05);
  d.pre_dy = (float)(p.max_dy * (1.0 + 1e-4) + 0.1);
  d.pre_dtx = (float)(p.max_dtx * (1.0 + 1e-4) + 1e-4);
  d.pre_dty = (float)(p.max_dty * (1.0 + 1e-4) + 1e-4);
  return d;
}

void free_slot_scratch(Slot &s) {
  for (void *p : s.allocs) (void)hipFree(p);
  s.allocs.clear();
}

void destroy_graphs(Slot &s) {
  for (Slot::Captured &g : s.graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  s.graphs.clear();
}

template <class T>
sm_status dalloc(Slot &s, T **p, size_t n, int64_t &bytes) {
  const size_t b = std::max<size_t>(n, 1) * sizeof(T);
  void *q = nullptr;
  if (hipMalloc(&q, b) != hipSuccess) {
    hipGetLastError();
    *p = nullptr;
    return SM_ERR_OOM;
  }
  s.allocs.push_back(q);
  bytes += (int64_t)b;
  *p = (T *)q;
  return SM_OK;
}

// (Re)allocate all scratch of a slot for its current caps.
sm_status alloc_slot(sm_ctx *c, Slot &s) {
  destroy_graphs(s);   // no graph outlives the scratch it was captured with
  free_slot_scratch(s);
  int64_t bytes = 0;
  const size_t G = (size_t)c->seed_wgs;
  const Caps &k = s.caps;
  Scratch &S = s.S;
  memset(&S, 0, sizeof(S));
  sm_status st = SM_OK;
#define A(ptr, n)                                   \
  if ((st = dalloc(s, &(ptr), (n), bytes)) != SM_OK) \
    return st;
  A(S.trip, G * k.trip);
  A(S.cand, G * k.cand);
  A(S.tbl, G * k.tbl);
  A(S.sst, G * k.sst);
  A(S.combo, G * k.combo);
  A(S.cscore, G * k.cand);
  A(S.cinfo, G * k.cand);
  A(S.bestn, G * k.cand);
  A(S.bestchi, G * k.cand);
  A(S.bestidx, G * k.cand);
  A(S.item_rec, k.items);
  A(S.item_cnt, k.items);
  A(S.item_base, k.items);
  A(S.ev_lcnt, k.events);
  A(S.ev_lbase, k.events);
  A(S.ev_done, k.events);
  S.pool_static = (long long)k.items * smk::kPoolPerItem;
  A(S.pool, (size_t)(S.pool_static + k.pool));
  A(S.lpool, (size_t)k.lpool);
  A(S.ms, G * k.ms);
  A(S.mf, G * 6 * (size_t)k.ms);
  A(S.best_s, G * k.ms);
  A(S.best_v, G * k.vs);
  A(S.surv, G * 2 * (size_t)k.surv);
  A(S.cnt, 1);
  // the preparation flag and the stall flag start clear (the kernels keep
  // the first at 0 between batches)
  if (hipMemset(S.cnt, 0, sizeof(Counters)) != hipSuccess) return SM_ERR_DEVICE;
  // big-item form: its own per-workgroup arrays, everything else shared
  Scratch &B = s.SB;
  B = S;
  const size_t GB = (size_t)std::max(c->big_wgs, 1);
  const Caps &kb = s.caps_big;
  A(B.trip, GB * kb.trip);
  A(B.cand, GB * kb.cand);
  A(B.tbl, GB * kb.tbl);
  A(B.sst, GB * kb.sst);
  A(B.combo, GB * kb.combo);
  A(B.cscore, GB * kb.cand);
  A(B.cinfo, GB * kb.cand);
  A(B.bestn, GB * kb.cand);
  A(B.bestchi, GB * kb.cand);
  A(B.bestidx, GB * kb.cand);
  A(B.ms, GB * kb.ms);
  A(B.mf, GB * 6 * (size_t)kb.ms);
  A(B.best_s, GB * kb.ms);
  A(B.best_v, GB * kb.vs);
  A(B.surv, GB * 2 * (size_t)kb.surv);
#undef A
  S.trip_cap = k.trip; S.cand_cap = k.cand; S.tbl_cap = k.tbl; S.sst_cap = k.sst;
  S.combo_cap = k.combo;
  S.pool_cap = S.pool_static + k.pool; S.lpool_cap = k.lpool;
  S.ms_cap = k.ms; S.vs_cap = k.vs; S.surv_cap = k.surv;
  B.trip_cap = kb.trip; B.cand_cap = kb.cand; B.tbl_cap = kb.tbl; B.sst_cap = kb.sst;
  B.combo_cap = kb.combo;
  B.ms_cap = kb.ms; B.vs_cap = kb.vs; B.surv_cap = kb.surv;
  B.item_rec = S.item_rec; B.item_cnt = S.item_cnt; B.item_base = S.item_base;
  B.ev_lcnt = S.ev_lcnt; B.ev_lbase = S.ev_lbase; B.ev_done = S.ev_done;
  B.pool = S.pool; B.pool_static = S.pool_static; B.lpool = S.lpool; B.pool_cap = S.pool_cap; B.lpool_cap = S.lpool_cap;
  B.cnt = S.cnt;
  // device addresses inside the counters (address arithmetic only)
  S.need = reinterpret_cast<unsigned *>(reinterpret_cast<char *>(S.cnt) + offsetof(Counters, need_trip));
  B.need = reinterpret_cast<unsigned *>(reinterpret_cast<char *>(S.cnt) + offsetof(Counters, need_big));
  // third iteration: the hit marks, the cleaned batch, its seeds' pool and
  // counters; its pass runs on a context whose pools, per-item counts and
  // counters are these (the per-workgroup scratch is the first pass's)
  smk::Third &T = s.T;
  memset(&T, 0, sizeof(T));
  smk::KCtx k3{};
  if (c->p.third_iter == 1) {
    const size_t zones = (size_t)k.events * 24 + 1;
    const long long pool3_static = (long long)k.items * smk::kPoolPerItem;
#define A3(ptr, n)                                  \
  if ((st = dalloc(s, &(ptr), (n), bytes)) != SM_OK) \
    return st;
    A3(S.used, (size_t)k.hits);
    A3(T.zcnt, zones);
    A3(T.zone_off, zones);
    A3(T.hx, (size_t)k.hits);
    A3(T.hz, (size_t)k.hits);
    A3(T.hid, (size_t)k.hits);
    A3(T.item_cnt, k.items);
    A3(T.item_base, k.items);
    A3(T.pool, (size_t)(pool3_static + k.pool3));
    A3(T.cnt, 1);
#undef A3
    // serials start at 1: no hit is marked by a batch yet
    if (hipMemset(S.used, 0, sizeof(uint32_t) * (size_t)k.hits) != hipSuccess ||
        hipMemset(T.cnt, 0, sizeof(Counters)) != hipSuccess)
      return SM_ERR_DEVICE;
    S.item_cnt3 = T.item_cnt; S.item_base3 = T.item_base; S.pool3 = T.pool;
    B.used = S.used; B.item_cnt3 = T.item_cnt; B.item_base3 = T.item_base; B.pool3 = T.pool;
    k3.S = S;
    k3.SB = B;
    for (Scratch *x : {&k3.S, &k3.SB}) {
      x->item_cnt = T.item_cnt;
      x->item_base = T.item_base;
      x->pool = T.pool;
      x->pool_static = pool3_static;
      x->pool_cap = pool3_static + k.pool3;
      x->cnt = T.cnt;
    }
    k3.S.need = reinterpret_cast<unsigned *>(reinterpret_cast<char *>(T.cnt) + offsetof(Counters, need_trip));
    k3.SB.need = reinterpret_cast<unsigned *>(reinterpret_cast<char *>(T.cnt) + offsetof(Counters, need_big));
    k3.P = c->dp;
    k3.T = T;
  }
  c->bytes += bytes;
  smk::KCtx kc;
  kc.S = S;
  kc.SB = B;
  kc.P = c->dp;
  kc.T = T;
  // the preparing launch writes the device descriptor, the copy kernel the
  // counters in pinned memory (both passes' with the third iteration)
  const bool third = c->p.third_iter == 1;
  kc.L = smk::Link{s.d_desc, s.h_cnt, third ? T.cnt : nullptr, third ? s.h_cnt3 : nullptr};
  k3.L = smk::Link{s.d_desc3, nullptr, nullptr, nullptr};
  if (hipMemcpy(s.d_kctx, &kc, sizeof(kc), hipMemcpyHostToDevice) != hipSuccess) return SM_ERR_DEVICE;
  if (c->p.third_iter == 1 &&
      hipMemcpy(s.d_kctx3, &k3, sizeof(k3), hipMemcpyHostToDevice) != hipSuccess)
    return SM_ERR_DEVICE;
  if (c->cfg.mem_budget > 0 && bytes > c->cfg.mem_budget) return SM_ERR_OOM;
  return SM_OK;
}

// Runs of one batch (the first and the re-runs after scratch growth) before
// a call gives up with SM_ERR_CAPACITY.
constexpr int kMaxTries = 8;

// Batches of up to this many events have their seeds written by the matching
// kernel (and only their long tracks by the copy kernel).
constexpr int kMatchSeedsEvents = 4096;

bool grow(int &cap, unsigned need) {
  if (need == 0) need = (unsigned)cap + 1;
  long long n = cap;
  while (n < (long long)need) n *= 2;
  n = std::min<long long>(n * 2, (long long)smk::kMaxItemHits * 4);
  if (n <= cap) return false;
  cap = (int)n;
  return true;
}

// LDS hit capacity of the seeding workgroup: the configured one, else 1.5x
// the mean (event, half) size rounded up to 256, 1024..4096 (items above it
// read their hits from global memory).
int lds_hits_for(const sm_ctx *c, const sm_batch &b) {
  int h = std::min(c->cfg.lds_hits, 4096);
  if (h <= 0) {
    const double mean = b.n_events > 0 ? (double)b.n_hits / (2.0 * b.n_events) : 0.0;
    h = 256 * (int)std::ceil(1.5 * mean / 256.0);
    h = std::max(1024, std::min(h, 4096));
  }
  return h;
}

// The launch shape of a batch: the first table entry whose class holds it,
// else the built-in one.
sm_shape choose_shape(const sm_ctx *c, const sm_batch &b) {
  const double mean = b.n_events > 0 ? (double)b.n_hits / (2.0 * b.n_events) : 0.0;
  // a batch beyond every class of its item size runs in the largest class
  // of the smallest item size that holds it (the same regime: many rounds of
  // items per workgroup)
  const sm_shape *far = nullptr;
  for (const sm_shape &e : c->shapes) {
    if (mean > (double)e.max_mean_item_hits) continue;
    if (b.n_events <= e.max_events) return e;
    if (!far || e.max_mean_item_hits < far->max_mean_item_hits ||
        (e.max_mean_item_hits == far->max_mean_item_hits && e.max_events > far->max_events))
      far = &e;
  }
  if (far) return *far;
  sm_shape d{};
  d.seed_wgs = c->base_wgs;
  d.lds_hits = lds_hits_for(c, b);
  return d;
}

// Workgroups of the matching kernel for a seeding grid: the grid, or the
// configured count (it uses the seeding workgroups' matching scratch).
int match_grid(const sm_ctx *c, int grid) {
  return c->cfg.match_wgs > 0 ? std::min(c->cfg.match_wgs, grid) : grid;
}

// The matching variant of the kernels: bit 0 the network form of the final
// selection, bit 1 the UT search; each is an instantiation of its own.
int sel_of(const sm_ctx *c) {
  return (c->p.final_sel == 1 ? 1 : 0) | (c->p.ut_mode == 1 ? 2 : 0);
}

// Where a batch is matched: inside the seeding kernel, by the workgroup that
// completes an event, when the main form runs more than four rounds of items
// (matching then overlaps the seeding tail) or when the batch's mean item
// size marks it as one with big items (matching overlaps the big items'
// tail); otherwise in k_match after all seeding, which needs no per-item
// release and per-event acquire.  sm_config.match_wgs can force either.
// Only the chosen main-form instantiation is launched.
int fuse_for(const sm_ctx *c, const sm_batch &b, int grid) {
  if (c->dp.match_mode != 0) return c->dp.match_mode < 0 ? 1 : 0;
  const long long items = 2LL * b.n_events;
  if (items > 4LL * std::max(grid, 1)) return 1;
  return b.n_hits > 2048LL * b.n_events ? 1 : 0;
}

// Make the slot's batch-sized buffers large enough for this batch.
sm_status fit_batch(sm_ctx *c, Slot &s, const sm_batch &b) {
  Caps &k = s.caps;
  bool re = false;
  const int items = 2 * b.n_events;
  if (items > k.items) { k.items = std::max(items, 2 * k.items); re = true; }
  if (b.n_events > k.events) { k.events = std::max(b.n_events, 2 * k.events); re = true; }
  const long long pool = b.n_hits / 8 + 1024;   // overflow area of the seed pool
  if (pool > k.pool) { k.pool = std::max(pool, 2 * k.pool); re = true; }
  const long long lpool = b.n_velo + 1024;
  if (lpool > k.lpool) { k.lpool = std::max(lpool, 2 * k.lpool); re = true; }
  if (c->p.third_iter == 1) {
    if (b.n_hits > k.hits) { k.hits = std::max<long long>(b.n_hits, 2 * k.hits); re = true; }
    if (pool > k.pool3) { k.pool3 = std::max(pool, 2 * k.pool3); re = true; }
  }
  const sm_shape sh = choose_shape(c, b);
  s.lds_hits = sh.lds_hits;
  s.grid = sh.seed_wgs;
  // with the third iteration, matching waits for all three iterations' seeds
  s.fuse = c->p.third_iter == 1 ? 0 : fuse_for(c, b, s.grid);
  if (!re && !s.allocs.empty()) return SM_OK;
  return alloc_slot(c, s);
}

sm_status check_batch(const sm_ctx *c, const sm_batch *b, const sm_out *o) {
  if (!b || !o) return SM_ERR_INVALID;
  // the UT search needs the batch's UT hits (an event may have none)
  if (c->p.ut_mode == 1 && b->n_events > 0 && !b->ut_off) return SM_ERR_INVALID;
  if (b->n_ut < 0 || (b->n_ut > 0 && (!b->ut_x || !b->ut_id)) ||
      (b->n_events > 0 && b->ut_off == nullptr && b->n_ut > 0))
    return SM_ERR_INVALID;
  if (b->n_events < 0 || b->n_hits < 0 || b->n_velo < 0) return SM_ERR_INVALID;
  if (o->seed_cap < 0 || o->long_cap < 0) return SM_ERR_INVALID;
  if (!o->seed_off || !o->long_off) return SM_ERR_INVALID;
  if (b->n_events > 0 && (!b->zone_off || !b->velo_off)) return SM_ERR_INVALID;
  if (b->n_hits > 0 && (!b->hit_x || !b->hit_z || !b->hit_id)) return SM_ERR_INVALID;
  if (b->n_velo > 0 && (!b->velo_x || !b->velo_y || !b->velo_z || !b->velo_tx || !b->velo_ty ||
                        !b->velo_id))
    return SM_ERR_INVALID;
  if ((o->seed_cap > 0 && !o->seeds) || (o->long_cap > 0 && !o->longs)) return SM_ERR_INVALID;
  if (b->n_events > (1 << 26)) return SM_ERR_LIMIT;
  return SM_OK;
}

void fill_desc(Desc &d, const sm_batch &b, const sm_out &o, int grid, int fuse, int pass = 0,
               unsigned serial = 0) {
  d.b = b;
  d.seeds = o.seeds;
  d.longs = o.longs;
  d.seed_off = o.seed_off;
  d.long_off = o.long_off;
  d.seed_cap = o.seed_cap;
  d.long_cap = o.long_cap;
  d.n_events = b.n_events;
  d.n_items = 2 * b.n_events;
  d.grid = grid;
  d.fuse = fuse;
  d.pass = pass;
  d.serial = serial;
  d.mseeds = 0;
}

// The slot's descriptors for one batch: the batch itself and, with the third
// iteration, its pass over the cleaned batch (the hits left after the first
// two iterations, built on the device by the clean-up launches).
void fill_descs(sm_ctx *c, Slot &s, const sm_batch &b, const sm_out &o) {
  const bool third = c->p.third_iter == 1;
  unsigned serial = 0;
  if (third) {
    serial = ++c->serial;
    if (serial == 0) serial = ++c->serial;   // 0 is the marks' initial value
  }
  fill_desc(*s.h_desc, b, o, s.grid, s.fuse, third ? 1 : 0, serial);
  // the matching kernel writes the seeds itself: each event adds up the
  // earlier events' seed counts, so only for batches of a few thousand
  s.h_desc->mseeds = !s.fuse && b.n_events <= kMatchSeedsEvents ? 1 : 0;
  if (third) {
    Desc &d3 = *s.h_desc3;
    d3 = *s.h_desc;
    d3.b.zone_off = s.T.zone_off;
    d3.b.hit_x = s.T.hx;
    d3.b.hit_z = s.T.hz;
    d3.b.hit_id = s.T.hid;
    d3.pass = 2;
    d3.fuse = 0;
    d3.mseeds = 0;
  }
}

// The third iteration's launches: its descriptor, the clean-up (hits left
// per zone, their offsets, their copy) and its seeding pass (preparation and
// big form, then the main form), on its own context (pools, counts,
// counters).
int enqueue_third(sm_ctx *c, Slot &s, hipStream_t q) {
  int e = smk_launch_clean(s.d_desc, s.d_kctx, 1024, q);
  // its preparing launch reads the pass's descriptor from pinned memory and
  // writes the device copy
  if (!e) e = smk_launch_seed_big(s.h_desc3, s.d_kctx3, c->big_wgs, c->lds_big, 1, sel_of(c), q);
  if (!e) e = smk_launch_seed_nomatch(s.d_desc3, s.d_kctx3, s.grid, s.lds_hits, q);
  return e;
}

// The head of the batched sequence: the batch's preparation and the
// big-item form in one launch (its workgroup 0 prepares), or, with input
// validation or the Hough variant, k_prepare, k_validate and the big form.
// The preparing launch reads the descriptor at src: the slot's pinned copy
// (it then writes the device copy for the launches after it) or the device
// copy itself.
int enqueue_prepare_big(sm_ctx *c, Slot &s, hipStream_t q, const Desc *src) {
  const smk::KCtx *S = s.d_kctx;
  const Desc *d = s.d_desc;
  if (c->p.uv_mode == 0 && !c->cfg.validate)
    return smk_launch_seed_big(src, S, c->big_wgs, c->lds_big, 1, sel_of(c), q);
  int e = smk_launch_prepare(src, S, 0, q);
  if (!e && c->cfg.validate) e = smk_launch_validate(d, S, 1024, q);
  if (!e && c->p.uv_mode == 0)
    e = smk_launch_seed_big(d, S, c->big_wgs, c->lds_big, 0, sel_of(c), q);
  return e;
}

// The batched sequence, replayed from a captured graph: kernels only.  The
// preparing launch reads the batch descriptor from the slot's pinned copy
// when the graph runs (so one graph serves every batch of the slot) and
// writes its device copy; the copy kernel writes the counters back to pinned
// memory.
sm_status enqueue_batched(sm_ctx *c, Slot &s, hipStream_t st) {
  const smk::KCtx *S = s.d_kctx;
  const Desc *d = s.d_desc;
  auto seq = [&](hipStream_t q) -> hipError_t {
    int e = enqueue_prepare_big(c, s, q, s.h_desc);
    if (!e && !s.fuse) e = smk_launch_seed_nomatch(d, S, s.grid, s.lds_hits, q);
    if (!e && s.fuse)
      e = smk_launch_seed(d, S, 0, -1, 1, s.grid, s.lds_hits, 0, c->p.uv_mode, sel_of(c), q);
    if (!e && c->p.third_iter == 1) e = enqueue_third(c, s, q);
    if (!e && !s.fuse) e = smk_launch_match(d, S, match_grid(c, s.grid), sel_of(c), q);
    if (!e) e = smk_launch_copy(d, S, 1024, q);
    return (hipError_t)e;
  };
  for (const Slot::Captured &g : s.graphs)
    if (g.lds_hits == s.lds_hits && g.grid == s.grid && g.fuse == s.fuse)
      return hip_status(hipGraphLaunch(g.exec, st));
  hipStream_t cap;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return SM_ERR_DEVICE;
  Slot::Captured g{s.lds_hits, s.grid, s.fuse, nullptr, nullptr};
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    hipError_t e2 = seq(cap);
    e = hipStreamEndCapture(cap, &g.graph);
    if (e == hipSuccess && e2 != hipSuccess) e = e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess) {
    if (g.graph) (void)hipGraphDestroy(g.graph);
    return SM_ERR_DEVICE;
  }
  s.graphs.push_back(g);
  return hip_status(hipGraphLaunch(g.exec, st));
}

sm_status enqueue_plain(sm_ctx *c, Slot &s, int n_events, hipStream_t st) {
  const smk::KCtx *S = s.d_kctx;
  const Desc *d = s.d_desc;
  int e = smk_launch_prepare(d, S, 1, st);
  if (!e && c->cfg.validate) e = smk_launch_validate(d, S, 1024, st);
  for (int ev = 0; ev < n_events && !e; ++ev)
    e = smk_launch_seed(d, S, 2 * ev, 2, 0, 2, s.lds_hits, 1, c->p.uv_mode, sel_of(c), st);
  if (!e) e = smk_launch_plain_totals(d, S, st);
  return hip_status((hipError_t)e);
}

// The batched sequence as plain launches with an event after every kernel.
sm_status enqueue_timed(sm_ctx *c, Slot &s, hipStream_t q, hipEvent_t *ev) {
  const smk::KCtx *S = s.d_kctx;
  const Desc *d = s.d_desc;
  int e = hipEventRecord(ev[0], q);
  if (!e) e = enqueue_prepare_big(c, s, q, d);   // preparation and big form
  if (!e) e = hipEventRecord(ev[1], q);
  if (!e) e = hipEventRecord(ev[2], q);
  if (!e && !s.fuse) e = smk_launch_seed_nomatch(d, S, s.grid, s.lds_hits, q);
  if (!e && c->p.third_iter == 1) e = enqueue_third(c, s, q);   // timed with seeding
  if (!e) e = hipEventRecord(ev[3], q);
  if (!e && s.fuse)
    e = smk_launch_seed(d, S, 0, -1, 1, s.grid, s.lds_hits, 0, c->p.uv_mode, sel_of(c), q);
  if (!e) e = hipEventRecord(ev[4], q);
  if (!e && !s.fuse) e = smk_launch_match(d, S, match_grid(c, s.grid), sel_of(c), q);
  if (!e) e = hipEventRecord(ev[5], q);
  if (!e) e = smk_launch_copy(d, S, 1024, q);   // offset scans and copy
  if (!e) e = hipEventRecord(ev[6], q);
  return hip_status((hipError_t)e);
}

// After the counters came back: grow what overflowed (returns true to re-run)
// or map the flags to a status.
bool needs_rerun(sm_ctx *c, Slot &s, sm_status &st) {
  const Counters &k = *s.h_cnt;
  // the third iteration's pass has counters of its own
  static const Counters none{};
  const bool third = c->p.third_iter == 1;
  const Counters &k3 = third ? *s.h_cnt3 : none;
  st = SM_OK;
  const unsigned f = k.flags | k3.flags;
  if (k.stall || k3.stall) {
    // a wait for the batch's preparation gave up: clear the counters
    (void)hipMemset(s.S.cnt, 0, sizeof(Counters));
    if (third) (void)hipMemset(s.T.cnt, 0, sizeof(Counters));
    st = SM_ERR_DEVICE;
    return false;
  }
  if (f & smk::F_INVALID) { st = SM_ERR_INVALID; return false; }
  if (f & smk::F_UNSORTED) { st = SM_ERR_UNSORTED; return false; }
  if (f & smk::F_LIMIT) { st = SM_ERR_LIMIT; return false; }
  bool re = false;
  Caps &cp = s.caps;
  // each form's scratch grows to what its own items needed
  auto grow_caps = [&](Caps &q, const unsigned *n) {
    bool r = false;
    if ((f & smk::F_TRIP) && n[0] > (unsigned)q.trip) r |= grow(q.trip, n[0]);
    if ((f & smk::F_CAND) && n[1] > (unsigned)q.cand) r |= grow(q.cand, n[1]);
    if ((f & smk::F_TBL) && n[2] > (unsigned)q.tbl) r |= grow(q.tbl, n[2]);
    if ((f & smk::F_SST) && n[3] > (unsigned)q.sst) r |= grow(q.sst, n[3]);
    if ((f & smk::F_MS) && n[4] > (unsigned)q.ms) r |= grow(q.ms, n[4]);
    if ((f & smk::F_VS) && n[5] > (unsigned)q.vs) r |= grow(q.vs, n[5]);
    if ((f & smk::F_SURV) && n[6] > (unsigned)q.surv) r |= grow(q.surv, n[6]);
    if ((f & smk::F_COMBO) && n[7] > (unsigned)q.combo) r |= grow(q.combo, n[7]);
    return r;
  };
  re |= grow_caps(cp, &k.need_trip);
  re |= grow_caps(s.caps_big, k.need_big);
  if (third) {
    re |= grow_caps(cp, &k3.need_trip);
    re |= grow_caps(s.caps_big, k3.need_big);
  }
  // seed pool: pool_top is what the overflow area needed
  if (k.flags & smk::F_POOL) { cp.pool = std::max<long long>(2 * cp.pool, (long long)k.pool_top + 1024); re = true; }
  if (k3.flags & smk::F_POOL) { cp.pool3 = std::max<long long>(2 * cp.pool3, (long long)k3.pool_top + 1024); re = true; }
  // long-track pool: every VELO state's slot, then the overflow area
  if (f & smk::F_LPOOL) { cp.lpool = std::max<long long>(2 * cp.lpool, cp.lpool + (long long)k.lpool_top + 1024); re = true; }
  if (re) {
    if (alloc_slot(c, s) != SM_OK) { st = SM_ERR_OOM; return false; }
    return true;
  }
  if (f & (smk::F_OUT_SEED | smk::F_OUT_LONG)) st = SM_ERR_CAPACITY;
  return false;
}

sm_status run_blocking(sm_ctx *c, const sm_batch *b, sm_out *o, void *stream, bool plain,
                       sm_kernel_times *times = nullptr) {
  sm_status st = check_batch(c, b, o);
  if (st != SM_OK) return st;
  // the per-event form matches each event as soon as it is seeded; the third
  // iteration needs the batch's clean-up between seeding and matching
  if (plain && c->p.third_iter == 1) return SM_ERR_INVALID;
  std::lock_guard<std::mutex> lk(c->mu);
  if (hipSetDevice(c->device) != hipSuccess) return SM_ERR_DEVICE;
  Slot &s = c->slots[0];
  hipStream_t q = (hipStream_t)stream;
  for (int tries = 0; tries < kMaxTries; ++tries) {
    if ((st = fit_batch(c, s, *b)) != SM_OK) return st;
    fill_descs(c, s, *b, *o);
    // the batched graph reads the pinned descriptor and writes the pinned
    // counters from its kernels; the plain and timed sequences move them here
    const bool graph = !times && !plain;
    if (!graph &&
        hipMemcpyAsync(s.d_desc, s.h_desc, sizeof(Desc), hipMemcpyHostToDevice, q) != hipSuccess)
      return SM_ERR_DEVICE;
    hipEvent_t ev[7] = {};
    if (times) {
      for (auto &x : ev)
        if (hipEventCreate(&x) != hipSuccess) return SM_ERR_DEVICE;
      st = enqueue_timed(c, s, q, ev);
    } else {
      st = plain ? enqueue_plain(c, s, b->n_events, q) : enqueue_batched(c, s, q);
    }
    if (st == SM_OK && !graph &&
        hipMemcpyAsync(s.h_cnt, s.S.cnt, sizeof(Counters), hipMemcpyDeviceToHost, q) != hipSuccess)
      st = SM_ERR_DEVICE;
    if (st == SM_OK && !graph && c->p.third_iter == 1 &&
        hipMemcpyAsync(s.h_cnt3, s.T.cnt, sizeof(Counters), hipMemcpyDeviceToHost, q) != hipSuccess)
      st = SM_ERR_DEVICE;
    if (st == SM_OK && hipStreamSynchronize(q) != hipSuccess) st = SM_ERR_DEVICE;
    if (times) {
      if (st == SM_OK) {
        float *f = &times->prepare;   // prepare, seed_big, seed, seed_fused, match, copy
        for (int k = 0; k < 6; ++k) hipEventElapsedTime(&f[k], ev[k], ev[k + 1]);
        hipEventElapsedTime(&times->total, ev[0], ev[6]);
      }
      for (auto &x : ev) hipEventDestroy(x);
    }
    if (st != SM_OK) return st;
    o->n_seeds = s.h_cnt->total_seeds;
    o->n_longs = s.h_cnt->total_longs;
    if (!needs_rerun(c, s, st)) return st;
  }
  return SM_ERR_CAPACITY;
}


// ------------------------------------------------ allocation-free form ----
//
// sm_run_noalloc runs on one static device array per GPU instead of slot
// scratch.  Its layout: the kernel context, the descriptor and the counters,
// then every scratch array of a slot (each 256-byte aligned) for a fixed
// grid of kNaWgs workgroups and fixed per-workgroup capacities.

constexpr int kNaWgs = SM_NOALLOC_WORKGROUPS;
constexpr long long kNaEvents = SM_NOALLOC_MAX_EVENTS;
constexpr long long kNaVelo = SM_NOALLOC_MAX_VELO;
constexpr long long kNaPoolExtra = 1 << 16;   // seeds in the overflow area of the seed pool
// per-workgroup capacities: sm_run's starting sizes (they hold the items and
// events of the min-bias and uneven workloads: up to 630 VELO states and 524
// seeds per event), except the clone table (x hits of one item) and the seed
// staging (seeds of one item), which are halved
constexpr int kNaTrip = 8192, kNaCand = 2048, kNaTbl = 4096, kNaSst = 512, kNaCombo = 2048;
constexpr int kNaMs = 1024, kNaVs = 1024, kNaSurv = 2048;

constexpr size_t na_align(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t kNaKctxOff = 0;
constexpr size_t kNaDescOff = na_align(sizeof(smk::KCtx));
constexpr size_t kNaCntOff = kNaDescOff + na_align(sizeof(Desc));
constexpr size_t kNaArrOff = kNaCntOff + na_align(sizeof(Counters));

// Places the scratch arrays from kNaArrOff on; with S set, also points S's
// arrays at base + offset.  `off` ends as the array's size.
struct NaCarver {
  uintptr_t base;
  Scratch *S;
  size_t off;
  template <class T>
  constexpr void put(T *Scratch::*m, long long n) {
    off = na_align(off);
    if (S) S->*m = reinterpret_cast<T *>(base + off);
    off += (size_t)(n > 0 ? n : 1) * sizeof(T);
  }
};

constexpr void na_layout(NaCarver &k) {
  const long long G = kNaWgs, E = kNaEvents, I = 2 * kNaEvents;
  k.off = kNaArrOff;
  k.put(&Scratch::trip, G * kNaTrip);
  k.put(&Scratch::cand, G * kNaCand);
  k.put(&Scratch::tbl, G * kNaTbl);
  k.put(&Scratch::sst, G * kNaSst);
  k.put(&Scratch::combo, G * kNaCombo);
  k.put(&Scratch::cscore, G * kNaCand);
  k.put(&Scratch::cinfo, G * kNaCand);
  k.put(&Scratch::bestn, G * kNaCand);
  k.put(&Scratch::bestchi, G * kNaCand);
  k.put(&Scratch::bestidx, G * kNaCand);
  k.put(&Scratch::item_rec, I);
  k.put(&Scratch::item_cnt, I);
  k.put(&Scratch::item_base, I);
  k.put(&Scratch::ev_lcnt, E);
  k.put(&Scratch::ev_lbase, E);
  k.put(&Scratch::ev_done, E);
  k.put(&Scratch::pool, I * smk::kPoolPerItem + kNaPoolExtra);
  k.put(&Scratch::lpool, kNaVelo + 1024);
  k.put(&Scratch::ms, G * kNaMs);
  k.put(&Scratch::mf, G * 6 * kNaMs);
  k.put(&Scratch::best_s, G * kNaMs);
  k.put(&Scratch::best_v, G * kNaVs);
  k.put(&Scratch::surv, G * 2 * kNaSurv);
  k.off = na_align(k.off);
}

constexpr size_t na_bytes() {
  NaCarver k{0, nullptr, 0};
  na_layout(k);
  return k.off;
}
constexpr size_t kNaBytes = na_bytes();
static_assert(kNaBytes <= SM_NOALLOC_SCRATCH_BYTES, "static scratch above its stated maximum");

// Device address of `scratch` on each device, from hipGetSymbolAddress with
// that device current (each GPU holds its own copy of the array).
constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
void *g_na_ptr[kNaMaxDevices] = {};

}  // namespace

// The allocation-free form's scratch.  In host code this name is a host-side
// stand-in, not a device address: only the per-device address from
// hipGetSymbolAddress (g_na_ptr) is handed to kernels and copies.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

// Once per device, with that device current: the array's address, and its
// counters cleared.
sm_status na_setup(int dev) {
  if (dev < 0 || dev >= kNaMaxDevices) return SM_ERR_DEVICE;
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (g_na_ptr[dev]) return SM_OK;
  void *ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return SM_ERR_DEVICE;
  }
  if (hipMemset(static_cast<char *>(ptr) + kNaCntOff, 0, sizeof(Counters)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipGetLastError();
    return SM_ERR_DEVICE;
  }
  g_na_ptr[dev] = ptr;
  return SM_OK;
}

// The kernel context of the allocation-free form: the context's parameters,
// scratch pointers into the device's array, its own grid, matching always in
// the matching kernel and no big-item form.
void na_fill_kctx(const sm_ctx *c, void *ptr, smk::KCtx &kc) {
  memset(&kc, 0, sizeof(kc));
  Scratch &S = kc.S;
  NaCarver k{reinterpret_cast<uintptr_t>(ptr), &S, 0};
  na_layout(k);
  S.trip_cap = kNaTrip; S.cand_cap = kNaCand; S.tbl_cap = kNaTbl; S.sst_cap = kNaSst;
  S.combo_cap = kNaCombo;
  S.pool_static = 2 * kNaEvents * smk::kPoolPerItem;
  S.pool_cap = S.pool_static + kNaPoolExtra;
  S.lpool_cap = kNaVelo + 1024;
  S.ms_cap = kNaMs; S.vs_cap = kNaVs; S.surv_cap = kNaSurv;
  S.cnt = reinterpret_cast<Counters *>(static_cast<char *>(ptr) + kNaCntOff);
  S.need = reinterpret_cast<unsigned *>(reinterpret_cast<char *>(S.cnt) + offsetof(Counters, need_trip));
  kc.SB = S;   // the big-item form is never launched here
  kc.SB.need = reinterpret_cast<unsigned *>(reinterpret_cast<char *>(S.cnt) + offsetof(Counters, need_big));
  kc.P = c->dp;
  kc.P.main_slots = kNaWgs;
  kc.P.big_slots = 0;
  kc.P.match_mode = 1;
}

sm_status run_noalloc(sm_ctx *c, const sm_batch *b, sm_out *o, void *stream) {
  sm_status st = check_batch(c, b, o);
  if (st != SM_OK) return st;
  // the third iteration's clean-up needs batch-sized arrays of its own
  if (c->p.third_iter == 1) return SM_ERR_INVALID;
  if (b->n_events > kNaEvents || b->n_velo > kNaVelo) return SM_ERR_LIMIT;
  std::lock_guard<std::mutex> lk(c->mu);
  if (hipSetDevice(c->device) != hipSuccess) return SM_ERR_DEVICE;
  char *base = static_cast<char *>(g_na_ptr[c->device]);
  if (!base || !c->na_kctx) return SM_ERR_DEVICE;
  const smk::KCtx *dk = reinterpret_cast<const smk::KCtx *>(base + kNaKctxOff);
  Desc *dd = reinterpret_cast<Desc *>(base + kNaDescOff);
  Counters *dc = reinterpret_cast<Counters *>(base + kNaCntOff);
  fill_desc(*c->na_desc, *b, *o, kNaWgs, 0);
  hipStream_t q = (hipStream_t)stream;
  const int lds = lds_hits_for(c, *b);
  int e = hipMemcpyAsync((void *)dk, c->na_kctx, sizeof(smk::KCtx), hipMemcpyHostToDevice, q);
  if (!e) e = hipMemcpyAsync(dd, c->na_desc, sizeof(Desc), hipMemcpyHostToDevice, q);
  if (!e) e = smk_launch_zero(dc, (int)(sizeof(Counters) / sizeof(unsigned)), q);
  if (!e) e = smk_launch_prepare(dd, dk, 0, q);
  if (!e && c->cfg.validate) e = smk_launch_validate(dd, dk, 1024, q);
  if (!e) e = smk_launch_seed_nomatch(dd, dk, kNaWgs, lds, q);
  if (!e) e = smk_launch_match(dd, dk, kNaWgs, sel_of(c), q);
  if (!e) e = smk_launch_copy(dd, dk, 1024, q);
  if (!e) e = hipMemcpyAsync(c->na_cnt, dc, sizeof(Counters), hipMemcpyDeviceToHost, q);
  if (!e) e = hipStreamSynchronize(q);
  if (e) {
    (void)hipGetLastError();
    return SM_ERR_DEVICE;
  }
  const Counters &k = *c->na_cnt;
  o->n_seeds = k.total_seeds;
  o->n_longs = k.total_longs;
  const unsigned f = k.flags;
  if (k.stall) return SM_ERR_DEVICE;
  if (f & smk::F_INVALID) return SM_ERR_INVALID;
  if (f & smk::F_UNSORTED) return SM_ERR_UNSORTED;
  if (f & smk::F_LIMIT) return SM_ERR_LIMIT;
  // scratch that sm_run would grow and re-run with
  const unsigned scratch_flags = smk::F_TRIP | smk::F_CAND | smk::F_TBL | smk::F_SST | smk::F_POOL |
                                 smk::F_LPOOL | smk::F_MS | smk::F_VS | smk::F_SURV | smk::F_COMBO;
  if (f & scratch_flags) return SM_ERR_LIMIT;
  if (f & (smk::F_OUT_SEED | smk::F_OUT_LONG)) return SM_ERR_CAPACITY;
  return SM_OK;
}

}  // namespace

extern "C" {

void sm_default_geometry(sm_geometry *g) {
  static const double z[SM_N_LAYERS] = {7826.0, 7896.0, 7966.0, 8036.0, 8527.5, 8597.5,
                                        8667.5, 8737.5, 9229.0, 9299.0, 9369.0, 9439.0};
  const double t = std::tan(5.0 * M_PI / 180.0);
  for (int l = 0; l < SM_N_LAYERS; ++l) {
    g->z[l] = z[l];
    const int kind = l & 3;  // x u v x
    g->tan_stereo[l] = kind == 1 ? t : (kind == 2 ? -t : 0.0);
  }
  g->z_ref = 8525.0;
  // UT layers UTaX, UTaU, UTbV, UTbX (positions are a reading: none printed)
  static const double uz[SM_N_UT] = {2327.5, 2372.5, 2597.5, 2642.5};
  for (int i = 0; i < SM_N_UT; ++i) {
    g->ut_z[i] = uz[i];
    g->ut_tan[i] = i == 1 ? t : (i == 2 ? -t : 0.0);
  }
}

void sm_default_params(sm_params *p) {
  memset(p, 0, sizeof(*p));
  p->p_min = 3000.0;
  p->invp_a = 1.6322e-7;
  p->invp_b = -5.0217e-12;
  p->alpha0 = 2.180e6;
  p->alpha1 = -1073.0;
  p->d_ratio = -3.0e-4;
  p->kappa_c = 3.0e-3;
  p->t2_tol0 = 0.5;
  p->t2_tol1 = 0.5;
  p->ext_tol = 1.0;
  p->min_x_hits = 5;
  p->sigma_x = 0.07;
  p->chi2x_max = 6.0;
  p->uv_tol = 2.0;
  p->y_max = 2500.0;
  p->min_uv_hits = 4;
  p->chi2y_max = 6.0;
  const double zm[5] = {5287.6, -7.98878, 317.683, 0.0119379, -1418.42};
  for (int i = 0; i < 5; ++i) p->zm[i] = zm[i];
  p->z_ymatch = 10000.0;
  p->z_state = 9439.0;
  p->max_dx = 20.0;
  p->max_dy = 150.0;
  p->max_dtx = 1.5;
  p->max_dty = 0.02;
  p->tolx_scale = 0.8;
  p->tolx_a = 10.12;
  p->tolx_b = 101.0;
  p->toly_scale = 0.2;
  p->toly_a = 1.59;
  p->toly_b = 212.1;
  p->tol_tx = 0.5;
  p->tol_ty = 1.0 / 937.5;
  p->chi2m_max = 2.0;
  p->polarity = 1.0;
  p->uv_mode = 0;
  p->hough_bins = 64;
  p->hough_best = 8;
  p->hough_fine = 4;
  p->hough_min = 2;
  p->final_sel = 0;      // no network weights are published (reading)
  p->ghost_cut = 0.8;    // Sec. 4.4
  p->clone_gap = 0.05;   // Sec. 4.4
  p->third_iter = 0;     // Sec. 3: the HLT1 form runs two x-z iterations
  p->p_min3 = 1500.0;    // reading: the third iteration opens its windows for 1.5 GeV/c
  p->ut_mode = 0;        // Sec. 4.3: UT hits are optional
  p->ut_min_hits = 3;    // more than two
  p->a_gamma = 7.707063e-11;   // Table 1
  p->b_gamma = -7.817364e-3;
  // Table 2 by layer UTaX, UTaU, UTbV, UTbX; UTbX has no loose window and
  // UTaX no tight one (hi = 0)
  const double la[SM_N_UT] = {0.8333, 0.8333, 1.3333, 0.0}, lb[SM_N_UT] = {3.3333, 3.3333, 3.3333, 0.0};
  const double llo[SM_N_UT] = {1.2, 1.2, 1.5, 0.0}, lhi[SM_N_UT] = {8.5, 8.5, 9.5, 0.0};
  const double ta[SM_N_UT] = {0.0, 0.2, 0.4, 0.4}, tb[SM_N_UT] = {0.0, 0.6, 1.2, 1.2};
  const double tlo[SM_N_UT] = {0.0, 0.5, 1.0, 1.0}, thi[SM_N_UT] = {0.0, 2.0, 4.0, 4.0};
  for (int i = 0; i < SM_N_UT; ++i) {
    p->ut_loose_a[i] = la[i]; p->ut_loose_b[i] = lb[i]; p->ut_loose_lo[i] = llo[i]; p->ut_loose_hi[i] = lhi[i];
    p->ut_tight_a[i] = ta[i]; p->ut_tight_b[i] = tb[i]; p->ut_tight_lo[i] = tlo[i]; p->ut_tight_hi[i] = thi[i];
  }
}

// A usable network: every standardisation scale non-zero and every weight
// finite.
static bool ghost_nn_ok(const sm_ghost_nn &n) {
  for (int i = 0; i < SM_NN_INPUTS; ++i)
    if (!(n.scale[i] != 0.0) || !std::isfinite(n.scale[i]) || !std::isfinite(n.mean[i]))
      return false;
  for (int j = 0; j < SM_NN_HIDDEN; ++j) {
    for (int i = 0; i < SM_NN_INPUTS; ++i)
      if (!std::isfinite(n.w1[j][i])) return false;
    if (!std::isfinite(n.b1[j]) || !std::isfinite(n.w2[j])) return false;
  }
  return std::isfinite(n.b2);
}

sm_status sm_create(const sm_geometry *g, const sm_params *p, const sm_config *cfg, sm_ctx **out) {
  if (!out) return SM_ERR_INVALID;
  *out = nullptr;
  sm_ctx *c = new (std::nothrow) sm_ctx();
  if (!c) return SM_ERR_OOM;
  if (g) c->g = *g; else sm_default_geometry(&c->g);
  if (p) c->p = *p; else sm_default_params(&c->p);
  if (cfg) c->cfg = *cfg;
  // the per-event form launches two workgroups (one per detector half) on the
  // per-workgroup scratch, so a context needs scratch for at least two
  if ((c->cfg.seed_wgs != 0 && c->cfg.seed_wgs < 2) ||
      c->p.p_min <= 0 || c->p.sigma_x <= 0 || c->p.min_x_hits < 4 || c->p.min_x_hits > 6 ||
      c->p.min_uv_hits < 3 || c->p.min_uv_hits > 6 ||
      (c->p.final_sel != 0 && c->p.final_sel != 1) ||
      (c->p.ut_mode != 0 && c->p.ut_mode != 1) ||
      (c->p.third_iter != 0 && c->p.third_iter != 1) ||
      (c->p.third_iter == 1 &&
       (!(c->p.p_min3 > 0) ||
        c->p.invp_a * c->p.invp_a + 4.0 * c->p.invp_b / c->p.p_min3 < 0)) ||
      (c->p.ut_mode == 1 && (c->p.ut_min_hits < 1 || c->p.ut_min_hits > SM_N_UT)) ||
      (c->p.final_sel == 1 && (!ghost_nn_ok(c->p.ghost_nn) || !(c->p.clone_gap >= 0.0))) ||
      c->p.invp_a * c->p.invp_a + 4.0 * c->p.invp_b / c->p.p_min < 0 ||
      // the Hough-cluster UV kernel (uv_mode 1) is switched off: one run of
      // it under a 5-workgroup context ended in a GPU memory fault whose
      // cause is not yet found
      c->p.uv_mode != 0 ||
      (c->p.uv_mode == 1 &&
       (c->p.hough_bins < 1 || c->p.hough_bins > smk::kHoughBins || c->p.hough_best < 1 ||
        c->p.hough_fine < 1 || c->p.hough_best * c->p.hough_fine > 64 || c->p.hough_min < 1))) {
    delete c;
    return SM_ERR_INVALID;
  }
  c->device = c->cfg.device;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || c->device < 0 || c->device >= ndev ||
      hipSetDevice(c->device) != hipSuccess) {
    hipGetLastError();
    delete c;
    return SM_ERR_DEVICE;
  }
  hipDeviceProp_t prop;
  hipGetDeviceProperties(&prop, c->device);
  const int cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->base_wgs = c->cfg.seed_wgs > 0 ? c->cfg.seed_wgs : cus * 4;
  c->seed_wgs = c->base_wgs;
  // the main seeding forms may take dynamic LDS beyond 64 KB where the device
  // allows it (launch shapes of up to 6144 LDS hits)
  {
    const size_t want = smk_seed_lds_bytes(6144);
    const size_t dev = prop.sharedMemPerBlock > 0 ? (size_t)prop.sharedMemPerBlock : 65536;
    const size_t lim = std::min(want, dev);
    if (lim > 65536 && smk_seed_lds_limit((int)lim) == 0) c->lds_limit = lim;
    (void)hipGetLastError();
  }
  // big-item form: one 1024-thread workgroup per CU, hits in LDS up to what
  // the per-workgroup LDS limit leaves after its shared state
  c->big_wgs = std::max(cus / 2, 1);
  {
    const size_t lim0 = prop.sharedMemPerBlock > 0 ? (size_t)prop.sharedMemPerBlock : 65536;
    const size_t stat = (size_t)std::max(smk_seed_big_static_lds(), 0);
    const size_t lim = lim0 > stat ? lim0 - stat : 0;
    const size_t base = smk_seed_big_lds_bytes(0);
    long long h = lim > base ? (long long)((lim - base) / 12) : 0;   // x, z, id per hit
    h = std::min<long long>(h, 12288) / 256 * 256;
    c->lds_big = (int)std::max<long long>(h, 256);
    if (smk_seed_big_lds_bytes(c->lds_big) > 65536 &&
        smk_seed_big_lds_limit((int)smk_seed_big_lds_bytes(c->lds_big)) != 0) {
      (void)hipGetLastError();
      const size_t b64 = 65536 > base + stat ? (65536 - base - stat) / 12 / 256 * 256 : 0;
      c->lds_big = (int)std::max<size_t>(b64, 256);
    }
  }
  // whether the matching kernel or the seeding kernel matches is chosen per
  // batch (match_wgs 0), or fixed (> 0: the matching kernel, with at most the
  // batch's seeding grid of workgroups, whose matching scratch it uses; < 0:
  // the seeding kernel)
  c->dp = make_params(c->g, c->p);
  c->dp.match_mode = c->cfg.match_wgs > 0 ? 1 : (c->cfg.match_wgs < 0 ? -1 : 0);
  // the Hough-cluster form is built only with the matching code: its batches
  // are always matched inside the seeding kernel (with k_match chosen, that
  // instantiation would return at once and leave the batch unseeded)
  if (c->p.uv_mode != 0) c->dp.match_mode = -1;
  // item latency on one 256-thread workgroup, fitted to phase timers on
  // min-bias (778 hits: 93 us) and stress items (12,011 hits: 13.9 ms)
  c->dp.main_slots = c->base_wgs;
  c->dp.big_slots = c->big_wgs;
  c->dp.lat_a = 0.048f;
  c->dp.lat_b = 9.2e-5f;
  c->dp.big_speedup = 3.0f;   // 16 waves against 4 on the same item
  // the allocation-free form: the device's static array (once per device)
  // and this context's pinned copies of its kernel context and descriptor
  if (na_setup(c->device) != SM_OK ||
      hipHostMalloc(&c->na_kctx, sizeof(smk::KCtx), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&c->na_desc, sizeof(Desc), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&c->na_cnt, sizeof(Counters), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    sm_destroy(c);
    return SM_ERR_DEVICE;
  }
  na_fill_kctx(c, g_na_ptr[c->device], *c->na_kctx);
  const int n_slots = 1 + (c->cfg.n_slots > 0 ? c->cfg.n_slots : 2);
  c->slots.resize(n_slots);
  for (Slot &s : c->slots) {
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&s.d_desc, sizeof(Desc)) != hipSuccess ||
        hipMalloc(&s.d_kctx, sizeof(smk::KCtx)) != hipSuccess ||
        hipMalloc(&s.d_desc3, sizeof(Desc)) != hipSuccess ||
        hipMalloc(&s.d_kctx3, sizeof(smk::KCtx)) != hipSuccess ||
        // coherent: the batched sequence's kernels read the descriptors and
        // write the counters here directly
        hipHostMalloc(&s.h_desc, sizeof(Desc), hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc(&s.h_desc3, sizeof(Desc), hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc(&s.h_cnt, sizeof(Counters), hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc(&s.h_cnt3, sizeof(Counters), hipHostMallocCoherent) != hipSuccess) {
      hipGetLastError();
      sm_destroy(c);
      return SM_ERR_DEVICE;
    }
    s.caps.items = 2048;
    s.caps.events = 1024;
    s.caps.pool = 1 << 16;
    s.caps.lpool = 1 << 15;
    if (c->p.third_iter == 1) {
      s.caps.hits = 1 << 20;
      s.caps.pool3 = 1 << 16;
    }
    sm_status st = alloc_slot(c, s);
    if (st != SM_OK) {
      sm_destroy(c);
      return st;
    }
  }
  *out = c;
  return SM_OK;
}

sm_status sm_run(sm_ctx *ctx, const sm_batch *batch, sm_out *out, void *stream) {
  if (!ctx) return SM_ERR_INVALID;
  return run_blocking(ctx, batch, out, stream, false);
}

sm_status sm_run_plain(sm_ctx *ctx, const sm_batch *batch, sm_out *out, void *stream) {
  if (!ctx) return SM_ERR_INVALID;
  return run_blocking(ctx, batch, out, stream, true);
}

sm_status sm_run_noalloc(sm_ctx *ctx, const sm_batch *batch, sm_out *out, void *stream) {
  if (!ctx) return SM_ERR_INVALID;
  return run_noalloc(ctx, batch, out, stream);
}

sm_status sm_profile(sm_ctx *ctx, const sm_batch *batch, sm_out *out, void *stream,
                     sm_kernel_times *t) {
  if (!ctx || !t) return SM_ERR_INVALID;
  memset(t, 0, sizeof(*t));
  return run_blocking(ctx, batch, out, stream, false, t);
}

static sm_status start_slot(sm_ctx *c, Slot &s) {
  sm_status st = fit_batch(c, s, s.batch);
  if (st != SM_OK) return st;
  fill_descs(c, s, s.batch, *s.out);
  // the graph's kernels read the pinned descriptor and write the pinned counters
  if ((st = enqueue_batched(c, s, s.stream)) != SM_OK) return st;
  return hip_status(hipEventRecord(s.done, s.stream));
}

sm_status sm_submit(sm_ctx *ctx, const sm_batch *batch, sm_out *out, int64_t *ticket) {
  if (!ctx || !ticket) return SM_ERR_INVALID;
  sm_status st = check_batch(ctx, batch, out);
  if (st != SM_OK) return st;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (hipSetDevice(ctx->device) != hipSuccess) return SM_ERR_DEVICE;
  for (size_t i = 1; i < ctx->slots.size(); ++i) {
    Slot &s = ctx->slots[i];
    if (s.busy) continue;
    s.batch = *batch;
    s.out = out;
    s.tries = 0;
    if ((st = start_slot(ctx, s)) != SM_OK) return st;
    s.busy = true;
    s.ticket = ctx->next_ticket++;
    *ticket = s.ticket;
    return SM_OK;
  }
  return SM_ERR_BUSY;
}

sm_status sm_poll(sm_ctx *ctx, int64_t ticket, int wait) {
  if (!ctx) return SM_ERR_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (hipSetDevice(ctx->device) != hipSuccess) return SM_ERR_DEVICE;
  for (size_t i = 1; i < ctx->slots.size(); ++i) {
    Slot &s = ctx->slots[i];
    if (!s.busy || s.ticket != ticket) continue;
    for (;;) {
      hipError_t e = wait ? hipEventSynchronize(s.done) : hipEventQuery(s.done);
      if (e == hipErrorNotReady) return SM_ERR_NOT_READY;
      if (e != hipSuccess) { s.busy = false; return SM_ERR_DEVICE; }
      sm_status st;
      s.out->n_seeds = s.h_cnt->total_seeds;
      s.out->n_longs = s.h_cnt->total_longs;
      if (needs_rerun(ctx, s, st)) {
        if (++s.tries >= kMaxTries) {
          // scratch grown kMaxTries times and still too small: the last run
          // dropped work, so its outputs are not reported as complete
          s.busy = false;
          return SM_ERR_CAPACITY;
        }
        if ((st = start_slot(ctx, s)) != SM_OK) { s.busy = false; return st; }
        if (!wait) return SM_ERR_NOT_READY;
        continue;
      }
      s.busy = false;
      return st;
    }
  }
  return SM_ERR_INVALID;
}

sm_status sm_set_shapes(sm_ctx *ctx, const sm_shape *shapes, int32_t n) {
  if (!ctx || n < 0 || (n > 0 && !shapes)) return SM_ERR_INVALID;
  std::vector<sm_shape> t(shapes, shapes + n);
  int grid = ctx->base_wgs;
  for (const sm_shape &e : t) {
    if (e.max_mean_item_hits < 0 || e.max_events < 0 || e.seed_wgs < 2 || e.seed_wgs > 65536 ||
        e.lds_hits < 256 || e.lds_hits > 6144 || e.lds_hits % 256 != 0 ||
        smk_seed_lds_bytes(e.lds_hits) > ctx->lds_limit)
      return SM_ERR_INVALID;
    grid = std::max(grid, e.seed_wgs);
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (const Slot &s : ctx->slots)
    if (s.busy) return SM_ERR_BUSY;
  if (hipSetDevice(ctx->device) != hipSuccess) return SM_ERR_DEVICE;
  ctx->shapes = t;
  if (grid > ctx->seed_wgs) {
    // per-workgroup scratch for the larger grid (graphs are rebuilt)
    ctx->seed_wgs = grid;
    for (Slot &s : ctx->slots) {
      const sm_status st = alloc_slot(ctx, s);
      if (st != SM_OK) return st;
    }
  }
  return SM_OK;
}

sm_status sm_launch_shape(const sm_ctx *ctx, const sm_batch *batch, sm_shape *shape) {
  if (!ctx || !batch || !shape || batch->n_events < 0 || batch->n_hits < 0) return SM_ERR_INVALID;
  *shape = choose_shape(ctx, *batch);
  return SM_OK;
}

int64_t sm_batch_bytes(const sm_ctx *ctx, int32_t n_events, int64_t n_hits, int64_t n_velo) {
  (void)ctx;
  const int64_t items = 2 * (int64_t)n_events;
  return items * ((int64_t)sizeof(smk::ItemRec) + 2 * 4) + (int64_t)n_events * 3 * 4 +
         (items * smk::kPoolPerItem + n_hits / 8 + 1024) * (int64_t)sizeof(sm_seed) +
         (n_velo + 1024) * (int64_t)sizeof(sm_long);
}

sm_status sm_destroy(sm_ctx *ctx) {
  if (!ctx) return SM_ERR_INVALID;
  hipSetDevice(ctx->device);
  for (Slot &s : ctx->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    free_slot_scratch(s);
    destroy_graphs(s);
    if (s.done) hipEventDestroy(s.done);
    if (s.stream) hipStreamDestroy(s.stream);
    if (s.d_desc) hipFree(s.d_desc);
    if (s.d_kctx) hipFree(s.d_kctx);
    if (s.d_desc3) hipFree(s.d_desc3);
    if (s.d_kctx3) hipFree(s.d_kctx3);
    if (s.h_desc) hipHostFree(s.h_desc);
    if (s.h_desc3) hipHostFree(s.h_desc3);
    if (s.h_cnt) hipHostFree(s.h_cnt);
    if (s.h_cnt3) hipHostFree(s.h_cnt3);
  }
  if (ctx->na_kctx) hipHostFree(ctx->na_kctx);
  if (ctx->na_desc) hipHostFree(ctx->na_desc);
  if (ctx->na_cnt) hipHostFree(ctx->na_cnt);
  delete ctx;
  return SM_OK;
}

const char *sm_status_str(sm_status s) {
  switch (s) {
    case SM_OK: return "ok";
    case SM_ERR_INVALID: return "invalid argument or malformed batch";
    case SM_ERR_UNSORTED: return "hits not x-sorted inside a zone";
    case SM_ERR_CAPACITY: return "output capacity too small";
    case SM_ERR_OOM: return "out of device memory";
    case SM_ERR_DEVICE: return "HIP runtime error";
    case SM_ERR_BUSY: return "no free serving slot";
    case SM_ERR_NOT_READY: return "not ready";
    case SM_ERR_LIMIT: return "event exceeds the per-event hit limit";
  }
  return "unknown status";
}

}  // extern "C"
