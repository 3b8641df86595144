// HIP kernels of SciFi Seeding (Sec. 3) and VELO-SciFi Matching (Sec. 4)
// for gfx950 (CDNA4, wave64).
//
// Precision: hits are FP32.  The combinatorial search (T1 x T3 doublets, T2
// third hit, Sec. 3.3.2-3.3.3) runs in FP32; the per-triplet work (3-point
// model, 1 mm extension, least-squares fit, score), UV seeding and the
// chi2_match of the preselected pairs run in FP64, so that fits and the
// clone-vote scores keep the digits the vote compares.
#include "sm_device.h"

#include <type_traits>

namespace smk {

// Global-memory access through an address-space-1 pointer compiles to a
// global (not flat) instruction: a 32-bit offset from a scalar base, and not
// counted by the LDS wait counter, so a wait for an LDS result does not also
// wait for these loads and stores.  Pointers read from the descriptor structs
// are generic, so the hot accesses go through these helpers.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}
// whole records of library scratch, in 16-byte pieces (records a multiple
// of 16 B, 16 B aligned) or else 8-byte pieces (a multiple of 8 B, 8 B aligned)
typedef int gvec4 __attribute__((ext_vector_type(4)));
typedef int gvec2 __attribute__((ext_vector_type(2)));
template <class T>
using gpiece = typename std::conditional<sizeof(T) % 16 == 0, gvec4, gvec2>::type;
template <class T> __device__ __forceinline__ void gstore(T *p, const T &v) {
  static_assert(sizeof(T) % 8 == 0, "records are stored in 8- or 16-byte pieces");
  using V = gpiece<T>;
  const V *s = reinterpret_cast<const V *>(&v);
  __attribute__((address_space(1))) V *d = (__attribute__((address_space(1))) V *)p;
#pragma unroll
  for (unsigned k = 0; k < sizeof(T) / sizeof(V); ++k) d[k] = s[k];
}
template <class T> __device__ __forceinline__ T gload(const T *p) {
  static_assert(sizeof(T) % 8 == 0, "records are loaded in 8- or 16-byte pieces");
  using V = gpiece<T>;
  T v;
  V *d = reinterpret_cast<V *>(&v);
  const __attribute__((address_space(1))) V *s = (const __attribute__((address_space(1))) V *)p;
#pragma unroll
  for (unsigned k = 0; k < sizeof(T) / sizeof(V); ++k) d[k] = s[k];
  return v;
}


// The thread's index in its workgroup, as a value the compiler must treat as
// new at every call: addresses derived from it are then formed where they are
// used, instead of being hoisted out of the item loop and kept live (which
// spilled them to scratch memory, a global round trip per reload).
__device__ __forceinline__ int tidx() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// x-layer slots 0..5 <-> layers 0, 3, 4, 7, 8, 11; stereo slots 0..5 <->
// layers 1, 2, 5, 6, 9, 10 (Sec. 1: x-u-v-x in each station).
__device__ __forceinline__ int xlayer(int slot) { return (slot >> 1) * 4 + (slot & 1) * 3; }
__device__ __forceinline__ int uvlayer(int slot) { return (slot >> 1) * 4 + 1 + (slot & 1); }

__device__ __forceinline__ float gf(float u, float d) { return u * u * (1.0f + d * u); }
__device__ __forceinline__ double gd(double u, double d) { return u * u * (1.0 + d * u); }

__device__ __forceinline__ double xm(double a, double b, double c, double z, const DevParams &P) {
  const double u = z - P.zref;
  return a + b * u + c * gd(u, P.d);
}
// x(z) at layer L's nominal z, from that layer's u and g(u)
__device__ __forceinline__ double xm_layer(double a, double b, double c, int L, const DevParams &P) {
  return a + b * P.uz[L] + c * P.gz[L];
}

// popcount of the set bits of m below this lane
__device__ __forceinline__ unsigned lane_rank(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Wave-aggregated append: every active lane gets its own slot of *counter
// with one atomic per wave (ballot + prefix of the active mask).
__device__ __forceinline__ unsigned wave_append(unsigned *counter) {
  const unsigned long long m = __ballot(1);
  const unsigned r = lane_rank(m);
  unsigned base = 0;
  if (r == 0) base = atomicAdd(counter, (unsigned)__popcll(m));
  base = __builtin_amdgcn_readfirstlane(base);
  return base + r;
}

// A workgroup barrier that orders LDS accesses only: unlike __syncthreads it
// does not wait for the waves' outstanding global loads and stores, so loads
// issued before it keep streaming in.  Only for code that passes nothing
// through global memory between the workgroup's threads across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Exclusive scan of one int per thread over a workgroup of NT threads
// (kLdsOnly: its barriers are lds_barrier).
template <int NT, bool kLdsOnly = false>
__device__ __forceinline__ int block_excl_scan(int v, int *s_tmp, int &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_tmp[w] = x;
  if constexpr (kLdsOnly) lds_barrier(); else __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    const int t = s_tmp[i];
    pre += i < w ? t : 0;
    tot += t;
  }
  if constexpr (kLdsOnly) lds_barrier(); else __syncthreads();
  total = tot;
  return pre + x - v;
}

// first i in [lo, hi) with X[i] >= v
// first i in [lo, hi) with X[i] > v
__device__ __forceinline__ int upper_f(const float *X, int lo, int hi, float v) {
  while (lo < hi) {
    const int m = (lo + hi) >> 1;
    if (X[m] <= v) lo = m + 1; else hi = m;
  }
  return lo;
}
__device__ __forceinline__ int lower_f(const float *X, int lo, int hi, float v) {
  while (lo < hi) {
    const int m = (lo + hi) >> 1;
    if (X[m] < v) lo = m + 1; else hi = m;
  }
  return lo;
}

// Rank of value v among a[0..n): entries below v plus equal entries before
// position self.  Loads are issued eight at a time so that their latencies
// overlap (every lane reads the same a[j]: an LDS broadcast).
template <class T>
__device__ __forceinline__ unsigned rank_of(const T *a, unsigned n, T v, unsigned self) {
  unsigned r = 0, j = 0;
  for (; j + 8 <= n; j += 8) {
    T u[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) u[q] = a[j + q];
#pragma unroll
    for (int q = 0; q < 8; ++q) r += (u[q] < v) | ((u[q] == v) & (j + q < self));
  }
  for (; j < n; ++j) {
    const T u = a[j];
    r += (u < v) | ((u == v) & (j < self));
  }
  return r;
}

__device__ __forceinline__ void raise_flag(Counters *c, unsigned f) { atomicOr(&c->flags, f); }

// Least-squares fit of eq. trackequation over the x-layer hits present in
// `pos` (d_ratio fixed).  Coordinates are taken relative to the first hit and
// the basis is scaled by 1 m so that the normal equations stay well
// conditioned; the 3x3 system is solved by cofactors.  Returns false if it is
// singular.
__device__ __forceinline__ bool fit_x(const float *X, const float *Z, const int (&pos)[6],
                                      const DevParams &P, double &a, double &b, double &c,
                                      double &chi2, int &n) {
  const double S = 1e-3, S2 = 1e-6;
  double A00 = 0, A01 = 0, A02 = 0, A11 = 0, A12 = 0, A22 = 0, r0 = 0, r1 = 0, r2 = 0;
  double xref = 0.0;
  n = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    if (pos[k] < 0) continue;
    const double x = X[pos[k]], z = Z[pos[k]];
    if (n == 0) xref = x;
    const double u = z - P.zref;
    const double f1 = u * S, f2 = gd(u, P.d) * S2, xr = x - xref;
    A00 += 1.0; A01 += f1; A02 += f2; A11 += f1 * f1; A12 += f1 * f2; A22 += f2 * f2;
    r0 += xr; r1 += f1 * xr; r2 += f2 * xr;
    ++n;
  }
  const double C00 = A11 * A22 - A12 * A12, C01 = A02 * A12 - A01 * A22, C02 = A01 * A12 - A02 * A11;
  const double det = A00 * C00 + A01 * C01 + A02 * C02;
  if (det == 0.0) return false;
  const double C11 = A00 * A22 - A02 * A02, C12 = A01 * A02 - A00 * A12, C22 = A00 * A11 - A01 * A01;
  const double inv = 1.0 / det;
  const double q0 = (C00 * r0 + C01 * r1 + C02 * r2) * inv;
  const double q1 = (C01 * r0 + C11 * r1 + C12 * r2) * inv;
  const double q2 = (C02 * r0 + C12 * r1 + C22 * r2) * inv;
  a = q0 + xref;
  b = q1 * S;
  c = q2 * S2;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    if (pos[k] < 0) continue;
    const double r = (double)X[pos[k]] - xm(a, b, c, Z[pos[k]], P);
    s += r * r;
  }
  chi2 = s * P.inv_sigma2 / (double)(n - 3);
  return true;
}

// ---------------------------------------------------------------- XZ ------

// Per-zone x-bin index of an item whose hits sit in LDS: bins[L][b] is the
// zone-local index of the first hit whose bin number kbin(x) exceeds b.
// kbin is a monotonic function of x, so every hit before bins[L][kbin(v)-1]
// lies below v and a lower-bound search starts there and walks forward a
// hit or two instead of bisecting the zone.
constexpr int kBins = 128;
constexpr float kBinX0 = -3600.0f;
constexpr float kBinInv = (float)kBins / 7200.0f;

__device__ __forceinline__ int kbin(float x) {
  const float f = floorf((x - kBinX0) * kBinInv);
  return f < 0.0f ? 0 : (f >= (float)kBins ? kBins : (int)f + 1);
}

// Before the vote, the vote table's LDS holds the first kTripLds triplets
// and, after them, the doublet map of the triplet search: the workgroup
// slot of the T1 hit of each of the first doublets of a round (one byte,
// two with 1024-thread workgroups).
constexpr int kTripLds = kXtabLds / 2;
template <int NT>
using SlotMap = typename std::conditional<(NT <= 256), unsigned char, unsigned short>::type;
template <int NT>
constexpr int kDmap = (kXtabLds - kTripLds) * (int)sizeof(unsigned long long) / (int)sizeof(SlotMap<NT>);
// the track slot of each combination of a UV round (the first kCmap)
template <int NT>
constexpr int kCmap = 1024 / (int)sizeof(SlotMap<NT>);

// Everything one seeding workgroup keeps in LDS besides the hits (whose
// capacity is set per launch in dynamic LDS).
template <int NT>
struct SeedShared {
  unsigned short bins[kNL][kBins];
  unsigned long long cscore[kCandLds];   // candidate scores
  int cinfo[kCandLds];                   // n | it << 3 | lost << 4 | repeat << 5
  unsigned short cpos[kCandLds][6];      // x-hit positions + 1 (0: none)
  union {
    unsigned long long xtab[kXtabLds];   // clone-vote table over the item's x hits; before
                                         // the vote, triplets and the doublet map
    struct {
      double cabc[kCandLds][3];          // x-z parameters for UV
      unsigned long long bestchi[kCandLds];
      int bestn[kCandLds];
      int bestidx[kCandLds];
    } uv;
    unsigned long long skey[kSeedLds];   // seed keys for the canonical rank
  } u;
  int scan[NT], a0[NT], a1[NT], a2[NT];
  SlotMap<NT> cmap[kCmap<NT>];           // track slot of each combination of a UV round
  int tmp[16];
  int zoff[kNL + 1];
  int zabs[kNL + 1];                     // the item's zone offsets in the batch
  int zlo[kNL], zhi[kNL];                // z span of each layer (Hough UV), as zkey
  int xb[7];                             // first compact x index of each x slot
  int item;
  int pass;                              // the batch's pass (third iteration): 0, 1 or 2
  unsigned serial;                       // the batch's serial (hit marks of pass 1)
  unsigned ntrip, ncand, nseed, ncombo, nkept;
  unsigned long long pbase;
};


// first i of zone L with X[i] >= v
template <bool kLds, class T, int NT>
__device__ __forceinline__ int zlower(const float *X, const SeedShared<NT> &sh, int L, T v) {
  const int lo = sh.zoff[L], hi = sh.zoff[L + 1];
  if constexpr (kLds) {
    const int k = kbin((float)v);
    int i = lo + (k > 0 ? (int)sh.bins[L][k - 1] : 0);
    // from the bin's first hit, four hits per LDS round trip: the hits are
    // sorted, so the count of them below v is how far to move.  The loads
    // are not guarded: i never passes the zone's end, so they reach at most
    // three hits past it, inside the item's LDS hit arrays, and those read as v
    for (;;) {
      T x4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T xv = (T)X[i + q];
        x4[q] = i + q < hi ? xv : v;
      }
      int c = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) c += x4[q] < v;
      i += c;
      if (c < 4) return i;
    }
  } else {
    int a = lo, b = hi;
    while (a < b) {
      const int m = (a + b) >> 1;
      if ((T)X[m] < v) a = m + 1; else b = m;
    }
    return a;
  }
}

// Closest hit to pred in zone L inside [pred - tol, pred + tol]; -1 if none.
// Distances closer than kTieMm are a tie, won by the lower position: a later
// hit replaces the current one only if it is closer by more than kTieMm, so a
// prediction midway between two hits picks the same hit whatever the
// rounding of the prediction.  The x and z of the chosen hit come back in
// xb, zb (read with the walk).
template <bool kLds, int NT>
__device__ __forceinline__ int zclosest(const float *X, const float *Z, const SeedShared<NT> &sh,
                                        int L, double pred, double tol, float &xb, float &zb) {
  const int hi = sh.zoff[L + 1];
  const double lo_v = pred - tol, hi_v = pred + tol;
  int best = -1;
  double bd = 0.0;
  xb = 0.0f;
  zb = 0.0f;
  if constexpr (kLds) {
    // from the bin of pred - tol, four hits per LDS round trip, each tested
    // with selects rather than branches, in ascending order as the one-hit
    // walk does.  The distance to beat starts at +inf, so the first hit in
    // the window is taken as the walk takes it.  The four loads are not
    // guarded: past the zone's end (at most three hits) they stay inside the
    // item's LDS hit arrays, and those x are replaced by +inf.  The walk ends
    // past the window or at the zone's end.
    const int k = kbin((float)lo_v);
    int i = sh.zoff[L] + (k > 0 ? (int)sh.bins[L][k - 1] : 0);
    bd = __builtin_inf();
    for (;; i += 4) {
      float x4[4], z4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float xv = X[i + q];
        x4[q] = i + q < hi ? xv : __builtin_inff();
        z4[q] = Z[i + q];
      }
      double x;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        x = x4[q];
        const double d = fabs(x - pred);
        const bool take = x >= lo_v && x <= hi_v && d < bd - kTieMm;
        best = take ? i + q : best;
        bd = take ? d : bd;
        xb = take ? x4[q] : xb;
        zb = take ? z4[q] : zb;
      }
      if (!(x <= hi_v) || i + 4 >= hi) break;
    }
  } else {
    for (int i = zlower<kLds>(X, sh, L, lo_v); i < hi; ++i) {
      const double x = X[i];
      if (x > hi_v) break;
      const double d = fabs(x - pred);
      if (best < 0 || d < bd - kTieMm) { best = i; bd = d; }
    }
    if (best >= 0) { xb = X[best]; zb = Z[best]; }
  }
  return best;
}
template <bool kLds, int NT>
__device__ __forceinline__ int zclosest(const float *X, const float *Z, const SeedShared<NT> &sh,
                                        int L, double pred, double tol) {
  float xb, zb;
  return zclosest<kLds>(X, Z, sh, L, pred, tol, xb, zb);
}

// T1 x T3 doublets and T2 third hits of both iterations (Sec. 3.3.2-3.3.3),
// FP32.  The T1 hits of both iterations form one list taken 256 at a time;
// each thread finds the T3 window of its T1 hit, a workgroup scan flattens
// the doublets so every thread gets an equal share, and the T2 hits found
// for a doublet are appended with one atomic per wave, the first kTripLds
// triplets to LDS and the rest to the workgroup's global scratch.
template <bool kLds, int NT>
__device__ __forceinline__ void xz_triplets(const float *X, const float *Z, SeedShared<NT> &sh,
                                            const DevParams &P, unsigned long long *trip,
                                            int trip_cap) {
  const int *zoff = sh.zoff;
  // the third iteration (pass 2) starts from iteration 0's T1 layer only
  const bool third = sh.pass == 2;
  const int n1a = zoff[1] - zoff[0], n1b = third ? 0 : zoff[4] - zoff[3];
  const int N1 = n1a + n1b;
  const float zr = P.zreff, dd = P.df;
  for (int c0 = 0; c0 < N1; c0 += NT) {
    const int j = c0 + (int)threadIdx.x;
    int st = 0, cnt_j = 0, i1 = 0, it = 0;
    if (j < N1) {
      it = j >= n1a;
      i1 = it ? zoff[3] + (j - n1a) : zoff[0] + j;
      const int L3 = it ? 11 : 8;
      const float x1 = X[i1], z1 = Z[i1];
      // window around x1 (z3 + alpha_corr) / z1, half-width Delta x3^max
      // window constants: the iteration's, or the third iteration's
      const int ic = third ? 2 : it;
      const float centre = (P.zf[L3] + P.alphaf[ic]) / z1 * x1;
      const float dx3 = P.dx3f[ic];
      st = zlower<kLds>(X, sh, L3, centre - dx3);
      const float hi3 = centre + dx3;
      int en = st;
      const int e3 = zoff[L3 + 1];
      if constexpr (kLds) {
        en = zlower<kLds>(X, sh, L3, hi3);
        while (en < e3 && X[en] <= hi3) ++en;
      } else {
        int b = e3;
        while (en < b) {
          const int m = (en + b) >> 1;
          if (X[m] <= hi3) en = m + 1; else b = m;
        }
      }
      cnt_j = en > st ? en - st : 0;
    }
    int total;
    // LDS-only barriers up to the round's end; the triplets beyond the LDS
    // list go to global memory and are read after the round's __syncthreads
    const int excl = block_excl_scan<NT, true>(cnt_j, sh.tmp, total);
    sh.scan[threadIdx.x] = excl;
    sh.a0[threadIdx.x] = st;
    sh.a1[threadIdx.x] = i1 | (it << 30);
    SlotMap<NT> *dmap = reinterpret_cast<SlotMap<NT> *>(sh.u.xtab + kTripLds);
    for (int d = excl; d < excl + cnt_j && d < kDmap<NT>; ++d) dmap[d] = (SlotMap<NT>)threadIdx.x;
    lds_barrier();
    const int nj = min(NT, N1 - c0);
    for (int d0 = 0; d0 < total; d0 += NT) {
      const int d = d0 + (int)threadIdx.x;
      if (d < total) {
        // the doublet's T1 slot: from the map, else a search of the scan
        int jj;
        if (d < kDmap<NT>) {
          jj = dmap[d];
        } else {
          int lo = 0, hi = nj;
          while (lo < hi) {
            const int m = (lo + hi) >> 1;
            if (sh.scan[m] <= d) lo = m + 1; else hi = m;
          }
          jj = lo - 1;
        }
        const int w = sh.a1[jj];
        const int di = w >> 30, d1 = w & 0x3fffffff;
        const int d3 = sh.a0[jj] + (d - sh.scan[jj]);
        const int L2 = di ? 7 : 4;
        const float z2n = P.zf[L2];
        const float x1 = X[d1], z1 = Z[d1], x3 = X[d3], z3 = Z[d3];
        const float t13 = (x3 - x1) / (z3 - z1);
        const float x0 = x1 - z1 * t13;
        const float ip = P.invp_af * fabsf(x0) + P.invp_bf * x0 * x0;
        const float cpred = (x0 >= 0.0f ? -1.0f : 1.0f) * P.kappa_cf * ip;
        const float g1 = gf(z1 - zr, dd), g3 = gf(z3 - zr, dd);
        const float k3 = gf(z2n - zr, dd) - g1 - (z2n - z1) / (z3 - z1) * (g3 - g1);
        const float dev = k3 * cpred;
        const float pred = x1 + (z2n - z1) * t13 + dev;
        const float tol = P.t2_tol0f + P.t2_tol1f * fabsf(dev);
        const float hi2 = pred + tol;
        const int e2 = zoff[L2 + 1];
        int k = zlower<kLds>(X, sh, L2, pred - tol);
        bool more = k < e2 && X[k] <= hi2;
        const unsigned long long head = ((unsigned long long)di << 63) |
                                        ((unsigned long long)d1 << 42) |
                                        ((unsigned long long)d3 << 21);
        while (more) {
          const unsigned slot = wave_append(&sh.ntrip);
          const unsigned long long v = head | (unsigned long long)k;
          if (slot < (unsigned)kTripLds) sh.u.xtab[slot] = v;
          else if (slot < (unsigned)trip_cap) trip[slot] = v;
          ++k;
          more = k < e2 && X[k] <= hi2;
        }
      }
    }
    __syncthreads();
  }
}

// Extension, fit and score of one triplet (Sec. 3.2, eq. seed_clone_score).
template <bool kLds, int NT>
__device__ __forceinline__ bool xz_candidate(const float *X, const float *Z, const SeedShared<NT> &sh,
                                             const DevParams &P, unsigned long long key, Cand &cd) {
  const unsigned msk = (1u << kPosBits) - 1u;
  const int it = (int)(key >> 63);
  const int i1 = (int)(key >> 42) & msk, i3 = (int)(key >> 21) & msk, i2 = (int)key & msk;
  const double x1 = X[i1], z1 = Z[i1], x2 = X[i2], z2 = Z[i2], x3 = X[i3], z3 = Z[i3];
  const double u1 = z1 - P.zref, g1 = gd(u1, P.d), g2 = gd(z2 - P.zref, P.d), g3 = gd(z3 - P.zref, P.d);
  // model through the three hits: c from the T2 deviation of the T1-T3 chord
  const double r31 = 1.0 / (z3 - z1);
  const double t13 = (x3 - x1) * r31;
  const double k3 = (g2 - g1) - (z2 - z1) * r31 * (g3 - g1);
  double c = ((x2 - x1) - (z2 - z1) * t13) / k3;
  double b = t13 - c * (g3 - g1) * r31;
  double a = x1 - b * u1 - c * g1;
  int pos[6];
  // slots of the initial layers: it 0 -> layers 0, 4, 8 (slots 0, 2, 4)
  const int s1 = it ? 1 : 0, s2 = it ? 3 : 2, s3 = it ? 5 : 4;
#pragma unroll
  for (int k = 0; k < 6; ++k) pos[k] = -1;
  int n = 3;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    if (k == s1) pos[k] = i1;
    else if (k == s2) pos[k] = i2;
    else if (k == s3) pos[k] = i3;
    else if ((k & 1) != it) {
      const int L = xlayer(k);
      const int h = zclosest<kLds>(X, Z, sh, L, xm_layer(a, b, c, L, P), P.ext_tol);
      if (h >= 0) { pos[k] = h; ++n; }
    }
  }
  if (n < P.min_x_hits) return false;
  double chi2;
  int m;
  if (!fit_x(X, Z, pos, P, a, b, c, chi2, m)) return false;
  if (!(chi2 < P.chi2x_max)) return false;
  const double score = (m == 6 ? 1.0 : 10.0) * (1000.0 * chi2 + fabs(c));
  cd.a = a; cd.b = b; cd.c = c; cd.chi2 = chi2;
  cd.score = (unsigned long long)__double_as_longlong(score);
  cd.key = key;
#pragma unroll
  for (int k = 0; k < 6; ++k) cd.pos[k] = pos[k];
  cd.n = m;
  cd.it = it;
  return true;
}

// ---------------------------------------------------------------- UV ------

// One combination of the iterative UV search of Sec. 3.4, FP64: start from
// initial hit h0 of stereo layer L0, predict with t_y from the origin, take
// the closest hit within uv_tol in each of the five other stereo layers in
// ascending z, averaging t_y after each, then fit y = y0 + t_y (z - z_ref)
// with weights tan^2(alpha) / sigma^2.  Returns false if it has too few hits
// or fails the chi2 cut.
template <bool kLds, int NT>
__device__ __forceinline__ bool uv_combo(const float *X, const float *Z, const SeedShared<NT> &sh,
                                         const DevParams &P, double a, double b, double c,
                                         int L0, int h0, Combo &r) {
  const double xh0 = X[h0], zh0 = Z[h0];
  const double t0 = P.tand[L0];
  // a hit at its layer's nominal z (as on the workloads) reuses the layer's
  // x(z) and 1/z; y / z is taken as y * (1/z)
  const bool nom0 = zh0 == P.zd[L0];
  const double y0h = ((nom0 ? xm_layer(a, b, c, L0, P) : xm(a, b, c, zh0, P)) - xh0) * P.inv_tand[L0];
  double ty = y0h * (nom0 ? P.inv_z[L0] : 1.0 / zh0);
  // weighted sums of the line fit, y taken relative to the initial hit's y
  double s0 = t0 * t0, s1 = s0 * (zh0 - P.zref), s2 = s1 * (zh0 - P.zref);
  double q0 = 0.0, q1 = 0.0, q2 = 0.0;
  int n = 1;
#pragma unroll
  for (int k = 0; k < 6; ++k) r.pos[k] = uvlayer(k) == L0 ? h0 : -1;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int L = uvlayer(k);
    if (L == L0) continue;
    const double tl = P.tand[L];
    const double xl = xm_layer(a, b, c, L, P);
    const double pred = xl - ty * P.ztan[L];
    float xhf, zhf;
    const int h = zclosest<kLds>(X, Z, sh, L, pred, P.uv_tol, xhf, zhf);
    if (h < 0) continue;
    const double zh = zhf;
    const bool nom = zh == P.zd[L];
    const double yl = ((nom ? xl : xm(a, b, c, zh, P)) - (double)xhf) * P.inv_tand[L];
    ty = 0.5 * (ty + yl * (nom ? P.inv_z[L] : 1.0 / zh));
    r.pos[k] = h;
    const double w = tl * tl, u = zh - P.zref, yr = yl - y0h;
    s0 += w; s1 += w * u; s2 += w * u * u;
    q0 += w * yr; q1 += w * u * yr; q2 += w * yr * yr;
    ++n;
  }
  if (n < P.min_uv_hits) return false;
  const double det = s0 * s2 - s1 * s1;
  const double idet = 1.0 / det;
  const double fy = (q0 * s2 - q1 * s1) * idet;
  const double ft = (s0 * q1 - s1 * q0) * idet;
  // residual sum of squares of the weighted fit
  const double rss = fmax(q2 - fy * q0 - ft * q1, 0.0);
  const double chi2 = rss * P.inv_sigma2 / (double)(n - 2);
  if (!(chi2 < P.chi2y_max)) return false;
  r.chi2 = chi2;
  r.y0 = fy + y0h;
  r.ty = ft;
  r.n = n;
  return true;
}


// Selection keys of the first kComboLds combinations of an item, kept in LDS
// regions the vote no longer needs: chi2 bits in cscore, (track, hits,
// order) in cpos viewed as three int arrays.
constexpr int kComboLds = kCandLds;
template <int NT>
__device__ __forceinline__ int *combo_keys(SeedShared<NT> &sh) {
  return reinterpret_cast<int *>(&sh.cpos[0][0]);
}
template <int NT>
__device__ __forceinline__ void push_combo(SeedShared<NT> &sh, Combo *combo, int cap, const Combo &r) {
  const unsigned slot = wave_append(&sh.ncombo);
  if (slot < (unsigned)cap) gstore(&combo[slot], r);
  if (slot < (unsigned)kComboLds) {
    int *ck = combo_keys(sh);
    sh.cscore[slot] = (unsigned long long)__double_as_longlong(r.chi2);
    ck[slot] = r.c;
    ck[kComboLds + slot] = r.n;
    ck[2 * kComboLds + slot] = r.tb;
  }
}
static_assert(sizeof(unsigned short) * kCandLds * 6 >= sizeof(int) * 3 * kComboLds,
              "combination keys must fit the candidate position area");

// ------------------------------------------------ Hough-cluster UV ------

// Per-wave LDS of the Hough-cluster UV search (one x-z track per wave).
struct HoughWave {
  int hist[kHoughBins];          // coarse t_y histogram
  long long fsum[64];            // t_y sums of the fine bins, in units of 2^-40
  int fcnt[64];                  // entries of the fine bins
  signed char rank[kHoughBins];  // order of a kept coarse bin, -1 if not kept
};
static_assert((kSeedWG / 64) * sizeof(HoughWave) <= sizeof(double) * kCandLds * 3,
              "Hough per-wave state must fit the UV parameter area");

// float order as int order, and back
__device__ __forceinline__ int zkey(float z) {
  const int b = __float_as_int(z);
  return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float zunkey(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }

// x range of stereo layer L holding every hit whose y = (x(z_hit) - x_hit) /
// tan lies in [ylo, yhi] for a z_hit inside the layer's z span.  x(z) may
// depart from its chord over the span by at most span^2/8 max|x''|.  The
// range is a superset; the exact test is taken hit by hit.
template <int NT>
__device__ __forceinline__ void hough_xrange(const SeedShared<NT> &sh, const DevParams &P, int L,
                                             double a, double b, double c, double ylo,
                                             double yhi, double &lo, double &hi) {
  const double za = zunkey(sh.zlo[L]), zb = zunkey(sh.zhi[L]);
  const double xa = xm(a, b, c, za, P), xb = xm(a, b, c, zb, P);
  const double dz = zb - za, um = fmax(fabs(za - P.zref), fabs(zb - P.zref));
  const double e = 0.125 * dz * dz * fabs(c) * (2.0 + 6.0 * fabs(P.d) * um);
  const double t = P.tand[L], s1 = yhi * t, s2 = ylo * t;
  lo = fmin(xa, xb) - e - fmax(s1, s2);
  hi = fmax(xa, xb) + e - fmin(s1, s2);
  const double slack = 1e-9 * (fabs(lo) + fabs(hi)) + 1e-6;
  lo -= slack;
  hi += slack;
}

// Calls f(L, i) on the lanes of one wave for every hit i of the six stereo
// layers inside the x range of hough_xrange.
template <bool kLds, class F, int NT>
__device__ __forceinline__ void hough_scan(const float *X, const SeedShared<NT> &sh, const DevParams &P,
                                           double a, double b, double c, double ylo, double yhi,
                                           F &&f) {
  const int lane = threadIdx.x & 63;
  for (int k = 0; k < 6; ++k) {
    const int L = uvlayer(k);
    const int e = sh.zoff[L + 1];
    if (sh.zoff[L] == e) continue;
    double lo, hi;
    hough_xrange(sh, P, L, a, b, c, ylo, yhi, lo, hi);
    const int s = zlower<kLds>(X, sh, L, lo);
    for (int i0 = s; i0 < e; i0 += 64) {
      const int i = i0 + lane;
      const bool in = i < e && (double)X[i] <= hi;
      if (in) f(L, i);
      if (__ballot(in) != ~0ull) break;
    }
  }
}

// One t_y hypothesis: the closest hit within uv_tol in every stereo layer,
// then the weighted line fit of uv_combo.
template <bool kLds, int NT>
__device__ __forceinline__ bool hough_attach(const float *X, const float *Z, const SeedShared<NT> &sh,
                                             const DevParams &P, double a, double b, double c,
                                             double ty, Combo &r) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, q0 = 0.0, q1 = 0.0, q2 = 0.0, yref = 0.0;
  int n = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int L = uvlayer(k);
    const double zl = P.zd[L], tl = P.tand[L];
    const double pred = xm(a, b, c, zl, P) - ty * zl * tl;
    float xhf, zhf;
    const int h = zclosest<kLds>(X, Z, sh, L, pred, P.uv_tol, xhf, zhf);
    r.pos[k] = h;
    if (h < 0) continue;
    const double zh = zhf;
    const double yl = (xm(a, b, c, zh, P) - (double)xhf) * P.inv_tand[L];
    if (n == 0) yref = yl;
    const double w = tl * tl, u = zh - P.zref, yr = yl - yref;
    s0 += w; s1 += w * u; s2 += w * u * u;
    q0 += w * yr; q1 += w * u * yr; q2 += w * yr * yr;
    ++n;
  }
  if (n < P.min_uv_hits) return false;
  const double idet = 1.0 / (s0 * s2 - s1 * s1);
  const double fy = (q0 * s2 - q1 * s1) * idet;
  const double ft = (s0 * q1 - s1 * q0) * idet;
  const double rss = fmax(q2 - fy * q0 - ft * q1, 0.0);
  const double chi2 = rss * P.inv_sigma2 / (double)(n - 2);
  if (!(chi2 < P.chi2y_max)) return false;
  r.chi2 = chi2;
  r.y0 = fy + yref;
  r.ty = ft;
  r.n = n;
  return true;
}

// Hough-cluster UV seeding (Sec. 3.4, second variant) of the item's
// surviving x-z tracks, one track per wave: coarse t_y histogram of the
// stereo hits with y in the half, the hough_best most populated bins (ties
// to the lower bin, at least hough_min entries), hough_fine fine bins in
// each, the mean t_y of every non-empty fine bin tried by one lane.  The
// best hypothesis (most hits, lowest chi2_y, earliest) is the track's only
// combination.  Bins are decided in FP64; the fine-bin sums are exact
// fixed-point sums, so the result does not depend on the order of the adds.
template <bool kLds, int NT>
__device__ void uv_hough(const float *X, const float *Z, SeedShared<NT> &sh, const DevParams &P,
                         int half, unsigned nc, const int *cinfo, const Cand *cand, int *bestn,
                         unsigned long long *bestchi, int *bestidx, Combo *combo, int combo_cap) {
#pragma clang fp contract(off)
  static_assert(NT == kSeedWG, "the Hough search keeps one state per wave of a 256-thread workgroup");
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  HoughWave &hw = reinterpret_cast<HoughWave *>(&sh.u.uv.cabc[0][0])[wv];
  if (tid < kNL) {
    sh.zlo[tid] = 0x7fffffff;
    sh.zhi[tid] = -0x7fffffff - 1;
  }
  __syncthreads();
  for (int k = 0; k < 6; ++k) {
    const int L = uvlayer(k);
    for (int i = sh.zoff[L] + tid; i < sh.zoff[L + 1]; i += NT) {
      const int key = zkey(Z[i]);
      atomicMin(&sh.zlo[L], key);
      atomicMax(&sh.zhi[L], key);
    }
  }
  __syncthreads();
  const double ylo = half == 0 ? 0.0 : -P.y_max, yhi = half == 0 ? P.y_max : 0.0;
  const double lo = P.hough_lo[half], hi = P.hough_hi[half];
  const int NB = P.hough_bins, NF = P.hough_fine, NH = P.hough_best * P.hough_fine;
  const double w = (hi - lo) / NB, fw = w / NF;
  constexpr double kFix = 1099511627776.0;   // 2^40
  auto coarse = [&](double t) {
    const int k = (int)floor((t - lo) / w);
    return k < 0 ? 0 : (k >= NB ? NB - 1 : k);
  };
  for (unsigned c0 = 0; c0 < nc; c0 += NT / 64) {
    const unsigned ci = c0 + wv;
    const bool act = ci < nc && !(cinfo[ci] & ((1 << 4) | (1 << 5)));
    double a = 0.0, b = 0.0, c = 0.0;
    if (act) {
      a = gmem(cand)[ci].a; b = gmem(cand)[ci].b; c = gmem(cand)[ci].c;
    }
    for (int i = lane; i < kHoughBins; i += 64) hw.hist[i] = 0;
    hw.fsum[lane] = 0;
    hw.fcnt[lane] = 0;
    if (act && lane == 0) {
      bestn[ci] = 0;
      bestchi[ci] = ~0ull;
      bestidx[ci] = 0x7fffffff;
    }
    __syncthreads();
    if (act)
      hough_scan<kLds>(X, sh, P, a, b, c, ylo, yhi, [&](int L, int i) {
        const double zh = Z[i];
        const double y = (xm(a, b, c, zh, P) - (double)X[i]) / P.tand[L];
        if (y >= ylo && y <= yhi) atomicAdd(&hw.hist[coarse(y / zh)], 1);
      });
    __syncthreads();
    if (act) {
      for (int k = lane; k < NB; k += 64) {
        const int h = hw.hist[k];
        int r = 0;
        for (int j = 0; j < NB; ++j) {
          const int hj = hw.hist[j];
          r += (hj > h) | (hj == h && j < k);
        }
        hw.rank[k] = (h >= P.hough_min && r < P.hough_best) ? (signed char)r : (signed char)-1;
      }
    }
    __syncthreads();
    if (act)
      hough_scan<kLds>(X, sh, P, a, b, c, ylo, yhi, [&](int L, int i) {
        const double zh = Z[i];
        const double y = (xm(a, b, c, zh, P) - (double)X[i]) / P.tand[L];
        if (!(y >= ylo && y <= yhi)) return;
        const double t = y / zh;
        const int k = coarse(t);
        const int r = hw.rank[k];
        if (r < 0) return;
        int f = (int)floor((t - (lo + k * w)) / fw);
        f = f < 0 ? 0 : (f >= NF ? NF - 1 : f);
        atomicAdd(&hw.fcnt[r * NF + f], 1);
        atomicAdd((unsigned long long *)&hw.fsum[r * NF + f],
                  (unsigned long long)(long long)llrint(t * kFix));
      });
    __syncthreads();
    if (act) {
      Combo r;
      bool ok = false;
      if (lane < NH && hw.fcnt[lane] > 0) {
        const double ty = (double)hw.fsum[lane] / kFix / (double)hw.fcnt[lane];
        ok = hough_attach<kLds>(X, Z, sh, P, a, b, c, ty, r);
      }
      int kn = ok ? r.n : 0;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) kn = max(kn, __shfl_xor(kn, o, 64));
      double kc = (ok && r.n == kn) ? r.chi2 : __builtin_inf();
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) kc = fmin(kc, __shfl_xor(kc, o, 64));
      int kh = (ok && r.n == kn && r.chi2 == kc) ? lane : 64;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) kh = min(kh, __shfl_xor(kh, o, 64));
      if (kn > 0 && lane == kh) {
        r.c = (int)ci;
        r.tb = lane;
        push_combo(sh, combo, combo_cap, r);
        bestn[ci] = r.n;
      }
    }
    __syncthreads();
  }
}

// -------------------------------------------------------- seed kernel -----

// Clone killing, UV seeding, best combination and seed staging of one item
// (continuation of seed_item).  kSmall: the vote records, the vote table and
// the UV bookkeeping are in LDS.
template <bool kLds, int kUv, bool kSmall, int NT>
__device__ __forceinline__ void seed_rest(const float *X, const float *Z, const int32_t *hid,
                                          int item, unsigned nc, int nx, const DevParams &P,
                                          const Scratch &S, size_t wg, SeedShared<NT> &sh) {
  const int tid = tidx();
  const int half = item & 1;
  const int *zoff = sh.zoff;
  Counters *cnt = S.cnt;
  Cand *cand = S.cand + wg * (size_t)S.cand_cap;
  SeedStage *sst = S.sst + wg * (size_t)S.sst_cap;
  Combo *combo = S.combo + wg * (size_t)S.combo_cap;
  constexpr bool small = kSmall;
  const size_t co = wg * (size_t)S.cand_cap;
  unsigned long long *cscore = small ? sh.cscore : S.cscore + co;
  int *cinfo = small ? sh.cinfo : S.cinfo + co;
  unsigned long long *xt = small ? sh.u.xtab : S.tbl + wg * (size_t)S.tbl_cap;
  // barriers: in the LDS form the vote records and tables are in LDS, so the
  // barriers up to the UV search order LDS only; the global form keeps
  // __syncthreads throughout
  auto bar = [&]() {
    if constexpr (kSmall) lds_barrier(); else __syncthreads();
  };
  // the global form reads the candidate records written by other threads
  if constexpr (!kSmall) __syncthreads();
  if (!small && nx > S.tbl_cap) {
    if (tid == 0) { raise_flag(cnt, F_TBL); atomicMax(&S.need[2], (unsigned)nx); }
    nc = 0;
  }
  if (!small) {
    for (unsigned i = tid; i < nc; i += NT) {
      cscore[i] = gmem(cand)[i].score;
      cinfo[i] = gmem(cand)[i].n | (gmem(cand)[i].it << 3);
    }
  }
  for (int i = tid; i < nx && nc > 0; i += NT) xt[i] = ~0ull;
  bar();
  // compact x index of the hit in slot k of candidate i, or -1
  auto xidx = [&](unsigned i, int k) -> int {
    const int p = small ? (int)sh.cpos[i][k] - 1 : gmem(cand)[i].pos[k];
    return p < 0 ? -1 : p - zoff[xlayer(k)] + sh.xb[k];
  };

  // O(n) clone killing (Sec. 3.3.4): per-hit minimum score, then own counts
  for (unsigned i = tid; i < nc; i += NT) {
    const unsigned long long sc = cscore[i];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int p = xidx(i, k);
      if (p >= 0) atomicMin(&xt[p], sc);
    }
  }
  bar();
  for (unsigned i = tid; i < nc; i += NT) {
    const unsigned long long sc = cscore[i];
    int own = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int p = xidx(i, k);
      if (p >= 0 && xt[p] == sc) ++own;
    }
    const int n = cinfo[i] & 7;
    const bool kept = own >= 3 || (own >= 2 && n == 6);
    if (!kept) cinfo[i] |= 1 << 4;
    const unsigned long long km = __ballot(kept);
    if (kept && lane_rank(km) == 0) atomicAdd(&sh.nkept, (unsigned)__popcll(km));
  }
  bar();
  // the item's pool range, for the tracks that survived the vote (at least
  // as many as its seeds): its own kPoolPerItem slots, or, for an item with
  // more, a range of the overflow area claimed now (the atomic's latency
  // overlaps the UV search); the range may keep unused slots
  unsigned long long pool_claim = 0;
  if (tid == 0)
    pool_claim = sh.nkept <= (unsigned)kPoolPerItem
                     ? (unsigned long long)item * kPoolPerItem
                     : (unsigned long long)S.pool_static +
                           atomicAdd(&cnt->pool_top, (unsigned long long)sh.nkept);
  // repeated tracks of the two iterations: a kept iteration-1 track whose
  // x-hit set equals a kept iteration-0 track's is dropped.  Equal sets have
  // bit-identical scores, which filters the comparison: one wave takes one
  // iteration-1 track, ballots 64 list entries at a time on the score, and
  // compares hit sets (one slot per lane) only where the score matches.
  if constexpr (kSmall) {
    // LDS records: a hash table keyed by score over the kept iteration-0
    // tracks (in the vote table's LDS, free once own counts are taken), at
    // most half full, so a probe always ends at an empty slot
    constexpr int kHT = 2 * kCandLds;
    static_assert(kHT * (sizeof(unsigned long long) + sizeof(int)) <=
                      kXtabLds * sizeof(unsigned long long), "hash table must fit the vote table");
    unsigned long long *hk = sh.u.xtab;
    int *hv = reinterpret_cast<int *>(sh.u.xtab + kHT);
    auto slot_of = [](unsigned long long k) {
      const unsigned x = (unsigned)(k ^ (k >> 29) ^ (k >> 43)) * 0x9E3779B1u;
      return (int)(x >> 23);   // 9 bits: kHT = 512
    };
    static_assert(kHT == 512, "slot_of takes 9 bits");
    for (int i = tid; i < kHT; i += NT) hk[i] = ~0ull;
    lds_barrier();
    for (unsigned j = tid; j < nc; j += NT) {
      if (cinfo[j] & ((1 << 3) | (1 << 4))) continue;   // kept iteration-0 only
      const unsigned long long sc = cscore[j];
      for (int h = slot_of(sc);; h = (h + 1) & (kHT - 1)) {
        if (atomicCAS(&hk[h], ~0ull, sc) == ~0ull) { hv[h] = (int)j; break; }
      }
    }
    lds_barrier();
    for (unsigned i = tid; i < nc; i += NT) {
      const int ci = cinfo[i];
      if ((ci & (1 << 4)) || !(ci & (1 << 3))) continue;   // kept iteration-1 only
      const unsigned long long sc = cscore[i];
      bool dup = false;
      for (int h = slot_of(sc); !dup; h = (h + 1) & (kHT - 1)) {
        const unsigned long long k = hk[h];
        if (k == ~0ull) break;
        if (k != sc) continue;
        const unsigned j = (unsigned)hv[h];
        bool same = true;
#pragma unroll
        for (int k6 = 0; k6 < 6; ++k6) same = same && xidx(j, k6) == xidx(i, k6);
        dup = same;
      }
      if (dup) cinfo[i] |= 1 << 5;
    }
  } else {
    const int lane = tid & 63;
    for (unsigned i = tid >> 6; i < nc; i += NT / 64) {
      const int ci = cinfo[i];
      if ((ci & (1 << 4)) || !(ci & (1 << 3))) continue;
      const unsigned long long sc = cscore[i];
      const int mine = lane < 6 ? xidx(i, lane) : 0;
      bool dup = false;
      for (unsigned j0 = 0; j0 < nc && !dup; j0 += 64) {
        const unsigned j = j0 + lane;
        const bool cand_j = j < nc && cscore[j] == sc && !(cinfo[j] & ((1 << 3) | (1 << 4)));
        unsigned long long m = __ballot(cand_j);
        while (m != 0ull && !dup) {
          const unsigned jj = j0 + (unsigned)__builtin_ctzll(m);
          m &= m - 1ull;
          const bool differs = lane < 6 && xidx(jj, lane) != mine;
          dup = __ballot(differs) == 0ull;
        }
      }
      if (dup && lane == 0) cinfo[i] |= 1 << 5;
    }
  }
  __syncthreads();

  // UV seeding (Sec. 3.4), one thread per (track, initial hit) combination
  double *cabc = small ? &sh.u.uv.cabc[0][0] : nullptr;
  int *bestn = small ? sh.u.uv.bestn : S.bestn + co;
  unsigned long long *bestchi = small ? sh.u.uv.bestchi : S.bestchi + co;
  int *bestidx = small ? sh.u.uv.bestidx : S.bestidx + co;
  const double ylo = half == 0 ? 0.0 : -P.y_max, yhi = half == 0 ? P.y_max : 0.0;
  if constexpr (kUv == 1)
    uv_hough<kLds>(X, Z, sh, P, half, nc, cinfo, cand, bestn, bestchi, bestidx, combo,
                   S.combo_cap);
  for (unsigned c0 = 0; c0 < nc && kUv == 0; c0 += NT) {
    const unsigned ci = c0 + tid;
    int cnt0 = 0, cnt1 = 0, st0 = 0, st1 = 0;
    if (ci < nc && !(cinfo[ci] & ((1 << 4) | (1 << 5)))) {
      const double a = gmem(cand)[ci].a, b = gmem(cand)[ci].b, c = gmem(cand)[ci].c;
      if (small) { cabc[3 * ci] = a; cabc[3 * ci + 1] = b; cabc[3 * ci + 2] = c; }
#pragma unroll
      for (int pass = 0; pass < 2; ++pass) {
        const int L0 = 1 + pass;
        const double t0 = P.tand[L0];
        const double xp = xm_layer(a, b, c, L0, P);
        const double e1 = xp - yhi * t0, e2 = xp - ylo * t0;
        const double lo = fmin(e1, e2), hi = fmax(e1, e2);
        const int s = zlower<kLds>(X, sh, L0, lo);
        // window end: from the lower bound of hi (bin lookup), past hits equal to hi
        int e = kLds ? zlower<kLds>(X, sh, L0, hi) : s;
        if (e < s) e = s;
        while (e < zoff[L0 + 1] && (double)X[e] <= hi) ++e;
        if (pass == 0) { st0 = s; cnt0 = e - s; } else { st1 = s; cnt1 = e - s; }
      }
      bestn[ci] = 0;
      bestchi[ci] = ~0ull;
      bestidx[ci] = 0x7fffffff;
    }
    int total;
    const int excl = block_excl_scan<NT, kSmall>(cnt0 + cnt1, sh.tmp, total);
    sh.scan[tid] = excl;
    sh.a0[tid] = st0;
    sh.a1[tid] = cnt0;
    sh.a2[tid] = st1;
    for (int d = excl; d < excl + cnt0 + cnt1 && d < kCmap<NT>; ++d) sh.cmap[d] = (SlotMap<NT>)tid;
    bar();
    const int nj = min((int)NT, (int)(nc - c0));
    for (int d0 = 0; d0 < total; d0 += NT) {
      const int d = d0 + tid;
      if (d >= total) continue;
      // the combination's track slot: from the map, else a search of the scan
      int jj;
      if (d < kCmap<NT>) {
        jj = sh.cmap[d];
      } else {
        int lo = 0, hi = nj;
        while (lo < hi) {
          const int m = (lo + hi) >> 1;
          if (sh.scan[m] <= d) lo = m + 1; else hi = m;
        }
        jj = lo - 1;
      }
      const int k = d - sh.scan[jj];
      const int pass = k >= sh.a1[jj];
      const int h0 = pass ? sh.a2[jj] + (k - sh.a1[jj]) : sh.a0[jj] + k;
      const int c = c0 + jj;
      double a, b, cc;
      if (small) { a = cabc[3 * c]; b = cabc[3 * c + 1]; cc = cabc[3 * c + 2]; }
      else { a = gmem(cand)[c].a; b = gmem(cand)[c].b; cc = gmem(cand)[c].c; }
      Combo r;
      if (!uv_combo<kLds>(X, Z, sh, P, a, b, cc, 1 + pass, h0, r)) continue;
      r.c = c;
      r.tb = (pass << 24) | (h0 - zoff[1 + pass]);
      push_combo(sh, combo, S.combo_cap, r);
      atomicMax(&bestn[c], r.n);
    }
    bar();
  }
  unsigned ncb = sh.ncombo;
  // the combinations beyond the LDS key list are read from their global
  // records by other threads below
  if constexpr (kSmall) {
    if (ncb > (unsigned)kComboLds) __syncthreads();
  }
  if (ncb > (unsigned)S.combo_cap) {
    if (tid == 0) { raise_flag(cnt, F_COMBO); atomicMax(&S.need[7], ncb); }
    ncb = S.combo_cap;
  }
  // best combination per track: most hits, then lowest chi2_y, then the
  // earlier (pass, initial hit)
  const int *ck = combo_keys(sh);
  auto key_c = [&](unsigned i) { return i < (unsigned)kComboLds ? ck[i] : gmem(combo)[i].c; };
  auto key_n = [&](unsigned i) { return i < (unsigned)kComboLds ? ck[kComboLds + i] : gmem(combo)[i].n; };
  auto key_tb = [&](unsigned i) {
    return i < (unsigned)kComboLds ? ck[2 * kComboLds + i] : gmem(combo)[i].tb;
  };
  auto key_chi = [&](unsigned i) {
    return i < (unsigned)kComboLds ? sh.cscore[i]
                                   : (unsigned long long)__double_as_longlong(gmem(combo)[i].chi2);
  };
  for (unsigned i = tid; i < ncb; i += NT) {
    const int c = key_c(i);
    if (key_n(i) == bestn[c]) atomicMin(&bestchi[c], key_chi(i));
  }
  // __syncthreads: the winners' records are read by other threads below
  __syncthreads();
  for (unsigned i = tid; i < ncb; i += NT) {
    const int c = key_c(i);
    if (key_n(i) == bestn[c] && key_chi(i) == bestchi[c]) atomicMin(&bestidx[c], key_tb(i));
  }
  bar();
  // the seed record of winning combination i
  auto make_seed = [&](unsigned i) {
    // the track index from the key list, so that the candidate and the
    // combination are read together
    const Cand cd = gload(&cand[key_c(i)]);
    const Combo r = gload(&combo[i]);
    SeedStage st;
    st.key = cd.key;
    st.s.ax = (float)cd.a; st.s.bx = (float)cd.b; st.s.cx = (float)cd.c;
    st.s.y0 = (float)r.y0; st.s.ty = (float)r.ty;
    st.s.chi2_x = (float)cd.chi2; st.s.chi2_y = (float)r.chi2;
    st.s.score = (float)__longlong_as_double((long long)cd.score);
    // the third iteration's seeds carry iteration 2 (its x-z search runs
    // with iteration 0's layers)
    st.s.n_x = cd.n; st.s.n_uv = r.n; st.s.half = half; st.s.iter = cd.it + (sh.pass == 2 ? 2 : 0);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      st.s.hits[xlayer(k)] = cd.pos[k] >= 0 ? hid[cd.pos[k]] : -1;
      st.s.hits[uvlayer(k)] = r.pos[k] >= 0 ? hid[r.pos[k]] : -1;
    }
    if (sh.pass == 1) {
      // clean-up for the third iteration: this seed's hits are used
      auto *u = gmem(S.used) + sh.zabs[0];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        if (cd.pos[k] >= 0) u[cd.pos[k]] = sh.serial;
        if (r.pos[k] >= 0) u[r.pos[k]] = sh.serial;
      }
    }
    return st;
  };
  auto is_winner = [&](unsigned i) {
    const int c = key_c(i);
    return key_n(i) == bestn[c] && key_tb(i) == bestidx[c] && key_chi(i) == bestchi[c];
  };
  auto claim_pool = [&](unsigned ns) {
    if (tid == 0) {
      const unsigned long long b = pool_claim;
      const bool ok = b + ns <= (unsigned long long)S.pool_cap;
      if (!ok) raise_flag(cnt, F_POOL);
      sh.pbase = ok ? b : (unsigned long long)S.pool_cap;   // no writes when full
      // a full pool keeps no seeds of the item (the call grows it and runs
      // the batch again), so no reader looks past it
      S.item_cnt[item] = ok ? (int)ns : 0;
      S.item_base[item] = ok ? (int)b : 0;
    }
  };
  if (ncb <= (unsigned)(NT < kSeedLds ? NT : kSeedLds)) {
    // one combination per thread (and every key fits the LDS key list): each winner publishes its key in LDS, and
    // once the pool range is known writes its record straight to its
    // canonical place (rank of its (iteration, T1, T3, T2) key)
    const bool win = tid < ncb && is_winner(tid);
    unsigned slot = 0;
    SeedStage st;
    if (win) {
      // the candidate and combination records in one round trip; the key
      // (iteration, T1, T3, T2 positions) comes with them
      st = make_seed(tid);
      slot = wave_append(&sh.nseed);
      sh.u.skey[slot] = st.key;
    }
    // LDS only: the keys and the pool range pass through LDS; the records
    // go to the pool for later launches
    lds_barrier();
    const unsigned ns = sh.nseed;
    claim_pool(ns);
    lds_barrier();
    const unsigned long long base = sh.pbase;
    if (win && base + ns <= (unsigned long long)S.pool_cap)
      gstore(&S.pool[base + rank_of(sh.u.skey, ns, st.key, slot)], st.s);
    return;
  }
  for (unsigned i = tid; i < ncb; i += NT) {
    if (!is_winner(i)) continue;
    const SeedStage st = make_seed(i);
    const unsigned slot = wave_append(&sh.nseed);
    if (slot < (unsigned)S.sst_cap) sst[slot] = st;
  }
  __syncthreads();
  unsigned ns = sh.nseed;
  if (ns > (unsigned)S.sst_cap) {
    if (tid == 0) { raise_flag(cnt, F_SST); atomicMax(&S.need[3], ns); }
    ns = S.sst_cap;
  }
  const bool lds_keys = ns <= (unsigned)kSeedLds;
  for (unsigned i = tid; i < ns && lds_keys; i += NT) sh.u.skey[i] = sst[i].key;
  claim_pool(ns);
  __syncthreads();
  const unsigned long long base = sh.pbase;
  if (base + ns <= (unsigned long long)S.pool_cap) {
    // canonical order: rank of each seed's (iteration, T1, T3, T2) key
    for (unsigned i = tid; i < ns; i += NT) {
      const unsigned long long key = lds_keys ? sh.u.skey[i] : sst[i].key;
      unsigned r = 0;
      if (lds_keys)
        r = rank_of(sh.u.skey, ns, key, i);
      else
        for (unsigned j = 0; j < ns; ++j) r += sst[j].key < key;
      gstore(&S.pool[base + r], sst[i].s);
    }
  }
}

// Seeding of one (event, half) item.  kLds: the item's hits are in LDS (with
// the x-bin index); the candidate-side arrays are in LDS whenever they fit,
// else in this workgroup's global scratch.
template <bool kLds, int kUv, int NT>
__device__ __forceinline__ void seed_item(const float *X, const float *Z, const int32_t *hid,
                                          int item, int nh, const DevParams &P,
                                          const Scratch &S, size_t wg, SeedShared<NT> &sh) {
  const int tid = tidx();
  const int half = item & 1;
  const int *zoff = sh.zoff;
  Counters *cnt = S.cnt;
  unsigned long long *trip = S.trip + wg * (size_t)S.trip_cap;
  Cand *cand = S.cand + wg * (size_t)S.cand_cap;
  SeedStage *sst = S.sst + wg * (size_t)S.sst_cap;
  Combo *combo = S.combo + wg * (size_t)S.combo_cap;

  // XZ seeding: two independent iterations (Sec. 3)
  xz_triplets<kLds>(X, Z, sh, P, trip, S.trip_cap);
  unsigned ntrip = sh.ntrip;
  if (ntrip > (unsigned)S.trip_cap) {
    if (tid == 0) { raise_flag(cnt, F_TRIP); atomicMax(&S.need[0], ntrip); }
    ntrip = S.trip_cap;
  }
  for (unsigned t = tid; t < ntrip; t += NT) {
    Cand cd;
    if (xz_candidate<kLds>(X, Z, sh, P, t < (unsigned)kTripLds ? sh.u.xtab[t] : trip[t], cd)) {
      const unsigned slot = wave_append(&sh.ncand);
      if (slot < (unsigned)S.cand_cap) gstore(&cand[slot], cd);
      if (slot < (unsigned)kCandLds) {
        sh.cscore[slot] = cd.score;
        sh.cinfo[slot] = cd.n | (cd.it << 3);
#pragma unroll
        for (int k = 0; k < 6; ++k) sh.cpos[slot][k] = (unsigned short)(cd.pos[k] + 1);
      }
    }
  }
  // LDS only: the candidate records in global memory are read by other
  // threads only after a __syncthreads (the vote's in the global form, the
  // one before the UV search in the LDS form), so their stores complete
  // behind the vote
  lds_barrier();
  unsigned nc = sh.ncand;
  if (nc > (unsigned)S.cand_cap) {
    if (tid == 0) { raise_flag(cnt, F_CAND); atomicMax(&S.need[1], nc); }
    nc = S.cand_cap;
  }
  const int nx = sh.xb[6];
  // vote records and table in LDS when they fit, else in global scratch; the
  // two forms are separate instantiations so that LDS accesses compile to
  // LDS instructions rather than generic ones
  if constexpr (kLds) {
    if (nc <= (unsigned)kCandLds && nx <= kXtabLds)
      seed_rest<true, kUv, true>(X, Z, hid, item, nc, nx, P, S, wg, sh);
    else
      seed_rest<true, kUv, false>(X, Z, hid, item, nc, nx, P, S, wg, sh);
  } else {
    seed_rest<false, kUv, false>(X, Z, hid, item, nc, nx, P, S, wg, sh);
  }
}

// ------------------------------------------------------------ Matching ----

struct PairEval {
  double chi2, zm, dx, dy, dtx, dty, qop;
  bool ok;
};

// One VELO-seed combination (Sec. 4.1-4.2), FP64.
__device__ __forceinline__ PairEval eval_pair(const MState &m, double xv, double yv, double zv,
                                              double txv, double tyv, const DevParams &P) {
  PairEval r;
  r.ok = false;
  const double dtx = m.txs - txv;
  const double zm = P.zm[0] + P.zm[1] * fabs(dtx) + P.zm[2] * dtx * dtx + P.zm[3] * fabs(m.xs) +
                    P.zm[4] * txv * txv;
  const double dx = (m.xs + (zm - P.z_state) * m.txs) - (xv + (zm - zv) * txv);
  const double dy = m.y_m - (yv + tyv * (P.z_ymatch - zv));
  const double dty = m.ty - tyv;
  r.zm = zm; r.dx = dx; r.dy = dy; r.dtx = dtx; r.dty = dty;
  r.chi2 = 0.0; r.qop = 0.0;
  if (!(fabs(dx) < P.max_dx && fabs(dy) < P.max_dy && fabs(dtx) < P.max_dtx &&
        fabs(dty) < P.max_dty))
    return r;
  const double tolx = P.tolx_scale * (P.tolx_a * P.tolx_a + P.tolx_b * P.tolx_b * dtx * dtx);
  const double rho = txv * txv + tyv * tyv;
  const double toly = P.toly_scale * (P.toly_a * P.toly_a + P.toly_b * P.toly_b * rho);
  r.chi2 = dx * dx / tolx + dy * dy / toly + dtx * dtx / P.tol_tx + dty * dty / P.tol_ty;
  if (!(r.chi2 < P.chi2m_max)) return r;
  // momentum from the kick: eq. invp on the z = 0 distance of the two lines
  const double x0 = m.x0s - (xv - zv * txv);
  const double ip = P.invp_a * fabs(x0) + P.invp_b * x0 * x0;
  r.qop = (x0 >= 0.0 ? -1.0 : 1.0) * P.polarity * ip;
  r.ok = true;
  return r;
}

// Ghost probability of one surviving pair (Sec. 4.4), FP64: the eight
// inputs (z_match, dx, dy, dtx, dty, chi2_match, eta of the VELO state, the
// seed's hit count) standardised, one hidden layer of rectified units, a
// logistic output.  eta = asinh(1 / tan theta), tan theta = sqrt(tx^2 + ty^2)
// floored at 1e-9.
__device__ __forceinline__ double ghost_prob(const PairEval &r, double txv, double tyv,
                                             int nhits, const DevParams &P) {
  const double f[SM_NN_INPUTS] = {r.zm, r.dx, r.dy, r.dtx, r.dty, r.chi2,
                                  asinh(1.0 / fmax(sqrt(txv * txv + tyv * tyv), 1e-9)),
                                  (double)nhits};
  double x[SM_NN_INPUTS];
#pragma unroll
  for (int i = 0; i < SM_NN_INPUTS; ++i) x[i] = (f[i] - P.nn_mean[i]) / P.nn_scale[i];
  double out = P.nn_b2;
  // one hidden unit per trip: unrolled, the 256 weights' loads and products
  // would hold registers that the rest of the matching kernel needs
#pragma unroll 1
  for (int j = 0; j < SM_NN_HIDDEN; ++j) {
    double h = P.nn_b1[j];
#pragma unroll
    for (int i = 0; i < SM_NN_INPUTS; ++i) h += P.nn_w1[j][i] * x[i];
    out += P.nn_w2[j] * (h > 0.0 ? h : 0.0);
  }
  return 1.0 / (1.0 + exp(-out));
}

// from the seed's x-z parameters and its y line (the only fields read)
__device__ __forceinline__ MState seed_state(const sm_seed *s, const DevParams &P) {
  MState m;
  const auto *g = gmem(s);
  const double a = g->ax, b = g->bx, c = g->cx, y0 = g->y0, ty = g->ty;
  const double us = P.z_state - P.zref;
  m.xs = a + b * us + c * gd(us, P.d);
  m.txs = b + c * (2.0 * us + 3.0 * P.d * us * us);
  m.y_m = y0 + ty * (P.z_ymatch - P.zref);
  m.ty = ty;
  m.x0s = m.xs - P.z_state * m.txs;
  m.xsf = (float)m.xs; m.txsf = (float)m.txs; m.y_mf = (float)m.y_m; m.tyf = (float)m.ty;
  return m;
}

// ---------------------------------------------------------- UT search ----

// Half-width of a UT window (Table 2): kind 0 loose, 1 tight; 0 where the
// layer has none.  min(max(a + b / p, lo), hi), p in GeV/c.
__device__ __forceinline__ double ut_window(const DevParams &P, int kind, int i, double qop) {
  const double hi = P.ut_hi[kind][i];
  if (!(hi > 0.0)) return 0.0;
  return fmin(fmax(P.ut_a[kind][i] + P.ut_b[kind][i] * 1000.0 * fabs(qop), P.ut_lo[kind][i]), hi);
}

// Closest hit to pred among positions [lo, hi) of an x-sorted layer, inside
// [pred - w, pred + w]; distances within kTieMm are a tie won by the lower
// position.  X(h): the hit's x.  -1 if none.
template <class FX>
__device__ __forceinline__ int ut_closest(FX X, int lo, int hi, double pred, double w) {
  const double xlo = pred - w, xhi = pred + w;
  int a = lo, b = hi;
  while (a < b) {
    const int m = (a + b) >> 1;
    if ((double)X(m) < xlo) a = m + 1; else b = m;
  }
  int best = -1;
  double bd = 0.0;
  for (int h = a; h < hi; ++h) {
    const double x = (double)X(h);
    if (!(x <= xhi)) break;
    const double d = fabs(x - pred);
    if (best < 0 || d < bd - kTieMm) { best = h; bd = d; }
  }
  return best;
}

// UT hits of one VELO-seed pair (Sec. 4.3): the VELO state extrapolated with
// eq. velo_ut_extrapolation (from the state's own z), gamma_x from eq.
// gamma_parametrisation with the pair's q/p, compared with the layer's
// measured coordinate x - y tan(alpha).  Until a hit is found each layer's
// loose window is searched; the closest hit found there refits gamma_x so
// that the parabola passes through it, and every later layer takes the
// closest hit in its tight window.  uo: the event's layer offsets into X/ID.
// Returns the number of hits attached, their ids in ids (-1 where none).
template <class FX, class FI>
__device__ __forceinline__ int ut_search(const DevParams &P, FX X, FI ID,
                                         const int (&uo)[SM_N_UT + 1], double xv, double yv,
                                         double zv, double txv, double tyv, double qop,
                                         int32_t (&ids)[SM_N_UT]) {
  double gam = P.a_gamma + P.b_gamma * qop;
  bool loose = true;
  int n = 0;
#pragma unroll
  for (int i = 0; i < SM_N_UT; ++i) {
    ids[i] = -1;
    const double w = ut_window(P, loose ? 0 : 1, i, qop);
    if (!(w > 0.0)) continue;
    const double dz = P.ut_z[i] - zv;
    const double yp = yv + tyv * dz;
    const double mp = xv + txv * dz + gam * dz * dz - yp * P.ut_tan[i];
    const int h = ut_closest(X, uo[i], uo[i + 1], mp, w);
    if (h < 0) continue;
    ids[i] = ID(h);
    ++n;
    if (loose) {
      const double xh = (double)X(h) + yp * P.ut_tan[i];
      gam = (xh - xv - txv * dz) / (dz * dz);
      loose = false;
    }
  }
  return n;
}

struct MatchShared {
  // per-seed prefilter state; after the prefilter pass it holds the event's
  // UT hits (x, then id) in the UT search variant
  float xsf[kMsLds], txsf[kMsLds], ymf[kMsLds], tyf[kMsLds], sty[kMsLds];
  int sidx[kMsLds];
  unsigned long long best_s[kMsLds];
  unsigned long long best_v[kVsLds];
  Surv surv[kSurvLds];
  unsigned long long kkey[kSurvLds];
  // flattened pair search: VELO states of the event, their window starts and
  // the scan of the window sizes
  float vx[kVflat], vy[kVflat], vz[kVflat], vtx[kVflat], vty[kVflat];
  int vk0[kVflat], vscan[kVflat];
  unsigned char pv[kPvLds];   // VELO state of each flattened pair
  int tmp[16];
  int ev;
  unsigned nsurv, nkeep, nplist;
  unsigned long long lbase;
};
// the UT hits' LDS home: the six per-seed prefilter arrays, contiguous
static_assert(offsetof(MatchShared, sidx) == offsetof(MatchShared, xsf) + 5 * kMsLds * sizeof(float) &&
                  2 * kUtLds * sizeof(float) == 6 * kMsLds * sizeof(float),
              "the UT hits overlay xsf .. sidx");

// zone offsets non-decreasing from 0, hits x-sorted inside each zone
__global__ __launch_bounds__(256) void k_validate(const Desc *__restrict__ D, const KCtx *__restrict__ K) {
  const Scratch &S = K->S;
  const int nz = D->n_events * 24;
  const int32_t *zo = D->b.zone_off;
  const float *x = D->b.hit_x;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nz; k += gridDim.x * blockDim.x) {
    if ((k == 0 && zo[0] != 0) || zo[k + 1] < zo[k]) {
      raise_flag(S.cnt, F_INVALID);
      continue;
    }
    for (int i = zo[k] + 1; i < zo[k + 1]; ++i)
      if (!(x[i] >= x[i - 1])) { raise_flag(S.cnt, F_UNSORTED); break; }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const int32_t *vo = D->b.velo_off;
    for (int e = 0; e < D->n_events; ++e)
      if (vo[e + 1] < vo[e]) { raise_flag(S.cnt, F_INVALID); break; }
    if (D->n_events > 0 && vo[0] != 0) raise_flag(S.cnt, F_INVALID);
  }
}

// Matching of one event (Sec. 4), run by the workgroup that completes the
// second half of the event.  plain: outputs go straight to the caller's
// buffers at offsets chained from the previous event; batched: long tracks go
// to the pool and the seeds stay in theirs until the offsets are known.
// kSmallM: the event's seeds and VELO states fit the LDS arrays, which the
// instantiation then addresses as LDS (not through generic pointers).  kSel:
// bit 0 the network form of the final selection, bit 1 the UT search (each
// variant an instantiation of its own, so that the default one carries none
// of their registers or LDS).
template <bool kSmallM, int NT, int kSel, bool kMk = false>
__device__ __forceinline__ void match_event_impl(const Desc *__restrict__ D, const Scratch &S,
                                                 const DevParams &P, int e, int plain, size_t wg,
                                                 MatchShared &sh) {
  const int tid = tidx();
  MState *ms = S.ms + wg * (size_t)S.ms_cap;
  float *mf = S.mf + wg * (size_t)S.ms_cap * 6;
  Counters *cnt = S.cnt;
  if (tid == 0) {
    sh.nsurv = 0;
    sh.nkeep = 0;
    sh.nplist = 0;
  }
  const int n0 = gmem(S.item_cnt)[2 * e], n1 = gmem(S.item_cnt)[2 * e + 1];
  const int b0 = gmem(S.item_base)[2 * e], b1 = gmem(S.item_base)[2 * e + 1];
  // with the third iteration, its seeds of the event follow (both halves)
  const bool t3 = D->pass == 1;
  const int n2 = t3 ? gmem(S.item_cnt3)[2 * e] : 0, n3 = t3 ? gmem(S.item_cnt3)[2 * e + 1] : 0;
  const int b2 = t3 ? gmem(S.item_base3)[2 * e] : 0, b3 = t3 ? gmem(S.item_base3)[2 * e + 1] : 0;
  const int ns = n0 + n1 + n2 + n3;
  // the event's seed i, in this order: half 0, half 1, then the third
  // iteration's half 0, half 1
  auto seed_at = [&](int i) -> const sm_seed * {
    if (i < n0) return &S.pool[b0 + i];
    if (i < n0 + n1) return &S.pool[b1 + i - n0];
    if (i < n0 + n1 + n2) return &S.pool3[b2 + i - n0 - n1];
    return &S.pool3[b3 + i - n0 - n1 - n2];
  };
  const int v0 = gmem(D->b.velo_off)[e], nv = gmem(D->b.velo_off)[e + 1] - v0;
  // the matching kernel (kMk) with mseeds: the event's seeds go to the
  // caller from here, after every earlier event's seeds; each wave's share
  // of that count is in sh.tmp[8 + wave] (free of the block scans) until the
  // end
  const bool mseeds = kMk && NT <= 512 && !plain && D->mseeds != 0;
  if (mseeds) {
    int sp = 0;
    for (int j = tid; j < e; j += NT) {
      sp += gmem(S.item_cnt)[2 * j] + gmem(S.item_cnt)[2 * j + 1];
      if (t3) sp += gmem(S.item_cnt3)[2 * j] + gmem(S.item_cnt3)[2 * j + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sp += __shfl_xor(sp, o, 64);
    if ((tid & 63) == 0) sh.tmp[8 + (tid >> 6)] = sp;
  }
  const bool pool_ok = !(cnt->flags & F_POOL);
  const int so = plain ? D->seed_off[e] : 0;
  if (tid == 0 && plain) D->seed_off[e + 1] = so + ns;
  const bool fits = ns <= S.ms_cap && nv <= S.vs_cap && pool_ok;
  if (tid == 0 && !fits && pool_ok) {
    if (ns > S.ms_cap) { raise_flag(cnt, F_MS); atomicMax(&S.need[4], (unsigned)ns); }
    if (nv > S.vs_cap) { raise_flag(cnt, F_VS); atomicMax(&S.need[5], (unsigned)nv); }
  }
  // per-seed arrays in LDS, or in this workgroup's global scratch for events
  // with many seeds / VELO states
  const bool sm_s = kSmallM || ns <= kMsLds, sm_v = kSmallM || nv <= kVsLds;
  float *xsf = sm_s ? sh.xsf : mf, *txsf = sm_s ? sh.txsf : mf + S.ms_cap;
  float *ymf = sm_s ? sh.ymf : mf + 2 * (size_t)S.ms_cap;
  float *tyf = sm_s ? sh.tyf : mf + 3 * (size_t)S.ms_cap;
  float *sty = sm_s ? sh.sty : mf + 4 * (size_t)S.ms_cap;
  int *sidx = sm_s ? sh.sidx : (int *)(mf + 5 * (size_t)S.ms_cap);
  unsigned long long *best_s = sm_s ? sh.best_s : S.best_s + wg * (size_t)S.ms_cap;
  unsigned long long *best_v = sm_v ? sh.best_v : S.best_v + wg * (size_t)S.vs_cap;
  // VELO states of the event for the flattened pair search, loaded here so
  // that the loads overlap the seed loads below
  const bool vlds = fits && ns > 0 && kSmallM && nv <= kVflat && nv <= NT;
  float vxr = 0.0f, vyr = 0.0f, vzr = 0.0f, vtxr = 0.0f, vtyr = 0.0f;
  if (vlds && tid < nv) {
    vxr = gmem(D->b.velo_x)[v0 + tid];
    vyr = gmem(D->b.velo_y)[v0 + tid];
    vzr = gmem(D->b.velo_z)[v0 + tid];
    vtxr = gmem(D->b.velo_tx)[v0 + tid];
    vtyr = gmem(D->b.velo_ty)[v0 + tid];
  }
  // UT search variant: the event's UT layer offsets (into the batch's UT
  // arrays until the hits are staged in LDS, see below)
  constexpr bool kUt = (kSel & 2) != 0;
  int ut_o[SM_N_UT + 1] = {};
  bool ut_lds = false;
  float *ut_xs = sh.xsf;
  int32_t *ut_ids = reinterpret_cast<int32_t *>(sh.xsf + kUtLds);
  if constexpr (kUt) {
#pragma unroll
    for (int k = 0; k <= SM_N_UT; ++k) ut_o[k] = gmem(D->b.ut_off)[(size_t)e * SM_N_UT + k];
  }
  // UT hits of a pair (its q/p from the evaluation)
  auto ut_of = [&](double xv, double yv, double zv, double txv, double tyv, double qop,
                   int32_t (&ids)[SM_N_UT]) {
    if (ut_lds)
      return ut_search(P, [&](int h) { return ut_xs[h]; }, [&](int h) { return ut_ids[h]; }, ut_o,
                       xv, yv, zv, txv, tyv, qop, ids);
    return ut_search(P, [&](int h) { return gmem(D->b.ut_x)[h]; },
                     [&](int h) { return gmem(D->b.ut_id)[h]; }, ut_o, xv, yv, zv, txv, tyv, qop,
                     ids);
  };
  // the event's seeds in canonical order (half 0 then half 1); the plain form
  // copies whole records to the caller, matching reads five fields of each
  if (plain)
    for (int i = tid; i < ns && pool_ok; i += NT)
      if ((long long)so + i < D->seed_cap) D->seeds[so + i] = *seed_at(i);
  for (int i = tid; i < ns && pool_ok && fits; i += NT) {
    const MState m = seed_state(seed_at(i), P);
    gstore(&ms[i], m);
    xsf[i] = m.xsf; txsf[i] = m.txsf; ymf[i] = m.y_mf; tyf[i] = m.tyf;
    best_s[i] = ~0ull;
  }
  // LDS only when the per-seed arrays are in LDS: the seed states' global
  // records are read by other threads only after the __syncthreads that ends
  // the t_y order, so their stores complete behind the sort
  if (sm_s) lds_barrier(); else __syncthreads();
  // seeds sorted by t_y (ties by index), so each VELO state visits only its
  // |dty| window.  Up to 256 seeds: each wave sorts 64 (t_y, index) keys in
  // registers (bitonic, lane exchanges), and a key's place is its place in
  // its wave plus, by binary search, the keys below it in the other waves'
  // sorted runs (in the final selection's key space, free until then).  More
  // seeds: each seed's rank among all.
  if (fits && ns <= 256) {
    unsigned long long *run = sh.kkey;
    static_assert(kSurvLds >= 256, "four sorted runs of 64 keys");
    const int lane = tid & 63, w = tid >> 6, nrun = (ns + 63) >> 6;
    if (tid < 256) {
      unsigned long long k = ~0ull;   // past the seeds: sorts last
      if (tid < ns) {
        float t = tyf[tid];
        if (t == 0.0f) t = 0.0f;      // -0 and +0 tie, as they compare
        unsigned b = __float_as_uint(t);
        b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);   // float order as unsigned order
        k = ((unsigned long long)b << 32) | (unsigned)tid;
      }
#pragma unroll
      for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
          const unsigned long long o = __shfl_xor(k, stride, 64);
          const bool keep_min = ((lane & stride) == 0) == ((lane & size) == 0);
          k = keep_min ? (o < k ? o : k) : (o > k ? o : k);
        }
      }
      if (w < nrun) run[tid] = k;
    }
    lds_barrier();
    if (tid < 256 && w < nrun) {
      const unsigned long long k = run[tid];
      if (k != ~0ull) {
        unsigned r = (unsigned)lane;
        int lo[4] = {0, 0, 0, 0}, hi[4] = {64, 64, 64, 64};
        // lower bound in each other run: seven halvings of 64
#pragma unroll
        for (int step = 0; step < 7; ++step) {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            if (c < nrun && c != w && lo[c] < hi[c]) {
              const int m = (lo[c] + hi[c]) >> 1;
              if (run[c * 64 + m] < k) lo[c] = m + 1; else hi[c] = m;
            }
          }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) r += (c < nrun && c != w) ? (unsigned)lo[c] : 0u;
        const unsigned b = (unsigned)(k >> 32);
        sty[r] = __uint_as_float((b & 0x80000000u) ? (b & 0x7fffffffu) : ~b);
        sidx[r] = (int)(unsigned)k;
      }
    }
  } else if (fits) {
    for (int i = tid; i < ns; i += NT) {
      const float t = tyf[i];
      const int r = (int)rank_of(tyf, (unsigned)ns, t, (unsigned)i);
      sty[r] = t;
      sidx[r] = i;
    }
  }
  __syncthreads();
  Surv *surv = S.surv + wg * (size_t)(2 * S.surv_cap);
  // one pair test: the FP32 prefilter, then the FP64 evaluation
  auto prefilter = [&](int s, float xvf, float yvf, float zvf, float txvf, float tyvf) {
    const float yvm = yvf + tyvf * (P.z_ymatchf - zvf);
    const float dtx = txsf[s] - txvf;
    if (!(fabsf(dtx) < P.pre_dtx)) return false;
    if (!(fabsf(ymf[s] - yvm) < P.pre_dy)) return false;
    const float zm = P.zmf[0] + P.zmf[4] * txvf * txvf + P.zmf[1] * fabsf(dtx) +
                     P.zmf[2] * dtx * dtx + P.zmf[3] * fabsf(xsf[s]);
    const float dx = (xsf[s] + (zm - P.z_statef) * txsf[s]) - (xvf + (zm - zvf) * txvf);
    return fabsf(dx) < P.pre_dx;
  };
  auto evaluate = [&](int v, int s, float xvf, float yvf, float zvf, float txvf, float tyvf,
                      unsigned long long &bits) {
    const PairEval r = eval_pair(gload(&ms[s]), xvf, yvf, zvf, txvf, tyvf, P);
    if (!r.ok) return false;
    if constexpr (kUt) {
      // Sec. 4.3: more than two UT hits (ut_min_hits) or the pair leaves
      int32_t ids[SM_N_UT];
      if (ut_of(xvf, yvf, zvf, txvf, tyvf, r.qop, ids) < P.ut_min_hits) return false;
    }
    bits = (unsigned long long)__double_as_longlong(r.chi2);
    atomicMin(&best_s[s], bits);
    const unsigned slot = atomicAdd(&sh.nsurv, 1u);
    if (slot < (unsigned)kSurvLds) sh.surv[slot] = Surv{v, s, r.chi2};
    else if (slot < (unsigned)(kSurvLds + S.surv_cap)) gstore(&surv[slot - kSurvLds], Surv{v, s, r.chi2});
    return true;
  };
  auto test_pair = [&](int v, int s, float xvf, float yvf, float zvf, float txvf, float tyvf,
                       unsigned long long &bits) {
    return prefilter(s, xvf, yvf, zvf, txvf, tyvf) &&
           evaluate(v, s, xvf, yvf, zvf, txvf, tyvf, bits);
  };
  if (vlds) {
    // every (VELO state, seed in its t_y window) pair gets its own thread:
    // window bounds per VELO state, a scan of the window sizes, then the
    // pairs in rounds of NT
    int cnt_v = 0;
    if (tid < nv) {
      const int v = tid;
      const float tyvf = vtyr;
      sh.vx[v] = vxr;
      sh.vy[v] = vyr;
      sh.vz[v] = vzr;
      sh.vtx[v] = vtxr;
      sh.vty[v] = tyvf;
      const int k0 = lower_f(sty, 0, ns, tyvf - P.pre_dty);
      const int k1 = upper_f(sty, k0, ns, tyvf + P.pre_dty);
      sh.vk0[v] = k0;
      cnt_v = k1 - k0;
      best_v[v] = ~0ull;
    }
    int total;
    const int ex = block_excl_scan<NT>(cnt_v, sh.tmp, total);
    if (tid < nv) {
      sh.vscan[tid] = ex;
      // the VELO state of each of its pairs (the first kPvLds pairs)
      for (int d = ex; d < ex + cnt_v && d < kPvLds; ++d) sh.pv[d] = (unsigned char)tid;
    }
    __syncthreads();
    // pass 1, LDS only: the FP32 prefilter; passing pairs are listed (in the
    // final-selection keys' space, free until then) for pass 2, or evaluated
    // at once if the list is full
    unsigned *plist = reinterpret_cast<unsigned *>(sh.kkey);
    constexpr unsigned kPlist = sizeof(sh.kkey) / sizeof(unsigned);
    for (int d0 = 0; d0 < total; d0 += NT) {
      const int d = d0 + tid;
      if (d >= total) continue;
      int v;
      if (d < kPvLds) {
        v = sh.pv[d];
      } else {
        int lo = 0, hi = nv;
        while (lo < hi) {
          const int m = (lo + hi) >> 1;
          if (sh.vscan[m] <= d) lo = m + 1; else hi = m;
        }
        v = lo - 1;
      }
      const int s = sidx[sh.vk0[v] + (d - sh.vscan[v])];
      if (!prefilter(s, sh.vx[v], sh.vy[v], sh.vz[v], sh.vtx[v], sh.vty[v])) continue;
      const unsigned slot = wave_append(&sh.nplist);
      unsigned long long bits;
      if (slot < kPlist) plist[slot] = ((unsigned)v << 16) | (unsigned)s;
      else if (evaluate(v, s, sh.vx[v], sh.vy[v], sh.vz[v], sh.vtx[v], sh.vty[v], bits))
        atomicMin(&best_v[v], bits);
    }
    __syncthreads();
    if constexpr (kUt) {
      // the prefilter's per-seed arrays are dead from here on: the event's UT
      // hits move into them when they fit (offsets then relative to the
      // first), so that the searches of pass 2 and of the output read LDS
      const int nu = ut_o[SM_N_UT] - ut_o[0];
      if (nu <= kUtLds) {
        const int u0 = ut_o[0];
        for (int i = tid; i < nu; i += NT) {
          ut_xs[i] = gmem(D->b.ut_x)[u0 + i];
          ut_ids[i] = gmem(D->b.ut_id)[u0 + i];
        }
#pragma unroll
        for (int k = 0; k <= SM_N_UT; ++k) ut_o[k] -= u0;
        ut_lds = true;
        __syncthreads();
      }
    }
    // pass 2: the FP64 evaluation of the listed pairs
    const unsigned np = sh.nplist < kPlist ? sh.nplist : kPlist;
    for (unsigned i = tid; i < np; i += NT) {
      const unsigned w = plist[i];
      const int v = (int)(w >> 16), s = (int)(w & 0xffffu);
      unsigned long long bits;
      if (evaluate(v, s, sh.vx[v], sh.vy[v], sh.vz[v], sh.vtx[v], sh.vty[v], bits))
        atomicMin(&best_v[v], bits);
    }
  } else if (fits && ns > 0) {
    for (int v = tid; v < nv; v += NT) {
      const float xvf = gmem(D->b.velo_x)[v0 + v], yvf = gmem(D->b.velo_y)[v0 + v],
                  zvf = gmem(D->b.velo_z)[v0 + v];
      const float txvf = gmem(D->b.velo_tx)[v0 + v], tyvf = gmem(D->b.velo_ty)[v0 + v];
      unsigned long long bv = ~0ull;
      const float thi = tyvf + P.pre_dty;
      for (int k = lower_f(sty, 0, ns, tyvf - P.pre_dty); k < ns && sty[k] <= thi; ++k) {
        unsigned long long bits;
        if (test_pair(v, sidx[k], xvf, yvf, zvf, txvf, tyvf, bits)) bv = bits < bv ? bits : bv;
      }
      best_v[v] = bv;
    }
  }
  __syncthreads();
  unsigned nsv = sh.nsurv;
  if (nsv > (unsigned)(kSurvLds + S.surv_cap)) {
    if (tid == 0) { raise_flag(cnt, F_SURV); atomicMax(&S.need[6], nsv - kSurvLds); }
    nsv = kSurvLds + S.surv_cap;
  }
  // the seed's hit count and the VELO state's slopes, for the network
  auto nhits_of = [&](int si) {
    const sm_seed *sd = seed_at(si);
    return gmem(sd)->n_x + gmem(sd)->n_uv;
  };
  // a pair's evaluation and its VELO state (x, y, z, tx, ty)
  auto pair_of = [&](int vi, int si, double (&vs)[5]) {
    const int v = v0 + vi;
    if (vlds) {
      vs[0] = sh.vx[vi]; vs[1] = sh.vy[vi]; vs[2] = sh.vz[vi]; vs[3] = sh.vtx[vi]; vs[4] = sh.vty[vi];
    } else {
      vs[0] = gmem(D->b.velo_x)[v]; vs[1] = gmem(D->b.velo_y)[v]; vs[2] = gmem(D->b.velo_z)[v];
      vs[3] = gmem(D->b.velo_tx)[v]; vs[4] = gmem(D->b.velo_ty)[v];
    }
    return eval_pair(gload(&ms[si]), vs[0], vs[1], vs[2], vs[3], vs[4], P);
  };
  constexpr bool nnsel = (kSel & 1) != 0;
  if (nnsel && fits) {
    // the network form (Sec. 4.4): each survivor's ghost probability replaces
    // its chi2 in the list; the retained ones (below the cut) give the lowest
    // ghost probability on each seed and each VELO state
    for (int i = tid; i < ns; i += NT) best_s[i] = ~0ull;
    for (int i = tid; i < nv; i += NT) best_v[i] = ~0ull;
    __syncthreads();
    for (unsigned i = tid; i < nsv; i += NT) {
      Surv sv = i < (unsigned)kSurvLds ? sh.surv[i] : gload(&surv[i - kSurvLds]);
      double vs[5];
      const PairEval pe = pair_of(sv.v, sv.s, vs);
      sv.chi2 = ghost_prob(pe, vs[3], vs[4], nhits_of(sv.s), P);
      if (i < (unsigned)kSurvLds) sh.surv[i] = sv;
      else gstore(&surv[i - kSurvLds], sv);
      if (sv.chi2 < P.ghost_cut) {
        const unsigned long long bits = (unsigned long long)__double_as_longlong(sv.chi2);
        atomicMin(&best_v[sv.v], bits);
        atomicMin(&best_s[sv.s], bits);
      }
    }
    __syncthreads();
  }
  // final selection.  chi2 form: a pair survives if its chi2 is the best of
  // its seed and of its VELO track.  Network form: a retained pair survives
  // unless a retained pair on its seed or its VELO track has a ghost
  // probability lower by the clone gap or more.
  unsigned long long *kkey =
      nsv <= (unsigned)kSurvLds ? sh.kkey : (unsigned long long *)(surv + S.surv_cap);
  // The long tracks go out in (VELO state, seed) order.  When the event's
  // VELO states fit one per thread, a key's place is the count of kept pairs
  // on lower VELO states (a count per state and its scan, in the pair
  // search's window arrays, free now) plus, on a state with several (exact
  // chi2 ties, or the network form), the count of its lower seeds; else the
  // key's rank among all keys.
  const bool vrank = nv <= kVflat && nv <= NT;
  int *vcnt = sh.vk0, *vbase = sh.vscan;
  if (vrank && tid < nv) vcnt[tid] = 0;
  for (unsigned i = tid; i < nsv; i += NT) {
    const Surv sv = i < (unsigned)kSurvLds ? sh.surv[i] : gload(&surv[i - kSurvLds]);
    const unsigned long long bits = (unsigned long long)__double_as_longlong(sv.chi2);
    bool keep;
    if (nnsel) {
      const double g = sv.chi2;
      keep = g < P.ghost_cut &&
             g - __longlong_as_double((long long)best_v[sv.v]) < P.clone_gap &&
             g - __longlong_as_double((long long)best_s[sv.s]) < P.clone_gap;
    } else {
      keep = best_v[sv.v] == bits && best_s[sv.s] == bits;
    }
    if (keep) {
      const unsigned slot = atomicAdd(&sh.nkeep, 1u);
      kkey[slot] = ((unsigned long long)sv.v << 32) | (unsigned)sv.s;
    }
  }
  __syncthreads();
  const unsigned nk = sh.nkeep;
  if (vrank)
    for (unsigned i = tid; i < nk; i += NT) atomicAdd(&vcnt[(int)(kkey[i] >> 32)], 1);
  if (tid == 0) {
    if (plain) {
      const long long lo = D->long_off[e];
      sh.lbase = (unsigned long long)lo;
      D->long_off[e + 1] = (int)(lo + nk);
    } else {
      // a VELO state is in at most one long track unless chi2 values tie
      // exactly, so the event's long tracks go to its VELO range of the pool;
      // an event with more goes to the overflow area after all VELO states
      const unsigned long long b =
          nk <= (unsigned)nv ? (unsigned long long)v0
                             : (unsigned long long)D->b.n_velo +
                                   atomicAdd(&cnt->lpool_top, (unsigned long long)nk);
      if (b + nk > (unsigned long long)S.lpool_cap) raise_flag(cnt, F_LPOOL);
      sh.lbase = b;
      S.ev_lcnt[e] = (int)nk;
      S.ev_lbase[e] = (int)(b < (unsigned long long)S.lpool_cap ? b : 0);
    }
  }
  __syncthreads();
  if (vrank) {
    int total;
    const int ex = block_excl_scan<NT, true>(tid < nv ? vcnt[tid] : 0, sh.tmp, total);
    if (tid < nv) vbase[tid] = ex;
    lds_barrier();
  }
  const unsigned long long lb = sh.lbase;
  const long long cap = plain ? D->long_cap : S.lpool_cap;
  sm_long *dst = plain ? D->longs : S.lpool;
  for (unsigned i = tid; i < nk; i += NT) {
    const unsigned long long key = kkey[i];
    unsigned r;
    if (vrank) {
      const unsigned vk = (unsigned)(key >> 32);
      r = (unsigned)vbase[vk];
      if (vcnt[vk] > 1)
        for (unsigned j = 0; j < nk; ++j) {
          const unsigned long long u = kkey[j];
          r += (unsigned)((u >> 32) == vk && u < key);
        }
    } else {
      r = rank_of(kkey, nk, key, i);
    }
    if ((long long)(lb + r) >= cap) continue;
    const int vi = (int)(key >> 32), si = (int)(key & 0xffffffffu);
    const int v = v0 + vi;
    double vs[5];
    const PairEval pe = pair_of(vi, si, vs);
    sm_long L;
    L.velo_idx = vi; L.seed_idx = si; L.velo_id = gmem(D->b.velo_id)[v];
    L.qop = (float)pe.qop; L.chi2 = (float)pe.chi2; L.z_match = (float)pe.zm;
    L.dx = (float)pe.dx; L.dy = (float)pe.dy; L.dtx = (float)pe.dtx; L.dty = (float)pe.dty;
    L.ghost_prob = nnsel ? (float)ghost_prob(pe, vs[3], vs[4], nhits_of(si), P) : -1.0f;
    L.n_ut = 0;
#pragma unroll
    for (int k = 0; k < SM_N_UT; ++k) L.ut_hits[k] = -1;
    if constexpr (kUt) {
      int32_t ids[SM_N_UT];
      L.n_ut = ut_of(vs[0], vs[1], vs[2], vs[3], vs[4], pe.qop, ids);
#pragma unroll
      for (int k = 0; k < SM_N_UT; ++k) L.ut_hits[k] = ids[k];
    }
    if (plain) dst[lb + r] = L;
    else gstore(&dst[lb + r], L);
  }
  if (plain && tid == 0 && (long long)(lb + nk) > D->long_cap) raise_flag(cnt, F_OUT_LONG);
  if (mseeds) {
    int sb = 0;   // the event's first seed
#pragma unroll
    for (int i = 0; i < (NT <= 512 ? NT / 64 : 1); ++i) sb += sh.tmp[8 + i];
    if (tid == 0) D->seed_off[e] = (int32_t)sb;
    if (pool_ok && (long long)sb + ns <= D->seed_cap)
      for (int i = tid; i < ns; i += NT) D->seeds[sb + i] = gload(seed_at(i));
  }
}

// ----------------------------------------------------- the fused kernel ----

// (kMk: called by the matching kernel, which may also write the seeds)
template <int NT, int kSel, bool kMk = false>
__device__ __forceinline__ void match_event(const Desc *__restrict__ D, const Scratch &S,
                                            const DevParams &P, int e, int plain, size_t wg,
                                            MatchShared &sh) {
  int ns = S.item_cnt[2 * e] + S.item_cnt[2 * e + 1];
  if (D->pass == 1) ns += S.item_cnt3[2 * e] + S.item_cnt3[2 * e + 1];
  const int nv = D->b.velo_off[e + 1] - D->b.velo_off[e];
  if (ns <= kMsLds && nv <= kVsLds)
    match_event_impl<true, NT, kSel, kMk>(D, S, P, e, plain, wg, sh);
  else
    match_event_impl<false, NT, kSel, kMk>(D, S, P, e, plain, wg, sh);
}

// The preparing launch's copy of the batch descriptor from pinned host
// memory (its D) to the device copy that the later launches read; nothing
// when D is that copy already.
__device__ __forceinline__ void link_desc(const Desc *__restrict__ D, const KCtx *__restrict__ K) {
  static_assert(sizeof(Desc) % 4 == 0, "the descriptor is copied in 4-byte words");
  Desc *dst = K->L.desc;
  if (dst == nullptr || dst == D) return;
  const unsigned *src = reinterpret_cast<const unsigned *>(D);
  auto *out = gmem(reinterpret_cast<unsigned *>(dst));
  for (int i = threadIdx.x; i < (int)(sizeof(Desc) / 4); i += blockDim.x) out[i] = src[i];
}

// Size class of an item for the longest-first order: kFineSub classes per
// octave of (hits + 1), from its leading four bits; monotone in the size.
constexpr int kFineSub = 16;
constexpr int kFineCls = 32 * kFineSub;
__device__ __forceinline__ int fine_class(int sz) {
  const unsigned v = (unsigned)sz + 1u;
  const int b = 31 - __clz(v);
  const unsigned sub = b >= 4 ? (v >> (b - 4)) & 15u : (v << (4 - b)) & 15u;
  return b * kFineSub + (int)sub;
}

// Counters, per-event hand-off counts and (batched) the longest-first item
// order with the big-form cut: one workgroup of 1024 threads.
__device__ __forceinline__ unsigned prepare_batch(const Desc *__restrict__ D,
                                                  const KCtx *__restrict__ K, int plain) {
  const Scratch &S = K->S;
  __shared__ int fb[kFineCls];
  __shared__ int s_scan[16];
  __shared__ int s_best;
  const int ne = D->n_events, n = D->n_items;
  const auto *zo = gmem(D->b.zone_off);
  // every parameter of the cut is read here, before the first store (after
  // it the loads could not move ahead of the stores they might alias), so
  // that their latency overlaps the zone-offset loads
  const DevParams &P = K->P;
  const float lat_a = P.lat_a, lat_b = P.lat_b, big_r = P.big_speedup;
  const int big_slots = P.big_slots, uv_mode = P.uv_mode;
  const int main_grid = max(D->grid > 0 ? D->grid : P.main_slots, 1);
  const unsigned fuse = (unsigned)D->fuse;
  if (threadIdx.x == 0) {
    Counters *c = S.cnt;
    c->seed_queue = 0; c->match_queue = 0; c->flags = 0;
    c->pool_top = 0; c->lpool_top = 0;
    c->big_queue = 0; c->n_big = 0;
    for (int k = 0; k < 8; ++k) c->need_big[k] = 0;
    c->need_trip = c->need_cand = c->need_tbl = c->need_sst = 0;
    c->need_ms = c->need_vs = c->need_surv = c->need_combo = 0;
    c->total_seeds = 0; c->total_longs = 0;
    c->fuse = plain ? 1u : fuse;
    if (plain) { D->seed_off[0] = 0; D->long_off[0] = 0; }
  }
  if (plain) {
    for (int e = threadIdx.x; e < ne; e += blockDim.x) gmem(S.ev_done)[e] = 0;
    return 0u;
  }
  // Size classes are log2 buckets.  The big-item form takes every class from
  // a cut B upwards; it runs before the main form.  B is chosen by a latency
  // model of one item on a 256-thread workgroup, L(n) = a n + b n^2 (us):
  // T(B) = max(L_max(>=B) / r, W(>=B) / (r S_big)) + max(L_max(<B), W(<B) / S_main),
  // r the speed-up of the 16-wave form, S the workgroups of each form, W the
  // summed latencies; "no big form" is B = 32.  The Hough variant keeps every
  // item in the main form.  Order: big classes, then the rest, longest first.
  // The order uses finer classes, kFineSub per octave, so that items of one
  // octave (most of a min-bias batch) are still taken longest first; the
  // model's per-octave sums are taken over these classes, each item counted at
  // the top size of its class (one LDS atomic per item and nothing else: the
  // wave reductions of exact sums cost more than the whole model).
  __shared__ int fh[kFineCls];
  for (int f = threadIdx.x; f < kFineCls; f += blockDim.x) fh[f] = 0;
  __syncthreads();
  auto latency = [&](float nh) { return lat_a * nh + lat_b * nh * nh; };
  // The zone offsets of the first kPrepCache * blockDim items stay in
  // registers for both passes below; later items are reloaded.  The item
  // sizes need only the first and last offset: those two loads go first, and
  // the eleven in between only after the histogram, so that the statistics
  // do not wait behind them (thirteen loads 48 B apart per thread queue up
  // in the workgroup's memory path) and the middle ones stream in while the
  // cut and the order's scan run.
  constexpr int kPrepCache = 2;
  int zc[kPrepCache][kNL + 1];
#pragma unroll
  for (int c = 0; c < kPrepCache; ++c) {
    const int i = c * (int)blockDim.x + (int)threadIdx.x;
    zc[c][0] = i < n ? zo[i * kNL] : 0;
    zc[c][kNL] = i < n ? zo[i * kNL + kNL] : 0;
  }
  auto stat = [&](int i, int z0, int z1) {
    if (i < n) atomicAdd(&fh[fine_class(max(z1 - z0, 0))], 1);
  };
  auto reload = [&](int i, int (&z)[kNL + 1]) {
#pragma unroll
    for (int k = 0; k <= kNL; ++k) z[k] = i < n ? zo[i * kNL + k] : 0;
  };
#pragma unroll
  for (int c = 0; c < kPrepCache; ++c)
    stat(c * (int)blockDim.x + (int)threadIdx.x, zc[c][0], zc[c][kNL]);
  for (int i0 = kPrepCache * (int)blockDim.x; i0 < n; i0 += blockDim.x) {
    const int i = i0 + (int)threadIdx.x;
    stat(i, i < n ? zo[i * kNL] : 0, i < n ? zo[i * kNL + kNL] : 0);
  }
  // From here to the order's records nothing passes through global memory
  // between threads: the barriers order LDS only.  The middle offsets are
  // needed only for those records; their loads (eleven per item, 48 B apart)
  // take the workgroup's memory path several microseconds to issue, so they
  // are issued after the histogram's barrier (by wave 0 after the cut) and
  // stream in behind the cut and the scan; with a 16-byte aligned offset
  // array they are three 16-byte loads per item.
  lds_barrier();
  __builtin_amdgcn_sched_barrier(0);
  // the cut: wave 0, one lane per octave; its count, summed latency and
  // largest size from its fine classes; prefix maximum of the latencies below
  // an octave, suffix sum and maximum from it upwards, then the argmin of T
  // over the lanes (ties to the higher cut)
  if (threadIdx.x < 64) {
    const int b = threadIdx.x;
    const bool v = b < 32;
    float ws = 0.0f, lm = 0.0f;
    if (v) {
      // the octave's sixteen counts in one go (independent LDS reads)
      int cnt[kFineSub];
#pragma unroll
      for (int j = 0; j < kFineSub; ++j) cnt[j] = fh[b * kFineSub + j];
#pragma unroll
      for (int j = 0; j < kFineSub; ++j) {
        // largest size of fine class (b, j): sizes + 1 in [2^b (1 + j/16),
        // 2^b (1 + (j+1)/16)) from octave 4 up, exact below
        const float top = b >= 4 ? ldexpf(1.0f + (float)(j + 1) / kFineSub, b) - 2.0f
                                 : (float)((1 << b) + (j >> (4 - b)) - 1);
        const float l = latency(top);
        ws += (float)cnt[j] * l;
        lm = cnt[j] ? l : lm;   // classes ascend in size
      }
    }
    float wtot = ws, lall = lm, pre = lm, wsuf = ws, lsuf = lm;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      wtot += __shfl_xor(wtot, o, 64);
      lall = fmaxf(lall, __shfl_xor(lall, o, 64));
    }
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
      const float t0 = __shfl_up(pre, o, 64);
      const float t1 = __shfl_down(wsuf, o, 64), t2 = __shfl_down(lsuf, o, 64);
      if (b >= o) pre = fmaxf(pre, t0);
      if (b + o < 32) { wsuf += t1; lsuf = fmaxf(lsuf, t2); }
    }
    float l_lo = __shfl_up(pre, 1, 64);
    if (b == 0) l_lo = 0.0f;
    const float sb = (float)max(big_slots, 1), sm = (float)main_grid;
    const float t_none = fmaxf(lall, wtot / sm);
    float t = __builtin_inff();
    if (v && b >= kBigBucket && uv_mode == 0 && big_slots > 0 && wsuf > 0.0f)
      t = fmaxf(lsuf / big_r, wsuf / (big_r * sb)) + fmaxf(l_lo, (wtot - wsuf) / sm);
    float tb = t;
    int bb = t < t_none ? b : 32;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const float ot = __shfl_xor(tb, o, 64);
      const int ob = __shfl_xor(bb, o, 64);
      if (ot < tb || (ot == tb && ob > bb)) { tb = ot; bb = ob; }
    }
    if (b == 0) s_best = tb < t_none ? bb : 32;
  }
  __builtin_amdgcn_sched_barrier(0);
  if ((reinterpret_cast<uintptr_t>(D->b.zone_off) & 15u) == 0u) {
    // an item's offsets start 48 B apart: three 16-byte loads each
    static_assert(kNL == 12, "an item's twelve zone offsets are three 16-byte pieces");
    const auto *z4 = (const __attribute__((address_space(1))) gvec4 *)D->b.zone_off;
#pragma unroll
    for (int c = 0; c < kPrepCache; ++c) {
      const int i = c * (int)blockDim.x + (int)threadIdx.x;
      gvec4 q0 = {0, 0, 0, 0}, q1 = q0, q2 = q0;
      if (i < n) {
        q0 = z4[3 * i];
        q1 = z4[3 * i + 1];
        q2 = z4[3 * i + 2];
      }
      zc[c][1] = q0.y; zc[c][2] = q0.z; zc[c][3] = q0.w;
      zc[c][4] = q1.x; zc[c][5] = q1.y; zc[c][6] = q1.z; zc[c][7] = q1.w;
      zc[c][8] = q2.x; zc[c][9] = q2.y; zc[c][10] = q2.z; zc[c][11] = q2.w;
    }
  } else {
#pragma unroll
    for (int c = 0; c < kPrepCache; ++c) {
      const int i = c * (int)blockDim.x + (int)threadIdx.x;
#pragma unroll
      for (int k = 1; k < kNL; ++k) zc[c][k] = i < n ? zo[i * kNL + k] : 0;
    }
  }
  // first position of each fine class: the items of all larger classes
  {
    const int f = kFineCls - 1 - (int)threadIdx.x;   // descending
    const int v = f >= 0 ? fh[f] : 0;
    int total;
    const int ex = block_excl_scan<1024, true>(v, s_scan, total);
    if (f >= 0) fb[f] = ex;
  }
  lds_barrier();
  if (threadIdx.x == 0) {
    const int best = s_best;
    // the big form takes the classes >= best: the positions before the
    // first fine class of octave best
    const unsigned nb = best < 32 ? (unsigned)fb[kFineSub * best - 1] : 0u;
    S.cnt->n_big = nb;
    s_best = (int)nb;
  }
  lds_barrier();
  const unsigned n_big = (unsigned)s_best;
  // positions in the order, one LDS atomic per item on its fine class; each
  // position's record holds the item and its zone offsets
  auto place = [&](int i, const int (&z)[kNL + 1]) {
    const bool in = i < n;
    auto put = [&](int p) {
      ItemRec r;
      r.item = i;
#pragma unroll
      for (int k = 0; k <= kNL; ++k) r.zabs[k] = z[k];
      r.pad[0] = r.pad[1] = 0;
      gstore(&S.item_rec[p], r);
    };
    if (in) put(atomicAdd(&fb[fine_class(max(z[kNL] - z[0], 0))], 1));
  };
#pragma unroll
  for (int c = 0; c < kPrepCache; ++c) place(c * (int)blockDim.x + (int)threadIdx.x, zc[c]);
  for (int i0 = kPrepCache * (int)blockDim.x; i0 < n; i0 += blockDim.x) {
    int z[kNL + 1];   // loads before the record stores (which may alias them)
    reload(i0 + (int)threadIdx.x, z);
    place(i0 + (int)threadIdx.x, z);
  }
  // per-event hand-off counts (matching inside seeding only), last: no
  // barrier above waits for these stores
  if (fuse)
    for (int e = threadIdx.x; e < ne; e += blockDim.x) gmem(S.ev_done)[e] = 0;
  return n_big;
}

// Persistent Seeding (+ Matching): each workgroup pulls (event, half) items
// from the queue (or takes item_begin + blockIdx in the plain form) and seeds
// them; when the batch is matched inside seeding (kFuse instantiation), the
// workgroup that completes the second half of an event then matches that
// event.  The seeding state and the matching state share the same LDS.
// NT = kSeedWG: the main form, 4 workgroups per CU, over the items after the
// big ones in the longest-first order.  NT = kBigWG: one workgroup of 16
// waves per CU with its own scratch, over the big items (at the head of the
// order); it runs first, so a big item gets a whole CU instead of holding one
// 256-thread workgroup for the whole batch.
template <int kUv, int NT, bool kFuse = true, int kSel = 0>
__global__ __launch_bounds__(NT, NT == kSeedWG ? 4 : 1) void k_seed(const Desc *__restrict__ D,
                                                     const KCtx *__restrict__ K, int item_begin,
                                                     int item_count, int use_queue, int lds_hits,
                                                     int plain, int prep) {
  constexpr bool kBig = NT == kBigWG;
  const Scratch &S = kBig ? K->SB : K->S;
  const DevParams &P = K->P;
  extern __shared__ __align__(16) unsigned char smem[];
  SeedShared<NT> &sh = *reinterpret_cast<SeedShared<NT> *>(smem);
  MatchShared &mh = *reinterpret_cast<MatchShared *>(smem);
  float *s_x = reinterpret_cast<float *>(smem + sizeof(SeedShared<NT>));
  float *s_z = s_x + lds_hits;
  int32_t *s_id = reinterpret_cast<int32_t *>(s_z + lds_hits);
  __shared__ int s_last;

  const int tid = tidx();
  const size_t wg = blockIdx.x;
  // a preparing launch's D is the pinned host copy of the descriptor (same
  // contents as the device copy it writes; its reads stay in the scalar cache)
  const int32_t *zone_off = D->b.zone_off;
  const float *hx = D->b.hit_x, *hz = D->b.hit_z;
  const int32_t *hid = D->b.hit_id;
  if constexpr (kBig) {
    if (prep) {
      // this launch also prepares the batch: workgroup 0 does what k_prepare
      // does and then releases the others, which poll for it (bounded: on
      // giving up they flag the batch and leave, and the call fails)
      // The flag holds 1 + the number of big items: with none, every
      // workgroup leaves at once, with no acquire (an L2 invalidate) and no
      // counter loads behind it.
      __shared__ int s_stall;
      if (blockIdx.x == 0) {
        // the device copy of the descriptor for the later launches first,
        // then the preparation
        link_desc(D, K);
        const unsigned nb = prepare_batch(D, K, 0);
        __syncthreads();
        if (tid == 0)
          __hip_atomic_store(&S.cnt->prep_ready, nb + 1u, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
        if (nb == 0u) return;
      } else {
        if (tid == 0) {
          s_stall = 0;
          unsigned n = 0, f;
          // relaxed polls (an acquire per poll would invalidate caches that
          // workgroup 0 is reading through), one acquire after the flag
          while ((f = __hip_atomic_load(&S.cnt->prep_ready, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT)) == 0u) {
            __builtin_amdgcn_s_sleep(16);
            if (++n == kPrepSpin) {
              atomicExch(&S.cnt->stall, 1u);
              s_stall = 1;
              break;
            }
          }
          if (f == 1u) s_stall = 2;   // prepared, no big items
          else if (!s_stall) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (s_stall) return;
      }
    }
  }
  // input that the validation kernel rejected is not processed
  if (S.cnt->flags & (F_INVALID | F_UNSORTED)) return;
  const int n_big = use_queue ? (int)S.cnt->n_big : 0;
  // matching here (hand-off to the workgroup completing an event) or in
  // k_match; the main form has one instantiation with the matching code and
  // one without (which keeps the seeding phases' registers free of it); the
  // host launches the one that fits the batch, and the other would return
  // at once
  const bool fuse = use_queue ? S.cnt->fuse != 0u : true;
  if (!kBig && fuse != kFuse) return;
  // queue of this form: the big items [0, n_big) or the rest of the order
  const int n_items = item_count >= 0 ? item_count : (kBig ? n_big : D->n_items - n_big);
  const int q0 = kBig ? 0 : n_big;
  bool first = true;
  for (;;) {
    // the next item and its zone offsets (once from global memory, then from
    // LDS): from its record in the order, or from the zone offsets
    if (tid == 0) {
      int q;
      // the first item of each workgroup is its own index; later ones come
      // from the queue, which counts from the grid size
      if (first) q = (int)blockIdx.x;
      else if (use_queue)
        q = (int)gridDim.x + (int)atomicAdd(kBig ? &S.cnt->big_queue : &S.cnt->seed_queue, 1u);
      else q = n_items;
      int it = -1, z[kNL + 1];
      if (q < n_items) {
        // every load issued before the first LDS store
        if (use_queue) {
          const ItemRec r = gload(&S.item_rec[q0 + q]);
          it = r.item;
#pragma unroll
          for (int k = 0; k <= kNL; ++k) z[k] = r.zabs[k];
        } else {
          it = item_begin + q;
#pragma unroll
          for (int k = 0; k <= kNL; ++k) z[k] = zone_off[it * kNL + k];
        }
#pragma unroll
        for (int k = 0; k <= kNL; ++k) sh.zabs[k] = z[k];
      }
      sh.item = it;
      sh.pass = D->pass;
      sh.serial = D->serial;
      sh.ntrip = 0; sh.ncand = 0; sh.nseed = 0; sh.ncombo = 0; sh.nkept = 0;
    }
    // the last quarter of the workgroups is the youngest on its CU, whose
    // waves the issue order serves last: its first item runs at a raised wave
    // priority so that the first round of items ends more evenly
    if (!kBig && use_queue) {
      if (first && blockIdx.x >= 3 * gridDim.x / 4) __builtin_amdgcn_s_setprio(2);
      if (!first) __builtin_amdgcn_s_setprio(0);
    }
    first = false;
    // LDS only: what the workgroup's last item left in global memory (its
    // seeds) is read by later launches, not by this workgroup
    lds_barrier();
    const int item = sh.item;
    if (item < 0) break;
    const int base = sh.zabs[0];
    const int nh = sh.zabs[kNL] - base;
    if (tid <= kNL) sh.zoff[tid] = sh.zabs[tid] - base;
    if (tid == 0) {
      int acc = 0;
      for (int k = 0; k < 6; ++k) {
        sh.xb[k] = acc;
        const int L = (k >> 1) * 4 + (k & 1) * 3;
        acc += sh.zabs[L + 1] - sh.zabs[L];
      }
      sh.xb[6] = acc;
    }
    if (nh >= kMaxItemHits || nh < 0) {
      if (tid == 0) {
        raise_flag(S.cnt, nh < 0 ? F_INVALID : F_LIMIT);
        S.item_cnt[item] = 0;
        S.item_base[item] = 0;
      }
      lds_barrier();
    } else if (nh <= lds_hits) {
      // stage the item's hits; every bin entry starts at its zone's size
      for (int i = tid; i < nh; i += NT) {
        s_x[i] = gmem(hx)[base + i];
        s_z[i] = gmem(hz)[base + i];
        s_id[i] = gmem(hid)[base + i];
      }
      for (int i = tid; i < kNL * kBins; i += NT) {
        const int L = i / kBins;
        sh.bins[L][i % kBins] = (unsigned short)(sh.zabs[L + 1] - sh.zabs[L]);
      }
      lds_barrier();
      // hit i opens the bins in (kbin(previous hit), kbin(hit i)]
      int zb[kNL];
#pragma unroll
      for (int k = 0; k < kNL; ++k) zb[k] = sh.zoff[k + 1];
      for (int i = tid; i < nh; i += NT) {
        int L = 0;
#pragma unroll
        for (int k = 0; k < kNL - 1; ++k) L += i >= zb[k];
        const int li = i - sh.zoff[L];
        const int kc = kbin(s_x[i]);
        const int kp = li > 0 ? kbin(s_x[i - 1]) : 0;
        for (int b = kp; b < kc; ++b) sh.bins[L][b] = (unsigned short)li;
      }
      lds_barrier();
      seed_item<true, kUv>(s_x, s_z, s_id, item, nh, P, S, wg, sh);
    } else {
      lds_barrier();
      seed_item<false, kUv>(hx + base, hz + base, hid + base, item, nh, P, S, wg, sh);
    }
    // hand-off: after the barrier, one release increment of the per-event
    // count publishes the whole workgroup's writes (barrier synchronisation
    // and the release compose); the workgroup that completes the event's
    // second half acquires once and matches.  One L2 write-back per item and
    // one invalidate per event, instead of a device-wide fence per wave.
    // Without the hand-off the next item only reuses the LDS.
    if (kFuse && fuse) __syncthreads(); else lds_barrier();
    if (!kFuse || !fuse) continue;
    if (tid == 0) {
      const int prev = __hip_atomic_fetch_add(&S.ev_done[item >> 1], 1, __ATOMIC_RELEASE,
                                              __HIP_MEMORY_SCOPE_AGENT);
      s_last = prev == 1;
      if (prev == 1) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if constexpr (kFuse) {
      if (s_last) match_event<NT, kSel>(D, S, P, item >> 1, plain, wg, mh);
    }
    __syncthreads();
  }
}

// Matching (Sec. 4) as a kernel of its own, after the seeding kernels, when
// the preparation chose it for the batch: a persistent grid pulls events from a
// queue.  The kernel boundary orders every seed before every match, so the
// seeding kernel needs no per-event hand-off (one agent-scope release per
// item and one acquire per event, each an L2 write-back or invalidate on a
// chip with one L2 per XCD).
template <int kSel>
__global__ __launch_bounds__(kSeedWG, 4) void k_match(const Desc *__restrict__ D,
                                                      const KCtx *__restrict__ K) {
  const Scratch &S = K->S;
  const DevParams &P = K->P;
  extern __shared__ __align__(16) unsigned char smem[];
  MatchShared &mh = *reinterpret_cast<MatchShared *>(smem);
  __shared__ int s_e;
  if (S.cnt->fuse || (S.cnt->flags & (F_INVALID | F_UNSORTED))) return;
  // the first event of each workgroup is its own index (1024 workgroups on
  // one queue counter would queue behind each other at launch); later ones
  // come from the queue, which counts from the grid size
  for (bool first = true;; first = false) {
    if (threadIdx.x == 0)
      s_e = first ? (int)blockIdx.x : (int)gridDim.x + (int)atomicAdd(&S.cnt->match_queue, 1u);
    __syncthreads();
    const int e = s_e;
    if (e >= D->n_events) break;
    match_event<kSeedWG, kSel, true>(D, S, P, e, 0, blockIdx.x, mh);
    __syncthreads();
  }
}

// ------------------------------------------------------ batch plumbing ----

// Clear counters and per-event hand-off counts; in the batched form also
// order the (event, half) items by hit count, largest first (log2 buckets),
// so the longest items start first and the persistent grid drains evenly.
__global__ __launch_bounds__(1024) void k_prepare(const Desc *__restrict__ D,
                                                  const KCtx *__restrict__ K, int plain) {
  link_desc(D, K);
  prepare_batch(D, K, plain);
}

// Per-event seed and long-track offsets and the copy from the pools to the
// caller's CSR outputs, in one kernel.  Workgroup b takes a contiguous range
// of events: it sums the counts of every earlier event (a reduction over the
// prefix, read from L2), scans its own range, writes those offsets and copies
// the range's records.  The workgroup holding the last event writes the
// totals and the capacity checks; an event whose records would pass the
// caller's capacity is not copied (the call then reports the capacity).
__global__ __launch_bounds__(256) void k_copy(const Desc *__restrict__ D,
                                              const KCtx *__restrict__ K) {
  const Scratch &S = K->S;
  const int n = D->n_events, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int per = (n + (int)gridDim.x - 1) / (int)gridDim.x;
  const int e_lo = min(n, (int)blockIdx.x * per), e_hi = min(n, e_lo + per);
  const bool last = (e_lo < e_hi && e_hi == n) || (n == 0 && blockIdx.x == 0);
  if (e_lo >= e_hi && !last) return;
  // pool or input errors of the earlier kernels: no copy (read first, so
  // that the load overlaps the others)
  const bool bad = (S.cnt->flags & (F_POOL | F_LPOOL | F_INVALID | F_UNSORTED)) != 0u;
  // with the third iteration, each event's seeds also come from its two
  // items in the third pool, after the first two iterations' ones
  const bool t3 = D->pass == 1;
  // the matching kernel wrote the seeds and their offsets (mseeds), unless
  // the input was rejected before matching
  const bool ms = D->mseeds != 0 && !(S.cnt->flags & (F_INVALID | F_UNSORTED));
  auto seeds3 = [&](int e) {
    return t3 ? gmem(S.item_cnt3)[2 * e] + gmem(S.item_cnt3)[2 * e + 1] : 0;
  };
  __shared__ long long s_part[2][4];
  __shared__ int s_tmp[16];
  // the first pass's counts and pool bases of this range, issued with the
  // loads below (one round trip for both: clamped addresses, no branch, and
  // nothing computed from them before the prefix is reduced)
  int f_n0 = 0, f_n1 = 0, f_m = 0, f_n3a = 0, f_n3b = 0, f_b0 = 0, f_b1 = 0, f_src = 0;
  if (e_lo < e_hi) {
    const int e = min(e_lo + tid, e_hi - 1);
    f_n0 = gmem(S.item_cnt)[2 * e]; f_n1 = gmem(S.item_cnt)[2 * e + 1]; f_m = gmem(S.ev_lcnt)[e];
    f_b0 = gmem(S.item_base)[2 * e]; f_b1 = gmem(S.item_base)[2 * e + 1];
    f_src = gmem(S.ev_lbase)[e];
    if (t3) { f_n3a = gmem(S.item_cnt3)[2 * e]; f_n3b = gmem(S.item_cnt3)[2 * e + 1]; }
  }
  // the counts of the events before this range, four loads in flight per
  // thread at a time (independent accumulators, clamped addresses)
  long long ps = 0, pl = 0;
  for (int e0 = tid; e0 < e_lo; e0 += 1024) {
    int a[4], b[4], c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = min(e0 + 256 * u, e_lo - 1);
      a[u] = gmem(S.item_cnt)[2 * e];
      b[u] = gmem(S.item_cnt)[2 * e + 1] + seeds3(e);
      c[u] = gmem(S.ev_lcnt)[e];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (e0 + 256 * u < e_lo) { ps += a[u] + b[u]; pl += c[u]; }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ps += __shfl_xor(ps, o, 64);
    pl += __shfl_xor(pl, o, 64);
  }
  if (lane == 0) { s_part[0][w] = ps; s_part[1][w] = pl; }
  __syncthreads();
  long long cs = s_part[0][0] + s_part[0][1] + s_part[0][2] + s_part[0][3];
  long long cl = s_part[1][0] + s_part[1][1] + s_part[1][2] + s_part[1][3];
  // the range: offsets by block scans; each event's counts, pool bases and
  // offsets stay in LDS for the copy when the range fits one pass
  __shared__ int s_n0[256], s_n1[256], s_m[256];
  __shared__ long long s_b0[256], s_b1[256], s_src[256], s_so[256], s_lo[256];
  const bool one = e_hi - e_lo <= 256;
  for (int c0 = e_lo; c0 < e_hi; c0 += 256) {
    const int e = c0 + tid;
    const bool in = e < e_hi;
    int n0 = in ? f_n0 : 0, n1 = in ? f_n1 : 0, m = in ? f_m : 0, n3 = in ? f_n3a + f_n3b : 0;
    long long b0 = in ? f_b0 : 0, b1 = in ? f_b1 : 0, src = in ? f_src : 0;
    if (c0 != e_lo) {
      n0 = n1 = m = n3 = 0;
      b0 = b1 = src = 0;
      if (e < e_hi) {
        n0 = gmem(S.item_cnt)[2 * e]; n1 = gmem(S.item_cnt)[2 * e + 1]; m = gmem(S.ev_lcnt)[e];
        b0 = gmem(S.item_base)[2 * e]; b1 = gmem(S.item_base)[2 * e + 1];
        src = gmem(S.ev_lbase)[e];
        n3 = seeds3(e);
      }
    }
    int ts, tl;
    const int xs = block_excl_scan<256>(n0 + n1 + n3, s_tmp, ts);
    __syncthreads();
    const int xl = block_excl_scan<256>(m, s_tmp, tl);
    if (e < e_hi) {
      if (!ms) D->seed_off[e] = (int32_t)(cs + xs);
      D->long_off[e] = (int32_t)(cl + xl);
      if (one) {
        s_n0[tid] = n0; s_n1[tid] = n1; s_m[tid] = m;
        s_b0[tid] = b0; s_b1[tid] = b1; s_src[tid] = src;
        s_so[tid] = cs + xs; s_lo[tid] = cl + xl;
      }
    }
    cs += ts;
    cl += tl;
    __syncthreads();
  }
  if (last && tid == 0) {
    S.cnt->prep_ready = 0u;   // for the next batch's preparing launch
    D->seed_off[n] = (int32_t)cs;
    D->long_off[n] = (int32_t)cl;
    S.cnt->total_seeds = cs;
    S.cnt->total_longs = cl;
    if (cs > D->seed_cap) raise_flag(S.cnt, F_OUT_SEED);
    if (cl > D->long_cap) raise_flag(S.cnt, F_OUT_LONG);
    __threadfence();
  }
  if (last && K->L.hcnt != nullptr) {
    // the counters are final: this workgroup writes them to the slot's
    // pinned host memory, a word per thread, read through L2 (this
    // workgroup read the flags above)
    static_assert(sizeof(Counters) % 4 == 0 && sizeof(Counters) / 4 <= 128,
                  "the counters are copied in 4-byte words, two structs per workgroup");
    constexpr int kW = (int)(sizeof(Counters) / 4);
    __syncthreads();
    const bool second = tid >= 128;
    const int i = tid & 127;
    const Counters *src = second ? K->L.cnt3 : S.cnt;
    Counters *dst = second ? K->L.hcnt3 : K->L.hcnt;
    if (i < kW && src != nullptr && dst != nullptr) {
      reinterpret_cast<unsigned *>(dst)[i] =
          __hip_atomic_load(reinterpret_cast<const unsigned *>(src) + i, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
      __threadfence_system();
    }
  }
  if (bad) return;
  for (int e = e_lo; e < e_hi; ++e) {
    const int k = e - e_lo;
    int n0, n1, m;
    long long b0, b1, src, so, dst;
    if (one) {
      n0 = s_n0[k]; n1 = s_n1[k]; m = s_m[k];
      b0 = s_b0[k]; b1 = s_b1[k]; src = s_src[k]; so = s_so[k]; dst = s_lo[k];
    } else {
      n0 = gmem(S.item_cnt)[2 * e]; n1 = gmem(S.item_cnt)[2 * e + 1]; m = gmem(S.ev_lcnt)[e];
      b0 = gmem(S.item_base)[2 * e]; b1 = gmem(S.item_base)[2 * e + 1]; src = gmem(S.ev_lbase)[e];
      so = D->seed_off[e]; dst = D->long_off[e];
    }
    if (!ms && so + n0 + n1 <= D->seed_cap)
      for (int i = tid; i < n0 + n1; i += 256)
        D->seeds[so + i] = gload(i < n0 ? &S.pool[b0 + i] : &S.pool[b1 + i - n0]);
    if (t3 && !ms) {
      // the third iteration's seeds of the event: half 0, then half 1
      const int m0 = gmem(S.item_cnt3)[2 * e], m1 = gmem(S.item_cnt3)[2 * e + 1];
      const int c0 = gmem(S.item_base3)[2 * e], c1 = gmem(S.item_base3)[2 * e + 1];
      const long long s3 = so + n0 + n1;
      if (s3 + m0 + m1 <= D->seed_cap)
        for (int i = tid; i < m0 + m1; i += 256)
          D->seeds[s3 + i] = gload(i < m0 ? &S.pool3[c0 + i] : &S.pool3[c1 + i - m0]);
    }
    if (dst + m <= D->long_cap)
      for (int i = tid; i < m; i += 256) D->longs[dst + i] = gload(&S.lpool[src + i]);
  }
}

// ------------------------------------------ third-iteration clean-up ----

// Hits left per zone of each (event, half) item: those the first two
// iterations' seeds did not mark with this batch's serial.  Workgroup per
// item (persistent over the items); one wave per zone.  Workgroup 0 also
// clears the third pass's preparation flag (its preparing launch comes next).
__global__ __launch_bounds__(256) void k_clean_count(const Desc *__restrict__ D,
                                                      const KCtx *__restrict__ K) {
  const Third &T = K->T;
  if (blockIdx.x == 0 && threadIdx.x == 0) T.cnt->prep_ready = 0u;
  const int nz = D->n_events * 24;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t serial = D->serial;
  for (int z = (int)blockIdx.x * 4 + w; z < nz; z += (int)gridDim.x * 4) {
    const int lo = gmem(D->b.zone_off)[z], hi = gmem(D->b.zone_off)[z + 1];
    int n = 0;
    for (int i = lo + lane; i < hi; i += 64) n += gmem(K->S.used)[i] != serial;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
    if (lane == 0) gmem(T.zcnt)[z] = n;
  }
}

// The cleaned batch's zone offsets: an exclusive scan of the zone counts, one
// 1024-thread workgroup.
__global__ __launch_bounds__(1024) void k_clean_scan(const Desc *__restrict__ D,
                                                     const KCtx *__restrict__ K) {
  const Third &T = K->T;
  __shared__ int s_tmp[16];
  const int nz = D->n_events * 24;
  int carry = 0;
  for (int z0 = 0; z0 < nz; z0 += 1024) {
    const int z = z0 + (int)threadIdx.x;
    const int v = z < nz ? gmem(T.zcnt)[z] : 0;
    int total;
    const int ex = block_excl_scan<1024>(v, s_tmp, total);
    if (z < nz) gmem(T.zone_off)[z] = carry + ex;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) gmem(T.zone_off)[nz] = carry;
}

// The hits left, zone by zone in x order, into the cleaned batch: one wave
// per zone, a ballot prefix per 64 hits.
__global__ __launch_bounds__(256) void k_clean_copy(const Desc *__restrict__ D,
                                                     const KCtx *__restrict__ K) {
  const Third &T = K->T;
  const int nz = D->n_events * 24;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t serial = D->serial;
  for (int z = (int)blockIdx.x * 4 + w; z < nz; z += (int)gridDim.x * 4) {
    const int lo = gmem(D->b.zone_off)[z], hi = gmem(D->b.zone_off)[z + 1];
    int out = gmem(T.zone_off)[z];
    for (int i0 = lo; i0 < hi; i0 += 64) {
      const int i = i0 + lane;
      const bool keep = i < hi && gmem(K->S.used)[i] != serial;
      const unsigned long long m = __ballot(keep);
      if (keep) {
        const int o = out + (int)__popcll(m & ((1ull << lane) - 1ull));
        gmem(T.hx)[o] = gmem(D->b.hit_x)[i];
        gmem(T.hz)[o] = gmem(D->b.hit_z)[i];
        gmem(T.hid)[o] = gmem(D->b.hit_id)[i];
      }
      out += (int)__popcll(m);
    }
  }
}

// Clears n words (a fill kernel rather than a memset, so that a captured
// sequence records no memset node).
__global__ __launch_bounds__(256) void k_zero(unsigned *p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// totals of the plain form (offsets were chained event by event)
__global__ void k_plain_totals(const Desc *__restrict__ D, const KCtx *__restrict__ K) {
  const Scratch &S = K->S;
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int n = D->n_events;
    S.cnt->total_seeds = D->seed_off[n];
    S.cnt->total_longs = D->long_off[n];
    if (S.cnt->total_seeds > D->seed_cap) raise_flag(S.cnt, F_OUT_SEED);
    if (S.cnt->total_longs > D->long_cap) raise_flag(S.cnt, F_OUT_LONG);
  }
}

}  // namespace smk

using namespace smk;

static size_t match_lds_bytes(int) { return sizeof(MatchShared); }
size_t smk_seed_lds_bytes(int lds_hits, int sel) {
  const size_t a = sizeof(SeedShared<kSeedWG>) + (size_t)lds_hits * 3 * sizeof(float);
  return a > match_lds_bytes(sel) ? a : match_lds_bytes(sel);
}
size_t smk_seed_big_lds_bytes(int lds_hits, int sel) {
  const size_t a = sizeof(SeedShared<kBigWG>) + (size_t)lds_hits * 3 * sizeof(float);
  return a > match_lds_bytes(sel) ? a : match_lds_bytes(sel);
}

template <int kSel>
static void launch_seed_sel(const Desc *d, const KCtx *k, int item_begin, int item_count,
                            int use_queue, int grid, int lds_hits, int plain, hipStream_t st) {
  hipLaunchKernelGGL((k_seed<0, kSeedWG, true, kSel>), dim3(grid), dim3(kSeedWG),
                     smk_seed_lds_bytes(lds_hits, kSel), st, d, k, item_begin, item_count,
                     use_queue, lds_hits, plain, 0);
}
template <int kSel>
static void launch_big_sel(const Desc *d, const KCtx *k, int grid, int lds_hits, int prep,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_seed<0, kBigWG, true, kSel>), dim3(grid), dim3(kBigWG),
                     smk_seed_big_lds_bytes(lds_hits, kSel), st, d, k, 0, -1, 1, lds_hits, 0, prep);
}

extern "C" {
int smk_launch_prepare(const Desc *d, const KCtx *k, int plain, hipStream_t st) {
  hipLaunchKernelGGL(k_prepare, dim3(1), dim3(1024), 0, st, d, k, plain);
  return (int)hipGetLastError();
}
int smk_launch_seed(const Desc *d, const KCtx *k, int item_begin, int item_count, int use_queue,
                    int grid, int lds_hits, int plain, int uv_mode, int sel, hipStream_t st) {
  if (uv_mode == 1)
    hipLaunchKernelGGL((k_seed<1, kSeedWG>), dim3(grid), dim3(kSeedWG), smk_seed_lds_bytes(lds_hits),
                       st, d, k, item_begin, item_count, use_queue, lds_hits, plain, 0);
  else if (sel == 1)
    launch_seed_sel<1>(d, k, item_begin, item_count, use_queue, grid, lds_hits, plain, st);
  else if (sel == 2)
    launch_seed_sel<2>(d, k, item_begin, item_count, use_queue, grid, lds_hits, plain, st);
  else if (sel == 3)
    launch_seed_sel<3>(d, k, item_begin, item_count, use_queue, grid, lds_hits, plain, st);
  else
    launch_seed_sel<0>(d, k, item_begin, item_count, use_queue, grid, lds_hits, plain, st);
  return (int)hipGetLastError();
}
int smk_launch_seed_nomatch(const Desc *d, const KCtx *k, int grid, int lds_hits, hipStream_t st) {
  hipLaunchKernelGGL((k_seed<0, kSeedWG, false>), dim3(grid), dim3(kSeedWG),
                     smk_seed_lds_bytes(lds_hits), st, d, k, 0, -1, 1, lds_hits, 0, 0);
  return (int)hipGetLastError();
}
int smk_launch_seed_big(const Desc *d, const KCtx *k, int grid, int lds_hits, int prep, int sel,
                        hipStream_t st) {
  if (sel == 1) launch_big_sel<1>(d, k, grid, lds_hits, prep, st);
  else if (sel == 2) launch_big_sel<2>(d, k, grid, lds_hits, prep, st);
  else if (sel == 3) launch_big_sel<3>(d, k, grid, lds_hits, prep, st);
  else launch_big_sel<0>(d, k, grid, lds_hits, prep, st);
  return (int)hipGetLastError();
}
int smk_launch_match(const Desc *d, const KCtx *k, int grid, int sel, hipStream_t st) {
  const size_t lds = match_lds_bytes(sel);
  if (sel == 1) hipLaunchKernelGGL(k_match<1>, dim3(grid), dim3(kSeedWG), lds, st, d, k);
  else if (sel == 2) hipLaunchKernelGGL(k_match<2>, dim3(grid), dim3(kSeedWG), lds, st, d, k);
  else if (sel == 3) hipLaunchKernelGGL(k_match<3>, dim3(grid), dim3(kSeedWG), lds, st, d, k);
  else hipLaunchKernelGGL(k_match<0>, dim3(grid), dim3(kSeedWG), lds, st, d, k);
  return (int)hipGetLastError();
}
int smk_seed_big_static_lds() {
  hipFuncAttributes a;
  if (hipFuncGetAttributes(&a, (const void *)k_seed<0, kBigWG>) != hipSuccess) {
    (void)hipGetLastError();
    return 1024;   // a margin above what the kernel declares
  }
  return (int)a.sharedSizeBytes;
}
int smk_seed_lds_limit(int bytes) {
  int e = (int)hipFuncSetAttribute((const void *)k_seed<0, kSeedWG, false>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (!e) e = (int)hipFuncSetAttribute((const void *)k_seed<0, kSeedWG, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (!e) e = (int)hipFuncSetAttribute((const void *)k_seed<0, kSeedWG, true, 1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (!e) e = (int)hipFuncSetAttribute((const void *)k_seed<0, kSeedWG, true, 2>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (!e) e = (int)hipFuncSetAttribute((const void *)k_seed<0, kSeedWG, true, 3>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (!e) e = (int)hipFuncSetAttribute((const void *)k_seed<1, kSeedWG, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return e;
}
int smk_seed_big_lds_limit(int bytes) {
  int e = (int)hipFuncSetAttribute((const void *)k_seed<0, kBigWG>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (!e) e = (int)hipFuncSetAttribute((const void *)k_seed<0, kBigWG, true, 1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (!e) e = (int)hipFuncSetAttribute((const void *)k_seed<0, kBigWG, true, 2>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (!e) e = (int)hipFuncSetAttribute((const void *)k_seed<0, kBigWG, true, 3>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return e;
}
int smk_launch_copy(const Desc *d, const KCtx *k, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, st, d, k);
  return (int)hipGetLastError();
}
int smk_launch_validate(const Desc *d, const KCtx *k, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_validate, dim3(grid), dim3(256), 0, st, d, k);
  return (int)hipGetLastError();
}
int smk_launch_clean(const Desc *d, const KCtx *k, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_clean_count, dim3(grid), dim3(256), 0, st, d, k);
  int e = (int)hipGetLastError();
  if (!e) {
    hipLaunchKernelGGL(k_clean_scan, dim3(1), dim3(1024), 0, st, d, k);
    e = (int)hipGetLastError();
  }
  if (!e) {
    hipLaunchKernelGGL(k_clean_copy, dim3(grid), dim3(256), 0, st, d, k);
    e = (int)hipGetLastError();
  }
  return e;
}
int smk_launch_zero(void *p, int n_words, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, st, (unsigned *)p, n_words);
  return (int)hipGetLastError();
}
int smk_launch_plain_totals(const Desc *d, const KCtx *k, hipStream_t st) {
  hipLaunchKernelGGL(k_plain_totals, dim3(1), dim3(64), 0, st, d, k);
  return (int)hipGetLastError();
}
}
