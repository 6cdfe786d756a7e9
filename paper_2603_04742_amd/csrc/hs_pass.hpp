// Two-pass (multi-workgroup) negacyclic NTT for gfx950.
//
// The stages of a length-N transform split at S = floor(log N / 2): the forward "high" pass runs
// stages [0, S) (index bits [logn - S, logn)), the forward "low" pass stages [S, logn) (bits
// [0, logn - S)); the inverse runs the low pass first.  A pass acts on independent groups:
//   high groups: the elements sharing their low logn - S bits, 2^S of them at stride 2^(logn-S);
//   low groups : 2^(logn-S) contiguous elements.
// A workgroup transforms a block of BE = min(N, 2048) elements: GB consecutive groups.  In LDS,
// element u of group g sits at u * GB + g (high: consecutive g are consecutive addresses in HBM)
// or g * G + u (low).  Between the passes the data goes through HBM/L2 as balanced doubles.
// Each kernel pass therefore needs only N / BE workgroups per limb, spreading one transform over
// many CUs (latency) while fused kernels chain several transforms of the same block.
#pragma once
#include "hs_device.hpp"

namespace hs {

static constexpr int kBlockElems = 2048;

struct PassGeom {
  static constexpr int kMaxBE = kBlockElems;  // bound for per-thread register arrays
  int logn, S;        // split
  int BE;             // elements per block
  int lbe;            // log2 BE
  int nblk;           // blocks per limb (same for both passes)
  __host__ __device__ int gb_high() const { return BE >> S; }            // high groups per block
  __host__ __device__ int gb_low() const { return BE >> (logn - S); }    // low groups per block
  __host__ __device__ int lgb_high() const { return lbe - S; }           // their log2 (all index
  __host__ __device__ int lgb_low() const { return lbe - (logn - S); }   // arithmetic is shifts)
};

__host__ __device__ inline PassGeom make_geom(int logn) {
  PassGeom g;
  g.logn = logn;
  g.S = logn >> 1;
  g.BE = (1 << logn) < kBlockElems ? (1 << logn) : kBlockElems;
  g.lbe = 0;
  while ((1 << g.lbe) < g.BE) g.lbe++;
  g.nblk = (1 << logn) / g.BE;
  return g;
}

// The same geometry as compile-time constants (ring sizes of the two-pass path): every shift and
// loop bound of the pass code folds, as with the whole-limb transforms.
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }
__host__ __device__ constexpr int clog2(int x) { return x <= 1 ? 0 : 1 + clog2(x >> 1); }
template <int LOGN, int LBE = 11>
struct PassGeomC {
  static constexpr int logn = LOGN, S = LOGN >> 1;
  static constexpr int BE = cmin(1 << LOGN, 1 << LBE);
  static constexpr int kMaxBE = BE;  // bound for per-thread register arrays
  static constexpr int lbe = clog2(BE);
  static constexpr int nblk = (1 << LOGN) / BE;
  __host__ __device__ static constexpr int gb_high() { return BE >> S; }
  __host__ __device__ static constexpr int gb_low() { return BE >> (logn - S); }
  __host__ __device__ static constexpr int lgb_high() { return lbe - S; }
  __host__ __device__ static constexpr int lgb_low() { return lbe - (logn - S); }
};

// LDS padding of a pass layout.  Low layout: one pad double per 16.  High layout: one per 32 --
// its first round reads elements 8 rows (8 x 16 doubles) apart across lanes, which one pad per 16
// maps onto a quarter of the banks (4-way conflicts); one per 32 halves that and keeps the
// unit-stride rounds conflict-free.
template <bool HIGH>
__device__ __forceinline__ int lpadx(int i) { return HIGH ? i + (i >> 5) : i + (i >> 4); }

// The same ring with half-size blocks (1024 elements): kernels whose workgroups hold several blocks
// use it to double their grid and halve each workgroup's serial work.  Runtime geometry: unchanged.
template <class GT> struct HalfBlocks { using type = GT; };
template <int LOGN> struct HalfBlocks<PassGeomC<LOGN, 11>> { using type = PassGeomC<LOGN, 10>; };

// Global index of element u of group g in block `blk`.
template <class GT>
__device__ __forceinline__ int gidx_high(const GT& G, int blk, int g, int u) {
  return ((blk << G.lgb_high()) + g) + (u << (G.logn - G.S));
}
template <class GT>
__device__ __forceinline__ int gidx_low(const GT& G, int blk, int g, int u) {
  return (((blk << G.lgb_low()) + g) << (G.logn - G.S)) + u;
}
// LDS address of element u of group g (HIGH: strided layout, LOW: contiguous layout).
template <bool HIGH, class GT>
__device__ __forceinline__ int laddr(const GT& G, int g, int u) {
  return HIGH ? (u << G.lgb_high()) + g : (g << (G.logn - G.S)) + u;
}
// Block element e (0..BE-1) <-> (g, u) in the LDS order of the layout: LDS address e.
template <bool HIGH, class GT>
__device__ __forceinline__ int gidx_of_lds(const GT& G, int blk, int e) {
  if (HIGH) {
    const int l = G.lgb_high();
    return gidx_high(G, blk, e & ((1 << l) - 1), e >> l);
  } else {
    const int l = G.logn - G.S;
    return gidx_low(G, blk, e >> l, e & ((1 << l) - 1));
  }
}

// ---- twiddles of one pass, staged in LDS
// High passes (forward stages [0, S), inverse stages [logn - S, logn)) use table entries [1, 2^S):
// copied to LDS at the same indices.  Low passes use, per stage, one contiguous range of the table
// that depends on the block:
//   forward stage st in [S, logn): entries 2^st + blk GB 2^(st-S) + [0, GB 2^(st-S)),
//                                   LDS offset GB (2^(st-S) - 1)
//   inverse stage st in [0, logn-S): with d = logn - S - st - 1, entries N/2^(st+1) + blk GB 2^d +
//                                   [0, GB 2^d), LDS offset GB (2^(logn-S) - 2^(d+1))
// Each range has at most BE/2 entries and all ranges of a pass at most BE.
__host__ __device__ constexpr int tw_lds_entries(int BE) { return BE; }

template <bool HIGH, bool FWD, class GT>
__device__ __forceinline__ int tw_lds_index(const GT& G, int blk, int st, int gtw) {
  if (HIGH) return gtw;
  const int lgb = G.lgb_low();
  const int nl = G.logn - G.S;
  if (FWD) {
    const int e = st - G.S;
    return (((1 << e) - 1) << lgb) + (gtw - (1 << st) - (blk << (lgb + e)));
  } else {
    const int d = nl - st - 1;
    return (((1 << nl) - (2 << d)) << lgb) + (gtw - ((1 << G.logn) >> (st + 1)) - (blk << (lgb + d)));
  }
}

// LDS twiddle slots of a pass: high passes use slots [0, 2^S) = table entries [0, 2^S); the
// stage ranges of a low pass are adjacent, [(2^k - 1) GB, (2^(k+1) - 1) GB) for forward stage
// S + k and [(2^nl - 2^(d+1)) GB, (2^nl - 2^d) GB) for inverse stage nl - 1 - d (nl = logn - S).
template <bool HIGH, class GT>
__host__ __device__ inline int tw_slots(const GT& G) {
  return HIGH ? (1 << G.S) : (((1 << (G.logn - G.S)) - 1) << G.lgb_low());
}
// Table index of slot L (the inverse of tw_lds_index over the slots in use).
template <bool HIGH, bool FWD, class GT>
__host__ __device__ inline int tw_src_index(const GT& G, int blk, int L) {
  if (HIGH) return L;
  const int lgb = G.lgb_low(), nl = G.logn - G.S;
  const int q = L >> lgb;
  if (FWD) {
    const int k = 31 - __builtin_clz((unsigned)(q + 1));
    return (1 << (G.S + k)) + (blk << (lgb + k)) + (L - (((1 << k) - 1) << lgb));
  }
  const int d = 31 - __builtin_clz((unsigned)((1 << nl) - q - 1));
  const int st = nl - 1 - d;
  return ((1 << G.logn) >> (st + 1)) + (blk << (lgb + d)) + (L - (((1 << nl) - (2 << d)) << lgb));
}

// A pass's twiddles held in registers: load() issues every global load at once (early in a
// kernel, so their latency overlaps the data loads), store() writes them to the LDS slots.
template <int NT, bool HIGH, bool FWD, class GT>
struct TwPre {
  static constexpr int kSlotsMax = HIGH ? cmin(GT::kMaxBE, 256) : GT::kMaxBE;  // 2^S <= 256 for logn <= 16
  static constexpr int kPer = (kSlotsMax + NT - 1) / NT;
  double2 v[kPer];
  __device__ __forceinline__ void load(const GT& G, int blk, const double2* __restrict__ tw) {
    const int total = tw_slots<HIGH>(G);
#pragma unroll
    for (int r = 0; r < kPer; r++) {
      const int L = threadIdx.x + r * NT;
      if (L < total) v[r] = ldtw(tw, tw_src_index<HIGH, FWD>(G, blk, L));
    }
  }
  __device__ __forceinline__ void store(double2* twl, const GT& G) const {
    const int total = tw_slots<HIGH>(G);
#pragma unroll
    for (int r = 0; r < kPer; r++) {
      const int L = threadIdx.x + r * NT;
      if (L < total) twl[L] = v[r];
    }
  }
};

// Copy the pass's twiddles to twl (cooperative; the caller synchronises afterwards).
template <int NT, bool HIGH, bool FWD, class GT>
__device__ __forceinline__ void stage_twiddles(double2* twl, const GT& G, int blk, const double2* __restrict__ tw) {
  TwPre<NT, HIGH, FWD, GT> p;
  p.load(G, blk, tw);
  p.store(twl, G);
}

// One register round of a group transform: group bits [lo, lo + nb) of the global index (lo = 0
// for low groups, logn - S for high groups); the round covers local bits [lb, lb + R).
// Forward: stage k pairs global bit lo + lb + R - 1 - k (global stage logn - lo - lb - R + k).
// Inverse: stage k pairs global bit lo + lb + k.
template <int R, int NT, bool FWD, bool HIGH, class GT>
__device__ __forceinline__ void pass_round(double* s, const GT& G, int blk, int lb, int lazy, bool scale,
                                           const double2* twl, double2 ninv, ModD m) {
  const int n = 1 << G.logn;
  const int nb = HIGH ? G.S : G.logn - G.S;
  const int lo = HIGH ? G.logn - G.S : 0;
  const int GB = HIGH ? G.gb_high() : G.gb_low();
  const int lpg = nb - R;  // log2 of the register groups per transform group
  for (int sg = threadIdx.x; sg < (GB << lpg); sg += NT) {
    const int g = sg >> lpg, r = sg & ((1 << lpg) - 1);
    const int base_u = ((r >> lb) << (lb + R)) | (r & ((1 << lb) - 1));
    const int gb = HIGH ? gidx_high(G, blk, g, base_u) : gidx_low(G, blk, g, base_u);
    const int hb = gb >> (lo + lb + R);
    const int l0 = laddr<HIGH>(G, g, base_u);
    const int ls = HIGH ? (GB << lb) : (1 << lb);
    double x[1 << R];
#pragma unroll
    for (int v = 0; v < (1 << R); v++) x[v] = s[lpadx<HIGH>(l0 + v * ls)];
    if (FWD) {
      int lz = lazy;
#pragma unroll
      for (int k = 0; k < R; k++) {
        if (lz >= 2) {
#pragma unroll
          for (int v = 0; v < (1 << R); v++) x[v] = reduce(x[v], m);
          lz = 0;
        }
        const int st = G.logn - lo - lb - R + k;
        const double2* twk = twl + tw_lds_index<HIGH, true>(G, blk, st, (1 << st) + (hb << k));
#pragma unroll
        for (int j = 0; j < (1 << k); j++) {
          const double2 w = twk[j];
#pragma unroll
          for (int v = 0; v < (1 << (R - 1 - k)); v++) {
            const int u = (j << (R - k)) | v;
            const int u2 = u | (1 << (R - 1 - k));
            const double t = mul_tw(x[u2], w.x, w.y, m);
            x[u2] = x[u] - t;
            x[u] = x[u] + t;
          }
        }
        lz++;
      }
    } else {
#pragma unroll
      for (int k = 0; k < R; k++) {
        const int st = lo + lb + k;
        const double2* twk = twl + tw_lds_index<HIGH, false>(G, blk, st, (n >> (st + 1)) + (hb << (R - 1 - k)));
#pragma unroll
        for (int j = 0; j < (1 << (R - 1 - k)); j++) {
          const double2 w = twk[j];
#pragma unroll
          for (int v = 0; v < (1 << k); v++) {
            const int u = (j << (k + 1)) | v;
            const int u2 = u | (1 << k);
            const double a = x[u], b = x[u2];
            x[u] = reduce(a + b, m);
            x[u2] = mul_tw(a - b, w.x, w.y, m);
          }
        }
      }
      if (scale) {
#pragma unroll
        for (int v = 0; v < (1 << R); v++) x[v] = mul_tw(x[v], ninv.x, ninv.y, m);
      }
    }
#pragma unroll
    for (int v = 0; v < (1 << R); v++) s[lpadx<HIGH>(l0 + v * ls)] = x[v];
  }
}

// Forward pass on the block in LDS (inputs |x| <= q); ends with every element reduced to
// |x| <= q/2 + 1 and a barrier.  twl: LDS scratch of tw_lds_entries(BE) double2 for the staged
// twiddles (must not be in use by other threads).  The caller synchronises before.
template <int NT, bool HIGH, class GT>
__device__ __forceinline__ void pass_fwd(double* s, double2* twl, const GT& G, int blk, const double2* __restrict__ tw, ModD m,
                         bool stage = true) {
  const int nb = HIGH ? G.S : G.logn - G.S;
  if (stage) {
    stage_twiddles<NT, HIGH, true>(twl, G, blk, tw);
    __syncthreads();
  }
  int done = 0, lazy = 0;
  while (done < nb) {
    const int R = min(HS_NTT_RADIX_BITS, nb - done);
    const int lb = nb - done - R;  // forward: from the top local bits down
    switch (R) {
      case 3: pass_round<3, NT, true, HIGH>(s, G, blk, lb, lazy, false, twl, double2{0, 0}, m); break;
      case 2: pass_round<2, NT, true, HIGH>(s, G, blk, lb, lazy, false, twl, double2{0, 0}, m); break;
      default: pass_round<1, NT, true, HIGH>(s, G, blk, lb, lazy, false, twl, double2{0, 0}, m); break;
    }
    for (int k = 0; k < R; k++) { if (lazy >= 2) lazy = 0; lazy++; }
    done += R;
    __syncthreads();
  }
  for (int e = threadIdx.x; e < G.BE; e += NT) s[lpadx<HIGH>(e)] = reduce(s[lpadx<HIGH>(e)], m);
  __syncthreads();
}

// Inverse pass on the block in LDS (inputs |x| <= q, outputs |x| <= 0.625 q); `scale` multiplies
// by N^-1 (the last inverse pass).  Ends with a barrier.
template <int NT, bool HIGH, class GT>
__device__ __forceinline__ void pass_inv(double* s, double2* twl, const GT& G, int blk, bool scale, const double2* __restrict__ tw, double2 ninv, ModD m,
                         bool stage = true) {
  const int nb = HIGH ? G.S : G.logn - G.S;
  if (stage) {
    stage_twiddles<NT, HIGH, false>(twl, G, blk, tw);
    __syncthreads();
  }
  int done = 0;
  while (done < nb) {
    const int R = min(HS_NTT_RADIX_BITS, nb - done);
    const bool last = scale && (done + R == nb);
    switch (R) {
      case 3: pass_round<3, NT, false, HIGH>(s, G, blk, done, 0, last, twl, ninv, m); break;
      case 2: pass_round<2, NT, false, HIGH>(s, G, blk, done, 0, last, twl, ninv, m); break;
      default: pass_round<1, NT, false, HIGH>(s, G, blk, done, 0, last, twl, ninv, m); break;
    }
    done += R;
    __syncthreads();
  }
}

// ---- several blocks of the same pass at once (same modulus and block position, so the staged
// twiddles are shared): block j at s + j * LB, skipped when bit j of `skip` is set.  Spreads the
// register groups of all blocks over the workgroup, so NB independent transforms run
// concurrently instead of one after another.
template <int R, int NT, bool FWD, bool HIGH, class GT, bool PM = false>
__device__ __forceinline__ void pass_round_multi(double* s, int LB, int NB, unsigned skip, const GT& G, int blk, int lb, int lazy,
                                                 bool scale, const double2* twl, double2 ninv, ModD m, int twstride = 0,
                                                 const double2* mods = nullptr) {
  const int nb = HIGH ? G.S : G.logn - G.S;
  const int GB = HIGH ? G.gb_high() : G.gb_low();
  const int lpg = nb - R;
  const int lpb = (HIGH ? G.lgb_high() : G.lgb_low()) + lpg;  // log2 register groups per block
  for (int t = threadIdx.x; t < (NB << lpb); t += NT) {
    const int j = t >> lpb;
    if ((skip >> j) & 1u) continue;
    // PM: block j has its own modulus (mods[j] = (q, fl(1/q)) in LDS) and twiddle table
    ModD mj = m;
    const double2* twj = twl;
    if (PM) {
      const double2 mq = mods[j];
      mj = ModD{mq.x, mq.y};
      twj = twl + (size_t)j * twstride;
    }
    const int sg = t & ((1 << lpb) - 1);
    const int g = sg >> lpg, r = sg & ((1 << lpg) - 1);
    const int n = 1 << G.logn;
    const int lo = HIGH ? G.logn - G.S : 0;
    const int base_u = ((r >> lb) << (lb + R)) | (r & ((1 << lb) - 1));
    const int gb = HIGH ? gidx_high(G, blk, g, base_u) : gidx_low(G, blk, g, base_u);
    const int hb = gb >> (lo + lb + R);
    double* sj = s + (size_t)j * LB;
    const int l0 = laddr<HIGH>(G, g, base_u);
    const int ls = HIGH ? (GB << lb) : (1 << lb);
    double x[1 << R];
#pragma unroll
    for (int v = 0; v < (1 << R); v++) x[v] = sj[lpadx<HIGH>(l0 + v * ls)];
    if (FWD) {
      int lz = lazy;
#pragma unroll
      for (int k = 0; k < R; k++) {
        if (lz >= 2) {
#pragma unroll
          for (int v = 0; v < (1 << R); v++) x[v] = reduce(x[v], mj);
          lz = 0;
        }
        const int st = G.logn - lo - lb - R + k;
        const double2* twk = twj + tw_lds_index<HIGH, true>(G, blk, st, (1 << st) + (hb << k));
#pragma unroll
        for (int jj = 0; jj < (1 << k); jj++) {
          const double2 w = twk[jj];
#pragma unroll
          for (int v = 0; v < (1 << (R - 1 - k)); v++) {
            const int u = (jj << (R - k)) | v;
            const int u2 = u | (1 << (R - 1 - k));
            const double tt = mul_tw(x[u2], w.x, w.y, mj);
            x[u2] = x[u] - tt;
            x[u] = x[u] + tt;
          }
        }
        lz++;
      }
    } else {
#pragma unroll
      for (int k = 0; k < R; k++) {
        const int st = lo + lb + k;
        const double2* twk = twj + tw_lds_index<HIGH, false>(G, blk, st, (n >> (st + 1)) + (hb << (R - 1 - k)));
#pragma unroll
        for (int jj = 0; jj < (1 << (R - 1 - k)); jj++) {
          const double2 w = twk[jj];
#pragma unroll
          for (int v = 0; v < (1 << k); v++) {
            const int u = (jj << (k + 1)) | v;
            const int u2 = u | (1 << k);
            const double a = x[u], bb = x[u2];
            x[u] = reduce(a + bb, mj);
            x[u2] = mul_tw(a - bb, w.x, w.y, mj);
          }
        }
      }
      if (scale) {
#pragma unroll
        for (int v = 0; v < (1 << R); v++) x[v] = mul_tw(x[v], ninv.x, ninv.y, mj);
      }
    }
#pragma unroll
    for (int v = 0; v < (1 << R); v++) sj[lpadx<HIGH>(l0 + v * ls)] = x[v];
  }
}

// Forward pass on NB blocks (twiddles already staged; inputs |x| <= q; outputs |x| <= q/2 + 1).
// Starts with no barrier of its own (the caller synchronises after staging) and ends with one.
template <int NT, bool HIGH, class GT>
__device__ __forceinline__ void pass_fwd_multi(double* s, int LB, int NB, unsigned skip, const double2* twl, const GT& G, int blk, ModD m) {
  const int nb = HIGH ? G.S : G.logn - G.S;
  int done = 0, lazy = 0;
  while (done < nb) {
    const int R = min(HS_NTT_RADIX_BITS, nb - done);
    const int lb = nb - done - R;
    switch (R) {
      case 3: pass_round_multi<3, NT, true, HIGH>(s, LB, NB, skip, G, blk, lb, lazy, false, twl, double2{0, 0}, m); break;
      case 2: pass_round_multi<2, NT, true, HIGH>(s, LB, NB, skip, G, blk, lb, lazy, false, twl, double2{0, 0}, m); break;
      default: pass_round_multi<1, NT, true, HIGH>(s, LB, NB, skip, G, blk, lb, lazy, false, twl, double2{0, 0}, m); break;
    }
    for (int k = 0; k < R; k++) { if (lazy >= 2) lazy = 0; lazy++; }
    done += R;
    __syncthreads();
  }
  for (int t = threadIdx.x; t < (NB << G.lbe); t += NT) {
    const int j = t >> G.lbe, e = t & (G.BE - 1);
    if (!((skip >> j) & 1u)) s[(size_t)j * LB + lpadx<HIGH>(e)] = reduce(s[(size_t)j * LB + lpadx<HIGH>(e)], m);
  }
  __syncthreads();
}

// Forward pass on NB blocks of different moduli: block j uses twiddle table twl + j * twstride and
// modulus mods[j] (LDS).  Same contract as pass_fwd_multi otherwise.
template <int NT, bool HIGH, class GT>
__device__ __forceinline__ void pass_fwd_multi_mod(double* s, int LB, int NB, const double2* twl, int twstride, const double2* mods, const GT& G,
                                                   int blk) {
  const int nb = HIGH ? G.S : G.logn - G.S;
  const ModD m0{0.0, 0.0};
  int done = 0, lazy = 0;
  while (done < nb) {
    const int R = min(HS_NTT_RADIX_BITS, nb - done);
    const int lb = nb - done - R;
    switch (R) {
      case 3: pass_round_multi<3, NT, true, HIGH, GT, true>(s, LB, NB, 0u, G, blk, lb, lazy, false, twl, double2{0, 0}, m0, twstride, mods); break;
      case 2: pass_round_multi<2, NT, true, HIGH, GT, true>(s, LB, NB, 0u, G, blk, lb, lazy, false, twl, double2{0, 0}, m0, twstride, mods); break;
      default: pass_round_multi<1, NT, true, HIGH, GT, true>(s, LB, NB, 0u, G, blk, lb, lazy, false, twl, double2{0, 0}, m0, twstride, mods); break;
    }
    for (int k = 0; k < R; k++) { if (lazy >= 2) lazy = 0; lazy++; }
    done += R;
    __syncthreads();
  }
  for (int t = threadIdx.x; t < (NB << G.lbe); t += NT) {
    const int j = t >> G.lbe, e = t & (G.BE - 1);
    const ModD mj{mods[j].x, mods[j].y};
    s[(size_t)j * LB + lpadx<HIGH>(e)] = reduce(s[(size_t)j * LB + lpadx<HIGH>(e)], mj);
  }
  __syncthreads();
}

// Inverse pass on NB blocks (twiddles already staged; inputs |x| <= q, outputs |x| <= 0.625 q).
template <int NT, bool HIGH, class GT>
__device__ __forceinline__ void pass_inv_multi(double* s, int LB, int NB, bool scale, const double2* twl, double2 ninv, const GT& G, int blk, ModD m) {
  const int nb = HIGH ? G.S : G.logn - G.S;
  int done = 0;
  while (done < nb) {
    const int R = min(HS_NTT_RADIX_BITS, nb - done);
    const bool last = scale && (done + R == nb);
    switch (R) {
      case 3: pass_round_multi<3, NT, false, HIGH>(s, LB, NB, 0u, G, blk, done, 0, last, twl, ninv, m); break;
      case 2: pass_round_multi<2, NT, false, HIGH>(s, LB, NB, 0u, G, blk, done, 0, last, twl, ninv, m); break;
      default: pass_round_multi<1, NT, false, HIGH>(s, LB, NB, 0u, G, blk, done, 0, last, twl, ninv, m); break;
    }
    done += R;
    __syncthreads();
  }
}

}  // namespace hs
