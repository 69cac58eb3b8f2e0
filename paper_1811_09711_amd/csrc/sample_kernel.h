// Device code of the sample pass shared by the single-job kernel (sample.hip)
// and the batched queue kernels (queue_f32.hip, queue_f64.hip): the kernel
// argument record, the per-call forward map and one work unit of a pass.
//
// Brass, Kilian, Reuter, arXiv:1811.09711, Sec. 3.5: for every call r_c of
// channel c, x_c = G_c^{-1}(r_c) with the VEGAS step map (Sec. 3.2, eq. g(x)),
// p = phi_c(x_c), f(p), then for every other channel c' the inverse map and the
// bin of x_c' in grid c' (eq. g(p)); the weight is w = f/g (eq. vamp-master).
// Sums of w and w^2 per channel (Sec. 3.1, eq. 4) and the per-bin sums of w^2
// along each axis (eq. 31) are accumulated for the adaptation.
#pragma once

#include <hip/hip_runtime.h>
#include <string.h>

#include "mcv_internal.h"
#include "mcv_point.h"

namespace mcv {

namespace {


template <typename T>
struct SampleArgs {
  int d, K, n, P;
  int sT;               // per-axis table stride (entries)
  int M, mshift;        // hint cells per axis and the log map's shift
  int n_orphan;
  int off_own, off_hist, off_red;
  uint32_t tag;         // iteration tag of trace and unweighting launches
  uint64_t seed;
  const int32_t* iter;  // sample pass: completed passes = this pass's tag
  const int64_t* start;
  const double* alpha;
  const DimMap<T>* cmap;
  const ChanType* ctype;
  const T* cnorm;
  const T* twin_pn;
  const PeakDim<T>* pmap;
  const T* pnorm;
  const int32_t* orphans;
  const Pair<T>* xtab;   // [K][d][sT]
  const Pair<T>* ptab;   // [K][d][sT]
  const Cell<T>* ctab;   // [K][d][M]
  const T* gbound;       // [K]
  const T* aterm;        // [3][K]: (T)alpha_c gbound_c, (T)alpha_c cnorm_c, alpha_c cnorm_c 2^s(1+m)
  const T* gab;          // [K][d][2] density-kernel constants
  const float* hab;      // [K][d][2] hint-map constants
  const int32_t* skx;    // [K][2] partial-exponent skip offsets
  double* part;
  double* hpart;
  // trace instantiation only: f, g, w of calls [tr_first, tr_first + tr_count)
  int64_t tr_first, tr_count;
  double* tr_out;        // [tr_count][3]
  int rng;               // 0 Philox4x32-10, 1 MRG32k3a streams
  const uint32_t* mrg;   // MRG32k3a jump tables and stream starts (JobDev::mrg)
  int strat;             // 0 uniform r; s >= 2 pseudo-stratified (>= s calls per box)
  const int64_t* nr;     // [K] stratified layout: boxes per axis
  const int64_t* spb;    // [K] calls per box
  const int64_t* bstart; // [K+1] box prefix
};

// Stratified sampling: bin j and fraction of one axis from the box digit b
// and the word u: r = (b + u 2^-32) / nr as the fixed-point R = b 2^32 + u
// over nr 2^32 (R n < 2^60 for nr <= 2^20, n <= 256); j = floor(R n /
// (nr 2^32)); fraction (rem + 1/2) / (nr 2^32), rem = R n - j nr 2^32 (one
// correctly rounded FP64 division); FP32 rounds it to FP32, the largest
// float below 1 if that gives 1.
template <typename T>
__device__ inline void strat_bin_frac(uint32_t b, uint32_t u, uint32_t nr, int n, uint32_t& j,
                                      T& fr) {
  const uint64_t Rn = (((uint64_t)b << 32) | u) * (uint64_t)n;
  const uint32_t hi32 = (uint32_t)(Rn >> 32);
  j = hi32 / nr;
  const uint64_t rem = ((uint64_t)(hi32 - j * nr) << 32) | (uint32_t)Rn;
  const double f = ((double)rem + 0.5) / ((double)nr * 4294967296.0);
  if constexpr (sizeof(T) == 4) {
    const float f32 = (float)f;
    fr = f32 >= 1.0f ? 0x1.fffffep-1f : f32;
  } else {
    fr = f;
  }
}

// The MRG32k3a state of the call with index i_c among channel c's calls at
// iteration tag t: stream start of c, 64 t steps in, substream i_c.
__device__ inline Mrg mrg_call_state(const uint32_t* mrg, int K_or_c, uint64_t i_c, uint32_t t) {
  CP<uint32_t> tab = cp(mrg);
  CP<uint32_t> st = tab + (size_t)kMrgTables * kMrgEntry + (size_t)K_or_c * 6;
  Mrg s{{st[0], st[1], st[2]}, {st[3], st[4], st[5]}};
  mrg_jump(tab, 0, 64ull * t, s);
  mrg_jump(tab, kMrgSubBase, i_c, s);
  return s;
}

// Cooperative copy global -> LDS in 16-byte units (both ends 16-byte aligned,
// bytes a multiple of 16).
__device__ inline void copy16(void* dst, const void* src, int bytes, int block) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(dst);
  const int n = bytes >> 4;
  for (int t = threadIdx.x; t < n; t += block) d[t] = s[t];
}

template <int MAXD>
__device__ __forceinline__ void draw_words(uint64_t seed, uint64_t i, uint32_t tag, int d,
                                  uint32_t (&u)[MAXD]) {
#pragma unroll
  for (int b = 0; b < (MAXD + 3) / 4; ++b) {
    if (4 * b < d) {
      const U4 r = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), tag, (uint32_t)b},
                                 (uint32_t)seed, (uint32_t)(seed >> 32));
      if (4 * b + 0 < MAXD) u[4 * b + 0] = r.x;
      if (4 * b + 1 < MAXD) u[4 * b + 1] = r.y;
      if (4 * b + 2 < MAXD) u[4 * b + 2] = r.z;
      if (4 * b + 3 < MAXD) u[4 * b + 3] = r.w;
    }
  }
}

// Forward part of one call of channel c: bins, x, p = phi_c(x) and the own
// grid density prod_k 1/(n Delta) (eq. g(x)), from the channel's x-space
// (edge, density) tables ot (per-axis stride sT).
template <typename T, int MAXD, bool REFINED = false>
__device__ inline T forward_point(const uint32_t (&u)[MAXD], int d, int n, CP<DimMap<T>> cm,
                                  const Pair<T>* ot, int sT, T (&p)[MAXD],
                                  uint32_t (&jpack)[(MAXD + 3) / 4]) {
  T own = T(1);
#pragma unroll
  for (int k = 0; k < (MAXD + 3) / 4; ++k) jpack[k] = 0u;
#pragma unroll
  for (int k = 0; k < MAXD; ++k) {
    if (k < d) {
      const uint32_t j = __umulhi(u[k], (uint32_t)n);
      const uint32_t lo = u[k] * (uint32_t)n;
      const T fr = Frac<T>::get(lo);
      const Pair<T> a0 = ot[k * sT + j], a1 = ot[k * sT + j + 1];
      const T w = a1.e - a0.e;
      const T x = a0.e + fr * w;
      const T xc = (T(1) - a1.e) + (T(1) - fr) * w;
      p[k] = map_forward<T, CP<DimMap<T>>, REFINED>(cm + k, x, xc);
      own *= a0.dens;
      jpack[k >> 2] |= j << (8 * (k & 3));
    } else {
      p[k] = T(0);
    }
  }
  return own;
}

// The same from given bins and fractions (stratified sampling).
template <typename T, int MAXD>
__device__ inline T forward_point_jf(const uint32_t (&jj)[MAXD], const T (&frs)[MAXD], int d,
                                     CP<DimMap<T>> cm, const Pair<T>* ot, int sT, T (&p)[MAXD],
                                     uint32_t (&jpack)[(MAXD + 3) / 4]) {
  T own = T(1);
#pragma unroll
  for (int k = 0; k < (MAXD + 3) / 4; ++k) jpack[k] = 0u;
#pragma unroll
  for (int k = 0; k < MAXD; ++k) {
    if (k < d) {
      const uint32_t j = jj[k];
      const T fr = frs[k];
      const Pair<T> a0 = ot[k * sT + j], a1 = ot[k * sT + j + 1];
      const T w = a1.e - a0.e;
      const T x = a0.e + fr * w;
      const T xc = (T(1) - a1.e) + (T(1) - fr) * w;
      p[k] = map_forward<T>(cm + k, x, xc);
      own *= a0.dens;
      jpack[k >> 2] |= j << (8 * (k & 3));
    } else {
      p[k] = T(0);
    }
  }
  return own;
}

// ---------------------------------------------------------------------------
// Full evaluation of one call from global-memory tables (trace and
// unweighting): every other channel's bin is found, none is skipped.
// ---------------------------------------------------------------------------
// own: the call's own grid density and packed own bins (forward map done).
template <typename T, int MAXD>
__device__ __forceinline__ void eval_channels(const SampleArgs<T>& a, const double* alpha_g, int c,
                                              T own, const uint32_t (&jp)[(MAXD + 3) / 4],
                                              const T (&p)[MAXD], T& f, T& g, int32_t* bins) {
  const int d = a.d, n = a.n, K = a.K;
  CP<double> alpha = cp(alpha_g);
  CP<DimMap<T>> cmap = cp(a.cmap);
  CP<ChanType> ctype = cp(a.ctype);
  CP<T> cnorm = cp(a.cnorm);
  CP<T> twin = cp(a.twin_pn);
  CP<T> gab = cp(a.gab);
  CP<float> hab = cp(a.hab);
  const int sT = a.sT;
  f = T(0);
  g = T(0);
  for (int cc = 0; cc < K; ++cc) {
    CP<T> gab_cc = gab + (size_t)cc * 2 * d;
    const T r = chan_r<T, MAXD>(gab_cc, ctype[cc].iso, ctype[cc].gmask, ctype[cc].bmask, d, p);
    f += twin[cc] * r;
    const T qd = cnorm[cc] * r;
    T Gd = T(1);
    if (cc == c) {
      Gd = own;
      if (bins)
        for (int k = 0; k < d; ++k) bins[c * d + k] = (jp[k >> 2] >> (8 * (k & 3))) & 0xFF;
    } else {
      int jb[MAXD];
      const Pair<T>* T0 = a.ptab + (size_t)cc * d * sT;
      const Cell<T>* C0 = a.ctab + (size_t)cc * d * a.M;
      Gd = ctype[cc].lin
               ? grid_density<T, MAXD, 1, true>(T0, C0, sT, n, d, a.M, a.mshift,
                                                hab + (size_t)cc * 2 * d, p, jb)
               : grid_density<T, MAXD, 1, false>(T0, C0, sT, n, d, a.M, a.mshift,
                                                 hab + (size_t)cc * 2 * d, p, jb);
      if (bins)
        for (int k = 0; k < d; ++k) bins[cc * d + k] = jb[k];
    }
    g += (T)alpha[cc] * Gd * qd;
  }
  CP<PeakDim<T>> pmap = cp(a.pmap);
  CP<T> pnorm = cp(a.pnorm);
  CP<int32_t> orphans = cp(a.orphans);
  for (int o = 0; o < a.n_orphan; ++o) {
    const int i2 = orphans[o];
    f += pnorm[i2] * peak_r<T, MAXD>(pmap + (size_t)i2 * d, d, p);
  }
}

template <typename T, int MAXD>
__device__ __forceinline__ void eval_call(const SampleArgs<T>& a, const double* alpha_g, int c,
                                          const uint32_t (&u)[MAXD], T (&p)[MAXD], T& f, T& g,
                                          int32_t* bins /* [K][d] or null */) {
  uint32_t jp[(MAXD + 3) / 4];
  const T own = forward_point<T, MAXD>(u, a.d, a.n, cp(a.cmap) + (size_t)c * a.d,
                                       a.xtab + (size_t)c * a.d * a.sT, a.sT, p, jp);
  eval_channels<T, MAXD>(a, alpha_g, c, own, jp, p, f, g, bins);
}

// The same from given bins and fractions of the call's own grid.
template <typename T, int MAXD>
__device__ __forceinline__ void eval_call_jf(const SampleArgs<T>& a, const double* alpha_g, int c,
                                             const uint32_t (&jj)[MAXD], const T (&fr)[MAXD],
                                             T (&p)[MAXD], T& f, T& g, int32_t* bins) {
  uint32_t jp[(MAXD + 3) / 4];
  const T own = forward_point_jf<T, MAXD>(jj, fr, a.d, cp(a.cmap) + (size_t)c * a.d,
                                          a.xtab + (size_t)c * a.d * a.sT, a.sT, p, jp);
  eval_channels<T, MAXD>(a, alpha_g, c, own, jp, p, f, g, bins);
}

// Axes of the partial exponent of the all-Gaussian skip test.
constexpr int kPartial = 3;

// floor(log2 max(x, smallest normal)) for x >= 0 (the smallest normal's half
// ulp is the denormals' half spacing, so a term below it leaves 0 and every
// denormal sum unchanged).
__device__ inline int floor_log2_normal(float x) {
  return __builtin_amdgcn_frexp_expf(fmaxf(x, 0x1p-126f)) - 1;
}
__device__ inline int floor_log2_normal(double x) {
  return __builtin_amdgcn_frexp_exp(fmax(x, 0x1p-1022)) - 1;
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int off) {
  const uint32_t lo = __shfl_xor((uint32_t)v, off);
  const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), off);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Every other channel's terms of one call of channel c at point p (eq. g(p)
// and the integrand's peaks): f += twin r for each channel's density kernel
// r, gg += alpha G q for the terms that can change gg (reading R25: exactly
// zero terms and, with TB, terms below half an ulp of gg are skipped, which
// leaves gg as the full sum gives it), then the peaks that share no
// channel's kernel.  GROUP hint-cell reads are issued together; EXACT: d is
// MAXD.  M, mshift: the job's hint cells per axis and the log map's shift.
// LAZY (with TB): crowded hint cells are walked only where their bound
// cannot rule the term out (see below).
template <typename T, int MAXD, int GROUP, bool EXACT, bool TB, bool LAZY = false>
__device__ __forceinline__ void other_terms(const SampleArgs<T>& a, int c, int d, int M,
                                            int mshift, const T (&p)[MAXD], T& f, T& gg) {
  const int n = a.n, K = a.K, sT = a.sT;
  const int chT = d * sT, chC = d * M;  // entries per channel table, cells per channel
  CP<ChanType> ctype = cp(a.ctype);
  CP<T> twin = cp(a.twin_pn);
  CP<PeakDim<T>> pmap = cp(a.pmap);
  CP<T> pnorm = cp(a.pnorm);
  CP<T> aterm = cp(a.aterm);
  CP<T> gab = cp(a.gab);
  CP<float> hab = cp(a.hab);
  CP<int32_t> skx = cp(a.skx);
  CP<int32_t> orphans = cp(a.orphans);
  for (int cc = 0; cc < K; ++cc) {
    if (cc == c) continue;
    const int iso = ctype[cc].iso;
    const uint32_t bm = ctype[cc].bmask;
    CP<T> gab_cc = gab + (size_t)cc * 2 * d;
    T r;
    if (TB && sizeof(T) == 8 && iso) {
      // The exponent of the first kPartial axes bounds r from above
      // (the full sum only adds non-negative terms): when that bound
      // shows, on every lane of the wavefront, both of the channel's
      // terms below half an ulp of f and of gg, neither sum can change
      // and the wavefront skips the channel.  Otherwise the sum
      // continues in the same order, so r is the value the full
      // evaluation gives.  FP64 only: in FP32 the test cost more than
      // it saved (d = 10, 32 channels: FP32 8.2 -> 8.6 ms per 1e8 calls,
      // and 6.55 -> 7.19 ms with the later kernel; FP64 24.3 -> 23.3 ms).
      // (the sum of (p_k - m_k)^2, scaled by ga^2, as chan_r)
      const T sc = gab_cc[d];
      T gs = T(0);
#pragma unroll
      for (int k = 0; k < kPartial && k < MAXD; ++k) {
        if (k < d) {
          const T z = p[k] - gab_cc[k];
          gs = fma(z, z, gs);
        }
      }
      const int thr = max(skx[2 * cc] - floor_log2_normal(f),
                          skx[2 * cc + 1] - floor_log2_normal(gg));
      if (__all(gs * sc >= (T)thr)) continue;
#pragma unroll
      for (int k = kPartial; k < MAXD; ++k) {
        if (k < d) {
          const T z = p[k] - gab_cc[k];
          gs = fma(z, z, gs);
        }
      }
      r = m_exp2(-(gs * sc));
    } else {
      r = chan_r<T, MAXD>(gab_cc, iso, ctype[cc].gmask, bm, d, p);
    }
    f += twin[cc] * r;
    // The term alpha G q of channel cc needs G (d lookups) only when it
    // can change gg.  Terms are non-negative, so gg only grows, and a
    // term below half an ulp of gg leaves it unchanged: skipping such a
    // term gives the same gg as adding it.  (alpha gbound) r < gg
    // bounds the term by gg 2^-25 (FP32; 2^-54 in FP64), below half an
    // ulp.  Exactly zero terms are skipped as well.  The factors
    // (T)alpha gbound and (T)alpha cnorm come formed with the allocation.
    if (r != T(0) && !(TB && aterm[cc] * r < gg)) {
      GP<Pair<T>> T0 = gptr(a.ptab + (size_t)cc * chT);
      GP<Cell<T>> C0 = gptr(a.ctab + (size_t)cc * chC);
      CP<float> hab_cc = hab + (size_t)cc * 2 * d;
      const bool lin = ctype[cc].lin;
      // LAZY: crowded cells first give their largest density (an upper bound
      // of G); the exact walks run only on the lanes where that bound, in the
      // same test with the looked-up densities in place of the maxima, shows
      // the term able to change gg.  Elsewhere the term is below half an ulp
      // of gg, exact or not, and gg is unchanged.
      static_assert(!LAZY || TB, "the lazy walks rest on the term bound");
      bool crowded = false;
      T Gd = lin ? grid_density<T, MAXD, GROUP, true, EXACT, LAZY>(T0, C0, sT, n, d, M, mshift,
                                                                  hab_cc, p, nullptr, &crowded)
                 : grid_density<T, MAXD, GROUP, false, EXACT, LAZY>(T0, C0, sT, n, d, M, mshift,
                                                                   hab_cc, p, nullptr, &crowded);
      if (LAZY && crowded && !(aterm[2 * K + cc] * r * Gd < gg))
        Gd = lin ? grid_density<T, MAXD, GROUP, true, EXACT>(T0, C0, sT, n, d, M, mshift, hab_cc,
                                                             p, nullptr)
                 : grid_density<T, MAXD, GROUP, false, EXACT>(T0, C0, sT, n, d, M, mshift,
                                                              hab_cc, p, nullptr);
      gg += aterm[K + cc] * Gd * r;
    }
  }
  for (int o = 0; o < a.n_orphan; ++o) {
    const int i2 = orphans[o];
    f += pnorm[i2] * peak_r<T, MAXD>(pmap + (size_t)i2 * d, d, p);
  }
}

// ---------------------------------------------------------------------------
// The sample pass.  Every thread takes one call of the segment's channel c per
// round: draws, forward map and own grid density, then one loop over the
// other channels computes each density kernel r once; the integrand collects
// the peaks that share a channel's exponential (then the remaining peaks),
// and every channel with a non-zero density adds alpha G q to g, its grid
// density G found from the channel's hint-cell records (global memory, L2),
// with its (edge, density) table for the rare exact walks.  The segment's own
// x-space table and its per-bin sums of w^2 live in LDS.
// ---------------------------------------------------------------------------

// One work unit of a pass: unit g of the job's G units takes the calls
// [g N/G, (g+1) N/G).  BLOCK > 0: the workgroup size as a constant, else
// blockDim.x.  EXACT: the job's dimension is MAXD (no per-axis guards).
// TB: a channel's lookups are guarded by its term bound (else only exactly
// zero terms are skipped); the results are the same either way.  TRACE:
// also write f, g and w of the calls in the argument record's trace window
// (the same code path otherwise).  MT > 0: the job's hint cells per axis as
// a constant (its offsets fold into immediates).  Every thread of the
// workgroup calls it with the same unit.
template <typename T, int MAXD, int BLOCK, bool EXACT, bool TB, bool TRACE = false, int RNG = 0,
          int MT = 0, bool LAZY = false, bool REFINED = false>
__device__ __forceinline__ void sample_unit(const SampleArgs<T>& a, int g, int G, uint32_t tag,
                                            unsigned char* smem) {
  static_assert(RNG == 0 || (BLOCK > 0 && (BLOCK & (BLOCK - 1)) == 0),
                "MRG32k3a substreams advance by a power-of-two workgroup");
  constexpr int GROUP = sizeof(T) == 4 ? 5 : 2;
  const int block = BLOCK > 0 ? BLOCK : (int)blockDim.x;
  const int waves = block >> 6;
  Pair<T>* ownT = reinterpret_cast<Pair<T>*>(smem + a.off_own);
  double* hist = reinterpret_cast<double*>(smem + a.off_hist);
  double* red = reinterpret_cast<double*>(smem + a.off_red);

  const int d = EXACT ? MAXD : a.d, n = a.n, K = a.K;
  const int tid = threadIdx.x;
  CP<int64_t> start = cp(a.start);
  CP<double> alpha = cp(a.alpha);
  CP<DimMap<T>> cmap = cp(a.cmap);
  CP<ChanType> ctype = cp(a.ctype);
  CP<T> cnorm = cp(a.cnorm);
  CP<T> twin = cp(a.twin_pn);
  CP<T> gab = cp(a.gab);

  const int64_t ntot = start[K];
  const int64_t lo = (int64_t)g * ntot / G;
  const int64_t hi = (int64_t)(g + 1) * ntot / G;
  if (lo >= hi) return;  // uniform over the workgroup
  const int dn = d * n;
  const int sT = a.sT;
  // hint cells per axis: the constant MT (256 or 512), else the job's
  const int M = MT > 0 ? MT : a.M;
  const int mshift = MT > 0 ? (MT == 512 ? 18 : 19) : a.mshift;
  const int chT = d * sT;  // entries per channel table

  for (int t = tid; t < dn; t += block) hist[t] = 0.0;

  int c = 0;
  while (c < K - 1 && start[c + 1] <= lo) ++c;
  for (; c < K && start[c] < hi; ++c) {
    const int64_t s0 = start[c] > lo ? start[c] : lo;
    const int64_t s1 = start[c + 1] < hi ? start[c + 1] : hi;
    __syncthreads();
    copy16(ownT, a.xtab + (size_t)c * chT, chT * (int)sizeof(Pair<T>), block);
    __syncthreads();

    // Per-lane sums of w and w^2 of the segment: plain FP64 sums over at
    // most kFold rounds, folded into compensated sums (little state live
    // across the channel loop).
    constexpr int kFold = 16;
    Neu S1{0.0, 0.0}, S2{0.0, 0.0};
    double q1 = 0.0, q2 = 0.0;
    int rounds = 0;
    T wmax = T(0);
    uint32_t nbad = 0u;
    const T al_c = (T)alpha[c];
    CP<DimMap<T>> cm_c = cmap + (size_t)c * d;
    const T own_norm = al_c * cnorm[c];
    const int iso_c = ctype[c].iso;
    const uint32_t gm_c = ctype[c].gmask, bm_c = ctype[c].bmask;
    const T tw_c = twin[c];
    // MRG32k3a: this lane's first call of the segment is substream
    // s0 + tid - start[c] of channel c's stream; each round moves BLOCK
    // substreams on
    Mrg mst{};
    if constexpr (RNG == 1)
      mst = mrg_call_state(a.mrg, c, (uint64_t)(s0 + tid - start[c]), tag);

    for (int64_t base = s0; base < s1; base += block) {
      const int64_t i = base + tid;
      const bool valid = i < s1;
      T p[MAXD];
      uint32_t jp[(MAXD + 3) / 4];
      T f = T(0), gg = T(1);
      if (valid) {
        uint32_t u[MAXD];
        if constexpr (RNG == 1) {
          Mrg w = mst;
#pragma unroll
          for (int k = 0; k < MAXD; ++k)
            if (k < d) u[k] = mrg_word(w);
        } else {
          draw_words<MAXD>(a.seed, (uint64_t)i, tag, d, u);
        }
        const T own = forward_point<T, MAXD, REFINED>(u, d, n, cm_c, ownT, sT, p, jp);
        const T r_c = chan_r<T, MAXD>(gab + (size_t)c * 2 * d, iso_c, gm_c, bm_c, d, p);
        f = tw_c * r_c;
        gg = own_norm * own * r_c;
        other_terms<T, MAXD, GROUP, EXACT, TB, LAZY>(a, c, d, M, mshift, p, f, gg);
      }
      // ---- weights and sums (FP64)
      if (valid) {
        const T wt = f / gg;
        if constexpr (TRACE) {
          if (i >= a.tr_first && i < a.tr_first + a.tr_count) {
            double* o = a.tr_out + (i - a.tr_first) * 3;
            o[0] = (double)f;
            o[1] = (double)gg;
            o[2] = (double)wt;
          }
        }
        const double w = (double)wt;
        if (!isfinite(wt)) {
          ++nbad;
        } else {
          q1 += w;
          const double w2 = w * w;
          q2 += w2;
          const T aw = fabs(wt);  // signed integrands: the largest |w|
          wmax = aw > wmax ? aw : wmax;
#pragma unroll
          for (int k = 0; k < MAXD; ++k) {
            if (k < d) {
              const int jb = (jp[k >> 2] >> (8 * (k & 3))) & 0xFF;
              __hip_atomic_fetch_add(hist + k * n + jb, w2, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
            }
          }
        }
      }
      if constexpr (RNG == 1) {
        constexpr int kLog2Block = __builtin_ctz((unsigned)(BLOCK > 0 ? BLOCK : 1));
        mrg_apply(cp(a.mrg) + (size_t)(kMrgSubBase + kLog2Block) * kMrgEntry, mst);
      }
      if (++rounds == kFold) {  // uniform
        S1.add(q1);
        S2.add(q2);
        q1 = 0.0;
        q2 = 0.0;
        rounds = 0;
      }
    }
    S1.add(q1);
    S2.add(q2);

    // segment reduction: wavefront butterflies, then LDS across waves
    double wmax_d = (double)wmax, nbad_d = (double)nbad;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const Neu o1{__shfl_xor(S1.s, off), __shfl_xor(S1.c, off)};
      const Neu o2{__shfl_xor(S2.s, off), __shfl_xor(S2.c, off)};
      S1 = neu_merge(S1, o1);
      S2 = neu_merge(S2, o2);
      wmax_d = fmax(wmax_d, __shfl_xor(wmax_d, off));
      nbad_d += __shfl_xor(nbad_d, off);
    }
    const int wave = tid >> 6;
    if ((tid & 63) == 0) {
      red[wave * 6 + 0] = S1.s;
      red[wave * 6 + 1] = S1.c;
      red[wave * 6 + 2] = S2.s;
      red[wave * 6 + 3] = S2.c;
      red[wave * 6 + 4] = wmax_d;
      red[wave * 6 + 5] = nbad_d;
    }
    __syncthreads();
    const size_t slot = (size_t)g + (size_t)c;
    if (tid == 0) {
      Neu A{red[0], red[1]}, B{red[2], red[3]};
      double wm = red[4], nb = red[5];
      for (int w = 1; w < waves; ++w) {
        A = neu_merge(A, Neu{red[w * 6 + 0], red[w * 6 + 1]});
        B = neu_merge(B, Neu{red[w * 6 + 2], red[w * 6 + 3]});
        wm = fmax(wm, red[w * 6 + 4]);
        nb += red[w * 6 + 5];
      }
      double* r = a.part + slot * kPartStride;
      r[0] = A.s;
      r[1] = A.c;
      r[2] = B.s;
      r[3] = B.c;
      r[4] = wm;
      r[5] = nb;
    }
    for (int t = tid; t < dn; t += block) {
      a.hpart[slot * dn + t] = hist[t];
      hist[t] = 0.0;
    }
  }
}

// A wave-uniform record read with scalar loads.
template <typename S>
__device__ __forceinline__ S load_uniform(const S* p) {
  static_assert(sizeof(S) % 4 == 0, "record of whole dwords");
  S out;
  uint32_t* o = reinterpret_cast<uint32_t*>(&out);
  CP<uint32_t> q = (CP<uint32_t>)(p);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(S) / 4); ++i) o[i] = q[i];
  return out;
}

// Batched pass: a persistent grid drains the work units spanning every job
// of a set.  Unit u belongs to the job jb with prefix[jb] <= u <
// prefix[jb+1] and is that job's unit u - prefix[jb] of prefix[jb+1] -
// prefix[jb]; each job's arguments (and LDS layout, after a 16-byte header
// that broadcasts the unit index) come from args[jb].  A unit's result does
// not depend on which workgroup runs it.
//
// The units are split into kQueues contiguous ranges, one queue each
// (counter[q] counts the units taken from range q).  Workgroups are
// dispatched to the chip's 8 XCDs in turn (workgroup w on XCD w mod 8), so
// workgroup w drains queue w mod 8 first: every XCD works on a contiguous
// stretch of jobs and its own L2 holds only their hint-cell tables.  A
// workgroup whose queue is empty takes units from the next queues in turn,
// and leaves once every queue is empty.  The counters are zeroed by the
// allocation kernel before each pass.  LB: the launch bound (largest
// workgroup size); 512 leaves the compiler more registers per lane, 256 caps
// them for at least 6 (FP32; 69.1 ms on the 256-job batch, against 69.9 at 7
// and 73.0 at 8) or 4 (FP64) waves per SIMD.  TB: lookups
// guarded by the channels' term bounds.
constexpr int kQueues = 8;

// One unit of a batched pass, compiled for the job's dimension: d <= 12
// exactly (no per-axis guards; the grouped hint-cell reads cover only the
// job's axes, where a 12-axis body would read 5, 10 or 15 cells for any d),
// a larger d through the generic body of the bucket MAXD.  d is uniform over
// the workgroup, and the set orders its jobs by d, so the workgroups of one
// XCD mostly run one body at a time.
template <typename T, int MAXD, bool TB>
__device__ __forceinline__ void queue_unit(const SampleArgs<T>& a, int u, int G, uint32_t tag,
                                           unsigned char* smem) {
#define MCV_EXACT_CASE(D)                                   \
  case D:                                                   \
    if constexpr (D <= MAXD) {                              \
      sample_unit<T, D, 0, true, TB>(a, u, G, tag, smem);   \
      return;                                               \
    }                                                       \
    break;
  switch (a.d) {
    MCV_EXACT_CASE(1)
    MCV_EXACT_CASE(2)
    MCV_EXACT_CASE(3)
    MCV_EXACT_CASE(4)
    MCV_EXACT_CASE(5)
    MCV_EXACT_CASE(6)
    MCV_EXACT_CASE(7)
    MCV_EXACT_CASE(8)
    MCV_EXACT_CASE(9)
    MCV_EXACT_CASE(10)
    MCV_EXACT_CASE(11)
    MCV_EXACT_CASE(12)
    default:
      break;
  }
#undef MCV_EXACT_CASE
  if constexpr (MAXD > 12) sample_unit<T, MAXD, 0, false, TB>(a, u, G, tag, smem);
}

template <typename T, int MAXD, int LB, bool TB>
__global__ __launch_bounds__(LB, LB == 256 ? (sizeof(T) == 4 ? 6 : 4) : 1) void k_sample_queue(
    const SampleArgs<T>* args, const int* prefix, int n_jobs, int n_units, int* counter) {
  extern __shared__ __align__(16) unsigned char smem[];
  int* bcast = reinterpret_cast<int*>(smem);
  CP<int> pf = cp(prefix);
  const int home = (int)(blockIdx.x % kQueues);
  int tried = 0;  // queues found empty (thread 0's view; the unit is broadcast)
  for (;;) {
    if (threadIdx.x == 0) {
      int unit = -1;
      while (tried < kQueues) {
        const int q = (home + tried) % kQueues;
        const int lo = (int)((int64_t)n_units * q / kQueues);
        const int hi = (int)((int64_t)n_units * (q + 1) / kQueues);
        const int k = lo < hi ? atomicAdd(counter + q, 1) : 0;
        if (lo + k < hi) {
          unit = lo + k;
          break;
        }
        ++tried;
      }
      bcast[0] = unit;
    }
    __syncthreads();
    const int u = __builtin_amdgcn_readfirstlane(bcast[0]);
    __syncthreads();
    if (u < 0) break;
    int lo = 0, hi = n_jobs;  // largest jb with prefix[jb] <= u
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (pf[mid] <= u) lo = mid;
      else hi = mid;
    }
    const int u0 = pf[lo];
    const int G = pf[lo + 1] - u0;
    const SampleArgs<T> a = load_uniform(args + lo);
    const uint32_t tag = (uint32_t)cp(a.iter)[0];
    queue_unit<T, MAXD, TB>(a, u - u0, G, tag, smem);
  }
}

// Launch shape of the single-job kernel per precision (measured best on the
// d = 10, 32-channel, 100-bin workload):
// 256-thread workgroups with the registers capped for 7 (FP32) or 4 (FP64)
// waves per SIMD (a few spills, more latency hidden; FP32 at 5, 6, 7 and 8
// waves: 6.45, 6.00, 5.62 and 5.75 ms).  With MRG32k3a streams (more state
// per lane) 6 was faster with one co-resident set of workgroups (6.85 ms
// against 7.05 at 7), 7 with up to 8 sets (5.24 against 5.31).
template <typename T>
struct Tune;
template <>
struct Tune<float> {
  static constexpr int BLOCK = 256, PPT = 1, MIN_WAVES = 7, MIN_WAVES_MRG = 7;
};
template <>
struct Tune<double> {
  static constexpr int BLOCK = 256, PPT = 1, MIN_WAVES = 4, MIN_WAVES_MRG = 4;
};
template <typename T, int RNG>
constexpr int kMinWaves = RNG == 1 ? Tune<T>::MIN_WAVES_MRG : Tune<T>::MIN_WAVES;

// Single-job pass: workgroup g of the grid is unit g.  RNG: 0 Philox words,
// 1 MRG32k3a streams.  Lazy walks in FP32 only (d = 10, 32 channels: FP32
// 6.16 -> 5.91 ms with them, FP64 22.4 -> 23.1 ms; the batched pass, whose
// channels all use the log map, 69 -> 76 ms, so it does without).
template <typename T>
constexpr bool kLazyWalks = sizeof(T) == 4;

template <typename T, int MAXD, int PPT, int BLOCK, bool EXACT, int RNG = 0, int MT = 0>
__global__ __launch_bounds__(BLOCK, (kMinWaves<T, RNG>)) void k_sample(SampleArgs<T> a) {
  static_assert(PPT == 1, "one call per thread and round");
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t tag = (uint32_t)cp(a.iter)[0];
  sample_unit<T, MAXD, BLOCK, EXACT, true, false, RNG, MT, kLazyWalks<T>, true>(
      a, blockIdx.x, gridDim.x, tag, smem);
}

// The single-job pass with its trace window written (k_sample's code path,
// launch bounds and grid; the iteration tag comes from the argument record).
template <typename T, int MAXD, int PPT, int BLOCK, bool EXACT, int RNG = 0, int MT = 0>
__global__ __launch_bounds__(BLOCK, (kMinWaves<T, RNG>)) void k_sample_trace(SampleArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  sample_unit<T, MAXD, BLOCK, EXACT, true, true, RNG, MT, kLazyWalks<T>, true>(
      a, blockIdx.x, gridDim.x, a.tag, smem);
}


// ---------------------------------------------------------------------------
// Host side: argument records, LDS layouts and launch shapes.
// ---------------------------------------------------------------------------
template <typename T>
SampleArgs<T> make_args(const JobDev& j, uint32_t tag) {
  SampleArgs<T> a{};
  a.d = j.d;
  a.K = j.K;
  a.n = j.n;
  a.P = j.P;
  a.sT = j.sT;
  a.M = j.M;
  a.mshift = j.mshift;
  a.tag = tag;
  a.seed = j.seed;
  a.iter = j.iter_dev;
  a.start = j.start;
  a.alpha = j.alpha;
  a.ctype = j.ctype;
  a.orphans = j.orphans;
  a.n_orphan = j.n_orphan;
  if (sizeof(T) == 8) {
    a.cmap = reinterpret_cast<const DimMap<T>*>(j.cmap64);
    a.cnorm = reinterpret_cast<const T*>(j.cnorm64);
    a.twin_pn = reinterpret_cast<const T*>(j.twin_pn64);
    a.pmap = reinterpret_cast<const PeakDim<T>*>(j.pmap64);
    a.pnorm = reinterpret_cast<const T*>(j.pnorm64);
  } else {
    a.cmap = reinterpret_cast<const DimMap<T>*>(j.cmap32);
    a.cnorm = reinterpret_cast<const T*>(j.cnorm32);
    a.twin_pn = reinterpret_cast<const T*>(j.twin_pn32);
    a.pmap = reinterpret_cast<const PeakDim<T>*>(j.pmap32);
    a.pnorm = reinterpret_cast<const T*>(j.pnorm32);
  }
  a.xtab = reinterpret_cast<const Pair<T>*>(j.xtab);
  a.ptab = reinterpret_cast<const Pair<T>*>(j.ptab);
  a.ctab = reinterpret_cast<const Cell<T>*>(j.ctab);
  a.gbound = reinterpret_cast<const T*>(j.gbound);
  a.aterm = reinterpret_cast<const T*>(j.aterm);
  a.gab = reinterpret_cast<const T*>(j.gab);
  a.hab = j.hab;
  a.skx = j.skx;
  a.part = j.part;
  a.hpart = j.hpart;
  a.rng = j.rng;
  a.mrg = j.mrg;
  a.strat = j.strat;
  a.nr = j.nr;
  a.spb = j.spb;
  a.bstart = j.bstart;
  return a;
}

static inline int align16(int x) { return (x + 15) & ~15; }


// LDS layout of the sample kernel from byte `base` on: the own channel's
// x-space table, the per-bin sums of w^2 and the cross-wave reduction.
// Returns the end of the layout (bytes used, base included).
template <typename T>
int lds_layout(SampleArgs<T>& a, int waves, int base = 0) {
  const int chT = a.d * a.sT * (int)sizeof(Pair<T>);
  int off = base;
  a.off_own = off;
  off += align16(chT);
  a.off_hist = off;
  off += align16(a.d * a.n * 8);
  a.off_red = off;
  off += align16(waves * 6 * 8);
  return off;
}

// Workgroups of one pass: as many as are co-resident (per_cu per CU) and no
// more than leave every workgroup a few rounds; with oversub, up to oversub
// times the co-resident count where every workgroup still gets 32 rounds
// (the hardware starts the later ones as earlier ones finish); at most the
// partial buffers' units.
int grid_for(const JobDev& j, int per_cu, int per_round, int64_t n_points, int oversub = 1) {
  if (per_cu < 1) per_cu = 1;
  int64_t G = (int64_t)j.n_cu * per_cu;
  const int64_t want = (n_points + 4 * (int64_t)per_round - 1) / (4 * (int64_t)per_round);
  if (want < G) G = want > 0 ? want : 1;
  if (oversub > 1) {
    int64_t more = (int64_t)j.n_cu * per_cu * oversub;
    const int64_t full = n_points / (32 * (int64_t)per_round);
    if (full < more) more = full;
    if (more > G) G = more;
  }
  if (G > j.gmax) G = j.gmax;
  return (int)G;
}

constexpr int kOversub = 8;

// Workgroups of k_sample for a pass of n_points (kOversub times its
// occupancy), or -1 if the kernel cannot get its LDS.
template <typename T, int MAXD, bool EXACT, int RNG, int MT>
int sample_grid_m(const JobDev& j, int64_t n_points) {
  constexpr int BLOCK = Tune<T>::BLOCK, PPT = Tune<T>::PPT;
  SampleArgs<T> a = make_args<T>(j, 0);
  const int lds = lds_layout<T>(a, BLOCK / 64);
  auto kern = k_sample<T, MAXD, PPT, BLOCK, EXACT, RNG, MT>;
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds) !=
          hipSuccess)
    return -1;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, BLOCK, lds) !=
      hipSuccess)
    return -1;
  // Units of unequal cost (the channels' calls differ by an order of
  // magnitude in cost) finish unevenly: with up to 8 workgroups per resident
  // slot the late ones overlap the tail.  d = 10, 32 channels, FP32: 1, 2, 4,
  // 8 and 16 times the resident count took 5.57, 5.10, 4.56, 4.37 and 4.41
  // ms (1e8 calls: 8 times is 27 rounds per workgroup; the 32-round floor
  // keeps 6.8 times).
  return grid_for(j, per_cu, BLOCK * PPT, n_points, kOversub);
}

template <typename T, int MAXD, bool EXACT, int RNG, int MT>
int launch_sample_m(const JobDev& j, int64_t n_points, hipStream_t s) {
  constexpr int BLOCK = Tune<T>::BLOCK, PPT = Tune<T>::PPT;
  const int G = sample_grid_m<T, MAXD, EXACT, RNG, MT>(j, n_points);
  if (G < 1) return -1;
  SampleArgs<T> a = make_args<T>(j, 0);
  const int lds = lds_layout<T>(a, BLOCK / 64);
  hipLaunchKernelGGL((k_sample<T, MAXD, PPT, BLOCK, EXACT, RNG, MT>), dim3(G), dim3(BLOCK), lds, s,
                     a);
  return G;
}

// The trace instantiation over the trace allocation (t_start, t_alpha) with
// G workgroups (k_sample's grid for the same pass).
template <typename T, int MAXD, bool EXACT, int RNG, int MT>
int launch_sample_trace_m(const JobDev& j, int G, uint32_t tag, int64_t first, int64_t count,
                          double* out, hipStream_t s) {
  constexpr int BLOCK = Tune<T>::BLOCK, PPT = Tune<T>::PPT;
  SampleArgs<T> a = make_args<T>(j, tag);
  a.start = j.t_start;
  a.alpha = j.t_alpha;
  a.aterm = reinterpret_cast<const T*>(j.t_aterm);
  a.tr_first = first;
  a.tr_count = count;
  a.tr_out = out;
  const int lds = lds_layout<T>(a, BLOCK / 64);
  auto kern = k_sample_trace<T, MAXD, PPT, BLOCK, EXACT, RNG, MT>;
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds) !=
          hipSuccess)
    return -1;
  hipLaunchKernelGGL(kern, dim3(G), dim3(BLOCK), lds, s, a);
  return G;
}

// The single-job pass with Philox words takes the job's hint cells per axis
// as a constant (256 or 512); MRG32k3a passes read it from the arguments.
template <typename T, int MAXD, bool EXACT, int RNG = 0>
int sample_grid_t(const JobDev& j, int64_t n_points) {
  if constexpr (RNG == 0)
    return j.M == 512 ? sample_grid_m<T, MAXD, EXACT, RNG, 512>(j, n_points)
                      : sample_grid_m<T, MAXD, EXACT, RNG, 256>(j, n_points);
  return sample_grid_m<T, MAXD, EXACT, RNG, 0>(j, n_points);
}

template <typename T, int MAXD, bool EXACT, int RNG = 0>
int launch_sample_t(const JobDev& j, int64_t n_points, hipStream_t s) {
  if constexpr (RNG == 0)
    return j.M == 512 ? launch_sample_m<T, MAXD, EXACT, RNG, 512>(j, n_points, s)
                      : launch_sample_m<T, MAXD, EXACT, RNG, 256>(j, n_points, s);
  return launch_sample_m<T, MAXD, EXACT, RNG, 0>(j, n_points, s);
}

template <typename T, int MAXD, bool EXACT, int RNG = 0>
int launch_sample_trace_t(const JobDev& j, int G, uint32_t tag, int64_t first, int64_t count,
                          double* out, hipStream_t s) {
  if constexpr (RNG == 0)
    return j.M == 512
               ? launch_sample_trace_m<T, MAXD, EXACT, RNG, 512>(j, G, tag, first, count, out, s)
               : launch_sample_trace_m<T, MAXD, EXACT, RNG, 256>(j, G, tag, first, count, out, s);
  return launch_sample_trace_m<T, MAXD, EXACT, RNG, 0>(j, G, tag, first, count, out, s);
}


}  // namespace
}  // namespace mcv
