// Device-side building blocks of the multi-channel VEGAS sample pass on
// gfx950: Philox4x32-10, the uniform -> (bin, fraction) rule, the 1-d channel
// maps, channel densities, the peak-mixture integrand and compensated sums.
//
// Method: Brass, Kilian, Reuter, arXiv:1811.09711, Sec. 3.2 (VEGAS step map,
// eq. g(x)), Sec. 3.4 (channel densities q_c = 1/phi_c'), Sec. 3.5 (eq. g(p)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcv {

// Hint cells per axis of a job's grids: 256 for at most 64 bins per axis,
// else 512, so that the cells stay finer than the bins (the linear map puts
// the centre +- 3 sigma on them; the log map gives M/16 cells per octave of
// |z| + 1, 8 octaves on either side of z = 0) while the tables of small
// grids stay small.  The log map's shift is 27 - log2 M.
inline int hint_cells_for_bins(int n) { return n > 64 ? 512 : 256; }
inline int hint_cell_shift(int M) { return M == 512 ? 18 : 19; }

enum { FLAT = 0, GAUSS = 1, BW = 2 };

constexpr uint32_t kTagUnweight = 0x80000000u;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32
// multiplies (multipliers 0xD2511F53, 0xCD9E8D57) with the key bumped by the
// Weyl constants 0x9E3779B9, 0xBB67AE85 between rounds.  Counter layout:
// (sample lo, sample hi, iteration tag, block index), key = seed.
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 32x32 -> 64 product as one 64-bit multiply (one v_mad_u64_u32
    // on the GPU, where separate low and high multiplies are two)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = U4{(uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
           (uint32_t)p0};
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Words 0..nw-1 of sample i (nw <= 36).
__device__ inline void philox_words(uint64_t seed, uint64_t i, uint32_t tag, int nw,
                                    uint32_t* out) {
  for (int b = 0; 4 * b < nw; ++b) {
    const U4 r = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), tag, (uint32_t)b},
                               (uint32_t)seed, (uint32_t)(seed >> 32));
    out[4 * b + 0] = r.x;
    if (4 * b + 1 < nw) out[4 * b + 1] = r.y;
    if (4 * b + 2 < nw) out[4 * b + 2] = r.z;
    if (4 * b + 3 < nw) out[4 * b + 3] = r.w;
  }
}

// ---------------------------------------------------------------------------
// MRG32k3a streams (Sec. 4.4, eq. mrg32k3a and eq. rngstream): two
// order-three recursions modulo m1 = 2^32 - 209 and m2 = 2^32 - 22853,
// x1_n = 1403580 x1_{n-2} - 810728 x1_{n-3}, x2_n = 527612 x2_{n-1} -
// 1370589 x2_{n-3}, combined into z_n = x1_n - x2_n mod m1 (m1 in place of
// 0).  The state of a component is (x_{n-2}, x_{n-1}, x_n); jumps of 2^b
// steps are 3x3 matrices modulo m applied to it (tables built on the host).
// A call's word is floor(z 2^32 / (m1 + 1)), so the bin / fraction rule of
// the Philox words applies unchanged.  Stream, substream and offset of a
// call: see JobDev::mrg.
// ---------------------------------------------------------------------------
constexpr uint32_t kMrgM1 = 4294967087u, kMrgM2 = 4294944443u;
constexpr int kMrgEntry = 18;      // uint32 per jump entry: 3x3 for each component
constexpr int kMrgSubBase = 64;    // entries 0..63: 2^b steps; 64..127: 2^(76+b)
constexpr int kMrgTables = 128;    // jump entries before the stream starts

struct Mrg {
  uint32_t a[3], b[3];
};

// x mod m1 (x < 2^64), from 2^32 = 209 mod m1: two folds leave x < 2 m1.
__host__ __device__ inline uint32_t mrg_mod1(uint64_t x) {
  x = (x >> 32) * 209u + (uint32_t)x;
  x = (x >> 32) * 209u + (uint32_t)x;
  return (uint32_t)(x >= kMrgM1 ? x - kMrgM1 : x);
}
// x mod m2 (x < 2^64), from 2^32 = 22853 mod m2: two folds leave x < 2 m2.
__host__ __device__ inline uint32_t mrg_mod2(uint64_t x) {
  x = (x >> 32) * 22853u + (uint32_t)x;
  x = (x >> 32) * 22853u + (uint32_t)x;
  return (uint32_t)(x >= kMrgM2 ? x - kMrgM2 : x);
}

// One fold of x < 2^64 toward x mod m1 (< 210 2^32) or mod m2 (< 22854
// 2^32): the same residue, small enough that three of them sum without
// overflow before the full reduction.
__device__ inline uint64_t mrg_fold1(uint64_t x) { return (x >> 32) * 209u + (uint32_t)x; }
__device__ inline uint64_t mrg_fold2(uint64_t x) { return (x >> 32) * 22853u + (uint32_t)x; }

// s <- M s for one jump entry M (both components).
template <typename PT>
__device__ inline void mrg_apply(PT M, Mrg& s) {
  uint32_t ra[3], rb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const uint64_t ta = mrg_fold1((uint64_t)M[3 * i] * s.a[0]) +
                        mrg_fold1((uint64_t)M[3 * i + 1] * s.a[1]) +
                        mrg_fold1((uint64_t)M[3 * i + 2] * s.a[2]);
    ra[i] = mrg_mod1(ta);
    const uint64_t tb = mrg_fold2((uint64_t)M[9 + 3 * i] * s.b[0]) +
                        mrg_fold2((uint64_t)M[9 + 3 * i + 1] * s.b[1]) +
                        mrg_fold2((uint64_t)M[9 + 3 * i + 2] * s.b[2]);
    rb[i] = mrg_mod2(tb);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s.a[i] = ra[i];
    s.b[i] = rb[i];
  }
}

// s <- A^(2^shift k) s with the table entries base..base+63 (A^(2^(shift+b))).
template <typename PT>
__device__ inline void mrg_jump(PT tab, int base, uint64_t k, Mrg& s) {
  for (int b = 0; k != 0; ++b, k >>= 1)
    if (k & 1) mrg_apply(tab + (size_t)(base + b) * kMrgEntry, s);
}

// One step; returns the 32-bit word of the new output.
__device__ inline uint32_t mrg_word(Mrg& s) {
  // (a12 x_{n-1} - a13 x_{n-2}) mod m1 as a12 x_{n-1} + a13 (m1 - x_{n-2})
  const uint32_t p1 = mrg_mod1((uint64_t)1403580u * s.a[1] + (uint64_t)810728u * (kMrgM1 - s.a[0]));
  s.a[0] = s.a[1];
  s.a[1] = s.a[2];
  s.a[2] = p1;
  const uint32_t p2 = mrg_mod2((uint64_t)527612u * s.b[2] + (uint64_t)1370589u * (kMrgM2 - s.b[0]));
  s.b[0] = s.b[1];
  s.b[1] = s.b[2];
  s.b[2] = p2;
  const uint32_t z = p1 > p2 ? p1 - p2 : p1 + (kMrgM1 - p2);
  // floor(z 2^32 / (m1 + 1)) with m1 + 1 = 2^32 - 208: z 2^32 / (2^32 - 208)
  // = z + 208 z / (2^32 - 208), and with 208 z = h 2^32 + l the last term's
  // floor is h + [l >= 2^32 - 208 - 208 h] (h < 208).  Exact for every z <
  // m1 (checked exhaustively against the division).
  const uint64_t t = (uint64_t)z * 208u;
  const uint32_t h = (uint32_t)(t >> 32), l = (uint32_t)t;
  return z + h + (l >= (kMrgM1 + 1u) - h * 208u ? 1u : 0u);
}

// ---------------------------------------------------------------------------
// Uniform word u -> bin j = floor(u n / 2^32) and fraction of the remainder.
// FP64: (lo + 1/2) 2^-32; FP32: (lo/2^9 + 1/2) 2^-23.  Both exact, in (0,1);
// the bin is the same integer in both precisions.
// ---------------------------------------------------------------------------
template <typename T>
struct Frac;
template <>
struct Frac<double> {
  __device__ static inline double get(uint32_t lo) { return ((double)lo + 0.5) * 0x1p-32; }
};
template <>
struct Frac<float> {
  __device__ static inline float get(uint32_t lo) {
    return ((float)(lo >> 9) + 0.5f) * 0x1p-23f;
  }
};

// ---------------------------------------------------------------------------
// Per (channel, dim) map constants, per channel density normalisation, and
// per (peak, dim) integrand constants.  Filled on the device by the set-up
// kernel in FP64 and rounded to FP32 for the mixed-precision mode.
// ---------------------------------------------------------------------------
template <typename T>
struct DimMap {
  int32_t kind;
  int32_t pad_;
  T loc;     // mu (Gauss), m (BW)
  T width;   // sigma (Gauss), Gamma (BW)
  T inv_w;   // 1/sigma (Gauss)
  T pa, qb, z;       // Gauss: Phi(a), 1 - Phi(b), Z = Phi(b) - Phi(a)
  T h, h2, ta, th;   // BW: Gamma/2, h^2, atan(-m/h), Theta = atan((1-m)/h) - ta
  T fa, fb;          // BW: atan2(h, m), atan2(h, 1-m) (distances of the ends to the poles)
  T ga, gb;          // Gauss exponent: z' = ga p + gb with z'^2 = log2(e) z^2 / 2
  float hb, hs;      // linear hint map of FP64 jobs (channels Gaussian on every axis)
  float lb, ls;      // log hint map (other channels): z = ls p + lb
};

// One table entry of an axis: a bin edge and the density of the bin that
// starts there.
template <typename T>
struct __align__(2 * sizeof(T)) Pair {
  T e, dens;
};

// Axis kinds of one channel: lin = Gaussian on every axis (its lookups use
// the linear hint map); iso = Gaussian on every axis with one width (its
// density constants take the isotropic form); bit k of gmask (bmask) marks a
// Gaussian (Breit-Wigner) axis k; the other axes are flat.
struct ChanType {
  int32_t iso;
  uint32_t gmask, bmask;
  int32_t lin;
};

// One cell of an axis' hint map, precomputed from its p-space edges:
// J = interior edges whose cell is lower (all of them lie below any x of the
// cell); with at most one edge inside the cell, e is that edge (+inf if
// none) and the bin of x is J (density dlo) below e, J + 1 (density dhi)
// from e on.  dlo < 0 marks a cell holding two or more edges.
template <typename T>
struct __align__(4 * sizeof(T)) Cell {
  T e, dlo, dhi;
  T J;  // the start bin, stored as a value of T (exact for J < 2^24)
};

template <typename T>
struct PeakDim {
  int32_t kind;
  int32_t pad_;
  T loc, h2, ga, gb;  // BW: centre, h^2; Gauss: exponent z' = ga p + gb as in DimMap
};

// Math wrappers resolving to the device math library for each precision.
__device__ inline double m_exp(double x) { return exp(x); }
__device__ inline float m_exp(float x) { return expf(x); }
__device__ inline double m_exp2(double x) { return exp2(x); }
// FP32: the hardware exp2 (one instruction, about 1 ulp; a result below
// 2^-126 may come back as 0).  Every use is a density kernel
// 2^(-sum z'^2) <= 1, so such a result is a term at least 2^-126 below the
// peak it belongs to, which the sums of f and g cannot notice at FP32
// precision; the library exp2f spends more instructions per call only to
// return those denormals.
__device__ inline float m_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
// 1/x: exact in FP64; the hardware reciprocal (1 ulp) in FP32.
__device__ inline double m_rcp(double x) { return 1.0 / x; }
__device__ inline float m_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double m_tan(double x) { return tan(x); }
__device__ inline float m_tan(float x) { return tanf(x); }
// FP32 erfcinv(y), 0 < y < 2, in the structure of M. Giles' erfinv
// approximation ("Approximating the erfinv function", GPU Computing Gems,
// Jade Edition, 2011): with w = -log2(y (2 - y)), erfcinv(y) = erfinv(1 - y)
// = (1 - y) P(w), P a polynomial in (w - 5) / 5 for w <= 10 (y >= 4.9e-4:
// all but a few lanes in a thousand) and in a normalised sqrt(w) for
// 10 < w <= 26; beyond (y < 7.5e-9) the library's erfcinvf.  Coefficients
// fitted by erfcinv_fit.py (largest relative error of the fits 2.9e-08 and
// 1.7e-08; in FP32 with the hardware log2 about 2.5e-7, median 4e-8).  The
// library function spends about 110 instructions over its three branches.
// The library erfcinvf for the far tail, kept out of line (rare; inlined
// into the branchy fast path it broke this compiler's instruction selection).
__device__ __noinline__ float erfcinv_far(float y) { return erfcinvf(y); }

__device__ inline float fast_erfcinv(float y) {
  const float L = __builtin_amdgcn_logf(y * (2.0f - y));  // log2, -w
  const float x = 1.0f - y;
  if (L >= -10.0f) {
    const float t = fmaf(L, -0.2f, -1.0f);
    float P = -1.689334030e-05f;
    P = fmaf(P, t, 1.472581541e-04f);
    P = fmaf(P, t, -1.411730478e-04f);
    P = fmaf(P, t, -7.059459609e-04f);
    P = fmaf(P, t, 2.037662157e-03f);
    P = fmaf(P, t, -8.269816707e-04f);
    P = fmaf(P, t, -7.870274752e-03f);
    P = fmaf(P, t, 2.327191661e-02f);
    P = fmaf(P, t, -2.094532432e-02f);
    P = fmaf(P, t, -8.007366265e-02f);
    P = fmaf(P, t, 8.172793550e-01f);
    P = fmaf(P, t, 1.734757719e+00f);
    return x * P;
  }
  if (L >= -26.0f) {
    const float t = (sqrtf(-L) - 4.130648587e+00f) * 1.032662147e+00f;
    float P = 7.523363763e-06f;
    P = fmaf(P, t, -5.389624879e-05f);
    P = fmaf(P, t, 1.529154143e-04f);
    P = fmaf(P, t, -2.954300123e-04f);
    P = fmaf(P, t, 5.583441763e-04f);
    P = fmaf(P, t, -1.234308599e-03f);
    P = fmaf(P, t, 2.392615197e-03f);
    P = fmaf(P, t, 8.118207278e-01f);
    P = fmaf(P, t, 3.274039353e+00f);
    return x * P;
  }
  return erfcinv_far(y);
}
// FP64 erfcinv: the FP32 value as the start of one Halley step on
// erfc(x) = y (erfc' = -2/sqrt(pi) e^{-x^2}, erfc'' = -2 x erfc', so the step
// is x - u / (1 + x u) with u = (erfc(x) - y) / erfc'(x)); from the FP32
// value's relative error of about 2.5e-7 the step's cubic convergence leaves
// the rounding of erfc and exp.  Outside the FP32 value's range (y below
// 1e-37, where FP32 has no normal number near y) the library function.
// Used by the single-job FP64 pass; the batched pass keeps the library
// function (with this one inlined it took 155 -> 161 ms on the 256-job
// batch).
__device__ inline double m_erfcinv_refined(double y) {
  if (!(y >= 1e-37 && y <= 1.0)) return erfcinv(y);
  const double x = (double)fast_erfcinv((float)y);
  const double u = (erfc(x) - y) / (-1.1283791670955125739 * exp(-x * x));
  return x - u / (1.0 + x * u);
}
__device__ inline double m_erfcinv(double x) { return erfcinv(x); }
__device__ inline float m_erfcinv(float x) { return fast_erfcinv(x); }

constexpr double kSqrt2 = 1.41421356237309504880;

// Forward map p = phi(x) for one dim.  x and xc = 1 - x are both supplied so
// the upper tail keeps its relative precision.  Gauss: truncated-normal
// inverse CDF, evaluated on the tail side of the median.  BW: arctan map; in
// FP32 near either pole it is written with the distance to the pole so that
// p - m keeps its precision.  In FP32 each case picks its argument first and
// then makes a single call of the special function (lanes of a wave that take
// different cases share that call).  PM: pointer to the axis' DimMap<T>
// (generic or constant address space).
// REFINED: in FP64, m_erfcinv_refined in place of the library function.
template <typename T, typename PM, bool REFINED = false>
__device__ inline T map_forward(PM m, T x, T xc) {
  const int kind = m->kind;
  if (kind == GAUSS) {
    const T t = m->pa + x * m->z;
    T zz;
    if constexpr (sizeof(T) == 4) {
      const bool lower = t <= T(0.5);
      const T arg = lower ? T(2) * t : T(2) * (m->qb + xc * m->z);
      zz = (lower ? -T(kSqrt2) : T(kSqrt2)) * m_erfcinv(arg);
    } else {  // FP64: two call sites keep the register use of the inlined calls down
      // (one call site with the argument selected first: 21.7 -> 40.2 ms at
      // d = 10, 32 channels)
      if (t <= T(0.5)) {
        const T y = T(2) * t;
        zz = -T(kSqrt2) * (REFINED ? m_erfcinv_refined(y) : m_erfcinv(y));
      } else {
        const T y = T(2) * (m->qb + xc * m->z);
        zz = T(kSqrt2) * (REFINED ? m_erfcinv_refined(y) : m_erfcinv(y));
      }
    }
    return m->loc + m->width * zz;
  }
  if (kind == BW) {
    if (sizeof(T) == 8) return m->loc + m->h * m_tan(m->ta + x * m->th);
    const T da = m->fa + x * m->th;   // theta + pi/2
    const T db = m->fb + xc * m->th;  // pi/2 - theta
    const T quarter = T(0.78539816339744830962);
    const bool near_a = da < quarter, near_b = !near_a && db < quarter;
    const T t = m_tan(near_a ? da : near_b ? db : m->ta + x * m->th);
    if (near_a) return m->loc - m->h / t;
    if (near_b) return m->loc + m->h / t;
    return m->loc + m->h * t;
  }
  return x;
}

// Neumaier compensated accumulator in FP64.
struct Neu {
  double s, c;
  __device__ inline void add(double v) {
    const double t = s + v;
    if (fabs(s) >= fabs(v)) c += (s - t) + v;
    else c += (v - t) + s;
    s = t;
  }
};

// Sum of two compensated pairs (a.s + a.c) + (b.s + b.c) by an error-free
// TwoSum of the leading parts.
__device__ inline Neu neu_merge(Neu a, Neu b) {
  const double s = a.s + b.s;
  const double bb = s - a.s;
  const double err = (a.s - (s - bb)) + (b.s - bb);
  return Neu{s, a.c + b.c + err};
}

}  // namespace mcv
