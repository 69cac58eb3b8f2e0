// Per-point pieces of the sample pass shared by the sample, trace and
// unweighting kernels: channel and peak density kernels and the bin search.
//
// Brass, Kilian, Reuter, arXiv:1811.09711: the integrand and the channel
// densities 1/phi_c' enter eq. g(p) (Sec. 3.5); the bin search finds the VEGAS
// bin B_j (Sec. 3.2) that holds a point's inverse map in another channel's
// grid.
#pragma once

#include "mcv_device.h"

namespace mcv {

// Read-only kernel inputs are read through the constant address space, so
// that wave-uniform reads become scalar loads.
template <typename T>
using CP = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ CP<T> cp(const T* p) {
  return (CP<T>)(p);
}

// Read-only device tables read with global-memory instructions.
template <typename T>
using GP = const __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ GP<T> gptr(const T* p) {
  return (GP<T>)(p);
}

// Unnormalised density kernel of a channel:
//   r_c(p) = exp(-sum_gauss z_k^2 / 2) / prod_bw ((p_k - m_k)^2 + h_k^2),
// so q_c(p) = cnorm_c * r_c(p) with cnorm_c = prod_gauss 1/(sqrt(2 pi) sigma Z)
// * prod_bw h/Theta.  The Gaussian exponent is evaluated as 2^(-sum z'^2) with
// z' = ga p + gb (ga, gb fold 1/sigma, the centre and log2(e)/2).  The
// per-axis constants come from the channel's contiguous pairs gab, (ga, gb)
// on a Gaussian axis and (m, h^2) on a Breit-Wigner one, so that they arrive
// in a few wide scalar loads.  The axis kinds come from the channel's masks
// (gm: Gaussian axes, bm: Breit-Wigner axes), one pass over each kind;
// iso: every axis Gaussian with one width.  Such a channel's 2d constants
// are the centres m_0..m_{d-1}, then ga^2, and the exponent is
// ga^2 sum (p_k - m_k)^2: a subtraction and an FMA per axis (the FMA of z'
// takes two scalar constants, and an instruction can read only one, so it
// costs a move besides); the centres are contiguous, so that they still
// arrive in wide scalar loads.
// Returns exactly 0 when the Gaussian factor underflows.
template <typename T, int MAXD>
__device__ __forceinline__ T chan_r(CP<T> gab, int iso, uint32_t gm, uint32_t bm, int d,
                                    const T (&p)[MAXD]) {
  T gs = T(0);
  if (iso) {
#pragma unroll
    for (int k = 0; k < MAXD; ++k) {
      if (k < d) {
        const T u = p[k] - gab[k];
        gs = fma(u, u, gs);
      }
    }
    return m_exp2(-(gs * gab[d]));
  }
  T den = T(1);
  if (gm) {
#pragma unroll
    for (int k = 0; k < MAXD; ++k) {
      if (k < d && ((gm >> k) & 1u)) {
        const T z = fma(p[k], gab[2 * k], gab[2 * k + 1]);
        gs = fma(z, z, gs);
      }
    }
  }
  if (bm) {
#pragma unroll
    for (int k = 0; k < MAXD; ++k) {
      if (k < d && ((bm >> k) & 1u)) {
        const T u = p[k] - gab[2 * k];
        den *= fma(u, u, gab[2 * k + 1]);
      }
    }
  }
  return gm ? m_exp2(-gs) * m_rcp(den) : m_rcp(den);  // no Gaussian axis: 2^-0 = 1
}

// The same kernel for a peak of the integrand: pdf_i(p) = pnorm_i * r_i(p)
// with pnorm_i = w_i prod_gauss 1/(sqrt(2 pi) sigma) * prod_bw h/pi
// (untruncated, normalised 1-d factors).
template <typename T, int MAXD>
__device__ __forceinline__ T peak_r(CP<PeakDim<T>> pm, int d, const T (&p)[MAXD]) {
  T gs = T(0), den = T(1);
#pragma unroll
  for (int k = 0; k < MAXD; ++k) {
    if (k < d) {
      const int kind = pm[k].kind;
      if (kind == GAUSS) {
        const T z = fma(p[k], pm[k].ga, pm[k].gb);
        gs = fma(z, z, gs);
      } else if (kind == BW) {
        const T u = p[k] - pm[k].loc;
        den *= fma(u, u, pm[k].h2);
      }
    }
  }
  return m_exp2(-gs) * m_rcp(den);
}

// Cell of x in the hint map of one axis: a cheap, monotone (non-decreasing)
// map of x onto the job's M cells, so that every edge of a lower (higher)
// cell lies below (above) any x of the cell.  Channels Gaussian on every
// axis: linear, the centre +- 3 sigma onto the M cells, cell = hs x + hb in
// FP32, clamped.  Other channels, on every axis: z = x ls + lb (z = (x - m) /
// h on a Breit-Wigner axis, 16 (x - mu) / sigma on a Gaussian one, 510 (x -
// 1/2) on a flat one), and the bit pattern of |z| + 1 (a monotone, piecewise
// linear log2) gives M/16 cells per doubling of |z| + 1 on either side of
// z = 0 -- fine cells near a peak, coarse ones over heavy tails.  The
// constants (a, b) = (hs, hb) or (ls, lb) come from the channel's contiguous
// hint-constant array.  Only the cost of the lookup depends on the map.
//
// The log map: q = the bits of |z| + 1 above those of 1.0, shifted by
// `shift` = 27 - log2 M (at most M/2 - 1); cell M/2 + q for z with a clear
// sign bit, M/2 - 1 - q = M/2 + ~q for a set one (the sign word s = 0 or ~0
// selects by xor).  Ordered as the sign bit orders floats (-0 below +0), so
// the map stays monotone.
template <typename T>
__device__ __forceinline__ unsigned hint_cell(float a, float b, T x, bool log_map, int M,
                                              int shift) {
  const float z = fmaf((float)x, a, b);
  if (log_map) {
    const uint32_t u = __float_as_uint(fabsf(z) + 1.0f) - 0x3F800000u;
    const uint32_t half = (uint32_t)M >> 1;
    const uint32_t q = min(u >> shift, half - 1u);
    const uint32_t s = (uint32_t)((int32_t)__float_as_uint(z) >> 31);
    return half + (q ^ s);
  }
  return (unsigned)__builtin_amdgcn_fmed3f(z, 0.0f, (float)(M - 1));
}

// Bin of x in one axis: the largest j in [0, n-1] with edge_j <= x, for an
// increasing table tab[off .. off+n] (entry 0 = -inf, entry n = +inf), found
// by walking from the start bin J (clamped to [0, n-1]); exact for any start.
// Returns that bin's density and, optionally, its index.  The axis offset
// is kept as an opaque per-lane value, so that the (rarely taken) walks do
// not make the compiler keep one scalar base address per axis across the
// channel loop.
template <typename T, typename PT>
__device__ __forceinline__ T walk_bin(PT base, int off, int n, int J, T x, int* jout) {
  asm("" : "+v"(off));
  const PT tab = base + off;
  J = J < 0 ? 0 : (J > n - 1 ? n - 1 : J);
  T lo_e = tab[J].e, lo_d = tab[J].dens, hi_e = tab[J + 1].e, hi_d = tab[J + 1].dens;
  while (J > 0 && x < lo_e) {
    --J;
    hi_e = lo_e;
    hi_d = lo_d;
    lo_e = tab[J].e;
    lo_d = tab[J].dens;
  }
  while (J < n - 1 && x >= hi_e) {
    ++J;
    lo_e = hi_e;
    lo_d = hi_d;
    hi_e = tab[J + 1].e;
    hi_d = tab[J + 1].dens;
  }
  if (jout) *jout = J;
  return lo_d;
}

// Grid density G_c(x_c) = prod_k dens of the bin holding p_k in axis k of one
// channel (eq. g(x) for another channel's grid, searched in p-space).  Per
// axis, one read of the point's hint cell gives the bin when the cell holds
// at most one edge (one comparison); otherwise an exact walk from the cell's
// start bin finds it (one branch per group of axes).  The reads of GROUP
// axes are issued together; the product runs in axis order.  ISO: the channel
// is Gaussian on every axis (linear hint map; otherwise the log map).
// LAZY: no walks; a crowded cell gives the largest density of the bins it
// can hold, so the result is an upper bound of G (exact unless *crowded is
// set on return).
template <typename T, int MAXD, int GROUP, bool ISO, bool FULL = false, bool LAZY = false,
          typename PT, typename PC>
__device__ __forceinline__ T grid_density(PT T0, PC C0, int sT, int n, int d, int M, int shift,
                                          CP<float> hab, const T (&p)[MAXD], int* bins,
                                          bool* crowded = nullptr) {
  T G = T(1);
  bool any_slow = false;
#pragma unroll
  for (int k0 = 0; k0 < MAXD; k0 += GROUP) {
    if (k0 >= d) break;  // uniform
    unsigned J[GROUP];
    T e[GROUP], dlo[GROUP], dhi[GROUP], dens[GROUP];
    int jj[GROUP];
    // Every axis of the group reads a record, so that the reads are issued
    // together without per-axis branches; an axis beyond d (p = 0 there)
    // reads a cell of axis d-1 and is ignored.  FULL: d == MAXD.
#pragma unroll
    for (int g = 0; g < GROUP; ++g) {
      const int k = k0 + g;
      if (k < MAXD && (!FULL || k < d)) {
        const int kk = FULL ? k : (k < d ? k : d - 1);
        const unsigned cell = hint_cell<T>(hab[2 * kk], hab[2 * kk + 1], p[k], !ISO, M, shift);
        // a 32-bit byte offset from the channel's cells (a scalar base), so
        // that the read takes the scalar-base form with no 64-bit address
        const uint32_t off = ((uint32_t)(kk * M) + cell) * (uint32_t)sizeof(Cell<T>);
        const PC rec = (PC)((GP<char>)C0 + off);
        e[g] = rec->e;
        dlo[g] = rec->dlo;
        dhi[g] = rec->dhi;
        J[g] = (unsigned)rec->J;
      }
    }
    bool slow = false;
#pragma unroll
    for (int g = 0; g < GROUP; ++g) {
      const int k = k0 + g;
      if (k < MAXD && (!FULL || k < d)) {
        const bool live = FULL || k < d;
        const bool up = p[k] >= e[g];
        jj[g] = (int)J[g] + (up ? 1 : 0);
        dens[g] = up ? dhi[g] : dlo[g];
        slow |= live && dlo[g] < T(0);
      }
    }
    any_slow |= slow;
    if (!LAZY && slow) {  // a cell holding several edges: exact walks
#pragma unroll
      for (int g = 0; g < GROUP; ++g) {
        const int k = k0 + g;
        if (k < MAXD && k < d && dlo[g] < T(0))
          dens[g] = walk_bin<T>(T0, k * sT, n, (int)J[g], p[k], &jj[g]);
      }
    }
#pragma unroll
    for (int g = 0; g < GROUP; ++g) {
      const int k = k0 + g;
      if (k < MAXD && k < d) {
        if (bins) bins[k] = jj[g];
        G *= dens[g];
      }
    }
  }
  if (LAZY) *crowded = any_slow;
  return G;
}

}  // namespace mcv
