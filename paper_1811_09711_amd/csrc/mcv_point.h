// Per-point pieces of the sample pass shared by the sample, trace and
// unweighting kernels: integrand, channel densities and the bin search.
//
// Brass, Kilian, Reuter, arXiv:1811.09711: the integrand and channel
// densities enter eq. g(p) (Sec. 3.5) as f and 1/phi_c'; the bin search finds
// the VEGAS bin B_j (Sec. 3.2) that holds a point's inverse map in an other
// channel's grid.
#pragma once

#include "mcv_device.h"

namespace mcv {

// Channel density q_c(p) = prod_k q_{c,k}(p_k) in one exponential:
// norm * exp(-sum_gauss z_k^2 / 2) / prod_bw ((p_k - m_k)^2 + h_k^2), where
// norm = prod_gauss 1/(sqrt(2 pi) sigma Z) * prod_bw h/Theta.  Returns exactly
// 0 when the Gaussian factor underflows, which lets callers skip the grid
// lookups of a channel whose term is exactly zero.
template <typename T, int MAXD>
__device__ inline T chan_density(const DimMap<T>* __restrict__ cm, T norm, int d, const T* p) {
  T gs = T(0), den = T(1);
#pragma unroll
  for (int k = 0; k < MAXD; ++k) {
    if (k < d) {
      const int kind = cm[k].kind;
      if (kind == GAUSS) {
        const T z = (p[k] - cm[k].loc) * cm[k].inv_w;
        gs += z * z;
      } else if (kind == BW) {
        const T u = p[k] - cm[k].loc;
        den *= u * u + cm[k].h2;
      }
    }
  }
  return norm * m_exp(T(-0.5) * gs) / den;
}

// Integrand f(p) = sum_i w_i prod_k pdf_ik(p_k) with untruncated normalised
// 1-d pdfs; pn[i] folds w_i and the normalisations.
template <typename T, int MAXD>
__device__ inline T integrand(const PeakDim<T>* __restrict__ pm, const T* __restrict__ pn, int P,
                              int d, const T* p) {
  T f = T(0);
  for (int i = 0; i < P; ++i) {
    const PeakDim<T>* m = pm + i * d;
    T gs = T(0), den = T(1);
#pragma unroll
    for (int k = 0; k < MAXD; ++k) {
      if (k < d) {
        const int kind = m[k].kind;
        if (kind == GAUSS) {
          const T z = (p[k] - m[k].loc) * m[k].inv_w;
          gs += z * z;
        } else if (kind == BW) {
          const T u = p[k] - m[k].loc;
          den *= u * u + m[k].h2;
        }
      }
    }
    f += pn[i] * m_exp(T(-0.5) * gs) / den;
  }
  return f;
}

// Largest j in [0, n-1] with P[j] <= x, for an increasing table P[0..n] whose
// P[n] is +inf and whose P[0] is never read.  Branch-free binary search over
// the next power of two npow2 >= n; indices beyond n read the +inf sentinel.
template <typename T>
__device__ inline int find_bin(const T* P, int n, int npow2, T x) {
  int j = 0;
  for (int s = npow2 >> 1; s > 0; s >>= 1) {
    const int t = min(j + s, n);
    j = (P[t] <= x) ? t : j;
  }
  return j;
}

}  // namespace mcv
