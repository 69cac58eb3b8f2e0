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

// Unnormalised density kernel of a channel:
//   r_c(p) = exp(-sum_gauss z_k^2 / 2) / prod_bw ((p_k - m_k)^2 + h_k^2),
// so q_c(p) = cnorm_c * r_c(p) with cnorm_c = prod_gauss 1/(sqrt(2 pi) sigma Z)
// * prod_bw h/Theta.  iso: every axis Gaussian (no per-axis branches).
// Returns exactly 0 when the Gaussian factor underflows.
template <typename T, int MAXD>
__device__ __forceinline__ T chan_r(CP<DimMap<T>> cm, int iso, int d, const T (&p)[MAXD]) {
  T gs = T(0);
  if (iso) {
#pragma unroll
    for (int k = 0; k < MAXD; ++k) {
      if (k < d) {
        const T z = (p[k] - cm[k].loc) * cm[k].inv_w;
        gs += z * z;
      }
    }
    return m_exp(T(-0.5) * gs);
  }
  T den = T(1);
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
  return m_exp(T(-0.5) * gs) / den;
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
        const T z = (p[k] - pm[k].loc) * pm[k].inv_w;
        gs += z * z;
      } else if (kind == BW) {
        const T u = p[k] - pm[k].loc;
        den *= u * u + pm[k].h2;
      }
    }
  }
  return m_exp(T(-0.5) * gs) / den;
}

// Largest j in [0, n-1] with P[j] <= x, for an increasing table P[0..n] whose
// P[n] is +inf and whose P[0] is never read.  Branch-free binary search over
// the next power of two npow2 >= n; indices beyond n read the +inf sentinel.
template <typename T>
__device__ __forceinline__ int find_bin(const T* P, int n, int npow2, T x) {
  int j = 0;
  for (int s = npow2 >> 1; s > 0; s >>= 1) {
    const int t = min(j + s, n);
    j = (P[t] <= x) ? t : j;
  }
  return j;
}

}  // namespace mcv
