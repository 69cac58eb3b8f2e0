// Small device kernels around the sample pass: set-up of the map constants
// and grids, p-space edge tables, the integer channel allocation, the
// reduction of a pass, VEGAS rebinning and the channel-weight update.
//
// Brass, Kilian, Reuter, arXiv:1811.09711: Sec. 3.1 (E_N, V_N), Sec. 3.2
// (eq. g(x), eq. 30, eq. 31), Sec. 3.4 (multi-channel estimator, eq. 15 and
// the integer N_c), Sec. 3.5 (eq. g(p); the organisation of an iteration).
#include <hip/hip_runtime.h>
#include <math.h>

#include "mcv_internal.h"
#include "mcv_point.h"

namespace mcv {

namespace {

constexpr double kInvSqrt2Pi = 0.39894228040143267794;
// sqrt(log2(e) / 2): exp(-z^2/2) = 2^(-(kExpScale z)^2)
constexpr double kExpScale = 0.84932180028801904272;
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Set-up
// ---------------------------------------------------------------------------
__global__ void k_setup_maps(JobDev j) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nc = j.K * j.d, np = j.P * j.d;
  if (t < nc) {
    DimMap<double> m{};
    m.kind = j.ckind[t];
    m.loc = j.cloc[t];
    m.width = j.cwidth[t];
    m.hs = (float)j.M;  // flat: the identity onto the cells
    m.hb = 0.0f;
    m.ls = 510.0f;      // flat, log map: z = 510 (x - 1/2)
    m.lb = -255.0f;
    if (m.kind == GAUSS) {
      const double a = (0.0 - m.loc) / m.width, b = (1.0 - m.loc) / m.width;
      m.inv_w = 1.0 / m.width;
      m.ga = kExpScale / m.width;
      m.gb = -m.loc * m.ga;
      // linear hint map: centre +- 3 sigma onto the M cells
      m.hs = (float)((double)j.M / (6.0 * m.width));
      m.hb = (float)((double)j.M * (0.5 - m.loc / (6.0 * m.width)));
      m.ls = (float)(16.0 / m.width);
      m.lb = (float)(-16.0 * m.loc / m.width);
      m.pa = 0.5 * erfc(-a / kSqrt2);
      m.qb = 0.5 * erfc(b / kSqrt2);
      m.z = (1.0 - m.qb) - m.pa;
    } else if (m.kind == BW) {
      m.h = 0.5 * m.width;
      m.h2 = m.h * m.h;
      m.ta = atan((0.0 - m.loc) / m.h);
      const double tb = atan((1.0 - m.loc) / m.h);
      m.th = tb - m.ta;
      m.fa = atan2(m.h, m.loc);
      m.fb = atan2(m.h, 1.0 - m.loc);
      m.ls = (float)(1.0 / m.h);
      m.lb = (float)(-m.loc / m.h);
    }
    j.cmap64[t] = m;
    DimMap<float> f{};
    f.kind = m.kind;
    f.loc = (float)m.loc;
    f.width = (float)m.width;
    f.inv_w = (float)m.inv_w;
    f.pa = (float)m.pa;
    f.qb = (float)m.qb;
    f.z = (float)m.z;
    f.h = (float)m.h;
    f.h2 = (float)m.h2;
    f.ta = (float)m.ta;
    f.th = (float)m.th;
    f.fa = (float)m.fa;
    f.fb = (float)m.fb;
    f.ga = (float)m.ga;
    f.gb = (float)m.gb;
    f.hb = m.hb;
    f.hs = m.hs;
    f.lb = m.lb;
    f.ls = m.ls;
    j.cmap32[t] = f;
    // density-kernel constants: (ga, gb) on a Gaussian axis, (m, h^2) on a
    // Breit-Wigner one, 0 on a flat one
    const bool bw = m.kind == BW;
    if (j.prec == 1) {
      ((float*)j.gab)[2 * t] = bw ? f.loc : f.ga;
      ((float*)j.gab)[2 * t + 1] = bw ? f.h2 : f.gb;
    } else {
      ((double*)j.gab)[2 * t] = bw ? m.loc : m.ga;
      ((double*)j.gab)[2 * t + 1] = bw ? m.h2 : m.gb;
    }
  }
  if (t < np) {
    PeakDim<double> m{};
    m.kind = j.pkind[t];
    m.loc = j.ploc[t];
    if (m.kind == GAUSS) {
      m.ga = kExpScale / j.pwidth[t];
      m.gb = -m.loc * m.ga;
    }
    if (m.kind == BW) m.h2 = 0.25 * j.pwidth[t] * j.pwidth[t];
    j.pmap64[t] = m;
    PeakDim<float> f{};
    f.kind = m.kind;
    f.loc = (float)m.loc;
    f.h2 = (float)m.h2;
    f.ga = (float)m.ga;
    f.gb = (float)m.gb;
    j.pmap32[t] = f;
  }
}

// Per-channel and per-peak normalisations (after the map constants).
__global__ void k_setup_twins(JobDev j) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < j.K) {
    const int i = j.twin_peak[t];
    j.twin_pn64[t] = i >= 0 ? j.pnorm64[i] : 0.0;
    j.twin_pn32[t] = i >= 0 ? j.pnorm32[i] : 0.0f;
  }
}

__global__ void k_setup_norms(JobDev j) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < j.K) {
    double norm = 1.0;
    for (int k = 0; k < j.d; ++k) {
      const DimMap<double>& m = j.cmap64[t * j.d + k];
      if (m.kind == GAUSS) norm *= kInvSqrt2Pi / (m.width * m.z);
      else if (m.kind == BW) norm *= m.h / m.th;
    }
    j.cnorm64[t] = norm;
    j.cnorm32[t] = (float)norm;
    j.alpha[t] = 1.0 / (double)j.K;
    ChanType ct{0, 0u, 0u, 1};
    for (int k = 0; k < j.d; ++k) {
      const int kind = j.cmap64[t * j.d + k].kind;
      ct.lin &= (kind == GAUSS) ? 1 : 0;
      if (kind == GAUSS) ct.gmask |= 1u << k;
      if (kind == BW) ct.bmask |= 1u << k;
    }
    if (ct.lin) {
      // one width on every axis: the centres m_0..m_{d-1}, then ga^2, in
      // place of the (ga, gb) pairs that the map set-up wrote
      bool eq = true;
      for (int k = 1; k < j.d; ++k) eq &= j.cmap64[t * j.d + k].ga == j.cmap64[t * j.d].ga;
      if (eq) {
        ct.iso = 1;
        const double s2 = j.cmap64[t * j.d].ga * j.cmap64[t * j.d].ga;
        for (int k = 0; k < 2 * j.d; ++k) {
          const double v = k < j.d ? j.cmap64[t * j.d + k].loc : k == j.d ? s2 : 0.0;
          if (j.prec == 1) ((float*)j.gab)[2 * t * j.d + k] = (float)v;
          else ((double*)j.gab)[2 * t * j.d + k] = v;
        }
      }
    }
    j.ctype[t] = ct;
    for (int k = 0; k < j.d; ++k) {
      const DimMap<double>& m = j.cmap64[t * j.d + k];
      j.hab[2 * (t * j.d + k)] = ct.lin ? m.hs : m.ls;
      j.hab[2 * (t * j.d + k) + 1] = ct.lin ? m.hb : m.lb;
    }
  }
  if (t < j.P) {
    double norm = j.pweight[t];
    for (int k = 0; k < j.d; ++k) {
      const int kind = j.pkind[t * j.d + k];
      const double w = j.pwidth[t * j.d + k];
      if (kind == GAUSS) norm *= kInvSqrt2Pi / w;
      else if (kind == BW) norm *= (0.5 * w) / kPi;
    }
    j.pnorm64[t] = norm;
    j.pnorm32[t] = (float)norm;
  }
}

// Rounds one axis to FP32 and keeps it strictly increasing (forward, then
// backward) -- the mixed-precision grid.
__device__ void snap_axis32(int n, double* e) {
  e[0] = 0.0;
  e[n] = 1.0;
  for (int i = 1; i < n; ++i) {
    float f = (float)e[i];
    const float prev = (float)e[i - 1];
    if (!(f > prev)) f = nextafterf(prev, 2.0f);
    e[i] = (double)f;
  }
  for (int i = n - 1; i >= 1; --i) {
    float f = (float)e[i];
    const float next = (float)e[i + 1];
    if (!(f < next)) f = nextafterf(next, -1.0f);
    e[i] = (double)f;
  }
}

// Equidistant bins (Sec. 3.2: adaptation starts from equidistant bins).
__global__ void k_init_grid(JobDev j) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= j.K * j.d) return;
  double* e = j.edges + (size_t)t * (j.n + 1);
  for (int i = 0; i <= j.n; ++i) e[i] = (double)i / (double)j.n;
  if (j.prec == 1) snap_axis32(j.n, e);
}

// Edge/density tables of every axis from the master edges (eq. g(x): the
// density of bin j is 1/(n Delta_j)); x-space edges for the forward map and
// p-space edges P_j = phi(X_j) for the other channels' bin search.  One thread
// per (axis, entry), entry < sT; grid row y = job.
template <typename T>
__global__ void k_tables(const JobDev* jobs) {
  const JobDev& j = jobs[blockIdx.y];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n = j.n, sT = j.sT;
  const int64_t tot = (int64_t)j.K * j.d * sT;
  if (t >= tot) return;
  const int64_t ax = t / sT;
  const int i = (int)(t - ax * sT);
  const double* e = j.edges + ax * (n + 1);
  Pair<T>* X = (Pair<T>*)j.xtab + ax * sT;
  Pair<T>* P = (Pair<T>*)j.ptab + ax * sT;
  const DimMap<double>* m = j.cmap64 + ax;
  const T dens = (i < n) ? (T)(1.0 / ((double)n * (e[i + 1] - e[i]))) : T(0);
  X[i] = Pair<T>{i <= n ? (T)e[i] : T(1), dens};
  T pe;
  if (i == 0) pe = (T)-INFINITY;
  else if (i >= n) pe = (T)INFINITY;
  else pe = (T)map_forward<double>(m, e[i], 1.0 - e[i]);
  P[i] = Pair<T>{pe, dens};
}

// Hint cells: for cell c of an axis, the start bin J (interior edges with a
// lower cell) and, when at most one interior edge falls into the cell, that
// edge and the densities of the bins on either side.  The cell map is
// monotone, so every edge of a lower (higher) cell lies below (above) any x
// of the cell.  One thread per (axis, cell); grid row y = job.
template <typename T>
__global__ void k_cells(const JobDev* jobs) {
  const JobDev& j = jobs[blockIdx.y];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int M = j.M, n = j.n;
  const int64_t tot = (int64_t)j.K * j.d * M;
  if (t >= tot) return;
  const int64_t ax = t / M;
  const unsigned c = (unsigned)(t - ax * M);
  const Pair<T>* P = (const Pair<T>*)j.ptab + ax * j.sT;
  const bool log_map = !j.ctype[ax / j.d].lin;  // the map the lookups of this channel use
  const float ha = j.hab[2 * ax], hb = j.hab[2 * ax + 1];
  // The cells of the interior edges 1..n-1 do not decrease (increasing
  // edges, monotone map): the edges below the cell and in it are two
  // binary searches.
  auto cell_of = [&](int i) { return hint_cell<T>(ha, hb, P[i].e, log_map, M, j.mshift); };
  int lo = 1, hi = n;
  while (lo < hi) {  // first edge whose cell is >= c (n if none)
    const int mid = (lo + hi) >> 1;
    if (cell_of(mid) < c) lo = mid + 1;
    else hi = mid;
  }
  const int lb = lo;
  hi = n;
  while (lo < hi) {  // first edge whose cell is > c
    const int mid = (lo + hi) >> 1;
    if (cell_of(mid) <= c) lo = mid + 1;
    else hi = mid;
  }
  const int below = lb - 1, inside = lo - lb, first = lb;
  Cell<T> r;
  r.J = (T)below;
  if (inside > 1) {
    // a crowded cell: the exact lookup walks from J over the bins J ..
    // J + inside; without the walk it reads dhi, the largest of their
    // densities (an upper bound), and the sign of dlo marks the cell
    T mx = P[below].dens;
    for (int b = below + 1; b <= below + inside; ++b) mx = mx > P[b].dens ? mx : P[b].dens;
    r.e = T(0);
    r.dlo = -mx;
    r.dhi = mx;
  } else if (inside == 0) {
    r.e = (T)INFINITY;
    r.dlo = P[below].dens;
    r.dhi = r.dlo;
  } else {
    r.e = P[first].e;
    r.dlo = P[first - 1].dens;
    r.dhi = P[first].dens;
  }
  ((Cell<T>*)j.ctab)[t] = r;
}

// Per-channel bound of the channel terms of g(p) (eq. g(p)) for the sample
// pass: gbound_c = 2^s (1 + m) cnorm_c prod_k max_j dens_kj, rounded up to
// the pass precision, with s = 25, m = 2^-16 in FP32 and s = 54, m = 2^-40 in
// FP64.  m covers the roundings of the term (at most d + 4 of the pass
// precision) and of this product, so (alpha_c gbound_c) r_c evaluated in the
// pass precision is at least 2^s times the term alpha_c cnorm_c G_c r_c as the
// pass evaluates it.  The same holds with any upper bounds of the looked-up
// densities in place of the maxima (the factor bound_factor(alpha_c cnorm_c)
// written with the allocation).  One wavefront per (channel, job).
template <typename T>
__device__ T bound_factor(double g) {
  if constexpr (sizeof(T) == 4) {
    g *= 0x1p25 * (1.0 + 0x1p-16);
    float f = (float)g;
    if ((double)f < g) f = nextafterf(f, INFINITY);
    return f;
  } else {
    return g * (0x1p54 * (1.0 + 0x1p-40));
  }
}

template <typename T>
__global__ void k_gbound(const JobDev* jobs) {
  const JobDev& j = jobs[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= j.K) return;  // uniform over the workgroup
  __shared__ double mx[64];
  const int lane = threadIdx.x, n = j.n;
  // per axis, the lanes take the bins in turn and a butterfly takes the
  // largest (a maximum, exact in any order)
  for (int k = 0; k < j.d; ++k) {
    const Pair<T>* P = (const Pair<T>*)j.ptab + ((size_t)c * j.d + k) * j.sT;
    double m = 0.0;
    for (int i = lane; i < n; i += 64) m = fmax(m, (double)P[i].dens);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if (lane == 0) mx[k] = m;
  }
  __syncthreads();
  if (lane != 0) return;
  constexpr bool f32 = sizeof(T) == 4;
  double g = f32 ? (double)j.cnorm32[c] : j.cnorm64[c];
  for (int a = 0; a < j.d; ++a) g *= mx[a];
  ((T*)j.gbound)[c] = bound_factor<T>(g);
}

// ---------------------------------------------------------------------------
// Allocation (Sec. 3.4): N_c = floor(alpha_c N), floor min_calls, the
// remainder to the largest fractional parts (ties to the lower channel);
// N_tot = sum N_c; alpha_c = N_c / N_tot.  One wavefront per job (workgroup
// x = job), the same IEEE operations per channel as a serial host
// implementation.  Handing the remainder out one call at a time to the
// largest fraction not yet served (all served: a new round) gives channel c
// floor(rem / K) calls plus one if its rank -- the channels with a larger
// fraction, or an equal one and a lower index -- is below rem mod K; the
// kernel computes that rank per channel.  N is n_override if positive, else
// the job's own calls per pass.  to_trace:
// the result goes to the trace allocation and alpha is left alone.  Also
// writes the partial-exponent skip offsets for the resulting weights and
// resets the 8 work-queue counters of the following sample pass.
// ---------------------------------------------------------------------------
// floor(log2 x) of a positive finite x; -100000 for 0, +100000 otherwise.
__device__ inline int floor_log2(double x) {
  if (x == 0.0) return -100000;
  if (!(x > 0.0) || !isfinite(x)) return 100000;
  int e = 0;
  (void)frexp(x, &e);
  return e - 1;
}

// Exponent offsets of the partial-exponent skip (all-Gaussian channels of
// the sample pass), from the pass-precision values the pass multiplies: the
// twin factor tw (the channel's term of f is tw r) and alpha gbound (the
// term of g is at most alpha gbound r 2^-s).  With r <= 2^(1 - floor(S)) for
// a partial exponent sum S, the term of f is below 2^(ex(tw) + 3 - floor(S))
// and must be at most 2^(ex(f) - P - 1) (half an ulp, P = 24 or 53, with a
// margin of 2), so EA = ex(tw) + P + 4; likewise EB = ex(alpha) + ex(gbound)
// + 4 - s + P.  A zero twin factor never blocks the skip.  alpha: the
// allocation's channel weights the pass will use.
__device__ inline void set_skip_exponents(const JobDev& j, const double* alpha, int c0,
                                          int stride) {
  const bool f32 = j.prec == 1;
  const int P = f32 ? 24 : 53, s = f32 ? 25 : 54;
  for (int c = c0; c < j.K; c += stride) {
    const double tw = f32 ? (double)j.twin_pn32[c] : j.twin_pn64[c];
    const double a = f32 ? (double)(float)alpha[c] : alpha[c];
    const double gb = f32 ? (double)((const float*)j.gbound)[c] : ((const double*)j.gbound)[c];
    const int ea = tw == 0.0 ? -100000 : floor_log2(tw) + P + 4;
    const int la = floor_log2(a), lg = floor_log2(gb);
    const int eb = (la >= 100000 || lg >= 100000) ? 100000 : la + lg + 4 - s + P;
    j.skx[2 * c] = ea;
    j.skx[2 * c + 1] = eb;
  }
}

// Stratified layout of a channel with n calls in d dimensions, at least
// s_min calls per box (Sec. 3.3): nr = the largest integer with s_min nr^d
// <= n (at most 2^20) boxes per axis, and floor(n / nr^d) calls per box.
__device__ inline void strat_layout(int64_t n, int d, int64_t s_min, int64_t* nr,
                                    int64_t* per_box, int64_t* boxes_out) {
  int64_t r = 1;
  for (;;) {
    const int64_t r1 = r + 1;
    if (r1 > ((int64_t)1 << 20)) break;
    int64_t boxes = 1;
    bool over = false;
    for (int k = 0; k < d && !over; ++k) {
      if (boxes > n / r1) over = true;
      else boxes *= r1;
    }
    if (over || boxes > n / s_min) break;
    r = r1;
  }
  int64_t boxes = 1;
  for (int k = 0; k < d; ++k) boxes *= r;
  *nr = r;
  *per_box = n / boxes;
  *boxes_out = boxes;
}

constexpr int kAllocMaxK = 1024;  // the channel limit of the interface

__global__ __launch_bounds__(64) void k_allocate(const JobDev* jobs, int64_t n_override,
                                                 int to_trace, int* counter) {
  __shared__ double frac[kAllocMaxK];
  __shared__ int64_t ncs[kAllocMaxK];
  __shared__ int64_t tot_s;
  const int tid = threadIdx.x;
  if (counter && blockIdx.x == 0 && tid < 8) counter[tid] = 0;  // the 8 unit queues
  const JobDev& j = jobs[blockIdx.x];
  const int K = j.K;
  const int64_t N = n_override > 0 ? n_override : j.n_points;
  const int64_t min_calls = j.min_calls;
  const double* alpha_in = j.alpha;
  int64_t* nc = to_trace ? j.t_nc : j.nc;
  int64_t* start = to_trace ? j.t_start : j.start;
  double* alpha_out = to_trace ? j.t_alpha : j.alpha;
  int64_t part = 0;
  for (int c = tid; c < K; c += 64) {
    const double v = alpha_in[c] * (double)N;
    const double fl = floor(v);
    int64_t b = (int64_t)fl;
    double fr = v - fl;
    if (b < min_calls) {
      b = min_calls;
      fr = -1.0;
    }
    frac[c] = fr;
    ncs[c] = b;
    part += b;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
  __syncthreads();
  const int64_t rem = N - part;  // every lane holds the sum
  if (rem > 0) {
    const int64_t q = rem / K, r = rem % K;
    for (int c = tid; c < K; c += 64) {
      const double fc = frac[c];
      int rank = 0;
      for (int c2 = 0; c2 < K; ++c2) {
        const double f2 = frac[c2];
        rank += (f2 > fc || (f2 == fc && c2 < c)) ? 1 : 0;
      }
      ncs[c] += q + (rank < r ? 1 : 0);
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (j.strat > 0) {
      // pseudo-stratified passes take whole boxes: N_c = calls per box x
      // boxes (Sec. 3.3 fixes N = s n^d; Sec. 3.4 lets N and alpha follow
      // whole numbers of calls)
      int64_t* nrv = to_trace ? j.t_nr : j.nr;
      int64_t* spbv = to_trace ? j.t_spb : j.spb;
      int64_t btot = 0;
      for (int c = 0; c < K; ++c) {
        int64_t boxes = 0;
        strat_layout(ncs[c], j.d, j.strat, &nrv[c], &spbv[c], &boxes);
        ncs[c] = spbv[c] * boxes;
        if (!to_trace) j.bstart[c] = btot;
        btot += boxes;
      }
      if (!to_trace) j.bstart[K] = btot;
    }
    int64_t acc = 0;
    start[0] = 0;
    for (int c = 0; c < K; ++c) {
      acc += ncs[c];
      start[c + 1] = acc;
    }
    tot_s = acc;
  }
  __syncthreads();
  const double tot = (double)tot_s;
  for (int c = tid; c < K; c += 64) {
    nc[c] = ncs[c];
    alpha_out[c] = (double)ncs[c] / tot;
  }
  // the factors of the channel terms in the pass precision, as the sample
  // loop forms them: (T)alpha_c gbound_c and (T)alpha_c cnorm_c
  if (j.prec == 1) {
    float* at = static_cast<float*>(to_trace ? j.t_aterm : j.aterm);
    const float* gb = static_cast<const float*>(j.gbound);
    for (int c = tid; c < K; c += 64) {
      const double a = (double)ncs[c] / tot;
      at[c] = (float)a * gb[c];
      at[K + c] = (float)a * j.cnorm32[c];
      at[2 * K + c] = bound_factor<float>(a * (double)j.cnorm32[c]);
    }
  } else {
    double* at = static_cast<double*>(to_trace ? j.t_aterm : j.aterm);
    const double* gb = static_cast<const double*>(j.gbound);
    for (int c = tid; c < K; c += 64) {
      const double a = (double)ncs[c] / tot;
      at[c] = a * gb[c];
      at[K + c] = a * j.cnorm64[c];
      at[2 * K + c] = bound_factor<double>(a * j.cnorm64[c]);
    }
  }
  // the skip offsets follow the weights of the pass that comes next (a real
  // pass or a trace); every real pass is preceded by its own allocation
  __syncthreads();
  set_skip_exponents(j, alpha_out, tid, 64);
}

// ---------------------------------------------------------------------------
// Finalize (Sec. 3.1 E_N and V_N per channel; Sec. 3.4 multi-channel
// estimator).  Workgroup (c, job) reduces the segment partials of channel c
// in work-unit order and the per-bin histograms; deterministic.  The pass of
// a job was split into G units: from the unit prefix of a job table, or the
// single job's G.
// ---------------------------------------------------------------------------
__device__ inline int64_t seg_of(int64_t i, int G, int64_t ntot) {
  return ((i + 1) * (int64_t)G - 1) / ntot;
}

__global__ void k_finalize_channels(const JobDev* jobs, const int* unit_prefix, int G1) {
  const JobDev& j = jobs[blockIdx.y];
  const int c = blockIdx.x;
  if (c >= j.K) return;
  const int G = unit_prefix ? unit_prefix[blockIdx.y + 1] - unit_prefix[blockIdx.y] : G1;
  // the pass split the calls (or, stratified, the boxes) into G units
  const bool strat = j.strat > 0;
  const int64_t ntot = strat ? j.bstart[j.K] : j.start[j.K];
  const int64_t g0 = seg_of(strat ? j.bstart[c] : j.start[c], G, ntot);
  const int64_t g1 = seg_of((strat ? j.bstart[c + 1] : j.start[c + 1]) - 1, G, ntot);
  const int dn = j.d * j.n;
  const double* hpart = j.hpart;
  double* hist = j.hist;
  // the reads of 16 (8) slots are issued together; the additions keep
  // slot order
  constexpr int kAheadH = 16, kAhead = 8;
  for (int t = threadIdx.x; t < dn; t += blockDim.x) {
    double h = 0.0;
    int64_t g = g0;
    for (; g + kAheadH - 1 <= g1; g += kAheadH) {
      double v[kAheadH];
#pragma unroll
      for (int u = 0; u < kAheadH; ++u) v[u] = hpart[(size_t)(g + u + c) * dn + t];
#pragma unroll
      for (int u = 0; u < kAheadH; ++u) h += v[u];
    }
    for (; g <= g1; ++g) h += hpart[(size_t)(g + c) * dn + t];
    hist[(size_t)c * dn + t] = h;
  }
  if (threadIdx.x == 0) {
    Neu s1{0.0, 0.0}, s2{0.0, 0.0}, sq{0.0, 0.0};
    double wmax = 0.0, nbad = 0.0;
    auto take = [&](const double* r) {
      s1.add(r[0]);
      s1.add(r[1]);
      s2.add(r[2]);
      s2.add(r[3]);
      wmax = fmax(wmax, r[4]);
      nbad += r[5];
      if (strat) sq.add(r[6]);
    };
    int64_t g = g0;
    for (; g + kAhead - 1 <= g1; g += kAhead) {
      double v[kAhead][7];
#pragma unroll
      for (int u = 0; u < kAhead; ++u) {
        const double* r = j.part + (size_t)(g + u + c) * kPartStride;
#pragma unroll
        for (int w = 0; w < 7; ++w) v[u][w] = r[w];
      }
#pragma unroll
      for (int u = 0; u < kAhead; ++u) take(v[u]);
    }
    for (; g <= g1; ++g) take(j.part + (size_t)(g + c) * kPartStride);
    const double N = (double)j.nc[c];
    const double S1 = s1.s + s1.c, S2 = s2.s + s2.c;
    const double E = S1 / N, W = S2 / N;
    double V;
    if (strat) {
      // stratified: Var(S1) = sum over boxes of m sigma_b^2, estimated by
      // m/(m-1) sum_b SSW_b with SSW_b the squared deviations of the box's
      // weights from its mean (slot word 6); V = that / N
      const double m = (double)j.spb[c];
      const double v = (m / (m - 1.0)) * (sq.s + sq.c) / N;
      V = v > 0.0 ? v : 0.0;
    } else {
      const double v = W - E * E;
      V = (j.nc[c] > 1) ? (v > 0.0 ? v : 0.0) * N / (N - 1.0) : 0.0;
    }
    double* st = j.chstats + (size_t)c * kStatStride;
    st[0] = S1;
    st[1] = S2;
    st[2] = wmax;
    st[3] = nbad;
    st[4] = E;
    st[5] = W;
    st[6] = V;
    st[7] = N;
  }
}

// Total estimate, error sqrt(sum_c (N_c/N)^2 V_c / N_c) and the history
// record of the pass, at row *iter_dev, which then counts the pass.  A full
// history is left untouched (the host rejects such a pass beforehand).
__global__ __launch_bounds__(64) void k_finalize_total(const JobDev* jobs) {
  // the channel records staged in LDS by every lane, the sums in channel
  // order by lane 0
  __shared__ double sts[kAllocMaxK][5];
  const JobDev& j = jobs[blockIdx.x];
  const int iter = *j.iter_dev;
  if (iter < 0 || iter >= j.max_iter) return;  // uniform
  for (int c = threadIdx.x; c < j.K; c += 64) {
    const double* st = j.chstats + (size_t)c * kStatStride;
    sts[c][0] = st[0];
    sts[c][1] = st[7];
    sts[c][2] = st[6];
    sts[c][3] = st[2];
    sts[c][4] = st[3];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double ntot = (double)j.start[j.K];
  double e = 0.0, var = 0.0, wmax = 0.0, nbad = 0.0;
  for (int c = 0; c < j.K; ++c) {
    e += sts[c][0];
    const double N = sts[c][1];
    const double fr = N / ntot;
    var += fr * fr * sts[c][2] / N;
    wmax = fmax(wmax, sts[c][3]);
    nbad += sts[c][4];
  }
  double* h = j.history + (size_t)iter * kHistStride;
  h[0] = e / ntot;
  h[1] = sqrt(var);
  h[2] = ntot;
  h[3] = wmax;
  h[4] = nbad;
  *j.iter_dev = iter + 1;
}

// ---------------------------------------------------------------------------
// Channel equivalences (Sec. 3.5: the bin weights of channels that share a
// structure are combined, with a permutation of the axes and an identity,
// invert, symmetric or invariant mapping, before rebinning).  The bin
// weights are the per-bin sums of w^2 (eq. 31).  A channel named on the left
// of any equivalence (c, c', perm, mode) gets the sum of its equivalences in
// list order, from zero (its own sums enter through an entry (c, c,
// identity)); per axis k, channel c' contributes its axis perm[k] as is
// (identity), mirrored, j -> n-1-j (invert), or as the mean of both
// (symmetric); an invariant axis gets weight 1 in every bin (its grid is
// kept).  Other channels keep their own sums.  One workgroup per (channel,
// axis) of a job (grid row y = job), one bin per lane; the additions of a
// bin run in list order.
// ---------------------------------------------------------------------------
constexpr int kEqIdentity = 0, kEqInvert = 1, kEqSymmetric = 2;

__global__ void k_equivalences(const JobDev* jobs) {
  const JobDev& j = jobs[blockIdx.y];
  const int ax = blockIdx.x;
  if (j.n_eq == 0 || ax >= j.K * j.d) return;  // uniform over the workgroup
  if (*j.iter_dev >= j.adapt_passes) return;
  const int d = j.d, n = j.n, rec = 2 + 2 * d;
  const int c = ax / d, k = ax - c * d;
  bool listed = false, invariant = false;
  for (int e = 0; e < j.n_eq; ++e) {
    const int32_t* r = j.eq + (size_t)e * rec;
    if (r[0] != c) continue;
    listed = true;
    invariant |= r[2 + d + k] > kEqSymmetric;
  }
  for (int b = threadIdx.x; b < n; b += blockDim.x) {
    double w = listed ? 0.0 : j.hist[(size_t)ax * n + b];
    for (int e = 0; e < j.n_eq; ++e) {
      const int32_t* r = j.eq + (size_t)e * rec;
      if (r[0] != c) continue;
      const double* h2 = j.hist + ((size_t)r[1] * d + r[2 + k]) * n;
      const int mode = r[2 + d + k];
      if (mode == kEqIdentity) w += h2[b];
      else if (mode == kEqInvert) w += h2[n - 1 - b];
      else if (mode == kEqSymmetric) w += 0.5 * (h2[b] + h2[n - 1 - b]);
    }
    j.hist_eq[(size_t)ax * n + b] = invariant ? 1.0 : w;
  }
}

// ---------------------------------------------------------------------------
// Grid refinement (eq. 30, eq. 31): one workgroup per (channel, dim) of a job
// (grid row y = job).  The per-bin measures are computed in parallel; lane 0
// does the ordered sums and the walk, over the edges staged in LDS, so that
// the result is the serial IEEE sequence.
// ---------------------------------------------------------------------------
__global__ void k_refine_grid(const JobDev* jobs) {
  __shared__ double om[256];
  __shared__ double m[256];
  __shared__ double out[257];
  __shared__ double es[257];
  __shared__ double pre[257];
  const JobDev& j = jobs[blockIdx.y];
  const int ax = blockIdx.x;
  if (ax >= j.K * j.d) return;
  if (*j.iter_dev >= j.adapt_passes) return;  // the job's last pass: grids stay
  const int n = j.n;
  double* e = j.edges + (size_t)ax * (n + 1);
  const double* h = (j.n_eq > 0 ? j.hist_eq : j.hist) + (size_t)ax * n;
  __shared__ double s_sum;
  for (int i = threadIdx.x; i < n; i += blockDim.x) om[i] = sqrt(h[i]);
  for (int i = threadIdx.x; i <= n; i += blockDim.x) es[i] = e[i];  // the walk reads LDS
  __syncthreads();
  if (threadIdx.x == 0) {  // the ordered sum
    double sum = 0.0;
    for (int i = 0; i < n; ++i) sum += om[i];
    s_sum = sum;
  }
  __syncthreads();
  const double sum = s_sum;
  if (!(sum > 0.0) || !isfinite(sum)) return;  // nothing to adapt to (uniform)
  const double a = j.grid_power;
  // the per-bin weights of eq. 30 are independent: one bin per lane
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double r = om[i] / sum;
    double v;
    if (r == 0.0) v = 0.0;
    else if (r == 1.0) v = 1.0;
    else v = pow((r - 1.0) / log(r), a);
    m[i] = v;
  }
  __syncthreads();
  // The serial walk: for new edge i, target = i M / n with M the ordered sum
  // of the m; acc runs through the ordered prefix sums S_b while m_b = 0 or
  // S_{b+1} < target, and the edge is interpolated in bin b.  Its stop is
  // the first b with S_{b+1} >= target (m_b > 0 there, S_{b+1} > S_b), else
  // n - 1: lane 0 forms the prefix sums in order, every lane finds its
  // edges' bins by bisection and interpolates with acc = S_b, the walk's
  // operands.
  if (threadIdx.x == 0) {
    double acc = 0.0;
    pre[0] = 0.0;
    for (int i = 0; i < n; ++i) {
      acc += m[i];
      pre[i + 1] = acc;
    }
    out[0] = 0.0;
    out[n] = 1.0;
  }
  __syncthreads();
  const double M = pre[n];
  for (int i = threadIdx.x + 1; i < n; i += blockDim.x) {
    const double target = ((double)i * M) / (double)n;
    int lo = 0, hi = n - 1;  // first b in [0, n - 1) with pre[b + 1] >= target, else n - 1
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (pre[mid + 1] >= target) hi = mid;
      else lo = mid + 1;
    }
    const int b = lo;
    out[i] = es[b] + ((target - pre[b]) / m[b]) * (es[b + 1] - es[b]);
  }
  __syncthreads();
  // The serial fix-ups (edges made strictly increasing forward, then
  // backward; in FP32 the edges rounded and fixed the same way) change
  // nothing when no pair violates them: every lane checks its pairs, and
  // lane 0 runs them only if some pair does.
  bool bad = false;
  for (int i = threadIdx.x + 1; i < n; i += blockDim.x)
    bad |= !(out[i] > out[i - 1]) || !(out[i] < out[i + 1]);
  if (__syncthreads_or(bad)) {
    if (threadIdx.x == 0) {
      for (int i = 1; i < n; ++i)
        if (!(out[i] > out[i - 1])) out[i] = nextafter(out[i - 1], 2.0);
      for (int i = n - 1; i >= 1; --i)
        if (!(out[i] < out[i + 1])) out[i] = nextafter(out[i + 1], -1.0);
    }
    __syncthreads();
  }
  if (j.prec == 1) {
    bool bad32 = false;
    for (int i = threadIdx.x + 1; i < n; i += blockDim.x) {
      const float f = (float)out[i];
      bad32 |= !(f > (float)out[i - 1]) || !(f < (float)out[i + 1]);
    }
    if (__syncthreads_or(bad32)) {
      if (threadIdx.x == 0) snap_axis32(n, out);
    } else {
      for (int i = threadIdx.x + 1; i < n; i += blockDim.x) out[i] = (double)(float)out[i];
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i <= n; i += blockDim.x) e[i] = out[i];
}

// Channel weights, eq. 15 with omega_c = W_c (second moment of the weights);
// one wavefront per job: the powers one channel per lane, the normalising
// sum in channel order by one lane, the division per lane (the oracle's
// operations in its order).
__global__ __launch_bounds__(64) void k_update_alpha(const JobDev* jobs) {
  __shared__ double pw[kAllocMaxK];
  __shared__ double den_s;
  const JobDev& j = jobs[blockIdx.x];
  if (*j.iter_dev >= j.adapt_passes) return;  // the job's last pass: alpha stays (uniform)
  const int K = j.K, tid = threadIdx.x;
  const double beta = j.channel_power;
  // the powers in parallel, the normalising sum in channel order (one lane)
  for (int c = tid; c < K; c += 64) pw[c] = pow(j.chstats[c * kStatStride + 5], beta);
  __syncthreads();
  if (tid == 0) {
    double den = 0.0;
    for (int c = 0; c < K; ++c) den += j.alpha[c] * pw[c];
    den_s = den;
  }
  __syncthreads();
  const double den = den_s;
  if (!(den > 0.0) || !isfinite(den)) return;  // uniform
  for (int c = tid; c < K; c += 64) j.alpha[c] = j.alpha[c] * pw[c] / den;
}

}  // namespace

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

void set_extents(JobSet& js) {
  js.maxK = js.maxKd = js.maxd = 0;
  js.maxTab = js.maxCells = 0;
  js.has_eq = false;
  for (int i = 0; i < js.n; ++i) {
    const JobDev& j = js.host[i];
    js.has_eq |= j.n_eq > 0;
    if (j.K > js.maxK) js.maxK = j.K;
    if (j.K * j.d > js.maxKd) js.maxKd = j.K * j.d;
    if (j.d > js.maxd) js.maxd = j.d;
    const int64_t t = (int64_t)j.K * j.d * j.sT, h = (int64_t)j.K * j.d * j.M;
    if (t > js.maxTab) js.maxTab = t;
    if (h > js.maxCells) js.maxCells = h;
  }
}

void launch_setup(const JobDev& j, hipStream_t s) {
  const int nmax = (j.K > j.P ? j.K : j.P) * j.d;
  hipLaunchKernelGGL(k_setup_maps, dim3(cdiv(nmax, 256)), dim3(256), 0, s, j);
  hipLaunchKernelGGL(k_setup_norms, dim3(cdiv(j.K > j.P ? j.K : j.P, 256)), dim3(256), 0, s, j);
  hipLaunchKernelGGL(k_setup_twins, dim3(cdiv(j.K, 256)), dim3(256), 0, s, j);
  hipLaunchKernelGGL(k_init_grid, dim3(cdiv(j.K * j.d, 128)), dim3(128), 0, s, j);
}

void launch_tables(const JobSet& js, hipStream_t s) {
  if (js.n < 1) return;
  const dim3 gt(cdiv(js.maxTab, 256), js.n), gh(cdiv(js.maxCells, 256), js.n);
  if (js.prec == 1) {
    hipLaunchKernelGGL(k_tables<float>, gt, dim3(256), 0, s, js.dev);
    hipLaunchKernelGGL(k_cells<float>, gh, dim3(256), 0, s, js.dev);
    hipLaunchKernelGGL(k_gbound<float>, dim3(js.maxK, js.n), dim3(64), 0, s, js.dev);
  } else {
    hipLaunchKernelGGL(k_tables<double>, gt, dim3(256), 0, s, js.dev);
    hipLaunchKernelGGL(k_cells<double>, gh, dim3(256), 0, s, js.dev);
    hipLaunchKernelGGL(k_gbound<double>, dim3(js.maxK, js.n), dim3(64), 0, s, js.dev);
  }
}

void launch_allocate(const JobSet& js, int64_t n_override, bool to_trace, hipStream_t s) {
  if (js.n < 1) return;
  hipLaunchKernelGGL(k_allocate, dim3(js.n), dim3(64), 0, s, js.dev, n_override,
                     to_trace ? 1 : 0, js.counter);
}

void launch_finalize(const JobSet& js, int G, hipStream_t s) {
  if (js.n < 1) return;
  hipLaunchKernelGGL(k_finalize_channels, dim3(js.maxK, js.n), dim3(1024), 0, s, js.dev,
                     js.unit_prefix, G);
  hipLaunchKernelGGL(k_finalize_total, dim3(js.n), dim3(64), 0, s, js.dev);
}

void launch_refine_grid(const JobSet& js, hipStream_t s) {
  if (js.n < 1) return;
  if (js.has_eq)
    hipLaunchKernelGGL(k_equivalences, dim3(js.maxKd, js.n), dim3(64), 0, s, js.dev);
  hipLaunchKernelGGL(k_refine_grid, dim3(js.maxKd, js.n), dim3(64), 0, s, js.dev);
}

void launch_update_alpha(const JobSet& js, hipStream_t s) {
  if (js.n < 1) return;
  hipLaunchKernelGGL(k_update_alpha, dim3(js.n), dim3(64), 0, s, js.dev);
}

}  // namespace mcv
