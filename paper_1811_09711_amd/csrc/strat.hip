// The pseudo-stratified sample pass (Sec. 3.3): r space of each channel is cut
// into nr^d equal boxes, every box gets the same number m of calls (at least
// the problem's strat, see the allocation kernel), each uniform inside its
// box; the VEGAS step map carries r to x (the boxes are not the grid's bins:
// pseudo-stratification), and the weights, sums and per-bin sums follow the
// importance-sampling pass.  The error of a channel comes from the spread of
// the weights inside each box: per box, the squared deviations from the box
// mean, taken one pass over the box as deviations from its first finite weight
// (sum d and sum d^2 give SSW = sum d^2 - (sum d)^2 / k); unlike S2 - Q/m
// this does not cancel when the boxes leave little spread.
//
// Work split: the pass's boxes, channel by channel, are split into G units;
// each lane takes one box per round and evaluates its m calls one after the
// other: the own map from the segment's x-space table staged in LDS, then
// every other channel's terms as the importance pass forms them (grouped
// hint-cell reads, the term bound of reading R25).  Call i_c of channel c
// (i_c = box m + t) is call start_c + i_c of the pass for the Philox words,
// and substream i_c of the channel's stream for MRG32k3a.
//
// Bin and fraction of axis k from the box digit b (digit k of the box index
// in base nr) and the word u: r = (b + u 2^-32) / nr as the fixed-point
// R = b 2^32 + u over nr 2^32; j = floor(R n / (nr 2^32)), fraction
// (rem + 1/2) / (nr 2^32) with rem = R n - j nr 2^32 (one correctly rounded
// FP64 division); FP32 mode rounds it to FP32 (the largest float below 1 if
// that rounds to 1).
#include <hip/hip_runtime.h>

#include "sample_kernel.h"

namespace mcv {

namespace {

constexpr int kStratBlock = 256;

// Registers capped for 6 waves per SIMD in FP32, 4 in FP64: uncapped, the
// kernel took 173 VGPRs at 12 axes (2 waves per SIMD); at 7 waves in FP32
// (the importance pass's cap) d = 10, 32 channels, s = 2 took 13.7 ms
// against 11.6.
template <typename T>
constexpr int kStratMinWaves = sizeof(T) == 4 ? 6 : 4;

template <typename T, int MAXD>
__global__ __launch_bounds__(kStratBlock, kStratMinWaves<T>) void k_sample_strat(SampleArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int GROUP = sizeof(T) == 4 ? 5 : 2;
  Pair<T>* ownT = reinterpret_cast<Pair<T>*>(smem + a.off_own);
  double* hist = reinterpret_cast<double*>(smem + a.off_hist);
  double* red = reinterpret_cast<double*>(smem + a.off_red);
  const int d = a.d, n = a.n, K = a.K, tid = threadIdx.x, dn = d * n;
  const int sT = a.sT, chT = d * sT;
  CP<double> alpha = cp(a.alpha);
  CP<DimMap<T>> cmap = cp(a.cmap);
  CP<ChanType> ctype = cp(a.ctype);
  CP<T> cnorm = cp(a.cnorm);
  CP<T> twin = cp(a.twin_pn);
  CP<T> gab = cp(a.gab);
  const int g = blockIdx.x, G = gridDim.x;
  CP<int64_t> start = cp(a.start);
  CP<int64_t> bstart = cp(a.bstart);
  const uint32_t tag = (uint32_t)cp(a.iter)[0];
  const int64_t btot = bstart[K];
  const int64_t lo = (int64_t)g * btot / G, hi = (int64_t)(g + 1) * btot / G;
  if (lo >= hi) return;  // uniform
  for (int t = tid; t < dn; t += kStratBlock) hist[t] = 0.0;
  int c = 0;
  while (c < K - 1 && bstart[c + 1] <= lo) ++c;
  for (; c < K && bstart[c] < hi; ++c) {
    const int64_t b0 = bstart[c] > lo ? bstart[c] : lo;
    const int64_t b1 = bstart[c + 1] < hi ? bstart[c + 1] : hi;
    const uint32_t nr = (uint32_t)cp(a.nr)[c];
    const int64_t m = cp(a.spb)[c];
    __syncthreads();  // the previous segment's histogram is flushed
    copy16(ownT, a.xtab + (size_t)c * chT, chT * (int)sizeof(Pair<T>), kStratBlock);
    __syncthreads();
    CP<DimMap<T>> cm_c = cmap + (size_t)c * d;
    const T own_norm = (T)alpha[c] * cnorm[c];
    const int iso_c = ctype[c].iso;
    const uint32_t gm_c = ctype[c].gmask, bm_c = ctype[c].bmask;
    const T tw_c = twin[c];
    const bool small_boxes = bstart[c + 1] - bstart[c] <= (int64_t)0xFFFFFFFF;
    Neu S1{0.0, 0.0}, S2{0.0, 0.0}, SW{0.0, 0.0};
    double wmax = 0.0, nbad = 0.0;
    for (int64_t box = b0 + tid; box < b1; box += kStratBlock) {
      const int64_t q = box - bstart[c];  // the box among the channel's
      uint32_t dig[MAXD];
      if (small_boxes) {  // uniform: 32-bit divisions (a 64-bit one is a long sequence)
        uint32_t rest = (uint32_t)q;
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
          if (k < d) {
            const uint32_t next = rest / nr;
            dig[k] = rest - next * nr;
            rest = next;
          }
        }
      } else {
        uint64_t rest = (uint64_t)q;
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
          if (k < d) {
            dig[k] = (uint32_t)(rest % nr);
            rest /= nr;
          }
        }
      }
      double bs = 0.0, bs2 = 0.0, w0 = 0.0, bd = 0.0, bd2 = 0.0;
      int64_t kf = 0;  // finite weights in the box
      for (int64_t t = 0; t < m; ++t) {
        const int64_t i_c = q * m + t;
        uint32_t u[MAXD];
        if (a.rng) {
          Mrg st = mrg_call_state(a.mrg, c, (uint64_t)i_c, tag);
#pragma unroll
          for (int k = 0; k < MAXD; ++k)
            if (k < d) u[k] = mrg_word(st);
        } else {
          draw_words<MAXD>(a.seed, (uint64_t)(start[c] + i_c), tag, d, u);
        }
        uint32_t jj[MAXD];
        T fr[MAXD];
#pragma unroll
        for (int k = 0; k < MAXD; ++k) {
          jj[k] = 0u;
          fr[k] = T(0);
          if (k < d) strat_bin_frac<T>(dig[k], u[k], nr, n, jj[k], fr[k]);
        }
        T p[MAXD];
        uint32_t jpk[(MAXD + 3) / 4];
        const T own = forward_point_jf<T, MAXD>(jj, fr, d, cm_c, ownT, sT, p, jpk);
        const T r_c = chan_r<T, MAXD>(gab + (size_t)c * 2 * d, iso_c, gm_c, bm_c, d, p);
        T f = tw_c * r_c, gg = own_norm * own * r_c;
        other_terms<T, MAXD, GROUP, false, true, kLazyWalks<T>>(a, c, d, a.M, a.mshift, p, f, gg);
        const T wt = f / gg;
        if (!isfinite(wt)) {
          nbad += 1.0;
          continue;
        }
        const double w = (double)wt;
        bs += w;
        bs2 += w * w;
        if (kf == 0) w0 = w;
        const double e = w - w0;
        bd += e;
        bd2 += e * e;
        ++kf;
        wmax = fmax(wmax, fabs(w));
#pragma unroll
        for (int k = 0; k < MAXD; ++k)
          if (k < d)
            __hip_atomic_fetch_add(hist + k * n + jj[k], w * w, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      S1.add(bs);
      S2.add(bs2);
      if (kf > 1) SW.add(fmax(bd2 - bd * bd / (double)kf, 0.0));
    }
    // segment reduction: wavefront butterflies, then LDS across waves
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      S1 = neu_merge(S1, Neu{__shfl_xor(S1.s, off), __shfl_xor(S1.c, off)});
      S2 = neu_merge(S2, Neu{__shfl_xor(S2.s, off), __shfl_xor(S2.c, off)});
      SW = neu_merge(SW, Neu{__shfl_xor(SW.s, off), __shfl_xor(SW.c, off)});
      wmax = fmax(wmax, __shfl_xor(wmax, off));
      nbad += __shfl_xor(nbad, off);
    }
    const int wave = tid >> 6;
    if ((tid & 63) == 0) {
      double* r = red + wave * 8;
      r[0] = S1.s;
      r[1] = S1.c;
      r[2] = S2.s;
      r[3] = S2.c;
      r[4] = wmax;
      r[5] = nbad;
      r[6] = SW.s;
      r[7] = SW.c;
    }
    __syncthreads();
    const size_t slot = (size_t)g + (size_t)c;
    if (tid == 0) {
      Neu A{red[0], red[1]}, B{red[2], red[3]}, C{red[6], red[7]};
      double wm = red[4], nb = red[5];
      for (int w = 1; w < kStratBlock / 64; ++w) {
        A = neu_merge(A, Neu{red[w * 8 + 0], red[w * 8 + 1]});
        B = neu_merge(B, Neu{red[w * 8 + 2], red[w * 8 + 3]});
        C = neu_merge(C, Neu{red[w * 8 + 6], red[w * 8 + 7]});
        wm = fmax(wm, red[w * 8 + 4]);
        nb += red[w * 8 + 5];
      }
      double* r = a.part + slot * kPartStride;
      r[0] = A.s;
      r[1] = A.c;
      r[2] = B.s;
      r[3] = B.c;
      r[4] = wm;
      r[5] = nb;
      r[6] = C.s + C.c;
      r[7] = 0.0;
    }
    for (int t = tid; t < dn; t += kStratBlock) {
      a.hpart[slot * dn + t] = hist[t];
      hist[t] = 0.0;
    }
  }
}

template <typename T, int MAXD>
int launch_t(const JobDev& j, int64_t n_points, hipStream_t s) {
  SampleArgs<T> a = make_args<T>(j, 0);
  // LDS: the segment's x-space table, the per-bin sums and the cross-wave
  // reduction (8 values per wave)
  a.off_own = 0;
  a.off_hist = (j.d * j.sT * (int)sizeof(Pair<T>) + 15) & ~15;
  a.off_red = a.off_hist + ((j.d * j.n * 8 + 15) & ~15);
  const int lds = a.off_red + (kStratBlock / 64) * 8 * 8;
  auto kern = k_sample_strat<T, MAXD>;
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds) !=
          hipSuccess)
    return -1;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, kStratBlock,
                                                   lds) != hipSuccess)
    return -1;
  // about n_points / strat boxes: a few rounds of boxes per workgroup, and
  // as in the importance pass up to kOversub times the co-resident count
  const int G =
      grid_for(j, per_cu, kStratBlock * (j.strat > 0 ? j.strat : 1), n_points, kOversub);
  hipLaunchKernelGGL(kern, dim3(G), dim3(kStratBlock), lds, s, a);
  return G;
}

template <typename T>
int launch_p(const JobDev& j, int64_t n, hipStream_t s) {
  const int d = j.d;
  if (d <= 2) return launch_t<T, 2>(j, n, s);
  if (d <= 4) return launch_t<T, 4>(j, n, s);
  if (d <= 6) return launch_t<T, 6>(j, n, s);
  if (d <= 8) return launch_t<T, 8>(j, n, s);
  if (d <= 10) return launch_t<T, 10>(j, n, s);
  if (d <= 12) return launch_t<T, 12>(j, n, s);
  if (d <= 16) return launch_t<T, 16>(j, n, s);
  return launch_t<T, 32>(j, n, s);
}

}  // namespace

int launch_sample_strat(const JobDev& j, int64_t n_points, hipStream_t s) {
  return j.prec == 1 ? launch_p<float>(j, n_points, s) : launch_p<double>(j, n_points, s);
}

}  // namespace mcv
