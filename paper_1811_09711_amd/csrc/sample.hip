// Host side of the sample pass (argument records, launches of the
// single-job kernels instantiated in single_f32.hip / single_f64.hip and of
// the batched queue kernels in queue_f32.hip / queue_f64.hip), plus the
// per-call trace and the unweighting trial kernels that share its point
// evaluation.
//
// Brass, Kilian, Reuter, arXiv:1811.09711, Sec. 3.5: for every call r_c of
// channel c, x_c = G_c^{-1}(r_c) with the VEGAS step map (Sec. 3.2, eq. g(x)),
// p = phi_c(x_c), f(p), then for every other channel c' the inverse map and the
// bin of x_c' in grid c' (eq. g(p)); the weight is w = f/g (eq. vamp-master).
// Sums of w and w^2 per channel (Sec. 3.1, eq. 4) and the per-bin sums of w^2
// along each axis (eq. 31) are accumulated for the adaptation.
//
// Work split on the GPU (the paper's OpenMP/MPI split is replaced): the
// calls of a pass are laid out channel by channel (call i belongs to channel c
// iff S_c <= i < S_{c+1}); workgroup g of G takes the contiguous range
// [g N/G, (g+1) N/G) and walks it channel segment by channel segment, so every
// segment is channel-uniform.  Each segment's sums are reduced in registers,
// wavefront shuffles and LDS into one partial record at slot g + c (unique,
// since each new segment increments g or c), its LDS histogram is written to
// the same slot, and a small kernel reduces the slots in order.
//
// The other channels' bins are found through their hint-cell records, read
// from global memory (L2); the segment's own x-space table is staged in LDS.
#include <hip/hip_runtime.h>
#include <string.h>

#include "sample_kernel.h"

namespace mcv {

namespace {

__device__ inline int channel_of(const int64_t* start, int K, int64_t i) {
  int lo = 0, hi = K;  // largest c with start[c] <= i
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename T, int MAXD>
__global__ __launch_bounds__(64) void k_trace(SampleArgs<T> a, const int64_t* tstart,
                                              const double* talpha, int64_t first, int64_t count,
                                              int n_words, uint32_t* words, int32_t* chan,
                                              int32_t* bins, double* pout, double* fgw) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const int64_t i = first + q;
  const int K = a.K, d = a.d;
  const int c = channel_of(tstart, K, i);
  uint32_t u[MAXD];
  if (a.rng) {  // MRG32k3a: substream i - S_c of channel c's stream
    Mrg st = mrg_call_state(a.mrg, c, (uint64_t)(i - tstart[c]), a.tag);
    const int nw = n_words > d ? n_words : d;
    for (int m = 0; m < nw; ++m) {
      const uint32_t wd = mrg_word(st);
      if (m < d && m < MAXD) u[m] = wd;
      if (m < n_words) words[q * n_words + m] = wd;
    }
  } else {
    draw_words<MAXD>(a.seed, (uint64_t)i, a.tag, d, u);
    for (int b = 0; 4 * b < n_words; ++b) {
      const U4 r = philox4x32_10(U4{(uint32_t)i, (uint32_t)(i >> 32), a.tag, (uint32_t)b},
                                 (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
      const uint32_t v[4] = {r.x, r.y, r.z, r.w};
      for (int l = 0; l < 4 && 4 * b + l < n_words; ++l) words[q * n_words + 4 * b + l] = v[l];
    }
  }
  T p[MAXD];
  T f, g;
  if (a.strat) {  // the call's box among the channel's (trace layout in a.nr, a.spb)
    uint64_t rest = (uint64_t)((i - tstart[c]) / a.spb[c]);
    const uint32_t nr = (uint32_t)a.nr[c];
    uint32_t jj[MAXD];
    T fr[MAXD];
#pragma unroll
    for (int k = 0; k < MAXD; ++k) {
      jj[k] = 0u;
      fr[k] = T(0);
      if (k < d) {
        strat_bin_frac<T>((uint32_t)(rest % nr), u[k], nr, a.n, jj[k], fr[k]);
        rest /= nr;
      }
    }
    eval_call_jf<T, MAXD>(a, talpha, c, jj, fr, p, f, g, bins + q * K * d);
  } else {
    eval_call<T, MAXD>(a, talpha, c, u, p, f, g, bins + q * K * d);
  }
  chan[q] = c;
  for (int k = 0; k < d; ++k) pout[q * d + k] = (double)p[k];
  fgw[q * 3 + 0] = (double)f;
  fgw[q * 3 + 1] = (double)g;
  fgw[q * 3 + 2] = (double)(f / g);
}

// Unweighting trials (Sec. 3.5, last paragraph; eq. efficiency): channel
// drawn by alpha through the prefix offsets, the same map and weight chain,
// accept iff u * w_max < |w| (weights may be negative, Sec. 3.1: the event
// then carries the sign).  accept[q]: 0 rejected, 1 kept with w > 0, 2 kept
// with w < 0; wts[q] = |w| (-1 if not finite).
template <typename T, int MAXD>
__global__ __launch_bounds__(256) void k_unweight(SampleArgs<T> a, uint64_t q0, int64_t count,
                                                  const double* wmax, uint8_t* accept, double* wts,
                                                  T* pts) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const uint64_t trial = q0 + (uint64_t)q;
  const int K = a.K, d = a.d;
  uint32_t u[MAXD];
  uint32_t extra[3];
  if (a.rng) {  // MRG32k3a: substream `trial` of the unweighting stream
    Mrg st = mrg_call_state(a.mrg, K, trial, 0);
    for (int m = 0; m < d && m < MAXD; ++m) u[m] = mrg_word(st);
    for (int l = 0; l < 3; ++l) extra[l] = mrg_word(st);
  } else {
    draw_words<MAXD>(a.seed, trial, kTagUnweight, d, u);
    const int b0 = d / 4;
    const U4 r0 = philox4x32_10(U4{(uint32_t)trial, (uint32_t)(trial >> 32), kTagUnweight,
                                   (uint32_t)b0},
                                (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
    const U4 r1 = philox4x32_10(U4{(uint32_t)trial, (uint32_t)(trial >> 32), kTagUnweight,
                                   (uint32_t)(b0 + 1)},
                                (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
    const uint32_t v[8] = {r0.x, r0.y, r0.z, r0.w, r1.x, r1.y, r1.z, r1.w};
    for (int l = 0; l < 3; ++l) extra[l] = v[(d + l) - 4 * b0];
  }
  const uint64_t u64 = (uint64_t)extra[0] | ((uint64_t)extra[1] << 32);
  const int64_t ntot = a.start[K];
  const int64_t r = (int64_t)__umul64hi(u64, (uint64_t)ntot);
  const int c = channel_of(a.start, K, r);
  T p[MAXD];
  T f, g;
  eval_call<T, MAXD>(a, a.alpha, c, u, p, f, g, nullptr);
  const double w = (double)(f / g);
  const double aw = fabs(w);
  const double acc = ((double)extra[2] + 0.5) * 0x1p-32;
  const bool ok = isfinite(w) && (acc * wmax[0] < aw);
  accept[q] = ok ? (w < 0.0 ? 2 : 1) : 0;
  wts[q] = isfinite(w) ? aw : -1.0;
  for (int k = 0; k < d; ++k) pts[q * d + k] = p[k];
}

// Ordered compaction of one unweighting batch, in tiles of kTile trials.
// k_compact_count: per tile, the accepted trials and the largest weight.
// k_compact_scatter: each tile's output offset is the sum of the earlier
// tiles' counts; within the tile a wavefront ballot and a scan of the wave
// totals give every accepted trial its position, and the first `need`
// accepted points are written in trial order; per tile, the last trial kept
// and the number kept above the batch's w_max.  k_compact_final: the batch's
// accepted count, largest weight, last trial kept and overweight count.
constexpr int kTile = 1024;

__device__ inline int64_t block_sum_i64(int64_t v, int64_t* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += shfl_xor_u64((uint64_t)v, off);
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  int64_t t = 0;
  for (int i = 0; i < nw; ++i) t += sh[i];
  return t;
}

__global__ __launch_bounds__(kTile) void k_compact_count(const uint8_t* accept,
                                                         const double* wts, int64_t count,
                                                         int64_t* tcount, double* tmax) {
  __shared__ int64_t sc[kTile / 64];
  __shared__ double sm[kTile / 64];
  const int64_t q = (int64_t)blockIdx.x * kTile + threadIdx.x;
  const bool in = q < count;
  int64_t a = (in && accept[q] != 0) ? 1 : 0;
  double m = in ? wts[q] : -1.0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  a = block_sum_i64(a, sc);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = sm[0];
    for (int i = 1; i < kTile / 64; ++i) mm = fmax(mm, sm[i]);
    tcount[blockIdx.x] = a;
    tmax[blockIdx.x] = mm;
  }
}

template <typename T>
__global__ __launch_bounds__(kTile) void k_compact_scatter(
    const uint8_t* accept, const double* wts, const T* pts, int64_t count, int d,
    const double* wmax, int64_t need, T* out, int64_t out_stride, int64_t out_base,
    int8_t* signs, const int64_t* tcount, int64_t* tlast, int64_t* tover) {
  __shared__ int64_t sh[kTile / 64];
  __shared__ int wsum[kTile / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int tile = blockIdx.x;
  int64_t before = 0;
  for (int i = t; i < tile; i += kTile) before += tcount[i];
  const int64_t off = block_sum_i64(before, sh);
  const int64_t q = (int64_t)tile * kTile + t;
  const bool acc = q < count && accept[q] != 0;
  const uint64_t mask = __ballot(acc);
  const int below = __popcll(mask & ((1ull << lane) - 1ull));
  if (lane == 0) wsum[w] = __popcll(mask);
  __syncthreads();
  int wbase = 0;
  for (int i = 0; i < w; ++i) wbase += wsum[i];
  const int64_t pos = off + wbase + below;
  int64_t my_last = -1, my_over = 0;
  if (acc && pos < need) {
    for (int k = 0; k < d; ++k) out[(int64_t)k * out_stride + out_base + pos] = pts[q * d + k];
    if (signs) signs[out_base + pos] = accept[q] == 2 ? -1 : 1;
    my_last = q;
    my_over = wts[q] > wmax[0] ? 1 : 0;
  }
  int64_t l = my_last;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t v = (int64_t)shfl_xor_u64((uint64_t)l, o);
    l = v > l ? v : l;
  }
  const int64_t ov = block_sum_i64(my_over, sh);
  __syncthreads();
  if (lane == 0) sh[w] = l;
  __syncthreads();
  if (t == 0) {
    int64_t lm = -1;
    for (int i = 0; i < kTile / 64; ++i) lm = sh[i] > lm ? sh[i] : lm;
    tlast[tile] = lm;
    tover[tile] = ov;
  }
}

__global__ __launch_bounds__(256) void k_compact_final(int ntiles, const int64_t* tcount,
                                                       const double* tmax, const int64_t* tlast,
                                                       const int64_t* tover, int64_t need,
                                                       double* res) {
  __shared__ int64_t st[256], sl[256], so[256];
  __shared__ double sm[256];
  const int t = threadIdx.x;
  int64_t total = 0, lst = -1, ov = 0;
  double bm = -1.0;
  for (int i = t; i < ntiles; i += 256) {
    total += tcount[i];
    bm = fmax(bm, tmax[i]);
    if (tlast[i] > lst) lst = tlast[i];
    ov += tover[i];
  }
  st[t] = total;
  sl[t] = lst;
  so[t] = ov;
  sm[t] = bm;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      st[t] += st[t + h];
      sl[t] = sl[t + h] > sl[t] ? sl[t + h] : sl[t];
      so[t] += so[t + h];
      sm[t] = fmax(sm[t], sm[t + h]);
    }
    __syncthreads();
  }
  if (t == 0) {
    res[0] = (double)(st[0] < need ? st[0] : need);
    res[1] = (double)st[0];
    res[2] = (double)sl[0];
    res[3] = (double)so[0];
    res[4] = sm[0];
    res[5] = 0.0;
  }
}

#define MCV_DISPATCH_D(D, FN, ...)   \
  do {                               \
    if ((D) <= 2) FN<2>(__VA_ARGS__); \
    else if ((D) <= 4) FN<4>(__VA_ARGS__); \
    else if ((D) <= 6) FN<6>(__VA_ARGS__); \
    else if ((D) <= 8) FN<8>(__VA_ARGS__); \
    else if ((D) <= 10) FN<10>(__VA_ARGS__); \
    else if ((D) <= 12) FN<12>(__VA_ARGS__); \
    else if ((D) <= 16) FN<16>(__VA_ARGS__); \
    else FN<32>(__VA_ARGS__); \
  } while (0)

// The batched kernel of a set: precision, launch bound (256, 512 or 1024,
// the smallest that holds the set's), term-bound option, largest dimension.
const void* queue_kernel(const JobSet& js) {
  const int lb = js.bound > 512 ? 1024 : js.bound > 256 ? 512 : 256;
  const int m = js.maxd;
  if (js.prec == 1) {
    if (js.term_bound)
      return lb == 1024 ? MCV_QUEUE_NAME(1, 1024, 1)(m)
             : lb == 512 ? MCV_QUEUE_NAME(1, 512, 1)(m) : MCV_QUEUE_NAME(1, 256, 1)(m);
    return lb == 1024 ? MCV_QUEUE_NAME(1, 1024, 0)(m)
           : lb == 512 ? MCV_QUEUE_NAME(1, 512, 0)(m) : MCV_QUEUE_NAME(1, 256, 0)(m);
  }
  if (js.term_bound)
    return lb == 1024 ? MCV_QUEUE_NAME(0, 1024, 1)(m)
           : lb == 512 ? MCV_QUEUE_NAME(0, 512, 1)(m) : MCV_QUEUE_NAME(0, 256, 1)(m);
  return lb == 1024 ? MCV_QUEUE_NAME(0, 1024, 0)(m)
         : lb == 512 ? MCV_QUEUE_NAME(0, 512, 0)(m) : MCV_QUEUE_NAME(0, 256, 0)(m);
}

template <typename T, int MAXD>
void trace_t(const JobDev& j, uint32_t tag, int64_t first, int64_t count, int n_words,
             uint32_t* words, int32_t* chan, int32_t* bins, double* p, double* fgw,
             hipStream_t s) {
  SampleArgs<T> a = make_args<T>(j, tag);
  a.nr = j.t_nr;  // the trace allocation's stratified layout
  a.spb = j.t_spb;
  const int blocks = (int)((count + 63) / 64);
  hipLaunchKernelGGL((k_trace<T, MAXD>), dim3(blocks), dim3(64), 0, s, a, j.t_start, j.t_alpha,
                     first, count, n_words, words, chan, bins, p, fgw);
}
template <int MAXD>
void trace_f64(const JobDev& j, uint32_t tag, int64_t first, int64_t count, int n_words,
               uint32_t* words, int32_t* chan, int32_t* bins, double* p, double* fgw,
               hipStream_t s) {
  trace_t<double, MAXD>(j, tag, first, count, n_words, words, chan, bins, p, fgw, s);
}
template <int MAXD>
void trace_f32(const JobDev& j, uint32_t tag, int64_t first, int64_t count, int n_words,
               uint32_t* words, int32_t* chan, int32_t* bins, double* p, double* fgw,
               hipStream_t s) {
  trace_t<float, MAXD>(j, tag, first, count, n_words, words, chan, bins, p, fgw, s);
}

template <typename T, int MAXD>
void unweight_t(const JobDev& j, uint64_t q0, int64_t count, const double* wmax, uint8_t* accept,
                double* wts, void* pts, hipStream_t s) {
  SampleArgs<T> a = make_args<T>(j, kTagUnweight);
  const int blocks = (int)((count + 255) / 256);
  hipLaunchKernelGGL((k_unweight<T, MAXD>), dim3(blocks), dim3(256), 0, s, a, q0, count, wmax,
                     accept, wts, reinterpret_cast<T*>(pts));
}
template <int MAXD>
void unweight_f64(const JobDev& j, uint64_t q0, int64_t count, const double* wmax,
                  uint8_t* accept, double* wts, void* pts, hipStream_t s) {
  unweight_t<double, MAXD>(j, q0, count, wmax, accept, wts, pts, s);
}
template <int MAXD>
void unweight_f32(const JobDev& j, uint64_t q0, int64_t count, const double* wmax,
                  uint8_t* accept, double* wts, void* pts, hipStream_t s) {
  unweight_t<float, MAXD>(j, q0, count, wmax, accept, wts, pts, s);
}

}  // namespace

int sample_lds_bytes(const JobDev& j) {
  if (j.prec == 1) {
    SampleArgs<float> a = make_args<float>(j, 0);
    return lds_layout<float>(a, Tune<float>::BLOCK / 64);
  }
  SampleArgs<double> a = make_args<double>(j, 0);
  return lds_layout<double>(a, Tune<double>::BLOCK / 64);
}

int launch_sample(const JobSet& js, int64_t n_points, hipStream_t s) {
  if (js.n != 1) return -1;
  const JobDev& j = js.host[0];
  return j.prec == 1 ? launch_sample_f32(j, n_points, s) : launch_sample_f64(j, n_points, s);
}

size_t sample_args_bytes(int prec) {
  return prec == 1 ? sizeof(SampleArgs<float>) : sizeof(SampleArgs<double>);
}

// The queue kernel keeps a 16-byte header (the unit broadcast) at LDS offset 0.
int sample_queue_layout(const JobDev& j, int block, void* args_host) {
  if (j.prec == 1) {
    SampleArgs<float> a = make_args<float>(j, 0);
    const int b = lds_layout<float>(a, block / 64, 16);
    memcpy(args_host, &a, sizeof a);
    return b;
  }
  SampleArgs<double> a = make_args<double>(j, 0);
  const int b = lds_layout<double>(a, block / 64, 16);
  memcpy(args_host, &a, sizeof a);
  return b;
}

int sample_queue_occupancy(const JobSet& js) {
  const void* kern = queue_kernel(js);
  if (js.lds > 64 * 1024 &&
      hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, js.lds) != hipSuccess)
    return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, js.block, js.lds) != hipSuccess)
    return 0;
  return nb;
}

int launch_sample_queue(const JobSet& js, hipStream_t s) {
  if (js.n < 1 || js.grid < 1 || !js.sargs || !js.unit_prefix || !js.counter) return -1;
  const void* kern = queue_kernel(js);
  void* args[] = {(void*)&js.sargs, (void*)&js.unit_prefix, (void*)&js.n, (void*)&js.n_units,
                  (void*)&js.counter};
  if (hipLaunchKernel(kern, dim3(js.grid), dim3(js.block), args, js.lds, s) != hipSuccess)
    return -1;
  return js.grid;
}

size_t compact_accept_bytes(int64_t count) {
  const int64_t ntiles = (count + kTile - 1) / kTile;
  return (((size_t)count + 255) & ~(size_t)255) + (size_t)ntiles * 4 * sizeof(int64_t);
}

void launch_compact(const JobDev& j, const uint8_t* accept, const double* wts, const void* pts,
                    int64_t count, const double* wmax, int64_t need, void* out,
                    int64_t out_stride, int64_t out_base, int8_t* signs, double* res,
                    hipStream_t s) {
  // per-tile scratch behind the accept flags (see compact_accept_bytes)
  const int ntiles = (int)((count + kTile - 1) / kTile);
  char* scratch = const_cast<char*>(reinterpret_cast<const char*>(accept)) +
                  (((size_t)count + 255) & ~(size_t)255);
  int64_t* tcount = reinterpret_cast<int64_t*>(scratch);
  double* tmax = reinterpret_cast<double*>(tcount + ntiles);
  int64_t* tlast = reinterpret_cast<int64_t*>(tmax + ntiles);
  int64_t* tover = tlast + ntiles;
  hipLaunchKernelGGL(k_compact_count, dim3(ntiles), dim3(kTile), 0, s, accept, wts, count, tcount,
                     tmax);
  if (j.prec == 1)
    hipLaunchKernelGGL(k_compact_scatter<float>, dim3(ntiles), dim3(kTile), 0, s, accept, wts,
                       reinterpret_cast<const float*>(pts), count, j.d, wmax, need,
                       reinterpret_cast<float*>(out), out_stride, out_base, signs, tcount, tlast,
                       tover);
  else
    hipLaunchKernelGGL(k_compact_scatter<double>, dim3(ntiles), dim3(kTile), 0, s, accept, wts,
                       reinterpret_cast<const double*>(pts), count, j.d, wmax, need,
                       reinterpret_cast<double*>(out), out_stride, out_base, signs, tcount, tlast,
                       tover);
  hipLaunchKernelGGL(k_compact_final, dim3(1), dim3(256), 0, s, ntiles, tcount, tmax, tlast, tover,
                     need, res);
}

void launch_trace(const JobDev& j, uint32_t tag, int64_t first, int64_t count, int n_words,
                  uint32_t* words, int32_t* chan, int32_t* bins, double* p, double* fgw,
                  hipStream_t s) {
  if (j.prec == 1)
    MCV_DISPATCH_D(j.d, trace_f32, j, tag, first, count, n_words, words, chan, bins, p, fgw, s);
  else
    MCV_DISPATCH_D(j.d, trace_f64, j, tag, first, count, n_words, words, chan, bins, p, fgw, s);
}

void launch_unweight_batch(const JobDev& j, uint64_t q0, int64_t count, const double* wmax,
                           uint8_t* accept, double* wts, void* pts, hipStream_t s) {
  if (j.prec == 1) MCV_DISPATCH_D(j.d, unweight_f32, j, q0, count, wmax, accept, wts, pts, s);
  else MCV_DISPATCH_D(j.d, unweight_f64, j, q0, count, wmax, accept, wts, pts, s);
}

}  // namespace mcv
