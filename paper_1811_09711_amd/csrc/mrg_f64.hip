// Single-job sample kernels in FP64 drawing from MRG32k3a streams (Sec. 4.4,
// eq. mrg32k3a and eq. rngstream), and their trace instantiations: the same
// pass as with Philox words (sample_kernel.h) with each lane carrying its
// substream state across rounds.  A translation unit of its own so that it
// compiles beside the Philox kernels.
#include "sample_kernel.h"

namespace mcv {

namespace {

template <int MAXD>
int run(const JobDev& j, int64_t n, hipStream_t s) {
  return j.d == MAXD ? launch_sample_t<double, MAXD, true, 1>(j, n, s)
                     : launch_sample_t<double, MAXD, false, 1>(j, n, s);
}

template <int MAXD>
int grid(const JobDev& j, int64_t n) {
  return j.d == MAXD ? sample_grid_t<double, MAXD, true, 1>(j, n)
                     : sample_grid_t<double, MAXD, false, 1>(j, n);
}

template <int MAXD>
int trace(const JobDev& j, int G, uint32_t tag, int64_t first, int64_t count, double* out,
          hipStream_t s) {
  return j.d == MAXD
             ? launch_sample_trace_t<double, MAXD, true, 1>(j, G, tag, first, count, out, s)
             : launch_sample_trace_t<double, MAXD, false, 1>(j, G, tag, first, count, out, s);
}

#define MCV_BY_DIM(FN, ...)                   \
  do {                                        \
    const int d_ = j.d;                       \
    if (d_ <= 2) return FN<2>(__VA_ARGS__);   \
    if (d_ <= 4) return FN<4>(__VA_ARGS__);   \
    if (d_ <= 6) return FN<6>(__VA_ARGS__);   \
    if (d_ <= 8) return FN<8>(__VA_ARGS__);   \
    if (d_ <= 10) return FN<10>(__VA_ARGS__); \
    if (d_ <= 12) return FN<12>(__VA_ARGS__); \
    if (d_ <= 16) return FN<16>(__VA_ARGS__); \
    return FN<32>(__VA_ARGS__);               \
  } while (0)

}  // namespace

int launch_sample_mrg_f64(const JobDev& j, int64_t n_points, hipStream_t s) {
  MCV_BY_DIM(run, j, n_points, s);
}

int sample_grid_mrg_f64(const JobDev& j, int64_t n_points) {
  MCV_BY_DIM(grid, j, n_points);
}

int launch_sample_trace_mrg_f64(const JobDev& j, int G, uint32_t tag, int64_t first,
                              int64_t count, double* out, hipStream_t s) {
  MCV_BY_DIM(trace, j, G, tag, first, count, out, s);
}

}  // namespace mcv
