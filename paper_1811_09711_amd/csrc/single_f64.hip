// Instantiations of the single-job sample kernel in FP64 (a translation unit
// of its own so that the precisions compile in parallel): one per dimension
// bucket, and an exact-dimension variant where the problem's dimension is the
// bucket (no per-axis guards).
#include "sample_kernel.h"

namespace mcv {

namespace {

template <int MAXD>
int run(const JobDev& j, int64_t n, hipStream_t s) {
  return j.d == MAXD ? launch_sample_t<double, MAXD, true>(j, n, s)
                     : launch_sample_t<double, MAXD, false>(j, n, s);
}

template <int MAXD>
int grid(const JobDev& j, int64_t n) {
  return j.d == MAXD ? sample_grid_t<double, MAXD, true>(j, n)
                     : sample_grid_t<double, MAXD, false>(j, n);
}

}  // namespace

int sample_grid_f64(const JobDev& j, int64_t n_points) {
  if (j.rng) return sample_grid_mrg_f64(j, n_points);
  const int d = j.d;
  if (d <= 2) return grid<2>(j, n_points);
  if (d <= 4) return grid<4>(j, n_points);
  if (d <= 6) return grid<6>(j, n_points);
  if (d <= 8) return grid<8>(j, n_points);
  if (d <= 10) return grid<10>(j, n_points);
  if (d <= 12) return grid<12>(j, n_points);
  if (d <= 16) return grid<16>(j, n_points);
  return grid<32>(j, n_points);
}

int launch_sample_f64(const JobDev& j, int64_t n_points, hipStream_t s) {
  if (j.rng) return launch_sample_mrg_f64(j, n_points, s);
  const int d = j.d;
  if (d <= 2) return run<2>(j, n_points, s);
  if (d <= 4) return run<4>(j, n_points, s);
  if (d <= 6) return run<6>(j, n_points, s);
  if (d <= 8) return run<8>(j, n_points, s);
  if (d <= 10) return run<10>(j, n_points, s);
  if (d <= 12) return run<12>(j, n_points, s);
  if (d <= 16) return run<16>(j, n_points, s);
  return run<32>(j, n_points, s);
}

}  // namespace mcv
