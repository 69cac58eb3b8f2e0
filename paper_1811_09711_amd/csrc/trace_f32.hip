// Trace instantiations of the single-job sample kernel in FP32: k_sample's
// code path (lookup groups, term-bound and partial-exponent skips, launch
// bounds) with each call's f, g and w written for a window of calls, for
// call-by-call checks of the kernel the pass runs.  A translation unit of its
// own so that it compiles beside the pass kernels.
#include "sample_kernel.h"

namespace mcv {

namespace {

template <int MAXD>
int run(const JobDev& j, int G, uint32_t tag, int64_t first, int64_t count, double* out,
        hipStream_t s) {
  return j.d == MAXD ? launch_sample_trace_t<float, MAXD, true>(j, G, tag, first, count, out, s)
                     : launch_sample_trace_t<float, MAXD, false>(j, G, tag, first, count, out, s);
}

}  // namespace

int launch_sample_trace_f32(const JobDev& j, int G, uint32_t tag, int64_t first, int64_t count,
                          double* out, hipStream_t s) {
  if (j.rng) return launch_sample_trace_mrg_f32(j, G, tag, first, count, out, s);
  const int d = j.d;
  if (d <= 2) return run<2>(j, G, tag, first, count, out, s);
  if (d <= 4) return run<4>(j, G, tag, first, count, out, s);
  if (d <= 6) return run<6>(j, G, tag, first, count, out, s);
  if (d <= 8) return run<8>(j, G, tag, first, count, out, s);
  if (d <= 10) return run<10>(j, G, tag, first, count, out, s);
  if (d <= 12) return run<12>(j, G, tag, first, count, out, s);
  if (d <= 16) return run<16>(j, G, tag, first, count, out, s);
  return run<32>(j, G, tag, first, count, out, s);
}

}  // namespace mcv
