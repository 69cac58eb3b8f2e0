// Instantiations of the batched sample kernel in FP32 (its own translation
// unit so that the two precisions compile in parallel).
#include "sample_kernel.h"

namespace mcv {

namespace {

template <int LB, bool TB>
const void* by_dim(int maxd) {
  if (maxd <= 4) return (const void*)k_sample_queue<float, 4, LB, TB>;
  if (maxd <= 8) return (const void*)k_sample_queue<float, 8, LB, TB>;
  if (maxd <= 12) return (const void*)k_sample_queue<float, 12, LB, TB>;
  if (maxd <= 16) return (const void*)k_sample_queue<float, 16, LB, TB>;
  return (const void*)k_sample_queue<float, 32, LB, TB>;
}

template <bool TB>
const void* by_bound(int maxd, int lb) {
  return lb > 512 ? by_dim<1024, TB>(maxd) : lb > 256 ? by_dim<512, TB>(maxd) : by_dim<256, TB>(maxd);
}

}  // namespace

// Dimension buckets are coarser than for the single-job kernel: every job of
// a set runs the bucket of the set's largest dimension.
const void* queue_kernel_f32(int maxd, int lb, bool term_bound) {
  return term_bound ? by_bound<true>(maxd, lb) : by_bound<false>(maxd, lb);
}

}  // namespace mcv
