// Instantiations of the batched sample kernel in FP32 (its own translation
// unit so that the two precisions compile in parallel).
#include "sample_kernel.h"

namespace mcv {

namespace {

template <int LB>
const void* by_dim(int maxd) {
  if (maxd <= 4) return (const void*)k_sample_queue<float, 4, LB>;
  if (maxd <= 8) return (const void*)k_sample_queue<float, 8, LB>;
  if (maxd <= 12) return (const void*)k_sample_queue<float, 12, LB>;
  if (maxd <= 16) return (const void*)k_sample_queue<float, 16, LB>;
  return (const void*)k_sample_queue<float, 32, LB>;
}

}  // namespace

// Dimension buckets are coarser than for the single-job kernel: every job of
// a set runs the bucket of the set's largest dimension.
const void* queue_kernel_f32(int maxd, int lb) {
  return lb > 512 ? by_dim<1024>(maxd) : lb > 256 ? by_dim<512>(maxd) : by_dim<256>(maxd);
}

}  // namespace mcv
