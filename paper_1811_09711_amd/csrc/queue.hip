// Instantiations of the batched sample kernel for one precision
// (MCV_QUEUE_FP32), launch bound (MCV_QUEUE_LB) and term-bound option
// (MCV_QUEUE_TB): the build compiles this file once per combination, so that
// the variants (each with a body per dimension) compile in parallel.
#include <type_traits>

#include "sample_kernel.h"

#if !defined(MCV_QUEUE_FP32) || !defined(MCV_QUEUE_LB) || !defined(MCV_QUEUE_TB)
#error "queue.hip is compiled with MCV_QUEUE_FP32, MCV_QUEUE_LB and MCV_QUEUE_TB defined"
#endif

namespace mcv {

namespace {
using QT = std::conditional_t<MCV_QUEUE_FP32 != 0, float, double>;
constexpr bool kTB = MCV_QUEUE_TB != 0;
}  // namespace

// Two buckets by the set's largest dimension: up to 12 (a body per d), and
// up to 32 (the same, plus one generic body for d > 12).
const void* MCV_QUEUE_NAME(MCV_QUEUE_FP32, MCV_QUEUE_LB, MCV_QUEUE_TB)(int maxd) {
  if (maxd <= 12) return (const void*)k_sample_queue<QT, 12, MCV_QUEUE_LB, kTB>;
  return (const void*)k_sample_queue<QT, 32, MCV_QUEUE_LB, kTB>;
}

}  // namespace mcv
