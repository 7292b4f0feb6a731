// The time-marching half stencil (dslash_march.h) for FP64 vectors and links.
#include "dslash_march.h"

namespace hisq {
namespace dslash_impl {
template hisq_status launch_march<double, vec2<double>, vec2<double>>(const DslashArgs<double, vec2<double>, vec2<double>> &, const DslashShape &, bool, bool,
                                      bool, hipStream_t);
}  // namespace dslash_impl
}  // namespace hisq
