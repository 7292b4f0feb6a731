// The time-marching half stencil (dslash_march.h) for FP32 vectors with 16-bit or FP32 links.
#include "dslash_march.h"

namespace hisq {
namespace dslash_impl {
template hisq_status launch_march<float, vec2<float>, q16c>(const DslashArgs<float, vec2<float>, q16c> &,
                                                            const DslashShape &, bool, bool, bool,
                                                            hipStream_t);
template hisq_status launch_march<float, vec2<float>, vec2<float>>(
    const DslashArgs<float, vec2<float>, vec2<float>> &, const DslashShape &, bool, bool, bool,
    hipStream_t);
}  // namespace dslash_impl
}  // namespace hisq
