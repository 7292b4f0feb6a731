// The time-marching half stencil (dslash_march.h) for 16-bit vectors and links.
#include "dslash_march.h"

namespace hisq {
namespace dslash_impl {
template hisq_status launch_march<float, h16p, q16s>(const DslashArgs<float, h16p, q16s> &,
                                                     const DslashShape &, bool, bool, bool,
                                                     hipStream_t);
}  // namespace dslash_impl
}  // namespace hisq
