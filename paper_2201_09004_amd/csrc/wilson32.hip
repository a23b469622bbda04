// FP32 instantiations of the Wilson-type stencil (templates in wilson_impl.h).
#include "wilson_impl.h"

namespace lq {

template int launch_wilson_prec<32>(const WilsonArgs& A, int nr, int bs, hipStream_t s);

}  // namespace lq
