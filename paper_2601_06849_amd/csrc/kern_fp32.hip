// The stage, adjoint and batch kernels and their host drivers instantiated
// for one mode-product precision: NativeMma<float>.
#include "library.hpp"

namespace etdds {

const PrecisionOps& ops_fp32() {
    static const PrecisionOps ops = make_ops<NativeMma<float>>();
    return ops;
}

}  // namespace etdds
