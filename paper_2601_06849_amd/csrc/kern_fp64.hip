// The stage, adjoint and batch kernels and their host drivers instantiated
// for one mode-product precision: NativeMma<double>.
#include "library.hpp"

namespace etdds {

const PrecisionOps& ops_fp64() {
    static const PrecisionOps ops = make_ops<NativeMma<double>>();
    return ops;
}

}  // namespace etdds
