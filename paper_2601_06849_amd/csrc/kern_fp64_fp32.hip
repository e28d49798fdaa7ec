// The stage, adjoint and batch kernels and their host drivers instantiated
// for one mode-product precision: F64F32Mma (FP64 state, FP32 products).
#include "library.hpp"

namespace etdds {

const PrecisionOps& ops_fp64_fp32() {
    static const PrecisionOps ops = make_ops<F64F32Mma>();
    return ops;
}

}  // namespace etdds
