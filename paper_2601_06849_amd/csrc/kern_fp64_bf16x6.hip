// The stage, adjoint and batch kernels and their host drivers instantiated
// for one mode-product precision: Bf16x6MmaOn<double> (FP64 state,
// split-BF16 products).
#include "library.hpp"

namespace etdds {

const PrecisionOps& ops_fp64_bf16x6() {
    static const PrecisionOps ops = make_ops<Bf16x6MmaOn<double>>();
    return ops;
}

}  // namespace etdds
