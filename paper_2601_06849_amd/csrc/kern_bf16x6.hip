// The stage, adjoint and batch kernels and their host drivers instantiated
// for one mode-product precision: Bf16x6Mma.
#include "library.hpp"

namespace etdds {

const PrecisionOps& ops_bf16x6() {
    static const PrecisionOps ops = make_ops<Bf16x6Mma>();
    return ops;
}

}  // namespace etdds
