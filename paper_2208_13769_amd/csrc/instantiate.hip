// instantiate.hip -- the kernels and launch helpers of one precision.
//
// Built once per precision with LBM_PREC naming the precision traits
// (PrecF64, PrecF32, PrecF32U64, PrecF16 or PrecBF16), so the five
// precisions' step kernels compile in parallel; the runtime sources only
// declare these instantiations.
#include "general_kernels.hpp"
#include "host_common.hpp"

namespace lbm {

template struct Kernels<LBM_PREC>;
template hipError_t general_step<LBM_PREC>(GenParams, char *, hipStream_t);

}  // namespace lbm
