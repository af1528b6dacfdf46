// Value-gradient-Hessian and general-cell VGL kernels for SPL_BF16 tables, one per tile shape.
#include "vgh_kernel.hpp"

namespace qs {

QS_VGH_REGISTRY(vgh_variants_bf16, QS_VGH_SHAPES_16, SPL_BF16)

}  // namespace qs
