// Value-gradient-Hessian and general-cell VGL kernels for SPL_F16 tables, one per tile shape.
#include "vgh_kernel.hpp"

namespace qs {

QS_VGH_REGISTRY(vgh_variants_f16, QS_VGH_SHAPES_16, SPL_F16)

}  // namespace qs
