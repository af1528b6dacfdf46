// Value-gradient-Hessian and general-cell VGL kernels for SPL_F64 tables, one per tile shape.
#include "vgh_kernel.hpp"

namespace qs {

QS_VGH_REGISTRY(vgh_variants_f64, QS_VGH_SHAPES_F64, SPL_F64)

}  // namespace qs
