// Value-gradient-Hessian and general-cell VGL kernels for SPL_F32 tables, one per tile shape.
#include "vgh_kernel.hpp"

namespace qs {

QS_VGH_REGISTRY(vgh_variants_f32, QS_VGH_SHAPES_F32, SPL_F32)

}  // namespace qs
