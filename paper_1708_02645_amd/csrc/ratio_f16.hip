// Determinant-ratio evaluation kernels for SPL_F16 tables, one per tile shape.
#include "shapes.hpp"

namespace qs {

QS_REGISTRY(ratio_variants_f16, QS_SHAPES_16, QS_RATIO_VARIANTS, SPL_F16)

}  // namespace qs
