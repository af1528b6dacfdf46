// Determinant-ratio evaluation kernels for SPL_F64 tables, one per tile shape.
#include "shapes.hpp"

namespace qs {

QS_REGISTRY(ratio_variants_f64, QS_SHAPES_F64, QS_RATIO_VARIANTS, SPL_F64)

}  // namespace qs
