// Determinant-ratio evaluation kernels for SPL_F32 tables, one per tile shape.
#include "shapes.hpp"

namespace qs {

QS_REGISTRY(ratio_variants_f32, QS_SHAPES_F32, QS_RATIO_VARIANTS, SPL_F32)

}  // namespace qs
