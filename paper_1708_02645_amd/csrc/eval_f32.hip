// Store and value-only evaluation kernels for SPL_F32 tables, one per tile shape.
#include "shapes.hpp"

namespace qs {

QS_REGISTRY(variants_f32, QS_SHAPES_F32, QS_EVAL_VARIANTS, SPL_F32)

}  // namespace qs
