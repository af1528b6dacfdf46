// Store and value-only evaluation kernels for SPL_F64 tables, one per tile shape.
#include "shapes.hpp"

namespace qs {

QS_REGISTRY(variants_f64, QS_SHAPES_F64, QS_EVAL_VARIANTS, SPL_F64)

}  // namespace qs
