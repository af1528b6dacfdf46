// Store and value-only evaluation kernels for SPL_BF16 tables, one per tile shape.
#include "shapes.hpp"

namespace qs {

QS_REGISTRY(variants_bf16, QS_SHAPES_16, QS_EVAL_VARIANTS, SPL_BF16)

}  // namespace qs
