// Compiled tile shapes of the evaluation kernels for BF16 tables (generated list;
// edit here and in the registry together).
#include "eval_kernel.hpp"

namespace qs {

#define QS_VARIANT(CW, NCH, LPP)                                                          \
    {SPL_BF16, CW, NCH, LPP, true, (const void*)&eval_kernel<SPL_BF16, CW, NCH, LPP, true>,          \
     (const void*)&plan_kernel<SPL_BF16, CW, NCH, LPP>, sizeof(PosW<Acc<SPL_BF16>::type>)},            \
    {SPL_BF16, CW, NCH, LPP, false, (const void*)&eval_kernel<SPL_BF16, CW, NCH, LPP, false>,        \
     nullptr, sizeof(PosW<Acc<SPL_BF16>::type>)},

static const Variant k_variants[] = {
    QS_VARIANT(1, 1, 64)
    QS_VARIANT(1, 2, 64)
    QS_VARIANT(1, 3, 64)
    QS_VARIANT(2, 1, 64)
    QS_VARIANT(2, 2, 64)
    QS_VARIANT(2, 3, 64)
    QS_VARIANT(3, 1, 64)
    QS_VARIANT(3, 2, 64)
    QS_VARIANT(4, 1, 64)
    QS_VARIANT(2, 1, 32)
    QS_VARIANT(3, 1, 32)
    QS_VARIANT(4, 1, 32)
    QS_VARIANT(4, 2, 32)
    QS_VARIANT(2, 1, 16)
    QS_VARIANT(4, 1, 16)
    QS_VARIANT(4, 2, 16)
};

const Variant* variants_bf16(int* count)
{
    *count = (int)(sizeof(k_variants) / sizeof(k_variants[0]));
    return k_variants;
}

}  // namespace qs
