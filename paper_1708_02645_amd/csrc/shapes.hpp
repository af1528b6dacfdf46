// Tile shapes (cw, nch, lpp) compiled for each storage type, as X-macro
// lists, and the registry entries a shape expands to.  The evaluation files
// (eval_*.hip) instantiate the store and value-only kernels, the ratio files
// (ratio_*.hip) the determinant-ratio kernels, of the same shapes.
#pragma once

#include "eval_kernel.hpp"

#define QS_SHAPES_F64(X, ST)                                                              \
    X(ST, 2, 1, 64) X(ST, 2, 2, 64) X(ST, 2, 3, 64) X(ST, 4, 1, 64) X(ST, 4, 2, 64)        \
    X(ST, 2, 1, 32) X(ST, 4, 1, 32) X(ST, 4, 2, 32) X(ST, 2, 1, 16) X(ST, 2, 2, 16)        \
    X(ST, 4, 1, 16) X(ST, 4, 2, 16)

#define QS_SHAPES_F32(X, ST)                                                              \
    X(ST, 1, 1, 64) X(ST, 1, 2, 64) X(ST, 1, 3, 64) X(ST, 1, 4, 64) X(ST, 1, 6, 64)        \
    X(ST, 2, 1, 64) X(ST, 2, 2, 64) X(ST, 2, 3, 64) X(ST, 3, 1, 64) X(ST, 3, 2, 64)        \
    X(ST, 4, 1, 64) X(ST, 4, 2, 64) X(ST, 1, 2, 32) X(ST, 2, 1, 32) X(ST, 2, 2, 32)        \
    X(ST, 3, 1, 32) X(ST, 4, 1, 32) X(ST, 4, 2, 32) X(ST, 2, 1, 16) X(ST, 4, 1, 16)        \
    X(ST, 4, 2, 16) X(ST, 1, 1, 16) X(ST, 3, 1, 16)

// BF16 and FP16
#define QS_SHAPES_16(X, ST)                                                               \
    X(ST, 1, 1, 64) X(ST, 1, 2, 64) X(ST, 1, 3, 64) X(ST, 2, 1, 64) X(ST, 2, 2, 64)        \
    X(ST, 2, 3, 64) X(ST, 3, 1, 64) X(ST, 3, 2, 64) X(ST, 4, 1, 64) X(ST, 2, 1, 32)        \
    X(ST, 3, 1, 32) X(ST, 4, 1, 32) X(ST, 4, 2, 32) X(ST, 2, 1, 16) X(ST, 4, 1, 16)        \
    X(ST, 4, 2, 16) X(ST, 1, 1, 16) X(ST, 3, 1, 16)

#define QS_EVAL_VARIANTS(ST, CW, NCH, LPP)                                                \
    {ST, CW, NCH, LPP, true, false, (const void*)&eval_kernel<ST, CW, NCH, LPP, true>,     \
     (const void*)&plan_kernel<ST, CW, NCH, LPP>, sizeof(PosW<Acc<ST>::type>), 0},         \
    {ST, CW, NCH, LPP, false, false, (const void*)&eval_kernel<ST, CW, NCH, LPP, false>,   \
     nullptr, sizeof(PosW<Acc<ST>::type>), 0},

#define QS_RATIO_VARIANTS(ST, CW, NCH, LPP)                                               \
    {ST, CW, NCH, LPP, true, true, (const void*)&eval_kernel<ST, CW, NCH, LPP, true, true>, \
     nullptr, sizeof(PosW<Acc<ST>::type>), 5 * sizeof(Acc<ST>::type)},                     \
    {ST, CW, NCH, LPP, false, true, (const void*)&eval_kernel<ST, CW, NCH, LPP, false, true>, \
     nullptr, sizeof(PosW<Acc<ST>::type>), sizeof(Acc<ST>::type)},

// Defines `const Variant* NAME(int* count)` over the list LIST for type ST.
#define QS_REGISTRY(NAME, LIST, KIND, ST)                                                 \
    static const Variant k_variants[] = {LIST(KIND, ST)};                                 \
    const Variant* NAME(int* count)                                                       \
    {                                                                                     \
        *count = (int)(sizeof(k_variants) / sizeof(k_variants[0]));                       \
        return k_variants;                                                                \
    }
