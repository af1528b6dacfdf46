// Kernels of the surrogate network: a periodic Fourier-feature MLP whose
// value, gradient and Laplacian are carried in forward mode (five streams:
// value, d/dx, d/dy, d/dz, Laplacian) through BF16 matrix-core products with
// FP32 accumulation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Network shape compiled into the kernels: 2*kFreq features, two hidden
// layers of kHidden units, up to kMaxOut outputs (a multiple of 16).
constexpr int kFreq = 48;
constexpr int kIn = 2 * kFreq;  // 96
constexpr int kHidden = 256;
constexpr int kMaxOut = 256;
constexpr int kStreams = 5;

// Flat FP32 parameter vector: W1 [H][96], b1 [H], W2 [H][H], b2 [H],
// W3 [N][H], b3 [N] (weights stored [out][in]).
struct MlpOffsets {
    int64_t W1, b1, W2, b2, W3, b3, total;
    int64_t hW1, hW2, hW3, htotal;  // BF16 copies of the weights
};

__host__ __device__ inline MlpOffsets mlp_offsets(int nout)
{
    MlpOffsets o;
    o.W1 = 0;
    o.b1 = o.W1 + (int64_t)kHidden * kIn;
    o.W2 = o.b1 + kHidden;
    o.b2 = o.W2 + (int64_t)kHidden * kHidden;
    o.W3 = o.b2 + kHidden;
    o.b3 = o.W3 + (int64_t)nout * kHidden;
    o.total = o.b3 + nout;
    o.hW1 = 0;
    o.hW2 = o.hW1 + (int64_t)kHidden * kIn;
    o.hW3 = o.hW2 + (int64_t)kHidden * kHidden;
    o.htotal = o.hW3 + (int64_t)nout * kHidden;
    return o;
}

struct MlpFwdArgs {
    const double* pos;    // [B][3]
    int64_t B;
    const int32_t* freqs;  // [kFreq][3]
    double cell[3];
    const __bf16* Wh;      // BF16 weights (hW1, hW2, hW3 offsets)
    const float* P;        // FP32 parameters (biases)
    const float* mu;       // [nout]
    const float* sd;       // [nout]
    float* V;              // [B][nout]
    float* G;              // [B][3][nout]
    float* L;              // [B][nout]
    int32_t nout;
};

// Generic matrix product for training: C = A B (+ bias on the first
// bias_rows rows), A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn],
// FP32 operands rounded to BF16 when staged, FP32 accumulation.  blockIdx.z
// selects a K chunk; chunk z writes C + z*split_stride.
struct GemmArgs {
    const float* A;
    int64_t sam, sak;
    const float* B;
    int64_t sbk, sbn;
    float* C;
    int64_t ldc;
    const float* bias;
    int32_t bias_rows;
    int32_t M, N, K;
    int32_t kchunk;
    int64_t split_stride;
};

}  // namespace qs
