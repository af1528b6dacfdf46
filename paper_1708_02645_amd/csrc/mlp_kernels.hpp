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

// Position of element i of a row-major [M][K] weight matrix (M a multiple
// of 16, K of 32) in its BF16 copy, which is kept in matrix-core fragment
// order: fragment (b, t) -- rows 16b..16b+15, columns 32t..32t+31 -- is 512
// consecutive values, b-major, in which lane 16g+c of a wave finds its A
// operand (row 16b+c, columns 32t+8g..+7) as 8 consecutive values, so one
// wave loads a fragment as one contiguous 1 KB block.
__host__ __device__ inline int64_t frag_index(int64_t i, int K)
{
    const int64_t r = i / K;
    const int k = (int)(i - r * K);
    const int64_t blk = r >> 4;
    const int c = (int)(r & 15), t = k >> 5, g = (k >> 3) & 3, j = k & 7;
    return (blk * (K >> 5) + t) * 512 + (16 * g + c) * 8 + j;
}

struct MlpFwdArgs {
    const double* pos;    // [B][3]
    int64_t B;
    const int32_t* freqs;  // [kFreq][3]
    double cell[3];
    double icell[3];       // 1 / cell
    double tpc[3];         // 2 pi / cell
    const __bf16* Wh;      // BF16 weights in fragment order (hW1, hW2, hW3 offsets)
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

// Launches the fused evaluation kernel (mlp_forward.hip) on a.B positions.
int launch_mlp_forward(const MlpFwdArgs& a, hipStream_t stream);

// SiLU x*s and its first two (three) derivatives, s = 1/(1 + e^-x) (the
// hardware reciprocal, 1 ulp).
__device__ inline float sigmoid(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }

__device__ inline float silu3(float x, float& d1, float& d2)
{
    const float s = sigmoid(x);
    const float oms = 1.0f - s;
    d1 = s * (1.0f + x * oms);
    d2 = s * oms * (2.0f + x * (1.0f - 2.0f * s));
    return x * s;
}

__device__ inline float silu4(float x, float& d1, float& d2, float& d3)
{
    const float s = sigmoid(x);
    const float oms = 1.0f - s;
    d1 = s * (1.0f + x * oms);
    d2 = s * oms * (2.0f + x * (1.0f - 2.0f * s));
    d3 = s * oms * (3.0f * (1.0f - 2.0f * s) + x * (1.0f - 6.0f * s + 6.0f * s * s));
    return x * s;
}

// One feature column k (0..2F-1) of one position, for the five streams:
// sin(2 pi k.u) for k < F, cos for k >= F; u = r / cell.  The phase k.u is
// reduced modulo 1 in FP64; the hardware sine/cosine take the angle in
// revolutions.
__device__ inline void feature5(const int32_t* freqs, const double* u, const double* cell, int k, float* out)
{
    const int f = k < kFreq ? k : k - kFreq;
    const int kx = freqs[3 * f], ky = freqs[3 * f + 1], kz = freqs[3 * f + 2];
    double x = (double)kx * u[0] + (double)ky * u[1] + (double)kz * u[2];
    x -= floor(x);
    const float s = __builtin_amdgcn_sinf((float)x);
    const float c = __builtin_amdgcn_cosf((float)x);
    const float gx = (float)(6.283185307179586 * kx / cell[0]);
    const float gy = (float)(6.283185307179586 * ky / cell[1]);
    const float gz = (float)(6.283185307179586 * kz / cell[2]);
    const float g2 = gx * gx + gy * gy + gz * gz;
    const float val = k < kFreq ? s : c;
    const float dv = k < kFreq ? c : -s;
    out[0] = val;
    out[1] = dv * gx;
    out[2] = dv * gy;
    out[3] = dv * gz;
    out[4] = -g2 * val;
}

}  // namespace qs
