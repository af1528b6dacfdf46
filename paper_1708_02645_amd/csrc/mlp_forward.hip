// Fused forward-mode evaluation of the surrogate network on the matrix cores
// (gfx950, v_mfma_f32_16x16x32_bf16, BF16 operands, FP32 accumulation).
//
// One wave evaluates 16 positions through all layers.  Operand layout of
// the instruction (lane l, g = l/16, c = l%16): A[c][8g..8g+7],
// B[8g..8g+7][c], C[4g..4g+3][c].  Each layer is computed transposed,
// H^T[unit][pos] = sum_k W[unit][k] Act[pos][k]: the weight rows are the A
// operand (read from global memory, 280 KB in all, L2-resident) and the
// layer input, held in registers for all K, is the B operand.  Each stream
// (value, d/dx, d/dy, d/dz, Laplacian) is its own product, so the five
// accumulators of a (unit, position) pair sit in the same lane and slot and
// the forward-mode SiLU combines them in registers.  A lane then holds four
// consecutive units of one position, which it writes to LDS with one 8-byte
// store per stream (a [stream][16][256] BF16 tile, 16-byte chunks XOR-swizzled
// by row), to be read back as the next layer's B operands.
//
// Output units are processed in groups of 64 with two accumulator sets: the
// epilogue of group k follows the first products of group k+1, so the vector
// ALU work of one overlaps the matrix-core work of the other, and weight
// fragments are loaded four steps ahead of their use.
#include "mlp_kernels.hpp"

#include "common.hpp"

namespace qs {

typedef float f32x4v __attribute__((ext_vector_type(4)));

__device__ inline int zoff(int s, int row, int col)
{
    return ((s * 16 + row) * kHidden + ((((col >> 3) ^ (row & 7)) << 3) | (col & 7)));
}

// A layer of NCG groups of 64 output units (4 blocks of 16) over KSTEPS
// steps of 32 inputs, as one unrolled sequence of NCG*KSTEPS steps; `blocks`
// clamps the weight rows of a partial last group (never stored).  The
// weight fragments of step i+4 are loaded while step i runs (a ring of five,
// across group boundaries), and the epilogue of group k is placed after the
// first products of group k+1 (two accumulator sets), so that loads, matrix
// products and vector work of neighbouring groups overlap.
template <int KSTEPS, int NCG, class Epi>
__device__ inline void layer(const bf16x8 (&X)[kStreams][KSTEPS], const __bf16* __restrict__ W, int blocks, int g,
                             int c, const Epi& epi)
{
    constexpr int K = 32 * KSTEPS;
    constexpr int S = NCG * KSTEPS;
    auto load = [&](int step, bf16x8 (&dst)[4]) {
        const int cg = step / KSTEPS, t = step % KSTEPS;
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int blk = cg * 4 + nb < blocks ? cg * 4 + nb : blocks - 1;
            dst[nb] = *reinterpret_cast<const bf16x8*>(W + (int64_t)(blk * 16 + c) * K + 32 * t + 8 * g);
        }
    };
    constexpr int R = 5;  // ring depth: fragments of step i+R-1 are loaded at step i
    bf16x8 ring[R][4];
#pragma unroll
    for (int i = 0; i < R - 1; ++i)
        if (i < S) load(i, ring[i]);
    f32x4 acc[2][kStreams][4];
    // fully unrolled: every register-array index below must be a constant
#pragma clang loop unroll(full)
    for (int step = 0; step < S; ++step) {
        const int cg = step / KSTEPS, t = step % KSTEPS;
        if (step + R - 1 < S) load(step + R - 1, ring[(step + R - 1) % R]);
        if (t == 0) {
#pragma unroll
            for (int s = 0; s < kStreams; ++s)
#pragma unroll
                for (int nb = 0; nb < 4; ++nb) acc[cg & 1][s][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int s = 0; s < kStreams; ++s)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                acc[cg & 1][s][nb] =
                    __builtin_amdgcn_mfma_f32_16x16x32_bf16(ring[step % R][nb], X[s][t], acc[cg & 1][s][nb], 0, 0, 0);
        if (t == 0 && cg >= 1) epi(cg - 1, acc[(cg - 1) & 1]);
    }
    epi(NCG - 1, acc[(NCG - 1) & 1]);
}

// Hidden layer epilogue: bias, forward-mode SiLU, BF16 into the LDS tile.
struct HiddenEpi {
    const float* bias;
    __bf16* zb;
    int g, c;
    __device__ void operator()(int cg, const f32x4 (&acc)[kStreams][4]) const
    {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int u0 = cg * 64 + nb * 16 + 4 * g;
            const f32x4v b = *reinterpret_cast<const f32x4v*>(bias + u0);
            __bf16 z[kStreams][4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float hv = acc[0][nb][j] + b[j];
                const float hx = acc[1][nb][j], hy = acc[2][nb][j], hz = acc[3][nb][j], hl = acc[4][nb][j];
                float d1, d2;
                z[0][j] = (__bf16)silu3(hv, d1, d2);
                z[1][j] = (__bf16)(d1 * hx);
                z[2][j] = (__bf16)(d1 * hy);
                z[3][j] = (__bf16)(d1 * hz);
                z[4][j] = (__bf16)(d1 * hl + d2 * (hx * hx + hy * hy + hz * hz));
            }
#pragma unroll
            for (int s = 0; s < kStreams; ++s) {
                uint64_t packed;
                __builtin_memcpy(&packed, z[s], 8);
                *reinterpret_cast<uint64_t*>(zb + zoff(s, c, u0)) = packed;
            }
        }
    }
};

// Output epilogue: bias and the per-orbital affine map; 16-byte stores of
// four consecutive orbitals of one position to V, G, L.
struct OutEpi {
    const MlpFwdArgs* a;
    const float* b3;
    int64_t b0;
    int blocks, g, c;
    __device__ void operator()(int cg, const f32x4 (&acc)[kStreams][4]) const
    {
        const int64_t b = b0 + c;
        if (b >= a->B) return;
        const int N = a->nout;
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            if (cg * 4 + nb >= blocks) continue;
            const int n0 = (cg * 4 + nb) * 16 + 4 * g;
            const f32x4v sd = *reinterpret_cast<const f32x4v*>(a->sd + n0);
            const f32x4v mu = *reinterpret_cast<const f32x4v*>(a->mu + n0);
            const f32x4v bb = *reinterpret_cast<const f32x4v*>(b3 + n0);
            f32x4v v, gx, gy, gz, l;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[j] = (acc[0][nb][j] + bb[j]) * sd[j] + mu[j];
                gx[j] = acc[1][nb][j] * sd[j];
                gy[j] = acc[2][nb][j] * sd[j];
                gz[j] = acc[3][nb][j] * sd[j];
                l[j] = acc[4][nb][j] * sd[j];
            }
            *reinterpret_cast<f32x4v*>(a->V + b * N + n0) = v;
            *reinterpret_cast<f32x4v*>(a->G + (3 * b + 0) * N + n0) = gx;
            *reinterpret_cast<f32x4v*>(a->G + (3 * b + 1) * N + n0) = gy;
            *reinterpret_cast<f32x4v*>(a->G + (3 * b + 2) * N + n0) = gz;
            *reinterpret_cast<f32x4v*>(a->L + b * N + n0) = l;
        }
    }
};

__device__ inline void load_x(bf16x8 (&X)[kStreams][kHidden / 32], const __bf16* zb, int g, int c)
{
#pragma unroll
    for (int s = 0; s < kStreams; ++s)
#pragma unroll
        for (int t = 0; t < kHidden / 32; ++t)
            X[s][t] = *reinterpret_cast<const bf16x8*>(zb + zoff(s, c, 32 * t + 8 * g));
}

template <int NCG_OUT>
__global__ __launch_bounds__(64) void mlp_vgl_kernel(MlpFwdArgs a)
{
    __shared__ __attribute__((aligned(16))) __bf16 zb[kStreams * 16 * kHidden];
    const int l = threadIdx.x, g = l >> 4, c = l & 15;
    const int64_t b0 = (int64_t)blockIdx.x * 16;
    const MlpOffsets o = mlp_offsets(a.nout);

    // Per-frequency constants, once per workgroup: the integer frequency and
    // its Cartesian factors 2 pi k_d / cell_d and their squared norm.  They
    // live at the start of the activation tile, which the first layer's
    // epilogue overwrites only after the features are in registers (and
    // after the barrier below), so the workgroup's LDS stays at one tile.
    int32_t (*fk)[3] = reinterpret_cast<int32_t (*)[3]>(zb);
    float (*fg)[4] = reinterpret_cast<float (*)[4]>(reinterpret_cast<unsigned char*>(zb) + kFreq * 3 * 4);
    if (l < kFreq) {
        float g2 = 0.f;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int k = a.freqs[3 * l + d];
            fk[l][d] = k;
            const float gd = (float)(6.283185307179586 * k / a.cell[d]);
            fg[l][d] = gd;
            g2 += gd * gd;
        }
        fg[l][3] = g2;
    }
    __syncthreads();

    // Layer-1 operands: the features of position b0 + c.  Phase k.u reduced
    // modulo 1 in FP64; the hardware sine/cosine take revolutions.
    int64_t bi = b0 + c;
    if (bi >= a.B) bi = a.B - 1;  // ragged tail: computed, never stored
    double u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = a.pos[3 * bi + d] * (1.0 / a.cell[d]);
    bf16x8 X1[kStreams][3];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 32 * t + 8 * g + j;
            const int fi = k < kFreq ? k : k - kFreq;
            double x = (double)fk[fi][0] * u[0] + (double)fk[fi][1] * u[1] + (double)fk[fi][2] * u[2];
            x -= floor(x);
            const float sn = __builtin_amdgcn_sinf((float)x), cs = __builtin_amdgcn_cosf((float)x);
            const float val = k < kFreq ? sn : cs, dv = k < kFreq ? cs : -sn;
            X1[0][t][j] = (__bf16)val;
            X1[1][t][j] = (__bf16)(dv * fg[fi][0]);
            X1[2][t][j] = (__bf16)(dv * fg[fi][1]);
            X1[3][t][j] = (__bf16)(dv * fg[fi][2]);
            X1[4][t][j] = (__bf16)(-fg[fi][3] * val);
        }

    __syncthreads();  // every lane's features are in registers before the tile is written
    layer<3, kHidden / 64>(X1, a.Wh + o.hW1, kHidden / 16, g, c, HiddenEpi{a.P + o.b1, zb, g, c});
    __syncthreads();
    bf16x8 X[kStreams][kHidden / 32];
    load_x(X, zb, g, c);
    __syncthreads();
    layer<kHidden / 32, kHidden / 64>(X, a.Wh + o.hW2, kHidden / 16, g, c, HiddenEpi{a.P + o.b2, zb, g, c});
    __syncthreads();
    load_x(X, zb, g, c);
    const int nblk = a.nout / 16;
    layer<kHidden / 32, NCG_OUT>(X, a.Wh + o.hW3, nblk, g, c, OutEpi{&a, a.P + o.b3, b0, nblk, g, c});
}

int launch_mlp_forward(const MlpFwdArgs& a, hipStream_t st)
{
    const int64_t blocks = (a.B + 15) / 16;
    if (blocks > 0x7fffffff) return fail(SPL_EINVAL, "batch too large");
    const int ncg = (a.nout / 16 + 3) / 4;
    switch (ncg) {
    case 1: hipLaunchKernelGGL(mlp_vgl_kernel<1>, dim3((unsigned)blocks), dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL(mlp_vgl_kernel<2>, dim3((unsigned)blocks), dim3(64), 0, st, a); break;
    case 3: hipLaunchKernelGGL(mlp_vgl_kernel<3>, dim3((unsigned)blocks), dim3(64), 0, st, a); break;
    case 4: hipLaunchKernelGGL(mlp_vgl_kernel<4>, dim3((unsigned)blocks), dim3(64), 0, st, a); break;
    default: return fail(SPL_EUNSUPPORTED, "output width out of range");
    }
    QS_HIP(hipGetLastError());
    return SPL_OK;
}

}  // namespace qs
