// Surrogate-network kernels for gfx950: the fused forward-mode evaluation
// (matrix cores, BF16 operands, FP32 accumulation) and the training kernels
// (features, generic BF16 matrix product, SiLU streams forward/backward,
// Sobolev loss, gradient reductions, Adam), plus the error map and the
// routing of positions to the spline fallback.
#include "mlp_kernels.hpp"

#include "common.hpp"

namespace qs {

constexpr float kTwoPi = 6.283185307179586f;

// SiLU x*s and its first two derivatives, s = 1/(1 + e^-x).
__device__ inline float silu3(float x, float& d1, float& d2)
{
    const float s = 1.0f / (1.0f + __expf(-x));
    const float oms = 1.0f - s;
    d1 = s * (1.0f + x * oms);
    d2 = s * oms * (2.0f + x * (1.0f - 2.0f * s));
    return x * s;
}

__device__ inline float silu4(float x, float& d1, float& d2, float& d3)
{
    const float s = 1.0f / (1.0f + __expf(-x));
    const float oms = 1.0f - s;
    d1 = s * (1.0f + x * oms);
    d2 = s * oms * (2.0f + x * (1.0f - 2.0f * s));
    d3 = s * oms * (3.0f * (1.0f - 2.0f * s) + x * (1.0f - 6.0f * s + 6.0f * s * s));
    return x * s;
}

// One feature column k (0..2F-1) of one position, for the five streams:
// sin(2 pi k.u) for k < F, cos for k >= F; u = r / cell.
__device__ inline void feature5(const int32_t* freqs, const double* u, const double* cell, int k, float* out)
{
    const int f = k < kFreq ? k : k - kFreq;
    const int kx = freqs[3 * f], ky = freqs[3 * f + 1], kz = freqs[3 * f + 2];
    double x = (double)kx * u[0] + (double)ky * u[1] + (double)kz * u[2];
    x -= floor(x);
    // hardware sine/cosine take the angle in revolutions: sin(2 pi x), x in [0, 1)
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

// ---------------------------------------------------------------------------
// Fused forward-mode evaluation: one wave evaluates 16 positions through all
// layers.  Operand layout of v_mfma_f32_16x16x32_bf16 (lane l, g = l/16,
// c = l%16): A[c][8g..8g+7], B[8g..8g+7][c], C[4g..4g+3][c].  Rows are the
// 16 positions, one product per stream, so the five accumulators of a
// (position, unit) pair sit in the same lane and slot and the SiLU streams
// are combined in registers.  The layer input lives in registers (A
// operands, all K); each layer's output is written once to LDS (a
// [stream][16][256] BF16 tile with an XOR swizzle of 16-byte chunks) and read
// back in A layout for the next layer.  Weights are read straight from
// global memory (280 KB, L2-resident) as B operands.

__device__ inline int zoff(int s, int row, int col)
{
    return ((s * 16 + row) * kHidden + ((((col >> 3) ^ (row & 7)) << 3) | (col & 7)));
}

// One layer on the matrix cores: ncg groups of 64 output columns (4 blocks
// of 16), KSTEPS steps of 32 inputs, five streams.  The B operands (weights,
// [out][in] rows of K BF16) of the next step are loaded while the current
// step's products run, across group boundaries too.  `blocks` clamps the
// column blocks of the last group (output layer); their results are unused.
template <int KSTEPS, class Epi>
__device__ inline void mfma_layer(const bf16x8 (&A)[kStreams][KSTEPS], const __bf16* __restrict__ W, int ncg,
                                  int blocks, int g, int c, Epi&& epi)
{
    constexpr int K = 32 * KSTEPS;
    auto loadB = [&](int cg, int t, bf16x8 (&dst)[4]) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            const int blk = cg * 4 + nb < blocks ? cg * 4 + nb : blocks - 1;
            dst[nb] = *reinterpret_cast<const bf16x8*>(W + (int64_t)(blk * 16 + c) * K + 32 * t + 8 * g);
        }
    };
    bf16x8 cur[4], nxt[4];
    loadB(0, 0, cur);
#pragma unroll 1
    for (int cg = 0; cg < ncg; ++cg) {
        f32x4 acc[kStreams][4];
#pragma unroll
        for (int s = 0; s < kStreams; ++s)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) acc[s][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < KSTEPS; ++t) {
            if (t + 1 < KSTEPS) loadB(cg, t + 1, nxt);
            else if (cg + 1 < ncg) loadB(cg + 1, 0, nxt);
#pragma unroll
            for (int s = 0; s < kStreams; ++s)
#pragma unroll
                for (int nb = 0; nb < 4; ++nb)
                    acc[s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[s][t], cur[nb], acc[s][nb], 0, 0, 0);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) cur[nb] = nxt[nb];
        }
        epi(cg, acc);
    }
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
            const int col = cg * 64 + nb * 16 + c;
            const float b = bias[col];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = 4 * g + j;
                const float hv = acc[0][nb][j] + b;
                const float hx = acc[1][nb][j], hy = acc[2][nb][j], hz = acc[3][nb][j], hl = acc[4][nb][j];
                float d1, d2;
                const float zv = silu3(hv, d1, d2);
                zb[zoff(0, row, col)] = (__bf16)zv;
                zb[zoff(1, row, col)] = (__bf16)(d1 * hx);
                zb[zoff(2, row, col)] = (__bf16)(d1 * hy);
                zb[zoff(3, row, col)] = (__bf16)(d1 * hz);
                zb[zoff(4, row, col)] = (__bf16)(d1 * hl + d2 * (hx * hx + hy * hy + hz * hz));
            }
        }
    }
};

// Output epilogue: bias and the per-orbital affine map, stores to V, G, L.
struct OutEpi {
    const MlpFwdArgs* a;
    const float* b3;
    int64_t b0;
    int blocks, g, c;
    __device__ void operator()(int cg, const f32x4 (&acc)[kStreams][4]) const
    {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            if (cg * 4 + nb >= blocks) continue;
            const int n = (cg * 4 + nb) * 16 + c;
            const float sd = a->sd[n], mu = a->mu[n], bb = b3[n];
            const int N = a->nout;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t b = b0 + 4 * g + j;
                if (b >= a->B) continue;
                a->V[b * N + n] = (acc[0][nb][j] + bb) * sd + mu;
                a->G[(3 * b + 0) * N + n] = acc[1][nb][j] * sd;
                a->G[(3 * b + 1) * N + n] = acc[2][nb][j] * sd;
                a->G[(3 * b + 2) * N + n] = acc[3][nb][j] * sd;
                a->L[b * N + n] = acc[4][nb][j] * sd;
            }
        }
    }
};

__device__ inline void load_a(bf16x8 (&A)[kStreams][kHidden / 32], const __bf16* zb, int g, int c)
{
#pragma unroll
    for (int s = 0; s < kStreams; ++s)
#pragma unroll
        for (int t = 0; t < kHidden / 32; ++t)
            A[s][t] = *reinterpret_cast<const bf16x8*>(zb + zoff(s, c, 32 * t + 8 * g));
}

__global__ __launch_bounds__(64) void mlp_vgl_kernel(MlpFwdArgs a)
{
    __shared__ __attribute__((aligned(16))) __bf16 zb[kStreams * 16 * kHidden];
    const int l = threadIdx.x, g = l >> 4, c = l & 15;
    const int64_t b0 = (int64_t)blockIdx.x * 16;
    const MlpOffsets o = mlp_offsets(a.nout);

    // Layer-1 operands: the features of position b0 + c, in A layout.
    int64_t bi = b0 + c;
    if (bi >= a.B) bi = a.B - 1;  // ragged tail: computed, never stored
    double u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = a.pos[3 * bi + d] / a.cell[d];
    bf16x8 A1[kStreams][3];
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float f[5];
            feature5(a.freqs, u, a.cell, 32 * t + 8 * g + j, f);
#pragma unroll
            for (int s = 0; s < kStreams; ++s) A1[s][t][j] = (__bf16)f[s];
        }

    mfma_layer<3>(A1, a.Wh + o.hW1, kHidden / 64, kHidden / 16, g, c, HiddenEpi{a.P + o.b1, zb, g, c});
    __syncthreads();
    bf16x8 A2[kStreams][kHidden / 32];
    load_a(A2, zb, g, c);
    __syncthreads();
    mfma_layer<kHidden / 32>(A2, a.Wh + o.hW2, kHidden / 64, kHidden / 16, g, c, HiddenEpi{a.P + o.b2, zb, g, c});
    __syncthreads();
    load_a(A2, zb, g, c);
    const int nblk = a.nout / 16;
    mfma_layer<kHidden / 32>(A2, a.Wh + o.hW3, (nblk + 3) / 4, nblk, g, c, OutEpi{&a, a.P + o.b3, b0, nblk, g, c});
}

// ---------------------------------------------------------------------------
// Training kernels.  Stream-major activations: X[s][B][width], FP32.

__global__ void mlp_features_kernel(const double* pos, int64_t B, const int32_t* freqs, double c0, double c1,
                                    double c2, float* X)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * kIn) return;
    const int64_t b = i / kIn;
    const int k = (int)(i - b * kIn);
    const double cell[3] = {c0, c1, c2};
    double u[3];
    for (int d = 0; d < 3; ++d) u[d] = pos[3 * b + d] / cell[d];
    float f[5];
    feature5(freqs, u, cell, k, f);
    for (int s = 0; s < kStreams; ++s) X[((int64_t)s * B + b) * kIn + k] = f[s];
}

// Tiled matrix product on the matrix cores (64x64 tiles, K step 32, four
// waves of 32x32).  Bounds-checked on M, N and K.
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs p)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[64][40];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[64][40];
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int g = l >> 4, c = l & 15;
    const int wm = w >> 1, wn = w & 1;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int kbeg = blockIdx.z * p.kchunk;
    const int kend = min(p.K, kbeg + p.kchunk);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int sr = tid >> 2, sk = (tid & 3) * 8;
    for (int k0 = kbeg; k0 < kend; k0 += 32) {
        {
            const int m = m0 + sr;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = k0 + sk + j;
                const float v = (m < p.M && k < kend) ? p.A[(int64_t)m * p.sam + (int64_t)k * p.sak] : 0.f;
                As[sr][sk + j] = (__bf16)v;
            }
            const int n = n0 + sr;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = k0 + sk + j;
                const float v = (n < p.N && k < kend) ? p.B[(int64_t)k * p.sbk + (int64_t)n * p.sbn] : 0.f;
                Bs[sr][sk + j] = (__bf16)v;
            }
        }
        __syncthreads();
        bf16x8 af[2], bf[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            af[i] = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + i * 16 + c][8 * g]);
            bf[i] = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + i * 16 + c][8 * g]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    float* C = p.C + (int64_t)blockIdx.z * p.split_stride;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn * 32 + j * 16 + c;
            if (n >= p.N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * 32 + i * 16 + 4 * g + r;
                if (m >= p.M) continue;
                float v = acc[i][j][r];
                if (p.bias && m < p.bias_rows) v += p.bias[n];
                C[(int64_t)m * p.ldc + n] = v;
            }
        }
}

// z streams from h streams (forward mode through SiLU).
__global__ void mlp_act_fwd_kernel(const float* H, float* Z, int64_t B, int W)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = B * W;
    if (i >= S) return;
    const float hv = H[i], hx = H[S + i], hy = H[2 * S + i], hz = H[3 * S + i], hl = H[4 * S + i];
    float d1, d2;
    Z[i] = silu3(hv, d1, d2);
    Z[S + i] = d1 * hx;
    Z[2 * S + i] = d1 * hy;
    Z[3 * S + i] = d1 * hz;
    Z[4 * S + i] = d1 * hl + d2 * (hx * hx + hy * hy + hz * hz);
}

// Adjoint of the SiLU streams: dh from dz and the saved h streams.
__global__ void mlp_act_bwd_kernel(const float* H, const float* dZ, float* dH, int64_t B, int W)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = B * W;
    if (i >= S) return;
    const float hv = H[i], hx = H[S + i], hy = H[2 * S + i], hz = H[3 * S + i], hl = H[4 * S + i];
    const float zv = dZ[i], zx = dZ[S + i], zy = dZ[2 * S + i], zz = dZ[3 * S + i], zl = dZ[4 * S + i];
    float f1, f2, f3;
    (void)silu4(hv, f1, f2, f3);
    const float s2 = hx * hx + hy * hy + hz * hz;
    dH[i] = zv * f1 + (zx * hx + zy * hy + zz * hz) * f2 + zl * (f2 * hl + f3 * s2);
    dH[S + i] = zx * f1 + 2.0f * zl * f2 * hx;
    dH[2 * S + i] = zy * f1 + 2.0f * zl * f2 * hy;
    dH[3 * S + i] = zz * f1 + 2.0f * zl * f2 * hz;
    dH[4 * S + i] = zl * f1;
}

// Sobolev loss of the normalised outputs Y[s][B][N] against spline targets
// (V[B][N], G[B][3][N], L[B][N]); writes dY and adds the loss to *loss.
__global__ void mlp_loss_kernel(const float* Y, const float* tV, const float* tG, const float* tL, const float* mu,
                                const float* sd, const float* w, int64_t B, int N, float* dY, float* loss)
{
    __shared__ float red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = B * N;
    float acc = 0.f;
    if (i < S) {
        const int64_t b = i / N;
        const int n = (int)(i - b * N);
        const float isd = 1.0f / sd[n];
        const float cv = 2.0f * w[0] / (float)S, cg = 2.0f * w[1] / (3.0f * (float)S), cl = 2.0f * w[2] / (float)S;
        const float ev = Y[i] - (tV[i] - mu[n]) * isd;
        dY[i] = cv * ev;
        acc += 0.5f * cv * ev * ev;
        for (int d = 0; d < 3; ++d) {
            const float eg = Y[(1 + d) * S + i] - tG[(3 * b + d) * N + n] * isd;
            dY[(1 + d) * S + i] = cg * eg;
            acc += 0.5f * cg * eg * eg;
        }
        const float el = Y[4 * S + i] - tL[i] * isd;
        dY[4 * S + i] = cl * el;
        acc += 0.5f * cl * el * el;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, red[0]);
}

// Column sums of the value-stream rows of dH [B][W], first stage: workgroup
// (x, y) sums columns 64x..64x+63 over rows y, y + gridDim.y, ... into
// part[y][W] (256 lanes: 64 columns x 4 row phases, combined in LDS).
__global__ void mlp_bias_grad_kernel(const float* dH, int64_t B, int W, float* part)
{
    __shared__ float red[4][64];
    const int cl = threadIdx.x & 63, rl = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + cl;
    float s = 0.f;
    if (n < W)
        for (int64_t b = (int64_t)blockIdx.y * 4 + rl; b < B; b += (int64_t)gridDim.y * 4) s += dH[b * W + n];
    red[rl][cl] = s;
    __syncthreads();
    if (rl == 0 && n < W) part[(int64_t)blockIdx.y * W + n] = red[0][cl] + red[1][cl] + red[2][cl] + red[3][cl];
}

__global__ void splitk_reduce_kernel(const float* part, int splits, int64_t count, int64_t stride, float* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[z * stride + i];
    out[i] = s;
}

__global__ void adam_kernel(float* P, const float* Gr, float* M1, float* M2, int64_t n, float lr, float b1, float b2,
                            float eps, float bc1, float bc2, __bf16* Wh)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = Gr[i];
    const float m = b1 * M1[i] + (1.0f - b1) * g;
    const float v = b2 * M2[i] + (1.0f - b2) * g * g;
    M1[i] = m;
    M2[i] = v;
    const float p = P[i] - lr * (m / bc1) / (sqrtf(v / bc2) + eps);
    P[i] = p;
    if (Wh) Wh[i] = (__bf16)p;
}

__global__ void bf16_copy_kernel(const float* P, __bf16* Wh, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) Wh[i] = (__bf16)P[i];
}

// Per-orbital statistics of a target batch: sums of V, V^2, G, G^2 (three
// components pooled), L, L^2 in FP64 -> stats[n][6].
__global__ void mlp_stats_kernel(const float* V, const float* G, const float* L, int64_t B, int N, double* stats)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t b = 0; b < B; ++b) {
        const double v = V[b * N + n], l = L[b * N + n];
        s[0] += v;
        s[1] += v * v;
        for (int d = 0; d < 3; ++d) {
            const double gg = G[(3 * b + d) * N + n];
            s[2] += gg;
            s[3] += gg * gg;
        }
        s[4] += l;
        s[5] += l * l;
    }
    for (int k = 0; k < 6; ++k) stats[6 * n + k] = s[k];
}

// ---------------------------------------------------------------------------
// Error map and routing.  Non-negative floats order like their bit patterns,
// so atomicMax on the unsigned bits is a float max.

__device__ inline int bin_of(const double* pos, int64_t b, const double* cell, int nb)
{
    int idx = 0;
    for (int d = 0; d < 3; ++d) {
        double f = pos[3 * b + d] / cell[d];
        f -= floor(f);
        int i = (int)(f * nb);
        i = i < 0 ? 0 : (i >= nb ? nb - 1 : i);  // NaN -> 0
        idx = idx * nb + i;
    }
    return idx;
}

__global__ void colmax_kernel(const float* V, const float* G, const float* L, int64_t B, int N, unsigned int* smax)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * N) return;
    const int64_t b = i / N;
    const int n = (int)(i - b * N);
    const float gm = fmaxf(fabsf(G[(3 * b) * N + n]), fmaxf(fabsf(G[(3 * b + 1) * N + n]), fabsf(G[(3 * b + 2) * N + n])));
    atomicMax(&smax[n], __float_as_uint(fabsf(V[i])));
    atomicMax(&smax[N + n], __float_as_uint(gm));
    atomicMax(&smax[2 * N + n], __float_as_uint(fabsf(L[i])));
}

__global__ void bin_error_kernel(const double* pos, double c0, double c1, double c2, int nbins, const float* Vm,
                                 const float* Gm, const float* Lm, const float* Vs, const float* Gs, const float* Ls,
                                 const unsigned int* smax, int64_t B, int N, unsigned int* bin_err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * N) return;
    const int64_t b = i / N;
    const int n = (int)(i - b * N);
    const double cell[3] = {c0, c1, c2};
    const float sv = fmaxf(__uint_as_float(smax[n]), 1e-30f);
    const float sg = fmaxf(__uint_as_float(smax[N + n]), 1e-30f);
    const float sl = fmaxf(__uint_as_float(smax[2 * N + n]), 1e-30f);
    float e = fabsf(Vm[i] - Vs[i]) / sv;
    for (int d = 0; d < 3; ++d) e = fmaxf(e, fabsf(Gm[(3 * b + d) * N + n] - Gs[(3 * b + d) * N + n]) / sg);
    e = fmaxf(e, fabsf(Lm[i] - Ls[i]) / sl);
    if (!(e == e)) e = 3.0e38f;  // NaN counts as the worst error
    atomicMax(&bin_err[bin_of(pos, b, cell, nbins)], __float_as_uint(e));
}

__global__ void fill_u32_kernel(unsigned int* p, unsigned int v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void bin_count_kernel(const double* pos, double c0, double c1, double c2, int nbins, int64_t B,
                                 unsigned int* count)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double cell[3] = {c0, c1, c2};
    atomicAdd(&count[bin_of(pos, b, cell, nbins)], 1u);
}

// A bin without validation points gets an infinite error (always routed).
__global__ void bin_finalize_kernel(const unsigned int* berr, const unsigned int* bcnt, float* out, int nb3)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nb3) out[k] = bcnt[k] ? __uint_as_float(berr[k]) : __builtin_inff();
}

// Appends the index of every position whose bin's estimated error exceeds tol.
__global__ void route_kernel(const double* pos, double c0, double c1, double c2, int nbins, const float* bin_err,
                             float tol, int64_t B, int32_t* list, int32_t* count)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double cell[3] = {c0, c1, c2};
    const float e = bin_err[bin_of(pos, b, cell, nbins)];
    if (!(e <= tol)) list[atomicAdd(count, 1)] = (int32_t)b;
}

}  // namespace qs
