// Surrogate-network training kernels for gfx950 (features, generic BF16
// matrix product on the matrix cores, SiLU streams forward/backward, Sobolev
// loss, gradient reductions, Adam), the error map and the routing of
// positions to the spline fallback.  The fused evaluation kernel is in
// mlp_forward.hip.
#include "mlp_kernels.hpp"

#include "common.hpp"

namespace qs {


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
                            float eps, float bc1, float bc2, __bf16* Wh, int32_t frag_k)
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
    if (Wh) Wh[frag_index(i, frag_k)] = (__bf16)p;
}

__global__ void bf16_copy_kernel(const float* P, __bf16* Wh, int64_t n, int32_t frag_k)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) Wh[frag_index(i, frag_k)] = (__bf16)P[i];
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
        const double x = f * nb;
        // f rounded up to 1 is the last bin; a non-finite coordinate is bin 0
        const int i = (x >= 0.0 && x < (double)nb) ? (int)x : (x >= (double)nb ? nb - 1 : 0);
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

// A point's error: the largest over orbitals of |dV| / sV, |dG_d| / sG and
// |dL| / sL, each normaliser the orbital's largest |quantity| over the
// validation set (1 if that is 0).  A NaN term makes the error +inf, whose
// bits order above every finite error.
__global__ void bin_error_kernel(const double* pos, double c0, double c1, double c2, int nbins, const float* Vm,
                                 const float* Gm, const float* Lm, const float* Vs, const float* Gs, const float* Ls,
                                 const unsigned int* smax, int64_t B, int N, unsigned int* bin_err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * N) return;
    const int64_t b = i / N;
    const int n = (int)(i - b * N);
    const double cell[3] = {c0, c1, c2};
    auto norm = [](unsigned int bits) {
        const float s = __uint_as_float(bits);
        return s == 0.0f ? 1.0f : s;
    };
    const float sv = norm(smax[n]), sg = norm(smax[N + n]), sl = norm(smax[2 * N + n]);
    float e = 0.0f;
    bool nan = false;
    auto take = [&](float x) {
        nan |= !(x == x);
        e = fmaxf(e, x);
    };
    take(fabsf(Vm[i] - Vs[i]) / sv);
    for (int d = 0; d < 3; ++d) take(fabsf(Gm[(3 * b + d) * N + n] - Gs[(3 * b + d) * N + n]) / sg);
    take(fabsf(Lm[i] - Ls[i]) / sl);
    if (nan) e = __builtin_inff();
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
