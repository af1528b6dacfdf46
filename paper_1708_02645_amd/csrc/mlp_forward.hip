// Fused forward-mode evaluation of the surrogate network on the matrix cores
// (gfx950, v_mfma_f32_16x16x32_bf16, BF16 operands, FP32 accumulation).
//
// A workgroup of four waves evaluates 16 positions through all layers; wave
// w owns a quarter of every layer's output units (64 of a hidden layer's
// 256).  Operand layout of the instruction (lane l, g = l/16, c = l%16):
// A[c][8g..8g+7], B[8g..8g+7][c], C[4g..4g+3][c].  Each layer is computed
// transposed, H^T[unit][pos] = sum_k W[unit][k] Act[pos][k]:
//  - weight rows are the A operand, read from global memory one K step
//    ahead of use (280 KB in all, L2-resident).  The BF16 weights are kept
//    in fragment order, so one wave's operand load is one contiguous 1 KB
//    block; row-major rows made it 16 half-used cache lines, and those loads
//    were the kernel's bound;
//  - the layer input, a [stream][16][256] BF16 tile in LDS shared by the
//    four waves (16-byte chunks XOR-swizzled by row), gives the B operands,
//    each stream's read one K step ahead.
// Each stream (value, d/dx, d/dy, d/dz, Laplacian) is its own product, so
// the five accumulators of a (unit, position) pair sit in the same lane and
// slot and the forward-mode SiLU combines them in registers; a lane then
// holds four consecutive units of one position and writes them back with one
// 8-byte store per stream.  One tile serves as every layer's input and
// output (a barrier separates the last operand reads from the epilogue's
// writes), 40 KB per workgroup, and the kernel is held to 168 registers (up
// to 192 outputs): three workgroups share a CU, three waves per SIMD, so two
// waves' loads and vector work hide behind the third's matrix products.
#include "mlp_kernels.hpp"

#include "common.hpp"

namespace qs {

typedef float f32x4v __attribute__((ext_vector_type(4)));

constexpr int kFwdWaves = 4;
constexpr int kFwdPos = 16;
constexpr int kTile = kStreams * kFwdPos * kHidden;  // BF16 elements of one activation tile

// Element offset of (stream s, position row, column col) in a tile: 16-byte
// chunks XOR-swizzled by the row, so the 16 rows a wave reads or writes at
// one column fall in distinct banks.
__device__ inline int zoff(int s, int row, int col)
{
    return ((s * kFwdPos + row) * kHidden + ((((col >> 3) ^ (row & 15)) << 3) | (col & 7)));
}

// acc[s][nb] = sum over KSTEPS*32 inputs of W[(blk0+nb)*16 + unit][k] xt[s][pos][k]
// for NB blocks of 16 units; `blocks` clamps the weight rows of blocks past
// the layer's end (their results are never used).
template <int KSTEPS, int NB>
__device__ inline void layer_products(const __bf16* __restrict__ xt, const __bf16* __restrict__ W, int blk0,
                                      int blocks, int g, int c, f32x4 (&acc)[kStreams][NB])
{
    constexpr int R = 2;  // ring depth: weight fragments of step t+1 are loaded at step t
    // W is in fragment order: fragment (blk, t) is 512 values, lane l's 8 at 8l.
    const __bf16* wrow[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int blk = blk0 + nb < blocks ? blk0 + nb : blocks - 1;
        wrow[nb] = W + (int64_t)blk * KSTEPS * 512 + 8 * (16 * g + c);
    }
    bf16x8 ring[R][NB];
#pragma unroll
    for (int i = 0; i < R - 1; ++i)
        if (i < KSTEPS)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) ring[i][nb] = *reinterpret_cast<const bf16x8*>(wrow[nb] + 512 * i);
    bf16x8 x[kStreams];  // one B operand per stream
#pragma unroll
    for (int s = 0; s < kStreams; ++s) x[s] = *reinterpret_cast<const bf16x8*>(xt + zoff(s, c, 8 * g));
#pragma unroll
    for (int s = 0; s < kStreams; ++s)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[s][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // The scheduling fences keep each load ahead of the products that follow
    // it (otherwise the scheduler sinks loads next to their use and every
    // step waits for a full L2 or LDS round trip).
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < KSTEPS; ++t) {
        if (t + R - 1 < KSTEPS)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                ring[(t + R - 1) % R][nb] = *reinterpret_cast<const bf16x8*>(wrow[nb] + 512 * (t + R - 1));
        __builtin_amdgcn_sched_barrier(0);
        // stream s's operand of step t+1 is read as soon as its products of
        // step t are issued, so only one operand per stream is live
#pragma unroll
        for (int s = 0; s < kStreams; ++s) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                acc[s][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ring[t % R][nb], x[s], acc[s][nb], 0, 0, 0);
            if (t + 1 < KSTEPS) x[s] = *reinterpret_cast<const bf16x8*>(xt + zoff(s, c, 32 * (t + 1) + 8 * g));
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Hidden layer epilogue: bias, forward-mode SiLU, BF16 into the output tile.
template <int NB>
__device__ inline void hidden_epilogue(const f32x4 (&acc)[kStreams][NB], const float* __restrict__ bias,
                                       __bf16* zo, int blk0, int g, int c)
{
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int u0 = (blk0 + nb) * 16 + 4 * g;
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
            *reinterpret_cast<uint64_t*>(zo + zoff(s, c, u0)) = packed;
        }
    }
}

// Output epilogue: bias and the per-orbital affine map, for output block nb
// of the wave: q[0] value, q[1..3] gradient, q[4] Laplacian of orbitals
// n0..n0+3 at the lane's position.
template <int NB>
__device__ inline int output_block(const MlpFwdArgs& a, const f32x4 (&acc)[kStreams][NB], const float* b3, int nb,
                                   int blk0, int g, f32x4v (&q)[kStreams])
{
    const int n0 = (blk0 + nb) * 16 + 4 * g;
    const f32x4v sd = *reinterpret_cast<const f32x4v*>(a.sd + n0);
    const f32x4v mu = *reinterpret_cast<const f32x4v*>(a.mu + n0);
    const f32x4v bb = *reinterpret_cast<const f32x4v*>(b3 + n0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        q[0][j] = (acc[0][nb][j] + bb[j]) * sd[j] + mu[j];
#pragma unroll
        for (int s = 1; s < kStreams; ++s) q[s][j] = acc[s][nb][j] * sd[j];
    }
    return n0;
}

// Staged outputs: rows of nout floats in the tile, padded by 4 floats so a
// wave's 16 rows fall in distinct banks.  Two rounds: the 16 value rows and
// the 16 Laplacian rows (32 rows), then the 48 gradient rows (row 3 pos + d,
// the order of G in memory); each round needs 48 (nout + 4) floats at most,
// within the tile for nout up to 208.
constexpr int kStagePad = 4;

// Copies `rows` staged rows to dst, where they are one contiguous run (the
// workgroup's positions are consecutive), in 16-byte pieces taken by
// consecutive threads.  Piece i is (row r, column 4k), i = r n/4 + k; the
// thread's (r, k) advance by a fixed step instead of a division per piece.
__device__ inline void copy_rows(const float* stage, float* dst, int rows, int N, int tid)
{
    constexpr int kStep = kFwdWaves * 64;
    const int n4 = N / 4, dr = kStep / n4, dk = kStep - dr * n4, total = rows * n4;
    int r = tid / n4, k = tid - r * n4;
    for (int i = tid; i < total; i += kStep) {
        const f32x4v v = *reinterpret_cast<const f32x4v*>(stage + r * (N + kStagePad) + 4 * k);
        __builtin_nontemporal_store(v, reinterpret_cast<f32x4v*>(dst + (int64_t)r * N + 4 * k));
        r += dr;
        k += dk;
        if (k >= n4) {
            k -= n4;
            ++r;
        }
    }
}

// Features of the workgroup's 16 positions into tile zt: thread t < 192
// takes position t/12 and the 8 feature columns 8(t%12)..+7 (sin for columns
// below kFreq, cos above), five streams each, one 16-byte store per stream.
// The phase k.u is reduced modulo 1 in FP64; the hardware sine/cosine take
// the angle in revolutions.
__device__ inline void stage_features(const MlpFwdArgs& a, int64_t b0, int tid, __bf16* zt)
{
    if (tid >= kFwdPos * (kIn / 8)) return;
    const int p = tid / (kIn / 8), ch = tid % (kIn / 8);
    int64_t bi = b0 + p;
    if (bi >= a.B) bi = a.B - 1;  // ragged tail: computed, never stored
    double u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = a.pos[3 * bi + d] * a.icell[d];
    bf16x8 f[kStreams];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = 8 * ch + j;
        const int fi = k < kFreq ? k : k - kFreq;
        const int kx = a.freqs[3 * fi], ky = a.freqs[3 * fi + 1], kz = a.freqs[3 * fi + 2];
        double x = (double)kx * u[0] + (double)ky * u[1] + (double)kz * u[2];
        x -= floor(x);
        const float sn = __builtin_amdgcn_sinf((float)x), cs = __builtin_amdgcn_cosf((float)x);
        const float gx = (float)(kx * a.tpc[0]), gy = (float)(ky * a.tpc[1]), gz = (float)(kz * a.tpc[2]);
        const float val = k < kFreq ? sn : cs, dv = k < kFreq ? cs : -sn;
        f[0][j] = (__bf16)val;
        f[1][j] = (__bf16)(dv * gx);
        f[2][j] = (__bf16)(dv * gy);
        f[3][j] = (__bf16)(dv * gz);
        f[4][j] = (__bf16)(-(gx * gx + gy * gy + gz * gz) * val);
    }
#pragma unroll
    for (int s = 0; s < kStreams; ++s) *reinterpret_cast<bf16x8*>(zt + zoff(s, p, 8 * ch)) = f[s];
}

// NBO: output blocks of 16 orbitals per wave, ceil(nout / 64).  STAGED:
// outputs go through the tile (nout up to 208); otherwise each lane stores
// four consecutive orbitals of one position directly.  Three waves per SIMD
// where the output epilogue fits in 168 registers without spilling (staged,
// nout up to 192), else two.
template <int NBO, bool STAGED>
constexpr int fwd_waves_per_simd = STAGED && NBO < 4 ? 3 : 2;

template <int NBO, bool STAGED>
__global__ __launch_bounds__(kFwdWaves * 64) __attribute__((
    amdgpu_waves_per_eu(fwd_waves_per_simd<NBO, STAGED>, fwd_waves_per_simd<NBO, STAGED>))) void mlp_vgl_kernel(MlpFwdArgs a)
{
    __shared__ __attribute__((aligned(16))) __bf16 tile[kTile];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, c = l & 15;
    const int64_t b0 = (int64_t)blockIdx.x * kFwdPos;
    const MlpOffsets o = mlp_offsets(a.nout);
    constexpr int NBH = kHidden / 16 / kFwdWaves;  // hidden blocks per wave

    stage_features(a, b0, tid, tile);
    __syncthreads();
    {
        f32x4 acc[kStreams][NBH];
        layer_products<kIn / 32, NBH>(tile, a.Wh + o.hW1, NBH * w, kHidden / 16, g, c, acc);
        __syncthreads();  // every wave has read its operands before the tile is overwritten
        hidden_epilogue<NBH>(acc, a.P + o.b1, tile, NBH * w, g, c);
    }
    __syncthreads();
    {
        f32x4 acc[kStreams][NBH];
        layer_products<kHidden / 32, NBH>(tile, a.Wh + o.hW2, NBH * w, kHidden / 16, g, c, acc);
        __syncthreads();
        hidden_epilogue<NBH>(acc, a.P + o.b2, tile, NBH * w, g, c);
    }
    __syncthreads();
    const int N = a.nout, nblk = N / 16, blk0 = NBO * w;
    const float* b3 = a.P + o.b3;
    f32x4 acc[kStreams][NBO];
    layer_products<kHidden / 32, NBO>(tile, a.Wh + o.hW3, blk0, nblk, g, c, acc);
    if constexpr (!STAGED) {
        const int64_t b = b0 + c;
        if (b >= a.B) return;
#pragma unroll
        for (int nb = 0; nb < NBO; ++nb) {
            if (blk0 + nb >= nblk) continue;
            f32x4v q[kStreams];
            const int n0 = output_block<NBO>(a, acc, b3, nb, blk0, g, q);
            __builtin_nontemporal_store(q[0], reinterpret_cast<f32x4v*>(a.V + b * N + n0));
#pragma unroll
            for (int d = 0; d < 3; ++d)
                __builtin_nontemporal_store(q[1 + d], reinterpret_cast<f32x4v*>(a.G + (3 * b + d) * N + n0));
            __builtin_nontemporal_store(q[4], reinterpret_cast<f32x4v*>(a.L + b * N + n0));
        }
    } else {
        float* stage = reinterpret_cast<float*>(tile);
        const int ld = N + kStagePad;
        const int64_t left = a.B - b0;
        const int np = left < kFwdPos ? (int)left : kFwdPos;
        __syncthreads();  // every wave has read its last operands
#pragma unroll
        for (int nb = 0; nb < NBO; ++nb) {
            if (blk0 + nb >= nblk) continue;
            f32x4v q[kStreams];
            const int n0 = output_block<NBO>(a, acc, b3, nb, blk0, g, q);
            *reinterpret_cast<f32x4v*>(stage + c * ld + n0) = q[0];
            *reinterpret_cast<f32x4v*>(stage + (kFwdPos + c) * ld + n0) = q[4];
        }
        __syncthreads();
        copy_rows(stage, a.V + b0 * N, np, N, tid);
        copy_rows(stage + kFwdPos * ld, a.L + b0 * N, np, N, tid);
        __syncthreads();
#pragma unroll
        for (int nb = 0; nb < NBO; ++nb) {
            if (blk0 + nb >= nblk) continue;
            f32x4v q[kStreams];
            const int n0 = output_block<NBO>(a, acc, b3, nb, blk0, g, q);
#pragma unroll
            for (int d = 0; d < 3; ++d) *reinterpret_cast<f32x4v*>(stage + (3 * c + d) * ld + n0) = q[1 + d];
        }
        __syncthreads();
        copy_rows(stage, a.G + 3 * b0 * N, 3 * np, N, tid);
    }
}

int launch_mlp_forward(const MlpFwdArgs& a, hipStream_t st)
{
    const int64_t blocks = (a.B + kFwdPos - 1) / kFwdPos;
    if (blocks > 0x7fffffff) return fail(SPL_EINVAL, "batch too large");
    if (a.nout < 16 || a.nout > kMaxOut || a.nout % 16) return fail(SPL_EUNSUPPORTED, "output width out of range");
    for (const float* p : {a.V, a.G, a.L})
        if (reinterpret_cast<uintptr_t>(p) & 15) return fail(SPL_EINVAL, "V, G and L must be 16-byte aligned");
    const int nbo = (a.nout / 16 + kFwdWaves - 1) / kFwdWaves;
    const bool staged = (size_t)3 * kFwdPos * (a.nout + kStagePad) * sizeof(float) <= kTile * sizeof(__bf16);
    const dim3 grid((unsigned)blocks), block(kFwdWaves * 64);
    switch (nbo * 2 + (staged ? 1 : 0)) {
    case 2: hipLaunchKernelGGL((mlp_vgl_kernel<1, false>), grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL((mlp_vgl_kernel<1, true>), grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL((mlp_vgl_kernel<2, false>), grid, block, 0, st, a); break;
    case 5: hipLaunchKernelGGL((mlp_vgl_kernel<2, true>), grid, block, 0, st, a); break;
    case 6: hipLaunchKernelGGL((mlp_vgl_kernel<3, false>), grid, block, 0, st, a); break;
    case 7: hipLaunchKernelGGL((mlp_vgl_kernel<3, true>), grid, block, 0, st, a); break;
    case 8: hipLaunchKernelGGL((mlp_vgl_kernel<4, false>), grid, block, 0, st, a); break;
    case 9: hipLaunchKernelGGL((mlp_vgl_kernel<4, true>), grid, block, 0, st, a); break;
    default: return fail(SPL_EUNSUPPORTED, "output width out of range");
    }
    QS_HIP(hipGetLastError());
    return SPL_OK;
}

}  // namespace qs
