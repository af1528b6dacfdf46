// Value, gradient and full Hessian of B-spline orbitals in any cell (gfx950).
//
// The gather, the staging of per-position weights and the pipelining are
// those of eval_block (eval_kernel.hpp); the contraction is extended to all
// ten grid-frame quantities: V, the three first derivatives and the six
// second derivatives d2/dt_d dt_e in grid units.  The three mixed ones come
// from the same anchored difference form: d2/dy dz is the quadratic y-weight
// sum of first z-differences, d2/dx dy and d2/dx dz the quadratic x-weight
// sums of differences of the y-level d/dy and d/dz sums -- each a difference
// of small derivative quantities, never of raw coefficients.
//
// A per-orbital epilogue maps the grid frame to Cartesian coordinates with
// the wave-uniform matrices of the launch:
//   G_c = sum_d M[c][d] g_d                 (M = Lat^-1 diag(n))
//   H_h = sum_k P[h][k] h_k                 (P: the 6x6 map of M (.) M^T on
//                                            symmetric matrices)
//   L   = sum_k K[k] h_k                    (K: the trace of that map)
// OUT selects the stores: VGH (V, G, H[6]), general-cell VGL (V, G, L), or
// the fused determinant ratio with derivatives (RATIO: the Cartesian V, G, L
// dotted with the position's row of A^-1, five numbers per position, summed
// as in eval_block: lanes by a butterfly, tiles in tile order after a
// barrier).
#pragma once

#include <vector>

#include "eval_kernel.hpp"

namespace qs {

enum { VGH_OUT_H = 0, VGH_OUT_L = 1, VGH_OUT_RATIO = 2 };

struct VghArgs {
    EvalArgs e;         // e.V, e.G as usual; e.general = 1; e.L unused for OUT_H
    void* H;            // [B][6][norb] for OUT_H, else [B][norb] (the Laplacian)
    float Mf[9], Pf[36], Kf[6];
    double Md[9], Pd[36], Kd[6];
};

template <typename TA> __device__ inline const TA* vgh_M(const VghArgs& a);
template <> __device__ inline const float* vgh_M<float>(const VghArgs& a) { return a.Mf; }
template <> __device__ inline const double* vgh_M<double>(const VghArgs& a) { return a.Md; }
template <typename TA> __device__ inline const TA* vgh_P(const VghArgs& a);
template <> __device__ inline const float* vgh_P<float>(const VghArgs& a) { return a.Pf; }
template <> __device__ inline const double* vgh_P<double>(const VghArgs& a) { return a.Pd; }
template <typename TA> __device__ inline const TA* vgh_K(const VghArgs& a);
template <> __device__ inline const float* vgh_K<float>(const VghArgs& a) { return a.Kf; }
template <> __device__ inline const double* vgh_K<double>(const VghArgs& a) { return a.Kd; }

template <spline_dtype S, int CW, int NCH, int LPP, int OUT>
__device__ inline void vgh_block(const VghArgs& va, int64_t b0, int np, PosW<typename Acc<S>::type>* W)
{
    using TA = typename Acc<S>::type;
    const EvalArgs& a = va.e;
    constexpr int VPC = vals_per_chunk<S>(CW);
    constexpr int VPL = VPC * NCH;
    constexpr int CHB = CW * 4;
    constexpr int GCB = LPP * CHB;
    constexpr int TB = GCB * NCH;
    constexpr int TO = LPP * VPL;
    static_assert(VPC >= 1, "chunk narrower than one value");

    const int tid = threadIdx.x;
    for (int p = tid; p < np; p += kBlock) stage_position<TA>(a, b0 + p, W[p]);
    __syncthreads();

    constexpr int groups = kBlock / LPP;
    const int g = tid / LPP;
    const int lane = tid % LPP;
    const int items = np * a.tiles;
    const uint32_t loff = (uint32_t)lane * CHB;
    // RATIO: per-(position, tile) sums in LDS after the staged weights.
    TA* part = reinterpret_cast<TA*>(W + a.pb);
    bool row_aligned = false;
    if constexpr (OUT == VGH_OUT_RATIO)
        row_aligned = a.ald % VPC == 0 && (uintptr_t)a.ainv % alignof(Pack<TA, VPC>) == 0;

    for (int it = g; it < items; it += groups) {
        const int item = (LPP == 64) ? uniform<int>(it) : it;
        const int p = item / a.tiles;
        const int tile = item - p * a.tiles;
        const PosW<TA>& w = W[p];

        int64_t off = w.off + (int64_t)tile * TB;
        if constexpr (LPP == 64) off = uniform<int64_t>(off);
        TA wy[9], wz[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            wy[k] = (LPP == 64) ? uniform<TA>(w.w[1][k]) : w.w[1][k];
            wz[k] = (LPP == 64) ? uniform<TA>(w.w[2][k]) : w.w[2][k];
        }
        // Row addresses as in eval_block: wave-uniform for LPP = 64, else one
        // 64-bit address per lane plus the wave-uniform row offset.
        const unsigned char* base = a.table + off;
        const unsigned char* lbase = base + loff;
        auto issue = [&](int xy, Chunk<CW> (&buf)[4][NCH]) {
            const int k0 = xy >> 2, k1 = xy & 3;
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) {
                const int64_t ro = k0 * a.xstride + k1 * a.ystride + k2 * a.row_bytes;
                if constexpr (LPP == 64) {
                    const unsigned char* row = base + ro;
#pragma unroll
                    for (int c = 0; c < NCH; ++c) buf[k2][c] = load_chunk<CW>(row + (loff + (uint32_t)(c * GCB)));
                } else {
                    const unsigned char* row = lbase + ro;
#pragma unroll
                    for (int c = 0; c < NCH; ++c) buf[k2][c] = load_chunk<CW>(row + c * GCB);
                }
            }
        };

        // x-level running sums: value (anchored), d/dx, d2/dx2, the y- and
        // z-derivative families, and the previous x's quantities whose
        // differences form the x-derivatives.
        TA vx[VPL], gxa[VPL], hxx[VPL], gya[VPL], gza[VPL], hyy[VPL], hzz[VPL], hyz[VPL], hxy[VPL], hxz[VPL];
        TA hxp[VPL], uxp[VPL], dxp[VPL], uyp[VPL], t1p[VPL];
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            vx[v] = gxa[v] = hxx[v] = gya[v] = gza[v] = hyy[v] = hzz[v] = hyz[v] = hxy[v] = hxz[v] = TA(0);
            hxp[v] = uxp[v] = dxp[v] = uyp[v] = t1p[v] = TA(0);
        }
        const TA wa0 = -wz[0], wa1 = wz[2] + wz[3], wa2 = wz[3];
        // Tail sums of the cubic weights (c_0 = 1): the y and x levels smooth
        // values as f_0 + sum_{k>=1} c_k (f_k - f_{k-1}).
        const TA cy3 = wy[3], cy2 = wy[2] + cy3, cy1 = wy[1] + cy2;
        const TA cy[4] = {TA(1), cy1, cy2, cy3};
        TA cx[4];
        cx[3] = (LPP == 64) ? uniform<TA>(w.w[0][3]) : w.w[0][3];
#pragma unroll
        for (int k = 2; k >= 1; --k) cx[k] = ((LPP == 64) ? uniform<TA>(w.w[0][k]) : w.w[0][k]) + cx[k + 1];
        cx[0] = TA(1);

        Chunk<CW> buf[2][4][NCH];
        issue(0, buf[0]);
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            // y-level state of this x
            TA h0[VPL], hp[VPL], lp[VPL], ep[VPL], ul[VPL], uy[VPL], uyy[VPL], t1[VPL], t2[VPL], t3[VPL], s1p[VPL];
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                const int xy = 4 * x + y;
                if (xy + 1 < 16) issue(xy + 1, buf[(xy + 1) & 1]);
                __builtin_amdgcn_sched_barrier(0);
                TA c[4][VPL];
#pragma unroll
                for (int k2 = 0; k2 < 4; ++k2)
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) decode<S, CW, TA>(buf[xy & 1][k2][ch], &c[k2][ch * VPC]);
#pragma unroll
                for (int v = 0; v < VPL; ++v) {
                    const TA d0 = c[1][v] - c[0][v], d1 = c[2][v] - c[1][v], d2 = c[3][v] - c[2][v];
                    const TA hz = c[1][v];
                    TA lz = wa0 * d0;
                    lz = fma(wa1, d1, lz);
                    lz = fma(wa2, d2, lz);
                    TA s1 = wz[4] * d0;
                    s1 = fma(wz[5], d1, s1);
                    s1 = fma(wz[6], d2, s1);
                    TA s2 = wz[7] * (d1 - d0);
                    s2 = fma(wz[8], d2 - d1, s2);
                    if (y == 0) {
                        h0[v] = hz;
                        ul[v] = lz;  // s0[0] = h0 + ul
                        t1[v] = wy[0] * s1;
                        t2[v] = wy[0] * s2;
                    } else {
                        const TA e = (hz - hp[v]) + (lz - lp[v]);  // s0[y] - s0[y-1]
                        const TA f = s1 - s1p[v];                   // s1[y] - s1[y-1]
                        ul[v] = fma(cy[y], e, ul[v]);
                        t1[v] = fma(wy[y], s1, t1[v]);
                        t2[v] = fma(wy[y], s2, t2[v]);
                        if (y == 1) {
                            uy[v] = wy[4] * e;
                            t3[v] = wy[4] * f;
                        } else {
                            uy[v] = fma(wy[4 + y - 1], e, uy[v]);
                            t3[v] = fma(wy[4 + y - 1], f, t3[v]);
                            if (y == 2) uyy[v] = wy[7] * (e - ep[v]);
                            else uyy[v] = fma(wy[8], e - ep[v], uyy[v]);
                        }
                        ep[v] = e;
                        pin(uy[v]);
                        pin(t3[v]);
                        pin(ep[v]);
                    }
                    hp[v] = hz;
                    lp[v] = lz;
                    s1p[v] = s1;
                    pin(ul[v]);
                    pin(t1[v]);
                    pin(t2[v]);
                    pin(hp[v]);
                    pin(lp[v]);
                    pin(s1p[v]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }

            const TA bx = (LPP == 64) ? uniform<TA>(w.w[0][x]) : w.w[0][x];
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                if (x == 0) vx[v] = h0[v] + ul[v];  // u[0]; then the tail weights times u[x] - u[x-1]
                gya[v] = fma(bx, uy[v], gya[v]);
                gza[v] = fma(bx, t1[v], gza[v]);
                hyy[v] = fma(bx, uyy[v], hyy[v]);
                hzz[v] = fma(bx, t2[v], hzz[v]);
                hyz[v] = fma(bx, t3[v], hyz[v]);
                if (x >= 1) {
                    const TA qx = (LPP == 64) ? uniform<TA>(w.w[0][4 + x - 1]) : w.w[0][4 + x - 1];
                    const TA d = (h0[v] - hxp[v]) + (ul[v] - uxp[v]);  // u[x] - u[x-1]
                    vx[v] = fma(cx[x], d, vx[v]);
                    gxa[v] = fma(qx, d, gxa[v]);
                    hxy[v] = fma(qx, uy[v] - uyp[v], hxy[v]);
                    hxz[v] = fma(qx, t1[v] - t1p[v], hxz[v]);
                    if (x >= 2) {
                        const TA lx = (LPP == 64) ? uniform<TA>(w.w[0][7 + x - 2]) : w.w[0][7 + x - 2];
                        hxx[v] = fma(lx, d - dxp[v], hxx[v]);
                    }
                    dxp[v] = d;
                }
                hxp[v] = h0[v];
                uxp[v] = ul[v];
                uyp[v] = uy[v];
                t1p[v] = t1[v];
            }
        }

        // Grid frame -> Cartesian.  M, P, K are launch constants (scalar
        // registers); the 16-bit scale multiplies every output.
        const TA* M = vgh_M<TA>(va);
        const TA* P = vgh_P<TA>(va);
        const TA* K = vgh_K<TA>(va);
        const int64_t b = w.row;
        const bool aligned = (a.norb % VPC) == 0;
        TA* Vo = reinterpret_cast<TA*>(a.V) + b * a.norb;
        TA* Go = reinterpret_cast<TA*>(a.G) + (3 * b) * a.norb;
        TA* Ho = reinterpret_cast<TA*>(va.H) + (OUT == VGH_OUT_H ? 6 : 1) * b * a.norb;
        [[maybe_unused]] TA rsum[5] = {TA(0), TA(0), TA(0), TA(0), TA(0)};
        [[maybe_unused]] const TA* ar = nullptr;
        if constexpr (OUT == VGH_OUT_RATIO)
            ar = reinterpret_cast<const TA*>(a.ainv) + (a.arows ? (int64_t)a.arows[b] : b) * a.ald;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int o = tile * TO + c * LPP * VPC + lane * VPC;
            if (OUT != VGH_OUT_RATIO && o >= a.norb) continue;
            TA sc[VPC];
#pragma unroll
            for (int i = 0; i < VPC; ++i) {
                if constexpr (S == SPL_BF16 || S == SPL_F16) sc[i] = a.scales[o + i];
                else sc[i] = TA(1);
            }
            TA ov[VPC], og[3][VPC], oh[6][VPC];
#pragma unroll
            for (int i = 0; i < VPC; ++i) {
                const int v = c * VPC + i;
                const TA s = sc[i];
                const TA gu[3] = {gxa[v] * s, gya[v] * s, gza[v] * s};
                const TA hu[6] = {hxx[v] * s, hxy[v] * s, hxz[v] * s, hyy[v] * s, hyz[v] * s, hzz[v] * s};
                ov[i] = vx[v] * s;
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    TA acc = M[cc * 3] * gu[0];
                    acc = fma(M[cc * 3 + 1], gu[1], acc);
                    og[cc][i] = fma(M[cc * 3 + 2], gu[2], acc);
                }
                if constexpr (OUT == VGH_OUT_H) {
#pragma unroll
                    for (int h = 0; h < 6; ++h) {
                        TA acc = P[h * 6] * hu[0];
#pragma unroll
                        for (int k = 1; k < 6; ++k) acc = fma(P[h * 6 + k], hu[k], acc);
                        oh[h][i] = acc;
                    }
                } else {
                    TA acc = K[0] * hu[0];
#pragma unroll
                    for (int k = 1; k < 6; ++k) acc = fma(K[k], hu[k], acc);
                    oh[0][i] = acc;
                }
            }
            if constexpr (OUT == VGH_OUT_RATIO) {
                // padding orbitals (o >= norb) hold zero coefficients and get
                // zero inverse-row entries
                TA av[VPC];
                load_vals<TA, VPC>(ar, av, o, a.norb, row_aligned);
#pragma unroll
                for (int i = 0; i < VPC; ++i) {
                    rsum[0] = fma(av[i], ov[i], rsum[0]);
                    rsum[1] = fma(av[i], og[0][i], rsum[1]);
                    rsum[2] = fma(av[i], og[1][i], rsum[2]);
                    rsum[3] = fma(av[i], og[2][i], rsum[3]);
                    rsum[4] = fma(av[i], oh[0][i], rsum[4]);
                }
                continue;
            }
            store_vals<TA, VPC>(Vo, ov, o, a.norb, aligned);
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) store_vals<TA, VPC>(Go + cc * a.norb, og[cc], o, a.norb, aligned);
#pragma unroll
            for (int h = 0; h < (OUT == VGH_OUT_H ? 6 : 1); ++h)
                store_vals<TA, VPC>(Ho + h * a.norb, oh[h], o, a.norb, aligned);
        }
        if constexpr (OUT == VGH_OUT_RATIO) {
#pragma unroll
            for (int m = LPP / 2; m >= 1; m >>= 1)
#pragma unroll
                for (int q = 0; q < 5; ++q) rsum[q] += __shfl_xor(rsum[q], m, LPP);
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < 5; ++q) part[(p * a.tiles + tile) * 5 + q] = rsum[q];
            }
        }
    }
    if constexpr (OUT == VGH_OUT_RATIO) {
        __syncthreads();
        for (int p = tid; p < np; p += kBlock) {
            TA sum[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) sum[q] = part[p * a.tiles * 5 + q];
            for (int t = 1; t < a.tiles; ++t)
#pragma unroll
                for (int q = 0; q < 5; ++q) sum[q] += part[(p * a.tiles + t) * 5 + q];
            TA* D = reinterpret_cast<TA*>(a.V) + W[p].row * 5;
#pragma unroll
            for (int q = 0; q < 5; ++q) D[q] = sum[q];
        }
    }
}

template <spline_dtype S, int CW, int NCH, int LPP, int OUT>
__global__ __launch_bounds__(kBlock) void vgh_kernel(VghArgs va)
{
    using TA = typename Acc<S>::type;
    extern __shared__ unsigned char lds_raw[];
    PosW<TA>* W = reinterpret_cast<PosW<TA>*>(lds_raw);
    const int64_t b0 = (int64_t)blockIdx.x * va.e.pb;
    const int64_t rem = va.e.B - b0;
    if (rem <= 0) return;
    const int np = rem < va.e.pb ? (int)rem : va.e.pb;
    vgh_block<S, CW, NCH, LPP, OUT>(va, b0, np, W);
}

// Several tables in one launch through the VGH-family kernel (the
// general-cell VGL, V, G and the trace of the Cartesian Hessian): the
// persistent work queue of plan_kernel (eval_kernel.hpp), each task running
// vgh_block on its table's arguments.
struct PlanVghArgs {
    const VghArgs* tabs;    // device, one per table
    const PlanTask* tasks;  // device, ntasks entries
    unsigned int* counter;  // device work counters (one per segment), zero at launch
    int32_t ntasks;
    int32_t nseg;
};

template <spline_dtype S, int CW, int NCH, int LPP>
__global__ __launch_bounds__(kBlock) void plan_vgh_kernel(PlanVghArgs pa)
{
    using TA = typename Acc<S>::type;
    extern __shared__ unsigned char lds_raw[];
    PosW<TA>* W = reinterpret_cast<PosW<TA>*>(lds_raw);
    __shared__ int s_task;
    const int home = (int)(blockIdx.x % (unsigned)pa.nseg);
    for (int k = 0; k < pa.nseg; ++k) {
        const int seg = (home + k) % pa.nseg;
        const int t0 = (int)((int64_t)pa.ntasks * seg / pa.nseg);
        const int t1 = (int)((int64_t)pa.ntasks * (seg + 1) / pa.nseg);
        for (;;) {
            if (threadIdx.x == 0) s_task = t0 + (int)atomicAdd(pa.counter + seg, 1u);
            __syncthreads();
            const int t = uniform<int>(s_task);
            __syncthreads();  // every thread has read s_task before it can be rewritten
            if (t >= t1) break;  // uniform across the workgroup
            const PlanTask tk = pa.tasks[t];
            vgh_block<S, CW, NCH, LPP, VGH_OUT_L>(pa.tabs[tk.table], tk.first, tk.count, W);
            __syncthreads();  // W is rewritten by the next task
        }
    }
}

// Registry entry of one compiled VGH-family kernel (plan_fn: the plan
// kernel of the shape, on the general-cell VGL entry).
struct VghVariant {
    spline_dtype store;
    int cw, nch, lpp, out;
    const void* fn;
    size_t lds_per_pos;
    const void* plan_fn;
};

// Host side (vgh_host.cpp): the kernel arguments of a VGH-family launch, and
// the compiled general-cell VGL variants (for plans).
VghArgs vgh_args(const spline_s* s, const spline_tile& t, const double* pos, int64_t B, void* V, void* G, void* H);
std::vector<const VghVariant*> vgh_plan_variants(spline_dtype store);
bool vgh_variant_fits(const spline_s* s, const VghVariant& v);

}  // namespace qs

// Tile shapes compiled for the VGH family (at most four values per lane: the
// ten running sums per value take the registers the store kernels spend on
// wider tiles).
#define QS_VGH_SHAPES_F64(X, ST)                                                          \
    X(ST, 2, 1, 64) X(ST, 2, 2, 64) X(ST, 4, 1, 64) X(ST, 2, 3, 64) X(ST, 4, 2, 64)        \
    X(ST, 2, 1, 32) X(ST, 4, 1, 32) X(ST, 2, 1, 16) X(ST, 4, 1, 16)
#define QS_VGH_SHAPES_F32(X, ST)                                                          \
    X(ST, 1, 1, 64) X(ST, 1, 2, 64) X(ST, 2, 1, 64) X(ST, 1, 3, 64) X(ST, 3, 1, 64)        \
    X(ST, 4, 1, 64) X(ST, 2, 1, 32) X(ST, 4, 1, 32) X(ST, 2, 1, 16) X(ST, 4, 1, 16)        \
    X(ST, 1, 1, 16) X(ST, 3, 1, 16)
#define QS_VGH_SHAPES_16(X, ST)                                                           \
    X(ST, 1, 1, 64) X(ST, 1, 2, 64) X(ST, 2, 1, 64) X(ST, 1, 1, 32) X(ST, 2, 1, 32)        \
    X(ST, 1, 1, 16) X(ST, 2, 1, 16) X(ST, 3, 1, 16)

#define QS_VGH_VARIANTS(ST, CW, NCH, LPP)                                                 \
    {ST, CW, NCH, LPP, VGH_OUT_H, (const void*)&vgh_kernel<ST, CW, NCH, LPP, VGH_OUT_H>,   \
     sizeof(PosW<Acc<ST>::type>), nullptr},                                                \
    {ST, CW, NCH, LPP, VGH_OUT_L, (const void*)&vgh_kernel<ST, CW, NCH, LPP, VGH_OUT_L>,   \
     sizeof(PosW<Acc<ST>::type>), (const void*)&plan_vgh_kernel<ST, CW, NCH, LPP>},        \
    {ST, CW, NCH, LPP, VGH_OUT_RATIO,                                                      \
     (const void*)&vgh_kernel<ST, CW, NCH, LPP, VGH_OUT_RATIO>, sizeof(PosW<Acc<ST>::type>), nullptr},

#define QS_VGH_REGISTRY(NAME, LIST, ST)                                                   \
    static const VghVariant k_vgh_variants[] = {LIST(QS_VGH_VARIANTS, ST)};               \
    const VghVariant* NAME(int* count)                                                    \
    {                                                                                     \
        *count = (int)(sizeof(k_vgh_variants) / sizeof(k_vgh_variants[0]));               \
        return k_vgh_variants;                                                            \
    }
