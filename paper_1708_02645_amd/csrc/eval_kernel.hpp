// Tricubic B-spline orbital evaluation kernels for gfx950 (CDNA4).
//
// One workgroup (256 lanes) takes `pb` consecutive positions.
//  Phase 1: one lane per position reduces it to (cell index, fractional
//    offset) in FP64 and stages in LDS, per axis, the cubic B-spline weights,
//    the quadratic weights of first differences and the linear weights of
//    second differences (scaled to Cartesian units), plus the byte offset of
//    the stencil corner in the halo layout.
//  Phase 2: groups of LPP lanes (a whole wave for LPP = 64) take
//    (position, orbital tile) items.  The 16 (x,y) pairs are visited x-major;
//    for each pair the group reads the 4 consecutive z rows of its tile: every
//    lane loads NCH chunks of CW dwords, lanes adjacent in memory, so each
//    chunk load of a wave is one contiguous LPP*CW*4-byte segment.  While one
//    pair is folded the loads of the next are in flight (two register
//    buffers).
//
// Contraction order and form: z, then y, then x.  Derivatives are taken in
// difference form -- the derivative of a cubic B-spline is the quadratic
// B-spline of first differences of the coefficients, the second derivative
// the linear B-spline of second differences -- and every partially smoothed
// value is carried as (raw anchor coefficient, small correction), so each
// derivative sum is built from differences of raw coefficients.  FP32
// rounding then scales with the variation of the data across the 4x4x4
// stencil instead of its magnitude, which matters for the Laplacian: its
// weights are O(n^2) while the result is much smaller.  Weights are
// wave-uniform for LPP = 64 and live in scalar registers.  No matrix cores:
// about 400 flop per orbital-VGL against 64 coefficient reads makes this a
// bandwidth-bound gather.
//
// Memory order of a row: orbital fastest; per tile, chunk c of lane l
// covers orbitals tile*TO + c*LPP*VPC + l*VPC + [0, VPC).
#pragma once

#include "common.hpp"

namespace qs {

template <spline_dtype S> struct Acc { using type = float; };
template <> struct Acc<SPL_F64> { using type = double; };

template <spline_dtype S> constexpr int vals_per_chunk(int cw)
{
    return S == SPL_F64 ? cw / 2 : (S == SPL_F32 ? cw : 2 * cw);
}

// Per-position weights staged in LDS.  Axis d: cubic weights b[0..3];
// quadratic weights of first differences q[0..2] times g_d = n_d / cell_d;
// linear weights of second differences l[0..1] times g_d^2.
template <typename TA> struct alignas(16) PosW {
    TA w[3][9];
    int64_t off;  // byte offset of the stencil corner row (halo indices i0, i1, i2)
    int64_t row;  // row of pos and of the outputs this position maps to
};

// Weights of one axis at offset t.  b: uniform cubic B-spline; the
// derivative of sum_k b_k c_k is sum_k q_k (c_{k+1} - c_k) and the second
// derivative sum_k l_k (c_{k+2} - 2 c_{k+1} + c_k).
template <typename T>
__device__ inline void axis_weights(T t, T g, T g2, T* w)
{
    const T s = T(1) - t;
    const T t2 = t * t, s2 = s * s;
    w[0] = s2 * s * T(1.0 / 6.0);
    w[1] = T(2.0 / 3.0) + t2 * (T(0.5) * t - T(1));
    w[2] = T(1.0 / 6.0) + T(0.5) * (t + t2 - t2 * t);
    w[3] = t2 * t * T(1.0 / 6.0);
    w[4] = T(0.5) * s2 * g;
    w[5] = (T(0.5) + t - t2) * g;
    w[6] = T(0.5) * t2 * g;
    w[7] = s * g2;
    w[8] = t * g2;
}

// FP64 lattice reduction of one coordinate: periodic wrap, lower cell,
// clamp to [0, n-1]; non-finite input gives cell 0 and t = NaN.  In a general
// cell the coordinate is the fractional one and cell = 1.
__device__ inline void lattice_reduce(double r, double cell, int n, int& i, double& t)
{
    if (!__builtin_isfinite(r)) {
        i = 0;
        t = __builtin_nan("");
        return;
    }
    double f = r / cell;
    f = f - floor(f);
    if (f >= 1.0) f = 0.0;
    const double u = (double)n * f;
    int ii = (int)floor(u);
    ii = ii > n - 1 ? n - 1 : (ii < 0 ? 0 : ii);
    i = ii;
    t = u - (double)ii;
}

template <typename TA>
__device__ inline void stage_position(const EvalArgs& a, int64_t b, PosW<TA>& w)
{
    int i[3];
    double r[3];
    const int64_t row = a.idx ? (int64_t)a.idx[b] : b;
#pragma unroll
    for (int d = 0; d < 3; ++d) r[d] = a.pos[3 * row + d];  // all three loads in flight together
    if (a.general) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double u = r[0] * a.ilat[d] + r[1] * a.ilat[3 + d] + r[2] * a.ilat[6 + d];
            double t;
            lattice_reduce(u, 1.0, a.n[d], i[d], t);
            axis_weights<TA>((TA)t, TA(1), TA(1), w.w[d]);
        }
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double t;
            lattice_reduce(r[d], a.cell[d], a.n[d], i[d], t);
            const double g = (double)a.n[d] / a.cell[d];
            axis_weights<TA>((TA)t, (TA)g, (TA)(g * g), w.w[d]);
        }
    }
    w.off = (int64_t)i[0] * a.xstride + (int64_t)i[1] * a.ystride + (int64_t)i[2] * a.row_bytes;
    w.row = row;
}

template <typename T> __device__ inline T uniform(T x);
template <> __device__ inline float uniform<float>(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
template <> __device__ inline int uniform<int>(int x) { return __builtin_amdgcn_readfirstlane(x); }
template <> __device__ inline int64_t uniform<int64_t>(int64_t x)
{
    const uint64_t u = (uint64_t)x;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <> __device__ inline double uniform<double>(double x)
{
    return __builtin_bit_cast(double, (uint64_t)uniform<int64_t>(__builtin_bit_cast(int64_t, x)));
}

// Materialise a value in a vector register at this point of the program.
// An empty volatile statement (no instruction, no memory access): it keeps the
// arithmetic of one pipeline stage from being sunk below the next stage's
// loads, which would keep every loaded value live at once.
template <typename T> __device__ inline void pin(T& x) { asm volatile("" : "+v"(x)); }

template <int CW> struct Chunk { uint32_t w[CW]; };

template <int CW>
__device__ inline Chunk<CW> load_chunk(const unsigned char* p)
{
    Chunk<CW> c;
    if constexpr (CW == 4) {
        const uint4 v = *reinterpret_cast<const uint4*>(p);
        c.w[0] = v.x; c.w[1] = v.y; c.w[2] = v.z; c.w[3] = v.w;
    } else if constexpr (CW == 2) {
        const uint2 v = *reinterpret_cast<const uint2*>(p);
        c.w[0] = v.x; c.w[1] = v.y;
    } else {
        const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
#pragma unroll
        for (int i = 0; i < CW; ++i) c.w[i] = q[i];
    }
    return c;
}

// Raw words -> accumulation type.
template <spline_dtype S, int CW, typename TA>
__device__ inline void decode(const Chunk<CW>& c, TA* v)
{
    if constexpr (S == SPL_F32) {
#pragma unroll
        for (int i = 0; i < CW; ++i) v[i] = __builtin_bit_cast(float, c.w[i]);
    } else if constexpr (S == SPL_F64) {
#pragma unroll
        for (int i = 0; i < CW / 2; ++i)
            v[i] = __builtin_bit_cast(double, ((uint64_t)c.w[2 * i + 1] << 32) | c.w[2 * i]);
    } else if constexpr (S == SPL_BF16) {
#pragma unroll
        for (int i = 0; i < CW; ++i) {
            v[2 * i] = __builtin_bit_cast(float, c.w[i] << 16);
            v[2 * i + 1] = __builtin_bit_cast(float, c.w[i] & 0xffff0000u);
        }
    } else {
#pragma unroll
        for (int i = 0; i < CW; ++i) {
            v[2 * i] = (float)__builtin_bit_cast(_Float16, (uint16_t)(c.w[i] & 0xffffu));
            v[2 * i + 1] = (float)__builtin_bit_cast(_Float16, (uint16_t)(c.w[i] >> 16));
        }
    }
}

constexpr int pack_align(int bytes) { return (bytes & (bytes - 1)) == 0 ? (bytes > 16 ? 16 : bytes) : 4; }
template <typename TA, int N> struct alignas(pack_align(N * (int)sizeof(TA))) Pack { TA v[N]; };

// Store VPC consecutive values: one naturally aligned vector store when the
// caller guarantees alignment (row length a multiple of VPC) and the values
// are inside the row, element-wise otherwise.
template <typename TA, int VPC>
__device__ inline void store_vals(TA* dst, const TA* v, int o, int norb, bool aligned)
{
    if (aligned && o + VPC <= norb) {
        if constexpr (VPC == 2 || VPC == 4) {
            // outputs are written once and not read back here: non-temporal
            typedef TA vec __attribute__((ext_vector_type(VPC)));
            vec x;
#pragma unroll
            for (int i = 0; i < VPC; ++i) x[i] = v[i];
            __builtin_nontemporal_store(x, reinterpret_cast<vec*>(dst + o));
            return;
        }
        if constexpr (VPC == 1) {
            __builtin_nontemporal_store(v[0], dst + o);
            return;
        }
        Pack<TA, VPC> p;
#pragma unroll
        for (int i = 0; i < VPC; ++i) p.v[i] = v[i];
        *reinterpret_cast<Pack<TA, VPC>*>(dst + o) = p;
    } else {
#pragma unroll
        for (int i = 0; i < VPC; ++i)
            if (o + i < norb) dst[o + i] = v[i];
    }
}

// Load VPC consecutive values of a caller row, zero beyond norb: one
// naturally aligned vector load when `aligned` and inside the row.
template <typename TA, int VPC>
__device__ inline void load_vals(const TA* src, TA* v, int o, int norb, bool aligned)
{
    if (aligned && o + VPC <= norb) {
        const Pack<TA, VPC> p = *reinterpret_cast<const Pack<TA, VPC>*>(src + o);
#pragma unroll
        for (int i = 0; i < VPC; ++i) v[i] = p.v[i];
    } else {
#pragma unroll
        for (int i = 0; i < VPC; ++i) v[i] = o + i < norb ? src[o + i] : TA(0);
    }
}

// Evaluates positions [b0, b0 + np) of one table with the whole workgroup.
// W: LDS staging for at least a.pb positions.  Contains one workgroup barrier
// (between staging and evaluation), two with RATIO; callers that reuse W must
// barrier again.
//
// RATIO: instead of storing the orbital values, dot them with the caller's
// row of the inverse Slater matrix (the determinant lemma: the ratio of the
// determinants after and before moving one electron is the dot product of
// that electron's row of A^-1 with the orbital values at the new position,
// and the same dot product with gradients and Laplacians gives the
// derivatives).  Each lane forms its partial sums in registers, the LPP lanes
// of a group combine them by a butterfly of cross-lane exchanges, and the
// per-tile sums of a position are added in tile order after a barrier, so
// the result does not depend on which group took which tile.  NQ = 5 (VGL)
// or 1 (value) sums per position are written to a.V[row][NQ].
template <spline_dtype S, int CW, int NCH, int LPP, bool VGL, bool RATIO = false>
__device__ inline void eval_block(const EvalArgs& a, int64_t b0, int np, PosW<typename Acc<S>::type>* W)
{
    using TA = typename Acc<S>::type;
    constexpr int VPC = vals_per_chunk<S>(CW);  // values per chunk per lane
    constexpr int VPL = VPC * NCH;              // values per lane
    constexpr int CHB = CW * 4;                 // chunk bytes per lane
    constexpr int GCB = LPP * CHB;              // bytes per group chunk
    constexpr int TB = GCB * NCH;               // tile bytes
    constexpr int TO = LPP * VPL;               // tile orbitals
    static_assert(VPC >= 1, "chunk narrower than one value");

    const int tid = threadIdx.x;
    for (int p = tid; p < np; p += kBlock) stage_position<TA>(a, b0 + p, W[p]);
    __syncthreads();

    constexpr int groups = kBlock / LPP;
    const int g = tid / LPP;
    const int lane = tid % LPP;
    const int items = np * a.tiles;
    const uint32_t loff = (uint32_t)lane * CHB;
    constexpr int NQ = VGL ? 5 : 1;
    // RATIO: per-(position, tile) sums, in LDS after the staged weights.
    TA* part = reinterpret_cast<TA*>(W + a.pb);
    bool row_aligned = false;
    if constexpr (RATIO)
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

        // Tiles divide the row exactly (checked on the host), so every chunk
        // is inside the table.
        // LPP = 64: the row address is wave-uniform (scalar registers) and each
        // lane adds its 32-bit offset.  Otherwise each lane keeps one 64-bit
        // address for its item and adds the wave-uniform row offset: one
        // vector add per row.
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

        // Every smoothed quantity is carried as (raw anchor coefficient,
        // correction): z level anchored at z = 1, y level at y = 0, x level at
        // x = 0.  All derivative sums are then built from differences of raw
        // coefficients or of corrections, so FP32 rounding scales with the
        // variation of the data across the stencil, not with its magnitude.
        //
        // Running x-level state.
        TA vx[VPL], gxa[VPL], lxx[VPL], hxp[VPL], uxp[VPL], dxp[VPL];
        // y-level sums carried across x: d/dy, d/dz and the y,z Laplacian parts.
        TA gya[VPL], gza[VPL], lyz[VPL];
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            vx[v] = gxa[v] = lxx[v] = hxp[v] = uxp[v] = dxp[v] = TA(0);
            gya[v] = gza[v] = lyz[v] = TA(0);
        }
        // z weights of the anchored value: s0 = c1 + wa0 d0 + wa1 d1 + wa2 d2.
        const TA wa0 = -wz[0], wa1 = wz[2] + wz[3], wa2 = wz[3];
        // Tail sums of the cubic weights, c_k = b_k + ... + b_3 (c_0 = 1): a
        // smoothed value sum_k b_k f_k equals f_0 + sum_{k>=1} c_k (f_k - f_{k-1}),
        // so the y and x levels smooth values from the same first differences
        // their derivative sums use.
        const TA cy3 = wy[3], cy2 = wy[2] + cy3, cy1 = wy[1] + cy2;
        const TA cy[4] = {TA(1), cy1, cy2, cy3};
        TA cx[4];
        cx[3] = (LPP == 64) ? uniform<TA>(w.w[0][3]) : w.w[0][3];
#pragma unroll
        for (int k = 2; k >= 1; --k) cx[k] = ((LPP == 64) ? uniform<TA>(w.w[0][k]) : w.w[0][k]) + cx[k + 1];
        cx[0] = TA(1);

        // Software pipeline over the 16 pairs (x-major), fully unrolled so that
        // every weight index is static: the loads of pair xy+1 are issued, then
        // pair xy is folded.  The scheduling fences keep that order (otherwise
        // the scheduler hoists many pairs' loads and trades occupancy for it).
        Chunk<CW> buf[2][4][NCH];
        issue(0, buf[0]);
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            // Running y-level state of this x.
            TA h0[VPL], hp[VPL], lp[VPL], ep[VPL], ul[VPL], uy[VPL], uyy[VPL], t1[VPL], t2[VPL];
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
                    const TA hz = c[1][v];  // z anchor
                    TA lz = wa0 * d0;       // z-smoothed value = hz + lz
                    lz = fma(wa1, d1, lz);
                    lz = fma(wa2, d2, lz);
                    TA s1 = TA(0), s2 = TA(0);
                    if constexpr (VGL) {
                        s1 = wz[4] * d0;
                        s1 = fma(wz[5], d1, s1);
                        s1 = fma(wz[6], d2, s1);
                        s2 = wz[7] * (d1 - d0);
                        s2 = fma(wz[8], d2 - d1, s2);
                    }
                    if (y == 0) {
                        h0[v] = hz;
                        ul[v] = lz;  // s0[0] = h0 + ul
                        if constexpr (VGL) {
                            t1[v] = wy[0] * s1;
                            t2[v] = wy[0] * s2;
                        }
                    } else {
                        const TA e = (hz - hp[v]) + (lz - lp[v]);  // s0[y] - s0[y-1]
                        ul[v] = fma(cy[y], e, ul[v]);
                        if constexpr (VGL) {
                            t1[v] = fma(wy[y], s1, t1[v]);
                            t2[v] = fma(wy[y], s2, t2[v]);
                            if (y == 1) {
                                uy[v] = wy[4] * e;
                            } else {
                                uy[v] = fma(wy[4 + y - 1], e, uy[v]);
                                if (y == 2) uyy[v] = wy[7] * (e - ep[v]);
                                else uyy[v] = fma(wy[8], e - ep[v], uyy[v]);
                            }
                            ep[v] = e;
                            pin(uy[v]);
                            pin(ep[v]);
                            pin(t1[v]);
                            pin(t2[v]);
                        }
                    }
                    hp[v] = hz;
                    lp[v] = lz;
                    pin(ul[v]);
                    pin(hp[v]);
                    pin(lp[v]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }

            // Fold this x into the running sums.  u = h0 + ul is the
            // y,z-smoothed value at this x; the value is u[0] plus the tail
            // weights times the differences u[x] - u[x-1].
            [[maybe_unused]] const TA bx = (LPP == 64) ? uniform<TA>(w.w[0][x]) : w.w[0][x];
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                TA d = TA(0);
                if (x == 0) {
                    vx[v] = h0[v] + ul[v];
                } else {
                    d = (h0[v] - hxp[v]) + (ul[v] - uxp[v]);  // u[x] - u[x-1]
                    vx[v] = fma(cx[x], d, vx[v]);
                }
                if constexpr (VGL) {
                    gya[v] = fma(bx, uy[v], gya[v]);
                    gza[v] = fma(bx, t1[v], gza[v]);
                    lyz[v] = fma(bx, uyy[v] + t2[v], lyz[v]);
                    if (x >= 1) {
                        const TA qx = (LPP == 64) ? uniform<TA>(w.w[0][4 + x - 1]) : w.w[0][4 + x - 1];
                        gxa[v] = fma(qx, d, gxa[v]);
                        if (x >= 2) {
                            const TA lx = (LPP == 64) ? uniform<TA>(w.w[0][7 + x - 2]) : w.w[0][7 + x - 2];
                            lxx[v] = fma(lx, d - dxp[v], lxx[v]);
                        }
                        dxp[v] = d;
                    }
                }
                hxp[v] = h0[v];
                uxp[v] = ul[v];
            }
        }
        TA acc[5][VPL];
#pragma unroll
        for (int v = 0; v < VPL; ++v) {
            acc[0][v] = vx[v];
            acc[1][v] = gxa[v];
            acc[2][v] = gya[v];
            acc[3][v] = gza[v];
            acc[4][v] = lxx[v] + lyz[v];
        }

        const int64_t b = w.row;
        if constexpr (RATIO) {
            const int64_t arow = a.arows ? (int64_t)a.arows[b] : b;
            const TA* ar = reinterpret_cast<const TA*>(a.ainv) + arow * a.ald;
            TA sum[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) sum[q] = TA(0);
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                const int o = tile * TO + c * LPP * VPC + lane * VPC;
                TA av[VPC];
                load_vals<TA, VPC>(ar, av, o, a.norb, row_aligned);
                if constexpr (S == SPL_BF16 || S == SPL_F16) {
                    // power-of-two scales: a*(s*x) == (a*s)*x exactly
#pragma unroll
                    for (int i = 0; i < VPC; ++i) av[i] *= a.scales[o + i];
                }
#pragma unroll
                for (int q = 0; q < NQ; ++q)
#pragma unroll
                    for (int i = 0; i < VPC; ++i) sum[q] = fma(av[i], acc[q][c * VPC + i], sum[q]);
            }
#pragma unroll
            for (int m = LPP / 2; m >= 1; m >>= 1)
#pragma unroll
                for (int q = 0; q < NQ; ++q) sum[q] += __shfl_xor(sum[q], m, LPP);
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) part[(p * a.tiles + tile) * NQ + q] = sum[q];
            }
            continue;
        }
        TA* Vo = reinterpret_cast<TA*>(a.V) + b * a.norb;
        TA* Gx = reinterpret_cast<TA*>(a.G) + (3 * b) * a.norb;
        TA* Gy = Gx + a.norb;
        TA* Gz = Gy + a.norb;
        TA* Lo = reinterpret_cast<TA*>(a.L) + b * a.norb;
        const bool aligned = (a.norb % VPC) == 0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int o = tile * TO + c * LPP * VPC + lane * VPC;
            if (o >= a.norb) continue;
            TA* r[5] = {Vo, Gx, Gy, Gz, Lo};
            if constexpr (S == SPL_BF16 || S == SPL_F16) {
                TA sc[VPC];
#pragma unroll
                for (int i = 0; i < VPC; ++i) sc[i] = a.scales[o + i];  // n_pad entries: always in range
#pragma unroll
                for (int q = 0; q < (VGL ? 5 : 1); ++q)
#pragma unroll
                    for (int i = 0; i < VPC; ++i) acc[q][c * VPC + i] *= sc[i];
            }
#pragma unroll
            for (int q = 0; q < (VGL ? 5 : 1); ++q) store_vals<TA, VPC>(r[q], &acc[q][c * VPC], o, a.norb, aligned);
        }
    }
    if constexpr (RATIO) {
        __syncthreads();
        for (int p = tid; p < np; p += kBlock) {
            TA sum[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) sum[q] = part[p * a.tiles * NQ + q];
            for (int t = 1; t < a.tiles; ++t)
#pragma unroll
                for (int q = 0; q < NQ; ++q) sum[q] += part[(p * a.tiles + t) * NQ + q];
            TA* D = reinterpret_cast<TA*>(a.V) + W[p].row * NQ;
#pragma unroll
            for (int q = 0; q < NQ; ++q) D[q] = sum[q];
        }
    }
}

// One table: workgroup i takes positions [i*pb, i*pb + pb).
template <spline_dtype S, int CW, int NCH, int LPP, bool VGL, bool RATIO = false>
__global__ __launch_bounds__(kBlock) void eval_kernel(EvalArgs a)
{
    using TA = typename Acc<S>::type;
    extern __shared__ unsigned char lds_raw[];
    PosW<TA>* W = reinterpret_cast<PosW<TA>*>(lds_raw);
    const int64_t b0 = (int64_t)blockIdx.x * a.pb;
    int64_t B = a.B;
    if (a.nidx) {
        const int64_t c = *a.nidx;
        B = c < B ? c : B;
    }
    const int64_t rem = B - b0;
    if (rem <= 0) return;  // whole workgroup beyond a device-side count
    const int np = rem < a.pb ? (int)rem : a.pb;
    eval_block<S, CW, NCH, LPP, VGL, RATIO>(a, b0, np, W);
}

// Several tables in one launch (ragged batches): a persistent grid pops
// tasks (table, first position, count <= pb) from device counters until the
// list is exhausted.  With nseg = 8 the list is cut into eight contiguous
// segments and workgroup i starts on segment i mod 8 (workgroups are
// dispatched to the eight XCDs in turn), so tasks that are neighbours in the
// list (in a locality-ordered plan: positions sharing table rows) run on one
// XCD and share its L2; a workgroup whose segment is exhausted moves on to
// the next one.  Every workgroup exits once it has found all nseg segments
// exhausted, so the grid always drains.  The counters must be zero at launch
// (plan_reset_kernel, captured in the same graph).
template <spline_dtype S, int CW, int NCH, int LPP>
__global__ __launch_bounds__(kBlock) void plan_kernel(PlanArgs pa)
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
            const EvalArgs a = pa.tabs[tk.table];
            eval_block<S, CW, NCH, LPP, true>(a, tk.first, tk.count, W);
            __syncthreads();  // W is rewritten by the next task
        }
    }
}

}  // namespace qs
