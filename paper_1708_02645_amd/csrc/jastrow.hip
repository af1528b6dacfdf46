// One- and two-body Jastrow factors with 1D cubic B-spline functors, and
// distance-table rows, for gfx950.
//
// Every kernel stages the functor coefficients and the ion positions in LDS
// (a few KB, shared by all walkers).  Pair terms are computed on the fly
// from structure-of-arrays electron positions: lanes of a wave take
// consecutive electrons, so every position load is one contiguous segment.
//  - move:     one wave per proposed move; each lane sums, over its
//              electrons and ions, U(new) - U(old) and the derivative terms
//              at the new position; a butterfly across the wave combines
//              the lanes in a fixed order.
//  - evaluate: one workgroup per walker; the walker's positions sit in LDS
//              and each thread owns electrons, looping over all partners
//              (every pair is formed twice, once from each side, so no
//              thread writes another's sums).
//  - rows:     one wave per position, lanes over partners, coalesced SoA
//              stores.
// FP32 throughout (positions, distances, sums).
#include <cmath>
#include <cstring>
#include <limits>
#include <type_traits>
#include <vector>

#include "../../include/qmcjastrow.h"

#include "common.hpp"

namespace qs {

constexpr int kJThreads = 256;
constexpr int kMaxSpecies = 16;
constexpr int kMaxIntervals = 256;
constexpr int kMaxIons = 1024;
constexpr int kMaxElecEval = 2048;  // jastrow_evaluate keeps a walker in LDS
constexpr int kJEvalMaxThreads = 1024;  // jastrow_evaluate: one thread per electron up to this

struct JFun {
    float rcut, hinv;
    int32_t m, off;  // intervals, first coefficient
};

struct JArgs {
    const JFun* fun;      // [nf]
    const float* coefs;   // [ncoef]
    const float* ion;     // [3][nip]
    const int32_t* spec;  // [nip]
    int32_t nf, ncoef, n_ion, nip, n_elec, n_up, ns;
    float L[3], Linv[3];
};

struct JStage {
    const JFun* fun;  // LDS
    float* coefs;
    float* ix;
    float* iy;
    float* iz;
    int32_t* isp;
};

// Copies functors and ions into LDS (whole workgroup; ends with a barrier).
__device__ inline void j_stage(const JArgs& a, unsigned char* lds, JStage& st)
{
    JFun* f = reinterpret_cast<JFun*>(lds);
    st.coefs = reinterpret_cast<float*>(f + a.nf);
    st.ix = st.coefs + a.ncoef;
    st.iy = st.ix + a.n_ion;
    st.iz = st.iy + a.n_ion;
    st.isp = reinterpret_cast<int32_t*>(st.iz + a.n_ion);
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < a.nf; i += nt) f[i] = a.fun[i];
    for (int i = tid; i < a.ncoef; i += nt) st.coefs[i] = a.coefs[i];
    for (int i = tid; i < a.n_ion; i += nt) {
        st.ix[i] = a.ion[i];
        st.iy[i] = a.ion[a.nip + i];
        st.iz[i] = a.ion[2 * a.nip + i];
        st.isp[i] = a.spec[i];
    }
    __syncthreads();
    st.fun = f;
}

__device__ inline float min_image(float d, float L, float Linv) { return d - L * rintf(d * Linv); }

// Basis of functor f at distance r: first coefficient and cubic weights.
// Branch-free: beyond the cutoff the interval index is clamped and `inside`
// is false (the caller zeroes the terms).
struct FBasis {
    const float* c;
    float x, s;
    bool inside;
};

__device__ inline FBasis fbasis(const JFun& f, const float* coefs, float r)
{
    FBasis b;
    const float t = r * f.hinv;
    int i = (int)t;
    i = i > f.m - 1 ? f.m - 1 : i;
    b.x = t - (float)i;
    b.s = 1.f - b.x;
    b.c = coefs + f.off + i;
    b.inside = r < f.rcut;
    return b;
}

// U only.
__device__ inline float fvalue(const JFun& f, const float* coefs, float r)
{
    const FBasis b = fbasis(f, coefs, r);
    const float x = b.x, s = b.s, x2 = x * x;
    const float u = (s * s * s) * (1.f / 6.f) * b.c[0] + (2.f / 3.f + x2 * (0.5f * x - 1.f)) * b.c[1] +
                    (1.f / 6.f + 0.5f * (x + x2 - x2 * x)) * b.c[2] + (x2 * x) * (1.f / 6.f) * b.c[3];
    return b.inside ? u : 0.f;
}

// U, U', U'' (derivatives from differences of the coefficients: the
// quadratic and linear B-splines of first and second differences).
__device__ inline void functor(const JFun& f, const float* coefs, float r, float& u, float& du, float& d2u)
{
    const FBasis b = fbasis(f, coefs, r);
    const float x = b.x, s = b.s, x2 = x * x;
    const float c0 = b.c[0], c1 = b.c[1], c2 = b.c[2], c3 = b.c[3];
    const float v = (s * s * s) * (1.f / 6.f) * c0 + (2.f / 3.f + x2 * (0.5f * x - 1.f)) * c1 +
                    (1.f / 6.f + 0.5f * (x + x2 - x2 * x)) * c2 + (x2 * x) * (1.f / 6.f) * c3;
    const float d0 = c1 - c0, d1 = c2 - c1, d2 = c3 - c2;
    const float g = f.hinv * (0.5f * s * s * d0 + (0.5f + x - x2) * d1 + 0.5f * x2 * d2);
    const float h = f.hinv * f.hinv * (s * (d1 - d0) + x * (d2 - d1));
    u = b.inside ? v : 0.f;
    du = b.inside ? g : 0.f;
    d2u = b.inside ? h : 0.f;
}

// Distance and its reciprocal from a displacement (hardware reciprocal
// square root; 0 and 0 for a zero displacement).
__device__ inline float pair_dist(float dx, float dy, float dz, float& rinv)
{
    const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float ri = __builtin_amdgcn_rsqf(d2);
    const bool nz = d2 > 0.f;
    rinv = nz ? ri : 0.f;
    return nz ? d2 * ri : 0.f;
}

// Adds the pair term of electron e at (dx, dy, dz) = r_e - r_other: U to v,
// U' (dx, dy, dz) / d to the gradient and U'' + 2 U' / d to the Laplacian
// (a zero distance adds U(0) only).
__device__ inline void pair_terms(const JFun& f, const float* coefs, float dx, float dy, float dz, float& v,
                                  float& gx, float& gy, float& gz, float& lap)
{
    float rinv;
    const float d = pair_dist(dx, dy, dz, rinv);
    float u, du, d2u;
    functor(f, coefs, d, u, du, d2u);
    v += u;
    const float q = du * rinv;
    gx = fmaf(q, dx, gx);
    gy = fmaf(q, dy, gy);
    gz = fmaf(q, dz, gz);
    lap += (rinv > 0.f ? d2u : 0.f) + 2.f * q;
}

// U of the pair at (dx, dy, dz).
__device__ inline float pair_value(const JFun& f, const float* coefs, float dx, float dy, float dz)
{
    float rinv;
    return fvalue(f, coefs, pair_dist(dx, dy, dz, rinv));
}

__device__ inline float wave_sum(float x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

struct MoveArgs {
    JArgs j;
    const float* R;
    int64_t ld, wstride;
    const int32_t* walkers;
    const int32_t* k;
    const double* rnew;
    int64_t count;
    float* out;
};

__global__ __launch_bounds__(kJThreads) void jastrow_move_kernel(MoveArgs a)
{
    extern __shared__ unsigned char lds[];
    JStage st;
    j_stage(a.j, lds, st);
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * (kJThreads / 64) + (threadIdx.x >> 6);
    if (s >= a.count) return;
    const int k = a.k[s];
    float* o = a.out + 5 * s;
    const int64_t w = a.walkers ? (int64_t)a.walkers[s] : s;
    if (k < 0 || k >= a.j.n_elec || w < 0) {
        if (lane < 5) o[lane] = __builtin_nanf("");
        return;
    }
    const float* Rx = a.R + w * a.wstride;
    const float* Ry = Rx + a.ld;
    const float* Rz = Ry + a.ld;
    const float xo = Rx[k], yo = Ry[k], zo = Rz[k];
    const float xn = (float)a.rnew[3 * s], yn = (float)a.rnew[3 * s + 1], zn = (float)a.rnew[3 * s + 2];
    const float L0 = a.j.L[0], L1 = a.j.L[1], L2 = a.j.L[2];
    const float I0 = a.j.Linv[0], I1 = a.j.Linv[1], I2 = a.j.Linv[2];
    float dv = 0.f, gx = 0.f, gy = 0.f, gz = 0.f, lap = 0.f;
    const bool up_k = k < a.j.n_up;
    const JFun fsame = st.fun[a.j.ns], fdiff = st.fun[a.j.ns + 1];
    for (int i = lane; i < a.j.n_elec; i += 64) {
        if (i == k) continue;
        const float xi = Rx[i], yi = Ry[i], zi = Rz[i];
        const JFun& f = ((i < a.j.n_up) == up_k) ? fsame : fdiff;
        float vn = 0.f;
        pair_terms(f, st.coefs, min_image(xn - xi, L0, I0), min_image(yn - yi, L1, I1), min_image(zn - zi, L2, I2),
                   vn, gx, gy, gz, lap);
        const float vo = pair_value(f, st.coefs, min_image(xo - xi, L0, I0), min_image(yo - yi, L1, I1),
                                    min_image(zo - zi, L2, I2));
        dv += vn - vo;
    }
    for (int I = lane; I < a.j.n_ion; I += 64) {
        const JFun& f = st.fun[st.isp[I]];
        float vn = 0.f;
        pair_terms(f, st.coefs, min_image(xn - st.ix[I], L0, I0), min_image(yn - st.iy[I], L1, I1),
                   min_image(zn - st.iz[I], L2, I2), vn, gx, gy, gz, lap);
        const float vo = pair_value(f, st.coefs, min_image(xo - st.ix[I], L0, I0), min_image(yo - st.iy[I], L1, I1),
                                    min_image(zo - st.iz[I], L2, I2));
        dv += vn - vo;
    }
    dv = wave_sum(dv);
    gx = wave_sum(gx);
    gy = wave_sum(gy);
    gz = wave_sum(gz);
    lap = wave_sum(lap);
    if (lane == 0) {
        o[0] = dv;
        o[1] = gx;
        o[2] = gy;
        o[3] = gz;
        o[4] = lap;
    }
}

struct EvalJArgs {
    JArgs j;
    const float* R;
    int64_t ld, wstride, W;
    float* J;
    float* G;
    float* L;
};

// One workgroup per walker with one thread per electron (whole waves,
// at most kJEvalMaxThreads), so every thread runs the same partner loops.
__global__ __launch_bounds__(kJEvalMaxThreads) void jastrow_eval_kernel(EvalJArgs a)
{
    extern __shared__ unsigned char lds[];
    JStage st;
    const int N = a.j.n_elec;
    // walker positions, (x, y, z, 0) per electron, after the staged functors and ions
    j_stage(a.j, lds, st);
    float4* p = reinterpret_cast<float4*>(lds + ((reinterpret_cast<uintptr_t>(st.isp + a.j.n_ion) -
                                                  reinterpret_cast<uintptr_t>(lds) + 15) & ~uintptr_t(15)));
    __shared__ float red[kJEvalMaxThreads / 64];
    const int nt = blockDim.x;
    const int64_t w = blockIdx.x;
    const float* Rx = a.R + w * a.wstride;
    for (int i = threadIdx.x; i < N; i += nt) p[i] = make_float4(Rx[i], Rx[a.ld + i], Rx[2 * a.ld + i], 0.f);
    __syncthreads();
    const float L0 = a.j.L[0], L1 = a.j.L[1], L2 = a.j.L[2];
    const float I0 = a.j.Linv[0], I1 = a.j.Linv[1], I2 = a.j.Linv[2];
    const int nup = a.j.n_up;
    float jpart = 0.f;
    for (int i = threadIdx.x; i < N; i += nt) {
        const float4 pi = p[i];
        const bool up = i < nup;
        const JFun fsame = st.fun[a.j.ns], fdiff = st.fun[a.j.ns + 1];
        const JFun f_lo = up ? fsame : fdiff;  // partners 0..nup-1
        const JFun f_hi = up ? fdiff : fsame;  // partners nup..N-1
        float v1 = 0.f, v2 = 0.f, gx = 0.f, gy = 0.f, gz = 0.f, lap = 0.f;
        // The partner j = i is included: at distance 0 it adds U_same(0) to
        // v2 (removed below) and nothing to the derivatives.
        for (int j = 0; j < nup; ++j) {
            const float4 pj = p[j];
            pair_terms(f_lo, st.coefs, min_image(pi.x - pj.x, L0, I0), min_image(pi.y - pj.y, L1, I1),
                       min_image(pi.z - pj.z, L2, I2), v2, gx, gy, gz, lap);
        }
        for (int j = nup; j < N; ++j) {
            const float4 pj = p[j];
            pair_terms(f_hi, st.coefs, min_image(pi.x - pj.x, L0, I0), min_image(pi.y - pj.y, L1, I1),
                       min_image(pi.z - pj.z, L2, I2), v2, gx, gy, gz, lap);
        }
        v2 -= fvalue(fsame, st.coefs, 0.f);
        for (int I = 0; I < a.j.n_ion; ++I)
            pair_terms(st.fun[st.isp[I]], st.coefs, min_image(pi.x - st.ix[I], L0, I0),
                       min_image(pi.y - st.iy[I], L1, I1), min_image(pi.z - st.iz[I], L2, I2), v1, gx, gy, gz, lap);
        jpart += v1 + 0.5f * v2;
        float* Gw = a.G + w * 3 * (int64_t)N;
        Gw[i] = gx;
        Gw[N + i] = gy;
        Gw[2 * N + i] = gz;
        a.L[w * (int64_t)N + i] = lap;
    }
    jpart = wave_sum(jpart);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = jpart;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = red[0];
#pragma unroll
        for (int q = 1; q < nt / 64; ++q) t += red[q];
        a.J[w] = t;
    }
}

// Symmetric evaluation for n_elec <= kSymMaxElec: every unordered
// electron pair is formed once and its terms go to both electrons (the
// gradient with opposite signs).  The electrons are cut into nb blocks of 64,
// one wave each (lane l owns electron 64 I + l of block I).  Wave I visits
// the partner blocks J = I + delta (mod nb), delta = 0 .. nb/2; in block J
// its lane l meets electron 64 J + ((l + s) mod 64) at step s, so at every
// step the lanes meet 64 different partners: each lane adds the pair to its
// own row sums and the partner's share to the column sums it holds for that
// partner, which then move down one lane; at the end of the block they go
// to LDS.  The
// diagonal block takes steps 1..32 (step 32 on lanes 0..31 only), and when
// nb is even the block half-way round is split between its two waves (steps
// 0..31 from one side, 1..32 from the other, which are the pairs of steps
// 32..63 seen from the first).  Each wave then adds, in the order delta =
// 0 .. nb/2, the column sums destined for its block to its row sums: the
// result is deterministic.
constexpr int kSymMaxElec = 512;
constexpr int kSymMaxBlocks = kSymMaxElec / 64;

__device__ inline JFun jsel(bool c, const JFun& a, const JFun& b)
{
    JFun f;
    f.rcut = c ? a.rcut : b.rcut;
    f.hinv = c ? a.hinv : b.hinv;
    f.m = c ? a.m : b.m;
    f.off = c ? a.off : b.off;
    return f;
}

__global__ __launch_bounds__(kSymMaxElec) void jastrow_eval_sym_kernel(EvalJArgs a)
{
    extern __shared__ unsigned char lds[];
    JStage st;
    const int N = a.j.n_elec, nb = (N + 63) / 64, D = nb / 2;
    j_stage(a.j, lds, st);
    float4* p = reinterpret_cast<float4*>(lds + ((reinterpret_cast<uintptr_t>(st.isp + a.j.n_ion) -
                                                  reinterpret_cast<uintptr_t>(lds) + 15) & ~uintptr_t(15)));
    float4* col = p + 64 * nb;  // column sums [wave][delta 0..D][64]
    __shared__ float red[kSymMaxBlocks];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t w = blockIdx.x;
    const float* Rx = a.R + w * a.wstride;
    for (int i = tid; i < 64 * nb; i += blockDim.x)
        p[i] = i < N ? make_float4(Rx[i], Rx[a.ld + i], Rx[2 * a.ld + i], 0.f) : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    const float L0 = a.j.L[0], L1 = a.j.L[1], L2 = a.j.L[2];
    const float I0 = a.j.Linv[0], I1 = a.j.Linv[1], I2 = a.j.Linv[2];
    const int nup = a.j.n_up;
    const JFun fsame = st.fun[a.j.ns], fdiff = st.fun[a.j.ns + 1];
    const int e = 64 * wv + lane;  // this lane's electron
    const bool e_ok = e < N, e_up = e < nup;
    const float4 pe = p[e];
    float v = 0.f, gx = 0.f, gy = 0.f, gz = 0.f, lap = 0.f;
    for (int delta = 0; delta <= D; ++delta) {
        const int J = (wv + delta) % nb;
        int s0 = 0, s1 = 64;  // steps [s0, s1)
        if (delta == 0) {
            s0 = 1;
            s1 = 33;
        } else if (2 * delta == nb) {
            if (wv < D) s1 = 32;
            else {
                s0 = 1;
                s1 = 33;
            }
        }
        // Column sums in registers: at step s lane l holds those of partner
        // (l + s) mod 64; after each step they move down one lane, so lane l
        // then holds those of (l + s + 1) mod 64.
        float cx = 0.f, cy = 0.f, cz = 0.f, cw = 0.f;
        // One step.  MASK: some pair of the step may not exist (padding
        // electrons, the half last diagonal step); SEL: the partner block
        // holds both spins, so the functor is chosen per pair.
        auto step = [&](int s, auto mask_t, auto sel_t, const JFun& fblk) {
            constexpr bool MASK = decltype(mask_t)::value, SEL = decltype(sel_t)::value;
            const int c = (lane + s) & 63, b = 64 * J + c;
            const float4 pb = p[b];
            const JFun f = SEL ? jsel(e_up == (b < nup), fsame, fdiff) : fblk;
            const float dx = min_image(pe.x - pb.x, L0, I0), dy = min_image(pe.y - pb.y, L1, I1),
                        dz = min_image(pe.z - pb.z, L2, I2);
            float rinv;
            const float d = pair_dist(dx, dy, dz, rinv);
            float u, du, d2u;
            functor(f, st.coefs, d, u, du, d2u);
            float q = du * rinv;
            float lt = (rinv > 0.f ? d2u : 0.f) + 2.f * q;  // as pair_terms at distance 0
            if constexpr (MASK) {
                // the last diagonal step pairs lane l with l + 32 and l + 32 with l: keep one
                const bool ok = e_ok && b < N && !(delta == 0 && s == 32 && lane >= 32);
                q = ok ? q : 0.f;
                lt = ok ? lt : 0.f;
                u = ok ? u : 0.f;
            }
            v += u;
            gx = fmaf(q, dx, gx);
            gy = fmaf(q, dy, gy);
            gz = fmaf(q, dz, gz);
            lap += lt;
            cx = __shfl(fmaf(-q, dx, cx), lane + 1, 64);
            cy = __shfl(fmaf(-q, dy, cy), lane + 1, 64);
            cz = __shfl(fmaf(-q, dz, cz), lane + 1, 64);
            cw = __shfl(cw + lt, lane + 1, 64);
        };
        using T = std::true_type;
        using F = std::false_type;
        // wave-uniform: every electron of this wave and of block J exists, and
        // block J holds one spin only
        const bool full = 64 * wv + 64 <= N && 64 * J + 64 <= N;
        const bool mixed = 64 * J < nup && nup < 64 * J + 64;
        const JFun fblk = jsel(e_up == (64 * J < nup), fsame, fdiff);
        const int s_end = delta == 0 ? s1 - 1 : s1;  // the half last diagonal step is masked
        if (full && !mixed) {
            for (int s = s0; s < s_end; ++s) step(s, F(), F(), fblk);
        } else {
            for (int s = s0; s < s_end; ++s) step(s, T(), T(), fblk);
        }
        if (s_end < s1) step(s_end, T(), T(), fblk);
        col[(wv * (D + 1) + delta) * 64 + ((lane + s1) & 63)] = make_float4(cx, cy, cz, cw);
    }
    __syncthreads();
    // column sums destined for this wave's block, in the order delta = 0 .. D
    for (int delta = 0; delta <= D; ++delta) {
        const int I = (wv - delta + nb) % nb;
        const float4 cc = col[(I * (D + 1) + delta) * 64 + lane];
        gx += cc.x;
        gy += cc.y;
        gz += cc.z;
        lap += cc.w;
    }
    float v1 = 0.f;
    if (e_ok) {
        for (int I = 0; I < a.j.n_ion; ++I)
            pair_terms(st.fun[st.isp[I]], st.coefs, min_image(pe.x - st.ix[I], L0, I0),
                       min_image(pe.y - st.iy[I], L1, I1), min_image(pe.z - st.iz[I], L2, I2), v1, gx, gy, gz, lap);
        float* Gw = a.G + w * 3 * (int64_t)N;
        Gw[e] = gx;
        Gw[N + e] = gy;
        Gw[2 * N + e] = gz;
        a.L[w * (int64_t)N + e] = lap;
    }
    float jpart = wave_sum(v + v1);
    if (lane == 0) red[wv] = jpart;
    __syncthreads();
    if (tid == 0) {
        float t = red[0];
        for (int q = 1; q < nb; ++q) t += red[q];
        a.J[w] = t;
    }
}

struct RowArgs {
    JArgs j;
    const float* R;
    int64_t ld, wstride;
    const int32_t* walkers;
    const double* r;
    int64_t count;
    float *de, *dre, *di, *dri;
};

__global__ __launch_bounds__(kJThreads) void jastrow_rows_kernel(RowArgs a)
{
    extern __shared__ unsigned char lds[];
    JStage st;
    j_stage(a.j, lds, st);
    const int lane = threadIdx.x & 63;
    const int64_t s = (int64_t)blockIdx.x * (kJThreads / 64) + (threadIdx.x >> 6);
    if (s >= a.count) return;
    const int64_t w = a.walkers ? (int64_t)a.walkers[s] : s;
    const float* Rx = a.R + (w < 0 ? 0 : w) * a.wstride;
    const float x = (float)a.r[3 * s], y = (float)a.r[3 * s + 1], z = (float)a.r[3 * s + 2];
    const int N = a.j.n_elec, NI = a.j.n_ion;
    if (w < 0) {  // no such walker: its electron rows are NaN
        for (int i = lane; i < N; i += 64) {
            a.de[s * N + i] = __builtin_nanf("");
            a.dre[(3 * s) * N + i] = __builtin_nanf("");
            a.dre[(3 * s + 1) * N + i] = __builtin_nanf("");
            a.dre[(3 * s + 2) * N + i] = __builtin_nanf("");
        }
    }
    for (int i = lane; i < N && w >= 0; i += 64) {
        const float dx = min_image(Rx[i] - x, a.j.L[0], a.j.Linv[0]);
        const float dy = min_image(Rx[a.ld + i] - y, a.j.L[1], a.j.Linv[1]);
        const float dz = min_image(Rx[2 * a.ld + i] - z, a.j.L[2], a.j.Linv[2]);
        a.de[s * N + i] = sqrtf(dx * dx + dy * dy + dz * dz);
        a.dre[(3 * s) * N + i] = dx;
        a.dre[(3 * s + 1) * N + i] = dy;
        a.dre[(3 * s + 2) * N + i] = dz;
    }
    if (!a.di) return;
    for (int I = lane; I < NI; I += 64) {
        const float dx = min_image(st.ix[I] - x, a.j.L[0], a.j.Linv[0]);
        const float dy = min_image(st.iy[I] - y, a.j.L[1], a.j.Linv[1]);
        const float dz = min_image(st.iz[I] - z, a.j.L[2], a.j.Linv[2]);
        a.di[s * NI + I] = sqrtf(dx * dx + dy * dy + dz * dz);
        a.dri[(3 * s) * NI + I] = dx;
        a.dri[(3 * s + 1) * NI + I] = dy;
        a.dri[(3 * s + 2) * NI + I] = dz;
    }
}

__global__ void jastrow_accept_kernel(float* R, int64_t ld, int64_t wstride, const int32_t* walkers,
                                      const int32_t* k, const double* rnew, int64_t count, int32_t n_elec)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const int kk = k[s];
    const int64_t w = walkers ? (int64_t)walkers[s] : s;
    if (kk < 0 || kk >= n_elec || w < 0) return;
    float* Rx = R + w * wstride;
    Rx[kk] = (float)rnew[3 * s];
    Rx[ld + kk] = (float)rnew[3 * s + 1];
    Rx[2 * ld + kk] = (float)rnew[3 * s + 2];
}

static int64_t a256(int64_t x) { return (x + 255) & ~int64_t(255); }

struct JLayout {
    int64_t fun, coefs, ion, spec, total;
    int32_t nf, ncoef, nip;
};

static bool j_layout(const jastrow_desc* d, const int32_t* intervals, JLayout* L)
{
    if (!d || !intervals) return false;
    if (d->n_elec < 1 || d->n_up < 0 || d->n_up > d->n_elec || d->n_ion < 0 || d->n_ion > kMaxIons ||
        d->n_species < 1 || d->n_species > kMaxSpecies)
        return false;
    for (int a = 0; a < 3; ++a)
        if (!(d->cell[a] > 0.0) || !std::isfinite(d->cell[a])) return false;
    L->nf = d->n_species + 2;
    int64_t nc = 0;
    for (int f = 0; f < L->nf; ++f) {
        if (intervals[f] < 1 || intervals[f] > kMaxIntervals) return false;
        nc += intervals[f] + 3;
    }
    L->ncoef = (int32_t)nc;
    L->nip = (d->n_ion + 3) & ~3;
    L->fun = 0;
    L->coefs = a256(L->fun + (int64_t)sizeof(JFun) * L->nf);
    L->ion = a256(L->coefs + 4 * nc);
    L->spec = a256(L->ion + 4 * 3 * (int64_t)L->nip);
    L->total = a256(L->spec + 4 * (int64_t)L->nip);
    return true;
}

}  // namespace qs

struct jastrow_s {
    jastrow_desc d;
    qs::JLayout lay;
    unsigned char* dev;
    int device;
};

namespace qs {

static JArgs j_args(const jastrow_s* j)
{
    JArgs a{};
    a.fun = reinterpret_cast<const JFun*>(j->dev + j->lay.fun);
    a.coefs = reinterpret_cast<const float*>(j->dev + j->lay.coefs);
    a.ion = reinterpret_cast<const float*>(j->dev + j->lay.ion);
    a.spec = reinterpret_cast<const int32_t*>(j->dev + j->lay.spec);
    a.nf = j->lay.nf;
    a.ncoef = j->lay.ncoef;
    a.n_ion = j->d.n_ion;
    a.nip = j->lay.nip;
    a.n_elec = j->d.n_elec;
    a.n_up = j->d.n_up;
    a.ns = j->d.n_species;
    for (int d = 0; d < 3; ++d) {
        a.L[d] = (float)j->d.cell[d];
        a.Linv[d] = (float)(1.0 / j->d.cell[d]);
    }
    return a;
}

static size_t stage_bytes(const jastrow_s* j)
{
    return sizeof(JFun) * j->lay.nf + 4 * (size_t)j->lay.ncoef + 16 * (size_t)j->d.n_ion;
}

static int j_common(const jastrow_s* j, const float* R, int64_t ld, int64_t wstride)
{
    if (!j) return fail(SPL_EINVAL, "handle is NULL");
    if (!R) return fail(SPL_EINVAL, "positions are NULL");
    if (ld < j->d.n_elec || wstride < 3 * ld) return fail(SPL_EINVAL, "need ld >= n_elec and wstride >= 3*ld");
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    if (dev != j->device) return fail(SPL_EINVAL, "current HIP device differs from the Jastrow factor's device");
    return SPL_OK;
}

static unsigned grid_of(int64_t count, int per)
{
    return (unsigned)((count + per - 1) / per);
}

}  // namespace qs

using namespace qs;

extern "C" {

size_t jastrow_bytes(const jastrow_desc* d, const int32_t* intervals)
{
    JLayout L;
    return j_layout(d, intervals, &L) ? (size_t)L.total : 0;
}

int jastrow_create(const jastrow_desc* d, const double* ions, const int32_t* species, const int32_t* intervals,
                   const double* rcut, const double* coefs, void* dev, size_t bytes, void* stream, jastrow_t** out)
{
    if (!out) return fail(SPL_EINVAL, "out is NULL");
    *out = nullptr;
    JLayout L;
    if (!j_layout(d, intervals, &L)) return fail(SPL_EINVAL, "invalid Jastrow sizes or cell");
    if (!rcut || !coefs || (d->n_ion > 0 && (!ions || !species))) return fail(SPL_EINVAL, "NULL host array");
    if (!dev || (reinterpret_cast<uintptr_t>(dev) & 255)) return fail(SPL_EINVAL, "device buffer NULL or not 256-byte aligned");
    if (bytes < (size_t)L.total) return fail(SPL_ENOMEM, "device buffer smaller than jastrow_bytes()");
    const double half = 0.5 * std::min(d->cell[0], std::min(d->cell[1], d->cell[2]));
    std::vector<unsigned char> host((size_t)L.total, 0);
    JFun* fun = reinterpret_cast<JFun*>(host.data() + L.fun);
    float* cf = reinterpret_cast<float*>(host.data() + L.coefs);
    int64_t off = 0;
    for (int f = 0; f < L.nf; ++f) {
        if (!(rcut[f] > 0.0) || rcut[f] > half * (1.0 + 1e-12) || !std::isfinite(rcut[f]))
            return fail(SPL_EINVAL, "every cutoff must be in (0, min(cell)/2]");
        fun[f].rcut = (float)rcut[f];
        fun[f].hinv = (float)(intervals[f] / rcut[f]);
        fun[f].m = intervals[f];
        fun[f].off = (int32_t)off;
        for (int c = 0; c < intervals[f] + 3; ++c) {
            const double v = coefs[off + c];
            if (!std::isfinite(v)) return fail(SPL_EINVAL, "non-finite functor coefficient");
            cf[off + c] = (float)v;
        }
        off += intervals[f] + 3;
    }
    float* ion = reinterpret_cast<float*>(host.data() + L.ion);
    int32_t* sp = reinterpret_cast<int32_t*>(host.data() + L.spec);
    for (int i = 0; i < d->n_ion; ++i) {
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(ions[3 * i + a])) return fail(SPL_EINVAL, "non-finite ion position");
            ion[a * L.nip + i] = (float)ions[3 * i + a];
        }
        if (species[i] < 0 || species[i] >= d->n_species) return fail(SPL_EINVAL, "ion species out of range");
        sp[i] = species[i];
    }
    int devid = -1;
    QS_HIP(hipGetDevice(&devid));
    hipStream_t st = static_cast<hipStream_t>(stream);
    QS_HIP(hipMemcpyAsync(dev, host.data(), host.size(), hipMemcpyHostToDevice, st));
    QS_HIP(hipStreamSynchronize(st));
    jastrow_s* j = new (std::nothrow) jastrow_s;
    if (!j) return fail(SPL_ENOMEM, "handle allocation failed");
    j->d = *d;
    j->lay = L;
    j->dev = static_cast<unsigned char*>(dev);
    j->device = devid;
    *out = j;
    return SPL_OK;
}

int jastrow_destroy(jastrow_t* j)
{
    delete j;
    return SPL_OK;
}

int jastrow_move(const jastrow_t* j, const float* R_dev, int64_t ld, int64_t wstride, const int32_t* walkers,
                 const int32_t* k_dev, const double* rnew, int64_t count, float* out, void* stream)
{
    if (count < 0) return fail(SPL_EINVAL, "count must be >= 0");
    int rc = j_common(j, R_dev, ld, wstride);
    if (rc) return rc;
    if (count == 0) return SPL_OK;
    if (!k_dev || !rnew || !out) return fail(SPL_EINVAL, "NULL electron, position or output pointer");
    if (count > (int64_t)std::numeric_limits<int32_t>::max()) return fail(SPL_EINVAL, "count too large");
    MoveArgs a{j_args(j), R_dev, ld, wstride, walkers, k_dev, rnew, count, out};
    void* params[] = {&a};
    QS_HIP(hipLaunchKernel((const void*)&jastrow_move_kernel, dim3(grid_of(count, kJThreads / 64)), dim3(kJThreads),
                           params, stage_bytes(j), static_cast<hipStream_t>(stream)));
    QS_HIP(hipGetLastError());
    return SPL_OK;
}

int jastrow_evaluate(const jastrow_t* j, const float* R_dev, int64_t ld, int64_t wstride, int64_t W, float* J,
                     float* G, float* L, void* stream)
{
    if (W < 0) return fail(SPL_EINVAL, "W must be >= 0");
    int rc = j_common(j, R_dev, ld, wstride);
    if (rc) return rc;
    if (W == 0) return SPL_OK;
    if (!J || !G || !L) return fail(SPL_EINVAL, "NULL output pointer");
    if (j->d.n_elec > kMaxElecEval) return fail(SPL_EUNSUPPORTED, "jastrow_evaluate supports n_elec <= 2048");
    if (W > (int64_t)std::numeric_limits<int32_t>::max()) return fail(SPL_EINVAL, "W too large");
    EvalJArgs a{j_args(j), R_dev, ld, wstride, W, J, G, L};
    void* params[] = {&a};
    const size_t lds = stage_bytes(j) + 16 + 16 * (size_t)j->d.n_elec;
    const int threads = std::min(kJEvalMaxThreads, std::max(64, (j->d.n_elec + 63) / 64 * 64));
    const int nb = (j->d.n_elec + 63) / 64;
    // symmetric pairs: positions padded to whole blocks, then the column sums
    const size_t slds = stage_bytes(j) + 16 + 16 * 64 * (size_t)nb * (1 + (nb / 2 + 1));
    if (j->d.n_elec <= kSymMaxElec && slds <= 64 * 1024) {
        QS_HIP(hipLaunchKernel((const void*)&jastrow_eval_sym_kernel, dim3((unsigned)W), dim3(64 * nb), params, slds,
                               static_cast<hipStream_t>(stream)));
        QS_HIP(hipGetLastError());
        return SPL_OK;
    }
    QS_HIP(hipLaunchKernel((const void*)&jastrow_eval_kernel, dim3((unsigned)W), dim3(threads), params, lds,
                           static_cast<hipStream_t>(stream)));
    QS_HIP(hipGetLastError());
    return SPL_OK;
}

int jastrow_dist_rows(const jastrow_t* j, const float* R_dev, int64_t ld, int64_t wstride, const int32_t* walkers,
                      const double* r, int64_t count, float* de, float* dre, float* di, float* dri, void* stream)
{
    if (count < 0) return fail(SPL_EINVAL, "count must be >= 0");
    int rc = j_common(j, R_dev, ld, wstride);
    if (rc) return rc;
    if (count == 0) return SPL_OK;
    if (!r || !de || !dre) return fail(SPL_EINVAL, "NULL position or electron-row pointer");
    if (j->d.n_ion > 0 && (!di || !dri)) return fail(SPL_EINVAL, "NULL ion-row pointer");
    if (count > (int64_t)std::numeric_limits<int32_t>::max()) return fail(SPL_EINVAL, "count too large");
    RowArgs a{j_args(j), R_dev, ld, wstride, walkers, r, count, de, dre, j->d.n_ion > 0 ? di : nullptr, dri};
    void* params[] = {&a};
    QS_HIP(hipLaunchKernel((const void*)&jastrow_rows_kernel, dim3(grid_of(count, kJThreads / 64)), dim3(kJThreads),
                           params, stage_bytes(j), static_cast<hipStream_t>(stream)));
    QS_HIP(hipGetLastError());
    return SPL_OK;
}

int jastrow_accept(const jastrow_t* j, float* R_dev, int64_t ld, int64_t wstride, const int32_t* walkers,
                   const int32_t* k_dev, const double* rnew, int64_t count, void* stream)
{
    if (count < 0) return fail(SPL_EINVAL, "count must be >= 0");
    int rc = j_common(j, R_dev, ld, wstride);
    if (rc) return rc;
    if (count == 0) return SPL_OK;
    if (!k_dev || !rnew) return fail(SPL_EINVAL, "NULL electron or position pointer");
    if (count > (int64_t)std::numeric_limits<int32_t>::max()) return fail(SPL_EINVAL, "count too large");
    hipLaunchKernelGGL(jastrow_accept_kernel, dim3(grid_of(count, 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       R_dev, ld, wstride, walkers, k_dev, rnew, count, j->d.n_elec);
    QS_HIP(hipGetLastError());
    return SPL_OK;
}

}  // extern "C"
