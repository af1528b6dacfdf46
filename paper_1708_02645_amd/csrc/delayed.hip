// Delayed (Woodbury) update of inverse Slater matrices.
//
// Against a stale inverse A0^-1 (rows a_i), j accepted moves are kept
// pending: the orbital vectors phi_l of the moved electrons k_l and the
// inverse of S (S[i][l] = a_{k_i} . phi_l).  Then
//   ratio for electron k with orbital quantities q:  a_k . q - t^T S^-1 y,
//     t_i = a_k . phi_i,  y_i = a_{k_i} . q;
//   accepting it borders S^-1 with the Schur complement (= the ratio);
//   a flush applies  A0^-1 -= (A0^-1 Phi - Q) S^-1 R  (R = rows k_i of
//   A0^-1, Q = columns e_{k_i}) once for all pending moves.
// Per accepted move the inverse is read in j + 1 rows instead of read and
// written whole (Sherman-Morrison); the whole matrix is read twice and
// written once per flush.
//
// Workspace, per walker (floats unless noted): Phi [d][n], Sinv [d][d] (row
// i, column l at i*d + l), M [d][n], T [n][d], K [d] int32, count int32.
#include <algorithm>
#include <limits>

#include "common.hpp"

namespace qs {

constexpr int kDThreads = 256;
constexpr int kDMaxN = 2048;
constexpr int kDMaxDelay = 64;
constexpr size_t kDMaxLds = 64 * 1024;  // dynamic LDS per workgroup asked for by ratio / accept

struct DluLayout {
    int64_t phi, sinv, m, t, k, cnt, stride;  // offsets in 4-byte words, per-walker stride
};

// Every region starts on a 256-byte boundary (64 words), so rows of Phi and M
// can be moved with 16-byte accesses when n is a multiple of 4.
static int64_t dlu_pad(int64_t words) { return (words + 63) & ~int64_t(63); }

static DluLayout dlu_layout(int n, int d)
{
    DluLayout L;
    L.phi = 0;
    L.sinv = L.phi + dlu_pad((int64_t)d * n);
    L.m = L.sinv + dlu_pad((int64_t)d * d);
    L.t = L.m + dlu_pad((int64_t)d * n);
    L.k = L.t + dlu_pad((int64_t)n * d);
    L.cnt = L.k + dlu_pad(d);
    L.stride = L.cnt + 64;
    return L;
}

struct DluArgs {
    float* ws;
    DluLayout L;
    int32_t n, d;
    float* ainv;
    int64_t wstride;
    const int32_t* walkers;
    const int32_t* k;
    const float* V;
    const float* G;
    const float* L_;
    int64_t count;
    float* out;
    int32_t stage_sinv;  // ratio / accept: copy S^-1 to LDS first (when it fits beside the rest)
    int64_t nwalkers;    // walkers of the workspace: a slot's walker must be in [0, nwalkers)
    const int32_t* kacc; // accepting step: electron of the move accepted in slot s (< 0: none)
    const float* Vacc;   //   and its orbital values [count][n]
};

__device__ inline float dwave_sum(float x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// `total` dot products p1 . p2 -> *dst, the pointers of dot e from
// job(e, p1, p2, dst).  Each wave takes eight dots at a time and loads R
// 64-column steps of all eight before using any, so a dot costs about
// n / (64 R) memory round trips; every dot is accumulated over m = lane,
// lane + 64, ... in that order and reduced by a butterfly, the same order
// whichever wave and slot takes it, and whichever other dots share the pass.
template <int R, typename Job>
__device__ inline void dlu_dot_set(int n, int total, Job job)
{
    constexpr int U = 8;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int e0 = wave * U; e0 < total; e0 += (kDThreads / 64) * U) {
        const float* p1[U];
        const float* p2[U];
        float* dst[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            job(e0 + u < total ? e0 + u : total - 1, p1[u], p2[u], dst[u]);  // a repeated last dot is not stored twice
        float s[U] = {};
        for (int m0 = lane; m0 < n; m0 += 64 * R) {
            float v1[U][R], v2[U][R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int m = m0 + 64 * r;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    v1[u][r] = m < n ? p1[u][m] : 0.f;
                    v2[u][r] = m < n ? p2[u][m] : 0.f;
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (m0 + 64 * r < n) s[u] = fmaf(v1[u][r], v2[u][r], s[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float r = dwave_sum(s[u]);
            if (lane == 0 && e0 + u < total) *dst[u] = r;
        }
    }
}

// The dots of a ratio or an accept against j pending moves: x[q] = a . q_q,
// t[i] = a . phi_i, y[i][q] = a_{K_i} . q_q (dot e of NQ + j + j NQ).
template <int NQ>
__device__ inline void dlu_dot_job(int e, int n, int j, const float* A, const float* Phi, const int32_t* K,
                                   const float* as, const float* qs, float* x, float* t, float* y, const float*& p1,
                                   const float*& p2, float*& dst)
{
    if (e < NQ) {
        p1 = as;
        p2 = qs + e * n;
        dst = x + e;
    } else if (e < NQ + j) {
        p1 = as;
        p2 = Phi + (int64_t)(e - NQ) * n;
        dst = t + (e - NQ);
    } else {
        const int f = e - NQ - j, i = f / NQ, q = f - i * NQ;
        p1 = A + (int64_t)K[i] * n;
        p2 = qs + q * n;
        dst = y + i * NQ + q;
    }
}

// Load steps per round: six (a 384-column dot in one round) where the
// registers allow it; the load batching does not change any dot's order.
template <int NQ> constexpr int dlu_rsteps() { return NQ == 1 ? 6 : 4; }

template <int NQ>
__device__ inline void dlu_dots(const DluArgs& a, const float* A, const float* st, int j, const int32_t* K,
                                const float* as, const float* qs, float* x, float* t, float* y)
{
    const int n = a.n;
    const float* Phi = st + a.L.phi;
    dlu_dot_set<dlu_rsteps<NQ>()>(n, NQ + j + j * NQ, [&](int e, const float*& p1, const float*& p2, float*& dst) {
        dlu_dot_job<NQ>(e, n, j, A, Phi, K, as, qs, x, t, y, p1, p2, dst);
    });
}

// An accept's dots (NQ = 1) and a ratio's dots (NQ) against the same j
// pending moves in one pass: the two sets read the same rows of Phi and of
// A0^-1, and each dot is formed exactly as in its own pass.
template <int NQ>
__device__ inline void dlu_dots_both(const DluArgs& a, const float* A, const float* st, int j, const int32_t* K,
                                     const float* aa, const float* qa, float* xa, float* ta, float* ya,
                                     const float* ar, const float* qs, float* x, float* t, float* y)
{
    const int n = a.n, ta_total = 1 + 2 * j;
    const float* Phi = st + a.L.phi;
    dlu_dot_set<dlu_rsteps<NQ>()>(n, ta_total + NQ + j + j * NQ,
                                  [&](int e, const float*& p1, const float*& p2, float*& dst) {
        if (e < ta_total) dlu_dot_job<1>(e, n, j, A, Phi, K, aa, qa, xa, ta, ya, p1, p2, dst);
        else dlu_dot_job<NQ>(e - ta_total, n, j, A, Phi, K, ar, qs, x, t, y, p1, p2, dst);
    });
}

// rows[r][m] = src[r][m] for r < NR, m < n: every load of a thread is issued
// before any of its LDS stores (up to four columns per row at a time).
template <int NR>
__device__ inline void dlu_copy_rows(float* rows, const float* const (&src)[NR], int n)
{
    for (int m0 = threadIdx.x; m0 < n; m0 += 4 * kDThreads) {
        float v[NR][4];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int u = 0; u < 4; ++u) v[r][u] = m0 + u * kDThreads < n ? src[r][m0 + u * kDThreads] : 0.f;
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (m0 + u * kDThreads < n) rows[r * n + m0 + u * kDThreads] = v[r][u];
    }
}

// `cnt` dot products of LDS vectors, p1[e] . p2[e], one wave each, in the
// order of dlu_dots (lane-strided over m, then a butterfly), so a dot formed
// here equals the same dot formed there bit for bit.
__device__ inline void dlu_lds_dots(const float* const* p1, const float* const* p2, float* const* dst, int cnt,
                                    int n)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int e = wave; e < cnt; e += kDThreads / 64) {
        float s = 0.f;
        for (int m = lane; m < n; m += 64) s = fmaf(p1[e][m], p2[e][m], s);
        s = dwave_sum(s);
        if (lane == 0) *dst[e] = s;
    }
}

// One step of the delayed update for slot s, in one workgroup: optionally
// accept the move kacc[s] (append phi = Vacc[s], border S^-1 with the Schur
// complement, which is that move's ratio), then optionally form the ratio
// (and derivative sums) of the proposal k[s] with quantities V/G/L[s]
// against the pending moves, the one just accepted included.  Memory is
// read in two rounds: the slot and the orbital rows first (they depend on
// the slot alone), then the pending count, electrons, S^-1 and the rows k of
// A0^-1; then one pass of dot products over the pending rows serves both
// the accept and the ratio.  The move accepted here enters the ratio from LDS (its phi and its
// row of A0^-1), in the order of the dot products of a separate ratio call,
// so a fused step equals an accept followed by a ratio bit for bit.
// ACCEPT alone is spline_dlu_accept, RATIO alone spline_dlu_ratio.  A fused
// step needs S^-1 staged in LDS (the host checks).
template <int NQ, bool ACCEPT, bool RATIO>
__global__ __launch_bounds__(kDThreads) void dlu_step_kernel(DluArgs a)
{
    extern __shared__ float lds[];
    const int n = a.n, tid = threadIdx.x, d = a.d;
    const int64_t s = blockIdx.x;
    float* qa = lds;                                   // accepted phi [n]
    float* aa = qa + (ACCEPT ? n : 0);                 // row kacc of A0^-1 [n]
    float* ar = aa + (ACCEPT ? n : 0);                 // row k of A0^-1 [n]
    float* qs = ar + (RATIO ? n : 0);                  // q [NQ][n]
    float* sc = qs + (RATIO ? NQ * n : 0);             // scalars:
    float* x = sc;                                     //   ratio: x [NQ]
    float* t = x + NQ;                                 //   t [d + 1]
    float* y = t + d + 1;                              //   y [d + 1][NQ]
    float* u = y + (d + 1) * NQ;                       //   u [d + 1]
    float* xa = u + d + 1;                             //   accept: x [1], t [d], y [d], u [d], w [d], rho [1]
    float* ta = xa + 1;
    float* ya = ta + d;
    float* ua = ya + d;
    float* wa = ua + d;
    float* rho = wa + d;
    int32_t* Ks = reinterpret_cast<int32_t*>(rho + 1);  // [d]
    float* Ss = reinterpret_cast<float*>(Ks + d);      // S^-1 [d][d] when staged

    // first wave of loads: the slot and the orbital rows
    const int k_a = ACCEPT ? a.kacc[s] : -1;
    const int k_r = RATIO ? a.k[s] : -1;
    const int64_t w = a.walkers ? (int64_t)a.walkers[s] : s;
    if constexpr (RATIO) {
        if constexpr (NQ == 5) {
            const float* const src[5] = {a.V + s * n, a.G + (3 * s) * n, a.G + (3 * s + 1) * n,
                                         a.G + (3 * s + 2) * n, a.L_ + s * n};
            dlu_copy_rows<5>(qs, src, n);
        } else {
            const float* const src[1] = {a.V + s * n};
            dlu_copy_rows<1>(qs, src, n);
        }
    }
    if constexpr (ACCEPT) {
        const float* const src[1] = {a.Vacc + s * n};
        dlu_copy_rows<1>(qa, src, n);
    }
    const bool wok = w >= 0 && w < a.nwalkers;
    const bool acc_ok = ACCEPT && wok && k_a >= 0 && k_a < n;
    const bool rat_ok = RATIO && wok && k_r >= 0 && k_r < n;
    if (!acc_ok && !rat_ok) {
        if (RATIO && tid < NQ) a.out[s * NQ + tid] = __builtin_nanf("");
        return;
    }
    // second wave of loads: the pending state and the rows of A0^-1
    float* st = a.ws + w * a.L.stride;
    const float* A = a.ainv + w * a.wstride;
    int32_t* cnt = reinterpret_cast<int32_t*>(st + a.L.cnt);
    float* Sinv = st + a.L.sinv;
    const int j = cnt[0];
    if (tid < d) Ks[tid] = reinterpret_cast<const int32_t*>(st + a.L.k)[tid];
    if (a.stage_sinv)
        for (int e = tid; e < d * d; e += kDThreads) Ss[e] = Sinv[e];
    if (acc_ok) {
        const float* const row[1] = {A + (int64_t)k_a * n};
        dlu_copy_rows<1>(aa, row, n);
    }
    if (rat_ok) {
        const float* const row[1] = {A + (int64_t)k_r * n};
        dlu_copy_rows<1>(ar, row, n);
    }
    const bool poisoned = cnt[1] != 0;  // an earlier accept could not be represented
    const float* Sr = a.stage_sinv ? Ss : Sinv;  // row stride d either way
    __syncthreads();

    // A second move of an electron that is already pending cannot be held
    // (the pending moves must be distinct electrons): it is not applied and
    // the walker is marked, so that its ratios are NaN from then on.
    bool dup = false;
    if (acc_ok)
        for (int l = 0; l < j; ++l) dup = dup || Ks[l] == k_a;
    if (dup && tid == 0) cnt[1] = 1;
    const bool acc_do = acc_ok && !dup;

    int jr = j;  // pending moves the ratio sees
    // Both steps: the ratio's dots against the moves pending before this step
    // do not depend on the accept, so they share its pass over the rows.
    const bool both = acc_do && j < d && rat_ok;  // the host keeps accepts between flushes <= d
    if (both) dlu_dots_both<NQ>(a, A, st, j, Ks, aa, qa, xa, ta, ya, ar, qs, x, t, y);
    if (acc_do && j < d) {
        if (!both) dlu_dots<1>(a, A, st, j, Ks, aa, qa, xa, ta, ya);
        __syncthreads();
        if (tid < j) {
            float v = 0.f;
            for (int i = 0; i < j; ++i) v = fmaf(ta[i], Sr[i * d + tid], v);
            ua[tid] = v;
        } else if (tid >= 64 && tid < 64 + j) {
            const int i = tid - 64;
            float v = 0.f;
            for (int l = 0; l < j; ++l) v = fmaf(Sr[i * d + l], ya[l], v);
            wa[i] = v;
        }
        __syncthreads();
        if (tid == 0) {  // the Schur complement: the same value as the ratio of this move
            float r = xa[0];
            for (int l = 0; l < j; ++l) r = fmaf(-ua[l], ya[l], r);
            rho[0] = r;
        }
        __syncthreads();
        const float ir = 1.f / rho[0];
        const int j1 = j + 1;
        for (int e = tid; e < j1 * j1; e += kDThreads) {
            const int i = e / j1, l = e - i * j1;
            float v;
            if (i < j && l < j) v = fmaf(wa[i] * ua[l], ir, Sr[i * d + l]);
            else if (i < j) v = -wa[i] * ir;
            else if (l < j) v = -ua[l] * ir;
            else v = ir;
            Sinv[i * d + l] = v;
            if (RATIO) Ss[i * d + l] = v;  // the ratio below reads the bordered S^-1 from LDS
        }
        float* Phi = st + a.L.phi + (int64_t)j * n;
        for (int m = tid; m < n; m += kDThreads) Phi[m] = qa[m];
        if (tid == 0) {
            reinterpret_cast<int32_t*>(st + a.L.k)[j] = k_a;
            Ks[j] = k_a;
            cnt[0] = j + 1;
        }
        jr = j + 1;
        __syncthreads();
    }
    if constexpr (RATIO) {
        if (!rat_ok || poisoned || dup) {
            if (tid < NQ) a.out[s * NQ + tid] = __builtin_nanf("");
            return;
        }
        if (!both) dlu_dots<NQ>(a, A, st, j, Ks, ar, qs, x, t, y);  // x, and the moves pending before this step
        if (jr > j) {  // the move accepted above, from LDS: t_j = a_k . phi_j, y_j = a_{k_j} . q
            const float* p1[NQ + 1];
            const float* p2[NQ + 1];
            float* dst[NQ + 1];
            p1[0] = ar;
            p2[0] = qa;
            dst[0] = t + j;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                p1[q + 1] = aa;
                p2[q + 1] = qs + q * n;
                dst[q + 1] = y + j * NQ + q;
            }
            dlu_lds_dots(p1, p2, dst, NQ + 1, n);
        }
        __syncthreads();
        // A pending electron's row of the current inverse carries the
        // correction of its replaced column: t_i - [k_i == k] (the Woodbury
        // form of row k of A^-1, Q = columns e_{k_i}).
        if (tid < jr && Ks[tid] == k_r) t[tid] -= 1.f;
        __syncthreads();
        if (tid < jr) {  // u = t^T S^-1
            float v = 0.f;
            for (int i = 0; i < jr; ++i) v = fmaf(t[i], Sr[i * d + tid], v);
            u[tid] = v;
        }
        __syncthreads();
        if (tid < NQ) {
            float r = x[tid];
            for (int l = 0; l < jr; ++l) r = fmaf(-u[l], y[l * NQ + tid], r);
            a.out[s * NQ + tid] = r;
        }
    }
}

// LDS bytes of a step kernel (without S^-1)
static size_t dlu_step_lds(int n, int d, int nq, bool acc, bool rat)
{
    const size_t rows = (acc ? 2 : 0) + (rat ? 1 + nq : 0);
    const size_t scal = nq + (size_t)(d + 1) * (nq + 2) + 1 + 4 * (size_t)d + 1;
    return sizeof(float) * (rows * n + scal) + sizeof(int32_t) * d;
}

// Flush, step 1: M = S^-1 R (R = rows K_i of A0^-1, read before any row
// changes).  S^-1 and K in LDS; each thread owns columns m, stages eight rows
// of R at a time in registers and accumulates every output row.
__global__ __launch_bounds__(kDThreads) void dlu_flush_m_kernel(DluArgs a)
{
    __shared__ float Ss[kDMaxDelay * kDMaxDelay];
    __shared__ int32_t Ks[kDMaxDelay];
    const int64_t w = blockIdx.x;
    float* st = a.ws + w * a.L.stride;
    const int j = reinterpret_cast<const int32_t*>(st + a.L.cnt)[0];
    if (j == 0) return;
    const int n = a.n, tid = threadIdx.x;
    const float* A = a.ainv + w * a.wstride;
    const float* Sinv = st + a.L.sinv;
    for (int e = tid; e < j * j; e += kDThreads) {
        const int l = e / j, i = e - l * j;
        Ss[l * kDMaxDelay + i] = Sinv[l * a.d + i];
    }
    if (tid < j) Ks[tid] = reinterpret_cast<const int32_t*>(st + a.L.k)[tid];
    __syncthreads();
    float* M = st + a.L.m;
    for (int m = blockIdx.y * kDThreads + tid; m < n; m += gridDim.y * kDThreads) {
        float acc[kDMaxDelay];
#pragma unroll
        for (int l = 0; l < kDMaxDelay; ++l) acc[l] = 0.f;
        for (int i0 = 0; i0 < j; i0 += 8) {
            float r[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) r[u] = i0 + u < j ? A[(int64_t)Ks[i0 + u] * n + m] : 0.f;
#pragma unroll
            for (int l = 0; l < kDMaxDelay; ++l)
                if (l < j)
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (i0 + u < j) acc[l] = fmaf(Ss[l * kDMaxDelay + i0 + u], r[u], acc[l]);
        }
#pragma unroll
        for (int l = 0; l < kDMaxDelay; ++l)
            if (l < j) M[(int64_t)l * n + m] = acc[l];
    }
}

typedef float f4v __attribute__((ext_vector_type(4)));

// Flush, step 2: T = A0^-1 Phi^T for a block of 64 rows, over LDS tiles of 64
// columns; the next tile's loads (16-byte when rows allow) are in flight
// while the current one is consumed.
template <bool VEC>
__global__ __launch_bounds__(kDThreads) void dlu_flush_t_kernel(DluArgs a)
{
    __shared__ float At[64][65];
    __shared__ float Pt[kDMaxDelay][65];
    const int64_t w = blockIdx.x;
    float* st = a.ws + w * a.L.stride;
    const int j = reinterpret_cast<const int32_t*>(st + a.L.cnt)[0];
    if (j == 0) return;
    const int n = a.n, tid = threadIdx.x, r0 = blockIdx.y * 64;
    const float* A = a.ainv + w * a.wstride;
    const float* Phi = st + a.L.phi;
    const int ri = tid & 63, lg = tid >> 6;
    float acc[kDMaxDelay / 4];
#pragma unroll
    for (int c = 0; c < kDMaxDelay / 4; ++c) acc[c] = 0.f;
    // registers for one tile: A 64 x 64 (4 x 16 values per thread), Phi j x 64 (<= 4 x 16)
    f4v ra[4], rp[4];
    auto fetch = [&](int m0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + u * kDThreads, r = e >> 4, c = (e & 15) * 4;
            const int64_t row = r0 + r;
            if constexpr (VEC) {
                ra[u] = (row < n && m0 + c < n) ? *reinterpret_cast<const f4v*>(A + row * n + m0 + c)
                                                : f4v{0.f, 0.f, 0.f, 0.f};
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) ra[u][q] = (row < n && m0 + c + q < n) ? A[row * n + m0 + c + q] : 0.f;
            }
            const int l = r;  // Phi rows: e >> 4 < j
#pragma unroll
            for (int q = 0; q < 4; ++q) rp[u][q] = (l < j && m0 + c + q < n) ? Phi[(int64_t)l * n + m0 + c + q] : 0.f;
        }
    };
    fetch(0);
    for (int m0 = 0; m0 < n; m0 += 64) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + u * kDThreads, r = e >> 4, c = (e & 15) * 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                At[r][c + q] = ra[u][q];
                if (r < j) Pt[r][c + q] = rp[u][q];
            }
        }
        __syncthreads();
        if (m0 + 64 < n) fetch(m0 + 64);
#pragma unroll
        for (int c = 0; c < kDMaxDelay / 4; ++c) {
            const int l = lg + 4 * c;
            if (l < j) {
                float v = acc[c];
#pragma unroll 16
                for (int mm = 0; mm < 64; ++mm) v = fmaf(At[ri][mm], Pt[l][mm], v);
                acc[c] = v;
            }
        }
        __syncthreads();
    }
    float* T = st + a.L.t;
    if (r0 + ri < n) {
#pragma unroll
        for (int c = 0; c < kDMaxDelay / 4; ++c) {
            const int l = lg + 4 * c;
            if (l < j) T[(int64_t)(r0 + ri) * a.d + l] = acc[c];
        }
    }
}

// Flush, step 3: A0^-1 -= (T - Q) M over a 64 x 64 tile; each thread owns a
// 4 x 4 block (rows rg + 16i, four consecutive columns), loaded before use.
template <bool VEC>
__global__ __launch_bounds__(kDThreads) void dlu_flush_update_kernel(DluArgs a)
{
    __shared__ float Ct[64][kDMaxDelay + 1];
    __shared__ __align__(16) float Mt[kDMaxDelay][64];
    const int64_t w = blockIdx.x;
    float* st = a.ws + w * a.L.stride;
    const int j = reinterpret_cast<const int32_t*>(st + a.L.cnt)[0];
    if (j == 0) return;
    const int n = a.n, tid = threadIdx.x, r0 = blockIdx.y * 64, c0 = blockIdx.z * 64;
    const float* T = st + a.L.t;
    const float* M = st + a.L.m;
    const int32_t* K = reinterpret_cast<const int32_t*>(st + a.L.k);
    float* A = a.ainv + w * a.wstride;
    const int cq = (tid & 15) * 4, rg = tid >> 4;
    f4v x[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t row = r0 + rg + 16 * i;
        if constexpr (VEC) {
            x[i] = (row < n && c0 + cq < n) ? *reinterpret_cast<const f4v*>(A + row * n + c0 + cq)
                                            : f4v{0.f, 0.f, 0.f, 0.f};
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) x[i][q] = (row < n && c0 + cq + q < n) ? A[row * n + c0 + cq + q] : 0.f;
        }
    }
    for (int e = tid; e < 64 * j; e += kDThreads) {
        const int r = e / j, l = e - r * j;
        const int i = r0 + r;
        Ct[r][l] = i < n ? T[(int64_t)i * a.d + l] - (K[l] == i ? 1.f : 0.f) : 0.f;
    }
    for (int e = tid; e < j * 64; e += kDThreads) {
        const int l = e >> 6, c = e & 63;
        Mt[l][c] = c0 + c < n ? M[(int64_t)l * n + c0 + c] : 0.f;
    }
    __syncthreads();
    for (int l = 0; l < j; ++l) {
        const f4v mv = *reinterpret_cast<const f4v*>(&Mt[l][cq]);
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] -= Ct[rg + 16 * i][l] * mv;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t row = r0 + rg + 16 * i;
        if (row >= n) continue;
        if constexpr (VEC) {
            if (c0 + cq < n) *reinterpret_cast<f4v*>(A + row * n + c0 + cq) = x[i];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (c0 + cq + q < n) A[row * n + c0 + cq + q] = x[i][q];
        }
    }
}

// Flush, steps 2 and 3 in one pass for n <= 512 (n a multiple of 4) and at
// most 16 pending moves: a workgroup holds 32 rows of A0^-1 in registers
// (thread: 4 rows x 4*NC columns, columns cg*4 + 128c), forms their rows of
// T = A0^-1 Phi^T, then C = T - Q and A0^-1 -= C M, and writes the rows back:
// A0^-1 is read once and written once.  Phi, then M, are staged through one
// LDS buffer; C goes through LDS as well.
//
// The 32 threads of a row group sum their four row partials by halving: the
// two lanes 16 apart exchange two rows each, lanes 8 apart one row, then the
// eight lanes that share a row reduce it (cross-lane moves within a 16-lane
// row), so every dot costs 1.5 exchanges instead of 5.
constexpr int kFuseMaxJ = 16;
constexpr int kFuseMaxN = 512;
constexpr int kFuseRows = 32;

template <int CTRL>
__device__ inline float dpp_f(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

// p[0..3]: this lane's partials of rows 0..3 of its row group (32 lanes).
// Returns the full sum of row 2*bit4 + bit3 of the lane id, the same in all
// eight lanes holding that row.
__device__ inline float row_group_sum(const float p[4], int lane)
{
    const bool h16 = lane & 16, h8 = lane & 8;
    const float k0 = h16 ? p[2] : p[0], k1 = h16 ? p[3] : p[1];
    const float s0 = h16 ? p[0] : p[2], s1 = h16 ? p[1] : p[3];
    const float r0 = k0 + __shfl_xor(s0, 16, 64);
    const float r1 = k1 + __shfl_xor(s1, 16, 64);
    float v = (h8 ? r1 : r0) + dpp_f<0x128>(h8 ? r0 : r1);  // row_ror:8 = lane xor 8 within 16
    v += dpp_f<0xB1>(v);                                     // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);                                     // quad_perm [2,3,0,1]
    v += dpp_f<0x141>(v);                                    // row_half_mirror
    return v;
}

// FULL: n == 128 NC and n a multiple of 32, so no row or column of a block
// needs a bounds check.
template <int NC, bool FULL>
__global__ __launch_bounds__(kDThreads) void dlu_flush_fused_kernel(DluArgs a)
{
    constexpr int kStage = kFuseMaxJ * kFuseMaxN / 4 / kDThreads;  // 16-byte loads per thread for Phi or M
    __shared__ __align__(16) float P[kFuseMaxJ * kFuseMaxN];
    __shared__ __align__(16) float Cs[kFuseMaxJ][kFuseRows];
    __shared__ int32_t Ks[kFuseMaxJ];
    const int64_t w = blockIdx.x;
    const float* st = a.ws + w * a.L.stride;
    const int j = reinterpret_cast<const int32_t*>(st + a.L.cnt)[0];
    if (j == 0 || j > kFuseMaxJ) return;  // the host takes this path only with <= 16 accepts since the last flush
    const int n = a.n, tid = threadIdx.x, cg = tid & 31, lane = tid & 63;
    const int rl = (tid >> 5) * 4, rb0 = blockIdx.y * kFuseRows, row0 = rb0 + rl;
    float* A = a.ainv + w * a.wstride;
    auto inside = [&](int i, int c) { return FULL || (row0 + i < n && cg * 4 + 128 * c < n); };
    // every global load of the block is issued here: 4 x NC row chunks, Phi and M
    f4v x[4][NC];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            x[i][c] = inside(i, c) ? *reinterpret_cast<const f4v*>(A + (int64_t)(row0 + i) * n + cg * 4 + 128 * c)
                                   : f4v{0.f, 0.f, 0.f, 0.f};
    const int nv = j * n / 4;
    const f4v* phi = reinterpret_cast<const f4v*>(st + a.L.phi);
    const f4v* mrows = reinterpret_cast<const f4v*>(st + a.L.m);
    f4v sp[kStage], sm[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
        const int e = tid + u * kDThreads;
        sp[u] = e < nv ? phi[e] : f4v{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
        const int e = tid + u * kDThreads;
        sm[u] = e < nv ? mrows[e] : f4v{0.f, 0.f, 0.f, 0.f};
    }
    f4v* P4 = reinterpret_cast<f4v*>(P);
#pragma unroll
    for (int u = 0; u < kStage; ++u)
        if (tid + u * kDThreads < nv) P4[tid + u * kDThreads] = sp[u];
    if (tid < j) Ks[tid] = reinterpret_cast<const int32_t*>(st + a.L.k)[tid];
    __syncthreads();
    const int mine = rl + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1);  // row (in the block) this lane's sums belong to
    for (int l = 0; l < j; ++l) {
        float p[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (inside(0, c)) {  // columns past n hold zeros in x; skip their LDS reads
                const f4v ph = P4[(l * n + cg * 4 + 128 * c) >> 2];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    p[i] = fmaf(x[i][c].x, ph.x, p[i]);
                    p[i] = fmaf(x[i][c].y, ph.y, p[i]);
                    p[i] = fmaf(x[i][c].z, ph.z, p[i]);
                    p[i] = fmaf(x[i][c].w, ph.w, p[i]);
                }
            }
        }
        const float t = row_group_sum(p, lane);
        if ((lane & 7) == 0) Cs[l][mine] = t - (Ks[l] == rb0 + mine ? 1.f : 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kStage; ++u)
        if (tid + u * kDThreads < nv) P4[tid + u * kDThreads] = sm[u];
    __syncthreads();
    for (int l = 0; l < j; ++l) {
        const f4v cv = *reinterpret_cast<const f4v*>(&Cs[l][rl]);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if (inside(0, c)) {
                const f4v mv = P4[(l * n + cg * 4 + 128 * c) >> 2];
                x[0][c] -= cv.x * mv;
                x[1][c] -= cv.y * mv;
                x[2][c] -= cv.z * mv;
                x[3][c] -= cv.w * mv;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (inside(i, c)) *reinterpret_cast<f4v*>(A + (int64_t)(row0 + i) * n + cg * 4 + 128 * c) = x[i][c];
}

// The whole flush on FP32 matrix cores, for n a multiple of 16 up to 384 and
// at most 16 pending moves (zero-padded to 16).  A workgroup owns a walker:
// it stages Phi and R (rows K of A0^-1) in LDS, forms M = S^-1 R in place,
// and each wave then takes blocks of 16 rows of A0^-1.  A block
// lives in registers in the accumulator layout of the transposed product:
// for column tile t (16 columns) lane (g = lane/16, c = lane%16) holds row c,
// columns 16t + 4g .. 16t + 4g + 3, one 16-byte load.  The same registers
// are the A operand of T = A0^-1 Phi^T when the 4-wide k-steps are taken as
// columns {16t + 4g + r}: step (t, r) multiplies register r of tile t with
// Phi[c][16t + 4g + r].  T (rows 4g + r, column c) goes through LDS to become
// the B operand -C^T of the update  A0^-1^T += M^T (-C^T), accumulated onto
// the block's registers, which are then stored.
constexpr int kMfmaMaxN = 384;

__device__ inline f4v mfma16x16x4(float a, float b, f4v c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// LDS row strides (words): Phi rows at 4 mod 64 (the 16-byte reads of a
// quarter wave, one per row, fall in distinct banks), M rows at 16 mod 64
// (the four row groups of a wave's 4-byte reads are 16 banks apart).
__host__ __device__ inline int dlu_mfma_ldp(int n) { return n + ((4 - n) & 63); }
__host__ __device__ inline int dlu_mfma_ldm(int n) { return n + ((16 - n) & 63); }

// EXACT: n == 16 NT, so no tile needs a guard; the guards of the other
// builds are branches, after which the compiler waits for every load in
// flight, the prefetch included.
template <int NT, bool EXACT, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4))) void dlu_flush_mfma_kernel(DluArgs a)
{
    constexpr int kThreads = 64 * NW;
    extern __shared__ __align__(16) float lds[];
    const int64_t w = blockIdx.x;
    const float* st = a.ws + w * a.L.stride;
    const int j = reinterpret_cast<const int32_t*>(st + a.L.cnt)[0];
    if (j == 0 || j > kFuseMaxJ) return;  // the host takes this path only with <= 16 accepts since the last flush
    const int n = EXACT ? 16 * NT : a.n, nt = EXACT ? NT : n >> 4, tid = threadIdx.x, lane = tid & 63,
              wave = tid >> 6;
    const int ldp = dlu_mfma_ldp(n), ldm = dlu_mfma_ldm(n);
    const int g = lane >> 4, c = lane & 15;
    float* Ph = lds;                                   // Phi [16][ldp]
    float* Ms = Ph + 16 * ldp;                         // M [16][ldm]
    float* Cw = Ms + 16 * ldm + wave * (16 * 20);      // -C of this wave's block [16][20]
    int32_t* Ks = reinterpret_cast<int32_t*>(Ms + 16 * ldm + NW * 16 * 20);
    float* Ss = Ms + 16 * ldm;  // S^-1 [16][17], zero-padded, in wave 0's C scratch (not in use yet)
    const int n4 = n >> 2;
    float* A = a.ainv + w * a.wstride;
    if (tid < 16) Ks[tid] = tid < j ? reinterpret_cast<const int32_t*>(st + a.L.k)[tid] : -1;
    if (tid < 256) {
        const int l = tid >> 4, i = tid & 15;
        Ss[l * 17 + i] = (l < j && i < j) ? st[a.L.sinv + l * a.d + i] : 0.f;
    }
    __syncthreads();
    // Phi, and R = rows K of A0^-1 (read before any row of this walker
    // changes: every row of it is updated by this workgroup, after the
    // barriers below) into the M buffer
    const f4v* phi = reinterpret_cast<const f4v*>(st + a.L.phi);
    for (int e = tid; e < 16 * n4; e += kThreads) {
        const int l = e / n4, q = e - l * n4;
        const f4v z = {0.f, 0.f, 0.f, 0.f};
        *reinterpret_cast<f4v*>(Ph + l * ldp + 4 * q) = l < j ? phi[e] : z;
        *reinterpret_cast<f4v*>(Ms + l * ldm + 4 * q) =
            l < j ? *reinterpret_cast<const f4v*>(A + (int64_t)Ks[l] * n + 4 * q) : z;
    }
    __syncthreads();
    // M = S^-1 R in place: a thread owns whole columns
    for (int m = tid; m < n; m += kThreads) {
        float r[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) r[i] = Ms[i * ldm + m];
#pragma unroll
        for (int l = 0; l < 16; ++l) {
            float v = 0.f;
#pragma unroll
            for (int i = 0; i < 16; ++i) v = fmaf(Ss[l * 17 + i], r[i], v);
            Ms[l * ldm + m] = v;
        }
    }
    __syncthreads();
    auto load = [&](int b, f4v* X) {
        const float* src = A + (int64_t)(16 * b + c) * n + 4 * g;
#pragma unroll
        for (int t = 0; t < NT; ++t)
            if (t < nt) X[t] = *reinterpret_cast<const f4v*>(src + 16 * t);
    };
    // one block, held in X: T, -C through LDS, the update, the stores
    auto block = [&](int b, f4v* X) {
        f4v acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t < nt) {
                const f4v ph = *reinterpret_cast<const f4v*>(Ph + c * ldp + 16 * t + 4 * g);
                acc0 = mfma16x16x4(X[t].x, ph.x, acc0);
                acc1 = mfma16x16x4(X[t].y, ph.y, acc1);
                acc0 = mfma16x16x4(X[t].z, ph.z, acc0);
                acc1 = mfma16x16x4(X[t].w, ph.w, acc1);
            }
        }
        const f4v T = acc0 + acc1;  // T[16b + 4g + r][c]
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 4 * g + r;
            Cw[row * 20 + c] = (Ks[c] == 16 * b + row ? 1.f : 0.f) - T[r];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float cb[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) cb[s4] = Cw[c * 20 + 4 * s4 + g];  // -C[row c][4 s4 + g]
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int t = 0; t < NT; ++t)
                if (t < nt) X[t] = mfma16x16x4(Ms[(4 * s4 + g) * ldm + 16 * t + c], cb[s4], X[t]);
        float* dst = A + (int64_t)(16 * b + c) * n + 4 * g;
#pragma unroll
        for (int t = 0; t < NT; ++t)
            if (t < nt) *reinterpret_cast<f4v*>(dst + 16 * t) = X[t];
    };
    // Blocks wave, wave + NW, ...; each wave loads a block, works on it and
    // stores it, and the eight waves of the workgroup (up to 16 per CU) hide
    // each other's loads.  (Holding a second block for a prefetch doubles
    // the registers and halves the waves; measured slower.)
    const int nblk = (nt - wave + NW - 1) / NW;
    f4v X[NT];
#pragma unroll 1
    for (int i = 0; i < nblk; ++i) {
        const int b = wave + NW * i;
        load(b, X);
        block(b, X);
    }
}

constexpr int kMfmaWaves = 8;  // waves per workgroup of the matrix-core flush
static size_t dlu_mfma_lds(int n)
{
    return sizeof(float) * (16 * (size_t)(dlu_mfma_ldp(n) + dlu_mfma_ldm(n)) + kMfmaWaves * 16 * 20) + 16 * 4;
}

// Clears the pending-move count of every walker (and, at creation, the mark
// left by an accept that could not be represented).
__global__ void dlu_clear_kernel(float* ws, DluLayout L, int64_t W, int32_t marks)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    int32_t* c = reinterpret_cast<int32_t*>(ws + w * L.stride + L.cnt);
    c[0] = 0;
    if (marks) c[1] = 0;
}

}  // namespace qs

struct spline_dlu_s {
    int32_t n, d;
    int64_t walkers;
    float* ws;
    qs::DluLayout L;
    int device;
    int32_t accepts;  // accept calls since the last flush (upper bound of every walker's count)
};

using namespace qs;

static int dlu_check(const spline_dlu_s* h, const float* ainv, int64_t wstride)
{
    if (!h) return fail(SPL_EINVAL, "handle is NULL");
    if (!ainv) return fail(SPL_EINVAL, "inverse pointer is NULL");
    if (wstride < (int64_t)h->n * h->n) return fail(SPL_EINVAL, "walker_stride must be >= n*n");
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    if (dev != h->device) return fail(SPL_EINVAL, "current HIP device differs from the workspace's device");
    return SPL_OK;
}

extern "C" {

size_t spline_dlu_workspace_bytes(int32_t n, int32_t delay, int64_t walkers)
{
    if (n < 1 || n > kDMaxN || delay < 1 || delay > kDMaxDelay || delay > n || walkers < 1) return 0;
    const DluLayout L = dlu_layout(n, delay);
    int64_t b;
    if (!mul_ok(L.stride * 4, walkers, &b)) return 0;
    return (size_t)b;
}

int spline_dlu_create(int32_t n, int32_t delay, int64_t walkers, void* ws_dev, size_t ws_bytes, void* stream,
                      spline_dlu_t** out)
{
    if (!out) return fail(SPL_EINVAL, "out is NULL");
    *out = nullptr;
    const size_t need = spline_dlu_workspace_bytes(n, delay, walkers);
    if (need == 0) return fail(SPL_EINVAL, "need 1 <= n <= 2048, 1 <= delay <= min(64, n), walkers >= 1");
    if (!ws_dev || (reinterpret_cast<uintptr_t>(ws_dev) & 255)) return fail(SPL_EINVAL, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < need) return fail(SPL_ENOMEM, "workspace smaller than spline_dlu_workspace_bytes()");
    spline_dlu_s* h = new (std::nothrow) spline_dlu_s;
    if (!h) return fail(SPL_ENOMEM, "handle allocation failed");
    h->n = n;
    h->d = delay;
    h->walkers = walkers;
    h->ws = static_cast<float*>(ws_dev);
    h->L = dlu_layout(n, delay);
    h->accepts = 0;
    QS_HIP(hipGetDevice(&h->device));
    hipLaunchKernelGGL(dlu_clear_kernel, dim3((unsigned)((walkers + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), h->ws, h->L, walkers, 1);
    QS_HIP(hipGetLastError());
    *out = h;
    return SPL_OK;
}

int spline_dlu_destroy(spline_dlu_t* h)
{
    delete h;
    return SPL_OK;
}

int spline_dlu_ratio(const spline_dlu_t* h, const float* ainv, int64_t walker_stride, const int32_t* walkers,
                     const int32_t* k, const float* V, const float* G, const float* L, int64_t count, float* out,
                     void* stream)
{
    int rc = dlu_check(h, ainv, walker_stride);
    if (rc) return rc;
    if (count < 0 || count > (int64_t)std::numeric_limits<int32_t>::max()) return fail(SPL_EINVAL, "bad count");
    if (count == 0) return SPL_OK;
    if (!k || !V || !out) return fail(SPL_EINVAL, "NULL electron, value or output pointer");
    if ((G == nullptr) != (L == nullptr)) return fail(SPL_EINVAL, "give both G and L, or neither");
    if (!walkers && count > h->walkers) return fail(SPL_EINVAL, "count exceeds the workspace's walkers");
    const bool vgl = G != nullptr;
    DluArgs a{h->ws, h->L, h->n, h->d, const_cast<float*>(ainv), walker_stride, walkers, k, V, G, L, count, out};
    a.nwalkers = h->walkers;
    void* params[] = {&a};
    size_t lds = dlu_step_lds(h->n, h->d, vgl ? 5 : 1, false, true);
    a.stage_sinv = lds + sizeof(float) * h->d * h->d <= kDMaxLds;
    if (a.stage_sinv) lds += sizeof(float) * h->d * h->d;
    QS_HIP(hipLaunchKernel(vgl ? (const void*)&dlu_step_kernel<5, false, true>
                               : (const void*)&dlu_step_kernel<1, false, true>,
                           dim3((unsigned)count), dim3(kDThreads), params, lds, static_cast<hipStream_t>(stream)));
    QS_HIP(hipGetLastError());
    return SPL_OK;
}

int spline_dlu_accept(spline_dlu_t* h, const float* ainv, int64_t walker_stride, const int32_t* walkers,
                      const int32_t* k, const float* V, int64_t count, void* stream)
{
    int rc = dlu_check(h, ainv, walker_stride);
    if (rc) return rc;
    if (count < 0 || count > (int64_t)std::numeric_limits<int32_t>::max()) return fail(SPL_EINVAL, "bad count");
    if (count == 0) return SPL_OK;
    if (!k || !V) return fail(SPL_EINVAL, "NULL electron or value pointer");
    if (h->accepts >= h->d) return fail(SPL_EINVAL, "delay reached: flush before accepting more moves");
    if (!walkers && count > h->walkers) return fail(SPL_EINVAL, "count exceeds the workspace's walkers");
    DluArgs a{h->ws, h->L, h->n, h->d, const_cast<float*>(ainv), walker_stride, walkers, nullptr, nullptr, nullptr,
              nullptr, count, nullptr};
    a.nwalkers = h->walkers;
    a.kacc = k;
    a.Vacc = V;
    void* params[] = {&a};
    size_t lds = dlu_step_lds(h->n, h->d, 1, true, false);
    a.stage_sinv = lds + sizeof(float) * h->d * h->d <= kDMaxLds;
    if (a.stage_sinv) lds += sizeof(float) * h->d * h->d;
    QS_HIP(hipLaunchKernel((const void*)&dlu_step_kernel<1, true, false>, dim3((unsigned)count), dim3(kDThreads),
                           params, lds, static_cast<hipStream_t>(stream)));
    QS_HIP(hipGetLastError());
    ++h->accepts;
    return SPL_OK;
}

int spline_dlu_accept_ratio(spline_dlu_t* h, const float* ainv, int64_t walker_stride, const int32_t* walkers,
                            const int32_t* k_acc, const float* V_acc, const int32_t* k, const float* V,
                            const float* G, const float* L, int64_t count, float* out, void* stream)
{
    int rc = dlu_check(h, ainv, walker_stride);
    if (rc) return rc;
    if (count < 0 || count > (int64_t)std::numeric_limits<int32_t>::max()) return fail(SPL_EINVAL, "bad count");
    if (count == 0) return SPL_OK;
    if (!k_acc || !V_acc || !k || !V || !out) return fail(SPL_EINVAL, "NULL electron, value or output pointer");
    if ((G == nullptr) != (L == nullptr)) return fail(SPL_EINVAL, "give both G and L, or neither");
    if (h->accepts >= h->d) return fail(SPL_EINVAL, "delay reached: flush before accepting more moves");
    if (!walkers && count > h->walkers) return fail(SPL_EINVAL, "count exceeds the workspace's walkers");
    const bool vgl = G != nullptr;
    const int nq = vgl ? 5 : 1;
    const size_t lds = dlu_step_lds(h->n, h->d, nq, true, true) + sizeof(float) * h->d * h->d;
    if (lds > kDMaxLds) {  // S^-1 would not fit in LDS beside the rest: the same step as two launches
        rc = spline_dlu_accept(h, ainv, walker_stride, walkers, k_acc, V_acc, count, stream);
        if (rc) return rc;
        return spline_dlu_ratio(h, ainv, walker_stride, walkers, k, V, G, L, count, out, stream);
    }
    DluArgs a{h->ws, h->L, h->n, h->d, const_cast<float*>(ainv), walker_stride, walkers, k, V, G, L, count, out};
    a.nwalkers = h->walkers;
    a.kacc = k_acc;
    a.Vacc = V_acc;
    a.stage_sinv = 1;
    void* params[] = {&a};
    QS_HIP(hipLaunchKernel(vgl ? (const void*)&dlu_step_kernel<5, true, true>
                               : (const void*)&dlu_step_kernel<1, true, true>,
                           dim3((unsigned)count), dim3(kDThreads), params, lds, static_cast<hipStream_t>(stream)));
    QS_HIP(hipGetLastError());
    ++h->accepts;
    return SPL_OK;
}

int spline_dlu_flush(spline_dlu_t* h, float* ainv, int64_t walker_stride, void* stream)
{
    int rc = dlu_check(h, ainv, walker_stride);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    DluArgs a{h->ws, h->L, h->n, h->d, ainv, walker_stride, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr};
    a.nwalkers = h->walkers;
    void* params[] = {&a};
    const unsigned W = (unsigned)h->walkers, nb = (unsigned)((h->n + 63) / 64);
    // 16-byte row accesses when every row of every walker starts 16-byte aligned
    const bool vec = h->n % 4 == 0 && walker_stride % 4 == 0 && (reinterpret_cast<uintptr_t>(ainv) & 15) == 0;
    const unsigned mb = (unsigned)((h->n + kDThreads - 1) / kDThreads);
    // matrix-core pass (M formed inside): n a multiple of 16 up to 384
    const int nt = h->n / 16;
    const bool mfma = vec && h->n % 16 == 0 && h->n <= kMfmaMaxN && h->accepts <= kFuseMaxJ;
    if (mfma) {
        constexpr int V = kMfmaWaves;
        // exact builds for n = 64, 128, ..., 384; otherwise the next larger
        // guarded build (a guarded 8-tile build spills)
        static const void* const exact[6] = {
            (const void*)&dlu_flush_mfma_kernel<4, true, V>,  (const void*)&dlu_flush_mfma_kernel<8, true, V>,
            (const void*)&dlu_flush_mfma_kernel<12, true, V>, (const void*)&dlu_flush_mfma_kernel<16, true, V>,
            (const void*)&dlu_flush_mfma_kernel<20, true, V>, (const void*)&dlu_flush_mfma_kernel<24, true, V>};
        static const void* const guarded[6] = {
            (const void*)&dlu_flush_mfma_kernel<4, false, V>,  (const void*)&dlu_flush_mfma_kernel<12, false, V>,
            (const void*)&dlu_flush_mfma_kernel<12, false, V>, (const void*)&dlu_flush_mfma_kernel<16, false, V>,
            (const void*)&dlu_flush_mfma_kernel<20, false, V>, (const void*)&dlu_flush_mfma_kernel<24, false, V>};
        const int ti = (nt + 3) / 4 - 1;
        const void* fn = nt == 4 * (ti + 1) ? exact[ti] : guarded[ti];
        QS_HIP(hipLaunchKernel(fn, dim3(W), dim3(64 * V), params, dlu_mfma_lds(h->n), st));
    } else {
        QS_HIP(hipLaunchKernel((const void*)&dlu_flush_m_kernel, dim3(W, mb), dim3(kDThreads), params, 0, st));
        if (vec && h->n <= kFuseMaxN && h->accepts <= kFuseMaxJ) {
            static const void* const fused[2][4] = {
                {(const void*)&dlu_flush_fused_kernel<1, false>, (const void*)&dlu_flush_fused_kernel<2, false>,
                 (const void*)&dlu_flush_fused_kernel<3, false>, (const void*)&dlu_flush_fused_kernel<4, false>},
                {(const void*)&dlu_flush_fused_kernel<1, true>, (const void*)&dlu_flush_fused_kernel<2, true>,
                 (const void*)&dlu_flush_fused_kernel<3, true>, (const void*)&dlu_flush_fused_kernel<4, true>}};
            const int nc = (h->n + 127) / 128;
            const bool full = h->n == 128 * nc;  // then also a multiple of 32
            const unsigned rb = (unsigned)((h->n + kFuseRows - 1) / kFuseRows);
            QS_HIP(hipLaunchKernel(fused[full][nc - 1], dim3(W, rb), dim3(kDThreads), params, 0, st));
        } else {
            QS_HIP(hipLaunchKernel(vec ? (const void*)&dlu_flush_t_kernel<true>
                                       : (const void*)&dlu_flush_t_kernel<false>,
                                   dim3(W, nb), dim3(kDThreads), params, 0, st));
            QS_HIP(hipLaunchKernel(vec ? (const void*)&dlu_flush_update_kernel<true>
                                       : (const void*)&dlu_flush_update_kernel<false>,
                                   dim3(W, nb, nb), dim3(kDThreads), params, 0, st));
        }
    }
    hipLaunchKernelGGL(dlu_clear_kernel, dim3((W + 255) / 256), dim3(256), 0, st, h->ws, h->L, h->walkers, 0);
    QS_HIP(hipGetLastError());
    h->accepts = 0;
    return SPL_OK;
}

}  // extern "C"
