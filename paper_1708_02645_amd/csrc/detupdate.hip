// Sherman-Morrison update of inverse Slater matrices after accepted moves.
//
// With t = A^-1 phi and rho = t_k, the new inverse is
//   A^-1[i][:] -= (t_i / rho) * rowk        for i != k
//   A^-1[k][:]  = rowk / rho
// where rowk is row k before the update.  Row i needs only its own dot
// product t_i and the original row k, so every row is read once and written
// once: a wave loads the row into registers, reduces the dot product with
// phi across its lanes, and writes the updated row back.  Rows of one walker
// are split over several workgroups; each stages phi and the original row k
// in LDS and computes rho itself, in a fixed order, so all of them agree bit
// for bit.  Row k is written by a second launch, after every workgroup of the
// first has read it.
#include <algorithm>
#include <limits>

#include "common.hpp"

namespace qs {

struct SmArgs {
    void* ainv;
    int64_t wstride;        // elements between walkers' inverses
    const int32_t* walkers; // [count] or null (slot j -> walker j)
    const int32_t* k;       // [count]
    const void* phi;        // [count][ld_phi]
    int64_t ld_phi;
    int64_t count;
    int32_t n;
    int32_t rows_per_group; // rows of one walker handled by one workgroup
};

constexpr int kSmThreads = 256;

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); static constexpr int n = 4; };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); static constexpr int n = 2; };

template <typename T>
__device__ inline T wave_sum(T x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// rho = rowk . phi over the workgroup, in a fixed order: per-thread strided
// partial sums, a butterfly per wave, then the four wave sums in order.
template <typename T>
__device__ inline T block_dot(const T* a, const T* b, int n, T* red)
{
    const int tid = threadIdx.x;
    T s = T(0);
    for (int j = tid; j < n; j += kSmThreads) s = fma(a[j], b[j], s);
    s = wave_sum(s);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    T r = red[0];
#pragma unroll
    for (int w = 1; w < kSmThreads / 64; ++w) r += red[w];
    return r;
}

// Slot j's walker, electron and phi; false when k is out of range (the
// walker is then left untouched).
template <typename T>
__device__ inline bool sm_slot(const SmArgs& a, int64_t j, T*& A, int& k, const T*& ph)
{
    const int64_t w = a.walkers ? (int64_t)a.walkers[j] : j;
    k = a.k[j];
    if (k < 0 || k >= a.n || w < 0) return false;
    A = reinterpret_cast<T*>(a.ainv) + w * a.wstride;
    ph = reinterpret_cast<const T*>(a.phi) + j * a.ld_phi;
    return true;
}

// Rows i != k.  C: 16-byte chunks per lane that hold a whole row in
// registers (row length n <= C * 64 * V and a multiple of V, 16-byte aligned
// rows); C = 0 streams the row twice (second pass from cache) for any n.
template <typename T, int C>
__global__ __launch_bounds__(kSmThreads) void sm_rows_kernel(SmArgs a)
{
    extern __shared__ unsigned char lds_raw[];
    T* phs = reinterpret_cast<T*>(lds_raw);
    T* rks = phs + a.n;
    T* red = rks + a.n;
    T* A;
    const T* ph;
    int k;
    if (!sm_slot<T>(a, blockIdx.x, A, k, ph)) return;  // uniform over the workgroup
    const int n = a.n, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int j = tid; j < n; j += kSmThreads) {
        phs[j] = ph[j];
        rks[j] = A[(int64_t)k * n + j];
    }
    __syncthreads();
    const T inv_rho = T(1) / block_dot(rks, phs, n, red);
    const int r0 = blockIdx.y * a.rows_per_group;
    const int r1 = min(n, r0 + a.rows_per_group);
    using V = typename Vec16<T>::type;
    constexpr int VN = Vec16<T>::n;
    constexpr int NW = kSmThreads / 64;
    if constexpr (C > 0) {
        // two rows per wave in flight: loads of both, then both reductions
        for (int i0 = r0 + wave; i0 < r1; i0 += 2 * NW) {
            const int rows[2] = {i0, i0 + NW};
            V x[2][C];
            T s[2] = {T(0), T(0)};
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                if (rows[r] >= r1 || rows[r] == k) continue;
                const T* Ai = A + (int64_t)rows[r] * n;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int j = (c * 64 + lane) * VN;
                    if (j < n) x[r][c] = *reinterpret_cast<const V*>(Ai + j);
                }
            }
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int j = (c * 64 + lane) * VN;
                    if (j < n && rows[r] < r1 && rows[r] != k)
#pragma unroll
                        for (int e = 0; e < VN; ++e) s[r] = fma(x[r][c][e], phs[j + e], s[r]);
                }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const T coef = wave_sum(s[r]) * inv_rho;  // every lane of the wave takes part
                if (rows[r] >= r1 || rows[r] == k) continue;
                T* Ai = A + (int64_t)rows[r] * n;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int j = (c * 64 + lane) * VN;
                    if (j < n) {
#pragma unroll
                        for (int e = 0; e < VN; ++e) x[r][c][e] = fma(-coef, rks[j + e], x[r][c][e]);
                        *reinterpret_cast<V*>(Ai + j) = x[r][c];
                    }
                }
            }
        }
        return;
    }
    for (int i = r0 + wave; i < r1; i += NW) {
        if (i == k) continue;
        T* Ai = A + (int64_t)i * n;
        {
            T s = T(0);
            for (int j = lane; j < n; j += 64) s = fma(Ai[j], phs[j], s);
            const T coef = wave_sum(s) * inv_rho;
            for (int j = lane; j < n; j += 64) Ai[j] = fma(-coef, rks[j], Ai[j]);
        }
    }
}

// Row k: rowk / rho, with rho computed exactly as in sm_rows_kernel.
template <typename T>
__global__ __launch_bounds__(kSmThreads) void sm_rowk_kernel(SmArgs a)
{
    extern __shared__ unsigned char lds_raw[];
    T* phs = reinterpret_cast<T*>(lds_raw);
    T* rks = phs + a.n;
    T* red = rks + a.n;
    T* A;
    const T* ph;
    int k;
    if (!sm_slot<T>(a, blockIdx.x, A, k, ph)) return;
    const int n = a.n;
    for (int j = threadIdx.x; j < n; j += kSmThreads) {
        phs[j] = ph[j];
        rks[j] = A[(int64_t)k * n + j];
    }
    __syncthreads();
    const T inv_rho = T(1) / block_dot(rks, phs, n, red);
    for (int j = threadIdx.x; j < n; j += kSmThreads) A[(int64_t)k * n + j] = rks[j] * inv_rho;
}

template <typename T>
static int sm_launch(const SmArgs& a0, bool vec_ok, hipStream_t st)
{
    SmArgs a = a0;
    constexpr int VN = Vec16<T>::n;
    const int chunks = (a.n + 64 * VN - 1) / (64 * VN);
    // Split each walker's rows so that the grid holds at least ~2048
    // workgroups, with at least 16 rows (four per wave) per workgroup.
    int64_t splits = (2048 + a.count - 1) / a.count;
    splits = std::max<int64_t>(1, std::min<int64_t>(splits, (a.n + 15) / 16));
    a.rows_per_group = (int32_t)((a.n + splits - 1) / splits);
    splits = (a.n + a.rows_per_group - 1) / a.rows_per_group;
    if (a.count > (int64_t)std::numeric_limits<int32_t>::max()) return fail(SPL_EINVAL, "too many walkers for one launch");
    const size_t lds = (2 * (size_t)a.n + kSmThreads / 64) * sizeof(T);
    void* params[] = {&a};
    const void* fn = (const void*)&sm_rows_kernel<T, 0>;
    if (vec_ok) {
        switch (chunks) {
        case 1: fn = (const void*)&sm_rows_kernel<T, 1>; break;
        case 2: fn = (const void*)&sm_rows_kernel<T, 2>; break;
        case 3: fn = (const void*)&sm_rows_kernel<T, 3>; break;
        case 4: fn = (const void*)&sm_rows_kernel<T, 4>; break;
        case 5: case 6: fn = (const void*)&sm_rows_kernel<T, 6>; break;
        case 7: case 8: fn = (const void*)&sm_rows_kernel<T, 8>; break;
        default: break;
        }
    }
    QS_HIP(hipLaunchKernel(fn, dim3((unsigned)a.count, (unsigned)splits), dim3(kSmThreads), params, lds, st));
    QS_HIP(hipGetLastError());
    QS_HIP(hipLaunchKernel((const void*)&sm_rowk_kernel<T>, dim3((unsigned)a.count), dim3(kSmThreads), params, lds,
                           st));
    QS_HIP(hipGetLastError());
    return SPL_OK;
}

}  // namespace qs

using namespace qs;

extern "C" int spline_det_update(void* ainv_dev, int32_t n, int64_t walker_stride, const int32_t* walkers_dev,
                                 const int32_t* k_dev, const void* phi_dev, int64_t ld_phi, int64_t count,
                                 spline_dtype dtype, void* stream)
{
    if (count < 0) return fail(SPL_EINVAL, "count must be >= 0");
    if (count == 0) return SPL_OK;
    if (!ainv_dev || !k_dev || !phi_dev) return fail(SPL_EINVAL, "NULL inverse, electron or orbital pointer");
    if (dtype != SPL_F32 && dtype != SPL_F64) return fail(SPL_EINVAL, "dtype must be SPL_F32 or SPL_F64");
    const size_t eb = dtype == SPL_F64 ? 8 : 4;
    if (n < 1 || (size_t)(2 * n + 4) * eb > kMaxLds) return fail(SPL_EINVAL, "n out of range");
    if (ld_phi < n) return fail(SPL_EINVAL, "ld_phi must be >= n");
    if (walker_stride < (int64_t)n * n) return fail(SPL_EINVAL, "walker_stride must be >= n*n");
    if ((uintptr_t)ainv_dev % eb || (uintptr_t)phi_dev % eb) return fail(SPL_EINVAL, "pointers must be element-aligned");
    SmArgs a{ainv_dev, walker_stride, walkers_dev, k_dev, phi_dev, ld_phi, count, n, 0};
    const int vn = (int)(16 / eb);
    const bool vec_ok = (uintptr_t)ainv_dev % 16 == 0 && n % vn == 0 && walker_stride % vn == 0;
    hipStream_t st = static_cast<hipStream_t>(stream);
    return dtype == SPL_F64 ? sm_launch<double>(a, vec_ok, st) : sm_launch<float>(a, vec_ok, st);
}
