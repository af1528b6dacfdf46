// Locality-ordered evaluation of a large batch.
//
// Each position needs the 4 x 4 x 4 table rows around its grid cell.  In a
// batch of random positions consecutive workgroups touch unrelated rows, so
// every gathered row comes from HBM.  Here the positions are first bucketed
// by the block of 2^s x 2^s x 2^s grid cells they fall in, blocks in Morton
// order (a counting sort on the device: key and rank within the bucket,
// exclusive scan of the bucket sizes, scatter), and the evaluation kernel
// then takes them in that order through its index list.  Positions that
// share rows run close together in time, so most rows are re-read from the
// L2 and Infinity caches instead of HBM.  Outputs go to each position's own
// row and the per-position arithmetic is the evaluation kernel's, so the
// results equal spline_eval_vgl / spline_eval_v bit for bit; the order
// within a bucket (atomic ranks) changes only the timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <fstream>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace qs {

constexpr int kLocThreads = 256;
constexpr int kLocScanThreads = 1024;
constexpr int kLocBits = 5;                            // coarse blocks per dimension <= 2^5
constexpr int kLocBuckets = 1 << (3 * kLocBits);       // Morton keys < 2^15

struct LocKey {
    double inv[3];    // 1 / cell length (orthorhombic cell)
    double ilat[9];   // general cell: fractional u_d = sum_c r_c ilat[c*3 + d]
    int32_t general;
    int32_t n[3];     // grid points per dimension
    int32_t shift;    // coarse block = 2^shift cells per dimension
};

// The low ten bits of v moved to every third bit position (Morton interleave).
__device__ inline uint32_t spread3(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ __launch_bounds__(kLocThreads) void loc_zero_kernel(int32_t* count, int n)
{
    const int i = blockIdx.x * kLocThreads + threadIdx.x;
    if (i < n) count[i] = 0;
}

// Bucket of each position and its rank among the positions of that bucket.
// A non-finite coordinate goes to block 0 (the evaluation kernel gives its
// outputs NaN either way).
__global__ __launch_bounds__(kLocThreads) void loc_key_kernel(const double* pos, int64_t B, LocKey k, int32_t* count,
                                                              int32_t* key, int32_t* rank)
{
    const int64_t b = (int64_t)blockIdx.x * kLocThreads + threadIdx.x;
    if (b >= B) return;
    uint32_t c[3];
    const double r[3] = {pos[3 * b], pos[3 * b + 1], pos[3 * b + 2]};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double u = k.general ? r[0] * k.ilat[d] + r[1] * k.ilat[3 + d] + r[2] * k.ilat[6 + d] : r[d] * k.inv[d];
        u -= floor(u);
        int i = (u >= 0.0 && u < 1.0) ? (int)(u * k.n[d]) : 0;
        i = i < 0 ? 0 : (i >= k.n[d] ? k.n[d] - 1 : i);
        c[d] = (uint32_t)i >> k.shift;
    }
    const int32_t kk = (int32_t)((spread3(c[0]) << 2) | (spread3(c[1]) << 1) | spread3(c[2]));
    key[b] = kk;
    rank[b] = atomicAdd(&count[kk], 1);
}

// Exclusive prefix sum of count[0 .. kLocBuckets) in place, one workgroup:
// each thread sums a run of buckets, the runs' totals are scanned in LDS,
// then every thread writes its run's offsets.
__global__ __launch_bounds__(kLocScanThreads) void loc_scan_kernel(int32_t* count)
{
    constexpr int kRun = kLocBuckets / kLocScanThreads;
    __shared__ int32_t part[kLocScanThreads];
    const int t = threadIdx.x;
    int32_t v[kRun];
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < kRun; ++i) {
        v[i] = count[t * kRun + i];
        s += v[i];
    }
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kLocScanThreads; off <<= 1) {  // inclusive scan of the run totals
        const int32_t x = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    int32_t run = part[t] - s;  // exclusive start of this thread's run
#pragma unroll
    for (int i = 0; i < kRun; ++i) {
        count[t * kRun + i] = run;
        run += v[i];
    }
}

// Sorted slot j = offset[key] + rank goes to the index list so that the
// workgroups on one XCD take a contiguous stretch of the sorted order:
// workgroups are dispatched to the eight XCDs in turn (workgroup i to XCD
// i mod 8), so whole chunks of pb slots are dealt out as chunk c -> workgroup
// 8k + x, where x is the XCD whose contiguous share of the chunks holds c and
// k is c's place in it.  The chunks of one XCD then share table rows in that
// XCD's L2.  A partial last chunk stays last (only the last workgroup takes
// fewer than pb positions).
__global__ __launch_bounds__(kLocThreads) void loc_scatter_kernel(int64_t B, int32_t pb, const int32_t* offset,
                                                                  const int32_t* key, const int32_t* rank,
                                                                  int32_t* perm)
{
    const int64_t b = (int64_t)blockIdx.x * kLocThreads + threadIdx.x;
    if (b >= B) return;
    const int64_t j = (int64_t)offset[key[b]] + rank[b];
    int64_t dst = j;
    const int64_t full = pb > 0 ? B / pb : 0, c = pb > 0 ? j / pb : 0, r = j - c * pb;
    if (c < full) {  // pb <= 0: plain sorted order (the caller deals the work)
        const int64_t c8 = full / 8, rem = full % 8, big = rem * (c8 + 1);  // XCDs x < rem take c8 + 1 chunks
        int64_t x, k;
        if (c < big) {
            x = c / (c8 + 1);
            k = c - x * (c8 + 1);
        } else {  // then c8 >= 1
            const int64_t e = c - big;
            x = rem + e / c8;
            k = e - (x - rem) * c8;
        }
        dst = (8 * k + x) * pb + r;
    }
    perm[dst] = (int32_t)b;
}

static_assert(kLocBuckets % kLocScanThreads == 0, "scan runs must tile the buckets");

// Workspace: count [kLocBuckets], key [B], rank [B], perm [B], int32 each.
size_t loc_bytes(int64_t B)
{
    const size_t words = (size_t)kLocBuckets + 3 * (size_t)B;
    return (words * 4 + 255) & ~(size_t)255;
}

static int sorted_check(const spline_s* s, const double* pos, int64_t B, void* V, void* G, void* L, void* ws,
                        size_t ws_bytes, bool vgl)
{
    if (!s) return fail(SPL_EINVAL, "handle is NULL");
    if (B < 0 || B > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(SPL_EINVAL, "B must be in [0, 2^31)");
    if (B == 0) return SPL_OK;
    if (!pos || !V || (vgl && (!G || !L))) return fail(SPL_EINVAL, "NULL position or output pointer");
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return fail(SPL_EINVAL, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < loc_bytes(B)) return fail(SPL_ENOMEM, "workspace smaller than spline_sorted_workspace_bytes()");
    int64_t tmp;
    if (!mul_ok(B, (int64_t)s->norb * 3 * 8, &tmp)) return fail(SPL_ENOMEM, "output size overflow");
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    if (dev != s->device) return fail(SPL_EINVAL, "current HIP device differs from the table's device");
    return SPL_OK;
}

const int32_t* loc_perm(const void* ws, int64_t B) { return static_cast<const int32_t*>(ws) + kLocBuckets + 2 * B; }

// The sort (four small launches) for workgroups of pb positions (pb <= 0:
// no dealing to XCDs); returns the index list inside the workspace.
int sort_positions(const spline_s* s, const double* pos, int64_t B, int pb, void* ws, hipStream_t st,
                          const int32_t** perm_out)
{
    LocKey k;
    k.general = s->general;
    for (int i = 0; i < 9; ++i) k.ilat[i] = s->ilat[i];
    int bits = 0;
    for (int d = 0; d < 3; ++d) {
        k.inv[d] = 1.0 / s->grid.cell[d];
        k.n[d] = s->grid.n[d];
        int bd = 0;
        while ((1 << bd) < s->grid.n[d]) ++bd;
        bits = bd > bits ? bd : bits;
    }
    k.shift = bits > kLocBits ? bits - kLocBits : 0;
    int32_t* count = static_cast<int32_t*>(ws);
    int32_t* key = count + kLocBuckets;
    int32_t* rank = key + B;
    int32_t* perm = rank + B;
    const unsigned gb = (unsigned)((B + kLocThreads - 1) / kLocThreads);
    hipLaunchKernelGGL(loc_zero_kernel, dim3(kLocBuckets / kLocThreads), dim3(kLocThreads), 0, st, count,
                       kLocBuckets);
    hipLaunchKernelGGL(loc_key_kernel, dim3(gb), dim3(kLocThreads), 0, st, pos, B, k, count, key, rank);
    hipLaunchKernelGGL(loc_scan_kernel, dim3(1), dim3(kLocScanThreads), 0, st, count);
    hipLaunchKernelGGL(loc_scatter_kernel, dim3(gb), dim3(kLocThreads), 0, st, B, (int32_t)pb, count, key, rank,
                       perm);
    QS_HIP(hipGetLastError());
    *perm_out = perm;
    return SPL_OK;
}

// The sort and the evaluation with tile t; arguments already checked.
static int sorted_run(const spline_s* s, const spline_tile& t, bool vgl, const double* pos, int64_t B, void* V,
                      void* G, void* L, void* ws, hipStream_t st)
{
    const Variant* v = find_variant(s->store, t.cw, t.nch, t.lpp, vgl);
    if (!v) return fail(SPL_EUNSUPPORTED, "tile shape not compiled");
    const int32_t* perm = nullptr;
    int rc = sort_positions(s, pos, B, t.pb, ws, st, &perm);
    if (rc) return rc;
    EvalArgs a = make_args(s, t, pos, B, V, G, L);
    a.idx = perm;
    return launch(*v, a, st);
}

// The VGH family in locality order (the Hessian, or the general-cell VGL).
static int sorted_vgh(const spline_s* s, bool hessian, const double* pos, int64_t B, void* V, void* G, void* H,
                      void* ws, hipStream_t st)
{
    const spline_tile t = vgh_sorted_tile(s);
    const int32_t* perm = nullptr;
    int rc = sort_positions(s, pos, B, t.pb, ws, st, &perm);
    if (rc) return rc;
    return vgh_launch_indexed(s, t, hessian, pos, B, V, G, H, perm, st);
}

static int sorted_common(const spline_s* s, const double* pos, int64_t B, void* V, void* G, void* L, void* ws,
                         size_t ws_bytes, void* stream, bool vgl)
{
    int rc = sorted_check(s, pos, B, V, G, L, ws, ws_bytes, vgl);
    if (rc || B == 0) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (s->general) {
        if (!vgl) return fail(SPL_EUNSUPPORTED, "value-only evaluation is built for orthorhombic cells");
        return sorted_vgh(s, false, pos, B, V, G, L, ws, st);
    }
    return sorted_run(s, vgl ? s->stile : s->svtile, vgl, pos, B, V, G, L, ws, st);
}

// Scratch of the entry point that allocates nothing: the sort's bucket
// counts, keys, ranks and index list for up to kStaticMaxPositions
// positions, one copy on every GPU the library runs on, held until the
// process ends.  In host code `scratch` names a host-side stand-in; its
// device address on the current GPU comes from hipGetSymbolAddress, looked
// up once per device and kept in g_scratch_dev.
constexpr int64_t kStaticMaxPositions = int64_t(1) << 19;
constexpr size_t kStaticWords = (size_t)kLocBuckets + 3 * (size_t)kStaticMaxPositions;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) int32_t scratch[kStaticWords];

static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices];

static int static_scratch(void** out)
{
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SPL_EUNSUPPORTED, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255)) return fail(SPL_EHIP, "static scratch not 256-byte aligned");
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return SPL_OK;
}

}  // namespace qs

using namespace qs;

extern "C" {

size_t spline_sorted_workspace_bytes(const spline_t* s, int64_t B)
{
    if (!s || B < 0 || B > (int64_t)std::numeric_limits<int32_t>::max()) return 0;
    return loc_bytes(B);
}

int spline_eval_vgl_sorted(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* L,
                           void* workspace_dev, size_t workspace_bytes, void* stream)
{
    return sorted_common(s, pos_dev, B, V, G, L, workspace_dev, workspace_bytes, stream, true);
}

int spline_eval_vgl_sorted_noalloc(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* L,
                                   void* stream)
{
    if (B > kStaticMaxPositions)
        return fail(SPL_ENOMEM, "B exceeds the static scratch of the no-allocation entry point (524288 positions)");
    if (!s || B <= 0) return sorted_check(s, pos_dev, B, V, G, L, nullptr, 0, true);
    void* ws = nullptr;
    int rc = static_scratch(&ws);
    if (rc) return rc;
    return sorted_common(s, pos_dev, B, V, G, L, ws, kStaticWords * sizeof(int32_t), stream, true);
}

int spline_eval_v_sorted(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* workspace_dev,
                         size_t workspace_bytes, void* stream)
{
    return sorted_common(s, pos_dev, B, V, nullptr, nullptr, workspace_dev, workspace_bytes, stream, false);
}

// Determinant ratio in locality order: as spline_eval_ratio_vgl / _v (the
// row of A^-1 for position b is still ainv + (rows ? rows[b] : b) * ld), with
// the sorted tile shape (the sorted value tile for the ratio alone).  The ratio's
// partial sums follow the tile shape, so the results equal the plain entry
// point's under the same shape.  Positions per workgroup are halved until
// the per-tile partial sums fit in LDS.
static int sorted_ratio(const spline_s* s, const double* pos, int64_t B, const void* ainv, int64_t ld,
                        const int32_t* rows, void* D, void* ws, size_t ws_bytes, void* stream, bool vgl)
{
    if (!s) return fail(SPL_EINVAL, "handle is NULL");
    if (ld < 0) return fail(SPL_EINVAL, "ld must be >= 0");
    int rc = sorted_check(s, pos, B, D, D, D, ws, ws_bytes, false);
    if (rc || B == 0) return rc;
    if (!ainv) return fail(SPL_EINVAL, "NULL inverse-row pointer");
    const uintptr_t eb = s->store == SPL_F64 ? 8 : 4;
    if ((uintptr_t)ainv % eb || (uintptr_t)D % eb)
        return fail(SPL_EINVAL, "inverse rows and outputs must be aligned to their element size");
    if (s->general && vgl) {
        // the VGH-family ratio kernel with the locality-ordered VGH shape
        spline_tile t = vgh_sorted_tile(s);
        rc = ratio_general_tile(s, t);
        if (rc) return rc;
        hipStream_t st = static_cast<hipStream_t>(stream);
        const int32_t* perm = nullptr;
        rc = sort_positions(s, pos, B, t.pb, ws, st, &perm);
        if (rc) return rc;
        return ratio_general(s, t, pos, B, ainv, ld, rows, D, perm, st);
    }
    spline_tile t = vgl ? s->stile : s->svtile;
    const Variant* v = find_variant(s->store, t.cw, t.nch, t.lpp, vgl, true);
    if (!v) return fail(SPL_EUNSUPPORTED, "no determinant-ratio kernel for this tile shape");
    const int64_t tiles = tiles_of(s, t);
    while (t.pb > 1 && launch_lds(*v, t.pb, tiles) > kMaxLds) t.pb /= 2;
    if (launch_lds(*v, t.pb, tiles) > kMaxLds) return fail(SPL_EUNSUPPORTED, "row too wide for the partial sums");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int32_t* perm = nullptr;
    rc = sort_positions(s, pos, B, t.pb, ws, st, &perm);
    if (rc) return rc;
    EvalArgs a = make_args(s, t, pos, B, D, nullptr, nullptr);
    a.ainv = ainv;
    a.ald = ld;
    a.arows = rows;
    a.idx = perm;
    return launch(*v, a, st);
}

int spline_eval_ratio_vgl_sorted(const spline_t* s, const double* pos_dev, int64_t B, const void* ainv_dev,
                                 int64_t ld, const int32_t* rows_dev, void* D, void* workspace_dev,
                                 size_t workspace_bytes, void* stream)
{
    return sorted_ratio(s, pos_dev, B, ainv_dev, ld, rows_dev, D, workspace_dev, workspace_bytes, stream, true);
}

int spline_eval_ratio_v_sorted(const spline_t* s, const double* pos_dev, int64_t B, const void* ainv_dev,
                               int64_t ld, const int32_t* rows_dev, void* R, void* workspace_dev,
                               size_t workspace_bytes, void* stream)
{
    return sorted_ratio(s, pos_dev, B, ainv_dev, ld, rows_dev, R, workspace_dev, workspace_bytes, stream, false);
}

int spline_eval_vgh_sorted(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* H,
                           void* workspace_dev, size_t workspace_bytes, void* stream)
{
    int rc = sorted_check(s, pos_dev, B, V, G, H, workspace_dev, workspace_bytes, true);
    if (rc || B == 0) return rc;
    int64_t tmp;
    if (!mul_ok(B, (int64_t)s->norb * 6 * 8, &tmp)) return fail(SPL_ENOMEM, "output size overflow");
    return sorted_vgh(s, true, pos_dev, B, V, G, H, workspace_dev, static_cast<hipStream_t>(stream));
}

int spline_set_sorted_tile(spline_t* s, const spline_tile* tile)
{
    if (!s) return fail(SPL_EINVAL, "handle is NULL");
    const int rc = check_tile(s, tile, true);
    if (rc) return rc;
    s->stile = *tile;
    if (find_variant(s->store, tile->cw, tile->nch, tile->lpp, false)) s->svtile = *tile;
    return SPL_OK;
}

int spline_get_sorted_tile(const spline_t* s, spline_tile* tile)
{
    if (!s || !tile) return fail(SPL_EINVAL, "NULL argument");
    *tile = s->stile;
    return SPL_OK;
}

// As spline_autotune, over the locality-ordered paths: the VGL shape and the
// value-only shape (also used by the value ratio) are tuned separately, each
// candidate's outputs on the first positions must equal the first
// candidate's bit for bit; cache lines "<key> sorted|cw nch lpp pb" and
// "<key> sorted V|cw nch lpp pb".
int spline_autotune_sorted(spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* L,
                           void* workspace_dev, size_t workspace_bytes, int32_t reps, const char* cache_path,
                           void* stream, spline_tile* chosen)
{
    int rc = sorted_check(s, pos_dev, B, V, G, L, workspace_dev, workspace_bytes, true);
    if (rc) return rc;
    if (B == 0) return fail(SPL_EINVAL, "autotune needs a non-empty batch");
    if (s->general) return fail(SPL_EUNSUPPORTED, "general cells use the VGH-family tile (spline_autotune_vgh)");
    if (reps < 1) reps = 1;
    hipStream_t st = static_cast<hipStream_t>(stream);
    cache_path = tune_cache_path(cache_path);
    const std::string key = tune_key(s, B) + " sorted", vkey = key + " V";
    spline_tile tv{}, tn{};
    const bool have_v = cache_path && cache_lookup(cache_path, key, &tv) && check_tile(s, &tv, true) == SPL_OK;
    const bool have_n = cache_path && cache_lookup(cache_path, vkey, &tn) && check_tile(s, &tn, false) == SPL_OK;
    if (!have_v || !have_n) {
        int32_t n = 0;
        rc = spline_tile_candidates(s, nullptr, 0, &n);
        if (rc) return rc;
        std::vector<spline_tile> cands(n);
        spline_tile_candidates(s, cands.data(), n, &n);
        // Shorter chunks too: fewer positions in flight per XCD keep more of
        // their shared rows in its L2.
        for (int32_t i = 0; i < n; ++i)
            if (cands[i].pb == 16) cands.push_back(spline_tile{cands[i].cw, cands[i].nch, cands[i].lpp, 8});
        if (cands.empty()) return fail(SPL_EUNSUPPORTED, "no candidate tile shapes");
        if (!have_v) {
            rc = tune_kind(s, true, cands, B, V, G, L, reps, st, [&](const spline_tile& t) {
                return sorted_run(s, t, true, pos_dev, B, V, G, L, workspace_dev, st);
            }, &tv);
            if (rc) return rc;
        }
        if (!have_n) {
            rc = tune_kind(s, false, cands, B, V, G, L, reps, st, [&](const spline_tile& t) {
                return sorted_run(s, t, false, pos_dev, B, V, nullptr, nullptr, workspace_dev, st);
            }, &tn);
            if (rc) return rc;
        }
    }
    s->stile = tv;
    s->svtile = tn;
    if (chosen) *chosen = tv;
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        if (f && !have_v) f << key << "|" << tv.cw << " " << tv.nch << " " << tv.lpp << " " << tv.pb << "\n";
        if (f && !have_n) f << vkey << "|" << tn.cw << " " << tn.nch << " " << tn.lpp << " " << tn.pb << "\n";
    }
    return SPL_OK;
}

int spline_get_sorted_vgh_tile(const spline_t* s, spline_tile* tile)
{
    if (!s || !tile) return fail(SPL_EINVAL, "NULL argument");
    *tile = vgh_sorted_tile(s);
    return SPL_OK;
}

int spline_get_sorted_value_tile(const spline_t* s, spline_tile* tile)
{
    if (!s || !tile) return fail(SPL_EINVAL, "NULL argument");
    *tile = s->svtile;
    return SPL_OK;
}

}  // extern "C"
