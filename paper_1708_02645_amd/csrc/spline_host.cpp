// Host runtime of the qmcspline C ABI: argument checks, table layout and
// quantization, kernel-variant selection, launches and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <limits>
#include <sstream>
#include <string>
#include <vector>

#include "common.hpp"

namespace qs {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    g_err = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return SPL_EHIP;
}

const Variant* variants_f32(int*);
const Variant* variants_f64(int*);
const Variant* variants_bf16(int*);
const Variant* variants_f16(int*);
const Variant* ratio_variants_f32(int*);
const Variant* ratio_variants_f64(int*);
const Variant* ratio_variants_bf16(int*);
const Variant* ratio_variants_f16(int*);

// Built once, on first use (a function-local static: thread-safe).
const Variant* variants(int* count)
{
    static const std::vector<Variant> all = [] {
        std::vector<Variant> a;
        for (auto f : {variants_f64, variants_f32, variants_bf16, variants_f16, ratio_variants_f64,
                       ratio_variants_f32, ratio_variants_bf16, ratio_variants_f16}) {
            int n = 0;
            const Variant* v = f(&n);
            a.insert(a.end(), v, v + n);
        }
        return a;
    }();
    *count = (int)all.size();
    return all.data();
}

int launch(const Variant& v, const EvalArgs& a, hipStream_t stream)
{
    const int64_t blocks = (a.B + a.pb - 1) / a.pb;
    if (blocks > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(SPL_EINVAL, "batch too large for one launch");
    EvalArgs args = a;
    void* params[] = {&args};
    const size_t lds = launch_lds(v, a.pb, a.tiles);
    QS_HIP(hipLaunchKernel(v.fn, dim3((unsigned)blocks), dim3(kBlock), params, lds, stream));
    QS_HIP(hipGetLastError());
    return SPL_OK;
}

static int elem_bytes(spline_dtype s)
{
    switch (s) {
    case SPL_F64: return 8;
    case SPL_F32: return 4;
    case SPL_BF16:
    case SPL_F16: return 2;
    default: return 0;  // not a storage type
    }
}

bool mul_ok(int64_t a, int64_t b, int64_t* out)
{
    if (a < 0 || b < 0) return false;
    if (a != 0 && b > std::numeric_limits<int64_t>::max() / a) return false;
    *out = a * b;
    return true;
}

static int compute_layout(const spline_grid* g, int32_t n_orb, spline_dtype store, spline_layout* L)
{
    if (!g) return fail(SPL_EINVAL, "grid is NULL");
    if (!L) return fail(SPL_EINVAL, "layout output is NULL");
    const int es = elem_bytes(store);
    if (es == 0) return fail(SPL_EINVAL, "unknown storage dtype");
    if (n_orb <= 0) return fail(SPL_EINVAL, "n_orb must be positive");
    for (int d = 0; d < 3; ++d) {
        if (g->n[d] <= 0) return fail(SPL_EINVAL, "grid points per axis must be positive");
        if (g->n[d] > (1 << 20)) return fail(SPL_ENOMEM, "grid axis too large");
        if (!(g->cell[d] > 0.0) || !std::isfinite(g->cell[d]))
            return fail(SPL_EINVAL, "cell lengths must be positive and finite");
    }
    int64_t row = 0;
    if (!mul_ok((int64_t)n_orb, es, &row)) return fail(SPL_ENOMEM, "row size overflow");
    // Rows longer than 256 B are padded to a multiple of 256 B.  Shorter rows
    // (a few orbitals per GPU, e.g. one share of an orbital split) are padded
    // only to the narrowest tile compiled for the storage type: 64 B (16
    // lanes x one word), 128 B for FP64 (16 lanes x one double), so a 192-B
    // row is not read as 256 B.
    const int64_t gran = row > 256 ? 256 : (store == SPL_F64 ? 128 : 64);
    row = (row + gran - 1) / gran * gran;
    int64_t rows = 1;
    for (int d = 0; d < 3; ++d)
        if (!mul_ok(rows, (int64_t)g->n[d] + 3, &rows)) return fail(SPL_ENOMEM, "table size overflow");
    int64_t tb = 0;
    if (!mul_ok(rows, row, &tb)) return fail(SPL_ENOMEM, "table size overflow");
    const int64_t n_pad = row / es;
    int64_t sb = 0;
    if (!mul_ok(n_pad, 4, &sb)) return fail(SPL_ENOMEM, "scale size overflow");
    sb = (sb + 255) / 256 * 256;
    if (tb > std::numeric_limits<int64_t>::max() - 256) return fail(SPL_ENOMEM, "table size overflow");
    const int64_t so = (tb + 255) / 256 * 256;  // scales start on a 256-byte boundary
    if (so > std::numeric_limits<int64_t>::max() - sb) return fail(SPL_ENOMEM, "table size overflow");
    L->row_bytes = row;
    L->n_pad = n_pad;
    L->table_bytes = tb;
    L->scales_offset = so;
    L->total_bytes = so + sb;
    L->elem_bytes = es;
    for (int d = 0; d < 3; ++d) L->padded[d] = g->n[d] + 3;
    return SPL_OK;
}

// Round |x| (x finite, nonzero) to p significant bits with minimum exponent
// emin, ties to even, and return the IEEE encoding of the narrow format
// whose exponent bias is 1 - emin (works for BF16 and FP16).
static uint32_t encode_narrow(double x, int p, int emin)
{
    uint64_t u;
    std::memcpy(&u, &x, 8);
    const uint32_t sign = (uint32_t)(u >> 63);
    const int ebits = (int)((u >> 52) & 0x7ff);
    const uint64_t mant = u & ((1ull << 52) - 1);
    if (ebits == 0) return sign << 15;  // zero or FP64 subnormal: far below either format
    const int e = ebits - 1023;
    const uint64_t M = (1ull << 52) | mant;  // value = M * 2^(e-52)
    const int E = e > emin ? e : emin;
    const int shift = 52 - e + E - (p - 1);  // units of 2^(E-p+1)
    uint64_t k;
    if (shift >= 64) {
        k = 0;
    } else {
        k = M >> shift;
        const uint64_t r = M & ((1ull << shift) - 1);
        const uint64_t half = 1ull << (shift - 1);
        if (r > half || (r == half && (k & 1))) ++k;
    }
    const int bias = 1 - emin;
    const uint32_t bits = (uint32_t)(((uint64_t)(E + bias - 1) << (p - 1)) + k);
    return (sign << 15) | bits;
}

// Smallest power of two >= m (m > 0, finite).
static double pow2_ceil(double m)
{
    uint64_t u;
    std::memcpy(&u, &m, 8);
    const int ebits = (int)((u >> 52) & 0x7ff);
    const uint64_t mant = u & ((1ull << 52) - 1);
    if (ebits == 0) return std::ldexp(1.0, -1022);  // subnormal: 2^-1022 bounds it
    if (mant == 0) return m;
    return std::ldexp(1.0, ebits - 1023 + 1);
}

}  // namespace qs

using namespace qs;

extern "C" {

const char* spline_last_error(void) { return g_err.c_str(); }

size_t spline_table_bytes(const spline_grid* grid, int32_t n_orb, spline_dtype store)
{
    spline_layout L;
    if (compute_layout(grid, n_orb, store, &L) != SPL_OK) return 0;
    return (size_t)L.total_bytes;
}

int spline_get_layout(const spline_grid* grid, int32_t n_orb, spline_dtype store, spline_layout* out)
{
    return compute_layout(grid, n_orb, store, out);
}

int spline_pack_host(const spline_grid* grid, int32_t n_orb, const double* coefs, spline_dtype store,
                     void* host_buf, size_t buf_bytes)
{
    spline_layout L;
    int rc = compute_layout(grid, n_orb, store, &L);
    if (rc) return rc;
    if (!coefs) return fail(SPL_EINVAL, "coefs is NULL");
    if (!host_buf) return fail(SPL_EINVAL, "host buffer is NULL");
    if (buf_bytes < (size_t)L.total_bytes) return fail(SPL_ENOMEM, "host buffer smaller than spline_table_bytes()");
    const int64_t n0 = grid->n[0], n1 = grid->n[1], n2 = grid->n[2];
    const int64_t N = n_orb;
    unsigned char* out = static_cast<unsigned char*>(host_buf);

    // Per-orbital scales (16-bit stores only; 1 otherwise and for padding).
    std::vector<double> scale(L.n_pad, 1.0);
    if (store == SPL_BF16 || store == SPL_F16) {
        std::vector<double> mx(N, 0.0);
        const int64_t npts = n0 * n1 * n2;
        for (int64_t j = 0; j < npts; ++j) {
            const double* c = coefs + j * N;
            for (int64_t m = 0; m < N; ++m) {
                const double a = std::fabs(c[m]);
                if (a > mx[m]) mx[m] = a;
            }
        }
        for (int64_t m = 0; m < N; ++m) {
            if (!std::isfinite(mx[m])) return fail(SPL_EINVAL, "non-finite coefficient");
            scale[m] = mx[m] > 0.0 ? pow2_ceil(mx[m]) : 1.0;
        }
    }
    float* sc = reinterpret_cast<float*>(out + L.scales_offset);
    std::memset(out + L.table_bytes, 0, (size_t)(L.total_bytes - L.table_bytes));  // gap before the scales too
    for (int64_t m = 0; m < L.n_pad; ++m) sc[m] = (float)scale[m];

    std::vector<double> inv(N);
    for (int64_t m = 0; m < N; ++m) inv[m] = 1.0 / scale[m];  // exact: powers of two

    const int64_t P0 = n0 + 3, P1 = n1 + 3, P2 = n2 + 3;
    const int64_t row = L.row_bytes;
    for (int64_t p0 = 0; p0 < P0; ++p0) {
        const int64_t j0 = ((p0 - 1) % n0 + n0) % n0;
        for (int64_t p1 = 0; p1 < P1; ++p1) {
            const int64_t j1 = ((p1 - 1) % n1 + n1) % n1;
            for (int64_t p2 = 0; p2 < P2; ++p2) {
                const int64_t j2 = ((p2 - 1) % n2 + n2) % n2;
                const double* c = coefs + ((j0 * n1 + j1) * n2 + j2) * N;
                unsigned char* r = out + ((p0 * P1 + p1) * P2 + p2) * row;
                std::memset(r, 0, (size_t)row);
                switch (store) {
                case SPL_F64:
                    for (int64_t m = 0; m < N; ++m)
                        if (!std::isfinite(c[m])) return fail(SPL_EINVAL, "non-finite coefficient");
                    std::memcpy(r, c, (size_t)(N * 8));
                    break;
                case SPL_F32: {
                    float* f = reinterpret_cast<float*>(r);
                    for (int64_t m = 0; m < N; ++m) {
                        if (!std::isfinite(c[m])) return fail(SPL_EINVAL, "non-finite coefficient");
                        f[m] = (float)c[m];  // round to nearest even
                    }
                    break;
                }
                case SPL_BF16:
                case SPL_F16: {
                    uint16_t* h = reinterpret_cast<uint16_t*>(r);
                    const int p = store == SPL_BF16 ? 8 : 11;
                    const int emin = store == SPL_BF16 ? -126 : -14;
                    for (int64_t m = 0; m < N; ++m) {
                        const double x = c[m] * inv[m];
                        if (!std::isfinite(x)) return fail(SPL_EINVAL, "non-finite coefficient");
                        h[m] = (uint16_t)encode_narrow(x, p, emin);
                    }
                    break;
                }
                default:
                    break;  // unreachable: compute_layout rejected the type
                }
            }
        }
    }
    return SPL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Tile shapes

namespace qs {

// A tile shape fits when whole tiles cover the padded row exactly.
bool tile_fits(const spline_s* s, const Variant& v)
{
    const int64_t tb = (int64_t)v.lpp * v.cw * 4 * v.nch;
    return v.store == s->store && s->layout.row_bytes % tb == 0;
}

const Variant* find_variant(spline_dtype st, int cw, int nch, int lpp, bool vgl, bool ratio)
{
    int n = 0;
    const Variant* vs = variants(&n);
    for (int i = 0; i < n; ++i)
        if (vs[i].store == st && vs[i].cw == cw && vs[i].nch == nch && vs[i].lpp == lpp && vs[i].vgl == vgl &&
            vs[i].ratio == ratio)
            return &vs[i];
    return nullptr;
}

int64_t tiles_of(const spline_s* s, const spline_tile& t)
{
    const int64_t tb = (int64_t)t.lpp * t.nch * t.cw * 4;
    return (s->layout.row_bytes + tb - 1) / tb;
}

// Default: whole-wave groups first, as few tiles as possible with at most 6
// dwords per lane, wasting as few loaded bytes as possible.
static spline_tile default_tile(const spline_s* s, bool vgl)
{
    int n = 0;
    const Variant* vs = variants(&n);
    spline_tile best{0, 0, 0, 32};
    double best_score = 1e300;
    for (int i = 0; i < n; ++i) {
        const Variant& v = vs[i];
        if (v.vgl != vgl || v.ratio || !tile_fits(s, v)) continue;
        const int words = v.cw * v.nch;
        if (words > 6) continue;
        spline_tile t{v.cw, v.nch, v.lpp, 32};
        const int64_t T = tiles_of(s, t);
        const int64_t tb = (int64_t)v.lpp * v.nch * v.cw * 4;
        const double waste = (double)(T * tb - s->layout.row_bytes) / (double)s->layout.row_bytes;
        // prefer: little waste, full waves when the row is wide enough, wide chunks
        double score = waste * 100.0 + (double)T * 0.5 + (v.lpp == 64 ? 0.0 : 2.0) - words * 0.1 +
                       (v.cw == 3 ? 0.05 : 0.0);
        if (s->layout.row_bytes < 64 * 4 * v.cw) score -= (v.lpp == 64 ? 0.0 : 3.0);
        if (score < best_score) {
            best_score = score;
            best = t;
        }
    }
    return best;
}

int check_tile(const spline_s* s, const spline_tile* t, bool vgl)
{
    if (!t) return fail(SPL_EINVAL, "tile is NULL");
    if (t->pb < 1 || t->pb > 256) return fail(SPL_EINVAL, "positions per workgroup must be in [1, 256]");
    const Variant* v = find_variant(s->store, t->cw, t->nch, t->lpp, vgl);
    if (!v) return fail(SPL_EUNSUPPORTED, "tile shape not compiled for this storage type");
    if (!tile_fits(s, *v)) return fail(SPL_EUNSUPPORTED, "tile chunk width does not divide the row");
    if (v->lds_per_pos * (size_t)t->pb > 64 * 1024) return fail(SPL_EUNSUPPORTED, "too many positions per workgroup");
    return SPL_OK;
}

EvalArgs make_args(const spline_s* s, const spline_tile& t, const double* pos, int64_t B, void* V, void* G,
                          void* L)
{
    EvalArgs a{};
    a.table = s->dev;
    a.scales = reinterpret_cast<const float*>(s->dev + s->layout.scales_offset);
    a.pos = pos;
    a.V = V;
    a.G = G;
    a.L = L;
    a.B = B;
    a.row_bytes = s->layout.row_bytes;
    a.ystride = (int64_t)s->layout.padded[2] * s->layout.row_bytes;
    a.xstride = (int64_t)s->layout.padded[1] * a.ystride;
    for (int d = 0; d < 3; ++d) {
        a.cell[d] = s->grid.cell[d];
        a.n[d] = s->grid.n[d];
    }
    a.norb = s->norb;
    a.tiles = (int32_t)tiles_of(s, t);
    a.pb = t.pb;
    if (s->general) set_general_args(s, a);
    return a;
}

static int run_eval(const spline_s* s, const spline_tile& t, bool vgl, const double* pos, int64_t B, void* V,
                    void* G, void* L, hipStream_t stream)
{
    const Variant* v = find_variant(s->store, t.cw, t.nch, t.lpp, vgl);
    if (!v) return fail(SPL_EUNSUPPORTED, "tile shape not compiled");
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    if (dev != s->device) return fail(SPL_EINVAL, "current HIP device differs from the table's device");
    return launch(*v, make_args(s, t, pos, B, V, G, L), stream);
}

}  // namespace qs

extern "C" {

int spline_create(const spline_grid* grid, int32_t n_orb, const double* coefs_host, spline_dtype store,
                  void* table_dev, size_t table_bytes, void* stream, spline_t** out)
{
    if (!out) return fail(SPL_EINVAL, "out is NULL");
    *out = nullptr;
    spline_layout L;
    int rc = compute_layout(grid, n_orb, store, &L);
    if (rc) return rc;
    if (!coefs_host) return fail(SPL_EINVAL, "coefs is NULL");
    if (!table_dev) return fail(SPL_EINVAL, "device buffer is NULL");
    if ((reinterpret_cast<uintptr_t>(table_dev) & 255) != 0) return fail(SPL_EINVAL, "device buffer not 256-byte aligned");
    if (table_bytes < (size_t)L.total_bytes) return fail(SPL_ENOMEM, "device buffer smaller than spline_table_bytes()");
    std::vector<unsigned char> host;
    try {
        host.resize((size_t)L.total_bytes);
    } catch (...) {
        return fail(SPL_ENOMEM, "host staging allocation failed");
    }
    rc = spline_pack_host(grid, n_orb, coefs_host, store, host.data(), host.size());
    if (rc) return rc;
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    hipStream_t st = static_cast<hipStream_t>(stream);
    QS_HIP(hipMemcpyAsync(table_dev, host.data(), host.size(), hipMemcpyHostToDevice, st));
    QS_HIP(hipStreamSynchronize(st));
    spline_s* s = new (std::nothrow) spline_s;
    if (!s) return fail(SPL_ENOMEM, "handle allocation failed");
    s->grid = *grid;
    s->norb = n_orb;
    s->store = store;
    s->layout = L;
    s->dev = static_cast<unsigned char*>(table_dev);
    s->device = dev;
    s->tile = default_tile(s, true);
    s->vtile = default_tile(s, false);
    s->htile = default_vgh_tile(s);
    s->stile = s->tile;
    s->svtile = s->vtile;
    s->general = 0;
    if (s->tile.cw == 0 || s->vtile.cw == 0 || s->htile.cw == 0) {
        delete s;
        return fail(SPL_EUNSUPPORTED, "no compiled tile shape fits this row width");
    }
    *out = s;
    return SPL_OK;
}

int spline_destroy(spline_t* s)
{
    delete s;
    return SPL_OK;
}

int spline_get_info(const spline_t* s, spline_grid* grid, int32_t* n_orb, spline_dtype* store, spline_layout* layout)
{
    if (!s) return fail(SPL_EINVAL, "handle is NULL");
    if (grid) *grid = s->grid;
    if (n_orb) *n_orb = s->norb;
    if (store) *store = s->store;
    if (layout) *layout = s->layout;
    return SPL_OK;
}

static int eval_common(const spline_t* s, const double* pos, int64_t B, void* V, void* G, void* L, void* stream,
                       bool vgl)
{
    if (!s) return fail(SPL_EINVAL, "handle is NULL");
    if (B < 0) return fail(SPL_EINVAL, "B must be >= 0");
    if (B == 0) return SPL_OK;
    if (!pos || !V || (vgl && (!G || !L))) return fail(SPL_EINVAL, "NULL position or output pointer");
    int64_t tmp;
    if (!mul_ok(B, (int64_t)s->norb * 3 * 8, &tmp)) return fail(SPL_ENOMEM, "output size overflow");
    if (s->general && vgl) return vgl_general(s, pos, B, V, G, L, static_cast<hipStream_t>(stream));
    return run_eval(s, vgl ? s->tile : s->vtile, vgl, pos, B, V, G, L, static_cast<hipStream_t>(stream));
}

int spline_eval_vgl(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* L, void* stream)
{
    return eval_common(s, pos_dev, B, V, G, L, stream, true);
}

int spline_eval_v(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* stream)
{
    return eval_common(s, pos_dev, B, V, nullptr, nullptr, stream, false);
}

// Determinant-ratio launches use the table's VGL (value) tile shape; the
// positions per workgroup are halved until the per-tile partial sums fit in
// LDS next to the staged weights.
static int ratio_common(const spline_t* s, const double* pos, int64_t B, const void* ainv, int64_t ld,
                        const int32_t* rows, void* D, void* stream, bool vgl)
{
    if (!s) return fail(SPL_EINVAL, "handle is NULL");
    if (B < 0) return fail(SPL_EINVAL, "B must be >= 0");
    if (ld < 0) return fail(SPL_EINVAL, "ld must be >= 0");
    if (B == 0) return SPL_OK;
    if (!pos || !ainv || !D) return fail(SPL_EINVAL, "NULL position, inverse-row or output pointer");
    const uintptr_t eb = s->store == SPL_F64 ? 8 : 4;
    if ((uintptr_t)ainv % eb || (uintptr_t)D % eb)
        return fail(SPL_EINVAL, "inverse rows and outputs must be aligned to their element size");
    int64_t tmp;
    if (!mul_ok(B, 5 * 8, &tmp)) return fail(SPL_ENOMEM, "output size overflow");
    if (s->general && vgl) {
        // the VGH-family kernel with the ratio epilogue (Cartesian G and L)
        spline_tile t = s->htile;
        int rc = ratio_general_tile(s, t);
        if (rc) return rc;
        int dev = -1;
        QS_HIP(hipGetDevice(&dev));
        if (dev != s->device) return fail(SPL_EINVAL, "current HIP device differs from the table's device");
        return ratio_general(s, t, pos, B, ainv, ld, rows, D, nullptr, static_cast<hipStream_t>(stream));
    }
    spline_tile t = vgl ? s->tile : s->vtile;
    const Variant* v = find_variant(s->store, t.cw, t.nch, t.lpp, vgl, true);
    if (!v) return fail(SPL_EUNSUPPORTED, "no determinant-ratio kernel for this tile shape");
    const int64_t tiles = tiles_of(s, t);
    while (t.pb > 1 && launch_lds(*v, t.pb, tiles) > kMaxLds) t.pb /= 2;
    if (launch_lds(*v, t.pb, tiles) > kMaxLds) return fail(SPL_EUNSUPPORTED, "row too wide for the partial sums");
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    if (dev != s->device) return fail(SPL_EINVAL, "current HIP device differs from the table's device");
    EvalArgs a = make_args(s, t, pos, B, D, nullptr, nullptr);
    a.ainv = ainv;
    a.ald = ld;
    a.arows = rows;
    return launch(*v, a, static_cast<hipStream_t>(stream));
}

int spline_eval_ratio_vgl(const spline_t* s, const double* pos_dev, int64_t B, const void* ainv_dev, int64_t ld,
                          const int32_t* rows_dev, void* D, void* stream)
{
    return ratio_common(s, pos_dev, B, ainv_dev, ld, rows_dev, D, stream, true);
}

int spline_eval_ratio_v(const spline_t* s, const double* pos_dev, int64_t B, const void* ainv_dev, int64_t ld,
                        const int32_t* rows_dev, void* R, void* stream)
{
    return ratio_common(s, pos_dev, B, ainv_dev, ld, rows_dev, R, stream, false);
}

int spline_tile_candidates(const spline_t* s, spline_tile* out, int32_t cap, int32_t* n)
{
    if (!s || !n) return fail(SPL_EINVAL, "NULL argument");
    if (cap > 0 && !out) return fail(SPL_EINVAL, "NULL output with positive capacity");
    int nv = 0;
    const Variant* vs = variants(&nv);
    int32_t k = 0;
    for (int i = 0; i < nv; ++i) {
        const Variant& v = vs[i];
        if (!v.vgl || v.ratio || !tile_fits(s, v)) continue;
        for (int pb : {16, 32, 64}) {
            if (v.lds_per_pos * (size_t)pb > 64 * 1024) continue;
            if (k < cap) out[k] = spline_tile{v.cw, v.nch, v.lpp, pb};
            ++k;
        }
    }
    *n = k;
    return SPL_OK;
}

int spline_set_tile(spline_t* s, const spline_tile* tile)
{
    if (!s) return fail(SPL_EINVAL, "handle is NULL");
    int rc = check_tile(s, tile, true);
    if (rc) return rc;
    s->tile = *tile;
    if (find_variant(s->store, tile->cw, tile->nch, tile->lpp, false)) {
        s->vtile = *tile;
    }
    return SPL_OK;
}

int spline_get_tile(const spline_t* s, spline_tile* tile)
{
    if (!s || !tile) return fail(SPL_EINVAL, "NULL argument");
    *tile = s->tile;
    return SPL_OK;
}

int spline_get_value_tile(const spline_t* s, spline_tile* tile)
{
    if (!s || !tile) return fail(SPL_EINVAL, "NULL argument");
    *tile = s->vtile;
    return SPL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner

namespace qs {

std::string tune_key(const spline_s* s, int64_t B)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, s->device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    int bucket = 0;
    while ((1ll << (bucket + 1)) <= B) ++bucket;
    std::ostringstream k;
    k << arch << " " << s->grid.n[0] << "x" << s->grid.n[1] << "x" << s->grid.n[2] << " N" << s->norb << " S"
      << (int)s->store << " B2^" << bucket;
    return k.str();
}

const char* tune_cache_path(const char* given)
{
    if (given) return given;
    const char* env = std::getenv("QMCSPLINE_TUNE_CACHE");
    return env && env[0] ? env : nullptr;
}

bool cache_lookup(const char* path, const std::string& key, spline_tile* t)
{
    std::ifstream f(path);
    if (!f) return false;
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        const size_t bar = line.find('|');
        if (bar == std::string::npos) continue;
        if (line.substr(0, bar) != key) continue;
        std::istringstream r(line.substr(bar + 1));
        spline_tile x{};
        if (r >> x.cw >> x.nch >> x.lpp >> x.pb) {
            *t = x;
            found = true;  // last matching entry wins
        }
    }
    return found;
}

}  // namespace qs

namespace qs {

// The accumulation order does not depend on the tile shape, so every
// candidate must give the first one's outputs bit for bit.
int tune_kind(const spline_s* s, bool vgl, const std::vector<spline_tile>& cands, int64_t B, void* V, void* G,
              void* L, int32_t reps, hipStream_t st, const std::function<int(const spline_tile&)>& run,
              spline_tile* best_t)
{
    const int64_t Bc = std::min<int64_t>(B, 512);
    const size_t ob = s->store == SPL_F64 ? 8 : 4;
    const size_t nv = (size_t)Bc * s->norb * ob;
    const size_t nq = vgl ? 5 : 1;
    std::vector<unsigned char> ref, cur(nv * nq);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(SPL_EHIP, "hipEventCreate failed");
    }
    int rc = SPL_OK;
    float best = 1e30f;
    *best_t = cands[0];
    for (size_t i = 0; i < cands.size(); ++i) {
        spline_tile t = cands[i];
        if (!vgl && !find_variant(s->store, t.cw, t.nch, t.lpp, false)) continue;
        rc = run(t);
        if (rc) break;
        bool copied = hipMemcpyAsync(cur.data(), V, nv, hipMemcpyDeviceToHost, st) == hipSuccess;
        if (vgl)
            copied = copied && hipMemcpyAsync(cur.data() + nv, G, 3 * nv, hipMemcpyDeviceToHost, st) == hipSuccess &&
                     hipMemcpyAsync(cur.data() + 4 * nv, L, nv, hipMemcpyDeviceToHost, st) == hipSuccess;
        if (!copied || hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(SPL_EHIP, "autotune: copy of outputs failed");
            break;
        }
        if (ref.empty()) {
            ref = cur;
        } else if (std::memcmp(ref.data(), cur.data(), ref.size()) != 0) {
            std::ostringstream m;
            m << "autotune: tile (" << t.cw << "," << t.nch << "," << t.lpp << "," << t.pb
              << ") differs bitwise from the first candidate";
            rc = fail(SPL_EUNSUPPORTED, m.str());
            break;
        }
        if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(SPL_EHIP, "event record"); break; }
        for (int r = 0; r < reps && rc == SPL_OK; ++r) rc = run(t);
        if (rc) break;
        float ms = 0.f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(SPL_EHIP, "autotune: event timing failed");
            break;
        }
        if (ms < best) {
            best = ms;
            *best_t = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace qs

// The VGL and the value-only shapes are tuned separately; cache lines are
// "<key>|cw nch lpp pb" for VGL and "<key> V|cw nch lpp pb" for value only.
extern "C" int spline_autotune(spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* L, int32_t reps,
                               const char* cache_path, void* stream, spline_tile* chosen)
{
    if (!s) return fail(SPL_EINVAL, "handle is NULL");
    if (B <= 0 || !pos_dev || !V || !G || !L) return fail(SPL_EINVAL, "autotune needs a non-empty batch and outputs");
    if (reps < 1) reps = 1;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (s->general) return vgh_autotune(s, 1 /* general-cell VGL */, pos_dev, B, V, G, L, reps, st, chosen);
    cache_path = tune_cache_path(cache_path);
    const std::string key = tune_key(s, B), vkey = key + " V";
    spline_tile tv{}, tn{};
    const bool have_v = cache_path && cache_lookup(cache_path, key, &tv) && check_tile(s, &tv, true) == SPL_OK;
    const bool have_n = cache_path && cache_lookup(cache_path, vkey, &tn) && check_tile(s, &tn, false) == SPL_OK;
    if (have_v && have_n) {
        s->tile = tv;
        s->vtile = tn;
        if (chosen) *chosen = tv;
        return SPL_OK;
    }
    int32_t n = 0;
    int rc = spline_tile_candidates(s, nullptr, 0, &n);
    if (rc) return rc;
    std::vector<spline_tile> cands(n);
    spline_tile_candidates(s, cands.data(), n, &n);
    if (n == 0) return fail(SPL_EUNSUPPORTED, "no candidate tile shapes");
    if (!have_v) {
        rc = tune_kind(s, true, cands, B, V, G, L, reps, st,
                       [&](const spline_tile& t) { return run_eval(s, t, true, pos_dev, B, V, G, L, st); }, &tv);
        if (rc) return rc;
    }
    if (!have_n) {
        rc = tune_kind(s, false, cands, B, V, G, L, reps, st,
                       [&](const spline_tile& t) { return run_eval(s, t, false, pos_dev, B, V, G, L, st); }, &tn);
        if (rc) return rc;
    }
    s->tile = tv;
    s->vtile = tn;
    if (chosen) *chosen = tv;
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        if (f && !have_v) f << key << "|" << tv.cw << " " << tv.nch << " " << tv.lpp << " " << tv.pb << "\n";
        if (f && !have_n) f << vkey << "|" << tn.cw << " " << tn.nch << " " << tn.lpp << " " << tn.pb << "\n";
    }
    return SPL_OK;
}
