// Host side of the value-gradient-Hessian family and of general (triclinic)
// cells: lattice set-up, the grid-to-Cartesian maps passed to the kernels,
// tile selection and autotuning, and the launches.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <sstream>
#include <vector>

#include "common.hpp"
#include "vgh_kernel.hpp"

namespace qs {

const VghVariant* vgh_variants_f64(int*);
const VghVariant* vgh_variants_f32(int*);
const VghVariant* vgh_variants_bf16(int*);
const VghVariant* vgh_variants_f16(int*);

// Built once, on first use (a function-local static: thread-safe).
static const std::vector<VghVariant>& vgh_all()
{
    static const std::vector<VghVariant> all = [] {
        std::vector<VghVariant> a;
        for (auto f : {vgh_variants_f64, vgh_variants_f32, vgh_variants_bf16, vgh_variants_f16}) {
            int n = 0;
            const VghVariant* v = f(&n);
            a.insert(a.end(), v, v + n);
        }
        return a;
    }();
    return all;
}

static const VghVariant* find_vgh(spline_dtype st, const spline_tile& t, int out)
{
    for (const VghVariant& v : vgh_all())
        if (v.store == st && v.cw == t.cw && v.nch == t.nch && v.lpp == t.lpp && v.out == out) return &v;
    return nullptr;
}

static bool vgh_fits(const spline_s* s, const VghVariant& v)
{
    const int64_t tb = (int64_t)v.lpp * v.cw * 4 * v.nch;
    return v.store == s->store && s->layout.row_bytes % tb == 0;
}

bool vgh_variant_fits(const spline_s* s, const VghVariant& v) { return vgh_fits(s, v); }

std::vector<const VghVariant*> vgh_plan_variants(spline_dtype store)
{
    std::vector<const VghVariant*> r;
    for (const VghVariant& v : vgh_all())
        if (v.store == store && v.out == VGH_OUT_L && v.plan_fn) r.push_back(&v);
    return r;
}

// Candidate VGH-family shapes for this table (OUT_H entries stand for both).
static std::vector<spline_tile> vgh_candidates(const spline_s* s)
{
    std::vector<spline_tile> c;
    for (const VghVariant& v : vgh_all()) {
        if (v.out != VGH_OUT_H || !vgh_fits(s, v)) continue;
        for (int pb : {16, 32, 64})
            if (v.lds_per_pos * (size_t)pb <= kMaxLds) c.push_back(spline_tile{v.cw, v.nch, v.lpp, pb});
    }
    return c;
}

// Default: whole waves, few tiles, as many values per lane as fit.
spline_tile default_vgh_tile(const spline_s* s)
{
    spline_tile best{0, 0, 0, 32};
    double best_score = 1e300;
    for (const VghVariant& v : vgh_all()) {
        if (v.out != VGH_OUT_H || !vgh_fits(s, v)) continue;
        spline_tile t{v.cw, v.nch, v.lpp, 32};
        const double T = (double)tiles_of(s, t);
        const double score = T * 0.5 + (v.lpp == 64 ? 0.0 : 2.0) - 0.1 * v.cw * v.nch;
        if (score < best_score) {
            best_score = score;
            best = t;
        }
    }
    return best;
}

// Inverse of a row-major 3x3 matrix by cofactors; false if singular or not finite.
static bool inv3(const double m[9], double r[9])
{
    const double c00 = m[4] * m[8] - m[5] * m[7];
    const double c01 = m[5] * m[6] - m[3] * m[8];
    const double c02 = m[3] * m[7] - m[4] * m[6];
    const double det = m[0] * c00 + m[1] * c01 + m[2] * c02;
    double scale = 0.0;
    for (int i = 0; i < 9; ++i) scale = std::max(scale, std::fabs(m[i]));
    if (!std::isfinite(det) || scale == 0.0 || std::fabs(det) <= 1e-12 * scale * scale * scale) return false;
    r[0] = c00 / det;
    r[1] = (m[2] * m[7] - m[1] * m[8]) / det;
    r[2] = (m[1] * m[5] - m[2] * m[4]) / det;
    r[3] = c01 / det;
    r[4] = (m[0] * m[8] - m[2] * m[6]) / det;
    r[5] = (m[2] * m[3] - m[0] * m[5]) / det;
    r[6] = c02 / det;
    r[7] = (m[1] * m[6] - m[0] * m[7]) / det;
    r[8] = (m[0] * m[4] - m[1] * m[3]) / det;
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(r[i])) return false;
    return true;
}

// Inverse lattice of a handle: the general one, or diag(1 / cell).
static void handle_ilat(const spline_s* s, double il[9])
{
    if (s->general) {
        std::memcpy(il, s->ilat, sizeof(s->ilat));
        return;
    }
    for (int i = 0; i < 9; ++i) il[i] = 0.0;
    for (int d = 0; d < 3; ++d) il[4 * d] = 1.0 / s->grid.cell[d];
}

void set_general_args(const spline_s* s, EvalArgs& a)
{
    handle_ilat(s, a.ilat);
    a.general = 1;
}

// Kernel arguments of a VGH-family launch: grid-frame weights (general
// staging) and the maps M, P, K to Cartesian coordinates.
static VghArgs make_vgh_args(const spline_s* s, const spline_tile& t, const double* pos, int64_t B, void* V, void* G,
                             void* H)
{
    VghArgs va{};
    va.e = make_args(s, t, pos, B, V, G, nullptr);
    set_general_args(s, va.e);
    va.H = H;
    double M[9];
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) M[c * 3 + d] = va.e.ilat[c * 3 + d] * (double)s->grid.n[d];
    static const int hc[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    double P[36], K[6] = {0, 0, 0, 0, 0, 0};
    for (int h = 0; h < 6; ++h) {
        const int c = hc[h][0], e = hc[h][1];
        for (int k = 0; k < 6; ++k) {
            const int d = hc[k][0], f = hc[k][1];
            double v = M[c * 3 + d] * M[e * 3 + f];
            if (d != f) v += M[c * 3 + f] * M[e * 3 + d];
            P[h * 6 + k] = v;
        }
    }
    for (int k = 0; k < 6; ++k) K[k] = P[0 * 6 + k] + P[3 * 6 + k] + P[5 * 6 + k];
    for (int i = 0; i < 9; ++i) {
        va.Md[i] = M[i];
        va.Mf[i] = (float)M[i];
    }
    for (int i = 0; i < 36; ++i) {
        va.Pd[i] = P[i];
        va.Pf[i] = (float)P[i];
    }
    for (int i = 0; i < 6; ++i) {
        va.Kd[i] = K[i];
        va.Kf[i] = (float)K[i];
    }
    return va;
}

// LDS of a VGH-family launch: the staged weights, and for the ratio the
// per-(position, tile) partial sums after them.
static size_t vgh_lds(const spline_s* s, const VghVariant& v, const spline_tile& t)
{
    size_t per = v.lds_per_pos;
    if (v.out == VGH_OUT_RATIO) per += (size_t)tiles_of(s, t) * 5 * (s->store == SPL_F64 ? 8 : 4);
    return per * (size_t)t.pb;
}

VghArgs vgh_args(const spline_s* s, const spline_tile& t, const double* pos, int64_t B, void* V, void* G, void* H)
{
    return make_vgh_args(s, t, pos, B, V, G, H);
}

static int vgh_launch(const spline_s* s, const spline_tile& t, int out, const double* pos, int64_t B, void* V,
                      void* G, void* H, hipStream_t st, const int32_t* idx = nullptr, const void* ainv = nullptr,
                      int64_t ld = 0, const int32_t* rows = nullptr)
{
    const VghVariant* v = find_vgh(s->store, t, out);
    if (!v || !vgh_fits(s, *v)) return fail(SPL_EUNSUPPORTED, "tile shape not compiled for the VGH kernels");
    if (t.pb < 1 || vgh_lds(s, *v, t) > kMaxLds) return fail(SPL_EUNSUPPORTED, "bad positions per workgroup");
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    if (dev != s->device) return fail(SPL_EINVAL, "current HIP device differs from the table's device");
    const int64_t blocks = (B + t.pb - 1) / t.pb;
    if (blocks > (int64_t)std::numeric_limits<int32_t>::max()) return fail(SPL_EINVAL, "batch too large for one launch");
    VghArgs va = make_vgh_args(s, t, pos, B, V, G, H);
    va.e.idx = idx;
    va.e.ainv = ainv;
    va.e.ald = ld;
    va.e.arows = rows;
    void* params[] = {&va};
    QS_HIP(hipLaunchKernel(v->fn, dim3((unsigned)blocks), dim3(kBlock), params, vgh_lds(s, *v, t), st));
    QS_HIP(hipGetLastError());
    return SPL_OK;
}

int ratio_general_tile(const spline_s* s, spline_tile& t)
{
    const VghVariant* v = find_vgh(s->store, t, VGH_OUT_RATIO);
    if (!v || !vgh_fits(s, *v)) return fail(SPL_EUNSUPPORTED, "tile shape not compiled for the VGH kernels");
    while (t.pb > 1 && vgh_lds(s, *v, t) > kMaxLds) t.pb /= 2;
    if (vgh_lds(s, *v, t) > kMaxLds) return fail(SPL_EUNSUPPORTED, "row too wide for the partial sums");
    return SPL_OK;
}

int ratio_general(const spline_s* s, const spline_tile& t, const double* pos, int64_t B, const void* ainv, int64_t ld,
                  const int32_t* rows, void* D, const int32_t* idx, hipStream_t st)
{
    return vgh_launch(s, t, VGH_OUT_RATIO, pos, B, D, nullptr, nullptr, st, idx, ainv, ld, rows);
}

// General-cell VGL (used by spline_eval_vgl for a handle with a lattice).
int vgl_general(const spline_s* s, const double* pos, int64_t B, void* V, void* G, void* L, hipStream_t st)
{
    return vgh_launch(s, s->htile, VGH_OUT_L, pos, B, V, G, L, st);
}

// The VGH family (Hessian, or the general-cell Laplacian) through an index
// list (locality-ordered evaluation).
int vgh_launch_indexed(const spline_s* s, const spline_tile& t, bool hessian, const double* pos, int64_t B, void* V,
                       void* G, void* H, const int32_t* idx, hipStream_t st)
{
    return vgh_launch(s, t, hessian ? VGH_OUT_H : VGH_OUT_L, pos, B, V, G, H, st, idx);
}

// In locality order the rows of neighbouring positions come from cache and
// the shape decides the speed (on the plain path, bound by HBM, the VGH
// tuner's candidates are equal within noise, and its pick can be 20% slower
// here): 16-lane groups with the widest chunk (16, 12, 8 or 4 bytes) that fits.
spline_tile vgh_sorted_tile(const spline_s* s)
{
    spline_tile t = s->htile;
    for (int cw : {4, 3, 2, 1}) {
        const spline_tile c{cw, 1, 16, t.pb};
        const VghVariant* v = find_vgh(s->store, c, VGH_OUT_H);
        if (v && vgh_fits(s, *v) && find_vgh(s->store, c, VGH_OUT_L)) {
            t = c;
            break;
        }
    }
    t.pb = std::min(t.pb, 8);  // fewer positions in flight per XCD keep more shared rows in its L2
    return t;
}

static int check_outputs(const spline_s* s, const double* pos, int64_t B, void* V, void* G, void* H)
{
    if (!s) return fail(SPL_EINVAL, "handle is NULL");
    if (B < 0) return fail(SPL_EINVAL, "B must be >= 0");
    if (B == 0) return SPL_OK;
    if (!pos || !V || !G || !H) return fail(SPL_EINVAL, "NULL position or output pointer");
    int64_t tmp;
    if (!mul_ok(B, (int64_t)s->norb * 6 * 8, &tmp)) return fail(SPL_ENOMEM, "output size overflow");
    return SPL_OK;
}

// Autotuner over the VGH-family shapes for output kind `out` (bitwise check
// across shapes: the accumulation order does not depend on the tile).
int vgh_autotune(spline_s* s, int out, const double* pos, int64_t B, void* V, void* G, void* H, int32_t reps,
                 hipStream_t st, spline_tile* chosen)
{
    const std::vector<spline_tile> cands = vgh_candidates(s);
    if (cands.empty()) return fail(SPL_EUNSUPPORTED, "no VGH tile shape fits this row width");
    if (reps < 1) reps = 1;
    const int64_t Bc = std::min<int64_t>(B, 512);
    const size_t ob = s->store == SPL_F64 ? 8 : 4;
    const size_t nv = (size_t)Bc * s->norb * ob;
    const size_t nh = out == VGH_OUT_H ? 6 : 1;
    std::vector<unsigned char> ref, cur(nv * (4 + nh));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(SPL_EHIP, "hipEventCreate failed");
    }
    int rc = SPL_OK;
    float best = 1e30f;
    spline_tile best_t = cands[0];
    for (size_t i = 0; i < cands.size() && rc == SPL_OK; ++i) {
        const spline_tile& t = cands[i];
        rc = vgh_launch(s, t, out, pos, B, V, G, H, st);
        if (rc) break;
        if (hipMemcpyAsync(cur.data(), V, nv, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(cur.data() + nv, G, 3 * nv, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(cur.data() + 4 * nv, H, nh * nv, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            rc = fail(SPL_EHIP, "autotune: copy of outputs failed");
            break;
        }
        if (i == 0) {
            ref = cur;
        } else if (std::memcmp(ref.data(), cur.data(), ref.size()) != 0) {
            std::ostringstream m;
            m << "autotune: VGH tile (" << t.cw << "," << t.nch << "," << t.lpp << "," << t.pb
              << ") differs bitwise from the first candidate";
            rc = fail(SPL_EUNSUPPORTED, m.str());
            break;
        }
        if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(SPL_EHIP, "event record"); break; }
        for (int r = 0; r < reps && rc == SPL_OK; ++r) rc = vgh_launch(s, t, out, pos, B, V, G, H, st);
        if (rc) break;
        float ms = 0.f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(SPL_EHIP, "autotune: event timing failed");
            break;
        }
        if (ms < best) {
            best = ms;
            best_t = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    s->htile = best_t;
    if (chosen) *chosen = best_t;
    return SPL_OK;
}

}  // namespace qs

using namespace qs;

extern "C" {

int spline_set_lattice(spline_t* s, const double* lattice)
{
    if (!s || !lattice) return fail(SPL_EINVAL, "NULL argument");
    double il[9];
    if (!inv3(lattice, il)) return fail(SPL_EINVAL, "lattice is singular or not finite");
    std::memcpy(s->lat, lattice, sizeof(s->lat));
    std::memcpy(s->ilat, il, sizeof(s->ilat));
    s->general = 1;
    return SPL_OK;
}

int spline_get_lattice(const spline_t* s, double* lattice)
{
    if (!s || !lattice) return fail(SPL_EINVAL, "NULL argument");
    if (s->general) {
        std::memcpy(lattice, s->lat, sizeof(s->lat));
    } else {
        for (int i = 0; i < 9; ++i) lattice[i] = 0.0;
        for (int d = 0; d < 3; ++d) lattice[4 * d] = s->grid.cell[d];
    }
    return SPL_OK;
}

int spline_eval_vgh(const spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* H, void* stream)
{
    int rc = check_outputs(s, pos_dev, B, V, G, H);
    if (rc || B == 0) return rc;
    return vgh_launch(s, s->htile, VGH_OUT_H, pos_dev, B, V, G, H, static_cast<hipStream_t>(stream));
}

int spline_vgh_tile_candidates(const spline_t* s, spline_tile* out, int32_t cap, int32_t* n)
{
    if (!s || !n) return fail(SPL_EINVAL, "NULL argument");
    if (cap > 0 && !out) return fail(SPL_EINVAL, "NULL output with positive capacity");
    const std::vector<spline_tile> c = vgh_candidates(s);
    for (size_t i = 0; i < c.size() && (int32_t)i < cap; ++i) out[i] = c[i];
    *n = (int32_t)c.size();
    return SPL_OK;
}

int spline_set_vgh_tile(spline_t* s, const spline_tile* tile)
{
    if (!s || !tile) return fail(SPL_EINVAL, "NULL argument");
    const VghVariant* v = find_vgh(s->store, *tile, VGH_OUT_H);
    if (!v) return fail(SPL_EUNSUPPORTED, "tile shape not compiled for the VGH kernels");
    if (!vgh_fits(s, *v)) return fail(SPL_EUNSUPPORTED, "tile does not divide the row");
    if (tile->pb < 1 || tile->pb > 256 || v->lds_per_pos * (size_t)tile->pb > kMaxLds)
        return fail(SPL_EUNSUPPORTED, "bad positions per workgroup");
    s->htile = *tile;
    return SPL_OK;
}

int spline_get_vgh_tile(const spline_t* s, spline_tile* tile)
{
    if (!s || !tile) return fail(SPL_EINVAL, "NULL argument");
    *tile = s->htile;
    return SPL_OK;
}

int spline_autotune_vgh(spline_t* s, const double* pos_dev, int64_t B, void* V, void* G, void* H, int32_t reps,
                        void* stream, spline_tile* chosen)
{
    int rc = check_outputs(s, pos_dev, B, V, G, H);
    if (rc) return rc;
    if (B == 0) return fail(SPL_EINVAL, "autotune needs a non-empty batch");
    return vgh_autotune(s, VGH_OUT_H, pos_dev, B, V, G, H, reps, static_cast<hipStream_t>(stream), chosen);
}

}  // extern "C"
