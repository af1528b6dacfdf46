// Internal declarations shared by the host runtime and the kernel files of
// the qmcspline library.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/qmcspline.h"

namespace qs {

// Thread-local last-error text and helpers that set it.
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define QS_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return qs::hip_fail(e_, #call); \
    } while (0)

// Kernel arguments of the single-table evaluation kernels.  The same
// struct serves VGL and value-only launches.
struct EvalArgs {
    const unsigned char* table;  // row (0,0,0) of the halo layout
    const float* scales;         // per-orbital scale (16-bit stores), else unused
    const double* pos;           // [B][3]
    void* V;                     // [B][norb]
    void* G;                     // [B][3][norb]
    void* L;                     // [B][norb]
    int64_t B;
    int64_t row_bytes;  // bytes per grid point row
    int64_t ystride;    // bytes between consecutive y rows (padded z extent * row_bytes)
    int64_t xstride;    // bytes between consecutive x planes
    double cell[3];
    int32_t n[3];
    int32_t norb;
    int32_t tiles;      // orbital tiles per position
    int32_t pb;         // positions per workgroup
    // Optional indirection (spline fallback of the surrogate): when idx is
    // set, logical position i is row idx[i] of pos and of the outputs, and
    // when nidx is set the number of logical positions is min(*nidx, B),
    // read on the device.
    const int32_t* idx;
    const int32_t* nidx;
    // Determinant-ratio launches: row of A^-1 for logical row r starts at
    // ainv + (arows ? arows[r] : r) * ald elements; the sums go to V.
    const void* ainv;
    int64_t ald;
    const int32_t* arows;
    // General (triclinic) cell: when `general` is set, a position r is reduced
    // through its fractional coordinates u_d = sum_c r_c ilat[c*3+d] (ilat =
    // inverse of the lattice matrix whose rows are the lattice vectors) and the
    // derivative weights are in grid units (d/dt_d).
    double ilat[9];
    int32_t general;
};

// One task of a multi-table plan: positions [first, first + count) of table
// `table` (count <= the plan's positions per workgroup).
struct PlanTask {
    int32_t table;
    int32_t count;
    int64_t first;
};

// Kernel arguments of the persistent multi-table kernel.
struct PlanArgs {
    const EvalArgs* tabs;   // device, one per table
    const PlanTask* tasks;  // device, ntasks entries, processed in order of popping
    unsigned int* counter;  // device work counters (one per segment), zero at launch
    int32_t ntasks;
    int32_t nseg;           // 1, or 8: the task list in eight contiguous segments, one per XCD
};
constexpr int kPlanSegs = 8;

// Task list of a plan for positions-per-task pb (plan_host.cpp): tables with
// the widest rows first (largest tasks first, the narrow ones fill the
// tail), each table's positions in blocks of at most pb; empty for pb < 1.
std::vector<PlanTask> plan_tasks(const int64_t* B, const int64_t* row_bytes, int32_t n, int pb);

// One compiled kernel variant.
struct Variant {
    spline_dtype store;
    int cw, nch, lpp;
    bool vgl;              // true: V, G, L; false: value only
    bool ratio;            // determinant-ratio epilogue instead of stores
    const void* fn;        // __global__ function symbol (single table)
    const void* plan_fn;   // persistent multi-table kernel (VGL variants only), else null
    size_t lds_per_pos;    // staged weights per position
    size_t lds_per_tile;   // ratio partial sums per (position, tile), else 0
};

// Registry of every compiled variant (filled by the kernel files).
const Variant* variants(int* count);

// LDS bytes of a launch of v with pb positions per workgroup and `tiles`
// orbital tiles per position.
inline size_t launch_lds(const Variant& v, int pb, int64_t tiles)
{
    return (size_t)pb * (v.lds_per_pos + (size_t)tiles * v.lds_per_tile);
}
constexpr size_t kMaxLds = 64 * 1024;

// Launch one variant; validates nothing (the caller did).
int launch(const Variant& v, const EvalArgs& a, hipStream_t stream);

constexpr int kBlock = 256;  // threads per workgroup of the evaluation kernels

}  // namespace qs

struct spline_s;

namespace qs {

bool mul_ok(int64_t a, int64_t b, int64_t* out);
// Whole tiles of variant v cover the padded rows of table s exactly.
bool tile_fits(const spline_s* s, const Variant& v);
const Variant* find_variant(spline_dtype st, int cw, int nch, int lpp, bool vgl, bool ratio = false);
int64_t tiles_of(const spline_s* s, const spline_tile& t);
EvalArgs make_args(const spline_s* s, const spline_tile& t, const double* pos, int64_t B, void* V, void* G,
                   void* L);
// General cells and the VGH family (vgh_host.cpp).
spline_tile default_vgh_tile(const spline_s* s);
void set_general_args(const spline_s* s, EvalArgs& a);
int vgl_general(const spline_s* s, const double* pos, int64_t B, void* V, void* G, void* L, hipStream_t st);
int vgh_launch_indexed(const spline_s* s, const spline_tile& t, bool hessian, const double* pos, int64_t B, void* V,
                       void* G, void* H, const int32_t* idx, hipStream_t st);
// Fused determinant ratio with derivatives in a general cell (the VGH-family
// kernel with the ratio epilogue): ratio_general_tile halves t.pb until the
// partial sums fit in LDS; ratio_general launches it (idx: optional
// position order, as in the locality-ordered evaluation).
int ratio_general_tile(const spline_s* s, spline_tile& t);
int ratio_general(const spline_s* s, const spline_tile& t, const double* pos, int64_t B, const void* ainv, int64_t ld,
                  const int32_t* rows, void* D, const int32_t* idx, hipStream_t st);
// Tile of the locality-ordered VGH family: 16-lane groups with the widest
// chunk compiled for the storage type where it fits the row (else the VGH
// tile's shape), at most 8 positions per workgroup.
spline_tile vgh_sorted_tile(const spline_s* s);
// Locality ordering (locality.hip): workspace bytes for B positions, and the
// device sort of B positions into an index list for workgroups of pb
// positions (pb <= 0: plain sorted order).
size_t loc_bytes(int64_t B);
const int32_t* loc_perm(const void* ws, int64_t B);  // where sort_positions leaves the index list
int sort_positions(const spline_s* s, const double* pos, int64_t B, int pb, void* ws, hipStream_t st,
                   const int32_t** perm_out);
int vgh_autotune(spline_s* s, int out, const double* pos, int64_t B, void* V, void* G, void* H, int32_t reps,
                 hipStream_t st, spline_tile* chosen);
// Tile validation and the tuning cache (spline_host.cpp).
int check_tile(const spline_s* s, const spline_tile* t, bool vgl);
// Times every candidate shape (run(t) launches one evaluation with shape t
// writing V, and G, L for VGL) and returns the fastest in *best; every
// candidate must reproduce the first one's outputs on the first positions
// bit for bit.  Candidates without a value-only kernel are skipped for !vgl.
int tune_kind(const spline_s* s, bool vgl, const std::vector<spline_tile>& cands, int64_t B, void* V, void* G,
              void* L, int32_t reps, hipStream_t st, const std::function<int(const spline_tile&)>& run,
              spline_tile* best);
std::string tune_key(const spline_s* s, int64_t B);
bool cache_lookup(const char* path, const std::string& key, spline_tile* t);
// The tuning cache to use: the given path, else $QMCSPLINE_TUNE_CACHE when
// set and not empty, else none.
const char* tune_cache_path(const char* given);

}  // namespace qs

// Handle (opaque in the C ABI).
struct spline_s {
    spline_grid grid;
    int32_t norb;
    spline_dtype store;
    spline_layout layout;
    unsigned char* dev;    // caller's device buffer
    int device;            // HIP device id the table lives on
    spline_tile tile;      // current VGL tile shape
    spline_tile vtile;     // current value-only tile shape
    spline_tile htile;     // current shape of the VGH family (also general-cell VGL)
    spline_tile stile;     // current VGL tile shape of the locality-ordered path
    spline_tile svtile;    // its value-only (and value-ratio) tile shape
    int general;           // 1 once a general lattice is set
    double lat[9];         // lattice vectors as rows (general cells)
    double ilat[9];        // its inverse
};
