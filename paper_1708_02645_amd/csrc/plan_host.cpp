// Ragged multi-table plans: several tables with their own batch sizes
// evaluated by one persistent work-queue launch, captured once in a HIP
// graph and replayed with a single graph launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <limits>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "common.hpp"
#include "vgh_kernel.hpp"

namespace qs {

// Zeroes the work counters of a plan (a kernel, not a memset node, so that
// the captured graph holds only kernel nodes).
__global__ void plan_reset_kernel(unsigned int* counter)
{
    if (threadIdx.x < kPlanSegs && blockIdx.x == 0) counter[threadIdx.x] = 0u;
}

// Smallest positions-per-task a plan may use; it sizes the task list in the
// workspace.  Locality-ordered plans also try 8-position tasks.
constexpr int kMinPb = 16, kMinPbSorted = 8;
static int min_pb(bool sorted) { return sorted ? kMinPbSorted : kMinPb; }

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

struct WsLayout {
    size_t counter, tabs, tasks, total;
    std::vector<size_t> loc;  // locality-ordered plans: each table's sort workspace
};

static bool ws_layout(int32_t n_tabs, const int64_t* B, bool sorted, WsLayout* w, int64_t* max_tasks)
{
    int64_t nt = 0;
    for (int32_t t = 0; t < n_tabs; ++t) {
        if (B[t] < 0) return false;
        if (sorted && B[t] > (int64_t)std::numeric_limits<int32_t>::max()) return false;
        nt += (B[t] + min_pb(sorted) - 1) / min_pb(sorted);
        if (nt > (int64_t)1 << 30) return false;
    }
    w->counter = 0;  // kPlanSegs counters in the first 256 bytes
    w->tabs = 256;
    // per-table kernel arguments: EvalArgs, or VghArgs for a plan with a general cell
    w->tasks = w->tabs + align256((size_t)n_tabs * std::max(sizeof(EvalArgs), sizeof(VghArgs)));
    w->total = w->tasks + align256((size_t)std::max<int64_t>(nt, 1) * sizeof(PlanTask));
    w->loc.clear();
    if (sorted)
        for (int32_t t = 0; t < n_tabs; ++t) {
            w->loc.push_back(w->total);
            w->total += loc_bytes(B[t]);
        }
    *max_tasks = nt;
    return true;
}

}  // namespace qs

struct spline_plan_s {
    std::vector<const spline_s*> tabs;
    std::vector<int64_t> B;
    std::vector<const double*> pos;
    std::vector<void*> V, G, L;
    unsigned char* ws = nullptr;
    qs::WsLayout lay{};
    spline_tile tile{};
    bool vgh = false;                 // a table has a general cell: every task runs the VGH-family kernel
    const void* fn = nullptr;         // the plan kernel of the chosen shape
    size_t lds_per_pos = 0;
    int32_t ntasks = 0;
    int64_t max_tasks = 0;            // capacity of the task list in the workspace
    int32_t nblocks = 0;
    bool sorted = false;              // positions sorted on the device before each launch
    std::vector<const int32_t*> perm; // locality-ordered plans: each table's index list
    int device = -1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace qs {

std::vector<PlanTask> plan_tasks(const int64_t* B, const int64_t* row_bytes, int32_t n, int pb)
{
    std::vector<int32_t> order((size_t)std::max(n, 0));
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return row_bytes[a] > row_bytes[b]; });
    std::vector<PlanTask> tasks;
    if (pb < 1) return tasks;
    for (int32_t t : order)
        for (int64_t f = 0; f < B[t]; f += pb)
            tasks.push_back(PlanTask{t, (int32_t)std::min<int64_t>(pb, B[t] - f), f});
    return tasks;
}

static std::vector<PlanTask> make_tasks(const spline_plan_s* p, int pb)
{
    std::vector<int64_t> rb;
    for (const spline_s* s : p->tabs) rb.push_back(s->layout.row_bytes);
    return plan_tasks(p->B.data(), rb.data(), (int32_t)p->tabs.size(), pb);
}

// A candidate plan kernel: its function, staged weights per position, shape.
struct PlanCand {
    const void* fn;
    size_t lds_per_pos;
    spline_tile t;
};

// Uploads the descriptors and tasks for a candidate and sizes the grid.
static int stage_config(spline_plan_s* p, const PlanCand& c, hipStream_t st)
{
    const spline_tile& t = c.t;
    if (t.pb < min_pb(p->sorted)) return fail(SPL_EINVAL, "positions per task below the plan's minimum");
    std::vector<PlanTask> tasks = make_tasks(p, t.pb);
    if ((int64_t)tasks.size() > p->max_tasks) return fail(SPL_EINVAL, "task list larger than its workspace region");
    if (p->vgh) {
        std::vector<VghArgs> args(p->tabs.size());
        for (size_t i = 0; i < p->tabs.size(); ++i) {
            args[i] = vgh_args(p->tabs[i], t, p->pos[i], p->B[i], p->V[i], p->G[i], p->L[i]);
            if (p->sorted) args[i].e.idx = p->perm[i];
        }
        QS_HIP(hipMemcpyAsync(p->ws + p->lay.tabs, args.data(), args.size() * sizeof(VghArgs),
                              hipMemcpyHostToDevice, st));
        QS_HIP(hipStreamSynchronize(st));  // the host vector dies at the end of this block
    } else {
        std::vector<EvalArgs> args(p->tabs.size());
        for (size_t i = 0; i < p->tabs.size(); ++i) {
            args[i] = make_args(p->tabs[i], t, p->pos[i], p->B[i], p->V[i], p->G[i], p->L[i]);
            if (p->sorted) args[i].idx = p->perm[i];
        }
        QS_HIP(hipMemcpyAsync(p->ws + p->lay.tabs, args.data(), args.size() * sizeof(EvalArgs),
                              hipMemcpyHostToDevice, st));
        QS_HIP(hipStreamSynchronize(st));
    }
    if (!tasks.empty())
        QS_HIP(hipMemcpyAsync(p->ws + p->lay.tasks, tasks.data(), tasks.size() * sizeof(PlanTask),
                              hipMemcpyHostToDevice, st));
    QS_HIP(hipStreamSynchronize(st));  // the host vectors die at return
    const size_t lds = c.lds_per_pos * (size_t)t.pb;
    int per_cu = 0;
    QS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, c.fn, kBlock, lds));
    hipDeviceProp_t prop;
    QS_HIP(hipGetDeviceProperties(&prop, p->device));
    const int64_t full = (int64_t)std::max(per_cu, 1) * prop.multiProcessorCount;
    p->ntasks = (int32_t)tasks.size();
    p->nblocks = (int32_t)std::max<int64_t>(1, std::min<int64_t>(full, p->ntasks));
    p->fn = c.fn;
    p->lds_per_pos = c.lds_per_pos;
    p->tile = t;
    return SPL_OK;
}

static int launch_plan(const spline_plan_s* p, hipStream_t st)
{
    if (p->ntasks == 0) return SPL_OK;
    if (p->sorted)  // each table's positions in locality order; the queue's segments deal them to the XCDs
        for (size_t i = 0; i < p->tabs.size(); ++i) {
            if (p->B[i] == 0) continue;
            const int32_t* perm = nullptr;
            const int rc = sort_positions(p->tabs[i], p->pos[i], p->B[i], 0, p->ws + p->lay.loc[i], st, &perm);
            if (rc) return rc;
        }
    unsigned int* counter = reinterpret_cast<unsigned int*>(p->ws + p->lay.counter);
    hipLaunchKernelGGL(plan_reset_kernel, dim3(1), dim3(64), 0, st, counter);
    QS_HIP(hipGetLastError());
    PlanArgs pa{reinterpret_cast<const EvalArgs*>(p->ws + p->lay.tabs),
                reinterpret_cast<const PlanTask*>(p->ws + p->lay.tasks), counter, p->ntasks,
                p->sorted ? kPlanSegs : 1};
    PlanVghArgs pv{reinterpret_cast<const VghArgs*>(p->ws + p->lay.tabs),
                   reinterpret_cast<const PlanTask*>(p->ws + p->lay.tasks), counter, p->ntasks,
                   p->sorted ? kPlanSegs : 1};
    void* params[] = {p->vgh ? static_cast<void*>(&pv) : static_cast<void*>(&pa)};
    const size_t lds = p->lds_per_pos * (size_t)p->tile.pb;
    QS_HIP(hipLaunchKernel(p->fn, dim3(p->nblocks), dim3(kBlock), params, lds, st));
    QS_HIP(hipGetLastError());
    return SPL_OK;
}

// Copies the first rows of every table's outputs to the host (autotuner check).
static int sample_outputs(const spline_plan_s* p, std::vector<unsigned char>& out, hipStream_t st)
{
    out.clear();
    for (size_t i = 0; i < p->tabs.size(); ++i) {
        const int64_t rows = std::min<int64_t>(p->B[i], 64);
        if (rows == 0) continue;
        const size_t es = p->tabs[i]->store == SPL_F64 ? 8 : 4;
        const size_t n = (size_t)rows * p->tabs[i]->norb * es;
        const size_t at = out.size();
        out.resize(at + 5 * n);
        QS_HIP(hipMemcpyAsync(out.data() + at, p->V[i], n, hipMemcpyDeviceToHost, st));
        QS_HIP(hipMemcpyAsync(out.data() + at + n, p->G[i], 3 * n, hipMemcpyDeviceToHost, st));
        QS_HIP(hipMemcpyAsync(out.data() + at + 4 * n, p->L[i], n, hipMemcpyDeviceToHost, st));
    }
    QS_HIP(hipStreamSynchronize(st));
    return SPL_OK;
}

static void free_graph(spline_plan_s* p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

}  // namespace qs

using namespace qs;

extern "C" {

}  // extern "C"

static size_t plan_ws_bytes(int32_t n_tabs, const int64_t* B_per_tab, bool sorted)
{
    if (n_tabs <= 0 || !B_per_tab) return 0;
    WsLayout w;
    int64_t nt = 0;
    if (!ws_layout(n_tabs, B_per_tab, sorted, &w, &nt)) return 0;
    return w.total;
}

static int plan_create(const spline_t* const* tabs, int32_t n_tabs, const int64_t* B_per_tab,
                       const double* const* pos_dev, void* const* V, void* const* G, void* const* L,
                       void* workspace_dev, size_t workspace_bytes, int32_t tune_reps, void* stream,
                       spline_plan_t** out, bool sorted)
{
    if (!out) return fail(SPL_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_tabs <= 0 || n_tabs > 4096) return fail(SPL_EINVAL, "n_tabs must be in [1, 4096]");
    if (!tabs || !B_per_tab || !pos_dev || !V || !G || !L) return fail(SPL_EINVAL, "NULL array argument");
    if (!workspace_dev) return fail(SPL_EINVAL, "workspace is NULL");
    if ((reinterpret_cast<uintptr_t>(workspace_dev) & 255) != 0)
        return fail(SPL_EINVAL, "workspace not 256-byte aligned");
    WsLayout lay;
    int64_t max_tasks = 0;
    if (!ws_layout(n_tabs, B_per_tab, sorted, &lay, &max_tasks)) return fail(SPL_EINVAL, "negative or huge batch size");
    if (workspace_bytes < lay.total) return fail(SPL_ENOMEM, "workspace smaller than spline_plan_workspace_bytes()");
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    for (int32_t t = 0; t < n_tabs; ++t) {
        if (!tabs[t]) return fail(SPL_EINVAL, "NULL table handle");
        if (tabs[t]->store != tabs[0]->store) return fail(SPL_EUNSUPPORTED, "tables of one plan must share the storage type");
        if (tabs[t]->device != dev) return fail(SPL_EINVAL, "table lives on another device");
        if (B_per_tab[t] > 0 && (!pos_dev[t] || !V[t] || !G[t] || !L[t]))
            return fail(SPL_EINVAL, "NULL position or output pointer");
        int64_t tmp;
        if (!mul_ok(B_per_tab[t], (int64_t)tabs[t]->norb * 3 * 8, &tmp)) return fail(SPL_ENOMEM, "output size overflow");
    }
    spline_plan_s* p = new (std::nothrow) spline_plan_s;
    if (!p) return fail(SPL_ENOMEM, "plan allocation failed");
    p->tabs.assign(tabs, tabs + n_tabs);
    p->B.assign(B_per_tab, B_per_tab + n_tabs);
    p->pos.assign(pos_dev, pos_dev + n_tabs);
    p->V.assign(V, V + n_tabs);
    p->G.assign(G, G + n_tabs);
    p->L.assign(L, L + n_tabs);
    p->ws = static_cast<unsigned char*>(workspace_dev);
    p->lay = lay;
    p->max_tasks = max_tasks;
    p->device = dev;
    p->sorted = sorted;
    if (sorted)  // the index lists sit at fixed places in each table's sort workspace
        for (int32_t t = 0; t < n_tabs; ++t)
            p->perm.push_back(loc_perm(p->ws + lay.loc[t], B_per_tab[t]));
    hipStream_t st = static_cast<hipStream_t>(stream);

    // A table with a general cell puts the whole plan on the VGH-family
    // kernel (the others take its general staging with their diagonal
    // lattice: the same results within rounding).
    for (int32_t t = 0; t < n_tabs; ++t) p->vgh = p->vgh || tabs[t]->general;

    // Candidate shapes: tiles that divide every table's row, times pb.
    std::vector<PlanCand> cands;
    auto add = [&](const void* fn, size_t lds_per_pos, int cw, int nch, int lpp) {
        for (int pb : {8, 16, 32, 64}) {
            if (pb == 8 && !sorted) continue;  // short tasks pay only when neighbours share rows
            if (lds_per_pos * (size_t)pb > 64 * 1024) continue;
            cands.push_back(PlanCand{fn, lds_per_pos, spline_tile{cw, nch, lpp, pb}});
        }
    };
    if (p->vgh) {
        for (const VghVariant* v : vgh_plan_variants(tabs[0]->store)) {
            bool ok = true;
            for (int32_t t = 0; t < n_tabs && ok; ++t) ok = vgh_variant_fits(tabs[t], *v);
            if (ok) add(v->plan_fn, v->lds_per_pos, v->cw, v->nch, v->lpp);
        }
    } else {
        int nv = 0;
        const Variant* vs = variants(&nv);
        for (int i = 0; i < nv; ++i) {
            const Variant& v = vs[i];
            if (!v.vgl || !v.plan_fn || v.store != tabs[0]->store) continue;
            bool ok = true;
            for (int32_t t = 0; t < n_tabs && ok; ++t) ok = tile_fits(tabs[t], v);
            if (ok) add(v.plan_fn, v.lds_per_pos, v.cw, v.nch, v.lpp);
        }
    }
    if (cands.empty()) {
        delete p;
        return fail(SPL_EUNSUPPORTED, "no compiled tile shape divides every table's row");
    }
    // Without tuning: the first table's own default shape (its VGH-family
    // shape for a plan with a general cell) if it fits all, else the
    // widest-chunk candidate with positions-per-task 32.
    size_t pick = 0;
    for (size_t i = 0; i < cands.size(); ++i) {
        const spline_tile& d = p->vgh ? tabs[0]->htile : tabs[0]->tile;
        const spline_tile& c = cands[i].t;
        if (c.cw == d.cw && c.nch == d.nch && c.lpp == d.lpp && c.pb == 32) {
            pick = i;
            break;
        }
        if (c.pb == 32 && c.cw * c.nch > cands[pick].t.cw * cands[pick].t.nch) pick = i;
    }
    int rc = SPL_OK;
    if (tune_reps > 0 && max_tasks > 0) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            delete p;
            return fail(SPL_EHIP, "hipEventCreate failed");
        }
        std::vector<unsigned char> ref, cur;
        float best = 1e30f;
        for (size_t i = 0; i < cands.size() && rc == SPL_OK; ++i) {
            rc = stage_config(p, cands[i], st);
            if (!rc) rc = launch_plan(p, st);
            if (!rc) rc = sample_outputs(p, i == 0 ? ref : cur, st);
            if (rc) break;
            if (i > 0 && cur != ref) {
                std::ostringstream m;
                m << "plan autotune: tile (" << cands[i].t.cw << "," << cands[i].t.nch << "," << cands[i].t.lpp
                  << "," << cands[i].t.pb << ") differs bitwise from the first";
                rc = fail(SPL_EUNSUPPORTED, m.str());
                break;
            }
            if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(SPL_EHIP, "event record"); break; }
            for (int r = 0; r < tune_reps && !rc; ++r) rc = launch_plan(p, st);
            float ms = 0.f;
            if (!rc && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = fail(SPL_EHIP, "plan autotune: event timing failed");
            if (!rc && ms < best) {
                best = ms;
                pick = i;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    if (!rc) rc = stage_config(p, cands[pick], st);
    if (rc) {
        delete p;
        return rc;
    }

    // Capture reset + persistent kernel once, on a private stream (the
    // caller's stream may be the null stream, which cannot be captured).
    if (p->ntasks > 0) {
        hipStream_t cs = nullptr;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
            delete p;
            return fail(SPL_EHIP, "hipStreamCreateWithFlags failed");
        }
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            rc = launch_plan(p, cs);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(cs, &g);
            p->graph = g;
            if (!rc && e2 != hipSuccess) rc = hip_fail(e2, "hipStreamEndCapture");
            if (!rc) {
                hipError_t e3 = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
                if (e3 != hipSuccess) rc = hip_fail(e3, "hipGraphInstantiate");
            }
        } else {
            rc = hip_fail(e, "hipStreamBeginCapture");
        }
        (void)hipStreamDestroy(cs);
        if (rc) {
            free_graph(p);
            delete p;
            return rc;
        }
    }
    *out = p;
    return SPL_OK;
}

extern "C" {

size_t spline_plan_workspace_bytes(int32_t n_tabs, const int64_t* B_per_tab)
{
    return plan_ws_bytes(n_tabs, B_per_tab, false);
}

size_t spline_plan_workspace_bytes_sorted(int32_t n_tabs, const int64_t* B_per_tab)
{
    return plan_ws_bytes(n_tabs, B_per_tab, true);
}

int spline_plan_create(const spline_t* const* tabs, int32_t n_tabs, const int64_t* B_per_tab,
                       const double* const* pos_dev, void* const* V, void* const* G, void* const* L,
                       void* workspace_dev, size_t workspace_bytes, int32_t tune_reps, void* stream,
                       spline_plan_t** out)
{
    return plan_create(tabs, n_tabs, B_per_tab, pos_dev, V, G, L, workspace_dev, workspace_bytes, tune_reps, stream,
                       out, false);
}

int spline_plan_create_sorted(const spline_t* const* tabs, int32_t n_tabs, const int64_t* B_per_tab,
                              const double* const* pos_dev, void* const* V, void* const* G, void* const* L,
                              void* workspace_dev, size_t workspace_bytes, int32_t tune_reps, void* stream,
                              spline_plan_t** out)
{
    return plan_create(tabs, n_tabs, B_per_tab, pos_dev, V, G, L, workspace_dev, workspace_bytes, tune_reps, stream,
                       out, true);
}

int spline_plan_launch(const spline_plan_t* p, void* stream)
{
    if (!p) return fail(SPL_EINVAL, "plan is NULL");
    if (p->ntasks == 0) return SPL_OK;
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    if (dev != p->device) return fail(SPL_EINVAL, "current HIP device differs from the plan's device");
    QS_HIP(hipGraphLaunch(p->exec, static_cast<hipStream_t>(stream)));
    return SPL_OK;
}

int spline_plan_launch_eager(const spline_plan_t* p, void* stream)
{
    if (!p) return fail(SPL_EINVAL, "plan is NULL");
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    if (dev != p->device) return fail(SPL_EINVAL, "current HIP device differs from the plan's device");
    return launch_plan(p, static_cast<hipStream_t>(stream));
}

int spline_plan_get_info(const spline_plan_t* p, spline_tile* tile, int32_t* n_tasks, int32_t* n_blocks)
{
    if (!p) return fail(SPL_EINVAL, "plan is NULL");
    if (tile) *tile = p->tile;
    if (n_tasks) *n_tasks = p->ntasks;
    if (n_blocks) *n_blocks = p->nblocks;
    return SPL_OK;
}

int spline_plan_destroy(spline_plan_t* p)
{
    if (!p) return SPL_OK;
    free_graph(p);
    delete p;
    return SPL_OK;
}

}  // extern "C"
