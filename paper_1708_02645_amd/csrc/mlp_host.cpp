// Host runtime of the surrogate network: parameter buffer layout, training
// step orchestration (forward, Sobolev loss, reverse pass, Adam), error map
// and spline fallback routing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "mlp_kernels.hpp"

namespace qs {

// Declared in mlp_kernels.hip.
__global__ void mlp_features_kernel(const double*, int64_t, const int32_t*, double, double, double, float*);
__global__ void gemm_bf16_kernel(GemmArgs p);
__global__ void mlp_act_fwd_kernel(const float*, float*, int64_t, int);
__global__ void mlp_act_bwd_kernel(const float*, const float*, float*, int64_t, int);
__global__ void mlp_loss_kernel(const float*, const float*, const float*, const float*, const float*, const float*,
                                const float*, int64_t, int, float*, float*);
__global__ void mlp_bias_grad_kernel(const float*, int64_t, int, float*);
__global__ void splitk_reduce_kernel(const float*, int, int64_t, int64_t, float*);
__global__ void adam_kernel(float*, const float*, float*, float*, int64_t, float, float, float, float, float, float,
                            __bf16*, int32_t);
__global__ void bf16_copy_kernel(const float*, __bf16*, int64_t, int32_t);
__global__ void mlp_stats_kernel(const float*, const float*, const float*, int64_t, int, double*);
__global__ void colmax_kernel(const float*, const float*, const float*, int64_t, int, unsigned int*);
__global__ void bin_error_kernel(const double*, double, double, double, int, const float*, const float*, const float*,
                                 const float*, const float*, const float*, const unsigned int*, int64_t, int,
                                 unsigned int*);
__global__ void fill_u32_kernel(unsigned int*, unsigned int, int64_t);
__global__ void route_kernel(const double*, double, double, double, int, const float*, float, int64_t, int32_t*,
                             int32_t*);
__global__ void bin_finalize_kernel(const unsigned int*, const unsigned int*, float*, int);
__global__ void bin_count_kernel(const double*, double, double, double, int, int64_t, unsigned int*);

constexpr int kMaxBins = 16;  // bins per axis of the error map
constexpr int kThreads = 256;

static size_t a256(size_t x) { return (x + 255) / 256 * 256; }

static unsigned grid1(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

struct MlpLay {
    size_t P, M1, M2, Wh, mu, sd, lw, freqs, bin_err, meta, stats, total;
};

static MlpLay mlp_lay(int nout)
{
    const MlpOffsets o = mlp_offsets(nout);
    MlpLay L;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t r = at;
        at += a256(bytes);
        return r;
    };
    L.P = take(o.total * 4);
    L.M1 = take(o.total * 4);
    L.M2 = take(o.total * 4);
    L.Wh = take(o.htotal * 2);
    L.mu = take((size_t)nout * 4);
    L.sd = take((size_t)nout * 4);
    L.lw = take(4 * 4);
    L.freqs = take((size_t)kFreq * 3 * 4);
    L.bin_err = take((size_t)kMaxBins * kMaxBins * kMaxBins * 4);
    L.meta = take(4 * 8);
    L.stats = take((size_t)nout * 6 * 8);  // scratch of spline_mlp_init_output
    L.total = at;
    return L;
}

static int check_desc(const spline_mlp_desc* d)
{
    if (!d) return fail(SPL_EINVAL, "desc is NULL");
    if (d->n_freq != kFreq || d->width[0] != kIn || d->width[1] != kHidden || d->width[2] != kHidden)
        return fail(SPL_EUNSUPPORTED, "compiled network shape is 48 frequencies, widths 96-256-256-N");
    if (d->width[3] < 16 || d->width[3] > kMaxOut || d->width[3] % 16 != 0)
        return fail(SPL_EUNSUPPORTED, "output width must be a multiple of 16 in [16, 256]");
    return SPL_OK;
}

static int gemm(const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk, int64_t sbn, float* C,
                int64_t ldc, const float* bias, int bias_rows, int M, int N, int K, int splits, int64_t split_stride,
                hipStream_t st)
{
    GemmArgs g{A, sam, sak, B, sbk, sbn, C, ldc, bias, bias_rows, M, N, K, 0, split_stride};
    const int chunk = ((K + splits - 1) / splits + 31) / 32 * 32;
    g.kchunk = chunk;
    const int nz = (K + chunk - 1) / chunk;
    hipLaunchKernelGGL(gemm_bf16_kernel, dim3((N + 63) / 64, (M + 63) / 64, nz), dim3(256), 0, st, g);
    QS_HIP(hipGetLastError());
    return nz;  // number of partial products written
}

struct TrainWs {
    size_t X0, H1, Z1, H2, Z2, Y, dY, dZ, dH, grad, part, loss, total;
    int splits;
};

static TrainWs train_ws(int64_t B, int nout)
{
    const MlpOffsets o = mlp_offsets(nout);
    TrainWs w;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t r = at;
        at += a256(bytes);
        return r;
    };
    const size_t R = (size_t)kStreams * (size_t)B;
    w.X0 = take(R * kIn * 4);
    w.H1 = take(R * kHidden * 4);
    w.Z1 = take(R * kHidden * 4);
    w.H2 = take(R * kHidden * 4);
    w.Z2 = take(R * kHidden * 4);
    w.Y = take(R * nout * 4);
    w.dY = take(R * nout * 4);
    w.dZ = take(R * kHidden * 4);
    w.dH = take(R * kHidden * 4);
    w.grad = take((size_t)o.total * 4);
    w.splits = (int)std::min<int64_t>(64, std::max<int64_t>(1, (int64_t)R / 1024));
    w.part = take((size_t)(w.splits + 1) * kHidden * kHidden * 4);
    w.loss = take(16);
    w.total = at;
    return w;
}

}  // namespace qs

struct spline_mlp_s {
    spline_mlp_desc desc;
    int nout;
    qs::MlpOffsets o;
    qs::MlpLay lay;
    unsigned char* dev;
    double cell[3];
    int device;
    int64_t step;
    int nbins;
    int64_t meta_host[4];  // step, nbins: staged for asynchronous copies
    // Host copy of the error map (nbins^3 bin errors) as of the last
    // creation, attach or spline_mlp_build_error_map: lets an evaluation
    // whose tolerance routes every bin (or none) skip the network (or the
    // routing).
    std::vector<float> bin_err_host;
};

namespace qs {

static MlpFwdArgs fwd_args(const spline_mlp_s* m, const double* pos, int64_t B, float* V, float* G, float* L)
{
    MlpFwdArgs a{};
    a.pos = pos;
    a.B = B;
    a.freqs = reinterpret_cast<const int32_t*>(m->dev + m->lay.freqs);
    for (int d = 0; d < 3; ++d) {
        a.cell[d] = m->cell[d];
        a.icell[d] = 1.0 / m->cell[d];
        a.tpc[d] = 6.283185307179586 / m->cell[d];
    }
    a.Wh = reinterpret_cast<const __bf16*>(m->dev + m->lay.Wh);
    a.P = reinterpret_cast<const float*>(m->dev + m->lay.P);
    a.mu = reinterpret_cast<const float*>(m->dev + m->lay.mu);
    a.sd = reinterpret_cast<const float*>(m->dev + m->lay.sd);
    a.V = V;
    a.G = G;
    a.L = L;
    a.nout = m->nout;
    return a;
}

static int launch_forward(const spline_mlp_s* m, const double* pos, int64_t B, float* V, float* G, float* L,
                          hipStream_t st)
{
    if (B == 0) return SPL_OK;
    return launch_mlp_forward(fwd_args(m, pos, B, V, G, L), st);
}

// Refreshes the host copy of the error map from the device (synchronous).
static int read_map(spline_mlp_s* m, hipStream_t st)
{
    m->bin_err_host.assign((size_t)m->nbins * m->nbins * m->nbins, 0.f);
    QS_HIP(hipMemcpyAsync(m->bin_err_host.data(), m->dev + m->lay.bin_err, m->bin_err_host.size() * sizeof(float),
                          hipMemcpyDeviceToHost, st));
    QS_HIP(hipStreamSynchronize(st));
    return SPL_OK;
}

static int write_meta(spline_mlp_s* m, hipStream_t st)
{
    m->meta_host[0] = m->step;
    m->meta_host[1] = m->nbins;
    QS_HIP(hipMemcpyAsync(m->dev + m->lay.meta, m->meta_host, sizeof(m->meta_host), hipMemcpyHostToDevice, st));
    QS_HIP(hipStreamSynchronize(st));
    return SPL_OK;
}

// Loss and gradient (into ws.grad) for one batch.
static int compute_grad(spline_mlp_s* m, const double* pos, const float* tV, const float* tG, const float* tL,
                        int64_t B, unsigned char* ws, const TrainWs& w, hipStream_t st)
{
    const int N = m->nout;
    const MlpOffsets& o = m->o;
    const float* P = reinterpret_cast<const float*>(m->dev + m->lay.P);
    auto F = [&](size_t off) { return reinterpret_cast<float*>(ws + off); };
    float *X0 = F(w.X0), *H1 = F(w.H1), *Z1 = F(w.Z1), *H2 = F(w.H2), *Z2 = F(w.Z2), *Y = F(w.Y), *dY = F(w.dY),
          *dZ = F(w.dZ), *dH = F(w.dH), *grad = F(w.grad), *part = F(w.part), *loss = F(w.loss);
    const int R = (int)(kStreams * B);
    const int32_t* freqs = reinterpret_cast<const int32_t*>(m->dev + m->lay.freqs);
    const float* mu = reinterpret_cast<const float*>(m->dev + m->lay.mu);
    const float* sd = reinterpret_cast<const float*>(m->dev + m->lay.sd);
    const float* lw = reinterpret_cast<const float*>(m->dev + m->lay.lw);

    hipLaunchKernelGGL(mlp_features_kernel, dim3(grid1(B * kIn)), dim3(kThreads), 0, st, pos, B, freqs, m->cell[0],
                       m->cell[1], m->cell[2], X0);
    QS_HIP(hipGetLastError());
    // forward: H = A W^T + b (value rows), Z = silu streams
    int rc = gemm(X0, kIn, 1, P + o.W1, 1, kIn, H1, kHidden, P + o.b1, (int)B, R, kHidden, kIn, 1, 0, st);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(mlp_act_fwd_kernel, dim3(grid1(B * kHidden)), dim3(kThreads), 0, st, H1, Z1, B, kHidden);
    rc = gemm(Z1, kHidden, 1, P + o.W2, 1, kHidden, H2, kHidden, P + o.b2, (int)B, R, kHidden, kHidden, 1, 0, st);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(mlp_act_fwd_kernel, dim3(grid1(B * kHidden)), dim3(kThreads), 0, st, H2, Z2, B, kHidden);
    rc = gemm(Z2, kHidden, 1, P + o.W3, 1, kHidden, Y, N, P + o.b3, (int)B, R, N, kHidden, 1, 0, st);
    if (rc < 0) return rc;
    // loss and its gradient with respect to the normalised outputs
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned int*>(loss), 0u, 4);
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(grid1(B * N)), dim3(kThreads), 0, st, Y, tV, tG, tL, mu, sd, lw, B, N,
                       dY, loss);
    QS_HIP(hipGetLastError());

    // reverse pass, layer by layer: dW = sum over streams and batch of dH^T A_in
    // (split over the batch), db = value-stream column sums, dA_in = dH W.
    auto wgrad = [&](const float* dHl, int Nout, const float* Ain, int Kin, float* out) -> int {
        const int nz = gemm(dHl, 1, Nout, Ain, Kin, 1, part, Kin, nullptr, 0, Nout, Kin, R, w.splits,
                            (int64_t)Nout * Kin, st);
        if (nz < 0) return nz;
        const int64_t cnt = (int64_t)Nout * Kin;
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid1(cnt)), dim3(kThreads), 0, st, part, nz, cnt, cnt, out);
        QS_HIP(hipGetLastError());
        return SPL_OK;
    };
    // bias gradients: column sums of the value-stream rows, in two stages
    auto bgrad = [&](const float* dHl, int Wd, float* out) -> int {
        constexpr int RB = 64;
        hipLaunchKernelGGL(mlp_bias_grad_kernel, dim3((Wd + 63) / 64, RB), dim3(kThreads), 0, st, dHl, B, Wd, part);
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid1(Wd)), dim3(kThreads), 0, st, part, RB, (int64_t)Wd,
                           (int64_t)Wd, out);
        QS_HIP(hipGetLastError());
        return SPL_OK;
    };
    rc = wgrad(dY, N, Z2, kHidden, grad + o.W3);
    if (rc < 0) return rc;
    rc = bgrad(dY, N, grad + o.b3);
    if (rc < 0) return rc;
    rc = gemm(dY, N, 1, P + o.W3, kHidden, 1, dZ, kHidden, nullptr, 0, R, kHidden, N, 1, 0, st);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(mlp_act_bwd_kernel, dim3(grid1(B * kHidden)), dim3(kThreads), 0, st, H2, dZ, dH, B, kHidden);
    rc = wgrad(dH, kHidden, Z1, kHidden, grad + o.W2);
    if (rc < 0) return rc;
    rc = bgrad(dH, kHidden, grad + o.b2);
    if (rc < 0) return rc;
    rc = gemm(dH, kHidden, 1, P + o.W2, kHidden, 1, dZ, kHidden, nullptr, 0, R, kHidden, kHidden, 1, 0, st);
    if (rc < 0) return rc;
    hipLaunchKernelGGL(mlp_act_bwd_kernel, dim3(grid1(B * kHidden)), dim3(kThreads), 0, st, H1, dZ, dH, B, kHidden);
    rc = wgrad(dH, kHidden, X0, kIn, grad + o.W1);
    if (rc < 0) return rc;
    rc = bgrad(dH, kHidden, grad + o.b1);
    if (rc < 0) return rc;
    QS_HIP(hipGetLastError());
    return SPL_OK;
}

static int check_dev(const spline_mlp_s* m)
{
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    if (dev != m->device) return fail(SPL_EINVAL, "current HIP device differs from the network's device");
    return SPL_OK;
}

}  // namespace qs

using namespace qs;

extern "C" {

size_t spline_mlp_param_bytes(const spline_mlp_desc* d)
{
    if (check_desc(d) != SPL_OK) return 0;
    return mlp_lay(d->width[3]).total;
}

int spline_mlp_get_layout(const spline_mlp_desc* d, spline_mlp_layout* out)
{
    int rc = check_desc(d);
    if (rc) return rc;
    if (!out) return fail(SPL_EINVAL, "out is NULL");
    const MlpLay L = mlp_lay(d->width[3]);
    const MlpOffsets o = mlp_offsets(d->width[3]);
    out->n_params = o.total;
    out->W1 = o.W1; out->b1 = o.b1; out->W2 = o.W2; out->b2 = o.b2; out->W3 = o.W3; out->b3 = o.b3;
    out->params = (int64_t)L.P;
    out->adam_m = (int64_t)L.M1;
    out->adam_v = (int64_t)L.M2;
    out->weights_bf16 = (int64_t)L.Wh;
    out->mu = (int64_t)L.mu;
    out->sd = (int64_t)L.sd;
    out->loss_w = (int64_t)L.lw;
    out->freqs = (int64_t)L.freqs;
    out->bin_err = (int64_t)L.bin_err;
    out->meta = (int64_t)L.meta;
    out->total = (int64_t)L.total;
    out->max_bins = kMaxBins;
    return SPL_OK;
}

static int mlp_new(const spline_mlp_desc* d, const double* cell, void* params_dev, size_t bytes, spline_mlp_s** out)
{
    int rc = check_desc(d);
    if (rc) return rc;
    if (!cell || !params_dev) return fail(SPL_EINVAL, "NULL argument");
    for (int k = 0; k < 3; ++k)
        if (!(cell[k] > 0.0) || !std::isfinite(cell[k])) return fail(SPL_EINVAL, "cell lengths must be positive");
    if ((reinterpret_cast<uintptr_t>(params_dev) & 255) != 0) return fail(SPL_EINVAL, "buffer not 256-byte aligned");
    const MlpLay L = mlp_lay(d->width[3]);
    if (bytes < L.total) return fail(SPL_ENOMEM, "buffer smaller than spline_mlp_param_bytes()");
    int dev = -1;
    QS_HIP(hipGetDevice(&dev));
    spline_mlp_s* m = new (std::nothrow) spline_mlp_s;
    if (!m) return fail(SPL_ENOMEM, "handle allocation failed");
    m->desc = *d;
    m->nout = d->width[3];
    m->o = mlp_offsets(m->nout);
    m->lay = L;
    m->dev = static_cast<unsigned char*>(params_dev);
    for (int k = 0; k < 3; ++k) m->cell[k] = cell[k];
    m->device = dev;
    m->step = 0;
    m->nbins = 0;
    *out = m;
    return SPL_OK;
}

int spline_mlp_create(const spline_mlp_desc* desc, const int32_t* freqs_host, const double* cell,
                      const float* params_host, void* params_dev, size_t bytes, void* stream, spline_mlp_t** out)
{
    if (!out) return fail(SPL_EINVAL, "out is NULL");
    *out = nullptr;
    if (!freqs_host || !params_host) return fail(SPL_EINVAL, "NULL frequencies or parameters");
    spline_mlp_s* m = nullptr;
    int rc = mlp_new(desc, cell, params_dev, bytes, &m);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = m->o.total;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(params_host[i])) {
            delete m;
            return fail(SPL_EINVAL, "non-finite initial parameter");
        }
    std::vector<float> ones(m->nout, 1.0f), zeros(m->nout, 0.0f), lw(4, 1.0f);
    unsigned char* D = m->dev;
    bool ok = hipMemcpyAsync(D + m->lay.P, params_host, n * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemsetAsync(D + m->lay.M1, 0, n * 4, st) == hipSuccess &&
              hipMemsetAsync(D + m->lay.M2, 0, n * 4, st) == hipSuccess &&
              hipMemcpyAsync(D + m->lay.mu, zeros.data(), m->nout * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(D + m->lay.sd, ones.data(), m->nout * 4, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(D + m->lay.lw, lw.data(), 16, hipMemcpyHostToDevice, st) == hipSuccess &&
              hipMemcpyAsync(D + m->lay.freqs, freqs_host, kFreq * 3 * 4, hipMemcpyHostToDevice, st) == hipSuccess;
    if (!ok) {
        delete m;
        return fail(SPL_EHIP, "upload of the network parameters failed");
    }
    const float* P = reinterpret_cast<const float*>(D + m->lay.P);
    __bf16* Wh = reinterpret_cast<__bf16*>(D + m->lay.Wh);
    hipLaunchKernelGGL(bf16_copy_kernel, dim3(grid1(m->o.b1)), dim3(kThreads), 0, st, P + m->o.W1, Wh + m->o.hW1,
                       m->o.b1 - m->o.W1, kIn);
    hipLaunchKernelGGL(bf16_copy_kernel, dim3(grid1(m->o.b2 - m->o.W2)), dim3(kThreads), 0, st, P + m->o.W2,
                       Wh + m->o.hW2, m->o.b2 - m->o.W2, kHidden);
    hipLaunchKernelGGL(bf16_copy_kernel, dim3(grid1(m->o.b3 - m->o.W3)), dim3(kThreads), 0, st, P + m->o.W3,
                       Wh + m->o.hW3, m->o.b3 - m->o.W3, kHidden);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid1(kMaxBins * kMaxBins * kMaxBins)), dim3(kThreads), 0, st,
                       reinterpret_cast<unsigned int*>(D + m->lay.bin_err), 0x7f800000u,
                       (int64_t)kMaxBins * kMaxBins * kMaxBins);  // no map yet: every bin routes to the spline
    if (hipGetLastError() != hipSuccess) {
        delete m;
        return fail(SPL_EHIP, "initialisation kernels failed to launch");
    }
    m->nbins = 1;
    m->bin_err_host.assign(1, INFINITY);
    rc = write_meta(m, st);
    if (rc) {
        delete m;
        return rc;
    }
    *out = m;
    return SPL_OK;
}

int spline_mlp_attach(const spline_mlp_desc* desc, const double* cell, void* params_dev, size_t bytes, void* stream,
                      spline_mlp_t** out)
{
    if (!out) return fail(SPL_EINVAL, "out is NULL");
    *out = nullptr;
    spline_mlp_s* m = nullptr;
    int rc = mlp_new(desc, cell, params_dev, bytes, &m);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(m->meta_host, m->dev + m->lay.meta, sizeof(m->meta_host), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        delete m;
        return fail(SPL_EHIP, "reading the parameter buffer failed");
    }
    m->step = m->meta_host[0];
    m->nbins = (int)m->meta_host[1];
    if (m->step < 0 || m->nbins < 1 || m->nbins > kMaxBins) {
        delete m;
        return fail(SPL_EINVAL, "parameter buffer does not hold a network state");
    }
    rc = read_map(m, st);
    if (rc) {
        delete m;
        return rc;
    }
    *out = m;
    return SPL_OK;
}

int spline_mlp_init_output(spline_mlp_t* m, const float* V, const float* G, const float* L, int64_t B, void* stream)
{
    if (!m || !V || !G || !L || B < 2) return fail(SPL_EINVAL, "need a network and at least two target positions");
    int rc = check_dev(m);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int N = m->nout;
    double* stats = reinterpret_cast<double*>(m->dev + m->lay.stats);
    hipLaunchKernelGGL(mlp_stats_kernel, dim3(grid1(N)), dim3(kThreads), 0, st, V, G, L, B, N, stats);
    std::vector<double> s((size_t)N * 6);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(s.data(), stats, s.size() * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "output statistics");
    std::vector<float> mu(N), sd(N);
    double vg = 0, vl = 0;
    for (int n = 0; n < N; ++n) {
        const double mv = s[6 * n] / B;
        const double var = std::max(s[6 * n + 1] / B - mv * mv, 0.0);
        mu[n] = (float)mv;
        sd[n] = (float)std::max(std::sqrt(var), 1e-12);
        const double mg = s[6 * n + 2] / (3.0 * B), ml = s[6 * n + 4] / B;
        vg += std::max(s[6 * n + 3] / (3.0 * B) - mg * mg, 0.0) / ((double)sd[n] * sd[n]);
        vl += std::max(s[6 * n + 5] / B - ml * ml, 0.0) / ((double)sd[n] * sd[n]);
    }
    vg /= N;
    vl /= N;
    float lw[4] = {1.0f, (float)(1.0 / std::max(vg, 1e-30)), (float)(1.0 / std::max(vl, 1e-30)), 0.0f};
    QS_HIP(hipMemcpyAsync(m->dev + m->lay.mu, mu.data(), N * 4, hipMemcpyHostToDevice, st));
    QS_HIP(hipMemcpyAsync(m->dev + m->lay.sd, sd.data(), N * 4, hipMemcpyHostToDevice, st));
    QS_HIP(hipMemcpyAsync(m->dev + m->lay.lw, lw, 16, hipMemcpyHostToDevice, st));
    QS_HIP(hipStreamSynchronize(st));
    return SPL_OK;
}

size_t spline_mlp_train_workspace_bytes(const spline_mlp_t* m, int64_t B)
{
    if (!m || B <= 0 || B > (1 << 24)) return 0;
    return train_ws(B, m->nout).total;
}

static int grad_common(spline_mlp_t* m, const double* pos, const float* tV, const float* tG, const float* tL,
                       int64_t B, void* ws, size_t ws_bytes, hipStream_t st, TrainWs& w)
{
    if (!m || !pos || !tV || !tG || !tL || !ws) return fail(SPL_EINVAL, "NULL argument");
    if (B <= 0 || B > (1 << 24)) return fail(SPL_EINVAL, "training batch must be in [1, 2^24]");
    int rc = check_dev(m);
    if (rc) return rc;
    w = train_ws(B, m->nout);
    if (ws_bytes < w.total) return fail(SPL_ENOMEM, "workspace smaller than spline_mlp_train_workspace_bytes()");
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(SPL_EINVAL, "workspace not 256-byte aligned");
    return compute_grad(m, pos, tV, tG, tL, B, static_cast<unsigned char*>(ws), w, st);
}

int spline_mlp_grad(spline_mlp_t* m, const double* pos, const float* tV, const float* tG, const float* tL, int64_t B,
                    void* ws, size_t ws_bytes, float* grad_out, float* loss_out, void* stream)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    TrainWs w;
    int rc = grad_common(m, pos, tV, tG, tL, B, ws, ws_bytes, st, w);
    if (rc) return rc;
    unsigned char* W = static_cast<unsigned char*>(ws);
    if (grad_out) QS_HIP(hipMemcpyAsync(grad_out, W + w.grad, m->o.total * 4, hipMemcpyDeviceToDevice, st));
    if (loss_out) QS_HIP(hipMemcpyAsync(loss_out, W + w.loss, 4, hipMemcpyDeviceToDevice, st));
    return SPL_OK;
}

int spline_mlp_train_step(spline_mlp_t* m, const double* pos, const float* tV, const float* tG, const float* tL,
                          int64_t B, float lr, void* ws, size_t ws_bytes, float* loss_out, void* stream)
{
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(SPL_EINVAL, "learning rate must be finite and >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    TrainWs w;
    int rc = grad_common(m, pos, tV, tG, tL, B, ws, ws_bytes, st, w);
    if (rc) return rc;
    unsigned char* W = static_cast<unsigned char*>(ws);
    const float* grad = reinterpret_cast<const float*>(W + w.grad);
    float* P = reinterpret_cast<float*>(m->dev + m->lay.P);
    float* M1 = reinterpret_cast<float*>(m->dev + m->lay.M1);
    float* M2 = reinterpret_cast<float*>(m->dev + m->lay.M2);
    __bf16* Wh = reinterpret_cast<__bf16*>(m->dev + m->lay.Wh);
    m->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)m->step));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)m->step));
    const MlpOffsets& o = m->o;
    struct Seg {
        int64_t p, n, h;
        int32_t k;  // columns of the weight matrix (its BF16 copy is in fragment order)
    } segs[6] = {{o.W1, o.b1 - o.W1, o.hW1, kIn},     {o.b1, o.W2 - o.b1, -1, 0},
                 {o.W2, o.b2 - o.W2, o.hW2, kHidden}, {o.b2, o.W3 - o.b2, -1, 0},
                 {o.W3, o.b3 - o.W3, o.hW3, kHidden}, {o.b3, o.total - o.b3, -1, 0}};
    for (const Seg& sg : segs)
        hipLaunchKernelGGL(adam_kernel, dim3(grid1(sg.n)), dim3(kThreads), 0, st, P + sg.p, grad + sg.p, M1 + sg.p,
                           M2 + sg.p, sg.n, lr, b1, b2, eps, bc1, bc2, sg.h >= 0 ? Wh + sg.h : nullptr,
                           sg.k > 0 ? sg.k : 1);
    QS_HIP(hipGetLastError());
    if (loss_out) QS_HIP(hipMemcpyAsync(loss_out, W + w.loss, 4, hipMemcpyDeviceToDevice, st));
    m->meta_host[0] = m->step;
    m->meta_host[1] = m->nbins;
    QS_HIP(hipMemcpyAsync(m->dev + m->lay.meta, m->meta_host, 16, hipMemcpyHostToDevice, st));
    return SPL_OK;
}

int spline_mlp_forward(const spline_mlp_t* m, const double* pos, int64_t B, float* V, float* G, float* L, void* stream)
{
    if (!m) return fail(SPL_EINVAL, "network is NULL");
    if (B < 0) return fail(SPL_EINVAL, "B must be >= 0");
    if (B == 0) return SPL_OK;
    if (!pos || !V || !G || !L) return fail(SPL_EINVAL, "NULL position or output pointer");
    int rc = check_dev(m);
    if (rc) return rc;
    return launch_forward(m, pos, B, V, G, L, static_cast<hipStream_t>(stream));
}

size_t spline_mlp_errmap_workspace_bytes(const spline_mlp_t* m, int64_t n_val)
{
    if (!m || n_val <= 0 || n_val > (1 << 26)) return 0;
    const size_t N = m->nout;
    return a256((size_t)n_val * N * 10 * 4) + a256(3 * N * 4) + 2 * a256((size_t)kMaxBins * kMaxBins * kMaxBins * 4);
}

int spline_mlp_build_error_map(spline_mlp_t* m, const spline_t* table, const double* val_pos, int64_t n_val,
                               int32_t bins_per_dim, void* ws, size_t ws_bytes, void* stream)
{
    if (!m || !table || !val_pos || !ws) return fail(SPL_EINVAL, "NULL argument");
    if (n_val <= 0 || n_val > (1 << 26)) return fail(SPL_EINVAL, "validation count must be in [1, 2^26]");
    if (bins_per_dim < 1 || bins_per_dim > kMaxBins) return fail(SPL_EINVAL, "bins per axis must be in [1, 16]");
    if (table->norb != m->nout || table->store == SPL_F64) return fail(SPL_EINVAL, "table must have N orbitals and FP32 outputs");
    for (int d = 0; d < 3; ++d)
        if (table->grid.cell[d] != m->cell[d]) return fail(SPL_EINVAL, "table and network cells differ");
    if (ws_bytes < spline_mlp_errmap_workspace_bytes(m, n_val)) return fail(SPL_ENOMEM, "workspace too small");
    int rc = check_dev(m);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int N = m->nout;
    const size_t QN = (size_t)n_val * N;
    float* base = static_cast<float*>(ws);
    float *Vm = base, *Gm = Vm + QN, *Lm = Gm + 3 * QN, *Vs = Lm + QN, *Gs = Vs + QN, *Ls = Gs + 3 * QN;
    unsigned char* after = static_cast<unsigned char*>(ws) + a256(QN * 10 * 4);
    unsigned int* smax = reinterpret_cast<unsigned int*>(after);
    const int nb3 = bins_per_dim * bins_per_dim * bins_per_dim;
    unsigned int* berr = reinterpret_cast<unsigned int*>(after + a256(3 * (size_t)N * 4));
    unsigned int* bcnt = berr + a256((size_t)kMaxBins * kMaxBins * kMaxBins * 4) / 4;
    rc = launch_forward(m, val_pos, n_val, Vm, Gm, Lm, st);
    if (rc) return rc;
    rc = spline_eval_vgl(table, val_pos, n_val, Vs, Gs, Ls, stream);
    if (rc) return rc;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid1(3 * N)), dim3(kThreads), 0, st, smax, 0u, (int64_t)3 * N);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid1(nb3)), dim3(kThreads), 0, st, berr, 0u, (int64_t)nb3);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid1(nb3)), dim3(kThreads), 0, st, bcnt, 0u, (int64_t)nb3);
    hipLaunchKernelGGL(colmax_kernel, dim3(grid1(n_val * N)), dim3(kThreads), 0, st, Vs, Gs, Ls, n_val, N, smax);
    hipLaunchKernelGGL(bin_error_kernel, dim3(grid1(n_val * N)), dim3(kThreads), 0, st, val_pos, m->cell[0],
                       m->cell[1], m->cell[2], bins_per_dim, Vm, Gm, Lm, Vs, Gs, Ls, smax, n_val, N, berr);
    hipLaunchKernelGGL(bin_count_kernel, dim3(grid1(n_val)), dim3(kThreads), 0, st, val_pos, m->cell[0], m->cell[1],
                       m->cell[2], bins_per_dim, n_val, bcnt);
    hipLaunchKernelGGL(bin_finalize_kernel, dim3(grid1(nb3)), dim3(kThreads), 0, st, berr, bcnt,
                       reinterpret_cast<float*>(m->dev + m->lay.bin_err), nb3);
    QS_HIP(hipGetLastError());
    m->nbins = bins_per_dim;
    rc = write_meta(m, st);
    return rc ? rc : read_map(m, st);
}

size_t spline_mlp_eval_workspace_bytes(int64_t B)
{
    if (B < 0 || B > 0x7fffffff) return 0;
    return a256((size_t)std::max<int64_t>(B, 1) * 4) + 256;
}

int spline_mlp_eval_vgl(const spline_mlp_t* m, const spline_t* fallback, float tol, const double* pos, int64_t B,
                        float* V, float* G, float* L, void* ws, size_t ws_bytes, int32_t* n_fallback, void* stream)
{
    if (!m) return fail(SPL_EINVAL, "network is NULL");
    if (B < 0 || B > 0x7fffffff) return fail(SPL_EINVAL, "B must be in [0, 2^31)");
    if (B == 0) return SPL_OK;
    if (!pos || !V || !G || !L) return fail(SPL_EINVAL, "NULL position or output pointer");
    int rc = check_dev(m);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!fallback) return launch_forward(m, pos, B, V, G, L, st);
    if (fallback->norb != m->nout || fallback->store == SPL_F64)
        return fail(SPL_EINVAL, "fallback table must have N orbitals and FP32 outputs");
    if (fallback->general) return fail(SPL_EUNSUPPORTED, "the fallback table must have an orthorhombic cell");
    for (int d = 0; d < 3; ++d)
        if (fallback->grid.cell[d] != m->cell[d]) return fail(SPL_EINVAL, "fallback table and network cells differ");
    if (!ws || ws_bytes < spline_mlp_eval_workspace_bytes(B)) return fail(SPL_ENOMEM, "workspace too small");
    int32_t* list = static_cast<int32_t*>(ws);
    int32_t* count = n_fallback ? n_fallback
                                : reinterpret_cast<int32_t*>(static_cast<unsigned char*>(ws) + a256((size_t)B * 4));
    const spline_tile t = fallback->tile;
    const Variant* v = find_variant(fallback->store, t.cw, t.nch, t.lpp, true);
    if (!v) return fail(SPL_EUNSUPPORTED, "fallback tile shape not compiled");
    // Bins above tol, from the host copy of the map: when it routes every
    // bin the network is not run (every row is the table's), when it routes
    // none the routing is skipped (every row is the network's).  The outputs
    // are those of the general path either way.
    size_t routed = 0;
    for (float e : m->bin_err_host) routed += !(e <= tol);
    if (!m->bin_err_host.empty() && routed == m->bin_err_host.size()) {
        hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned int*>(count),
                           (unsigned int)B, 1);
        QS_HIP(hipGetLastError());
        return launch(*v, make_args(fallback, t, pos, B, V, G, L), st);
    }
    rc = launch_forward(m, pos, B, V, G, L, st);
    if (rc) return rc;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned int*>(count), 0u, 1);
    if (!m->bin_err_host.empty() && routed == 0) {
        QS_HIP(hipGetLastError());
        return SPL_OK;
    }
    hipLaunchKernelGGL(route_kernel, dim3(grid1(B)), dim3(kThreads), 0, st, pos, m->cell[0], m->cell[1], m->cell[2],
                       m->nbins, reinterpret_cast<const float*>(m->dev + m->lay.bin_err), tol, B, list, count);
    QS_HIP(hipGetLastError());
    EvalArgs a = make_args(fallback, t, pos, B, V, G, L);
    a.idx = list;
    a.nidx = count;
    return launch(*v, a, st);
}

int spline_mlp_get_info(const spline_mlp_t* m, int64_t* step, int32_t* bins_per_dim)
{
    if (!m) return fail(SPL_EINVAL, "network is NULL");
    if (step) *step = m->step;
    if (bins_per_dim) *bins_per_dim = m->nbins;
    return SPL_OK;
}

int spline_mlp_destroy(spline_mlp_t* m)
{
    delete m;
    return SPL_OK;
}

}  // extern "C"
