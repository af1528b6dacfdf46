// Setup of the surrogate's features: the integer frequency pairs +-k that
// carry the most energy in a coefficient table (host code, run once before
// training; nothing here is on the evaluation path).
//
// The discrete Fourier transform of orbital m's coefficient grid,
//     c_hat_m(k) = sum_j c_m[j] exp(-2 pi i (k0 j0 / n0 + k1 j1 / n1 + k2 j2 / n2)),
// is needed only at the (2 kmax + 1)^3 integer vectors |k_d| <= kmax, so it
// is taken directly, one axis at a time (z, then y, then x), for a chunk of
// orbitals at a time.  The energy of a pair is sum_m |c_hat_m(k)|^2 +
// |c_hat_m(-k)|^2.
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "common.hpp"

namespace qs {
namespace {

using cplx = std::complex<double>;

// tw[kk][j] = exp(-2 pi i (kk - kmax) j / n), the angle reduced as an
// integer fraction of a turn first.
std::vector<cplx> twiddles(int n, int kmax)
{
    const int K = 2 * kmax + 1;
    std::vector<cplx> tw((size_t)K * n);
    for (int kk = 0; kk < K; ++kk) {
        const int64_t k = kk - kmax;
        for (int j = 0; j < n; ++j) {
            const int64_t r = ((k * j) % n + n) % n;
            const double a = -2.0 * M_PI * (double)r / (double)n;
            tw[(size_t)kk * n + j] = cplx(std::cos(a), std::sin(a));
        }
    }
    return tw;
}

// Energy per k of orbitals [m0, m0 + mc), added into E[K^3].
void chunk_energy(const int32_t n[3], int32_t norb, const double* c, int m0, int mc, int kmax,
                  const std::vector<cplx> tw[3], std::vector<double>& E, int threads)
{
    const int K = 2 * kmax + 1;
    const int n0 = n[0], n1 = n[1], n2 = n[2];
    // pass over z: T1[j0][j1][k2][m]
    std::vector<cplx> T1((size_t)n0 * n1 * K * mc);
    auto zpass = [&](int a0, int a1) {
        for (int j0 = a0; j0 < a1; ++j0)
            for (int j1 = 0; j1 < n1; ++j1) {
                cplx* out = &T1[(((size_t)j0 * n1 + j1) * K) * mc];
                for (int j2 = 0; j2 < n2; ++j2) {
                    const double* row = c + (((size_t)j0 * n1 + j1) * n2 + j2) * norb + m0;
                    for (int k2 = 0; k2 < K; ++k2) {
                        const cplx w = tw[2][(size_t)k2 * n2 + j2];
                        cplx* o = out + (size_t)k2 * mc;
                        for (int m = 0; m < mc; ++m) o[m] += w * row[m];
                    }
                }
            }
    };
    const int nt = std::max(1, std::min(threads, n0));
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t) pool.emplace_back(zpass, (int)((int64_t)n0 * t / nt), (int)((int64_t)n0 * (t + 1) / nt));
    for (auto& th : pool) th.join();
    // pass over y: T2[j0][k1][k2][m]
    std::vector<cplx> T2((size_t)n0 * K * K * mc);
    for (int j0 = 0; j0 < n0; ++j0)
        for (int j1 = 0; j1 < n1; ++j1) {
            const cplx* in = &T1[(((size_t)j0 * n1 + j1) * K) * mc];
            for (int k1 = 0; k1 < K; ++k1) {
                const cplx w = tw[1][(size_t)k1 * n1 + j1];
                cplx* o = &T2[(((size_t)j0 * K + k1) * K) * mc];
                for (size_t i = 0; i < (size_t)K * mc; ++i) o[i] += w * in[i];
            }
        }
    // pass over x, then |.|^2 summed over the chunk's orbitals
    std::vector<cplx> F((size_t)K * K * mc);
    for (int k0 = 0; k0 < K; ++k0) {
        std::fill(F.begin(), F.end(), cplx(0.0, 0.0));
        for (int j0 = 0; j0 < n0; ++j0) {
            const cplx w = tw[0][(size_t)k0 * n0 + j0];
            const cplx* in = &T2[((size_t)j0 * K * K) * mc];
            for (size_t i = 0; i < (size_t)K * K * mc; ++i) F[i] += w * in[i];
        }
        for (int k12 = 0; k12 < K * K; ++k12) {
            double e = 0.0;
            for (int m = 0; m < mc; ++m) e += std::norm(F[(size_t)k12 * mc + m]);
            E[(size_t)k0 * K * K + k12] += e;
        }
    }
}

}  // namespace
}  // namespace qs

using namespace qs;

extern "C" int spline_mlp_select_frequencies(const spline_grid* grid, int32_t n_orb, const double* coefs_host,
                                             int32_t count, int32_t kmax, int32_t* freqs_out, double* energy_out)
{
    if (!grid || !coefs_host || !freqs_out) return fail(SPL_EINVAL, "NULL argument");
    if (n_orb <= 0) return fail(SPL_EINVAL, "n_orb must be positive");
    if (kmax < 1 || kmax > 16) return fail(SPL_EINVAL, "kmax must be in [1, 16]");
    for (int d = 0; d < 3; ++d)
        if (grid->n[d] < 1 || grid->n[d] > 4096) return fail(SPL_EINVAL, "grid size must be in [1, 4096]");
    const int K = 2 * kmax + 1;
    // the +-k pairs with 0 < |k|^2 <= kmax^2, each by the lexicographically larger of k and -k
    std::vector<std::array<int, 3>> reps;
    for (int a = -kmax; a <= kmax; ++a)
        for (int b = -kmax; b <= kmax; ++b)
            for (int c = -kmax; c <= kmax; ++c) {
                const int r2 = a * a + b * b + c * c;
                const std::array<int, 3> k{a, b, c}, mk{-a, -b, -c};
                if (r2 > 0 && r2 <= kmax * kmax && k > mk) reps.push_back(k);
            }
    if (count < 1 || (size_t)count > reps.size())
        return fail(SPL_EINVAL, "count must be in [1, number of +-k pairs with 0 < |k| <= kmax]");
    const int32_t* n = grid->n;
    const std::vector<cplx> tw[3] = {twiddles(n[0], kmax), twiddles(n[1], kmax), twiddles(n[2], kmax)};
    std::vector<double> E((size_t)K * K * K, 0.0);
    const unsigned hc = std::thread::hardware_concurrency();
    const int threads = (int)std::min(16u, std::max(1u, hc));
    constexpr int kChunk = 32;
    for (int m0 = 0; m0 < n_orb; m0 += kChunk)
        chunk_energy(n, n_orb, coefs_host, m0, std::min(kChunk, n_orb - m0), kmax, tw, E, threads);
    auto at = [&](int a, int b, int c) { return E[((size_t)(a + kmax) * K + (b + kmax)) * K + (c + kmax)]; };
    std::vector<std::pair<double, std::array<int, 3>>> pe;
    pe.reserve(reps.size());
    for (const auto& k : reps) pe.push_back({at(k[0], k[1], k[2]) + at(-k[0], -k[1], -k[2]), k});
    // most energy first; equal energies in increasing lexicographic order of k
    std::sort(pe.begin(), pe.end(), [](const auto& x, const auto& y) {
        return x.first != y.first ? x.first > y.first : x.second < y.second;
    });
    for (int i = 0; i < count; ++i)
        for (int d = 0; d < 3; ++d) freqs_out[3 * i + d] = pe[i].second[d];
    if (energy_out) {
        for (int i = 0; i < count; ++i) energy_out[i] = pe[i].first;
        // k = 0, and the whole spectrum by Parseval: n0 n1 n2 sum_j c_j^2
        energy_out[count] = at(0, 0, 0);
        const size_t total = (size_t)n[0] * n[1] * n[2] * n_orb;
        double s = 0.0;
        for (size_t i = 0; i < total; ++i) s += coefs_host[i] * coefs_host[i];
        energy_out[count + 1] = s * (double)n[0] * n[1] * n[2];
    }
    return SPL_OK;
}
