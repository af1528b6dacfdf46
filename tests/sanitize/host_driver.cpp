// Runs the library's host-only code -- table layout and sizes, the host
// packer for every storage type, frequency selection, network and Jastrow
// layouts, plan workspace sizes and task lists, the tuning-cache parser --
// on ordinary and edge-case inputs under AddressSanitizer and
// UndefinedBehaviorSanitizer (CPU only, no GPU call).  Exit 0 when every
// check holds; a sanitizer report aborts.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <limits>
#include <string>
#include <vector>

#include "../../include/qmcjastrow.h"
#include "../../include/qmcspline.h"

namespace qs {
struct PlanTask {
    int32_t table;
    int32_t count;
    int64_t first;
};
std::vector<PlanTask> plan_tasks(const int64_t* B, const int64_t* row_bytes, int32_t n, int pb);
bool cache_lookup(const char* path, const std::string& key, spline_tile* t);
const char* tune_cache_path(const char* given);
}  // namespace qs

static int fails = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);   \
            ++fails;                                                              \
        }                                                                         \
    } while (0)

static uint64_t g_seed = 99;
static double urand()
{
    g_seed = g_seed * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(g_seed >> 11) / 9007199254740992.0;
}

static spline_grid grid3(int a, int b, int c, double L = 1.0)
{
    spline_grid g;
    g.n[0] = a;
    g.n[1] = b;
    g.n[2] = c;
    g.cell[0] = g.cell[1] = g.cell[2] = L;
    return g;
}

static void layouts_and_packing()
{
    const int shapes[][3] = {{1, 1, 1}, {2, 3, 1}, {5, 4, 6}, {8, 8, 8}};
    const int norbs[] = {1, 3, 16, 48, 130};
    const spline_dtype types[] = {SPL_F64, SPL_F32, SPL_BF16, SPL_F16};
    for (auto& sh : shapes)
        for (int N : norbs)
            for (spline_dtype st : types) {
                spline_grid g = grid3(sh[0], sh[1], sh[2]);
                spline_layout L;
                CHECK(spline_get_layout(&g, N, st, &L) == SPL_OK);
                const size_t tb = spline_table_bytes(&g, N, st);
                CHECK(tb == (size_t)L.total_bytes && L.row_bytes >= N * L.elem_bytes);
                CHECK(L.scales_offset % 256 == 0 && L.scales_offset >= L.table_bytes);
                const int64_t npts = (int64_t)sh[0] * sh[1] * sh[2];
                std::vector<double> c((size_t)(npts * N));
                for (double& x : c) x = 4 * urand() - 2;
                // exactly the required bytes on the heap: any overrun is reported
                unsigned char* buf = static_cast<unsigned char*>(std::malloc(tb));
                CHECK(spline_pack_host(&g, N, c.data(), st, buf, tb) == SPL_OK);
                CHECK(spline_pack_host(&g, N, c.data(), st, buf, tb - 1) == SPL_ENOMEM);
                c[c.size() / 2] = std::nan("");
                CHECK(spline_pack_host(&g, N, c.data(), st, buf, tb) == SPL_EINVAL);
                std::free(buf);
            }
    // invalid and overflowing sizes
    spline_layout L;
    spline_grid g = grid3(0, 4, 4);
    CHECK(spline_get_layout(&g, 4, SPL_F32, &L) == SPL_EINVAL);
    g = grid3(4, 4, 4);
    CHECK(spline_get_layout(&g, 0, SPL_F32, &L) == SPL_EINVAL);
    CHECK(spline_get_layout(&g, 4, (spline_dtype)9, &L) == SPL_EINVAL);
    CHECK(spline_get_layout(nullptr, 4, SPL_F32, &L) == SPL_EINVAL);
    CHECK(spline_get_layout(&g, 4, SPL_F32, nullptr) == SPL_EINVAL);
    g = grid3(1 << 20, 1 << 20, 1 << 20);
    CHECK(spline_table_bytes(&g, std::numeric_limits<int32_t>::max(), SPL_F64) == 0);
    g = grid3(4, 4, 4, -1.0);
    CHECK(spline_table_bytes(&g, 4, SPL_F32) == 0);
    g = grid3(4, 4, 4);
    g.cell[1] = std::numeric_limits<double>::infinity();
    CHECK(spline_table_bytes(&g, 4, SPL_F32) == 0);
}

static void frequencies_and_network()
{
    spline_grid g = grid3(8, 6, 10);
    const int N = 3;
    std::vector<double> c((size_t)8 * 6 * 10 * N);
    for (double& x : c) x = urand() - 0.5;
    for (int kmax : {1, 2, 4})
        for (int count : {1, 3, 9}) {
            if (kmax == 1 && count > 3) continue;  // |k| <= 1 has three pairs
            std::vector<int32_t> f((size_t)count * 3, -99);
            std::vector<double> e((size_t)count + 2, -1.0);
            CHECK(spline_mlp_select_frequencies(&g, N, c.data(), count, kmax, f.data(), e.data()) == SPL_OK);
            for (int i = 0; i < count; ++i) {
                const int k2 = f[3 * i] * f[3 * i] + f[3 * i + 1] * f[3 * i + 1] + f[3 * i + 2] * f[3 * i + 2];
                CHECK(k2 >= 1 && k2 <= kmax * kmax);
            }
        }
    std::vector<int32_t> f(600 * 3);
    CHECK(spline_mlp_select_frequencies(&g, N, c.data(), 600, 2, f.data(), nullptr) != SPL_OK);  // more than the pairs
    CHECK(spline_mlp_select_frequencies(&g, N, c.data(), 4, 1, f.data(), nullptr) != SPL_OK);
    CHECK(spline_mlp_select_frequencies(&g, N, c.data(), 4, 0, f.data(), nullptr) != SPL_OK);
    CHECK(spline_mlp_select_frequencies(&g, N, nullptr, 4, 2, f.data(), nullptr) != SPL_OK);

    for (int out : {16, 192, 256, 8, 250, 0}) {
        spline_mlp_desc d;
        d.n_freq = 48;
        d.width[0] = 96;
        d.width[1] = 256;
        d.width[2] = 256;
        d.width[3] = out;
        spline_mlp_layout L;
        const bool ok = out >= 16 && out <= 256 && out % 16 == 0;
        CHECK((spline_mlp_param_bytes(&d) > 0) == ok);
        CHECK((spline_mlp_get_layout(&d, &L) == SPL_OK) == ok);
        if (ok) CHECK(L.total <= (int64_t)spline_mlp_param_bytes(&d) && L.n_params > 0);
    }

    jastrow_desc jd;
    jd.n_elec = 16;
    jd.n_up = 8;
    jd.n_ion = 4;
    jd.n_species = 2;
    jd.cell[0] = jd.cell[1] = jd.cell[2] = 1.0;
    int32_t iv[4] = {8, 8, 12, 3};
    CHECK(jastrow_bytes(&jd, iv) > 0);
    iv[2] = 0;
    CHECK(jastrow_bytes(&jd, iv) == 0);
    iv[2] = 8;
    jd.n_up = 17;
    CHECK(jastrow_bytes(&jd, iv) == 0);
}

static void plans()
{
    const int64_t B[] = {1000, 0, 1, 257, 64};
    const int64_t rb[] = {256, 1536, 256, 768, 192};
    CHECK(spline_plan_workspace_bytes(5, B) > 0);
    CHECK(spline_plan_workspace_bytes_sorted(5, B) > 0);
    const int64_t neg[] = {5, -1};
    CHECK(spline_plan_workspace_bytes(2, neg) == 0);
    CHECK(spline_plan_workspace_bytes(0, B) == 0);
    CHECK(spline_plan_workspace_bytes(2, nullptr) == 0);
    const int64_t huge[] = {(int64_t)1 << 40, 1};
    CHECK(spline_plan_workspace_bytes(2, huge) == 0);
    for (int pb : {1, 8, 16, 64, 1000, 0}) {
        const std::vector<qs::PlanTask> t = qs::plan_tasks(B, rb, 5, pb);
        if (pb < 1) {
            CHECK(t.empty());
            continue;
        }
        std::vector<std::vector<int>> seen(5);
        for (int i = 0; i < 5; ++i) seen[i].assign((size_t)B[i], 0);
        int64_t prev_rb = std::numeric_limits<int64_t>::max();
        for (const qs::PlanTask& x : t) {
            CHECK(x.table >= 0 && x.table < 5 && x.count >= 1 && x.count <= pb);
            CHECK(x.first >= 0 && x.first + x.count <= B[x.table]);
            CHECK(rb[x.table] <= prev_rb);  // widest rows first
            prev_rb = rb[x.table];
            for (int64_t p = x.first; p < x.first + x.count; ++p) ++seen[x.table][(size_t)p];
        }
        for (int i = 0; i < 5; ++i)
            for (int v : seen[i]) CHECK(v == 1);  // every position exactly once
    }
}

static void tuning_cache(const char* dir)
{
    const std::string path = std::string(dir) + "/tune_cache_test.txt";
    {
        std::ofstream f(path);
        f << "gfx950 8x8x8 N32 S1 B2^10|4 1 16 32\n";
        f << "no bar on this line\n";
        f << "gfx950 8x8x8 N32 S1 B2^11|not numbers\n";
        f << "gfx950 8x8x8 N32 S1 B2^12|1 2\n";
        f << "|\n\n";
        f << std::string(100000, 'x') << "|1 1 1 1\n";
        f << "gfx950 8x8x8 N32 S1 B2^10|2 2 64 16\n";  // the last match wins
        f << "gfx950 8x8x8 N32 S1 B2^10 V|1 6 64 8";     // no final newline
    }
    spline_tile t{};
    CHECK(qs::cache_lookup(path.c_str(), "gfx950 8x8x8 N32 S1 B2^10", &t));
    CHECK(t.cw == 2 && t.nch == 2 && t.lpp == 64 && t.pb == 16);
    CHECK(qs::cache_lookup(path.c_str(), "gfx950 8x8x8 N32 S1 B2^10 V", &t) && t.nch == 6 && t.pb == 8);
    CHECK(!qs::cache_lookup(path.c_str(), "gfx950 8x8x8 N32 S1 B2^11", &t));
    CHECK(!qs::cache_lookup(path.c_str(), "gfx950 8x8x8 N32 S1 B2^12", &t));
    CHECK(!qs::cache_lookup(path.c_str(), "missing", &t));
    CHECK(!qs::cache_lookup((path + ".absent").c_str(), "gfx950 8x8x8 N32 S1 B2^10", &t));
    std::remove(path.c_str());
    unsetenv("QMCSPLINE_TUNE_CACHE");
    CHECK(qs::tune_cache_path(nullptr) == nullptr);
    CHECK(std::strcmp(qs::tune_cache_path("given"), "given") == 0);
    setenv("QMCSPLINE_TUNE_CACHE", "", 1);
    CHECK(qs::tune_cache_path(nullptr) == nullptr);
    setenv("QMCSPLINE_TUNE_CACHE", "/tmp/from_env.txt", 1);
    CHECK(std::strcmp(qs::tune_cache_path(nullptr), "/tmp/from_env.txt") == 0);
    CHECK(std::strcmp(qs::tune_cache_path("given"), "given") == 0);
    unsetenv("QMCSPLINE_TUNE_CACHE");
}

int main(int argc, char** argv)
{
    layouts_and_packing();
    frequencies_and_network();
    plans();
    tuning_cache(argc > 1 ? argv[1] : "/tmp");
    std::printf("host driver: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
