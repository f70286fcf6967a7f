// Host paths of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer
// (no GPU): parameter checks, workspace sizes, the bond threshold, derived
// observables, argument checks that run before any HIP call, and calls on
// handles that do not exist.  Built from the library's sources compiled for the
// host only; every kernel launch would fail, and none is reached.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <vector>

#include "sw.h"
#include "sw_xy.h"

static int failures = 0;
#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                              \
        }                                                                            \
    } while (0)

static sw_params params(uint32_t L, uint32_t q, double K, uint32_t cap = 2, uint32_t ty = 0, uint32_t flags = 0)
{
    sw_params p{};
    p.L = L;
    p.q = q;
    p.K = K;
    p.seed = 1;
    p.init = 1;
    p.obs_capacity = cap;
    p.tile_rows = ty;
    p.flags = flags;
    return p;
}

int main()
{
    const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();

    // bond threshold
    for (double K : {0.0, 0.1, 0.8813735870195430, 2.0, 40.0, inf}) {
        sw_params p = params(16, 2, K);
        uint64_t thr = 0;
        CHECK(sw_threshold(&p, &thr) == SW_OK);
        CHECK(thr <= (uint64_t(1) << 32));
    }
    for (double K : {-1.0, nan}) {
        sw_params p = params(16, 2, K);
        uint64_t thr = 0;
        CHECK(sw_threshold(&p, &thr) == SW_EINVAL);
        CHECK(sw_last_error()[0] != '\0');
    }

    // workspace sizes, valid and invalid parameters
    for (uint32_t L : {2u, 3u, 64u, 100u, 129u, 4096u, 65536u}) {
        for (uint32_t ty : {0u, 32u, 64u, 128u}) {
            sw_params p = params(L, 3, 1.0, 4, ty);
            const size_t n = sw_workspace_bytes(&p);
            CHECK(n > 0 && n % 256 == 0);
        }
    }
    {
        sw_params whole = params(128, 2, 1.0, 4, SW_TILE_WHOLE), big = params(129, 2, 1.0, 4, SW_TILE_WHOLE);
        CHECK(sw_workspace_bytes(&whole) > 0);
        CHECK(sw_workspace_bytes(&big) == 0);
    }
    const sw_params bad[] = {params(1, 2, 1.0),  params(65537, 2, 1.0), params(8, 1, 1.0), params(8, 256, 1.0),
                             params(8, 2, -0.5), params(8, 2, nan),     params(8, 2, 1.0, 1),
                             params(8, 2, 1.0, 2, 48), params(8, 2, 1.0, 2, 0, 2), params(40000, 2, 1.0, 4, 0, SW_CLUSTER_SUMS),
                             params(64, 2, 1.0, 0, 0, SW_CLUSTER_SUMS)};
    for (const sw_params& p : bad) CHECK(sw_workspace_bytes(&p) == 0);

    // sw_init refuses bad workspaces and parameters before any HIP call
    {
        sw_params p = params(16, 2, 1.0);
        const size_t need = sw_workspace_bytes(&p);
        sw_lattice* h = nullptr;
        CHECK(sw_init(&p, nullptr, need, nullptr, &h) == SW_ESPACE);
        CHECK(sw_init(&p, reinterpret_cast<void*>(0x1001), need, nullptr, &h) == SW_ESPACE);
        CHECK(sw_init(&p, reinterpret_cast<void*>(0x10000), need - 256, nullptr, &h) == SW_ESPACE);
        CHECK(h == nullptr);
        sw_params badk = params(16, 2, -1.0);
        CHECK(sw_init(&badk, reinterpret_cast<void*>(0x10000), need, nullptr, &h) == SW_EINVAL);
        CHECK(h == nullptr);
        CHECK(sw_init(nullptr, reinterpret_cast<void*>(0x10000), need, nullptr, &h) == SW_EINVAL);
    }

    // calls on handles that do not exist
    {
        int64_t row[4];
        uint8_t s[4];
        uint32_t n = 0;
        CHECK(sw_sweep(nullptr, 1) != SW_OK);
        CHECK(sw_measure(nullptr, 0, 1, row) != SW_OK);
        CHECK(sw_read_spins(nullptr, s) != SW_OK);
        CHECK(sw_sweeps_done(nullptr, &n) != SW_OK);
        sw_destroy(nullptr);   // no handle: nothing to release, no crash
        CHECK(sw_batch_sweep_all(nullptr, 1) != SW_OK);
        CHECK(sw_group_sweep(nullptr, nullptr, nullptr, 0) != SW_OK);
    }

    // batch workspaces: mixed tile heights are refused
    {
        sw_params arr[2] = {params(16, 2, 1.0, 2, 32), params(16, 2, 1.0)};
        size_t n = 0;
        CHECK(sw_batch_workspace_bytes(arr, 2, &n) == SW_EINVAL);
        sw_params ok[3] = {params(16, 2, 1.0), params(40, 3, 0.5), params(300, 8, 1.2)};
        CHECK(sw_batch_workspace_bytes(ok, 3, &n) == SW_OK && n > 0 && n % 256 == 0);
        CHECK(sw_batch_workspace_bytes(ok, 0, &n) != SW_OK);
    }

    // autotune argument checks (before any launch)
    {
        sw_params arr[2] = {params(64, 2, 1.0), params(100, 3, 0.9)};
        uint32_t best = 7;
        double ms[9];
        const uint32_t c_bad[2] = {32, 48}, c9[9] = {32, 32, 32, 32, 32, 32, 32, 32, 32}, c_ok[1] = {64};
        void* ws = reinterpret_cast<void*>(0x10000);
        CHECK(sw_batch_autotune(arr, 2, c_bad, 2, 4, ws, size_t(1) << 40, nullptr, &best, ms) == SW_EINVAL);
        CHECK(sw_batch_autotune(arr, 2, c_ok, 0, 4, ws, size_t(1) << 40, nullptr, &best, ms) == SW_EINVAL);
        CHECK(sw_batch_autotune(arr, 2, c9, 9, 4, ws, size_t(1) << 40, nullptr, &best, ms) == SW_EINVAL);
        CHECK(sw_batch_autotune(arr, 2, c_ok, 1, 0, ws, size_t(1) << 40, nullptr, &best, ms) == SW_EINVAL);
        CHECK(sw_batch_autotune(arr, 0, c_ok, 1, 4, ws, size_t(1) << 40, nullptr, &best, ms) == SW_EINVAL);
        CHECK(sw_batch_autotune(arr, 2, c_ok, 1, 4, reinterpret_cast<void*>(0x10001), size_t(1) << 40, nullptr,
                                &best, ms) == SW_ESPACE);
        CHECK(best == 7);
    }

    // tiles and group workspaces
    {
        sw_params p = params(100, 2, 1.0, 2, 64);
        uint32_t tiles = 0;
        CHECK(sw_tile_count(&p, &tiles) == SW_OK && tiles == 2 * 2);
        size_t n = 0;
        CHECK(sw_group_workspace_bytes(16, 1024, &n) == SW_OK && n > 0);
    }

    // derived observables of a row (energy, order parameter, Ising magnetisation)
    {
        const uint32_t L = 4, q = 3;
        const int64_t row[2 + q] = {10, 20, 6, 5, 5};   // n_unsat, n_active, n_0..n_2 (16 sites)
        double out[3];
        CHECK(sw_derived(L, q, row, out) == SW_OK);
        CHECK(std::fabs(out[0] - 10.0 / 16) < 1e-15);
        CHECK(std::fabs(out[1] - (3.0 * 6 / 16 - 1) / 2) < 1e-15);
        const int64_t wrong[2 + q] = {10, 20, 6, 5, 4};  // counts do not add up to N
        CHECK(sw_derived(L, q, wrong, out) == SW_EINVAL);
        const int64_t r2[4] = {3, 9, 10, 6};
        CHECK(sw_derived(4, 2, r2, out) == SW_OK && out[2] == 4.0);
        CHECK(sw_derived(1, 2, r2, out) == SW_EINVAL);
    }

    // XY parameters, workspace and derived values
    {
        sw_xy_params p{};
        p.L = 64;
        p.K = 1.0;
        p.seed = 1;
        p.init = 1;
        p.obs_capacity = 2;
        p.tile_rows = 0;
        p.dir_bits = 32;
        CHECK(sw_xy_workspace_bytes(&p) > 0);
        for (uint32_t bits : {0u, 33u}) {
            sw_xy_params b = p;
            b.dir_bits = bits;
            CHECK(sw_xy_workspace_bytes(&b) == 0);
        }
        sw_xy_params bk = p;
        bk.K = nan;
        CHECK(sw_xy_workspace_bytes(&bk) == 0);
        sw_lattice* h = nullptr;
        CHECK(sw_xy_init(&p, nullptr, sw_xy_workspace_bytes(&p), nullptr, &h) == SW_ESPACE && h == nullptr);
        std::vector<int64_t> row(SW_XY_OBS_WORDS, 0);
        row[1] = int64_t(1) << 62;   // a sum far beyond what N sites can give: rejected
        double out[8];
        CHECK(sw_xy_derived(16, 1.0, row.data(), out) != SW_OK);
    }

    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("host C-ABI checks passed\n");
    return 0;
}
