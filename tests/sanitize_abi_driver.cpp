// Host-side checks of libhrw under AddressSanitizer / UndefinedBehaviorSanitizer
// (built with the sanitizers on the host pass only and run on a CPU by
// tests/test_sanitizers.py).  Exercises the C ABI's argument validation and
// size planning, which run before anything touches a device, and the parser
// of the launch-shape cache on well-formed, malformed and hostile files.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

#include "../paper_2405_19294_amd/csrc/hop_impl.h"
#include "hrw.h"

#define CHECK(cond)                                                               \
    do {                                                                          \
        if (!(cond)) {                                                            \
            fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #cond, \
                    hrw_last_error());                                           \
            return 1;                                                             \
        }                                                                         \
    } while (0)

static int abi_checks()
{
    CHECK(strlen(hrw_version()) > 0);
    int nr = 0;
    CHECK(hrw_rep_dim(3, HRW_REP_SYM, &nr) == HRW_OK && nr == 6);
    CHECK(hrw_rep_dim(1, HRW_REP_FUND, &nr) == HRW_EINVAL);
    CHECK(hrw_rep_dim(3, 7, &nr) == HRW_EINVAL);
    CHECK(hrw_rep_dim(3, 0, nullptr) == HRW_EINVAL);
    const int dims[4] = {4, 4, 2, 6}, odd[4] = {4, 3, 2, 6}, huge[4] = {1 << 10, 1 << 10, 1 << 10, 4};
    size_t bytes = 0;
    for (int nc = 2; nc <= 4; ++nc)
        for (int rep = 0; rep < 4; ++rep)
            for (unsigned mask : {1u, 3u, 15u, 1u | (1u << 4), 3u | (1u << 5)}) {
                const int rc = hrw_gauge_storage_size(dims, nc, rep, mask, &bytes);
                CHECK(rc == HRW_OK || rc == HRW_EUNSUPPORTED);
            }
    CHECK(hrw_gauge_storage_size(odd, 3, 0, 1, &bytes) == HRW_EINVAL);
    CHECK(hrw_gauge_storage_size(huge, 3, 0, 1, &bytes) == HRW_EINVAL);
    CHECK(hrw_gauge_storage_size(dims, 3, 0, 0, &bytes) == HRW_EINVAL);
    CHECK(hrw_gauge_storage_size(dims, 3, 0, 1u << 9, &bytes) == HRW_EINVAL);
    CHECK(hrw_gauge_storage_size(dims, 5, 0, 1, &bytes) == HRW_EUNSUPPORTED);
    CHECK(hrw_gauge_storage_size(nullptr, 3, 0, 1, &bytes) == HRW_EINVAL);
    hrw_solve_params p;
    memset(&p, 0, sizeof p);
    p.tol = 1e-10;
    p.max_iter = 100;
    p.reliable_every = 50;
    for (int sys = 0; sys <= 4; ++sys)
        for (int dt = 0; dt < 4; ++dt)
            for (int n : {1, 7, 64}) {
                p.system = sys;
                p.inner_dtype = dt;
                const int rc = hrw_workspace_size(dims, 3, 0, n, &p, &bytes);
                CHECK(rc == HRW_OK || rc == HRW_EUNSUPPORTED);
                CHECK(hrw_workspace_size(dims, 3, 0, n, nullptr, &bytes) == HRW_OK && bytes > 0);
            }
    CHECK(hrw_workspace_size(dims, 3, 0, 65, nullptr, &bytes) == HRW_EINVAL);
    CHECK(hrw_workspace_size(dims, 3, 0, 0, nullptr, &bytes) == HRW_EINVAL);
    p.tol = -1;
    CHECK(hrw_workspace_size(dims, 3, 0, 1, &p, &bytes) == HRW_EINVAL);
    p.tol = 1e-10;
    p.reliable_delta = 1.5;
    CHECK(hrw_workspace_size(dims, 3, 0, 1, &p, &bytes) == HRW_EINVAL);
    p.reliable_delta = 0;
    // calls that are refused before anything is enqueued
    hrw_gauge *g = nullptr;
    double buf[16] = {0};
    const double theta[4] = {0, 0, 0, 0};
    const double kap[1] = {0.1};
    CHECK(hrw_gauge_create(dims, 3, 0, nullptr, 1, buf, sizeof buf, nullptr, &g) == HRW_EINVAL);
    CHECK(hrw_gauge_create(dims, 3, 0, buf, 1, buf, 8, nullptr, &g) == HRW_ENOMEM);
    CHECK(hrw_gauge_create(dims, 2, 0, buf, 1u | (1u << 5), buf, sizeof buf, nullptr, &g) == HRW_EUNSUPPORTED);
    CHECK(hrw_gauge_create(dims, 3, 0, buf, 1u << 5, buf, sizeof buf, nullptr, &g) == HRW_EINVAL);
    CHECK(hrw_dw_apply(nullptr, 0.1, theta, 0, 1, 0, buf, buf + 8, buf, sizeof buf, nullptr) == HRW_EINVAL);
    CHECK(hrw_deo_apply(nullptr, kap, theta, 0, 1, 0, buf, buf + 8, buf, sizeof buf, nullptr) == HRW_EINVAL);
    CHECK(hrw_deo_apply_noalloc(nullptr, kap, theta, 0, 1, 0, buf, buf + 8, nullptr) == HRW_EINVAL);
    hrw_solve_result res[1];
    CHECK(hrw_cg_solve(nullptr, &p, 1, kap, buf, buf + 8, res, buf, sizeof buf, nullptr) == HRW_EINVAL);
    CHECK(hrw_gauge_destroy(nullptr) == HRW_OK);
    return 0;
}

static void put(const char *path, const std::string &text)
{
    FILE *f = fopen(path, "wb");
    fwrite(text.data(), 1, text.size(), f);
    fclose(f);
}

static int cache_checks(const char *dir)
{
    const std::string path = std::string(dir) + "/tune.json";
    hrw::TuneCache c;
    std::map<std::string, std::pair<hrw::MrShape, double>> m;
    put(path.c_str(), "{\n  \"a/nr6\": {\"threads\": 128, \"cmax\": 4, \"sites\": 32, \"us\": 1.5},\n"
                      "  \"b\": {\"us\": 2, \"sites\": 16, \"cmax\": 16, \"threads\": 256}\n}\n");
    c.read_file(path, m);
    CHECK(m.size() == 2 && m["a/nr6"].first.threads == 128 && m["b"].first.sites == 16);
    const char *bad[] = {"", "{", "{\"k\": {", "{\"k\": {\"threads\": 100, \"cmax\": 4, \"sites\": 16}}",
                         "{\"k\": {\"threads\": 64, \"cmax\": 4, \"sites\": 17}}", "}}}}{{{{\"\"\"\":::",
                         "{\"k\": {\"threads\": -64, \"cmax\": 4, \"sites\": 16}}", "[1, 2, 3]",
                         "{\"k\": {\"threads\": 1e999, \"cmax\": 4, \"sites\": 16}}",
                         "{\"k\": {\"threads\": 64, \"cmax\": 4, \"sites\": 16, \"planes\": 3}}",
                         "{\"k\": {\"threads\": 64, \"cmax\": 4, \"sites\": 16, \"planes\": -1e300}}"};
    for (const char *b : bad) {
        m.clear();
        put(path.c_str(), b);
        c.read_file(path, m);
        CHECK(m.empty());
    }
    std::string big = "{\"" + std::string(100000, 'x') + "\": {\"threads\": 64, \"cmax\": 4, \"sites\": 16}}";
    put(path.c_str(), big);
    m.clear();
    c.read_file(path, m);
    CHECK(m.size() == 1);
    std::string junk(70000, '\0');
    for (size_t i = 0; i < junk.size(); ++i) junk[i] = (char)((i * 2654435761u) >> 13);
    put(path.c_str(), junk);
    m.clear();
    c.read_file(path, m);
    // store then read back through a fresh cache object
    setenv("HRW_TUNE_CACHE", path.c_str(), 1);
    put(path.c_str(), "");
    hrw::TuneCache w;
    w.store("gfx950/nr3/rs3/f32/n8/v10", hrw::MrShape{192, 16, 16}, 12.5);
    w.store("gfx950/nr6/rs6/f32/n24/v19", hrw::MrShape{256, 4, 32}, 99.0);
    w.store("gfx950/nr6/rs6/f32/n12/v19/w2", hrw::MrShape{192, 32, 16, 4}, 50.0);
    hrw::TuneCache r;
    hrw::MrShape sh{0, 0, 0, 0};
    CHECK(r.lookup("gfx950/nr6/rs6/f32/n24/v19", &sh) && sh.threads == 256 && sh.cmax == 4 && sh.sites == 32 &&
          sh.planes == 1);
    CHECK(r.lookup("gfx950/nr6/rs6/f32/n12/v19/w2", &sh) && sh.threads == 192 && sh.cmax == 32 && sh.planes == 4);
    CHECK(!r.lookup("missing", &sh));
    return 0;
}

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    if (abi_checks() || cache_checks(argv[1])) return 1;
    printf("abi sanitizer driver: ok\n");
    return 0;
}
