// Host-only calls of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer (built host-only: no device code, no GPU call):
// parameter validation, create-time tables, workspace sizing, the hookstep
// subproblem, the Hessenberg eigenvalue routine and the tile-cache reader
// and writer, including malformed inputs.  Exit status 0 when every call
// returns the expected status; a sanitizer report aborts with a nonzero one.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/opf.h"

static int fails = 0;
#define EXPECT(cond)                                                        \
    do {                                                                    \
        if (!(cond)) {                                                      \
            std::fprintf(stderr, "expectation failed: %s (line %d)\n", #cond, __LINE__); \
            ++fails;                                                        \
        }                                                                   \
    } while (0)

int main(int argc, char** argv) {
    const char* dir = argc > 1 ? argv[1] : ".";
    opf_params p;
    EXPECT(opf_default_params(&p) == OPF_OK);
    for (int N : {12, 13, 24, 33, 48, 64}) {
        p.N = N;
        std::vector<double> r(N), q(N), d1(2 * N * 9), d2(2 * N * 9);
        std::vector<int32_t> s0(N);
        EXPECT(opf_tables(&p, r.data(), q.data(), d1.data(), d2.data(), s0.data()) == OPF_OK);
        size_t bytes = 0;
        EXPECT(opf_workspace_size(&p, &bytes) == OPF_OK && bytes > 0);
    }
    p.N = 65;  // beyond the largest radial grid
    size_t bytes = 0;
    EXPECT(opf_workspace_size(&p, &bytes) != OPF_OK);
    p.N = 24;
    p.M = 7;  // 3M = 21: no transform length
    EXPECT(opf_workspace_size(&p, &bytes) != OPF_OK);
    opf_default_params(&p);
    std::vector<opf_params> mem(5, p);
    mem[3].N = 32;
    EXPECT(opf_ensemble_workspace_size(mem.data(), 5, &bytes) == OPF_OK && bytes > 0);
    EXPECT(opf_ensemble_workspace_size(mem.data(), 0, &bytes) == OPF_E_INVALID);

    // hookstep subproblem on random Hessenberg matrices of several sizes
    unsigned s = 12345;
    auto rnd = [&]() { s = s * 1103515245u + 12345u; return ((s >> 8) & 0xffff) / 65536.0 - 0.5; };
    for (int k = 1; k <= 40; k += 3) {
        std::vector<double> hb((k + 1) * k, 0.0), y(k);
        for (int i = 0; i <= k; ++i)
            for (int j = 0; j < k; ++j)
                if (i <= j + 1) hb[i * k + j] = rnd();
        double mu = 0, res = 0;
        EXPECT(opf_hookstep_solve(hb.data(), k, 1.0, 0.1, y.data(), &mu, &res) == OPF_OK);
        EXPECT(opf_hookstep_solve(hb.data(), k, 1.0, INFINITY, y.data(), &mu, &res) == OPF_OK);
        std::vector<double> h(k * k), re(k), im(k);
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) h[i * k + j] = i <= j + 1 ? rnd() : 0.0;
        EXPECT(opf_hessenberg_eigvals(h.data(), k, re.data(), im.data()) == OPF_OK);
    }
    double mu = 0, res = 0, yv = 0, hv = 1.0;
    EXPECT(opf_hookstep_solve(nullptr, 1, 1.0, 1.0, &yv, &mu, &res) == OPF_E_INVALID);
    EXPECT(opf_hookstep_solve(&hv, 0, 1.0, 1.0, &yv, &mu, &res) == OPF_E_INVALID);

    // tile cache
    opf_tiles t[2] = {{32, 16, 24, 1, 1, 0, 2, 8, 4, 0.0}, {48, 24, 32, 2, 0, 0, 2, 4, 8, 0.0}};
    std::string path = std::string(dir) + "/tiles.json";
    EXPECT(opf_tile_cache_write(t, 2, path.c_str()) == OPF_OK);
    opf_tiles back[4];
    int32_t n = 0;
    EXPECT(opf_tile_cache_read(path.c_str(), back, 4, &n) == OPF_OK && n == 2);
    EXPECT(back[1].gm == 2 && back[1].tz == 4 && back[1].ztile == 8 && back[0].tz == 8);
    const char* bad[] = {"", "{", "[1,2", "{\"classes\": [{\"N\": 1e400}]}", "{\"classes\": [\"x\"]}",
                         "{\"classes\": [{\"N\": 32, \"M\": 16, \"K\": 24, \"mp\": 1, \"precision\": 1, "
                         "\"gm\": 2, \"tz\": 4, \"ztile\": -8}]}",
                         "\"unterminated", "{\"a\": [[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]}"};
    for (const char* b : bad) {
        std::string bp = std::string(dir) + "/bad.json";
        FILE* f = std::fopen(bp.c_str(), "wb");
        std::fwrite(b, 1, std::strlen(b), f);
        std::fclose(f);
        EXPECT(opf_tile_cache_read(bp.c_str(), back, 4, &n) == OPF_E_INVALID);
    }
    EXPECT(opf_tile_cache_read((std::string(dir) + "/missing.json").c_str(), back, 4, &n) == OPF_E_INVALID);
    EXPECT(std::strlen(opf_status_string(OPF_E_NUMERIC)) > 0);
    std::printf("host calls: %d expectation failures\n", fails);
    return fails ? 1 : 0;
}
