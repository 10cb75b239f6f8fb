// The library's host code under the compiler's sanitizers (AddressSanitizer
// with UndefinedBehaviorSanitizer, or ThreadSanitizer): the threaded list
// builder (polygons in parallel, and one large polygon split over threads),
// the MBR join, list files and list validation.  Built by
// tests/test_sanitizers.py from the library's host sources with g++ (no
// device code: the one device entry the list sources reach is stubbed
// below and never called).
//
// Input file (little-endian): uint64 n, uint64 nv, uint64 voff[n + 1],
// double xy[2 * nv], double x0, y0, side, uint64 order.  Usage:
//     sanitize_host INPUT TMPDIR
// Exit status 0 when every check holds; a sanitizer report makes the test
// fail on its own (halt_on_error / the report in stderr).
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "april.h"
#include "internal.hpp"

namespace april {
// compressed lists are decoded on a device; not reached here
int launch_decode_lists(const april_lists_t *, bool, uint32_t *, uint32_t *, hipStream_t) {
    return fail(APRIL_E_NODEV, "no device in the sanitizer build");
}
}  // namespace april

#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            std::exit(1);                                                 \
        }                                                                 \
    } while (0)

struct Arrays {
    std::vector<uint64_t> offA, offF;
    std::vector<uint32_t> sA, eA, sF, eF;
};

static Arrays export_lists(const april_lists_t *L) {
    april_lists_info_t inf;
    CHECK(april_lists_info(L, &inf) == APRIL_OK);
    Arrays a;
    a.offA.resize(inf.n_objects + 1);
    a.offF.resize(inf.n_objects + 1);
    a.sA.resize(inf.n_a);
    a.eA.resize(inf.n_a);
    a.sF.resize(inf.n_f);
    a.eF.resize(inf.n_f);
    CHECK(april_lists_export(L, a.offA.data(), a.sA.data(), a.eA.data(), a.offF.data(), a.sF.data(),
                             a.eF.data()) == APRIL_OK);
    return a;
}

static bool same(const Arrays &a, const Arrays &b) {
    return a.offA == b.offA && a.offF == b.offF && a.sA == b.sA && a.eA == b.eA && a.sF == b.sF && a.eF == b.eF;
}

static april_lists_t *build(const april_grid_t &g, const std::vector<double> &xy, const std::vector<uint64_t> &voff,
                            const char *threads) {
    setenv("APRIL_HOST_THREADS", threads, 1);
    april_lists_t *L = nullptr;
    CHECK(april_build_lists(&g, xy.data(), voff.data(), voff.size() - 1, APRIL_STRICT, &L) == APRIL_OK);
    return L;
}

int main(int argc, char **argv) {
    CHECK(argc == 3);
    FILE *f = std::fopen(argv[1], "rb");
    CHECK(f);
    uint64_t n = 0, nv = 0;
    CHECK(std::fread(&n, 8, 1, f) == 1 && std::fread(&nv, 8, 1, f) == 1);
    std::vector<uint64_t> voff(n + 1);
    std::vector<double> xy(2 * nv);
    CHECK(std::fread(voff.data(), 8, n + 1, f) == n + 1);
    CHECK(std::fread(xy.data(), 8, 2 * nv, f) == 2 * nv);
    double gd[3];
    uint64_t order = 0;
    CHECK(std::fread(gd, 8, 3, f) == 3 && std::fread(&order, 8, 1, f) == 1);
    std::fclose(f);
    april_grid_t g{};
    g.x0 = gd[0];
    g.y0 = gd[1];
    g.side = gd[2];
    g.order = uint32_t(order);

    // 1. the collection with one thread and with eight
    april_lists_t *L1 = build(g, xy, voff, "1");
    april_lists_t *L8 = build(g, xy, voff, "8");
    const Arrays a1 = export_lists(L1), a8 = export_lists(L8);
    CHECK(same(a1, a8));
    CHECK(a1.sA.size() > 0 && a1.sF.size() > 0);

    // 2. the first polygon alone, split over eight threads
    setenv("APRIL_PAR_BUILD_CELLS", "1", 1);
    std::vector<uint64_t> v0 = {0, voff[1]};
    std::vector<double> xy0(xy.begin(), xy.begin() + 2 * voff[1]);
    april_lists_t *P1 = build(g, xy0, v0, "1");
    april_lists_t *P8 = build(g, xy0, v0, "8");
    const Arrays p1 = export_lists(P1), p8 = export_lists(P8);
    CHECK(same(p1, p8));
    CHECK(p1.sA == std::vector<uint32_t>(a1.sA.begin(), a1.sA.begin() + a1.offA[1]));
    unsetenv("APRIL_PAR_BUILD_CELLS");

    // 3. MBR join against brute force
    std::vector<double> box(4 * n);
    for (uint64_t k = 0; k < n; k++) {
        double *b = &box[4 * k];
        b[0] = b[2] = xy[2 * voff[k]];
        b[1] = b[3] = xy[2 * voff[k] + 1];
        for (uint64_t v = voff[k]; v < voff[k + 1]; v++) {
            b[0] = std::min(b[0], xy[2 * v]);
            b[1] = std::min(b[1], xy[2 * v + 1]);
            b[2] = std::max(b[2], xy[2 * v]);
            b[3] = std::max(b[3], xy[2 * v + 1]);
        }
    }
    const uint64_t half = n / 2;
    uint64_t need = 0;
    CHECK(april_mbr_join(box.data(), half, box.data() + 4 * half, n - half, nullptr, nullptr, 0, &need) ==
          APRIL_E_NOMEM);
    std::vector<uint32_t> jr(need + 1), js(need + 1);
    uint64_t got = 0;
    CHECK(april_mbr_join(box.data(), half, box.data() + 4 * half, n - half, jr.data(), js.data(), need, &got) ==
          APRIL_OK);
    CHECK(got == need);
    uint64_t brute = 0;
    for (uint64_t i = 0; i < half; i++)
        for (uint64_t j = half; j < n; j++) {
            const double *a = &box[4 * i], *b = &box[4 * j];
            brute += a[0] <= b[2] && b[0] <= a[2] && a[1] <= b[3] && b[1] <= a[3];
        }
    CHECK(brute == got);

    // 4. list files: round trip, then a damaged copy
    const std::string path = std::string(argv[2]) + "/lists.april";
    CHECK(april_lists_save(L8, path.c_str()) == APRIL_OK);
    april_lists_t *back = nullptr;
    CHECK(april_lists_load(path.c_str(), 1, &back) == APRIL_OK);
    CHECK(same(export_lists(back), a8));
    april_lists_free(back);
    {
        FILE *h = std::fopen(path.c_str(), "r+b");
        CHECK(h);
        std::fseek(h, 200, SEEK_SET);
        unsigned char c = 0;
        CHECK(std::fread(&c, 1, 1, h) == 1);
        c ^= 0x10;
        std::fseek(h, 200, SEEK_SET);
        CHECK(std::fwrite(&c, 1, 1, h) == 1);
        std::fclose(h);
    }
    april_lists_t *bad = nullptr;
    CHECK(april_lists_load(path.c_str(), 1, &bad) == APRIL_E_CORRUPT && bad == nullptr);
    CHECK(april_lists_load((path + ".missing").c_str(), 1, &bad) == APRIL_E_IO);

    // 5. validation of caller arrays: valid lists pass, a swapped pair fails
    april_lists_t *V = nullptr;
    CHECK(april_lists_from_arrays(&g, n, a1.offA.data(), a1.sA.data(), a1.eA.data(), a1.offF.data(), a1.sF.data(),
                                  a1.eF.data(), 1, &V) == APRIL_OK);
    april_lists_free(V);
    Arrays broken = a1;
    CHECK(broken.sA.size() >= 2);
    std::swap(broken.sA[0], broken.sA[1]);
    std::swap(broken.eA[0], broken.eA[1]);
    V = nullptr;
    CHECK(april_lists_from_arrays(&g, n, broken.offA.data(), broken.sA.data(), broken.eA.data(), broken.offF.data(),
                                  broken.sF.data(), broken.eF.data(), 1, &V) == APRIL_E_CORRUPT);

    april_lists_free(L1);
    april_lists_free(L8);
    april_lists_free(P1);
    april_lists_free(P8);
    std::printf("sanitize_host ok: %llu polygons, %zu A intervals, %llu MBR pairs\n", (unsigned long long)n,
                a1.sA.size(), (unsigned long long)got);
    return 0;
}
