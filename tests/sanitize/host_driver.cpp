// Host-side driver of the library's integer geometry code (geom.cpp) for
// sanitizer builds (AddressSanitizer, UndefinedBehaviorSanitizer): seeded
// electrodes, biofilm layers, link masks and lists, percolation, the flow
// domain, reference nodes, descriptor words and growth picks on 2-D and
// 3-D grids including ragged and degenerate ones, and the rejections of
// invalid inputs.  Prints "ok" and exits 0 when every call behaved.
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "lbm_internal.h"

#define CHECK(c)                                                                 \
    do {                                                                         \
        if (!(c)) {                                                              \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);     \
            exit(1);                                                             \
        }                                                                        \
    } while (0)

static void run_grid(lbm_grid g, bool fibres, uint64_t seed)
{
    const size_t N = (size_t)g.nx * g.ny * g.nz;
    std::vector<uint8_t> cls(N);
    double frac = 0.0;
    if (fibres) {
        lbm_fibre_params fp = {1, 2, 0.2};
        CHECK(lbm_geom_fibres(g, &fp, seed, cls.data(), &frac) == LBM_OK);
    } else {
        lbm_disc_params dp = {2, 4, 0.3, (int)(seed & 1)};
        CHECK(lbm_geom_discs(g, &dp, seed, cls.data(), &frac) == LBM_OK);
    }
    CHECK(lbm_biofilm_layer(g, cls.data()) == LBM_OK);
    CHECK(lbmh::check_mask(g, cls.data()).empty());
    std::vector<uint32_t> lf(N), lc(N);
    CHECK(lbm_links(g, cls.data(), 0, lf.data()) == LBM_OK);
    CHECK(lbm_links(g, cls.data(), 1, lc.data()) == LBM_OK);
    for (int which = 0; which < 2; ++which) {
        const int64_t n = lbm_link_list(g, cls.data(), which, nullptr, 0);
        CHECK(n >= 0);
        std::vector<int64_t> list((size_t)(2 * n + 2));
        CHECK(lbm_link_list(g, cls.data(), which, list.data(), n) == n);
        if (n > 1)
            CHECK(lbm_link_list(g, cls.data(), which, list.data(), n / 2) >= 0);
    }
    std::vector<uint8_t> dom(N);
    CHECK(lbm_flow_domain(g, cls.data(), dom.data()) == LBM_OK);
    const int perc = lbm_percolates(g, cls.data());
    CHECK(perc == 0 || perc == 1);
    const std::vector<uint8_t> dv = lbmh::flow_domain(g, cls.data());
    const std::vector<int64_t> refn = lbmh::reference_nodes(g, dv);
    CHECK((int)refn.size() == g.nx);
    std::vector<uint32_t> desc(N);
    lbmh::build_desc(g, cls.data(), dv, refn, desc.data());
    std::vector<double> C(N);
    for (size_t i = 0; i < N; ++i)
        C[i] = (double)((i * 2654435761u) % 1000) / 1000.0;
    for (double xi : {0.0, 0.37, 0.999999})
        (void)lbm_growth_pick(g, cls.data(), C.data(), xi);
    std::vector<double> Z(N, 0.0);
    (void)lbm_growth_pick(g, cls.data(), Z.data(), 0.5);
}

int main()
{
    run_grid({96, 48, 1}, false, 1);
    run_grid({131, 67, 1}, false, 2);
    run_grid({64, 3, 1}, false, 3);
    run_grid({40, 20, 12}, true, 4);
    run_grid({33, 9, 5}, true, 5);
    // rejections
    std::vector<uint8_t> cls(96 * 48);
    lbm_disc_params bad = {5, 2, 0.3, 0};
    CHECK(lbm_geom_discs({96, 48, 1}, &bad, 1, cls.data(), nullptr) == LBM_EINVAL);
    lbm_disc_params full = {2, 4, 1.0, 0};
    CHECK(lbm_geom_discs({96, 48, 1}, &full, 1, cls.data(), nullptr) == LBM_EINVAL);
    CHECK(lbm_geom_discs({3, 48, 1}, &full, 1, cls.data(), nullptr) == LBM_EINVAL);
    lbm_disc_params dp = {2, 4, 0.3, 0};
    CHECK(lbm_geom_discs({96, 48, 1}, &dp, 1, cls.data(), nullptr) == LBM_OK);
    cls[48 * 96 / 2] = 7; // unknown class
    CHECK(!lbmh::check_mask({96, 48, 1}, cls.data()).empty());
    CHECK(lbm_geom_discs({96, 48, 1}, &dp, 1, cls.data(), nullptr) == LBM_OK);
    cls[96 * 10] = LBM_SOLID; // inlet column
    CHECK(!lbmh::check_mask({96, 48, 1}, cls.data()).empty());
    std::vector<uint64_t> sm(8);
    lbm_splitmix64(42, 8, sm.data());
    printf("ok\n");
    return 0;
}
