// Host planner of libfse driven from the command line, for CPU tests (built
// with g++ and the address and undefined-behaviour sanitizers):
//   plan_harness MASKFILE W H [opt RHO DELTA] B1 b1 [B2 b2 [B3 b3]]
// MASKFILE holds W*H bytes (row-major, 1 = lost).  Prints
//   "blocks N", then per block "y0 x0 class level", then "owner" and the
// fine-cell owner map row by row.  With "opt", the blocks are in the
// optimised processing order (and numbered so), with its dependency levels.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "fse_plan.h"

int main(int argc, char** argv) {
    int first = 4;
    bool opt = false;
    double rho = 0.8, delta = 0.5;
    if (argc > 7 && std::string(argv[4]) == "opt") {
        opt = true;
        rho = std::atof(argv[5]);
        delta = std::atof(argv[6]);
        first = 7;
    }
    if (argc < first + 2 || (argc - first) % 2 != 0) {
        std::fprintf(stderr, "usage: plan_harness MASKFILE W H [opt RHO DELTA] B1 b1 [B2 b2 [B3 b3]]\n");
        return 2;
    }
    const int W = std::atoi(argv[2]), H = std::atoi(argv[3]);
    std::vector<fse::ClassCfg> cls;
    for (int i = first; i + 1 < argc; i += 2) {
        const int B = std::atoi(argv[i]), b = std::atoi(argv[i + 1]);
        cls.push_back({B, b, 1, B + 2 * b});
    }
    std::vector<uint8_t> mask((size_t)W * H);
    std::FILE* f = std::fopen(argv[1], "rb");
    if (!f || std::fread(mask.data(), 1, mask.size(), f) != mask.size()) {
        std::fprintf(stderr, "cannot read %s\n", argv[1]);
        return 2;
    }
    std::fclose(f);
    fse::RegionPlan P;
    fse::PlanScratch S;
    if (!fse::plan_region(mask.data(), W, W, H, cls, P, S)) {
        std::fprintf(stderr, "plan_region failed\n");
        return 3;
    }
    int reach = 0;
    for (auto& c : cls) reach = c.b > reach ? c.b : reach;
    if (opt) {
        fse::OrderScratch O;
        fse::plan_priority_order(P, mask.data(), W, cls, rho, delta, O, 4);
    } else {
        fse::plan_levels(P, cls, reach, S.cell_level);
    }
    const size_t n = P.desc.size() / 4;
    std::printf("blocks %zu\n", n);
    for (size_t j = 0; j < n; ++j)
        std::printf("%d %d %d %d\n", P.desc[4 * j], P.desc[4 * j + 1], P.desc[4 * j + 2], P.level[j]);
    std::printf("owner %d %d\n", P.fw, P.fh);
    for (int y = 0; y < P.fh; ++y) {
        for (int x = 0; x < P.fw; ++x) std::printf("%d ", P.owner[(size_t)y * P.fw + x]);
        std::printf("\n");
    }
    return 0;
}
