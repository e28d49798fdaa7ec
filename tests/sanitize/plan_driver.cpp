// Host driver for the sanitizer build of the plan construction
// (paper_2601_06849_amd/csrc/plan.cpp): builds plans for valid problems of
// every precision, rational family and dimension (extents from one point to
// the largest supported) and for malformed ones, and reads the tables.
// Exit status 0 on success.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "plan.hpp"

using namespace etdds;

static etd_problem base(int dim, int nx, int ny, int nz) {
    etd_problem p;
    std::memset(&p, 0, sizeof(p));
    p.dim = dim;
    p.n[0] = nx;
    p.n[1] = ny;
    p.n[2] = nz;
    for (int d = 0; d < 3; ++d) {
        p.lo[d] = 0.0;
        p.hi[d] = 1.0 + d;
    }
    p.ncomp = 1;
    p.kappa[0] = 0.2;
    p.q = 0.3;
    p.tau = 0.01;
    p.rxn = ETD_RXN_FISHER;
    p.rxn_param[0] = 1.0;
    p.pade = 2;
    p.precision = ETD_FP64;
    return p;
}

int main() {
    int bad = 0;
    const int ext[][4] = {{2, 1, 1, 1}, {2, 63, 63, 1}, {2, 1023, 40, 1}, {3, 7, 1, 33}, {3, 255, 255, 255},
                          {3, 576, 9, 7}};
    for (const auto& e : ext)
        for (int prec = ETD_FP64; prec <= ETD_FP64_BF16X6; ++prec)
            for (int pade : {0, 2, 4})
                for (int rxn : {ETD_RXN_FISHER, ETD_RXN_AC_MMS, ETD_RXN_FHN_CUBIC}) {
                    etd_problem p = base(e[0], e[1], e[2], e[3]);
                    p.precision = prec;
                    p.pade = pade;
                    p.rxn = rxn;
                    p.ncomp = rxn == ETD_RXN_FHN_CUBIC ? 2 : 1;
                    p.kappa[1] = 0.01;
                    Plan pl;
                    std::string err;
                    const etd_status st = build_plan(p, pl, err);
                    if (st == ETD_OK) {
                        if (pl.image.size() != pl.table_bytes || pl.lay.total < pl.table_bytes) bad = 1;
                        for (int d = 0; d < p.dim; ++d)
                            for (int c = 0; c < pl.nc; ++c)
                                for (int l = 0; l < 3; ++l)
                                    for (double v : pl.inc[d][c][l])
                                        if (!std::isfinite(v)) bad = 1;
                    } else if (st != ETD_EUNSUPPORTED) {
                        std::fprintf(stderr, "unexpected status %d: %s\n", int(st), err.c_str());
                        bad = 1;
                    }
                }
    // malformed problems are rejected with a message
    for (int k = 0; k < 8; ++k) {
        etd_problem p = base(2, 10, 10, 1);
        switch (k) {
        case 0: p.dim = 4; break;
        case 1: p.n[1] = 0; break;
        case 2: p.tau = -1.0; break;
        case 3: p.kappa[0] = NAN; break;
        case 4: p.hi[0] = p.lo[0]; break;
        case 5: p.precision = 9; break;
        case 6: p.pade = 3; break;
        default: p.rxn = ETD_RXN_FHN_CUBIC; break;   // ncomp 1 with a two-component reaction
        }
        Plan pl;
        std::string err;
        if (build_plan(p, pl, err) != ETD_EINVAL || err.empty()) {
            std::fprintf(stderr, "malformed case %d accepted\n", k);
            bad = 1;
        }
    }
    std::printf("plan sanitizer driver: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
