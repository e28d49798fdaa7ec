/* Host driver for the sanitizer build of the CPU oracle (oracle/etdo.c):
 * runs every entry point on small 2-D and 3-D problems (every reaction, both
 * rational families, extents down to one interior point) and checks the
 * results are finite.  Exit status 0 on success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "etdo.h"

static int check_finite(const double* u, long n, const char* what) {
    for (long i = 0; i < n; ++i)
        if (!isfinite(u[i])) {
            fprintf(stderr, "%s: non-finite value at %ld\n", what, i);
            return 1;
        }
    return 0;
}

int main(void) {
    const int dims[][4] = {{2, 7, 5, 1}, {2, 1, 9, 1}, {2, 12, 1, 1}, {3, 5, 4, 3}, {3, 1, 1, 1}, {3, 2, 6, 9}};
    int bad = 0;
    for (size_t c = 0; c < sizeof(dims) / sizeof(dims[0]); ++c)
        for (int rxn = ETDO_RXN_NONE; rxn <= ETDO_RXN_FHN_CLASSIC; ++rxn)
            for (int pade = 2; pade <= 4; pade += 2) {
                etdo_problem p;
                memset(&p, 0, sizeof(p));
                p.dim = dims[c][0];
                for (int d = 0; d < 3; ++d) {
                    p.n[d] = d < p.dim ? dims[c][d + 1] : 1;
                    p.lo[d] = 0.1 * d;
                    p.hi[d] = 1.0 + 0.2 * d;
                }
                p.ncomp = rxn >= ETDO_RXN_FHN_CUBIC ? 2 : 1;
                p.kappa[0] = 0.3;
                p.kappa[1] = 0.05;
                p.q = 0.4;
                p.tau = 0.01;
                p.rxn = rxn;
                p.rxn_param[0] = rxn == ETDO_RXN_SATURATING ? 0.1 : (rxn == ETDO_RXN_FHN_CLASSIC ? 1.0 : 0.5);
                p.rxn_param[1] = rxn == ETDO_RXN_AC_MMS ? 1.0 : 0.01;
                p.rxn_param[2] = 0.5;
                p.pade = pade;
                const long npt = (long)p.ncomp * p.n[0] * p.n[1] * p.n[2];
                double* u = malloc(sizeof(double) * npt);
                double* g = malloc(sizeof(double) * npt);
                for (long i = 0; i < npt; ++i) u[i] = 0.25 + 0.5 * sin(0.37 * (double)i);
                if (etdo_advance(&p, u, 0.0, 3, 1) != 0) {
                    fprintf(stderr, "advance rejected case %zu rxn %d pade %d\n", c, rxn, pade);
                    bad = 1;
                }
                bad |= check_finite(u, npt, "advance");
                for (int d = 0; d < p.dim; ++d)
                    for (int ell = 1; ell <= 3; ++ell) {
                        if (etdo_apply(&p, ell, d, p.ncomp - 1, u, g, 1) != 0) bad = 1;
                        bad |= check_finite(g, npt, "apply");
                    }
                if (etdo_reaction(&p, 0.5, u, g) != 0) bad = 1;
                bad |= check_finite(g, npt, "reaction");
                free(u);
                free(g);
            }
    double s[4], r[12];
    if (etdo_poles(2, s, r) < 1 || etdo_poles(4, s, r) < 1) bad = 1;
    printf("oracle sanitizer driver: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
