/*
 * CPU oracle for the Pade-based dimension-split ETD2RK scheme (ETD2RK-DS).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  Plain C99, FP64.
 *
 * What it computes, in the paper's order:
 *   - the finite-difference operator of Sec. 2.1: per direction
 *     A_d = h_d^-2 tridiag(-kappa, 2 kappa + q h_d^2 / dim, -kappa);
 *   - the rational functions of Sec. 3.1 through their partial fractions
 *     Q_l(x) = 2 Re( sum_k r_{l,k} (x - s_k)^-1 ),
 *     P_{0,2}: one pole s = -1 + i, r = (-i, (1-i)/2, 1/2);
 *     P_{0,4} (Sec. 5): the two upper-half-plane roots of
 *     x^4 + 4x^3 + 12x^2 + 24x + 24 with residues N_l(s)/den'(s);
 *   - each shifted 1-D system (tau A_d - s I) v = r g of Sec. 3.2 solved by
 *     the Thomas algorithm on every grid line along d, the factorisation being
 *     computed once and reused (Sec. 3.3.1);
 *   - one step of the scheme (Sec. 3.1, 2-D and 3-D forms; Algorithms 1-2):
 *       F0 = f(t_n, U)
 *       3-D: w1 = Q1(tau A_z) U,  w2 = Q1(tau A_z) F0
 *            w3 = Q1(tau A_y) w1, w4 = Q1(tau A_y) w2
 *       2-D: w3 = Q1(tau A_y) U,  w4 = Q1(tau A_y) F0
 *       W  = Q1(tau A_x) w3 + tau Q2(tau A_x) w4
 *       F1 = f(t_{n+1}, W)
 *       U+ = W + tau Q3(tau A_x) (F1 - w4)
 *     The factor tau on the Q3 term follows the scheme's equations; the
 *     algorithm listings drop it, which the equations and the printed error
 *     tables contradict.
 */
#include "etdo.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Working precision.  The oracle is FP64.  Built with -DETDO_EXTENDED the
 * same source runs in x87 extended precision (64-bit significand); that build
 * only referees how much of a difference between two FP64 results is FP64
 * rounding.  The public entry points take and return doubles either way. */
#ifdef ETDO_EXTENDED
typedef long double real;
typedef long double complex cplx;
#define R_SIN sinl
#define R_EXP expl
#define R_CREAL creall
#define R_CIMAG cimagl
#define R_PI 3.141592653589793238462643383279502884L
#else
typedef double real;
typedef double complex cplx;
#define R_SIN sin
#define R_EXP exp
#define R_CREAL creal
#define R_CIMAG cimag
#define R_PI M_PI
#endif

/* ------------------------------------------------------------------------ */
/* Rational families: poles and residues                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int np;          /* number of poles in the upper half plane */
    cplx s[2];       /* poles */
    cplx r[3][2];    /* r[l-1][k]: residue of Q_l (or R_l) at pole k */
} rational_family;

static cplx poly_eval(const real* c, int deg, cplx x) {
    /* c[0] x^deg + ... + c[deg] */
    cplx v = c[0];
    for (int i = 1; i <= deg; ++i) v = v * x + c[i];
    return v;
}

/* Roots of a monic real quartic by the Weierstrass (Durand-Kerner) iteration. */
static void quartic_roots(const real* c, cplx roots[4]) {
    cplx z[4];
    const cplx seed = 0.4 + 0.9 * I;
    z[0] = 1.0;
    for (int k = 1; k < 4; ++k) z[k] = z[k - 1] * seed;
    for (int it = 0; it < 500; ++it) {
        for (int k = 0; k < 4; ++k) {
            cplx den = 1.0;
            for (int j = 0; j < 4; ++j)
                if (j != k) den *= (z[k] - z[j]);
            z[k] -= poly_eval(c, 4, z[k]) / den;
        }
    }
    for (int k = 0; k < 4; ++k) roots[k] = z[k];
}

static void make_family(int pade, rational_family* f) {
    memset(f, 0, sizeof(*f));
    if (pade == 4) {
        /* R_1 = 24/den, R_2 = (x^3+4x^2+12x+24)/den, R_3 = (x^3+3x^2+8x+12)/den */
        const real den[5] = {1.0, 4.0, 12.0, 24.0, 24.0};
        const real dden[4] = {4.0, 12.0, 24.0, 24.0};
        const real num[3][4] = {{0.0, 0.0, 0.0, 24.0},
                                  {1.0, 4.0, 12.0, 24.0},
                                  {1.0, 3.0, 8.0, 12.0}};
        cplx roots[4];
        quartic_roots(den, roots);
        int k = 0;
        for (int j = 0; j < 4 && k < 2; ++j)
            if (R_CIMAG(roots[j]) > 0.0) f->s[k++] = roots[j];
        f->np = 2;
        for (int l = 0; l < 3; ++l)
            for (int kk = 0; kk < 2; ++kk)
                f->r[l][kk] = poly_eval(num[l], 3, f->s[kk]) / poly_eval(dden, 3, f->s[kk]);
    } else {
        f->np = 1;
        f->s[0] = -1.0 + 1.0 * I;
        f->r[0][0] = -1.0 * I;
        f->r[1][0] = 0.5 - 0.5 * I;
        f->r[2][0] = 0.5;
    }
}

int etdo_poles(int pade, double* out_s, double* out_r) {
    rational_family f;
    make_family(pade, &f);
    for (int k = 0; k < f.np; ++k) {
        out_s[2 * k] = (double)R_CREAL(f.s[k]);
        out_s[2 * k + 1] = (double)R_CIMAG(f.s[k]);
    }
    for (int l = 0; l < 3; ++l)
        for (int k = 0; k < f.np; ++k) {
            out_r[2 * (l * f.np + k)] = (double)R_CREAL(f.r[l][k]);
            out_r[2 * (l * f.np + k) + 1] = (double)R_CIMAG(f.r[l][k]);
        }
    return f.np;
}

/* ------------------------------------------------------------------------ */
/* Thomas factorisation of tau A_d - s I                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int len;
    cplx off;       /* off-diagonal entry of tau A_d - s I */
    cplx* cp;       /* modified super-diagonal */
    cplx* inv;      /* inverse pivots */
} thomas_factor;

static void thomas_setup(thomas_factor* t, int len, real diag_real, real off_real, cplx s) {
    const cplx a = diag_real - s;
    const cplx b = off_real;
    t->len = len;
    t->off = b;
    t->cp = (cplx*)malloc(sizeof(cplx) * (size_t)len);
    t->inv = (cplx*)malloc(sizeof(cplx) * (size_t)len);
    cplx piv = a;
    t->inv[0] = 1.0 / piv;
    t->cp[0] = b * t->inv[0];
    for (int i = 1; i < len; ++i) {
        piv = a - b * t->cp[i - 1];
        t->inv[i] = 1.0 / piv;
        t->cp[i] = b * t->inv[i];
    }
}

static void thomas_free(thomas_factor* t) {
    free(t->cp);
    free(t->inv);
}

/* Solve in place: y holds the right-hand side on entry, the solution on exit. */
static void thomas_solve(const thomas_factor* t, cplx* y) {
    const int n = t->len;
    y[0] = y[0] * t->inv[0];
    for (int i = 1; i < n; ++i) y[i] = (y[i] - t->off * y[i - 1]) * t->inv[i];
    for (int i = n - 2; i >= 0; --i) y[i] -= t->cp[i] * y[i + 1];
}

/* ------------------------------------------------------------------------ */
/* Context: problem geometry and the reusable factorisations                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    const etdo_problem* p;
    int nx, ny, nz;
    size_t npts;                       /* points per component */
    rational_family fam;
    thomas_factor fac[3][2][2];        /* [direction][component][pole] */
    int nthreads;
} ctx;

static int check_problem(const etdo_problem* p) {
    if (!p) return -1;
    if (p->dim != 2 && p->dim != 3) return -1;
    if (p->ncomp != 1 && p->ncomp != 2) return -1;
    for (int d = 0; d < p->dim; ++d) {
        if (p->n[d] < 1) return -1;
        if (!(p->hi[d] > p->lo[d])) return -1;
    }
    for (int c = 0; c < p->ncomp; ++c)
        if (!(p->kappa[c] >= 0.0)) return -1;
    if (!(p->q >= 0.0) || !(p->tau > 0.0)) return -1;
    if (p->pade != 2 && p->pade != 4) return -1;
    const int two = (p->rxn == ETDO_RXN_FHN_CUBIC || p->rxn == ETDO_RXN_FHN_CLASSIC);
    if (two != (p->ncomp == 2)) return -1;
    if (p->rxn < ETDO_RXN_NONE || p->rxn > ETDO_RXN_FHN_CLASSIC) return -1;
    return 0;
}

static int ctx_init(ctx* c, const etdo_problem* p, int nthreads) {
    if (check_problem(p)) return -1;
    memset(c, 0, sizeof(*c));
    c->p = p;
    c->nx = p->n[0];
    c->ny = p->n[1];
    c->nz = p->dim == 3 ? p->n[2] : 1;
    c->npts = (size_t)c->nx * c->ny * c->nz;
    c->nthreads = etdo_threads(nthreads);
    make_family(p->pade, &c->fam);
    for (int d = 0; d < p->dim; ++d) {
        const real h = ((real)p->hi[d] - (real)p->lo[d]) / (p->n[d] + 1);
        for (int cc = 0; cc < p->ncomp; ++cc) {
            const real k = p->kappa[cc];
            /* tau * h^-2 * (2 kappa + q h^2/dim) on the diagonal, -tau kappa h^-2 off it */
            const real diag = (real)p->tau * (2.0 * k / (h * h) + (real)p->q / p->dim);
            const real off = -(real)p->tau * k / (h * h);
            for (int kp = 0; kp < c->fam.np; ++kp)
                thomas_setup(&c->fac[d][cc][kp], p->n[d], diag, off, c->fam.s[kp]);
        }
    }
    return 0;
}

static void ctx_free(ctx* c) {
    for (int d = 0; d < c->p->dim; ++d)
        for (int cc = 0; cc < c->p->ncomp; ++cc)
            for (int kp = 0; kp < c->fam.np; ++kp) thomas_free(&c->fac[d][cc][kp]);
}

int etdo_threads(int nthreads) {
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Line sweeps                                                               */
/* ------------------------------------------------------------------------ */

/* Lines along direction d: their count, length, element stride and the
 * offset of line number L. */
static void line_geometry(const ctx* c, int d, size_t* nlines, int* len, size_t* stride) {
    if (d == 0) {
        *len = c->nx; *stride = 1; *nlines = (size_t)c->ny * c->nz;
    } else if (d == 1) {
        *len = c->ny; *stride = (size_t)c->nx; *nlines = (size_t)c->nx * c->nz;
    } else {
        *len = c->nz; *stride = (size_t)c->nx * c->ny; *nlines = (size_t)c->nx * c->ny;
    }
}

static size_t line_offset(const ctx* c, int d, size_t L) {
    if (d == 0) return L * (size_t)c->nx;
    if (d == 1) {
        const size_t z = L / c->nx, x = L % c->nx;
        return z * (size_t)c->nx * c->ny + x;
    }
    return L; /* d == 2: L = y*nx + x */
}

/* out = sum_k 2 Re( (tau A_d - s_k)^-1 (alpha_k g1 + beta_k g2) ) along d for
 * one component (g2 may be NULL). */
static void apply_dir(const ctx* c, int d, int comp, const cplx* alpha, const real* g1,
                      const cplx* beta, const real* g2, real* out) {
    size_t nlines, stride;
    int len;
    line_geometry(c, d, &nlines, &len, &stride);
    const int np = c->fam.np;
#ifdef _OPENMP
#pragma omp parallel num_threads(c->nthreads)
#endif
    {
        cplx* y = (cplx*)malloc(sizeof(cplx) * (size_t)len);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (size_t L = 0; L < nlines; ++L) {
            const size_t base = line_offset(c, d, L);
            for (int i = 0; i < len; ++i) out[base + i * stride] = 0.0;
            for (int k = 0; k < np; ++k) {
                for (int i = 0; i < len; ++i) {
                    cplx rhs = alpha[k] * g1[base + i * stride];
                    if (g2) rhs += beta[k] * g2[base + i * stride];
                    y[i] = rhs;
                }
                thomas_solve(&c->fac[d][comp][k], y);
                for (int i = 0; i < len; ++i) out[base + i * stride] += 2.0 * R_CREAL(y[i]);
            }
        }
        free(y);
    }
}

/* out = Q_ell(tau A_d) g for one component */
static void apply_q(const ctx* c, int ell, int d, int comp, const real* g, real* out) {
    apply_dir(c, d, comp, c->fam.r[ell - 1], g, NULL, NULL, out);
}

/* ------------------------------------------------------------------------ */
/* Reactions                                                                 */
/* ------------------------------------------------------------------------ */

static real node(const etdo_problem* p, int d, int i) {
    const real h = ((real)p->hi[d] - (real)p->lo[d]) / (p->n[d] + 1);
    return p->lo[d] + (i + 1) * h;
}

static int reaction(const etdo_problem* p, real t, const real* u, real* f) {
    if (check_problem(p)) return -1;
    const int nx = p->n[0], ny = p->n[1], nz = p->dim == 3 ? p->n[2] : 1;
    const size_t np = (size_t)nx * ny * nz;
    real a[8];
    for (int i = 0; i < 8; ++i) a[i] = p->rxn_param[i];
    switch (p->rxn) {
    case ETDO_RXN_NONE:
        for (size_t i = 0; i < np; ++i) f[i] = 0.0;
        break;
    case ETDO_RXN_LINEAR:
        for (size_t i = 0; i < np; ++i) f[i] = a[0] * u[i];
        break;
    case ETDO_RXN_FISHER:
        for (size_t i = 0; i < np; ++i) f[i] = a[0] * u[i] * (1.0 - u[i]);
        break;
    case ETDO_RXN_ALLEN_CAHN:
        for (size_t i = 0; i < np; ++i) f[i] = u[i] - u[i] * u[i] * u[i];
        break;
    case ETDO_RXN_SATURATING:
        for (size_t i = 0; i < np; ++i) f[i] = a[0] * u[i] / (1.0 - u[i]);
        break;
    case ETDO_RXN_AC_MMS: {
        /* exact solution ue = e^{-lam t} prod_d sin(pi (x_d-lo_d)/L_d); psi makes
         * u_t - kappa Lap u + q u = u(1-u^2) + psi hold for it (Example 5.1). */
        const real lam = a[0];
        real mu = 0.0;
        for (int d = 0; d < p->dim; ++d) {
            const real L = (real)p->hi[d] - (real)p->lo[d];
            if (a[1] != 0.0) {
                const real h = L / (p->n[d] + 1);
                const real sn = R_SIN(R_PI * h / (2.0 * L));
                mu += 4.0 / (h * h) * sn * sn;
            } else {
                mu += (R_PI / L) * (R_PI / L);
            }
        }
        const real rate = -lam + (real)p->kappa[0] * mu + (real)p->q;
        const real et = R_EXP(-lam * t);
        for (int z = 0; z < nz; ++z) {
            const real sz = p->dim == 3 ? R_SIN(R_PI * (node(p, 2, z) - p->lo[2]) / ((real)p->hi[2] - p->lo[2])) : 1.0;
            for (int y = 0; y < ny; ++y) {
                const real sy = R_SIN(R_PI * (node(p, 1, y) - p->lo[1]) / ((real)p->hi[1] - p->lo[1]));
                for (int x = 0; x < nx; ++x) {
                    const real sx = R_SIN(R_PI * (node(p, 0, x) - p->lo[0]) / ((real)p->hi[0] - p->lo[0]));
                    const size_t i = ((size_t)z * ny + y) * nx + x;
                    const real ue = et * sx * sy * sz;
                    const real psi = rate * ue - ue * (1.0 - ue * ue);
                    f[i] = u[i] * (1.0 - u[i] * u[i]) + psi;
                }
            }
        }
        break;
    }
    case ETDO_RXN_FHN_CUBIC: {
        const real* uu = u;
        const real* vv = u + np;
        for (size_t i = 0; i < np; ++i) {
            f[i] = uu[i] * (1.0 - uu[i]) * (uu[i] - a[0]) - vv[i];
            f[np + i] = a[1] * (uu[i] - a[2] * vv[i]);
        }
        break;
    }
    case ETDO_RXN_FHN_CLASSIC: {
        const real* uu = u;
        const real* vv = u + np;
        for (size_t i = 0; i < np; ++i) {
            f[i] = uu[i] - uu[i] * uu[i] * uu[i] / 3.0 - vv[i];
            f[np + i] = a[0] * (uu[i] - a[1] * vv[i]);
        }
        break;
    }
    default:
        return -1;
    }
    return 0;
}

/* Field conversions between the public FP64 arrays and the working precision. */
static real* to_real(const double* x, size_t n) {
    real* r = (real*)malloc(sizeof(real) * n);
    for (size_t i = 0; i < n; ++i) r[i] = x[i];
    return r;
}

static void from_real(const real* r, double* x, size_t n) {
    for (size_t i = 0; i < n; ++i) x[i] = (double)r[i];
}

static size_t field_size(const etdo_problem* p) {
    return (size_t)p->n[0] * p->n[1] * (p->dim == 3 ? p->n[2] : 1) * p->ncomp;
}

int etdo_reaction(const etdo_problem* p, double t, const double* u, double* f) {
    if (check_problem(p)) return -1;
    const size_t n = field_size(p);
    real* ur = to_real(u, n);
    real* fr = (real*)malloc(sizeof(real) * n);
    const int rc = reaction(p, t, ur, fr);
    from_real(fr, f, n);
    free(ur);
    free(fr);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Public entry points                                                       */
/* ------------------------------------------------------------------------ */

int etdo_apply(const etdo_problem* p, int ell, int d, int comp, const double* g, double* out,
               int nthreads) {
    ctx c;
    if (ell < 1 || ell > 3 || !p || d < 0 || d >= p->dim || comp < 0 || comp >= p->ncomp)
        return -1;
    if (ctx_init(&c, p, nthreads)) return -1;
    const size_t n = c.npts;
    real* gr = to_real(g + (size_t)comp * n, n);
    real* orr = (real*)malloc(sizeof(real) * n);
    apply_q(&c, ell, d, comp, gr, orr);
    from_real(orr, out + (size_t)comp * n, n);
    free(gr);
    free(orr);
    ctx_free(&c);
    return 0;
}

int etdo_advance(const etdo_problem* p, double* u_io, double t0, int nsteps, int nthreads) {
    ctx c;
    if (nsteps < 0) return -1;
    if (ctx_init(&c, p, nthreads)) return -1;
    const size_t N = c.npts * p->ncomp;
    const real tau = p->tau;
    real* u = to_real(u_io, N);
    real* F0 = (real*)malloc(sizeof(real) * N);
    real* wa = (real*)malloc(sizeof(real) * N);  /* w1, then w3 */
    real* wb = (real*)malloc(sizeof(real) * N);  /* w2, then w4 */
    real* tmp = (real*)malloc(sizeof(real) * N);
    real* W = (real*)malloc(sizeof(real) * N);
    real* F1 = (real*)malloc(sizeof(real) * N);
    const cplx* r1 = c.fam.r[0];
    const cplx* r3 = c.fam.r[2];
    cplx tr2[2], tr3[2];
    for (int k = 0; k < c.fam.np; ++k) {
        tr2[k] = tau * c.fam.r[1][k];
        tr3[k] = tau * r3[k];
    }

    for (int step = 0; step < nsteps; ++step) {
        const real tn = (real)t0 + step * tau;
        const real tn1 = (real)t0 + (step + 1) * tau;
        reaction(p, tn, u, F0);
        for (int cc = 0; cc < p->ncomp; ++cc) {
            const size_t o = (size_t)cc * c.npts;
            if (p->dim == 3) {
                /* z-lines, then y-lines (Algorithm 2, steps 3.1-3.4) */
                apply_dir(&c, 2, cc, r1, u + o, NULL, NULL, tmp + o);
                apply_dir(&c, 1, cc, r1, tmp + o, NULL, NULL, wa + o);
                apply_dir(&c, 2, cc, r1, F0 + o, NULL, NULL, tmp + o);
                apply_dir(&c, 1, cc, r1, tmp + o, NULL, NULL, wb + o);
            } else {
                /* y-lines (Algorithm 1, steps 3.1-3.2) */
                apply_dir(&c, 1, cc, r1, u + o, NULL, NULL, wa + o);
                apply_dir(&c, 1, cc, r1, F0 + o, NULL, NULL, wb + o);
            }
            /* x-lines: W = Q1 w3 + tau Q2 w4, one solve per pole */
            apply_dir(&c, 0, cc, r1, wa + o, tr2, wb + o, W + o);
        }
        reaction(p, tn1, W, F1);
        for (size_t i = 0; i < N; ++i) tmp[i] = F1[i] - wb[i];
        for (int cc = 0; cc < p->ncomp; ++cc) {
            const size_t o = (size_t)cc * c.npts;
            apply_dir(&c, 0, cc, tr3, tmp + o, NULL, NULL, F1 + o);
        }
        for (size_t i = 0; i < N; ++i) u[i] = W[i] + F1[i];
    }
    from_real(u, u_io, N);

    free(u); free(F0); free(wa); free(wb); free(tmp); free(W); free(F1);
    ctx_free(&c);
    return 0;
}
