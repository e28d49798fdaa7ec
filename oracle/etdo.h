/*
 * CPU oracle for the Pade-based dimension-split ETD2RK scheme (ETD2RK-DS).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain FP64 reference
 * that the GPU path is checked against.  Only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the product path never
 * does.  It shares no source with the GPU library.
 *
 * Method (paper Sec. 3.1-3.3): each rational operator Q_l(tau*A_d) is applied
 * through its partial-fraction form 2 Re( r_l (tau*A_d - s I)^{-1} g ), the
 * shifted tridiagonal systems being solved line by line with the Thomas
 * algorithm (Sec. 3.3.1: one factorisation per direction and component,
 * reused for every line and every step).
 *
 * Layout: a field is ncomp x nz x ny x nx doubles, x fastest (Sec. 2.1),
 * with nz = 1 in 2-D.  n[d] counts interior points, h_d = (hi-lo)/(n_d+1).
 */
#ifndef ETDO_H
#define ETDO_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ETDO_RXN_NONE = 0,
    ETDO_RXN_LINEAR = 1,       /* f = c u                              p0 = c          */
    ETDO_RXN_FISHER = 2,       /* f = a u (1-u)                        p0 = a          */
    ETDO_RXN_ALLEN_CAHN = 3,   /* f = u - u^3                                          */
    ETDO_RXN_AC_MMS = 4,       /* f = u(1-u^2) + psi(x,t)              p0 = lambda,
                                  p1 = 1 uses the discrete Laplacian eigenvalue in psi */
    ETDO_RXN_SATURATING = 5,   /* f = rho u/(1-u)                      p0 = rho        */
    ETDO_RXN_FHN_CUBIC = 6,    /* fu = u(1-u)(u-a) - v, fv = eps(u - g v)  p = a,eps,g */
    ETDO_RXN_FHN_CLASSIC = 7   /* fu = u - u^3/3 - v, fv = eps(u - alpha v) p = eps,alpha */
};

typedef struct {
    int dim;              /* 2 or 3 */
    int n[3];             /* interior points per direction x, y, z */
    double lo[3], hi[3];  /* box */
    int ncomp;            /* 1 or 2 */
    double kappa[2];      /* diffusivity per component (>= 0) */
    double q;             /* potential >= 0, split q/dim per direction */
    double tau;           /* time step */
    int rxn;              /* ETDO_RXN_* */
    double rxn_param[8];
    int pade;             /* 2: P_{0,2} rational family; 4: P_{0,4} family */
} etdo_problem;

/* Advance u (host, ncomp*nz*ny*nx doubles, in place) by nsteps steps of size
 * tau from time t0.  nthreads <= 0 means "all available".  Returns 0 on
 * success, a negative value on invalid arguments. */
int etdo_advance(const etdo_problem* p, double* u, double t0, int nsteps, int nthreads);

/* out = Q_ell(tau A_d) g for component comp, ell in {1,2,3}, d in {0,1,2}. */
int etdo_apply(const etdo_problem* p, int ell, int d, int comp, const double* g,
               double* out, int nthreads);

/* f evaluated at time t: out has the same shape as u. */
int etdo_reaction(const etdo_problem* p, double t, const double* u, double* out);

/* Poles and residues of the rational family in use: for pade = 2 one pole,
 * for pade = 4 two poles (upper half plane).  out_s: 2*npoles doubles (re,im);
 * out_r: 3*2*npoles doubles, residue of family member ell, pole k at
 * [(ell-1)*npoles + k]*2.  Returns npoles. */
int etdo_poles(int pade, double* out_s, double* out_r);

/* Number of threads the OpenMP runtime would use for nthreads (<= 0: all). */
int etdo_threads(int nthreads);

#ifdef __cplusplus
}
#endif
#endif
