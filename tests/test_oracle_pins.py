"""Pins of the CPU oracle against closed forms, special cases and brute force.

None of these re-use the oracle's arithmetic: the rational functions are
evaluated from their polynomial definitions (Sec. 3.1 and Sec. 5) rather than
from partial fractions, the eigenpairs are the textbook sine-transform ones,
and the dense checks build the full Kronecker operators of Sec. 2.1 and apply
the scheme's equations (Sec. 3.1) with dense solves, without any slicing.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import workloads as W

# ---------------------------------------------------------------------------
# rational functions from their polynomial definitions
# ---------------------------------------------------------------------------


def q_scalar(pade, ell, x):
    x = np.asarray(x, dtype=np.float64)
    if pade == 2:
        den = x * x + 2 * x + 2
        num = {1: 2.0 + 0 * x, 2: x + 2, 3: x + 1}[ell]
    else:
        den = x ** 4 + 4 * x ** 3 + 12 * x ** 2 + 24 * x + 24
        num = {1: 24.0 + 0 * x, 2: x ** 3 + 4 * x ** 2 + 12 * x + 24, 3: x ** 3 + 3 * x ** 2 + 8 * x + 12}[ell]
    return num / den


def q_matrix(pade, ell, M):
    """Q_ell(M) = den(M)^{-1} num(M) for a dense symmetric M."""
    I = np.eye(M.shape[0])
    M2 = M @ M
    if pade == 2:
        den = M2 + 2 * M + 2 * I
        num = {1: 2 * I, 2: M + 2 * I, 3: M + I}[ell]
    else:
        M3 = M2 @ M
        M4 = M3 @ M
        den = M4 + 4 * M3 + 12 * M2 + 24 * M + 24 * I
        num = {1: 24 * I, 2: M3 + 4 * M2 + 12 * M + 24 * I, 3: M3 + 3 * M2 + 8 * M + 12 * I}[ell]
    return np.linalg.solve(den, num)


def stencil(p, d, c=0):
    """A_d = h^-2 tridiag(-kappa, 2 kappa + q h^2/dim, -kappa) (Sec. 2.1)."""
    n = p.n[d]
    h = p.h(d)
    k = p.kappa[c]
    A = np.zeros((n, n))
    i = np.arange(n)
    A[i, i] = (2 * k + p.q * h * h / p.dim) / (h * h)
    A[i[:-1], i[:-1] + 1] = -k / (h * h)
    A[i[:-1] + 1, i[:-1]] = -k / (h * h)
    return A


def split_ops(p, c=0):
    """Dense A_1 (x direction) and the other directional operators, acting on
    the x-fastest vectorisation (Sec. 2.1 and Sec. 2.2)."""
    Ix = np.eye(p.n[0])
    Iy = np.eye(p.n[1])
    Ax = stencil(p, 0, c)
    Ay = stencil(p, 1, c)
    if p.dim == 2:
        return np.kron(Iy, Ax), [np.kron(Ay, Ix)]
    Iz = np.eye(p.n[2])
    Az = stencil(p, 2, c)
    A1 = np.kron(Iz, np.kron(Iy, Ax))
    A2y = np.kron(Iz, np.kron(Ay, Ix))
    A2z = np.kron(Az, np.kron(Iy, Ix))
    return A1, [A2y, A2z]


def dense_reaction(p, t, u):
    a = p.params
    if p.reaction == "none":
        return np.zeros_like(u)
    if p.reaction == "linear":
        return a[0] * u
    if p.reaction == "fisher":
        return a[0] * u * (1 - u)
    if p.reaction == "allen_cahn":
        return u - u ** 3
    if p.reaction == "saturating":
        return a[0] * u / (1 - u)
    if p.reaction == "fhn_cubic":
        uu, vv = u[0], u[1]
        return np.stack([uu * (1 - uu) * (uu - a[0]) - vv, a[1] * (uu - a[2] * vv)])
    if p.reaction == "fhn_classic":
        uu, vv = u[0], u[1]
        return np.stack([uu - uu ** 3 / 3 - vv, a[0] * (uu - a[1] * vv)])
    raise NotImplementedError(p.reaction)


def dense_step(p, u, t):
    """One step of the Pade ETD2RK-DS scheme in the unsliced Kronecker form of
    Sec. 3.1 (2-D and 3-D equations), per component."""
    tau = p.tau
    F0 = dense_reaction(p, t, u)
    W_ = np.empty_like(u)
    w2 = np.empty_like(u)
    for c in range(p.ncomp):
        A1, rest = split_ops(p, c)
        Q1r = np.eye(A1.shape[0])
        for A in rest:
            Q1r = Q1r @ q_matrix(p.pade, 1, tau * A)
        uc = u[c].reshape(-1)
        fc = F0[c].reshape(-1)
        w = q_matrix(p.pade, 1, tau * A1) @ (Q1r @ uc) + tau * q_matrix(p.pade, 2, tau * A1) @ (Q1r @ fc)
        W_[c] = w.reshape(u[c].shape)
        w2[c] = (Q1r @ fc).reshape(u[c].shape)
    F1 = dense_reaction(p, t + tau, W_)
    out = np.empty_like(u)
    for c in range(p.ncomp):
        A1, _ = split_ops(p, c)
        corr = tau * q_matrix(p.pade, 3, tau * A1) @ (F1[c] - w2[c]).reshape(-1)
        out[c] = W_[c] + corr.reshape(u[c].shape)
    return out


def sine_mode(p, js):
    """Joint eigenvector prod_d sin(j_d pi i_d/(n_d+1)) of every A_d."""
    vecs = [np.sin(js[d] * math.pi * np.arange(1, p.n[d] + 1) / (p.n[d] + 1)) for d in range(p.dim)]
    if p.dim == 2:
        return np.outer(vecs[1], vecs[0])[None]
    return np.einsum("k,j,i->kji", vecs[2], vecs[1], vecs[0])[None]


def eig1d(p, d, j, c=0):
    """lambda_j = kappa (4/h^2) sin^2(j pi/(2(n+1))) + q/dim: the closed-form
    eigenvalue of A_d for the sine eigenvector with index j."""
    h = p.h(d)
    return p.kappa[c] * 4 / (h * h) * math.sin(j * math.pi / (2 * (p.n[d] + 1))) ** 2 + p.q / p.dim


# ---------------------------------------------------------------------------
# P1: closed-form eigenpairs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("pade", [2, 4])
@pytest.mark.parametrize("dim", [2, 3])
def test_apply_on_eigenvector(oracle_mod, pade, dim):
    n = (13, 9) if dim == 2 else (11, 7, 6)
    p = W.Problem(dim=dim, n=n, kappa=(0.37,), q=0.8, tau=0.013, reaction="none", pade=pade,
                  lo=(0.2, -1.0, 0.5), hi=(1.1, 0.5, 1.75))
    rng = np.random.default_rng(1)
    for trial in range(4):
        js = [int(rng.integers(1, p.n[d] + 1)) for d in range(dim)]
        g = sine_mode(p, js)
        for d in range(dim):
            for ell in (1, 2, 3):
                got = oracle_mod.apply(p, ell, d, g)
                want = q_scalar(pade, ell, p.tau * eig1d(p, d, js[d])) * g
                assert np.abs(got - want).max() <= 1e-13 * np.abs(g).max(), (d, ell, js)


def test_apply_second_component_uses_its_kappa(oracle_mod):
    p = W.Problem(dim=2, n=(10, 12), kappa=(0.05, 2.5), q=0.3, tau=0.02, reaction="fhn_cubic")
    g1 = sine_mode(p, (3, 5))[0]
    g = np.stack([0 * g1, g1])
    got = oracle_mod.apply(p, 1, 1, g, comp=1)
    want = q_scalar(2, 1, p.tau * eig1d(p, 1, 5, c=1)) * g1
    assert np.abs(got[1] - want).max() <= 1e-13
    assert np.abs(got[0]).max() == 0.0


@pytest.mark.parametrize("pade", [2, 4])
def test_partial_fractions_match_rational_functions(oracle_mod, pade):
    s, r = oracle_mod.poles(pade)
    # the poles are the roots of the denominator polynomial
    den = [1, 2, 2] if pade == 2 else [1, 4, 12, 24, 24]
    roots = np.roots(den)
    for sk in s:
        assert np.min(np.abs(roots - sk)) < 1e-12
        assert sk.imag > 0
    x = np.linspace(0.0, 50.0, 201)
    for ell in (1, 2, 3):
        pf = sum(2 * np.real(r[ell - 1, k] / (x - s[k])) for k in range(len(s)))
        assert np.allclose(pf, q_scalar(pade, ell, x), rtol=1e-13, atol=1e-15)


def test_rational_family_invariants():
    """0 < Q1 <= 1, 0 < Q2 <= 1, 0 < Q3 <= 1/2 for x >= 0 (P_{0,2}), consistent
    with the bounds used in Proposition 4.3, and Q_l(0) = phi_l(0)."""
    x = np.concatenate([np.linspace(0, 10, 1001), np.logspace(1, 8, 50)])
    for pade in (2, 4):
        q1, q2, q3 = (q_scalar(pade, l, x) for l in (1, 2, 3))
        assert np.all(q1 > 0) and np.all(q1 <= 1)
        assert np.all(q2 > 0) and np.all(q2 <= 1 + 1e-15)
        assert np.all(q3 > 0) and np.all(q3 <= 0.5 + 1e-15)
        assert q1[0] == 1 and q2[0] == 1 and q3[0] == 0.5
        # third-order agreement with exp(-x) near 0 for the P_{0,2} family
    xs = np.array([1e-2, 5e-3])
    err = np.abs(np.exp(-xs) - q_scalar(2, 1, xs))
    assert 7.5 < err[0] / err[1] < 8.5


# ---------------------------------------------------------------------------
# P5: brute force with dense Kronecker operators
# ---------------------------------------------------------------------------

DENSE_CASES = [
    dict(dim=2, n=(5, 7), kappa=(0.3,), q=0.6, tau=0.05, reaction="fisher", rxn_param=(1.3,)),
    dict(dim=2, n=(6, 4), kappa=(0.02, 0.9), q=0.1, tau=0.1, reaction="fhn_cubic"),
    dict(dim=2, n=(6, 5), kappa=(0.5, 0.1), q=0.0, tau=0.08, reaction="fhn_classic", rxn_param=(0.7, 1.4)),
    dict(dim=2, n=(7, 5), kappa=(1.0,), q=1.0, tau=0.03, reaction="saturating", rxn_param=(0.1,)),
    dict(dim=3, n=(3, 4, 5), kappa=(0.2,), q=0.9, tau=0.04, reaction="fisher"),
    dict(dim=3, n=(4, 3, 3), kappa=(0.05, 0.4), q=0.2, tau=0.06, reaction="fhn_cubic"),
    dict(dim=3, n=(4, 4, 3), kappa=(0.7,), q=0.0, tau=0.02, reaction="allen_cahn", pade=4),
    dict(dim=2, n=(5, 6), kappa=(0.4,), q=0.3, tau=0.07, reaction="fisher", pade=4),
]


@pytest.mark.parametrize("case", DENSE_CASES, ids=lambda c: f"{c['dim']}d-{c['reaction']}-p{c.get('pade', 2)}")
def test_dense_brute_force(oracle_mod, case):
    p = W.Problem(lo=(0.1, -0.3, 0.0), hi=(1.0, 0.9, 2.0), **case)
    rng = np.random.default_rng(7)
    u = rng.uniform(0.0, 0.8, size=p.shape)
    want = u.copy()
    t = 0.3
    for s in range(3):
        want = dense_step(p, want, t + s * p.tau)
    got = oracle_mod.advance(p, u, 3, t0=t)
    assert np.abs(got - want).max() <= 1e-13 * max(1.0, np.abs(want).max())


def test_dense_brute_force_mms_forcing(oracle_mod):
    """The forcing term psi of Example 5.1 is checked through its defining
    property: with f = u(1-u^2) + psi the continuous solution is
    e^{-lambda t} prod sin; here with the discrete eigenvalue in psi, the
    semi-discrete solution is exactly that on the grid, so a fine-step run
    must approach it at second order (see the EOC test) and one dense step
    must match the oracle's step."""
    p = W.Problem(dim=2, n=(6, 5), kappa=(0.8,), q=0.4, tau=0.05, reaction="ac_mms", rxn_param=(1.5, 1.0))
    u0 = W.sine_product(p)[None]
    lam = 1.5
    mu = sum(4 / p.h(d) ** 2 * math.sin(math.pi * p.h(d) / 2) ** 2 for d in range(2))

    def psi(t):
        ue = math.exp(-lam * t) * u0
        return (-lam + p.kappa[0] * mu + p.q) * ue - ue * (1 - ue ** 2)

    f_or = oracle_mod.reaction(p, u0 * 0.7, t=0.2)
    assert np.allclose(f_or, (0.7 * u0) * (1 - (0.7 * u0) ** 2) + psi(0.2), rtol=1e-14, atol=1e-14)


# ---------------------------------------------------------------------------
# P2-P4: special cases with closed-form answers
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [2, 3])
def test_linear_reaction_mode_amplification(oracle_mod, dim):
    """f = c u on a joint sine mode: with a_d = Q1(tau lambda_d), A = prod_{d>0} a_d,
    b = Q2(tau lambda_x), e = Q3(tau lambda_x):
    W = (a_x A + tau c b A) U and U+ = W + tau e c (W - A U)."""
    n = (9, 8) if dim == 2 else (7, 6, 5)
    c = -2.3
    p = W.Problem(dim=dim, n=n, kappa=(0.21,), q=0.7, tau=0.04, reaction="linear", rxn_param=(c,))
    js = (2, 5) if dim == 2 else (3, 2, 4)
    U = sine_mode(p, js)
    tl = [p.tau * eig1d(p, d, js[d]) for d in range(dim)]
    ax = q_scalar(2, 1, tl[0])
    A = np.prod([q_scalar(2, 1, t) for t in tl[1:]])
    b = q_scalar(2, 2, tl[0])
    e = q_scalar(2, 3, tl[0])
    Wf = ax * A + p.tau * c * b * A
    amp = Wf + p.tau * e * c * (Wf - A)
    got = oracle_mod.advance(p, U, 1)
    assert np.abs(got - amp * U).max() <= 1e-13


def test_heun_special_case(oracle_mod):
    """kappa = q = 0 gives Q1 = Q2 = 1, Q3 = 1/2: the step is Heun's method
    W = U + tau f(U), U+ = W + tau/2 (f(W) - f(U)) pointwise."""
    for reaction, params in (("fisher", (1.7,)), ("fhn_cubic", (0.1, 0.01, 0.5)),
                             ("fhn_classic", (1.0, 1.0)), ("saturating", (0.1,))):
        ncomp = 2 if reaction.startswith("fhn") else 1
        p = W.Problem(dim=2, n=(6, 7), kappa=(0.0,) * ncomp, q=0.0, tau=0.1, reaction=reaction,
                      rxn_param=params)
        rng = np.random.default_rng(3)
        u = rng.uniform(0.0, 0.7, size=p.shape)
        f0 = dense_reaction(p, 0.0, u)
        w = u + p.tau * f0
        want = w + 0.5 * p.tau * (dense_reaction(p, p.tau, w) - f0)
        got = oracle_mod.advance(p, u, 1)
        assert np.abs(got - want).max() <= 1e-15, reaction


@pytest.mark.parametrize("pade", [2, 4])
def test_pure_diffusion_product(oracle_mod, pade):
    """f = 0: U^N = (prod_d Q1(tau lambda_d))^N U^0 on a joint mode."""
    p = W.Problem(dim=3, n=(8, 7, 9), kappa=(0.6,), q=1.2, tau=0.003, reaction="none", pade=pade)
    js = (4, 1, 7)
    U = sine_mode(p, js)
    g = np.prod([q_scalar(pade, 1, p.tau * eig1d(p, d, js[d])) for d in range(3)])
    got = oracle_mod.advance(p, U, 12)
    assert np.abs(got - g ** 12 * U).max() <= 1e-13


# ---------------------------------------------------------------------------
# convergence order and boundedness (Theorem 4.7 and Sec. 5)
# ---------------------------------------------------------------------------

def test_second_order_against_exact_exponential_linear(oracle_mod):
    """f = c u: the semi-discrete solution is expm(-T (A_h - c)) u0 (dense,
    scipy); the observed order in tau is about 2."""
    c = 0.8
    p = W.Problem(dim=2, n=(9, 11), kappa=(0.05,), q=0.5, tau=0.1, reaction="linear", rxn_param=(c,))
    A1, (A2,) = split_ops(p)
    Ah = A1 + A2
    rng = np.random.default_rng(11)
    u0 = W.sine_product(p)[None] + 0.1 * rng.uniform(-1, 1, size=p.shape)
    T = 1.0
    exact = (scipy.linalg.expm(-T * (Ah - c * np.eye(Ah.shape[0]))) @ u0.reshape(-1)).reshape(p.shape)
    errs = []
    for N in (8, 16, 32, 64):
        got = oracle_mod.advance(p.replace(tau=T / N), u0, N)
        errs.append(np.abs(got - exact).max())
    eoc = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(1.8 < e < 2.3 for e in eoc), eoc


def test_second_order_discrete_manufactured(oracle_mod):
    """Allen-Cahn with the discrete-eigenvalue forcing: the grid function
    e^{-t} prod sin solves the semi-discrete system exactly, so the error is
    purely temporal and the EOC is about 2 (Sec. 5, Example 5.1)."""
    p = W.Problem(dim=2, n=(31, 31), kappa=(1.0,), q=0.0, tau=0.1, reaction="ac_mms", rxn_param=(1.0, 1.0))
    u0 = W.sine_product(p)[None]
    errs = []
    for N in (32, 64, 128):
        got = oracle_mod.advance(p.replace(tau=1.0 / N), u0, N)
        errs.append(np.abs(got - math.exp(-1.0) * u0).max())
    eoc = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 < e < 2.3 for e in eoc), eoc


def test_long_run_stays_bounded(oracle_mod):
    """Example 5.2's long run (tau = 0.1 to t = 100) stays in (0, 1) and
    bounded (Theorem 4.2, Sec. 5)."""
    p = W.Problem(dim=2, n=(63, 63), kappa=(1.0,), q=1.0, tau=0.1, reaction="saturating", rxn_param=(0.1,))
    u = 0.99 * W.sine_product(p)[None]
    u = oracle_mod.advance(p, u, 1000)
    assert np.all(np.isfinite(u))
    assert u.max() < 0.99 and u.min() >= -1e-12
