"""Pins of the exact-exponential oracle (``oracle.phi``), which forms
e^{-tau A_d}, phi_1(tau A_d) and phi_2(tau A_d) from one block exponential:

- the matrix functions on the closed-form sine eigenvectors equal the scalar
  definitions e^{-z}, (1 - e^{-z})/z and (z - 1 + e^{-z})/z^2 at z = tau lambda_j;
- kappa = q = 0 reduces the scheme to Heun's method;
- f = c u on a joint mode has the closed-form per-step amplification;
- three steps equal the fully discrete equations of Sec. 2.2 evaluated with
  Kronecker-assembled A_1, A_2 (dense expm and dense solves), 2-D and 3-D;
- the temporal order is 2 against the exact semi-discrete solution.
"""
import math

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def phi(oracle_mod):
    from oracle import phi as m
    return m


def phi1(z):
    return -math.expm1(-z) / z if z > 1e-3 else sum((-z) ** k / math.factorial(k + 1) for k in range(12))


def phi2(z):
    if z > 1e-2:
        return (z + math.expm1(-z)) / (z * z)
    return sum((-z) ** k / math.factorial(k + 2) for k in range(12))


def sine_basis(n):
    i = np.arange(1, n + 1)
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * np.outer(i, i) / (n + 1))


@pytest.mark.parametrize("tau", [1e-5, 1e-3, 0.05, 1.0])
def test_matrix_functions_on_eigenvectors(phi, tau):
    p = W.Problem(dim=2, n=(23, 5), kappa=(0.7,), q=0.4, tau=tau, reaction="fisher", lo=(0.0, 0.0), hi=(2.0, 1.0))
    A = phi.stencil(p, 0)
    E, F1, F2 = phi.phi_matrices(A, tau)
    n, h = p.n[0], 2.0 / 24
    V = sine_basis(n)
    for j in range(n):
        lam = 0.7 * 4 / h ** 2 * math.sin((j + 1) * math.pi / (2 * (n + 1))) ** 2 + 0.4 / 2
        z = tau * lam
        v = V[:, j]
        for M, ref in ((E, math.exp(-z)), (F1, phi1(z)), (F2, phi2(z))):
            assert np.abs(M @ v - ref * v).max() <= 1e-13 * max(1.0, abs(ref)), (j, z)


def test_heun_when_the_operator_vanishes(oracle_mod, phi):
    p = W.Problem(dim=2, n=(9, 11), kappa=(0.0,), q=0.0, tau=0.1, reaction="fisher", pade=0)
    u = W.u0_random(p, 4, 0.0, 1.0)
    got = phi.advance(p, u, 3)
    rp = p.replace(pade=2)
    for k in range(3):
        f0 = oracle_mod.reaction(rp, u, k * p.tau)
        w = u + p.tau * f0
        u = u + 0.5 * p.tau * (f0 + oracle_mod.reaction(rp, w, (k + 1) * p.tau))
    assert np.abs(got - u).max() <= 1e-14


def test_linear_mode_amplification(phi):
    c = 0.8
    p = W.Problem(dim=2, n=(15, 12), kappa=(0.3,), q=0.5, tau=0.02, reaction="linear", rxn_param=(c,), pade=0)
    jx, jy = 3, 2
    lam = []
    for d, j in ((0, jx), (1, jy)):
        n, h = p.n[d], 1.0 / (p.n[d] + 1)
        lam.append(0.3 * 4 / h ** 2 * math.sin(j * math.pi / (2 * (n + 1))) ** 2 + 0.5 / 2)
    zx, zy = p.tau * lam[0], p.tau * lam[1]
    w = math.exp(-zx - zy) + p.tau * c * phi1(zx) * math.exp(-zy)
    G = w + p.tau * c * phi2(zx) * (w - math.exp(-zy))
    x = np.sin(jx * np.pi * np.arange(1, 16) / 16)
    y = np.sin(jy * np.pi * np.arange(1, 13) / 13)
    u0 = np.outer(y, x)[None]
    got = phi.advance(p, u0, 7)
    assert np.abs(got - G ** 7 * u0).max() <= 1e-14


def kron_ops(p, comp):
    """Dense A_1 (x) and A_2 (the other directions) on the x-fastest vector."""
    from oracle.phi import stencil
    I = [np.eye(p.n[d]) for d in range(p.dim)]
    Ax = stencil(p, 0, comp)
    Ay = stencil(p, 1, comp)
    if p.dim == 2:
        return np.kron(I[1], Ax), np.kron(Ay, I[0])
    Az = stencil(p, 2, comp)
    A1 = np.kron(I[2], np.kron(I[1], Ax))
    A2 = np.kron(I[2], np.kron(Ay, I[0])) + np.kron(Az, np.kron(I[1], I[0]))
    return A1, A2


BRUTE = [
    dict(dim=2, n=(5, 6), kappa=(0.4,), q=0.3, tau=0.05, reaction="fisher"),
    dict(dim=2, n=(6, 4), kappa=(0.05, 0.02), q=0.1, tau=0.1, reaction="fhn_cubic"),
    dict(dim=3, n=(4, 5, 3), kappa=(0.3,), q=0.6, tau=0.02, reaction="allen_cahn", lo=(0, -1, 0), hi=(1, 1, 2)),
    dict(dim=3, n=(3, 4, 5), kappa=(0.1,), q=0.2, tau=0.01, reaction="ac_mms", rxn_param=(1.0, 0.0)),
]


@pytest.mark.parametrize("kw", BRUTE, ids=lambda k: f"{k['dim']}d-{k['reaction']}")
def test_brute_force_kronecker_equations(oracle_mod, phi, kw):
    import scipy.linalg
    p = W.Problem(pade=0, **kw)
    u = W.u0_random(p, 8, 0.0, 0.9)
    got = phi.advance(p, u, 3, t0=0.2)
    rp = p.replace(pade=2)
    tau = p.tau
    ops = []
    for c in range(p.ncomp):
        A1, A2 = kron_ops(p, c)
        N = A1.shape[0]
        e1, e2 = scipy.linalg.expm(-tau * A1), scipy.linalg.expm(-tau * A2)
        inv1 = np.linalg.solve(A1, np.eye(N))
        ops.append((e1, e2, inv1, tau * inv1 - inv1 @ inv1 + inv1 @ inv1 @ e1))
    U = u.reshape(p.ncomp, -1).copy()
    for k in range(3):
        tn = 0.2 + k * tau
        F0 = oracle_mod.reaction(rp, U.reshape(p.shape), tn).reshape(p.ncomp, -1)
        Wn = np.stack([e1 @ e2 @ U[c] + inv1 @ (np.eye(len(U[c])) - e1) @ e2 @ F0[c]
                       for c, (e1, e2, inv1, _) in enumerate(ops)])
        F1 = oracle_mod.reaction(rp, Wn.reshape(p.shape), tn + tau).reshape(p.ncomp, -1)
        U = np.stack([Wn[c] + B @ (F1[c] - e2 @ F0[c]) / tau for c, (e1, e2, inv1, B) in enumerate(ops)])
    ref = U.reshape(p.shape)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= 1e-12, err


def test_second_order_in_time(phi):
    """f = c u with a multi-mode start: error at T against the exact
    semi-discrete solution expm((c I - A) T) u0 falls by ~4 per halving."""
    import scipy.linalg
    c = 1.5
    base = W.Problem(dim=2, n=(7, 6), kappa=(0.2,), q=0.1, tau=0.1, reaction="linear", rxn_param=(c,), pade=0)
    u0 = W.u0_random(base, 9, -1.0, 1.0)
    A1, A2 = kron_ops(base, 0)
    T = 0.4
    exact = (scipy.linalg.expm(T * (c * np.eye(A1.shape[0]) - A1 - A2)) @ u0.ravel()).reshape(base.shape)
    errs = []
    for k in range(4):
        N = 4 * 2 ** k
        p = base.replace(tau=T / N)
        errs.append(np.abs(phi.advance(p, u0, N) - exact).max())
    eoc = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(1.8 < e < 2.3 for e in eoc), (errs, eoc)


def test_dispatch_through_the_oracle_entry_point(oracle_mod, phi):
    p = W.Problem(dim=2, n=(9, 8), kappa=(0.1,), tau=0.01, reaction="fisher", pade=0)
    u = W.u0_sine_noise(p, 2)
    assert np.array_equal(oracle_mod.advance(p, u, 4, t0=0.1), phi.advance(p, u, 4, t0=0.1))
    with pytest.raises(ValueError):
        oracle_mod.advance(p, u, 1, precision="extended")
