"""CPU oracle for the exact-exponential dimension-split ETD2RK scheme.

TEST INFRASTRUCTURE ONLY (like the rest of this package): the tests, the
smoke check and the benchmark's CPU-baseline leg may use it; the product path
never does.  It shares no code with the GPU library.

What it computes (Sec. 2.2, the two fully discrete equations that define
ETD2RK-DS before any Pade approximation).  With A_1 the x-direction operator
and A_2 the sum of the other directions' operators (Sec. 2.2's splitting):

    W   = e^{-tau A_1} e^{-tau A_2} U + A_1^{-1} (I - e^{-tau A_1}) e^{-tau A_2} f(t_n, U)
    U+  = W + (A_1^{-1} tau - A_1^{-2} + A_1^{-2} e^{-tau A_1})
              (f(t_{n+1}, W) - e^{-tau A_2} f(t_n, U)) / tau

Written with the phi-functions phi_1(z) = (1 - e^{-z})/z and
phi_2(z) = (z - 1 + e^{-z})/z^2 of z = tau A_1 (A_1^{-1}(I - e^{-tau A_1}) =
tau phi_1 and the bracket / tau = tau phi_2), and e^{-tau A_2} = prod over the
other directions of e^{-tau A_d} (Sec. 2.2, property (i) of the commuting
Kronecker terms).  Each 1-D matrix function is formed densely from ONE matrix
exponential of the block matrix

    B = [[-tau A, I, 0], [0, 0, I], [0, 0, 0]],
    expm(B) = [[e^{-tau A}, phi_1(tau A), phi_2(tau A)], [.., .., ..], ..],

(scipy.linalg.expm, scaling and squaring), so no phi-function is evaluated
by a scalar formula here.  A_d = h^-2 tridiag(-kappa, 2 kappa + q h^2/dim,
-kappa) (Sec. 2.1), per component.  The reactions come from the C oracle.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import reaction as _reaction


def stencil(p, d: int, comp: int = 0) -> np.ndarray:
    """Dense A_d of direction d for component comp (Sec. 2.1)."""
    n = p.n[d]
    h = (p.hi[d] - p.lo[d]) / (n + 1)
    k = p.kappa[comp]
    A = np.diag(np.full(n, (2.0 * k + p.q * h * h / p.dim) / (h * h)))
    off = np.full(n - 1, -k / (h * h))
    return A + np.diag(off, 1) + np.diag(off, -1)


def phi_matrices(A: np.ndarray, tau: float):
    """(e^{-tau A}, phi_1(tau A), phi_2(tau A)) from one block exponential."""
    n = A.shape[0]
    B = np.zeros((3 * n, 3 * n))
    B[:n, :n] = -tau * A
    B[:n, n:2 * n] = np.eye(n)
    B[n:2 * n, 2 * n:] = np.eye(n)
    E = scipy.linalg.expm(B)
    return E[:n, :n], E[:n, n:2 * n], E[:n, 2 * n:]


def _axis(p, d: int) -> int:
    """Array axis of direction d in a (ncomp, [nz,] ny, nx) field."""
    return p.dim - d


def mode(M: np.ndarray, g: np.ndarray, axis: int) -> np.ndarray:
    """The mode product along `axis`: g_{..i..} -> sum_j M_ij g_{..j..}."""
    return np.moveaxis(np.tensordot(M, g, axes=([1], [axis])), 0, axis)


class PhiStepper:
    """The scheme above for one problem (matrix functions formed once)."""

    def __init__(self, p):
        self.p = p
        # the C oracle's reactions do not depend on the time-stepping family
        self.rp = p.replace(pade=2)
        self.E, self.F1, self.F2 = {}, {}, {}
        for c in range(p.ncomp):
            for d in range(p.dim):
                e, f1, f2 = phi_matrices(stencil(p, d, c), p.tau)
                self.E[c, d], self.F1[c, d], self.F2[c, d] = e, f1, f2

    def split2(self, c: int, g: np.ndarray) -> np.ndarray:
        """e^{-tau A_2} g for component c (the y and z directions)."""
        for d in range(1, self.p.dim):
            g = mode(self.E[c, d], g, _axis(self.p, d) - 1)
        return g

    def step(self, U: np.ndarray, tn: float) -> np.ndarray:
        p = self.p
        tau = p.tau
        F0 = _reaction(self.rp, U, tn)
        W = np.empty_like(U)
        e2F = np.empty_like(U)
        ax = _axis(p, 0) - 1
        for c in range(p.ncomp):
            e2F[c] = self.split2(c, F0[c])
            W[c] = mode(self.E[c, 0], self.split2(c, U[c]), ax) + tau * mode(self.F1[c, 0], e2F[c], ax)
        F1 = _reaction(self.rp, W, tn + tau)
        out = np.empty_like(U)
        for c in range(p.ncomp):
            out[c] = W[c] + tau * mode(self.F2[c, 0], F1[c] - e2F[c], ax)
        return out


def advance(p, u: np.ndarray, nsteps: int, t0: float = 0.0) -> np.ndarray:
    """U after nsteps steps of the exact-exponential scheme (input untouched)."""
    st = PhiStepper(p)
    U = np.array(u, dtype=np.float64).reshape(p.shape)
    for n in range(nsteps):
        U = st.step(U, t0 + n * p.tau)
    return U
