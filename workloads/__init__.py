"""Problem descriptions and seeded synthetic inputs.

This module is shared by the CPU oracle harness and the GPU path.  It holds
problem *data* (grid sizes, coefficients, reaction names) and seeded input
fields only; none of the time-stepping arithmetic lives here.

Grid convention (Sec. 2.1 of the paper, with ``n`` counting interior points):
direction d has ``n[d]`` interior nodes ``x_i = lo[d] + i*h[d]``, i = 1..n[d],
``h[d] = (hi[d] - lo[d]) / (n[d] + 1)``; the field is stored with x fastest,
shape ``(ncomp, ny, nx)`` in 2-D and ``(ncomp, nz, ny, nx)`` in 3-D.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

REACTIONS = (
    "none",          # f = 0
    "linear",        # f = c*u                         p = (c,)
    "fisher",        # f = a*u*(1-u)                   p = (a,)
    "allen_cahn",    # f = u - u^3
    "ac_mms",        # f = u(1-u^2) + psi(x,t)         p = (lam, discrete)
    "saturating",    # f = rho*u/(1-u)                 p = (rho,)
    "fhn_cubic",     # fu = u(1-u)(u-a) - v, fv = eps(u - g v)   p = (a, eps, g)
    "fhn_classic",   # fu = u - u^3/3 - v, fv = eps(u - alpha v) p = (eps, alpha)
)

DEFAULT_PARAMS = {
    "none": (),
    "linear": (1.0,),
    "fisher": (1.0,),
    "allen_cahn": (),
    "ac_mms": (1.0, 0.0),
    "saturating": (0.1,),
    "fhn_cubic": (0.1, 0.01, 0.5),
    "fhn_classic": (1.0, 1.0),
}

TWO_COMPONENT = ("fhn_cubic", "fhn_classic")


@dataclass(frozen=True)
class Problem:
    """One reaction-diffusion problem u_t - kappa*Lap(u) + q*u = f (Sec. 1)."""

    dim: int
    n: tuple                      # interior points (nx, ny[, nz])
    kappa: tuple = (1.0,)         # one diffusivity per component
    q: float = 0.0
    tau: float = 0.01
    reaction: str = "fisher"
    rxn_param: tuple = ()
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    pade: int = 2                 # 2: P_{0,2} (Sec. 3.1); 4: P_{0,4} (Sec. 5); 0: exact exponentials (Sec. 2.2)
    precision: str = "fp64"       # GPU mode-product precision: fp64|fp32|bf16x6|fp64_fp32|fp64_bf16x6

    def __post_init__(self):
        if self.dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        if len(self.n) != self.dim:
            raise ValueError("n must have dim entries")
        if self.reaction not in REACTIONS:
            raise ValueError(f"unknown reaction {self.reaction!r}")
        if len(self.kappa) != self.ncomp:
            raise ValueError("kappa needs one entry per component")

    @property
    def ncomp(self) -> int:
        return 2 if self.reaction in TWO_COMPONENT else 1

    @property
    def params(self) -> tuple:
        return tuple(self.rxn_param) if self.rxn_param else DEFAULT_PARAMS[self.reaction]

    @property
    def shape(self) -> tuple:
        return (self.ncomp,) + tuple(reversed(self.n))

    @property
    def npoints(self) -> int:
        return int(np.prod(self.n))

    def h(self, d: int) -> float:
        return (self.hi[d] - self.lo[d]) / (self.n[d] + 1)

    def coords(self, d: int) -> np.ndarray:
        """Interior node coordinates along direction d (Sec. 2.1)."""
        i = np.arange(1, self.n[d] + 1, dtype=np.float64)
        return self.lo[d] + i * self.h(d)

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def mesh(p: Problem):
    """Coordinate arrays broadcast to the field layout (x fastest)."""
    if p.dim == 2:
        y, x = np.meshgrid(p.coords(1), p.coords(0), indexing="ij")
        return (x, y)
    z, y, x = np.meshgrid(p.coords(2), p.coords(1), p.coords(0), indexing="ij")
    return (x, y, z)


def sine_product(p: Problem) -> np.ndarray:
    """prod_d sin(pi (x_d - lo_d)/L_d) on the interior nodes."""
    out = 1.0
    for d, xd in enumerate(mesh(p)):
        out = out * np.sin(math.pi * (xd - p.lo[d]) / (p.hi[d] - p.lo[d]))
    return np.asarray(out, dtype=np.float64)


# --------------------------------------------------------------------------
# Seeded initial data.  Generators draw in a fixed order from
# numpy.random.default_rng(seed) and return float64 arrays of shape p.shape.
# --------------------------------------------------------------------------

def u0_sine_noise(p: Problem, seed: int, amp: float = 0.01) -> np.ndarray:
    """sin-product plus uniform noise U(-amp, amp) on the interior."""
    rng = np.random.default_rng(seed)
    base = sine_product(p)
    noise = rng.uniform(-amp, amp, size=base.shape)
    return (base + noise)[None].copy()


def u0_sine_bumps(p: Problem, seed: int, ncenters: int = 8, sigma: float = 0.05,
                  box=(0.15, 0.85), amp: float = 1.0) -> np.ndarray:
    """sin-product plus Gaussian bumps exp(-|x-c|^2/sigma^2), centers ~ U(box)^d."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(box[0], box[1], size=(ncenters, p.dim))
    xs = mesh(p)
    out = sine_product(p)
    for c in centers:
        r2 = 0.0
        for d in range(p.dim):
            r2 = r2 + (xs[d] - c[d]) ** 2
        out = out + amp * np.exp(-r2 / sigma ** 2)
    return out[None].copy()


def u0_fhn_patch(p: Problem, seed: int, patch: float = 0.1, corner=(0.05, 0.85),
                 vmax: float = 0.1) -> np.ndarray:
    """u = 1 on a seeded patch^dim box (lower corner ~ U(corner)^dim) else 0;
    v ~ U(0, vmax) on the interior."""
    rng = np.random.default_rng(seed)
    lower = rng.uniform(corner[0], corner[1], size=p.dim)
    xs = mesh(p)
    inside = np.ones(xs[0].shape, dtype=bool)
    for d in range(p.dim):
        inside &= (xs[d] >= lower[d]) & (xs[d] <= lower[d] + patch)
    u = inside.astype(np.float64)
    v = rng.uniform(0.0, vmax, size=u.shape)
    return np.stack([u, v])


def u0_gaussian(p: Problem, sigma: float = 0.05, center=0.5) -> np.ndarray:
    """Gaussian bump exp(-|x-c|^2/sigma^2) for u, zero for v (Example 5.3)."""
    xs = mesh(p)
    r2 = 0.0
    for d in range(p.dim):
        r2 = r2 + (xs[d] - center) ** 2
    u = np.exp(-r2 / sigma ** 2)
    if p.ncomp == 1:
        return u[None].copy()
    return np.stack([u, np.zeros_like(u)])


def u0_random(p: Problem, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Plain uniform random field (parity and edge-case tests)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=p.shape)


# --------------------------------------------------------------------------
# Named workloads.  Seeds are 20260101 + index.
# --------------------------------------------------------------------------

SEED0 = 20260101


@dataclass(frozen=True)
class Workload:
    name: str
    problem: Problem
    nsteps: int
    init: str            # name of the generator above
    seed: int
    note: str = ""

    def u0(self) -> np.ndarray:
        return initial_field(self.problem, self.init, self.seed)


def initial_field(p: Problem, init: str, seed: int) -> np.ndarray:
    if init == "sine_noise":
        return u0_sine_noise(p, seed)
    if init == "sine_bumps":
        return u0_sine_bumps(p, seed)
    if init == "fhn_patch":
        return u0_fhn_patch(p, seed)
    if init == "gaussian":
        return u0_gaussian(p)
    if init == "sine":
        return sine_product(p)[None].copy()
    if init == "sine099":
        return (0.99 * sine_product(p))[None].copy()
    if init == "random":
        return u0_random(p, seed)
    raise ValueError(init)


def fisher2d_small(precision="fp64") -> Workload:
    """2-D scalar Fisher-KPP, 63^2 interior points (h = 1/64), 100 steps."""
    p = Problem(dim=2, n=(63, 63), kappa=(0.01,), q=0.0, tau=0.01, reaction="fisher",
                precision=precision)
    return Workload("fisher2d_n63", p, 100, "sine_noise", SEED0 + 0)


def fhn2d(precision="fp64") -> Workload:
    """2-D coupled FitzHugh-Nagumo, 511^2 interior points, 2000 steps."""
    p = Problem(dim=2, n=(511, 511), kappa=(1e-4, 1e-5), q=0.0, tau=0.05,
                reaction="fhn_cubic", rxn_param=(0.1, 0.01, 0.5), precision=precision)
    return Workload("fhn2d_n511", p, 2000, "fhn_patch", SEED0 + 1)


def fisher3d(precision="fp64", n=255, nsteps=200) -> Workload:
    """3-D scalar Fisher-KPP, 255^3 interior points (16.6M unknowns), 200 steps."""
    p = Problem(dim=3, n=(n, n, n), kappa=(0.005,), q=0.5, tau=0.005, reaction="fisher",
                precision=precision)
    return Workload(f"fisher3d_n{n}", p, nsteps, "sine_bumps", SEED0 + 2)


def fhn3d(precision="fp32", n=127, nsteps=400) -> Workload:
    """3-D FitzHugh-Nagumo, 127^3, the 2-D FHN reaction parameters, 400 steps."""
    p = Problem(dim=3, n=(n, n, n), kappa=(1e-4, 1e-5), q=0.0, tau=0.02,
                reaction="fhn_cubic", rxn_param=(0.1, 0.01, 0.5), precision=precision)
    return Workload(f"fhn3d_n{n}", p, nsteps, "fhn_patch", SEED0 + 4)


def batched2d(count: int = 256, extents=(127, 255, 511, 1023), nsteps: int = 100, precision: str = "fp32",
              seed: int = SEED0 + 3):
    """Many uneven 2-D Fisher-KPP instances advanced together: per instance,
    drawn in this order from one generator, n ~ U{extents} (square grid),
    kappa log-uniform on [1e-3, 1e-1], q ~ U[0, 1], then its initial field
    (sine product plus U(-0.01, 0.01) noise, from a seed drawn here too);
    tau = 0.01, f = u(1-u).  Returns (problems, u0 list, nsteps)."""
    rng = np.random.default_rng(seed)
    problems, u0s = [], []
    for _ in range(count):
        n = int(rng.choice(extents))
        kappa = float(10.0 ** rng.uniform(-3.0, -1.0))
        q = float(rng.uniform(0.0, 1.0))
        init_seed = int(rng.integers(0, 2 ** 31 - 1))
        p = Problem(dim=2, n=(n, n), kappa=(kappa,), q=q, tau=0.01, reaction="fisher", precision=precision)
        problems.append(p)
        u0s.append(u0_sine_noise(p, init_seed))
    return problems, u0s, nsteps


# Paper examples (Sec. 5), used as printed-value pins.  The paper's m counts
# intervals, so m = 512 means 511 interior points and m = 80 means 79.

def paper_allen_cahn(dim: int, pade: int = 2) -> Problem:
    n = (511, 511) if dim == 2 else (79, 79, 79)
    return Problem(dim=dim, n=n, kappa=(1.0,), q=0.0, tau=1.0, reaction="ac_mms",
                   rxn_param=(1.0, 0.0), pade=pade)


def paper_saturating(dim: int) -> Problem:
    n = (511, 511) if dim == 2 else (79, 79, 79)
    return Problem(dim=dim, n=n, kappa=(1.0,), q=1.0, tau=1.0, reaction="saturating",
                   rxn_param=(0.1,))


def paper_fhn() -> Problem:
    return Problem(dim=2, n=(511, 511), kappa=(0.01, 10.0), q=0.0, tau=1.0,
                   reaction="fhn_classic", rxn_param=(1.0, 1.0))
