"""CPU oracle for the Pade-based dimension-split ETD2RK scheme.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg use this module; the product path never imports it.  It
wraps ``etdo.c`` (plain C99, FP64 complex Thomas line solves, see that file's
header for the formulas and their places in the paper) through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "etdo.c")
_LIB = os.path.join(_HERE, "libetdo.so")
# The same source built with x87 extended precision: a referee that shows how
# much of a difference between two FP64 results is FP64 rounding.
_LIB_EXT = os.path.join(_HERE, "libetdo_ext.so")

_RXN = {
    "none": 0, "linear": 1, "fisher": 2, "allen_cahn": 3, "ac_mms": 4,
    "saturating": 5, "fhn_cubic": 6, "fhn_classic": 7,
}


class _Problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3),
        ("ncomp", ctypes.c_int),
        ("kappa", ctypes.c_double * 2),
        ("q", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("rxn", ctypes.c_int),
        ("rxn_param", ctypes.c_double * 8),
        ("pade", ctypes.c_int),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over independent lines), in
    FP64 and in the extended-precision referee build."""
    for out, extra in ((_LIB, []), (_LIB_EXT, ["-DETDO_EXTENDED"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-D_DEFAULT_SOURCE", *extra,
                   "-o", out + ".tmp", _SRC, "-lm"]
            subprocess.check_call(cmd, cwd=_HERE)
            os.replace(out + ".tmp", out)
    return _LIB


_libs = {}


def lib(precision: str = "fp64"):
    if precision not in _libs:
        path = {"fp64": _LIB, "extended": _LIB_EXT}[precision]
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build(force=False)
        L = ctypes.CDLL(path)
        P = ctypes.POINTER(_Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        L.etdo_advance.argtypes = [P, dp, ctypes.c_double, ctypes.c_int, ctypes.c_int]
        L.etdo_apply.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int]
        L.etdo_reaction.argtypes = [P, ctypes.c_double, dp, dp]
        L.etdo_poles.argtypes = [ctypes.c_int, dp, dp]
        L.etdo_threads.argtypes = [ctypes.c_int]
        _libs[precision] = L
    return _libs[precision]


def _struct(p) -> _Problem:
    s = _Problem()
    s.dim = p.dim
    for d in range(3):
        s.n[d] = p.n[d] if d < p.dim else 1
        s.lo[d] = p.lo[d]
        s.hi[d] = p.hi[d]
    s.ncomp = p.ncomp
    for c in range(p.ncomp):
        s.kappa[c] = p.kappa[c]
    s.q = p.q
    s.tau = p.tau
    s.rxn = _RXN[p.reaction]
    for i, v in enumerate(p.params):
        s.rxn_param[i] = v
    s.pade = p.pade
    return s


def _f64(a: np.ndarray, shape) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.size != int(np.prod(shape)):
        raise ValueError(f"field has {a.size} values, expected shape {shape}")
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def advance(p, u: np.ndarray, nsteps: int, t0: float = 0.0, nthreads: int = 0,
            precision: str = "fp64") -> np.ndarray:
    """Return U after nsteps steps of the scheme from time t0 (input untouched).
    precision="extended" runs the referee build (x87 extended arithmetic).
    pade = 0 selects the exact-exponential scheme (``oracle.phi``, FP64)."""
    if p.pade == 0:
        if precision != "fp64":
            raise ValueError("the exact-exponential oracle runs in FP64 only")
        from . import phi
        return phi.advance(p, u, nsteps, t0)
    out = _f64(u, p.shape).copy()
    rc = lib(precision).etdo_advance(ctypes.byref(_struct(p)), _ptr(out), float(t0), int(nsteps), int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return out.reshape(p.shape)


def apply(p, ell: int, d: int, g: np.ndarray, comp: int = 0, nthreads: int = 0) -> np.ndarray:
    """Q_ell(tau A_d) g for one component (other components of the result are 0)."""
    g = _f64(g, p.shape)
    out = np.zeros(p.shape, dtype=np.float64)
    rc = lib().etdo_apply(ctypes.byref(_struct(p)), int(ell), int(d), int(comp), _ptr(g), _ptr(out),
                          int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def reaction(p, u: np.ndarray, t: float = 0.0) -> np.ndarray:
    u = _f64(u, p.shape)
    out = np.zeros(p.shape, dtype=np.float64)
    rc = lib().etdo_reaction(ctypes.byref(_struct(p)), float(t), _ptr(u), _ptr(out))
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    return out


def poles(pade: int):
    """(poles, residues[l-1][k]) of the rational family."""
    s = np.zeros(4)
    r = np.zeros(12)
    npl = lib().etdo_poles(int(pade), _ptr(s), _ptr(r))
    sp = s[0:2 * npl:2] + 1j * s[1:2 * npl:2]
    rr = (r[0:6 * npl:2] + 1j * r[1:6 * npl:2]).reshape(3, npl)
    return sp, rr


def threads(nthreads: int = 0) -> int:
    return int(lib().etdo_threads(int(nthreads)))
