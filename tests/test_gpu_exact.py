"""The exact-exponential variant (pade = 0: e^{-z}, phi_1, phi_2 in place of
the Pade factors; the fully discrete scheme of Sec. 2.2) on the GPU, against
the exact-exponential oracle (block matrix exponentials, FP64).

Bar: relative L2 <= 1e-12 in FP64, <= 1e-6 for the reduced-precision mode
products; the adjoint against finite differences of the oracle at 1e-6.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def etd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2601_06849_amd as m
    m.lib()
    return m


def run_gpu(etd, p, u0, nsteps, t0=0.0):
    import torch
    st = etd.Stepper(p)
    u = st.field(u0)
    st.advance(u, nsteps, t0)
    torch.cuda.synchronize()
    out = u.cpu().numpy().astype(np.float64)
    st.close()
    return out


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


CASES = [
    ("2d-fisher-n63", dict(dim=2, n=(63, 63), kappa=(0.01,), tau=0.01, reaction="fisher"), "sine_noise", 100, 0.0),
    ("2d-fhn-n255", dict(dim=2, n=(255, 200), kappa=(1e-4, 1e-5), tau=0.05, reaction="fhn_cubic"), "fhn", 60, 0.0),
    ("3d-fhnc", dict(dim=3, n=(20, 14, 17), kappa=(0.01, 0.003), q=0.2, tau=0.05, reaction="fhn_classic",
                     rxn_param=(0.7, 1.2)), "fhn", 10, 0.0),
    ("3d-ac-mms", dict(dim=3, n=(31, 17, 24), kappa=(0.2,), q=0.1, tau=0.01, reaction="ac_mms",
                       rxn_param=(1.0, 0.0)), "sine", 8, 0.3),
    ("3d-fisher-n95", dict(dim=3, n=(95, 64, 80), kappa=(0.005,), q=0.5, tau=0.005, reaction="fisher"),
     "sine_bumps", 5, 0.0),
]


def init(p, kind, seed=3):
    if kind == "fhn":
        return W.u0_fhn_patch(p, seed, patch=0.3)
    return W.initial_field(p, kind, seed)


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_exact_exponential_fp64_parity(etd, oracle_mod, case):
    name, kw, kind, N, t0 = case
    p = W.Problem(pade=0, **kw)
    u0 = init(p, kind)
    ref = oracle_mod.advance(p, u0, N, t0=t0)
    got = run_gpu(etd, p, u0, N, t0)
    err = rel_l2(got, ref)
    print(f"  rel_l2 {err:.2e}")
    assert err <= 1e-12


@pytest.mark.parametrize("precision", ["fp32", "bf16x6"])
@pytest.mark.parametrize("case", [CASES[1], CASES[4]], ids=lambda c: c[0])
def test_exact_exponential_reduced_precision(etd, oracle_mod, precision, case):
    name, kw, kind, N, t0 = case
    p = W.Problem(pade=0, precision=precision, **kw)
    u0 = init(p, kind)
    ref = oracle_mod.advance(p.replace(precision="fp64"), u0, N, t0=t0)
    err = rel_l2(run_gpu(etd, p, u0, N, t0), ref)
    print(f"  {precision} rel_l2 {err:.2e}")
    assert err <= 1e-6


def test_exact_exponential_tiny_steps_fp32(etd, oracle_mod):
    """tau*lambda down to 1e-9 (series region of phi_1 - 1, phi_2 - 1/2): the
    FP32 increments stay accurate and the run matches the FP64 oracle."""
    p = W.Problem(dim=2, n=(255, 127), kappa=(1e-3,), q=0.2, tau=1e-6, reaction="fisher", pade=0, precision="fp32")
    u0 = W.u0_sine_noise(p, 6)
    ref = oracle_mod.advance(p.replace(precision="fp64"), u0, 20)
    err = rel_l2(run_gpu(etd, p, u0, 20), ref)
    print(f"  rel_l2 {err:.2e}")
    assert err <= 1e-6


def fd_gradient(field_at, x0, target, h, one_sided=False):
    """Richardson-combined differences of L = 1/2 ||u_N - target||^2 formed
    from field differences (see test_gpu_adjoint)."""
    cache = {}

    def u(x):
        if x not in cache:
            cache[x] = field_at(x)
        return cache[x]

    def dL(a, b):
        ua, ub = u(a), u(b)
        return float(((ua - ub) * (0.5 * (ua + ub) - target)).sum())

    def diff(k):
        if one_sided:
            return (4 * dL(x0 + k, x0) - dL(x0 + 2 * k, x0)) / (2 * k)
        return dL(x0 + k, x0 - k) / (2 * k)

    return (4 * diff(h / 2) - diff(h)) / 3


@pytest.mark.parametrize("case", [
    ("2d-fisher-N8", dict(dim=2, n=(31, 37), kappa=(0.05,), q=0.3, tau=0.01, reaction="fisher"), "sine_noise", 8),
    ("3d-fhn-N5", dict(dim=3, n=(20, 14, 17), kappa=(0.01, 0.003), q=0.2, tau=0.05, reaction="fhn_cubic"), "fhn", 5),
], ids=lambda c: c[0])
def test_exact_exponential_adjoint_against_finite_differences(etd, oracle_mod, case):
    import torch
    name, kw, kind, N = case
    p = W.Problem(pade=0, **kw)
    u0 = init(p, kind, 5)
    target = 0.9 * u0
    st = etd.Stepper(p)
    u = st.advance(st.field(u0), N)
    ubar = u - st.field(target)
    ubar0, grad = st.adjoint(st.field(u0), ubar, N)
    ubar0 = ubar0.cpu().numpy()
    st.close()
    run = lambda pp, uu: oracle_mod.advance(pp, uu, N)
    rows = []
    for c in range(p.ncomp):
        def at_k(k, c=c):
            kk = list(p.kappa)
            kk[c] = k
            return run(p.replace(kappa=tuple(kk)), u0)
        rows.append((f"kappa{c}", grad[c], fd_gradient(at_k, p.kappa[c], target, 1e-3 * p.kappa[c])))
    rows.append(("q", grad[p.ncomp], fd_gradient(lambda q: run(p.replace(q=q), u0), p.q, target, 1e-3 * p.q)))
    dl = np.random.default_rng(1).standard_normal(u0.shape)
    rows.append(("u0", float((ubar0 * dl).sum()), fd_gradient(lambda e: run(p, u0 + e * dl), 0.0, target, 1e-4)))
    for nm, a, b in rows:
        print(f"  {nm}: adjoint {a:.10e} fd {b:.10e} rel {abs(a - b) / abs(b):.2e}")
        assert abs(a - b) <= 1e-6 * abs(b), nm
