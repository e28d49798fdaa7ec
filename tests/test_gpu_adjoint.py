"""The hand-written adjoint of the ETD2RK-DS step (gradients of a loss of
U_N with respect to u0, kappa_c and q) against central finite differences of
the CPU oracle's forward map, and its torch.autograd wrapper.

Bar: 1e-6 relative in FP64 (the finite-difference truncation and rounding are
below 1e-8 at the steps used).  The 3-D FitzHugh-Nagumo workload runs in FP32
as specified; its gradient is compared with the same FP64 oracle differences
at a bound derived from FP32 rounding over the run (see the test).
"""
import json
import os

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


def half_sq(uN, target):
    d = uN - target
    return 0.5 * float((d * d).sum()), d


def fd_gradient(field_at, x0, target, h, one_sided=False):
    """dL/dx at x0 for L = 1/2 ||u_N(x) - target||^2, from the oracle's final
    fields.  Loss differences are formed from field differences,
    L(a) - L(b) = sum (u_a - u_b) ((u_a + u_b)/2 - target), which is exact and
    avoids subtracting two large losses when the gradient is small; steps h and
    h/2 are Richardson-combined (truncation O(h^4) central, O(h^3) one-sided,
    used where x may not go below x0)."""
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


def adjoint_vs_fd(etd, oracle_mod, p, u0, target, N, h_rel=1e-3, seed=1, fd_precision="extended"):
    """Adjoint gradients of the GPU path against finite differences of the
    oracle's forward map (by default its extended-precision build, so that
    the differences resolve gradients far below the loss's own size)."""
    import torch
    st = etd.Stepper(p)
    u = st.field(u0)
    st.advance(u, N)
    torch.cuda.synchronize()
    uN = u.cpu().numpy().astype(np.float64)
    _, ubar = half_sq(uN, target)
    ubar0, grad = st.adjoint(st.field(u0), st.field(ubar), N)
    ubar0 = ubar0.cpu().numpy().astype(np.float64)
    st.close()
    p64 = p.replace(precision="fp64")

    def run(pp, uu):
        return oracle_mod.advance(pp, uu, N, precision=fd_precision)

    rows = []
    for c in range(p.ncomp):
        def at_k(k, c=c):
            kk = list(p.kappa)
            kk[c] = k
            return run(p64.replace(kappa=tuple(kk)), u0)
        rows.append((f"kappa{c}", grad[c], fd_gradient(at_k, p.kappa[c], target, h_rel * p.kappa[c])))
    hq = h_rel * max(p.q, 1e-2)
    rows.append(("q", grad[p.ncomp], fd_gradient(lambda q: run(p64.replace(q=q), u0), p.q, target, hq,
                                                 one_sided=p.q < hq)))
    dl = np.random.default_rng(seed).standard_normal(u0.shape)
    rows.append(("u0", float((ubar0 * dl).sum()), fd_gradient(lambda e: run(p64, u0 + e * dl), 0.0, target, 1e-4)))
    for name, a, b in rows:
        print(f"  {name}: adjoint {a:.10e} fd {b:.10e} rel {abs(a - b) / abs(b):.2e}")
    return rows


CASES = [
    ("2d-fisher-N1", dict(dim=2, n=(31, 37), kappa=(0.05,), q=0.3, tau=0.01, reaction="fisher"), "sine_noise", 0.8, 1),
    ("2d-fisher-N16", dict(dim=2, n=(31, 37), kappa=(0.05,), q=0.3, tau=0.01, reaction="fisher"), "sine_noise", 0.8, 16),
    ("3d-fisher-N6", dict(dim=3, n=(15, 17, 13), kappa=(0.02,), q=0.4, tau=0.01, reaction="fisher"), "sine_noise", 0.5, 6),
    ("2d-fhn-N9", dict(dim=2, n=(30, 33), kappa=(0.01, 0.002), q=0.1, tau=0.05, reaction="fhn_cubic"), "fhn", 0.9, 9),
    ("3d-fhnc-N5", dict(dim=3, n=(20, 14, 17), kappa=(0.01, 0.003), q=0.2, tau=0.05, reaction="fhn_classic",
                        rxn_param=(0.7, 1.2)), "fhn", 0.9, 5),
    ("2d-allen-cahn-p04-N8", dict(dim=2, n=(40, 25), kappa=(0.03,), q=0.6, tau=0.02, reaction="allen_cahn", pade=4),
     "sine_noise", 0.7, 8),
    # the saturating source has a pole at u = 1; this start (peak 0.6) stays clear
    # of it, where finite differences are well conditioned
    ("2d-saturating-N12", dict(dim=2, n=(33, 31), kappa=(0.1,), q=1.0, tau=0.01, reaction="saturating"), "sine06", 0.9,
     12),
    ("3d-ac-mms-N4", dict(dim=3, n=(12, 13, 14), kappa=(0.2,), q=0.1, tau=0.01, reaction="ac_mms",
                          rxn_param=(1.0, 0.0)), "sine", 0.5, 4),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_adjoint_matches_oracle_finite_differences_fp64(etd, oracle_mod, case):
    name, kw, init, scale, N = case
    p = W.Problem(**kw)
    if init == "fhn":
        u0 = W.u0_fhn_patch(p, 5, patch=0.4)
    elif init == "sine06":
        u0 = 0.6 * W.initial_field(p, "sine", 0)
    else:
        u0 = W.initial_field(p, init, 3)
    rows = adjoint_vs_fd(etd, oracle_mod, p, u0, scale * u0, N)
    for pname, a, b in rows:
        assert abs(a - b) <= 1e-6 * abs(b), (pname, a, b)


@pytest.mark.parametrize("precision,n,N,bound", [
    ("fp64", (255, 12, 10), 4, 1e-6),        # x padded to 256 (FP64 state)
    ("fp64", (20, 255, 9), 3, 1e-6),         # y padded to 256
    ("fp64_fp32", (255, 12, 10), 4, 1e-5),
    ("fp32", (511, 10, 9), 3, 1e-4),         # x padded to 512 (FP32 state)
])
def test_adjoint_large_extents(etd, oracle_mod, precision, n, N, bound):
    """The adjoint tiles hold four fields of one component, so the adjoint
    runs up to 256 points per direction with an FP64 state and 512 with an
    FP32 one.  Two-component 3-D FitzHugh-Nagumo against finite differences
    of the oracle.  Reduced-precision bounds: the products round to FP32
    (relative ~6e-8 each, ~1e-7 per step through the operator chain); an FP32
    state adds the same per step to the forward field and so to U+bar."""
    p = W.Problem(dim=3, n=n, kappa=(0.004, 0.001), q=0.2, tau=0.02, reaction="fhn_cubic",
                  rxn_param=(0.1, 0.01, 0.5), precision=precision)
    u0 = W.u0_fhn_patch(p, 7, patch=0.5)
    rows = adjoint_vs_fd(etd, oracle_mod, p, u0, 0.8 * u0, N,
                         fd_precision="extended" if precision == "fp64" else "fp64")
    for pname, a, b in rows:
        assert abs(a - b) <= bound * abs(b), (pname, a, b)


def test_adjoint_fhn3d_n127_fp32(etd, oracle_mod):
    """The 3-D FitzHugh-Nagumo workload (127^3, FP32) over 40 of its steps;
    loss = 1/2 ||u(T) - u_target||^2 with u_target from a run at 1.1 kappa_u.

    Budget: after 40 FP32 steps the state carries ~1e-6 of ||u|| rounding
    error, while the residual u(T) - u_target is only ~8.5e-3 of ||u||, so the
    adjoint's input ubar = u(T) - u_target is ~1.2e-4 off relative; every
    gradient is linear in ubar.  The bound 1e-3 covers that with margin; the
    adjoint's own FP32 arithmetic is below 1e-5 (kappa and q rows)."""
    wl = W.fhn3d(nsteps=40)
    p = wl.problem
    u0 = wl.u0()
    N = 40
    target = oracle_mod.advance(p.replace(precision="fp64", kappa=(p.kappa[0] * 1.1, p.kappa[1])), u0, N)
    rows = adjoint_vs_fd(etd, oracle_mod, p, u0, target, N, fd_precision="fp64")
    for pname, a, b in rows:
        assert abs(a - b) <= 1e-3 * abs(b), (pname, a, b)


FD_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fhn3d_n127_fd.json")
_FHN3D_TARGET = {}


def fhn3d_target(oracle_mod, g):
    """u_target of the 400-step gradient workload: the oracle's u_N at
    1.1 kappa_u (computed once per session)."""
    if "t" not in _FHN3D_TARGET:
        wl = W.fhn3d()
        p = wl.problem.replace(precision="fp64")
        _FHN3D_TARGET["t"] = oracle_mod.advance(
            p.replace(kappa=(p.kappa[0] * g["target_kappa_scale"], p.kappa[1])), wl.u0(), g["nsteps"])
    return _FHN3D_TARGET["t"]


# relative bound per precision: FP64 at the 1e-6 gradient target; the reduced
# modes at bounds derived from their rounding (see the test's docstring;
# measured: FP64 <= 6.8e-8, FP64 state with FP32 products <= 1.3e-6, FP32
# state <= 8.2e-6)
FHN3D_BOUNDS = {"fp64": 1e-6, "fp64_fp32": 1e-5, "fp32": 1e-4}


@pytest.mark.parametrize("precision", ["fp64", "fp64_fp32", "fp32"])
def test_adjoint_fhn3d_n127_all_400_steps(etd, oracle_mod, precision):
    """The 3-D FitzHugh-Nagumo gradient workload over all 400 steps (127^3 x
    2, tau = 0.02, sqrt(N) = 20-step checkpoint segments): dL/dkappa_u,
    dL/dkappa_v, dL/dq and dL/du0 along a seeded direction against central
    finite differences of the FP64 oracle (tests/golden/fhn3d_n127_fd.json,
    written by tests/golden/make_fhn3d_fd.py from the oracle alone).

    FP64: <= 1e-6 (the differences' truncation is ~1e-8).  The loss is
    ill-conditioned for reduced precision: u_N - u_target is only 1.3% of
    u_N (residual_rel in the golden file), and every gradient is linear in
    U+bar = u_N - u_target, so a relative forward error e of u_N can become
    e / 0.013 in the gradients.  FP32 products on an FP64 state leave
    e ~ 5e-8 (the 2-D workload's 2000 steps: 5.2e-8), so up to ~4e-6; an
    FP32 state adds ~6e-8 per step of rounding (e ~ 2.5e-7 after 40 steps,
    growing with the run), so a few 1e-5.  The bounds take those amplified
    errors with a factor ~2-4 of margin."""
    import torch
    with open(FD_GOLDEN) as f:
        g = json.load(f)
    wl = W.fhn3d(precision=precision)
    p = wl.problem
    u0 = wl.u0()
    N = g["nsteps"]
    assert N == wl.nsteps and list(p.kappa) == g["kappa"] and p.q == g["q"]
    target = fhn3d_target(oracle_mod, g)
    st = etd.Stepper(p)
    u = st.field(u0)
    st.advance(u, N)
    torch.cuda.synchronize()
    uN = u.cpu().numpy().astype(np.float64)
    ubar = uN - target
    ubar0, grad = st.adjoint(st.field(u0), st.field(ubar), N)
    ubar0 = ubar0.cpu().numpy().astype(np.float64)
    st.close()
    dl = np.random.default_rng(g["dir_seed"]).standard_normal(u0.shape)
    got = {"kappa0": grad[0], "kappa1": grad[1], "q": grad[2], "u0_dir": float((ubar0 * dl).sum())}
    fwd = float(np.linalg.norm(uN - target) / np.linalg.norm(uN))
    print(f"  {precision}: residual_rel {fwd:.3e} (oracle {g['residual_rel']:.3e})")
    bound = FHN3D_BOUNDS[precision]
    for name, ref in g["gradient"].items():
        rel = abs(got[name] - ref) / abs(ref)
        print(f"  {precision} {name}: adjoint {got[name]:.10e} fd {ref:.10e} rel {rel:.2e}")
    for name, ref in g["gradient"].items():
        assert abs(got[name] - ref) <= bound * abs(ref), (name, got[name], ref)


def test_autograd_function_matches_adjoint(etd):
    import torch
    p = W.Problem(dim=2, n=(30, 33), kappa=(0.01, 0.002), q=0.1, tau=0.05, reaction="fhn_cubic")
    u0 = torch.tensor(W.u0_fhn_patch(p, 5, patch=0.4), device="cuda", requires_grad=True)
    kappa = torch.tensor(p.kappa, dtype=torch.float64, requires_grad=True)
    q = torch.tensor(p.q, dtype=torch.float64, requires_grad=True)
    target = 0.9 * u0.detach()
    uN = etd.advance_autograd(u0, kappa, q, p, 9)
    loss = 0.5 * ((uN - target) ** 2).sum()
    loss.backward()
    st = etd.Stepper(p)
    ubar0, grad = st.adjoint(u0.detach(), (uN - target).detach(), 9)
    st.close()
    assert torch.equal(u0.grad, ubar0)
    assert kappa.grad.tolist() == grad[:2] and float(q.grad) == grad[2]


def test_adjoint_is_repeatable(etd):
    import torch
    wl = W.fhn3d(n=31, nsteps=10)
    st = etd.Stepper(wl.problem)
    u0 = st.field(wl.u0())
    ub = torch.ones_like(u0)
    a0, ga = st.adjoint(u0, ub, 10)
    b0, gb = st.adjoint(u0, ub, 10)
    st.close()
    assert torch.equal(a0, b0) and ga == gb


def test_autograd_fp32_problem_with_float64_u0(etd):
    """An FP32 problem given a float64 u0 (what the workload generators
    return): the forward rounds u0 once to FP32, and the gradients equal those
    of Stepper.adjoint on that rounded u0, returned as float64."""
    import torch
    p = W.Problem(dim=2, n=(30, 33), kappa=(0.01, 0.002), q=0.1, tau=0.05, reaction="fhn_cubic",
                  precision="fp32")
    u0 = torch.tensor(W.u0_fhn_patch(p, 5, patch=0.4), device="cuda", dtype=torch.float64, requires_grad=True)
    kappa = torch.tensor(p.kappa, dtype=torch.float64, requires_grad=True)
    q = torch.tensor(p.q, dtype=torch.float64, requires_grad=True)
    uN = etd.advance_autograd(u0, kappa, q, p, 9)
    assert uN.dtype == torch.float64
    target = 0.9 * u0.detach()
    loss = 0.5 * ((uN - target) ** 2).sum()
    loss.backward()
    assert u0.grad.dtype == torch.float64
    st = etd.Stepper(p)
    u32 = u0.detach().float().contiguous()
    ref = st.advance(u32.clone(), 9)
    assert torch.equal(uN.float(), ref)
    ubar0, grad = st.adjoint(u32, (uN - target).detach().float().contiguous(), 9)
    st.close()
    assert torch.equal(u0.grad, ubar0.double())
    assert kappa.grad.tolist() == grad[:2] and float(q.grad) == grad[2]


@pytest.mark.parametrize("dim,precision", [(3, "fp64"), (2, "fp32"), (3, "fp64_bf16x6")])
def test_adjoint_segment_lengths_agree(etd, dim, precision):
    """Checkpoint segments of ceil(sqrt(N)), an intermediate length and N steps
    (one forward pass that keeps every step's stage fields) replay the same
    states with the same kernels, so the gradients agree bit for bit; a
    workspace between two layouts' sizes takes the longer segment that fits."""
    import torch
    if dim == 3:
        p = W.fhn3d(n=31, nsteps=20, precision=precision).problem
    else:
        p = W.Problem(dim=2, n=(60, 45), kappa=(0.01, 0.002), q=0.1, tau=0.05, reaction="fhn_cubic",
                      precision=precision)
    N = 20
    st = etd.Stepper(p)
    u0 = st.field(W.u0_fhn_patch(p, 5, patch=0.4))
    ub = st.advance(u0.clone(), N) - 0.5
    sizes = [etd.etd_adjoint_workspace_bytes_segment(st.plan, N, k) for k in (5, 6, 7, 11, 20)]
    assert sizes[0] == etd.etd_adjoint_workspace_bytes(st.plan, N)
    assert sizes == sorted(sizes) and sizes[0] < sizes[-1]
    for bad in (4, 21, 0):
        with pytest.raises(etd.EtdError) as ei:
            etd.etd_adjoint_workspace_bytes_segment(st.plan, N, bad)
        assert ei.value.status == etd.ETD_EINVAL
    ref0, ref = st.adjoint(u0, ub, N)
    for seg in (7, 11, 20):
        b0, g = st.adjoint(u0, ub, N, segment=seg)
        assert torch.equal(b0, ref0), seg
        assert g == ref, seg
    st.close()
