"""The resident schedule: every step of an etd_advance call in one cooperative
launch whose workgroups run the stages' tiles in turn, a grid-wide barrier
between stages (small grids: one padded extent of at most 128 points).

It runs the same tile bodies as the per-stage launches, and every tile shape
computes each output with the same operations in the same order, so the two
schedules must agree bit for bit.  The one exception is the manufactured
Allen-Cahn source, whose factor e^{-lambda t} the resident kernel forms on the
device (the per-stage launches take it from the host).  The small workload
(63^2 Fisher-KPP, 100 steps) is also checked against the FP64 oracle at the
parity bar (relative L2 and max error <= 1e-12).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

PRECISIONS = ["fp64", "fp32", "bf16x6", "fp64_fp32", "fp64_bf16x6"]


@pytest.fixture(scope="module")
def etd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2601_06849_amd as m
    m.lib()
    return m


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def run(etd, p, u0, nsteps, schedule, t0=0.0, chunks=None):
    st = etd.Stepper(p)
    st.set_schedule(schedule)
    assert st.schedule() == schedule
    u = st.field(u0)
    t = t0
    for k in (chunks or [nsteps]):
        st.advance(u, k, t)
        t += k * p.tau
    out = host(u)
    st.close()
    return out


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())), \
        float(np.abs(a - b).max() / np.abs(b).max())


def test_small_workload_resident_vs_oracle(etd, oracle_mod):
    """63^2 Fisher-KPP, all 100 steps in one launch, against the FP64 oracle."""
    wl = W.fisher2d_small()
    u0 = wl.u0()
    ref = oracle_mod.advance(wl.problem, u0, wl.nsteps)
    got = run(etd, wl.problem, u0, wl.nsteps, "resident")
    e2, em = rel(got, ref)
    print(f"  rel_l2={e2:.3e} rel_max={em:.3e}")
    assert np.all(np.isfinite(got))
    assert e2 <= 1e-12 and em <= 1e-12, (e2, em)


CASES = [
    # (dim, n, reaction, params, kappa)
    (2, (63, 63), "fisher", (1.0,), (0.01,)),
    (2, (50, 61), "fhn_cubic", (0.1, 0.01, 0.5), (1e-2, 1e-3)),
    (2, (127, 113), "allen_cahn", (), (0.02,)),
    (3, (31, 31, 31), "fhn_classic", (1.0, 1.0), (0.01, 0.1)),
    (3, (63, 50, 60), "fisher", (1.3,), (0.005,)),
    (3, (1, 1, 1), "fisher", (1.0,), (0.3,)),
    (3, (127, 120, 113), "fhn_cubic", (0.1, 0.01, 0.5), (1e-3, 1e-4)),   # 1024 tiles a stage
]


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("dim,n,rxn,params,kappa", CASES, ids=lambda v: str(v))
def test_resident_equals_stages(etd, precision, dim, n, rxn, params, kappa):
    p = W.Problem(dim=dim, n=n, kappa=kappa, q=0.2, tau=0.01, reaction=rxn, rxn_param=params,
                  precision=precision)
    if rxn.startswith("fhn"):
        u0 = W.u0_fhn_patch(p, seed=3, patch=0.3)
    else:
        u0 = 0.9 * W.sine_product(p)[None] + 0.05 * W.u0_random(p, seed=4, lo=0, hi=1)
    nsteps = 6 if max(n) > 100 else 25
    a = run(etd, p, u0, nsteps, "stages", t0=0.5)
    b = run(etd, p, u0, nsteps, "resident", t0=0.5)
    assert np.all(np.isfinite(b))
    assert np.array_equal(a, b), rel(b, a)


@pytest.mark.parametrize("dim,n", [(2, (63, 63)), (3, (31, 20, 17))])
def test_resident_manufactured_source(etd, oracle_mod, dim, n):
    """AC_MMS: the time factor is formed on the device, so the schedules agree
    to rounding; both meet the oracle."""
    p = W.Problem(dim=dim, n=n, kappa=(0.4,), q=0.2, tau=0.01, reaction="ac_mms", rxn_param=(2.0, 1.0))
    u0 = 0.9 * W.sine_product(p)[None] + 0.05 * W.u0_random(p, seed=4, lo=0, hi=1)
    a = run(etd, p, u0, 20, "stages", t0=0.25)
    b = run(etd, p, u0, 20, "resident", t0=0.25)
    e2, em = rel(b, a)
    print(f"  resident vs stages rel_l2={e2:.3e} rel_max={em:.3e}")
    assert e2 <= 1e-14 and em <= 1e-14
    ref = oracle_mod.advance(p, u0, 20, t0=0.25)
    e2, em = rel(b, ref)
    assert e2 <= 1e-12 and em <= 1e-12, (e2, em)


def test_resident_resumes_exactly(etd):
    """Three calls of 30 + 1 + 69 steps equal one call of 100 (times carried)."""
    p = W.Problem(dim=2, n=(63, 63), kappa=(0.01,), tau=0.01, reaction="fisher")
    u0 = W.u0_sine_noise(p, 5)
    a = run(etd, p, u0, 100, "resident")
    b = run(etd, p, u0, 100, "resident", chunks=[30, 1, 69])
    assert np.array_equal(a, b)


def test_resident_capture_and_timing(etd):
    """AUTO is the per-stage schedule; a forced resident schedule refuses
    graph capture and records no stage times, and all agree bit for bit."""
    import torch
    p = W.Problem(dim=2, n=(63, 63), kappa=(0.01,), tau=0.01, reaction="fisher")
    u0 = W.u0_sine_noise(p, 5)
    st = etd.Stepper(p)
    assert st.schedule() == "stages"
    st.set_schedule("resident")
    assert st.schedule() == "resident"
    res = st.field(u0)
    st.advance(res, 40)
    # timing on: the resident launch is not a stage launch, so nothing is timed
    etd.etd_timing_enable(st.plan, 1)
    timed = st.field(u0)
    st.advance(timed, 40)
    ms, counts = etd.etd_timing_read(st.plan)
    etd.etd_timing_enable(st.plan, 0)
    assert list(counts) == [0, 0, 0]
    assert np.array_equal(host(timed), host(res))
    s = torch.cuda.Stream()
    with pytest.raises(etd.EtdError) as ei:
        st.capture(st.field(u0), 40, s)
    assert ei.value.status == etd.ETD_EUNSUPPORTED
    torch.cuda.synchronize()
    # AUTO: per-stage launches, eagerly and from a graph, equal the resident run
    st.set_schedule("auto")
    eager = st.field(u0)
    for _ in range(4):
        st.advance(eager, 10)
    assert np.array_equal(host(eager), host(res))
    u = st.field(u0)
    torch.cuda.synchronize()
    g = st.capture(u, 40, s)
    for r in range(2):
        if r:
            u.copy_(st.field(u0))
            torch.cuda.synchronize()
        g.launch(s)
        s.synchronize()
        assert np.array_equal(host(u), host(res)), r
    g.close()
    st.close()
