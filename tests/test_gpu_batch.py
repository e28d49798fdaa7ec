"""Tile shapes, the autotuner, batched (grouped persistent) launches and HIP
graphs, through the C ABI.

- Every valid tile shape computes each output with the same operations in
  the same order, so results are bit-identical across shapes; the autotuner's
  choice is checked the same way.
- A batch of uneven instances matches, instance by instance, the single-plan
  path bit for bit (same kernels, same tiles), and the FP64 oracle to 1e-12.
- Graph replays match eager calls bit for bit, with eager work and host
  synchronisation between replays.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-6


@pytest.fixture(scope="module")
def etd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_2601_06849_amd as m
    m.lib()
    return m


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def valid_shapes(etd, st, d):
    """Tile shapes accepted for direction d (others at their current choice)."""
    cur = st.tiles()
    out = []
    for rb in (2, 4, 8):
        for cb in (1, 2, 4):
            trial = list(cur)
            trial[d] = (rb, cb)
            try:
                st.set_tiles(trial)
            except etd.EtdError as e:
                assert e.status == etd.ETD_EUNSUPPORTED
                continue
            out.append((rb, cb))
    st.set_tiles(cur)
    return out


SHAPE_CASES = [
    ("3d-fisher-fp64", dict(dim=3, n=(63, 47, 33), kappa=(0.02,), q=0.4, tau=0.01, reaction="fisher")),
    ("2d-fhn-fp32", dict(dim=2, n=(255, 127), kappa=(1e-3, 1e-4), tau=0.05, reaction="fhn_cubic",
                         precision="fp32")),
    ("2d-fisher-bf16x6", dict(dim=2, n=(127, 511), kappa=(0.01,), q=0.2, tau=0.01, reaction="fisher",
                              precision="bf16x6")),
    ("3d-ac-fp32", dict(dim=3, n=(127, 64, 40), kappa=(0.05,), tau=0.01, reaction="allen_cahn", precision="fp32")),
]


@pytest.mark.parametrize("case", SHAPE_CASES, ids=lambda c: c[0])
def test_every_tile_shape_is_bit_identical(etd, case):
    name, kw = case
    p = W.Problem(**kw)
    u0 = W.initial_field(p, "sine_noise" if p.ncomp == 1 else "fhn_patch", 11)
    st = etd.Stepper(p)
    ref = host(st.advance(st.field(u0), 3))
    default = st.tiles()
    ntried = 0
    for d in range(p.dim):
        for shape in valid_shapes(etd, st, d):
            trial = list(default)
            trial[d] = shape
            st.set_tiles(trial)
            got = host(st.advance(st.field(u0), 3))
            print(f"  dir {d} shape {shape}: identical={np.array_equal(got, ref)}")
            assert np.array_equal(got, ref), (d, shape)
            ntried += 1
    st.set_tiles([(0, 0)] * p.dim)
    assert st.tiles() == default
    assert ntried >= p.dim + 1
    tuned = st.autotune()
    print(f"  default {default} autotuned {tuned}")
    got = host(st.advance(st.field(u0), 3))
    assert np.array_equal(got, ref)
    st.close()


def mixed_batch(precision="fp64"):
    """Uneven 2-D instances: four extents, per-instance coefficients,
    reactions and Pade orders, two instances sharing each extent."""
    rng = np.random.default_rng(7)
    probs = []
    for i, n in enumerate((31, 100, 63, 31, 127, 100, 63, 127)):
        rxn = ("fisher", "allen_cahn", "saturating", "linear")[i % 4]
        probs.append(W.Problem(dim=2, n=(n, n if i % 3 else n + 32), kappa=(float(10 ** rng.uniform(-3, -1)),),
                               q=float(rng.uniform(0, 1)), tau=float(rng.choice([0.01, 0.02])), reaction=rxn,
                               pade=4 if i % 2 else 2, precision=precision))
    u0s = [W.u0_sine_noise(p, 100 + i) * (0.5 if p.reaction == "saturating" else 1.0) for i, p in enumerate(probs)]
    return probs, u0s


def test_batch_matches_single_plans_and_oracle(etd, oracle_mod):
    probs, u0s = mixed_batch()
    b = etd.Batch(probs)
    print(f"  {len(probs)} instances in {b.groups()} groups")
    assert b.groups() == 4       # padded shapes 32x64, 128x128, 64x64, 64x96
    f = b.fields(u0s)
    b.advance(f, 9, t0=0.3)
    for i, (p, u0) in enumerate(zip(probs, u0s)):
        got = host(f[i])
        st = etd.Stepper(p)
        st.set_tiles(b.tiles(i)[:p.dim])
        single = host(st.advance(st.field(u0), 9, 0.3))
        st.close()
        ref = oracle_mod.advance(p, u0, 9, t0=0.3)
        err = rel_l2(got, ref)
        print(f"  instance {i} n={p.n[:2]} {p.reaction} P0{p.pade}: rel_l2 {err:.2e}")
        assert np.array_equal(got, single), i
        assert err <= FP64_TOL, i
    b.close()


def test_batch_3d_two_component_fp32_and_time_dependent(etd, oracle_mod):
    fhn = [W.Problem(dim=3, n=(n, n, 31), kappa=(k, k / 10), tau=0.02, reaction="fhn_cubic", precision="fp32")
           for n, k in ((31, 1e-3), (63, 5e-3), (31, 2e-3))]
    b = etd.Batch(fhn)
    u0s = [W.u0_fhn_patch(p, 30 + i, patch=0.3) for i, p in enumerate(fhn)]
    f = b.fields(u0s)
    b.advance(f, 12)
    for i, p in enumerate(fhn):
        err = rel_l2(host(f[i]), oracle_mod.advance(p, u0s[i], 12))
        print(f"  fhn instance {i}: rel_l2 {err:.2e}")
        assert err <= FP32_TOL
    b.close()
    mms = [W.Problem(dim=3, n=(n, 23, 17), kappa=(0.1,), q=0.2, tau=0.01, reaction="ac_mms", rxn_param=(1.0, 0.0))
           for n in (15, 40)]
    b = etd.Batch(mms)
    u0s = [W.initial_field(p, "sine", 0) * np.exp(-0.7) for p in mms]
    f = b.fields(u0s)
    b.advance(f, 6, t0=0.7)
    for i, p in enumerate(mms):
        err = rel_l2(host(f[i]), oracle_mod.advance(p, u0s[i], 6, t0=0.7))
        print(f"  mms instance {i}: rel_l2 {err:.2e}")
        assert err <= FP64_TOL
    b.close()


def test_batch_autotune_keeps_results(etd):
    probs, u0s = mixed_batch("fp32")
    b = etd.Batch(probs)
    f = b.fields(u0s)
    b.advance(f, 4)
    ref = [host(x) for x in f]
    before = [b.tiles(i) for i in range(len(probs))]
    b.autotune()
    after = [b.tiles(i) for i in range(len(probs))]
    print(f"  tiles before {before[0]} after {after[0]}")
    f = b.fields(u0s)
    b.advance(f, 4)
    for i in range(len(probs)):
        assert np.array_equal(host(f[i]), ref[i]), i
    b.close()


def test_plan_graph_replays_match_eager(etd):
    import torch
    p = W.Problem(dim=2, n=(63, 63), kappa=(0.01,), tau=0.01, reaction="fisher")
    u0 = W.u0_sine_noise(p, 5)
    st = etd.Stepper(p)
    eager = st.field(u0)
    s = torch.cuda.Stream()
    u = st.field(u0)
    torch.cuda.synchronize()
    g = st.capture(u, 10, s)
    assert np.array_equal(host(u), u0.reshape(p.shape))       # nothing ran during capture
    for r in range(3):
        g.launch(s)
        s.synchronize()
        st.advance(eager, 10, 0.0)      # eager work on the other stream between replays
        torch.cuda.synchronize()
        assert np.array_equal(host(u), host(eager)), r
    g.close()
    st.close()


def test_batch_graph_replays_and_staleness(etd):
    import torch
    probs, u0s = mixed_batch("fp32")
    b = etd.Batch(probs)
    eager = b.fields(u0s)
    f = b.fields(u0s)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = b.capture(f, 5, s)
    for r in range(3):
        g.launch(s)
        s.synchronize()
        b.advance(eager, 5)
        torch.cuda.synchronize()
        for i in range(len(probs)):
            assert np.array_equal(host(f[i]), host(eager[i])), (r, i)
    b.autotune()
    with pytest.raises(etd.EtdError) as ei:
        g.launch(s)
    assert ei.value.status == etd.ETD_EINVAL
    g.close()
    b.close()


def test_batched_workload_sampled_against_oracle(etd, oracle_mod):
    """The 256-instance uneven workload (n in {127, 255, 511, 1023}, FP32,
    100 steps) in one batch; the first instance of each extent is checked
    against the FP64 oracle over all steps, every instance for finiteness."""
    import torch
    probs, u0s, nsteps = W.batched2d()
    b = etd.Batch(probs)
    assert b.groups() == 4
    f = b.fields(u0s)
    b.advance(f, nsteps)
    torch.cuda.synchronize()
    seen = set()
    for i, p in enumerate(probs):
        got = f[i]
        assert bool(torch.isfinite(got).all()), i
        if p.n[0] in seen:
            continue
        seen.add(p.n[0])
        err = rel_l2(host(got), oracle_mod.advance(p, u0s[i], nsteps))
        print(f"  instance {i} n={p.n[0]} kappa={p.kappa[0]:.2e} q={p.q:.2f}: rel_l2 {err:.2e}")
        assert err <= FP32_TOL
    b.close()


@pytest.mark.parametrize("precision,reaction,n", [
    ("fp64", "fisher", (511, 480)), ("fp32", "fhn_cubic", (511, 480)), ("bf16x6", "fisher", (511, 480)),
    # four-wave launches in y as well (NP_y a multiple of 64), one and two components (a two-component FP64
    # 511^2 tile exceeds the LDS, so no batch of it exists to compare with)
    ("fp64", "fisher", (480, 511)), ("fp32", "fhn_cubic", (511, 511))])
def test_product_parallel_2d_matches_fused_stages(etd, precision, reaction, n):
    """Large 2-D single plans run every mode product as a launch of its own;
    a batch of the same single problem runs the fused stage kernels.  Both
    compute every output with the same operations, except that the
    product-parallel launches split each contraction in two halves summed at
    the end (and the compiler fuses a few epilogue multiply-adds): FP64
    results agree to a few units in the last place, FP32 ones within 1e-6."""
    kw = dict(kappa=(1e-3, 1e-4)) if reaction == "fhn_cubic" else dict(kappa=(0.01,), q=0.3)
    p = W.Problem(dim=2, n=n, tau=0.02, reaction=reaction, precision=precision, **kw)
    u0 = W.u0_fhn_patch(p, 3, patch=0.3) if reaction == "fhn_cubic" else W.u0_sine_noise(p, 3)
    st = etd.Stepper(p)
    single = host(st.advance(st.field(u0), 6, 0.1))
    st.close()
    b = etd.Batch([p])
    f = b.fields([u0])
    b.advance(f, 6, t0=0.1)
    fused = host(f[0])
    b.close()
    diff = np.abs(single - fused).max() / np.abs(fused).max()
    print(f"  max rel diff {diff:.2e}")
    assert diff <= (1e-14 if precision == "fp64" else 1e-6)


def test_independent_plans_and_a_batch_on_concurrent_streams(etd):
    """Plans share no mutable device state: two plans and a batch advanced in
    interleaved calls on three streams give, bit for bit, what each gives
    alone on the default stream."""
    import torch
    p3 = W.Problem(dim=3, n=(63, 40, 33), kappa=(0.02,), q=0.3, tau=0.01, reaction="fisher")
    p2 = W.Problem(dim=2, n=(255, 127), kappa=(1e-3, 1e-4), tau=0.05, reaction="fhn_cubic", precision="fp32")
    probs, u0s = mixed_batch("fp32")
    u3 = W.initial_field(p3, "sine_noise", 5)
    u2 = W.initial_field(p2, "fhn_patch", 6)

    def alone():
        a = etd.Stepper(p3)
        b = etd.Stepper(p2)
        c = etd.Batch(probs)
        x, y, z = a.field(u3), b.field(u2), c.fields(u0s)
        a.advance(x, 12)
        b.advance(y, 12)
        c.advance(z, 12)
        torch.cuda.synchronize()
        out = (host(x), host(y), [host(f) for f in z])
        a.close(), b.close(), c.close()
        return out

    ref = alone()
    a, b, c = etd.Stepper(p3), etd.Stepper(p2), etd.Batch(probs)
    x, y, z = a.field(u3), b.field(u2), c.fields(u0s)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(3)]
    for k in range(4):
        with torch.cuda.stream(streams[0]):
            a.advance(x, 3, 3 * k * p3.tau)
        with torch.cuda.stream(streams[1]):
            b.advance(y, 3, 3 * k * p2.tau)
        with torch.cuda.stream(streams[2]):
            c.advance(z, 3, 3 * k * 0.0)
    torch.cuda.synchronize()
    assert np.array_equal(host(x), ref[0])
    assert np.array_equal(host(y), ref[1])
    for got, want in zip(z, ref[2]):
        assert np.array_equal(host(got), want)
    a.close(), b.close(), c.close()


# ---------------------------------------------------------------------------
# the flow schedule: one persistent dataflow launch per step (disabled)
#
# A batch schedule that ran every stage and shape group of a step in ONE
# persistent launch (workgroups taking tiles from a queue; a tile of a later
# stage polling per-instance counters of finished tiles of the stage before)
# did not complete on the GPU: the one-instance 63^2 case below ran past
# 180 s without output, twice (the second time with counter polls that no
# longer invalidate the L2).  The cause is not established, so the schedule
# is not in the library; these tests stay, skipped, for a version whose
# cross-workgroup synchronisation is shown to work.
# ---------------------------------------------------------------------------

FLOW_SKIP = pytest.mark.skip(reason="flow schedule removed: its first runs did not complete (cross-workgroup "
                                    "counter waits never saw the producers' counts; cause not established)")

@FLOW_SKIP
def test_flow_schedule_matches_grouped_launches(etd, oracle_mod):
    """Uneven 2-D FP32 instances (n in {127, 255, 511, 1023}) in one launch per
    call: bit-identical to the grouped per-stage launches (tile shapes change
    no output's arithmetic), and the first instance of each extent against
    the FP64 oracle."""
    probs, u0s, _ = W.batched2d(count=24, nsteps=7)
    b = etd.Batch(probs)
    f = b.fields(u0s)
    b.advance(f, 7, t0=0.05)
    ref = [host(x) for x in f]
    b.set_schedule("flow")
    print(f"  flow tiles {[b.tiles(i)[:2] for i in range(4)]}")
    f = b.fields(u0s)
    b.advance(f, 7, t0=0.05)
    seen = set()
    for i, p in enumerate(probs):
        got = host(f[i])
        assert np.array_equal(got, ref[i]), i
        if p.n[0] not in seen:
            seen.add(p.n[0])
            err = rel_l2(got, oracle_mod.advance(p, u0s[i], 7, t0=0.05))
            print(f"  instance {i} n={p.n[0]}: rel_l2 {err:.2e}")
            assert err <= FP32_TOL
    # back to the grouped schedule: same results again
    b.set_schedule("groups")
    f = b.fields(u0s)
    b.advance(f, 7, t0=0.05)
    for i in range(len(probs)):
        assert np.array_equal(host(f[i]), ref[i]), i
    b.close()


@FLOW_SKIP
@pytest.mark.parametrize("case", [
    ("3d-fhn-fp64", [dict(dim=3, n=(63, 127, 63), kappa=(1e-3, 1e-4), tau=0.02, reaction="fhn_cubic"),
                     dict(dim=3, n=(60, 100, 50), kappa=(2e-3, 3e-4), tau=0.01, reaction="fhn_cubic")]),
    ("3d-mms-fp64", [dict(dim=3, n=(63, 60, 33), kappa=(0.1,), q=0.2, tau=0.01, reaction="ac_mms",
                          rxn_param=(1.0, 0.0))]),
    ("2d-fisher-fp64_bf16x6", [dict(dim=2, n=(255, 127), kappa=(0.01,), q=0.3, tau=0.01, reaction="fisher",
                                    precision="fp64_bf16x6"),
                               dict(dim=2, n=(127, 255), kappa=(0.02,), q=0.1, tau=0.02, reaction="saturating",
                                    precision="fp64_bf16x6")]),
], ids=lambda c: c[0])
def test_flow_schedule_3d_systems_and_time_dependent(etd, oracle_mod, case):
    """3-D two-component, time-dependent forcing and FP64-state reduced-product
    batches in the flow schedule against the oracle, over several steps so
    that every stage waits on the one before it."""
    name, kws = case
    probs = [W.Problem(**kw) for kw in kws]
    b = etd.Batch(probs)
    b.set_schedule("flow")
    u0s = [W.u0_fhn_patch(p, 40 + i, patch=0.4) if p.ncomp == 2 else
           (W.initial_field(p, "sine", 0) * np.exp(-0.3) if p.reaction == "ac_mms" else
            0.5 * W.u0_sine_noise(p, 40 + i)) for i, p in enumerate(probs)]
    f = b.fields(u0s)
    b.advance(f, 9, t0=0.3)
    tol = FP64_TOL if probs[0].precision == "fp64" else FP32_TOL
    for i, p in enumerate(probs):
        err = rel_l2(host(f[i]), oracle_mod.advance(p.replace(precision="fp64"), u0s[i], 9, t0=0.3))
        print(f"  {name} instance {i} n={p.n}: rel_l2 {err:.2e}")
        assert err <= tol, i
    b.close()


@FLOW_SKIP
def test_flow_schedule_small_grid_latency_path(etd, oracle_mod):
    """The 63^2 Fisher-KPP workload as a one-instance batch in the flow
    schedule: all 100 steps in one launch, four-wave tiles; bit-identical to
    the single plan and within 1e-12 of the oracle; replayed from a graph."""
    import torch
    wl = W.fisher2d_small()
    p = wl.problem
    b = etd.Batch([p])
    b.set_schedule("flow")
    f = b.fields([wl.u0()])
    b.advance(f, wl.nsteps)
    got = host(f[0])
    st = etd.Stepper(p)
    single = host(st.advance(st.field(wl.u0()), wl.nsteps))
    st.close()
    err = rel_l2(got, oracle_mod.advance(p, wl.u0(), wl.nsteps))
    print(f"  rel_l2 vs oracle {err:.2e}; tiles {b.tiles(0)[:4]}")
    assert err <= FP64_TOL
    assert np.array_equal(got, single)
    s = torch.cuda.Stream()
    g_f = b.fields([wl.u0()])
    torch.cuda.synchronize()
    g = b.capture(g_f, wl.nsteps, s)
    for r in range(3):
        for x in g_f:
            x.copy_(torch.as_tensor(wl.u0().reshape(p.shape), device=x.device))
        torch.cuda.synchronize()
        g.launch(s)
        s.synchronize()
        assert np.array_equal(host(g_f[0]), got), r
    g.close()
    b.close()


@FLOW_SKIP
def test_flow_schedule_refused_where_no_wave_count_fits(etd):
    """Padded extents 32 and 96 fit no common W in {8, 4}; the batch keeps its
    grouped schedule."""
    probs = [W.Problem(dim=2, n=(31, 95), kappa=(0.01,), tau=0.01, reaction="fisher")]
    b = etd.Batch(probs)
    with pytest.raises(etd.EtdError) as ei:
        b.set_schedule("flow")
    assert ei.value.status == etd.ETD_EUNSUPPORTED
    f = b.fields([W.u0_sine_noise(probs[0], 1)])
    b.advance(f, 2)
    assert np.isfinite(host(f[0])).all()
    b.close()
