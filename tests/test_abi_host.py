"""Host-side checks of the C ABI: the library loads and exports every entry
point the header declares; plan construction (host FP64, no GPU) builds the
closed-form eigenpairs and the rational factors of Sec. 3.3.2 / Sec. 3.1
correctly; malformed arguments are rejected on the host before any device
work."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def etd():
    import paper_2601_06849_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_2601_06849_amd import build
        build.build()
    m.lib()
    return m


def declared_functions():
    src = open(os.path.join(ROOT, "include", "etdds.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(etd_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(etd):
    names = declared_functions()
    assert len(names) >= 9
    L = ctypes.CDLL(etd.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(etd.EXPORTS)


def dense_stencil(p, d, c=0):
    n, h, k = p.n[d], p.h(d), p.kappa[c]
    A = np.diag(np.full(n, (2 * k + p.q * h * h / p.dim) / h ** 2))
    A += np.diag(np.full(n - 1, -k / h ** 2), 1) + np.diag(np.full(n - 1, -k / h ** 2), -1)
    return A


def q_poly(pade, ell, x):
    if pade == 2:
        den = x * x + 2 * x + 2
        return {1: 2 / den, 2: (x + 2) / den, 3: (x + 1) / den}[ell]
    den = x ** 4 + 4 * x ** 3 + 12 * x ** 2 + 24 * x + 24
    return {1: 24 / den, 2: (x ** 3 + 4 * x ** 2 + 12 * x + 24) / den, 3: (x ** 3 + 3 * x ** 2 + 8 * x + 12) / den}[ell]


@pytest.mark.parametrize("pade", [2, 4])
def test_plan_tables_match_dense_eigendecomposition(etd, pade):
    p = W.Problem(dim=3, n=(17, 40, 9), kappa=(0.3, 2.0), q=0.9, tau=0.02, reaction="fhn_cubic", pade=pade,
                  lo=(0.0, -1.0, 0.5), hi=(2.0, 1.5, 1.0))
    plan = etd.etd_plan_create(p)
    try:
        for d in range(3):
            n = p.n[d]
            P = etd.etd_plan_table(plan, 1, d, 0, n * n).reshape(n, n)
            assert np.abs(P @ P.T - np.eye(n)).max() < 1e-14 * n
            assert np.abs(P - P.T).max() == 0.0
            for c in range(2):
                A = dense_stencil(p, d, c)
                lam = etd.etd_plan_table(plan, 0, d, c, n)
                # A P = P diag(lam) and the spectrum equals the dense one
                assert np.abs(A @ P - P * lam).max() < 1e-12 * np.abs(A).max()
                assert np.allclose(np.sort(lam), np.linalg.eigvalsh(A), rtol=1e-12, atol=1e-12)
                for ell in (1, 2, 3):
                    qv = etd.etd_plan_table(plan, 1 + ell, d, c, n)
                    assert np.allclose(qv, q_poly(pade, ell, p.tau * lam), rtol=1e-14, atol=0)
                    # the operator P diag(q) P^T equals Q_ell(tau A) from its polynomial definition
                    M = p.tau * A
                    I = np.eye(n)
                    if pade == 2:
                        den = M @ M + 2 * M + 2 * I
                        num = {1: 2 * I, 2: M + 2 * I, 3: M + I}[ell]
                    else:
                        M2 = M @ M
                        den = M2 @ M2 + 4 * M2 @ M + 12 * M2 + 24 * M + 24 * I
                        num = {1: 24 * I, 2: M2 @ M + 4 * M2 + 12 * M + 24 * I,
                               3: M2 @ M + 3 * M2 + 8 * M + 12 * I}[ell]
                    assert np.abs((P * qv) @ P.T - np.linalg.solve(den, num)).max() < 1e-12
    finally:
        etd.etd_plan_destroy(plan)


def test_rational_factors_bounded(etd):
    """0 < Q1 <= 1, 0 < Q2 <= 1, 0 < Q3 <= 1/2 at tau*lambda >= 0 (Prop. 4.3)."""
    p = W.Problem(dim=2, n=(200, 3), kappa=(5.0,), q=0.2, tau=0.5, reaction="fisher")
    plan = etd.etd_plan_create(p)
    try:
        q1, q2, q3 = (etd.etd_plan_table(plan, w, 0, 0, 200) for w in (2, 3, 4))
        assert np.all((q1 > 0) & (q1 <= 1)) and np.all((q2 > 0) & (q2 <= 1)) and np.all((q3 > 0) & (q3 <= 0.5))
    finally:
        etd.etd_plan_destroy(plan)


BAD = [
    dict(dim=4),
    dict(ncomp=3),
    dict(tau=0.0),
    dict(tau=float("nan")),
    dict(kappa0=-1.0),
    dict(q=-0.5),
    dict(n0=0),
    dict(pade=3),
    dict(precision=7),
    dict(rxn=42),
    dict(rxn=6),          # FitzHugh-Nagumo with one component
    dict(hi0=0.0),        # empty box
]


@pytest.mark.parametrize("mod", BAD, ids=lambda m: ",".join(m))
def test_plan_rejects_malformed_problem(etd, mod):
    s = etd.problem_struct(W.Problem(dim=2, n=(10, 12), kappa=(0.1,), tau=0.01, reaction="fisher"))
    for k, v in mod.items():
        if k == "kappa0":
            s.kappa[0] = v
        elif k == "n0":
            s.n[0] = v
        elif k == "hi0":
            s.hi[0] = v
        else:
            setattr(s, k, v)
    with pytest.raises(etd.EtdError) as ei:
        etd.etd_plan_create(s)
    assert ei.value.status == etd.ETD_EINVAL


@pytest.mark.parametrize("n,precision", [((1100, 10), "fp32"), ((10, 700), "fp64"), ((700, 10), "fp64")])
def test_plan_reports_unsupported_sizes(etd, n, precision):
    """Padded extents beyond 1024, or an FP64 tile of one component beyond the
    LDS budget (extents above 576), are reported as unsupported."""
    p = W.Problem(dim=2, n=n, kappa=(0.1,), tau=0.01, reaction="fisher", precision=precision)
    with pytest.raises(etd.EtdError) as ei:
        etd.etd_plan_create(p)
    assert ei.value.status == etd.ETD_EUNSUPPORTED


@pytest.mark.parametrize("n,precision", [((1023, 1023), "fp32"), ((576, 576), "fp64"), ((511, 511), "fp64")])
def test_plan_accepts_large_supported_sizes(etd, n, precision):
    p = W.Problem(dim=2, n=n, kappa=(0.1, 0.2), tau=0.01, reaction="fhn_cubic", precision=precision)
    plan = etd.etd_plan_create(p)
    etd.etd_plan_destroy(plan)


def test_host_side_argument_errors_touch_nothing(etd):
    """Workspace and step-count errors are caught before any HIP call, so fake
    device addresses are never dereferenced."""
    L = etd.lib()
    p = W.Problem(dim=2, n=(31, 31), kappa=(0.1,), tau=0.01, reaction="fisher")
    plan = etd.etd_plan_create(p)
    try:
        nbytes = etd.etd_plan_workspace_bytes(plan)
        assert nbytes > 0 and nbytes % 256 == 0
        fake_u = ctypes.c_void_p(0x1000)
        misaligned = ctypes.c_void_p(0x1008)
        assert L.etd_advance(plan, fake_u, 0.0, 1, misaligned, None) == etd.ETD_EWORKSPACE
        assert L.etd_advance(plan, fake_u, 0.0, 1, None, None) == etd.ETD_EWORKSPACE
        assert L.etd_advance(plan, fake_u, 0.0, -1, ctypes.c_void_p(0x10000), None) == etd.ETD_EINVAL
        assert L.etd_advance(plan, None, 0.0, 1, ctypes.c_void_p(0x10000), None) == etd.ETD_EINVAL
        assert L.etd_advance(plan, fake_u, float("inf"), 1, ctypes.c_void_p(0x10000), None) == etd.ETD_EINVAL
        assert L.etd_advance(None, fake_u, 0.0, 1, ctypes.c_void_p(0x10000), None) == etd.ETD_EINVAL
        # nsteps = 0 is a no-op that returns before touching the device
        assert L.etd_advance(plan, fake_u, 0.0, 0, ctypes.c_void_p(0x10000), None) == etd.ETD_OK
        assert L.etd_plan_upload(plan, ctypes.c_void_p(0x10000), nbytes - 1, None) == etd.ETD_EWORKSPACE
        assert "smaller" in etd.etd_last_error()
        # an aligned workspace that etd_plan_upload never filled for this plan
        ws = ctypes.c_void_p(0x10000)
        assert L.etd_advance(plan, fake_u, 0.0, 1, ws, None) == etd.ETD_EWORKSPACE
        assert "not uploaded" in etd.etd_last_error()
        out = (ctypes.c_double * 4)()
        assert L.etd_compare(plan, fake_u, fake_u, out, ws, None) == etd.ETD_EWORKSPACE
        assert L.etd_plan_autotune(plan, ws, None) == etd.ETD_EWORKSPACE
        g = (ctypes.c_double * 2)()
        assert L.etd_adjoint(plan, fake_u, 0.0, 2, fake_u, fake_u, g, ws, ws, 1 << 30, None) == etd.ETD_EWORKSPACE
        h = ctypes.c_void_p()
        assert L.etd_graph_capture(plan, fake_u, 0.0, 1, ws, ctypes.c_void_p(0x20), ctypes.byref(h)) == \
            etd.ETD_EWORKSPACE
        assert etd.etd_status_string(etd.ETD_EWORKSPACE) == "bad workspace"
    finally:
        etd.etd_plan_destroy(plan)


def test_adjoint_workspace_query(etd):
    """The adjoint's tiles hold four fields of one component: FP64-state
    systems fit up to 288 points per direction, FP32-state ones up to 576
    (the forward x tile of two components must also fit, for the replay)."""
    ok = W.Problem(dim=3, n=(127, 127, 127), kappa=(1e-4, 1e-5), tau=0.02, reaction="fhn_cubic", precision="fp32")
    plan = etd.etd_plan_create(ok)
    try:
        n1 = etd.etd_adjoint_workspace_bytes(plan, 400)
        n2 = etd.etd_adjoint_workspace_bytes(plan, 100)
        assert n1 > n2 > 0
        with pytest.raises(etd.EtdError) as ei:
            etd.etd_adjoint_workspace_bytes(plan, 0)
        assert ei.value.status == etd.ETD_EINVAL
        # checkpoint segments of 20 (the shortest) to 400 steps (one forward
        # pass keeping five stage fields and the state of every step)
        assert etd.etd_adjoint_workspace_bytes_segment(plan, 400, 20) == n1
        full = etd.etd_adjoint_workspace_bytes_segment(plan, 400, 400)
        field = 2 * 128 ** 3 * 4
        assert 6 * 400 * field < full < 6 * 400 * field + 16 * field
        for bad in (19, 401, -1):
            with pytest.raises(etd.EtdError) as ei:
                etd.etd_adjoint_workspace_bytes_segment(plan, 400, bad)
            assert ei.value.status == etd.ETD_EINVAL
    finally:
        etd.etd_plan_destroy(plan)
    for prec, n_ok, n_big in (("fp64", (255, 40, 288), (300, 40, 40)), ("fp64_fp32", (288, 255, 30), (30, 320, 30)),
                              ("fp32", (511, 40, 576), (40, 640, 40)), ("bf16x6", (576, 30, 30), (30, 30, 700))):
        for n, good in ((n_ok, True), (n_big, False)):
            plan = etd.etd_plan_create(ok.replace(n=n, precision=prec))
            try:
                if good:
                    assert etd.etd_adjoint_workspace_bytes(plan, 10) > 0
                else:
                    with pytest.raises(etd.EtdError) as ei:
                        etd.etd_adjoint_workspace_bytes(plan, 10)
                    assert ei.value.status == etd.ETD_EUNSUPPORTED
            finally:
                etd.etd_plan_destroy(plan)


def test_tile_shapes_host_validation(etd):
    """Tile requests are validated on the host: default shapes are reported,
    invalid ones rejected without changing the plan."""
    p = W.Problem(dim=3, n=(255, 100, 1000), kappa=(0.1,), tau=0.01, reaction="fisher", precision="fp32")
    plan = etd.etd_plan_create(p)
    try:
        d = etd.etd_plan_tiles(plan)
        assert d == [(2, 4), (2, 2), (4, 1)]
        etd.etd_plan_set_tiles(plan, [(4, 1), (2, 1), (4, 1)])
        assert etd.etd_plan_tiles(plan) == [(4, 1), (2, 1), (4, 1)]
        for bad in ([(2, 8)], [(3, 1)], [(2, 1), (2, 1), (2, 1)], [(2, 1), (2, 4)]):
            with pytest.raises(etd.EtdError) as ei:
                etd.etd_plan_set_tiles(plan, bad)
            assert ei.value.status == etd.ETD_EUNSUPPORTED
        assert etd.etd_plan_tiles(plan) == [(4, 1), (2, 1), (4, 1)]
        # eight row blocks per wave: one column block, FP32 states only
        etd.etd_plan_set_tiles(plan, [(4, 1), (2, 1), (8, 1)])
        assert etd.etd_plan_tiles(plan) == [(4, 1), (2, 1), (8, 1)]
        for bad in ([(4, 1), (2, 1), (8, 2)], [(8, 2)], [(8, 4)]):
            with pytest.raises(etd.EtdError) as ei:
                etd.etd_plan_set_tiles(plan, bad)
            assert ei.value.status == etd.ETD_EUNSUPPORTED
        assert etd.etd_plan_tiles(plan) == [(4, 1), (2, 1), (8, 1)]
        etd.etd_plan_set_tiles(plan, [(0, 0)] * 3)
        assert etd.etd_plan_tiles(plan) == d
    finally:
        etd.etd_plan_destroy(plan)
    p64 = p.replace(n=(255, 96, 64), precision="fp64")
    plan = etd.etd_plan_create(p64)
    try:
        assert etd.etd_plan_tiles(plan) == [(1, 2), (1, 2), (1, 2)]
        for bad in ([(4, 1)], [(8, 1)]):   # rb = 4 at <= 8 waves and rb = 8: FP32 states only
            with pytest.raises(etd.EtdError) as ei:
                etd.etd_plan_set_tiles(plan, bad)
            assert ei.value.status == etd.ETD_EUNSUPPORTED
    finally:
        etd.etd_plan_destroy(plan)


def test_schedule_host_validation(etd):
    """The resident schedule (all steps in one cooperative launch) applies to
    grids whose directions share one padded extent of at most 128; AUTO is
    the per-stage schedule."""
    cases = [((63, 63), True), ((64, 50), True), ((127, 120), True), ((1, 1), True), ((63, 63, 63), True),
             ((31, 20, 17), True), ((127, 127, 127), True),
             ((63, 65), False), ((255, 255), False), ((63, 63, 80), False), ((255, 255, 255), False)]
    for n, eligible in cases:
        p = W.Problem(dim=len(n), n=n, kappa=(0.01,), tau=0.01, reaction="fisher")
        plan = etd.etd_plan_create(p)
        try:
            assert etd.etd_plan_schedule(plan) == "stages", n
            etd.etd_plan_set_schedule(plan, "stages")
            assert etd.etd_plan_schedule(plan) == "stages"
            if eligible:
                etd.etd_plan_set_schedule(plan, "resident")
                assert etd.etd_plan_schedule(plan) == "resident"
            else:
                with pytest.raises(etd.EtdError) as ei:
                    etd.etd_plan_set_schedule(plan, "resident")
                assert ei.value.status == etd.ETD_EUNSUPPORTED
                assert etd.etd_plan_schedule(plan) == "stages"      # unchanged
            etd.etd_plan_set_schedule(plan, "auto")
            assert etd.etd_plan_schedule(plan) == "stages"
            for bad in (-1, 3, 7):
                with pytest.raises(etd.EtdError) as ei:
                    etd.etd_plan_set_schedule(plan, bad)
                assert ei.value.status == etd.ETD_EINVAL
            assert etd.etd_plan_schedule(plan) == "stages"
        finally:
            etd.etd_plan_destroy(plan)


def test_small_grid_default_tiles(etd):
    """A launch of at most 256 one-block tiles takes one row block per wave
    over one block (the larger default tiles would leave CUs idle); a batch
    group counts the tiles of all its instances."""
    for n, prec in (((63, 63), "fp64"), ((255, 255), "fp64"), ((63, 63, 63), "fp32"), ((31, 31), "bf16x6"),
                    ((63, 63), "fp64_fp32"), ((127, 63), "fp64_bf16x6")):
        p = W.Problem(dim=len(n), n=n, kappa=(0.01,), tau=0.01, reaction="fisher", precision=prec)
        plan = etd.etd_plan_create(p)
        try:
            assert etd.etd_plan_tiles(plan)[:len(n)] == [(1, 1)] * len(n), (n, prec)
        finally:
            etd.etd_plan_destroy(plan)
    p = W.Problem(dim=3, n=(255, 255, 255), kappa=(0.01,), tau=0.01, reaction="fisher")
    plan = etd.etd_plan_create(p)
    try:
        assert etd.etd_plan_tiles(plan) == [(1, 2), (1, 2), (1, 2)]
    finally:
        etd.etd_plan_destroy(plan)
    # 300 instances of 63^2: 1200 tiles per stage launch, so the group keeps the larger tiles
    probs = [W.Problem(dim=2, n=(63, 63), kappa=(0.01,), tau=0.01, reaction="fisher")] * 300
    b = etd.etd_batch_create(probs)
    try:
        assert etd.etd_batch_tiles(b, 0)[:2] == [(1, 2), (1, 2)]
    finally:
        etd.etd_batch_destroy(b)


def test_fp32_512_point_defaults(etd):
    """FP32-product, one-component plans take four row blocks over two line
    blocks in x stages of 512 padded points; outer stages of 512 points and
    FP64 states keep their shapes."""
    for n, prec, want in (((511, 100, 40), "fp32", [(4, 2), (2, 2), (2, 2)]),
                          ((100, 64, 511), "fp32", [(2, 4), (2, 2), (2, 1)]),
                          ((511, 100, 40), "fp64_fp32", [(2, 1), (2, 1), (2, 1)]),
                          ((511, 100, 40), "fp64", [(2, 1), (1, 2), (1, 2)]),
                          ((100, 64, 511), "fp64", [(1, 2), (1, 2), (2, 1)])):
        p = W.Problem(dim=3, n=n, kappa=(0.01,), tau=0.01, reaction="fisher", precision=prec)
        plan = etd.etd_plan_create(p)
        try:
            assert etd.etd_plan_tiles(plan) == want, (n, prec, etd.etd_plan_tiles(plan))
        finally:
            etd.etd_plan_destroy(plan)


def test_batch_fp32_x_tiles_follow_tile_count(etd):
    """Batch groups of FP32 instances with fewer than 1024 four-block x tiles
    take two line blocks; larger groups and single grids keep four."""
    for n, count, want in ((255, 96, (2, 2)), (127, 48, (2, 2)), (255, 300, (2, 4))):
        ps = [W.Problem(dim=2, n=(n, n), kappa=(0.01,), tau=0.01, reaction="fisher", precision="fp32")
              for _ in range(count)]
        b = etd.etd_batch_create(ps)
        try:
            assert etd.etd_batch_tiles(b, 0)[0] == want, (n, count, etd.etd_batch_tiles(b, 0))
        finally:
            etd.etd_batch_destroy(b)
    p = W.Problem(dim=3, n=(255, 127, 127), kappa=(0.01,), tau=0.01, reaction="fisher", precision="fp32")
    plan = etd.etd_plan_create(p)
    try:
        assert etd.etd_plan_tiles(plan)[0] == (2, 4)
    finally:
        etd.etd_plan_destroy(plan)


def test_one_array_x_tile_default(etd):
    """FP32-product, one-component plans whose x lines are too long for a
    two-array tile of two line blocks default to the one-array (8, 2) tile;
    it is valid nowhere else."""
    for n, prec, want in (((1023, 100, 40), "fp32", (8, 2)), ((767, 64, 40), "fp32", (8, 2)),
                          ((1023, 100, 40), "bf16x6", None), ((255, 100, 40), "fp32", None),
                          ((511, 100, 40), "fp64_fp32", None)):
        p = W.Problem(dim=3, n=n, kappa=(0.01,), tau=0.01, reaction="fisher", precision=prec)
        plan = etd.etd_plan_create(p)
        try:
            x = etd.etd_plan_tiles(plan)[0]
            if want:
                assert x == want, (n, prec, x)
            else:
                assert x != (8, 2), (n, prec)
                if prec != "bf16x6":
                    with pytest.raises(etd.EtdError) as ei:
                        etd.etd_plan_set_tiles(plan, [(8, 2)])
                    assert ei.value.status == etd.ETD_EUNSUPPORTED
        finally:
            etd.etd_plan_destroy(plan)
    p = W.Problem(dim=3, n=(1023, 100, 40), kappa=(0.01, 0.001), tau=0.01, reaction="fhn_cubic", precision="fp32")
    plan = etd.etd_plan_create(p)
    try:
        with pytest.raises(etd.EtdError) as ei:
            etd.etd_plan_set_tiles(plan, [(8, 2)])
        assert ei.value.status == etd.ETD_EUNSUPPORTED
    finally:
        etd.etd_plan_destroy(plan)


def test_bench_refuses_more_than_one_gpu():
    """The benchmark is a one-GPU measurement: --gpus above 1 exits with a
    message (before anything touches a device)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_batch_host_validation(etd):
    """Batches: grouping by padded shape, shared limits and host-side errors."""
    a = W.Problem(dim=2, n=(100, 100), kappa=(0.1,), tau=0.01, reaction="fisher")
    probs = [a, a.replace(n=(97, 100), q=0.5), a.replace(n=(127, 100)),
             a.replace(n=(100, 140), pade=4, reaction="allen_cahn")]
    b = etd.etd_batch_create(probs)
    try:
        assert etd.etd_batch_groups(b) == 2          # 97, 100, 127 pad to 128; 140 to 160
        assert etd.etd_batch_workspace_bytes(b) % 256 == 0
        assert etd.etd_batch_tiles(b, 0) == etd.etd_batch_tiles(b, 1)
        with pytest.raises(etd.EtdError):
            etd.etd_batch_tiles(b, 4)
        L = etd.lib()
        ptrs = (ctypes.c_void_p * 4)(0x1000, 0x2000, 0x3000, 0x4000)
        # not uploaded: every workspace is rejected before any device work
        assert L.etd_batch_advance(b, ptrs, 0.0, 1, ctypes.c_void_p(0x10000), None) == etd.ETD_EWORKSPACE
        ptrs[2] = None
        assert L.etd_batch_advance(b, ptrs, 0.0, 1, ctypes.c_void_p(0x10000), None) == etd.ETD_EINVAL
        h = ctypes.c_void_p()
        assert L.etd_batch_graph_capture(b, ptrs, 0.0, 1, ctypes.c_void_p(0x10000), None, ctypes.byref(h)) == \
            etd.ETD_EINVAL   # the null stream cannot be captured
    finally:
        etd.etd_batch_destroy(b)
    for bad in ([a, a.replace(precision="fp32")], [a, a.replace(dim=3, n=(10, 10, 10))], []):
        with pytest.raises((etd.EtdError, ValueError)) as ei:
            etd.etd_batch_create(bad)
    with pytest.raises(etd.EtdError) as ei:
        etd.etd_batch_create([a, a.replace(tau=-1.0)])
    assert "instance 1" in str(ei.value)
    fhn = W.Problem(dim=2, n=(700, 32), kappa=(0.1, 0.1), tau=0.01, reaction="fhn_cubic", precision="fp32")
    with pytest.raises(etd.EtdError) as ei:
        etd.etd_batch_create([fhn])
    assert ei.value.status == etd.ETD_EUNSUPPORTED


def _phi_decimal(z, ell):
    """Q_1 - 1, Q_2 - 1, Q_3 - 1/2 of the exact family at z, to 50 digits."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    Z = Decimal(float(z))   # the exact binary value
    # e^{-z} by its Taylor series with argument halving
    k = 0
    while Z / (2 ** k) > 1:
        k += 1
    x = -Z / (2 ** k)
    term, e = Decimal(1), Decimal(1)
    for i in range(1, 80):
        term *= x / i
        e += term
    for _ in range(k):
        e *= e
    if ell == 1:
        return e - 1
    if ell == 2:
        return (1 - e) / Z - 1
    return (Z - 1 + e) / (Z * Z) - Decimal("0.5")


def test_exact_exponential_increments_to_full_precision(etd):
    """The exact-exponential increments (expm1 and series) against 50-digit
    decimal arithmetic, from tau*lambda = 1e-9 to 60, within a few ulps (a
    cancelling closed form would lose up to all digits as tau*lambda -> 0)."""
    for tau in (1e-10, 1e-6, 1e-3, 0.05, 2.0):
        p = W.Problem(dim=2, n=(40, 3), kappa=(0.7,), q=0.3, tau=tau, reaction="fisher", pade=0)
        plan = etd.etd_plan_create(p)
        try:
            lam = etd.etd_plan_table(plan, 0, 0, 0, 40)
            for ell in (1, 2, 3):
                got = etd.etd_plan_table(plan, 4 + ell, 0, 0, 40)
                for j in range(0, 40, 3):
                    ref = float(_phi_decimal(tau * lam[j], ell))
                    assert abs(got[j] - ref) <= 1e-15 * abs(ref), (tau, j, ell, got[j], ref)
        finally:
            etd.etd_plan_destroy(plan)


def test_exact_exponential_tables_match_block_expm(etd, oracle_mod):
    """P diag(Q_l) P^T equals e^{-tau A}, phi_1(tau A), phi_2(tau A) formed by
    the oracle from one block matrix exponential."""
    from oracle import phi
    p = W.Problem(dim=2, n=(30, 17), kappa=(0.4, 2.0), q=0.9, tau=0.03, reaction="fhn_cubic", pade=0,
                  lo=(0.0, -1.0, 0.0), hi=(2.0, 1.5, 1.0))
    plan = etd.etd_plan_create(p)
    try:
        for d in range(2):
            n = p.n[d]
            P = etd.etd_plan_table(plan, 1, d, 0, n * n).reshape(n, n)
            for c in range(2):
                ref = phi.phi_matrices(phi.stencil(p, d, c), p.tau)
                for ell in (1, 2, 3):
                    qv = etd.etd_plan_table(plan, 1 + ell, d, c, n)
                    assert np.abs((P * qv) @ P.T - ref[ell - 1]).max() < 1e-13
    finally:
        etd.etd_plan_destroy(plan)


def test_missing_library_fails_loudly():
    """Without the built HIP library the package raises; there is no fallback."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import paper_2601_06849_amd as m\n"
            "m.LIB_PATH = '/nonexistent/libetdds.so'\n"
            "try:\n    m.lib()\nexcept RuntimeError as e:\n    print('raised:', e)\nelse:\n    print('loaded')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("raised:") and "missing" in r.stdout


def test_product_path_never_touches_the_oracle():
    """The package (Python binding and HIP sources) neither imports nor links
    the oracle: the two share no code."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_2601_06849_amd")
    files = [os.path.join(pkg, f) for f in os.listdir(pkg) if f.endswith(".py")]
    files += [os.path.join(pkg, "csrc", f) for f in os.listdir(os.path.join(pkg, "csrc"))]
    for f in files:
        text = open(f).read()
        assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), f
        assert "etdo" not in text, f
        assert "oracle/" not in text, f


def test_batch_holds_one_p_per_extent(etd):
    """Instances that borrow every direction's P hold no copy: a batch of k
    equal instances needs k plan workspaces minus (k - 1) P tables."""
    p = W.Problem(dim=2, n=(255, 255), kappa=(0.01,), tau=0.01, reaction="fisher", precision="fp32")
    plan = etd.etd_plan_create(p)
    try:
        single = etd.etd_plan_workspace_bytes(plan)
    finally:
        etd.etd_plan_destroy(plan)
    p_bytes = 2 * 256 * 256 * 4          # P_x and P_y of one instance
    for k in (1, 3):
        b = etd.etd_batch_create([p] * k)
        try:
            total = etd.etd_batch_workspace_bytes(b)
        finally:
            etd.etd_batch_destroy(b)
        assert total % 256 == 0
        # k regions, the last k - 1 without their P tables, plus the descriptor table (< 64 KiB here)
        assert k * single - (k - 1) * p_bytes <= total < k * single - (k - 1) * p_bytes + 65536


def test_plan_problem_round_trip(etd):
    """etd_plan_problem returns the problem the plan was built from."""
    p = W.Problem(dim=3, n=(20, 14, 17), kappa=(0.01, 0.003), q=0.2, tau=0.05, reaction="fhn_classic",
                  rxn_param=(0.7, 1.2), precision="fp32", pade=4)
    plan = etd.etd_plan_create(p)
    try:
        got = etd.etd_plan_problem(plan)
        ref = etd.problem_struct(p)
        assert bytes(got) == bytes(ref)
    finally:
        etd.etd_plan_destroy(plan)


def test_binding_rejects_host_and_mismatched_tensors(etd):
    """The binding checks every tensor before any library call: host tensors,
    a wrong element type or a wrong size raise ValueError (no device needed,
    so no fake address ever reaches a kernel)."""
    import torch
    p = W.Problem(dim=2, n=(31, 33), kappa=(0.1,), tau=0.01, reaction="fisher", precision="fp32")
    plan = etd.etd_plan_create(p)
    try:
        host = torch.zeros(p.shape, dtype=torch.float32)
        with pytest.raises(ValueError, match="device tensor"):
            etd.etd_advance(plan, host, 0.0, 1, host)
        with pytest.raises(ValueError, match="device tensor"):
            etd.etd_compare(plan, host, host, host)
        n, dt = etd._field_spec(plan)
        assert n == 31 * 33 and dt == torch.float32
    finally:
        etd.etd_plan_destroy(plan)
