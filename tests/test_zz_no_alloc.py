"""etd_compare_noalloc (partials in the library's fixed device array, results
written to a device buffer) against etd_compare (workspace partials, results
copied to the host): the same four values, bit for bit, on two calls in a row
whose second field is smaller, in FP64 and FP32 element types."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_compare_noalloc_matches_compare(precision):
    import torch
    import paper_2601_06849_amd as etd

    cases = [W.Problem(dim=3, n=(95, 70, 41), kappa=(0.01,), q=0.3, tau=0.01, reaction="fisher",
                       precision=precision),
             W.Problem(dim=2, n=(33, 20), kappa=(0.02,), q=0.0, tau=0.01, reaction="fisher",
                       precision=precision)]
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    for k, p in enumerate(cases):
        print(f"compare_noalloc case {k}: {p.n} {precision}", flush=True)
        st = etd.Stepper(p)
        rng = np.random.default_rng(123 + k)
        a0 = rng.standard_normal(p.shape)
        b0 = a0 + 1e-3 * rng.standard_normal(p.shape)
        a, b = st.field(a0), st.field(b0)
        ref = st.compare(a, b)
        out.fill_(float("nan"))
        etd.etd_compare_noalloc(st.plan, a, b, out, st.stream)
        torch.cuda.synchronize()
        got = tuple(out.cpu().tolist())
        assert got == ref, (k, got, ref)
        # and against a host reduction of the same device values
        ah, bh = a.cpu().double().numpy(), b.cpu().double().numpy()
        assert got[0] == pytest.approx(np.linalg.norm(ah - bh), rel=1e-12)
        assert got[1] == pytest.approx(np.linalg.norm(bh), rel=1e-12)
        assert got[2] == pytest.approx(np.abs(ah - bh).max(), rel=1e-15)
        assert got[3] == 0.0
        st.close()


def test_compare_noalloc_counts_nonfinite():
    import torch
    import paper_2601_06849_amd as etd

    p = W.Problem(dim=2, n=(40, 31), kappa=(0.02,), q=0.0, tau=0.01, reaction="fisher", precision="fp64")
    st = etd.Stepper(p)
    a0 = np.ones(p.shape)
    a0.flat[7] = np.nan
    a0.flat[100] = np.inf
    a, b = st.field(a0), st.field(np.zeros(p.shape))
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    etd.etd_compare_noalloc(st.plan, a, b, out, st.stream)
    torch.cuda.synchronize()
    got = out.cpu().tolist()
    ref = st.compare(a, b, allow_nonfinite=True)
    assert tuple(got) == ref
    assert got[3] == 2.0 and got[2] == 1.0
    st.close()
