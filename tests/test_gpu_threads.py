"""Plans driven from several host threads at once (each on its own stream)
give the same fields, bit for bit, as the same plans run one after another:
the library's per-kernel launch caches are shared across threads."""
import threading

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


CASES = [
    (3, (40, 31, 50), "fp64", "fisher"), (3, (33, 64, 20), "fp32", "fhn_cubic"),
    (3, (30, 30, 30), "bf16x6", "fisher"), (2, (70, 41), "fp64_fp32", "fhn_classic"),
    (2, (300, 520), "fp64", "fisher"), (2, (63, 63), "fp64_bf16x6", "allen_cahn"),
]


def problem(dim, n, prec, rxn):
    params = {"fisher": (1.0,), "fhn_cubic": (0.1, 0.01, 0.5), "fhn_classic": (1.0, 1.0), "allen_cahn": ()}[rxn]
    kappa = (0.01, 0.002) if rxn.startswith("fhn") else (0.02,)
    return W.Problem(dim=dim, n=n, kappa=kappa, q=0.2, tau=0.01, reaction=rxn, rxn_param=params, precision=prec)


def test_plans_on_concurrent_host_threads(etd):
    import torch
    probs = [problem(*c) for c in CASES]
    u0s = [W.u0_random(p, seed=11 + i, lo=0.0, hi=1.0) for i, p in enumerate(probs)]
    serial = []
    for p, u0 in zip(probs, u0s):
        st = etd.Stepper(p)
        u = st.field(u0)
        st.advance(u, 12)
        torch.cuda.synchronize()
        serial.append(u.cpu().numpy())
        st.close()
    for rep in range(3):
        streams = [torch.cuda.Stream() for _ in probs]
        steppers = [etd.Stepper(p, stream=s) for p, s in zip(probs, streams)]
        fields = [st.field(u0) for st, u0 in zip(steppers, u0s)]
        torch.cuda.synchronize()
        errors = []

        def run(i):
            try:
                for _ in range(3):
                    steppers[i].advance(fields[i], 4)
            except Exception as e:   # reported below
                errors.append((i, e))

        threads = [threading.Thread(target=run, args=(i,)) for i in range(len(probs))]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        torch.cuda.synchronize()
        assert not errors, errors
        for i, (f, ref) in enumerate(zip(fields, serial)):
            assert np.array_equal(f.cpu().numpy(), ref), (rep, CASES[i])
        for st in steppers:
            st.close()
