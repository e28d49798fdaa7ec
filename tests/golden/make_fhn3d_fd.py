"""Write fhn3d_n127_fd.json: central finite differences of the CPU oracle's
forward map for the 3-D FitzHugh-Nagumo gradient workload (127^3, two
components, tau = 0.02, all 400 steps), the expected values of the adjoint
tests.  Calls the oracle only (FP64, complex Thomas line solves).

Loss L = 1/2 ||u_N(kappa_u, kappa_v, q, u0) - u_target||^2, u_target the
oracle's u_N at 1.1 kappa_u.  Loss differences are formed from field
differences, L(a) - L(b) = sum (u_a - u_b) ((u_a + u_b)/2 - u_target), which
is exact.  kappa_u, kappa_v and the u0 direction (seeded standard normal
field) take central differences with relative step 1e-4 (truncation ~1e-8 of
the derivative); q = 0 is the edge of its domain, so dL/dq takes the
second-order one-sided difference (4 (L(k) - L(0)) - (L(2k) - L(0))) / (2k)
with k = 1e-6.  About 10 oracle runs of 400 steps (~10 min on 8 cores).

Run from the repository root:  python tests/golden/make_fhn3d_fd.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "fhn3d_n127_fd.json")
H_REL = 1e-4
H_Q = 1e-6
H_U0 = 1e-4
DIR_SEED = 20260105


def main():
    wl = W.fhn3d()
    p = wl.problem.replace(precision="fp64")
    N = wl.nsteps
    u0 = wl.u0()
    t_start = time.time()

    def run(pp, uu):
        t0 = time.time()
        out = oracle.advance(pp, uu, N)
        print(f"  oracle run {time.time() - t0:.1f} s", flush=True)
        return out

    target = run(p.replace(kappa=(p.kappa[0] * 1.1, p.kappa[1])), u0)

    def dL(ua, ub):
        return float(((ua - ub) * (0.5 * (ua + ub) - target)).sum())

    base = run(p, u0)
    rows = {}
    for c in range(p.ncomp):
        h = H_REL * p.kappa[c]
        kp, km = list(p.kappa), list(p.kappa)
        kp[c] += h
        km[c] -= h
        up, um = run(p.replace(kappa=tuple(kp)), u0), run(p.replace(kappa=tuple(km)), u0)
        rows[f"kappa{c}"] = dL(up, um) / (2 * h)
    assert p.q == 0.0
    u1, u2 = run(p.replace(q=H_Q), u0), run(p.replace(q=2 * H_Q), u0)
    rows["q"] = (4 * dL(u1, base) - dL(u2, base)) / (2 * H_Q)
    dl = np.random.default_rng(DIR_SEED).standard_normal(u0.shape)
    up, um = run(p, u0 + H_U0 * dl), run(p, u0 - H_U0 * dl)
    rows["u0_dir"] = dL(up, um) / (2 * H_U0)
    loss = 0.5 * float(((base - target) ** 2).sum())
    out = {
        "_about": ("Finite differences of the FP64 CPU oracle's forward map (tests/golden/make_fhn3d_fd.py) for "
                   "L = 1/2 ||u_N - u_target||^2 on the 3-D FitzHugh-Nagumo workload fhn3d_n127 (127^3 x 2, "
                   "tau = 0.02, all 400 steps); u_target = the oracle's u_N at 1.1 kappa_u; u0_dir is the "
                   "derivative along a standard normal field drawn with numpy default_rng(dir_seed)."),
        "workload": wl.name, "nsteps": N, "kappa": list(p.kappa), "q": p.q, "tau": p.tau,
        "target_kappa_scale": 1.1, "dir_seed": DIR_SEED,
        "steps": {"kappa_rel": H_REL, "q": H_Q, "u0": H_U0},
        "loss": loss, "residual_rel": float(np.linalg.norm(base - target) / np.linalg.norm(base)),
        "gradient": rows,
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["gradient"]), f"{time.time() - t_start:.0f} s", flush=True)


if __name__ == "__main__":
    main()
