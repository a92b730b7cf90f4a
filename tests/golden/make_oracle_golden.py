"""Write the oracle's expected values for the workloads the GPU tests check.

Calls only the oracle (oracle/) and the seeded input generators; run it from
the repository root:  python tests/golden/make_oracle_golden.py
Outputs (text JSON, floats printed with 17 significant digits):
  tests/golden/ring12_oracle.json        N=12 s=1/2 ring, 120 steps, full reorth
  tests/golden/all_to_all20_oracle.json  N=20 all-to-all, 300 steps, gradient
  tests/golden/j1j2_ring32_oracle.json   N=32 J1-J2 ring (dim 601,080,390), the
                                         first two Lanczos steps (alpha, beta);
                                         about 30 GB of host memory, minutes
Pass workload names to write only some of them.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_0706_3293_amd import inputs  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def _floats(a):
    return [float(f"{v:.17g}") for v in np.asarray(a, dtype=np.float64)]


def ring12():
    N = 12
    J = inputs.ring_couplings(N, -1.0)
    sub = oracle.Subspace(N, 1, 6)
    res = oracle.lanczos(sub, J, inputs.start_vector(sub.dim, 0), 120,
                         full_reorth=True)
    return dict(workload="ring12", N=N, two_s=1, A=6, steps=120, full_reorth=True,
                seed=0, E0=float(res["E0"]), steps_done=res["steps_done"],
                alpha=_floats(res["alpha"]), beta=_floats(res["beta"]))


def all_to_all20():
    N = 20
    J, bonds, vals = inputs.all_to_all_couplings(N, 0)
    sub = oracle.Subspace(N, 1, 10)
    res = oracle.ground_state(sub, J, inputs.start_vector(sub.dim, 0), 300)
    psi = res["psi"]
    C = oracle.bond_correlations(sub, psi, bonds)
    resid = float(np.linalg.norm(sub.apply(J, psi) - res["E0"] * psi))
    evals, _ = oracle.ritz_all(res["alpha"], res["beta"])
    return dict(workload="all_to_all20", N=N, two_s=1, A=10, steps=300,
                full_reorth=False, seed=0, E0=float(res["E0"]),
                steps_done=res["steps_done"], alpha=_floats(res["alpha"]),
                beta=_floats(res["beta"]), bonds=[list(b) for b in bonds],
                J=_floats(vals), grad=_floats(-C),
                ritz_gap=float(evals[evals > evals[0] + 1e-8 * abs(evals[0])][0] - evals[0]),
                residual=resid)


def j1j2_ring32():
    """The first two oracle Lanczos steps of the largest single-GPU workload:
    two full H x applications on 601,080,390 rows (Sec. 4, Eq. (E-4-b))."""
    N = 32
    J = inputs.workload_couplings("j1j2_ring32")
    sub = oracle.Subspace(N, 1, 16)
    res = oracle.lanczos(sub, J, inputs.start_vector(sub.dim, 0), 2)
    return dict(workload="j1j2_ring32", N=N, two_s=1, A=16, J1=-1.0, J2=-0.25,
                dim=sub.dim, steps=2, full_reorth=False, seed=0,
                alpha=_floats(res["alpha"]), beta=_floats(res["beta"]))


WORKLOADS = {"ring12": ring12, "all_to_all20": all_to_all20, "j1j2_ring32": j1j2_ring32}


def main():
    names = sys.argv[1:] or list(WORKLOADS)
    for fn in (WORKLOADS[n] for n in names):
        t = time.time()
        data = fn()
        path = os.path.join(OUT, f"{data['workload']}_oracle.json")
        with open(path, "w") as f:
            json.dump(data, f, indent=1)
        print(f"wrote {path} in {time.time() - t:.1f} s", flush=True)


if __name__ == "__main__":
    main()
