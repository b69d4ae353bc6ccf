"""Writes lattice_n32_t3.json: the oracle's FP64 outer iterations (the
finite-beta Hartree-Fock reference and one correlated iteration) for member 3
of the 4x4x2 lattice hopping scan (N = 32, 32 electrons, beta = 100,
8192 Matsubara frequencies, 1025 tau points, Sigma damping 0.5).

Run from the repository root:  python tests/golden/make_lattice_reference.py
It calls only oracle/ (and the seeded input generator); a run takes a few
minutes on 8 cores.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from synthetic import LATTICE_T, lattice_sweep  # noqa: E402

INDEX = 3


def main():
    s = lattice_sweep(INDEX)
    p = O.Params(damp_Sigma=0.5)
    mu0 = float(np.mean(np.diag(s.h)))
    st = O.State(mu=mu0, F=s.h.copy())
    its = []
    for _ in range(2):
        r = O.outer_iteration(s, p, st)
        its.append({"energy": r.energy, "e2b": r.e2b, "mu": r.mu, "n_inner": r.n_inner,
                    "n_eval": r.n_eval})
        print(its[-1], flush=True)
    out = {"system": s.name, "index": INDEX, "t": LATTICE_T[INDEX], "mu0": mu0,
           "damp_Sigma": 0.5, "iterations": its,
           "written_by": "tests/golden/make_lattice_reference.py (oracle, FP64)"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lattice_n32_t3.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
