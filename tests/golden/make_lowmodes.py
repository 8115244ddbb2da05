"""Writes lowmodes_8x8x4x4.json: the lowest-|lambda| eigenvalues of Q on an
8x8x4x4 lattice (12,288 unknowns) from the oracle's dense matrix and LAPACK's
Hermitian eigensolver.  This is the exact reference of the completeness test
of the GPU eigensolver (every pair it returns must be one of these, and it
must return the lowest ones).  Calls only oracle/ and the seeded input
generator.

Usage: python tests/golden/make_lowmodes.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import lqsynth  # noqa: E402
from oracle.dirac import Lattice, dense_Q  # noqa: E402

DIMS, T_BC, EPS, SEED, M0, KEEP = (8, 8, 4, 4), 1, 0.4, 801, -0.30, 80


def main():
    lat = Lattice(DIMS, T_BC)
    U = lqsynth.gauge_field(DIMS, EPS, SEED)
    t0 = time.time()
    ev = np.linalg.eigvalsh(dense_Q(U, M0, lat))
    order = sorted(range(len(ev)), key=lambda i: (abs(ev[i]), ev[i]))
    low = [float(ev[i]) for i in order[:KEEP]]
    out = {"dims": list(DIMS), "t_bc": T_BC, "eps": EPS, "field_seed": SEED, "m0": M0,
           "lowest_by_abs": low, "n_total": int(len(ev)),
           "note": "eigenvalues of Q sorted by (|lambda|, lambda); dense LAPACK eigvalsh of the oracle's matrix"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lowmodes_8x8x4x4.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path} in {time.time() - t0:.0f} s; |lambda| 1..{KEEP}: {abs(low[0]):.4f} .. {abs(low[-1]):.4f}")


if __name__ == "__main__":
    main()
