"""Write tests/golden/mc_curve.json: the additive critical mass m_c(eps) of
the synthetic field ensemble at eps = 0.20, 0.25, ..., 0.40, for the learned
setup's training fields (16^4, eps between 0.2 and 0.4, t periodic), whose
bare mass is m_c(eps) + 0.005 with m_c interpolated linearly in eps.

m_c(eps) is found as for the large workloads in make_m0.py: the minimiser of
the smallest |lambda(Q)| over m0 on a 4^4 periodic lattice drawn with the
same recipe (field seed 900 + 100 eps), by golden-section search on the dense
spectrum.  Calls only oracle/ and the seeded field generator.

Run:  OPENBLAS_NUM_THREADS=4 python tests/golden/make_mc_curve.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lqsynth  # noqa: E402
from oracle.dirac import Lattice, dense_Q  # noqa: E402


def smallest(Q0, G5, m0):
    return float(np.min(np.abs(np.linalg.eigvalsh(Q0 + m0 * G5))))


def critical_mass(eps, seed):
    dims = (4, 4, 4, 4)
    lat = Lattice(dims, 1)
    Q0 = dense_Q(lqsynth.gauge_field(dims, eps, seed), 0.0, lat)
    G5 = np.diag(np.repeat([1.0, 1.0, -1.0, -1.0], 3 * lat.V)).astype(np.complex128)
    a, b = -1.0, 0.0
    g = (np.sqrt(5) - 1) / 2
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = smallest(Q0, G5, c), smallest(Q0, G5, d)
    while b - a > 1e-4:
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = smallest(Q0, G5, c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = smallest(Q0, G5, d)
    return 0.5 * (a + b)


def main():
    eps_grid = [0.20, 0.25, 0.30, 0.35, 0.40]
    mc = []
    for eps in eps_grid:
        mc.append(critical_mass(eps, 900 + int(round(100 * eps))))
        print(f"eps {eps:.2f}: m_c {mc[-1]:.5f}", flush=True)
    out = {"eps": eps_grid, "m_c": mc, "target": 0.005, "dims_4444_seed": "900 + 100 eps",
           "note": "m0(eps) = interp(eps, eps, m_c) + target; 4^4 periodic golden-section minimiser"}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "mc_curve.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
