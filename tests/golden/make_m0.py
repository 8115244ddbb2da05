"""Write tests/golden/m0.json: bare masses for the small lattice workloads.

Calls only the CPU oracle (dense eigenvalues of Q on a 4^4 lattice) and the
seeded field generator.  Recipe (one reading of the workload description):
  * 4^4, t antiperiodic, eps = 0.4, field seed 101: the smallest |lambda(Q)|
    stays near 0.49 for every m0, so m0 is the minimiser of that smallest
    |lambda| (golden-section search);
  * 4^4, t periodic, same field: m0 is bisected on the heavier side of the
    minimiser until the smallest |lambda| is 0.02 (relative accuracy 1e-3).
  * larger lattices (16^4 at eps = 0.3 and 32^3 x 64 at eps = 0.25, t
    periodic): the additive mass shift is a short-distance property of the
    field ensemble, so m_c(eps) is taken as the minimiser of the smallest
    |lambda| on a 4^4 periodic lattice drawn with the same recipe (seeds 201,
    301), and m0 = m_c + target; the smallest |lambda| actually reached on the
    large lattice is measured by the solver and reported, not assumed.
Run:  OPENBLAS_NUM_THREADS=1 python tests/golden/make_m0.py
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


def main():
    dims = (4, 4, 4, 4)
    U = lqsynth.gauge_field(dims, 0.4, 101)
    out = {}
    for name, bc in (("tiny_antiperiodic", -1), ("tiny_periodic", 1)):
        lat = Lattice(dims, bc)
        Q0 = dense_Q(U, 0.0, lat)
        G5 = np.diag(np.repeat([1.0, 1.0, -1.0, -1.0], 3 * lat.V)).astype(np.complex128)
        a, b = -1.0, 0.0
        g = (np.sqrt(5) - 1) / 2
        c, d = b - g * (b - a), a + g * (b - a)
        fc, fd = smallest(Q0, G5, c), smallest(Q0, G5, d)
        while b - a > 2e-3:
            if fc < fd:
                b, d, fd = d, c, fc
                c = b - g * (b - a)
                fc = smallest(Q0, G5, c)
            else:
                a, c, fc = c, d, fd
                d = a + g * (b - a)
                fd = smallest(Q0, G5, d)
        mstar = 0.5 * (a + b)
        smin = smallest(Q0, G5, mstar)
        target = 0.02
        if smin >= target:
            m0 = mstar
        else:
            lo, hi = mstar, mstar + 1.0
            while True:
                mid = 0.5 * (lo + hi)
                s = smallest(Q0, G5, mid)
                if abs(s - target) <= 1e-3 * target:
                    break
                if s < target:
                    lo = mid
                else:
                    hi = mid
            m0 = mid
        s = smallest(Q0, G5, m0)
        out[name] = {"dims": list(dims), "t_bc": bc, "eps": 0.4, "field_seed": 101,
                     "m0": round(m0, 6), "smallest_abs_lambda": s, "argmin_m0": mstar,
                     "floor": smin}
        print(name, out[name], flush=True)
    for name, eps, seed, target, big in (("medium", 0.3, 201, 0.005, (16, 16, 16, 16)),
                                         ("large", 0.25, 301, 0.002, (32, 32, 32, 64))):
        U4 = lqsynth.gauge_field(dims, eps, seed)
        lat = Lattice(dims, 1)
        Q0 = dense_Q(U4, 0.0, lat)
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
        mc = 0.5 * (a + b)
        out[name] = {"dims": list(big), "t_bc": 1, "eps": eps, "field_seed": seed, "m0": round(mc + target, 6),
                     "m_c_4444": mc, "target": target}
        print(name, out[name], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "m0.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
