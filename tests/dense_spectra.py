"""Dense matrix and full spectrum of the oracle's Q on the tiny periodic
workload, built once per test session and shared by the oracle pins that
need them (read-only)."""
import functools
import json
import os

import scipy.linalg

import lqsynth
from oracle.dirac import Lattice, dense_Q

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "m0.json")


@functools.lru_cache(maxsize=None)
def tiny_periodic_dense():
    """(cfg, U, Qd, ev, vecs): eigenvalues ascending, eigenvectors as columns."""
    cfg = json.load(open(GOLDEN))["tiny_periodic"]
    dims = tuple(cfg["dims"])
    lat = Lattice(dims, cfg["t_bc"])
    U = lqsynth.gauge_field(dims, cfg["eps"], cfg["field_seed"])
    Qd = dense_Q(U, cfg["m0"], lat)
    ev, vecs = scipy.linalg.eigh(Qd)
    for a in (U, Qd, ev, vecs):
        a.setflags(write=False)
    return cfg, U, Qd, ev, vecs
