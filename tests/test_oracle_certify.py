"""Pins of the eigenpair certificates against the dense spectrum of Q on the
tiny periodic lattice: the residual bound and the Kato-Temple bound hold for
perturbed eigenvectors, and deflated inverse iteration finds the next mode
after the exact lowest ones, or the missing one when a low mode is left out."""

import numpy as np
import pytest

from oracle import certify as C
from oracle.dirac import Lattice, WilsonOp


@pytest.fixture(scope="module")
def tiny():
    from dense_spectra import tiny_periodic_dense
    cfg, U, Qd, ev, vecs = tiny_periodic_dense()
    dims = tuple(cfg["dims"])
    lat = Lattice(dims, cfg["t_bc"])
    order = np.argsort(np.abs(ev), kind="stable")
    return dict(dims=dims, op=WilsonOp(U, cfg["m0"], lat), Qd=Qd, ev=ev[order], vecs=vecs[:, order])


def test_residual_and_kato_temple_bounds_hold(tiny):
    t = tiny
    rng = np.random.default_rng(1)
    n = 6
    V = t["vecs"][:, :n].T.copy()
    V = V + 1e-5 * (rng.standard_normal(V.shape) + 1j * rng.standard_normal(V.shape))
    V = V / np.linalg.norm(V, axis=1)[:, None]
    V = V.reshape(n, 12, -1)
    lam = np.array([np.vdot(v.ravel(), t["Qd"] @ v.ravel()).real for v in V])
    eps = C.residual_bound(t["op"], lam, V)
    err = np.abs(lam - t["ev"][:n])
    assert np.all(err <= eps)                            # some eigenvalue within eps
    kt = C.kato_temple(lam, eps)
    assert np.all(np.isfinite(kt))
    assert np.all(err <= kt * (1 + 1e-6))               # and within eps^2 / gap
    assert np.all(kt < eps)                              # which is the sharper bound here


def test_deflated_inverse_iteration_finds_the_next_or_the_missing_mode(tiny):
    t = tiny
    Qinv = np.linalg.inv(t["Qd"])

    def solve(b):
        return (Qinv @ b.ravel()).reshape(b.shape)

    k = 5
    V = t["vecs"][:, :k].T.reshape(k, 12, -1)
    mu, res = C.deflated_smallest(t["op"], V, solve, n_start=3, iters=60, tol=1e-10)
    assert abs(abs(mu) - abs(t["ev"][k])) < 1e-8          # the sixth lowest
    assert not C.missing_modes(t["ev"][:k], mu, 1e-10)
    # leave out the third lowest: it comes back, and the set is flagged
    keep = [0, 1, 3, 4, 5]
    V2 = t["vecs"][:, keep].T.reshape(len(keep), 12, -1)
    mu2, _ = C.deflated_smallest(t["op"], V2, solve, n_start=3, iters=60, tol=1e-10)
    assert abs(abs(mu2) - abs(t["ev"][2])) < 1e-8
    assert C.missing_modes(t["ev"][keep], mu2, 1e-10)
