"""Pins of the oracle's Alg. 1 (RQI + multigrid) and Rayleigh-Ritz against the
definition of the result: the eigenpairs of Hermitian Q with smallest |lambda|
(dense eigendecomposition of the 3072 x 3072 matrix)."""

import numpy as np
import pytest

import lqsynth
from oracle import mg as M
from oracle import rqi as R
from oracle.dirac import Lattice, WilsonOp


@pytest.fixture(scope="module")
def tiny_periodic():
    from dense_spectra import tiny_periodic_dense
    cfg, U, Qd, ev, vecs = tiny_periodic_dense()
    dims = tuple(cfg["dims"])
    lat = Lattice(dims, cfg["t_bc"])
    m0 = cfg["m0"]
    # eigenvectors of the 12 eigenvalues nearest zero; EV maps an index of ev to its eigenvector
    near = np.sort(np.argsort(np.abs(ev))[:12])
    EV = {int(i): vecs[:, int(i)] for i in near}
    return dict(dims=dims, lat=lat, U=U, m0=m0, ev=ev, EV=EV, op=WilsonOp(U, m0, lat))


def test_golden_mass_meets_its_target(tiny_periodic):
    s = np.abs(tiny_periodic["ev"]).min()
    assert abs(s - 0.02) <= 1e-3 * 0.02 + 1e-6


@pytest.mark.slow
def test_alg1_returns_the_lowest_exact_pairs(tiny_periodic):
    # Alg. 1 started from the first N_eig = 5 setup test vectors (sec. 2.1:
    # RQI starts from the setup's test vectors), with P rebuilt after every
    # update: every returned pair is an exact eigenpair of Q (residual at the
    # tolerance, eigenvalue equal to a dense one) and they are the five lowest
    # of the dense spectrum, with unit overlap with the dense eigenvectors.
    t = tiny_periodic
    p = M.MGParams(coarse_m=128, coarse_tol=1e-8, coarse_restarts=2, n_setup=4)
    mg, W = M.setup(t["op"], (2, 2, 2, 2), lqsynth.gaussian_spinors(8, t["dims"], 102), p)
    lam, v, eps, info = R.rqi(mg, W[:5], 1e-10, W_pad=W, solve_tol=1e-6, max_sweeps=12)
    assert info["converged"]
    ev = t["ev"]
    assert np.all(R.residuals(t["op"], lam, v) <= 1.01e-10)
    ref = np.array(sorted(ev[np.argsort(np.abs(ev))][:5], key=lambda x: (abs(x), x)))
    assert np.abs(lam - ref).max() < 1e-12
    for i in range(5):
        j = np.argmin(np.abs(ev - lam[i]))
        ov = abs(np.vdot(t["EV"][int(j)], v[i].ravel()))
        assert ov > 1 - 1e-9


@pytest.mark.slow
def test_alg1_with_rayleigh_ritz_returns_the_eight_lowest_pairs(tiny_periodic):
    # The tiny periodic workload's own target, the 8 lowest pairs at 1e-10:
    # Alg. 1 from the 8 setup test vectors plus 2 guard vectors, with a
    # Rayleigh-Ritz step after every pass (the literal iteration stalls near
    # 2e-8 on this cluster); it stops when the 8 smallest |lambda| converge.
    # Each eigenvalue against the dense spectrum, each residual, each vector
    # against the dense eigenvector.
    t = tiny_periodic
    p = M.MGParams(coarse_m=128, coarse_tol=1e-8, coarse_restarts=2, n_setup=4)
    mg, W = M.setup(t["op"], (2, 2, 2, 2), lqsynth.gaussian_spinors(8, t["dims"], 102), p)
    V0 = np.concatenate([W, lqsynth.gaussian_spinors(2, t["dims"], 103)])
    lam, v, eps, info = R.rqi(mg, V0, 1e-10, W_pad=W, solve_tol=1e-6, max_sweeps=10, rayleigh_ritz=True,
                              n_want=8)
    assert info["converged"]
    ev = t["ev"]
    ref = np.array(sorted(ev[np.argsort(np.abs(ev))][:8], key=lambda x: (abs(x), x)))
    assert np.all(np.abs(lam[:8] - ref) <= 1e-10 * np.abs(ref))
    assert np.all(R.residuals(t["op"], lam[:8], v[:8]) <= 1.01e-10)
    for i in range(8):
        j = np.argmin(np.abs(ev - lam[i]))
        assert abs(np.vdot(t["EV"][int(j)], v[i].ravel())) > 1 - 1e-9


def test_rayleigh_ritz_recovers_exact_pairs_and_interlaces(tiny_periodic):
    t = tiny_periodic
    ev, EV = t["ev"], t["EV"]
    idx = np.argsort(np.abs(ev))[:6]
    rng = np.random.default_rng(5)
    # a random unitary mix of six exact eigenvectors: Ritz pairs are exact
    Z = rng.standard_normal((6, 6)) + 1j * rng.standard_normal((6, 6))
    Qm, _ = np.linalg.qr(Z)
    basis = (np.stack([EV[int(i)] for i in idx], axis=1) @ Qm).T.reshape(6, 12, -1)
    w, vr = R.rayleigh_ritz(t["op"], basis)
    assert np.abs(np.sort(w) - np.sort(ev[idx])).max() < 1e-12
    assert np.all(R.residuals(t["op"], w, vr) < 1e-11)
    # on a random subspace the Ritz values lie inside the spectrum (Cauchy interlacing)
    X = lqsynth.gaussian_spinors(5, t["dims"], 6)
    w2, _ = R.rayleigh_ritz(t["op"], M.orthonormalise(X))
    assert w2.min() >= ev.min() - 1e-12 and w2.max() <= ev.max() + 1e-12


def test_selection_of_interpolation_vectors():
    lam = [0.5, -0.1, 0.3, 0.1, -0.05]
    assert R.select_for_P(lam, 5, 8) == [0, 1, 2, 3, 4]
    # the three smallest |lambda| (ties to the lower index), in index order
    assert R.select_for_P(lam, 5, 3) == [1, 3, 4]
