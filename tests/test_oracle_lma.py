"""Pins of the approximate low-mode averaging of paper sec. 3.2-3.3 against the
dense inverse of Q on the tiny periodic lattice: A is diagonal for exact
eigenvectors and Q~_low^{-1} is then the plain low-mode sum; for inexact ones
the low part plus Q^{-1} R~ is exactly Q^{-1} (so the stochastic high part
leaves the estimate unbiased); R~ annihilates Q V~; tr(Q Q~_low^{-1}) equals the
number of modes; the per-timeslice loop and connected correlator of the low
part equal their definitions written out with the dense low-mode matrix."""

import numpy as np
import pytest

import lqsynth
from oracle import lma
from oracle.dirac import Lattice, WilsonOp


@pytest.fixture(scope="module")
def tiny():
    from dense_spectra import tiny_periodic_dense
    cfg, U, Qd, ev, vecs = tiny_periodic_dense()
    dims = tuple(cfg["dims"])
    lat = Lattice(dims, cfg["t_bc"])
    o = np.argsort(np.abs(ev), kind="stable")
    return dict(dims=dims, lat=lat, op=WilsonOp(U, cfg["m0"], lat), Qd=Qd, ev=ev[o], vecs=vecs[:, o],
                T=dims[3], Vol=lat.V)


def _inexact(t, n, amp, seed):
    rng = np.random.default_rng(seed)
    X = t["vecs"][:, :n] + amp * (rng.standard_normal((t["Qd"].shape[0], n))
                                  + 1j * rng.standard_normal((t["Qd"].shape[0], n)))
    Qm, _ = np.linalg.qr(X)                              # orthonormal approximations
    return Qm.T.reshape(n, 12, -1)


def test_exact_modes_give_diagonal_A_and_the_plain_low_sum(tiny):
    t = tiny
    n = 8
    V = t["vecs"][:, :n].T.reshape(n, 12, -1)
    A = lma.projected_matrix(t["op"], V)
    assert np.abs(A - np.diag(t["ev"][:n])).max() < 1e-12
    x = lqsynth.gaussian_spinors(1, t["dims"], 3)[0]
    plain = sum(np.vdot(V[i].ravel(), x.ravel()) / t["ev"][i] * V[i] for i in range(n))
    assert np.abs(lma.low_inverse_apply(V, A, x) - plain).max() < 1e-12 * np.abs(plain).max()


def test_low_part_plus_high_part_is_the_inverse_for_inexact_modes(tiny):
    t = tiny
    n = 8
    V = _inexact(t, n, 1e-3, 4)
    A = lma.projected_matrix(t["op"], V)
    x = lqsynth.gaussian_spinors(1, t["dims"], 5)[0]
    exact = np.linalg.solve(t["Qd"], x.ravel()).reshape(x.shape)
    high = np.linalg.solve(t["Qd"], lma.oblique_projector_apply(t["op"], V, A, x).ravel()).reshape(x.shape)
    total = lma.low_inverse_apply(V, A, x) + high
    assert np.abs(total - exact).max() < 1e-10 * np.abs(exact).max()
    # R~ annihilates Q V~, and tr(Q Q~_low^{-1}) = tr(A^{-1} A) = n
    QV = t["op"].Q(V)
    for i in range(n):
        assert np.abs(lma.oblique_projector_apply(t["op"], V, A, QV[i])).max() < 1e-10 * np.abs(QV[i]).max()
    Vm = V.reshape(n, -1).T
    Qlow = Vm @ np.linalg.solve(A, Vm.conj().T)
    assert abs(np.trace(t["Qd"] @ Qlow) - n) < 1e-10


def test_timeslice_observables_of_the_low_part_match_their_definitions(tiny):
    t = tiny
    n, T, Vol = 8, tiny["T"], tiny["Vol"]
    V = _inexact(t, n, 1e-2, 6)
    A = lma.projected_matrix(t["op"], V)
    Vm = V.reshape(n, -1).T
    M = (Vm @ np.linalg.solve(A, Vm.conj().T)).reshape(12, Vol, 12, Vol)    # (c x, c' y)
    L3 = Vol // T
    Lref = np.array([sum(np.trace(M[:, x, :, x]) for x in range(s * L3, (s + 1) * L3)) for s in range(T)])
    assert np.abs(lma.loop_low(V, A, T) - Lref).max() < 1e-12 * np.abs(Lref).max()
    # C_low(t) = (1/Vol) sum over x, y with x_t - y_t = t of tr[M_xy M_yx]
    tslice = np.arange(Vol) // L3
    Wxy = np.einsum("axby,byax->xy", M, M)                 # tr[M_xy M_yx] for every pair
    dt = (tslice[:, None] - tslice[None, :]) % T
    Cref = np.array([Wxy[dt == s].sum() for s in range(T)]) / Vol
    assert np.abs(lma.connected_low(V, A, T, Vol) - Cref).max() < 1e-12 * np.abs(Cref).max()


def test_stochastic_high_part_is_unbiased(tiny):
    # L_low + mean over Z2 + i Z2 noise of the high-part samples approaches the
    # exact loop (dense inverse); the error falls like 1/sqrt(samples)
    t = tiny
    n, T = 8, tiny["T"]
    V = _inexact(t, n, 1e-2, 7)
    A = lma.projected_matrix(t["op"], V)
    Qinv = np.linalg.inv(t["Qd"])
    blocks = np.einsum("cxdx->xcd", Qinv.reshape(12, t["Vol"], 12, t["Vol"]))
    Lex = lma.loop_exact(blocks, T)
    eta = lqsynth.z2_spinors(64, t["dims"], 8)
    samples = []
    for e in eta:
        s = (Qinv @ lma.oblique_projector_apply(t["op"], V, A, e).ravel()).reshape(e.shape)
        samples.append(lma.loop_high_sample(t["op"], V, A, e, s, T))
    samples = np.array(samples)
    est = lma.loop_low(V, A, T) + samples.mean(axis=0)
    err = np.abs(est - Lex)
    sem = samples.std(axis=0) / np.sqrt(len(samples))
    assert np.all(err <= 5 * sem + 1e-12)


def test_cutoff_keeps_the_accurate_approximations():
    lam = [0.1, -0.2, 0.05, 0.3]
    eps = [0.05, 0.2, 0.01, 0.25]
    assert lma.select(lam, eps, 0.75) == [0, 2]
    assert lma.select(lam, eps, 1.0) == [0, 1, 2, 3]
