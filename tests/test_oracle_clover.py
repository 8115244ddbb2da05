"""Pins of the oracle's clover term (oracle/clover.py) against facts fixed by
the definition and by the mathematics, not by retyping it: closed loops walked
site by site, the exact field strength of a constant abelian field, sigma_munu
in the chiral basis worked out by hand, Hermiticity and chirality, gauge
covariance, and the spectrum of Q with the clover term."""
import numpy as np
import pytest

import lqsynth
from oracle import clover as CL
from oracle.dirac import GAMMA5, Lattice, WilsonOp

DIMS = (4, 4, 4, 4)


def walk(U, lat, x, steps):
    """Product of the links along a closed path from site x, step by step:
    +mu uses U_mu(y), -mu uses U_mu(y - mu)^dag."""
    M = np.eye(3, dtype=np.complex128)
    c = list(lat.coords(np.array(x)))
    for mu, sgn in steps:
        y = lat.index(c)
        if sgn > 0:
            L = U[mu].reshape(3, 3, lat.V)[:, :, y]
            c[mu] = (c[mu] + 1) % lat.dims[mu]
        else:
            c[mu] = (c[mu] - 1) % lat.dims[mu]
            L = U[mu].reshape(3, 3, lat.V)[:, :, lat.index(c)].conj().T
        M = M @ L
    assert lat.index(c) == x
    return M


@pytest.mark.parametrize("mu,nu", [(0, 1), (1, 3), (2, 3), (0, 2)])
def test_leaves_are_the_four_plaquettes_walked_site_by_site(mu, nu):
    lat = Lattice(DIMS, -1)
    U = lqsynth.gauge_field(DIMS, 0.5, 11)
    Q = CL.leaves(U, lat, mu, nu)
    paths = [[(mu, 1), (nu, 1), (mu, -1), (nu, -1)], [(nu, 1), (mu, -1), (nu, -1), (mu, 1)],
             [(mu, -1), (nu, -1), (mu, 1), (nu, 1)], [(nu, -1), (mu, 1), (nu, 1), (mu, -1)]]
    for x in (0, 37, 255):
        ref = sum(walk(U, lat, x, p) for p in paths)
        assert np.abs(Q[x] - ref).max() < 1e-13
    # the reversed orientation gives the conjugate: Q_numu = Q_munu^dag
    assert np.abs(CL.leaves(U, lat, nu, mu) - CL.dag(Q)).max() < 1e-13


def test_sigma_in_the_chiral_basis():
    # worked out by hand from gamma_k = [[0, i s_k], [-i s_k, 0]], gamma_t = [[0, 1], [1, 0]]:
    # sigma_kl = -eps_klm s_m in both chiral blocks, sigma_kt = -s_k (upper), +s_k (lower)
    s = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
    z = np.zeros((2, 2))
    blk = lambda a, b: np.block([[a, z], [z, b]])
    assert np.allclose(CL.sigma(0, 1), blk(-s[2], -s[2]))
    assert np.allclose(CL.sigma(0, 2), blk(s[1], s[1]))
    assert np.allclose(CL.sigma(1, 2), blk(-s[0], -s[0]))
    for k in range(3):
        assert np.allclose(CL.sigma(k, 3), blk(-s[k], s[k]))
        assert np.allclose(CL.sigma(3, k), -CL.sigma(k, 3))


def test_constant_abelian_field_has_the_closed_form_clover():
    # U_x(n) = exp(i b n_y) (b = 2 pi / L_y, a whole flux quantum), all else 1:
    # every x-y plaquette is exp(-i b), so F_xy = -i sin(b), the other planes
    # vanish, and C = c_sw sin(b)/2 sigma_xy (x) 1, eigenvalues +-c_sw sin(b)/2
    lat = Lattice(DIMS, 1)
    b = 2 * np.pi / DIMS[1]
    U = np.zeros((4, 9, lat.V), dtype=np.complex128)
    for mu in range(4):
        U[mu, [0, 4, 8], :] = 1.0
    _, y, _, _ = lat.coords(np.arange(lat.V))
    U[0, [0, 4, 8], :] = np.exp(1j * b * y)
    csw = 1.7
    C = CL.clover_matrix(U, lat, csw)
    ref = csw * np.sin(b) / 2 * np.kron(CL.sigma(0, 1), np.eye(3))
    assert np.abs(C - ref[None]).max() < 1e-13
    ev = np.linalg.eigvalsh(C[5])
    assert np.allclose(np.sort(ev), np.repeat([-1, 1], 6) * csw * np.sin(b) / 2)


def test_free_field_has_no_clover_term():
    lat = Lattice(DIMS, -1)
    U = lqsynth.gauge_field(DIMS, 0.0, 1)
    assert np.abs(CL.clover_matrix(U, lat, 1.0)).max() < 1e-14


def test_clover_is_hermitian_traceless_and_chiral():
    lat = Lattice(DIMS, -1)
    U = lqsynth.gauge_field(DIMS, 0.6, 12)
    C = CL.clover_matrix(U, lat, 1.3)
    assert np.abs(C - np.conj(np.swapaxes(C, 1, 2))).max() < 1e-14
    assert np.abs(np.trace(C, axis1=1, axis2=2)).max() < 1e-13
    g5 = np.kron(GAMMA5, np.eye(3))
    assert np.abs(C @ g5 - g5 @ C).max() < 1e-14
    assert np.abs(C).max() > 1e-2


def test_clover_is_gauge_covariant():
    lat = Lattice(DIMS, -1)
    U = lqsynth.gauge_field(DIMS, 0.6, 13)
    Om = lqsynth.gauge_field(DIMS, 2.0, 14)[0].reshape(3, 3, lat.V)    # random SU(3) per site
    Ug = np.empty_like(U)
    for mu in range(4):
        n, _ = lat.neighbour(np.arange(lat.V), mu, +1)
        Um = U[mu].reshape(3, 3, lat.V)
        Ug[mu] = np.einsum("abn,bcn,dcn->adn", Om, Um, Om[:, :, n].conj()).reshape(9, lat.V)
    C, Cg = CL.clover_matrix(U, lat, 1.0), CL.clover_matrix(Ug, lat, 1.0)
    W = np.einsum("st,abn->nsatb", np.eye(4), Om).reshape(lat.V, 12, 12)
    assert np.abs(Cg - W @ C @ np.conj(np.swapaxes(W, 1, 2))).max() < 1e-13


def test_q_with_clover_is_hermitian_and_its_spectrum_gauge_invariant():
    dims = (4, 4, 2, 2)
    lat = Lattice(dims, -1)
    U = lqsynth.gauge_field(dims, 0.5, 15)
    op = WilsonOp(U, -0.2, lat, csw=1.5)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((12, lat.V)) + 1j * rng.standard_normal((12, lat.V))
    y = rng.standard_normal((12, lat.V)) + 1j * rng.standard_normal((12, lat.V))
    assert abs(np.vdot(x, op.Q(y)) - np.vdot(op.Q(x), y)) < 1e-11 * np.linalg.norm(x) * np.linalg.norm(y)
    Om = lqsynth.gauge_field(dims, 2.0, 16)[0].reshape(3, 3, lat.V)
    Ug = np.empty_like(U)
    for mu in range(4):
        n, _ = lat.neighbour(np.arange(lat.V), mu, +1)
        Ug[mu] = np.einsum("abn,bcn,dcn->adn", Om, U[mu].reshape(3, 3, lat.V),
                           Om[:, :, n].conj()).reshape(9, lat.V)
    opg = WilsonOp(Ug, -0.2, lat, csw=1.5)

    def dense(o):
        n = 12 * lat.V
        E = np.eye(n, dtype=np.complex128).reshape(n, 12, lat.V)
        return o.Q(E).reshape(n, n).T

    e1 = np.linalg.eigvalsh(dense(op))
    e2 = np.linalg.eigvalsh(dense(opg))
    assert np.abs(e1 - e2).max() < 1e-11
    # and the clover term changes the spectrum
    e0 = np.linalg.eigvalsh(dense(WilsonOp(U, -0.2, lat)))
    assert np.abs(e1 - e0).max() > 1e-3
