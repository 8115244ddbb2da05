"""Pins of the oracle's Wilson-Dirac operator against facts the paper and the
mathematics fix (sec. 2: Q = gamma5 D Hermitian, gamma5 = diag(1,1,-1,-1))."""
import itertools

import numpy as np
import pytest

import lqsynth
from oracle import dirac
from oracle.dirac import GAMMA, GAMMA5, Lattice, WilsonOp, apply_D, apply_Q, dense_Q


def _unit_links(V):
    U = np.zeros((4, 9, V), dtype=np.complex128)
    U[:, [0, 4, 8], :] = 1.0
    return U


def test_gamma_basis_matches_paper_convention():
    # sec. 2: gamma5 = -g1 g2 g3 g4 must be diag(1, 1, -1, -1).
    assert np.allclose(GAMMA5, np.diag([1, 1, -1, -1]))
    for mu, nu in itertools.product(range(4), range(4)):
        assert np.allclose(GAMMA[mu], GAMMA[mu].conj().T)
        anti = GAMMA[mu] @ GAMMA[nu] + GAMMA[nu] @ GAMMA[mu]
        assert np.allclose(anti, 2.0 * np.eye(4) * (mu == nu))


def _free_spectrum(dims, m0, t_bc):
    ps = [2 * np.pi * np.arange(L) / L for L in dims[:3]]
    T = dims[3]
    ps.append((2 * np.arange(T) + (1 if t_bc == -1 else 0)) * np.pi / T)
    P = np.meshgrid(*ps, indexing="ij")
    E = np.sqrt((m0 + sum(1 - np.cos(p) for p in P)) ** 2
                + sum(np.sin(p) ** 2 for p in P)).ravel()
    # each momentum: +-E, each with spin multiplicity 2 and colour 3
    return np.sort(np.concatenate([np.repeat(E, 6), -np.repeat(E, 6)]))


@pytest.mark.parametrize("dims,m0,t_bc", [
    ((4, 2, 2, 4), 0.1, -1), ((2, 4, 4, 2), -0.3, 1), ((4, 4, 4, 4), 0.25, -1),
])
def test_free_field_closed_form(dims, m0, t_bc):
    lat = Lattice(dims, t_bc)
    Q = dense_Q(_unit_links(lat.V), m0, lat)
    ev = np.linalg.eigvalsh(Q)
    assert np.abs(ev - _free_spectrum(dims, m0, t_bc)).max() < 1e-12


def test_hermiticity_and_gamma5_hermiticity():
    dims = (4, 6, 2, 8)
    lat = Lattice(dims, -1)
    U = lqsynth.gauge_field(dims, 0.4, 11)
    x, y = lqsynth.gaussian_spinors(2, dims, 12)
    lhs = np.vdot(x, apply_Q(U, -0.3, y, lat))
    rhs = np.vdot(apply_Q(U, -0.3, x, lat), y)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # D^dag = gamma5 D gamma5  <=>  <x, D y> = <gamma5 D gamma5 x, y>
    g5 = dirac.gamma5
    lhs = np.vdot(x, apply_D(U, -0.3, y, lat))
    rhs = np.vdot(g5(apply_D(U, -0.3, g5(x), lat)), y)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _gauge_transform(U, Om, lat):
    """U_mu(n) -> Om(n) U_mu(n) Om(n + mu)^dag."""
    fwd, _, _, _ = lat.tables()
    Ut = np.empty_like(U)
    for mu in range(4):
        Um = U[mu].reshape(3, 3, lat.V).transpose(2, 0, 1)
        On = Om[fwd[mu]]
        Ut[mu] = (Om @ Um @ On.conj().transpose(0, 2, 1)).transpose(1, 2, 0).reshape(9, lat.V)
    return Ut


def _colour_rotate(Om, psi, V):
    p = psi.reshape(4, 3, V)
    return np.einsum("nab,sbn->san", Om, p).reshape(12, V)


def test_gauge_covariance_and_spectrum_invariance():
    dims = (4, 2, 4, 4)
    lat = Lattice(dims, -1)
    U = lqsynth.gauge_field(dims, 0.4, 21)
    Om = lqsynth.random_su3(lat.V, 22)
    Ut = _gauge_transform(U, Om, lat)
    psi = lqsynth.gaussian_spinors(1, dims, 23)[0]
    lhs = apply_Q(Ut, -0.2, _colour_rotate(Om, psi, lat.V), lat)
    rhs = _colour_rotate(Om, apply_Q(U, -0.2, psi, lat), lat.V)
    assert np.abs(lhs - rhs).max() < 1e-12
    e1 = np.linalg.eigvalsh(dense_Q(U, -0.2, lat))
    e2 = np.linalg.eigvalsh(dense_Q(Ut, -0.2, lat))
    assert np.abs(e1 - e2).max() < 1e-11


def test_sparse_route_equals_definition_route():
    dims = (6, 4, 2, 4)
    for t_bc in (-1, 1):
        lat = Lattice(dims, t_bc)
        U = lqsynth.gauge_field(dims, 0.3, 31)
        op = WilsonOp(U, -0.45, lat)
        x = lqsynth.gaussian_spinors(3, dims, 32)
        assert np.abs(op.Q(x) - apply_Q(U, -0.45, x, lat)).max() < 1e-13
        assert np.abs(op.D(x) - apply_D(U, -0.45, x, lat)).max() < 1e-13


def test_site_sampled_apply():
    dims = (4, 4, 2, 6)
    lat = Lattice(dims, -1)
    U = lqsynth.gauge_field(dims, 0.3, 41)
    x = lqsynth.gaussian_spinors(1, dims, 42)[0]
    sites = np.array([0, 3, 17, 55, lat.V - 1])
    full = apply_Q(U, 0.1, x, lat)[:, sites]
    assert np.abs(dirac.apply_Q_sites(U, 0.1, x, lat, sites) - full).max() < 1e-14


def test_boundary_sign_only_on_t_hops():
    # With unit links, flipping the t boundary sign changes the spectrum
    # (momenta shift by pi/T) while an x-translation leaves Q invariant.
    dims = (4, 2, 2, 4)
    U = _unit_links(16 * 4)
    x = lqsynth.gaussian_spinors(1, dims, 51)[0]
    lat = Lattice(dims, -1)
    y = apply_Q(U, 0.2, x, lat).reshape(12, 4, 2, 2, 4, order="F")
    xs = np.roll(x.reshape(12, 4, 2, 2, 4, order="F"), 1, axis=1)
    ys = apply_Q(U, 0.2, xs.reshape(12, -1, order="F"), lat).reshape(12, 4, 2, 2, 4, order="F")
    assert np.abs(np.roll(y, 1, axis=1) - ys).max() < 1e-13
