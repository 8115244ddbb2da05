"""Clover term of the clover-improved Wilson-Dirac operator (the operator of
sec. 2 is the clover-improved Wilson operator; the paper does not write the
term out, so the standard Sheikholeslami-Wohlert form is taken).

TEST INFRASTRUCTURE ONLY (see the package docstring).

  * Q_munu(x): the sum of the four plaquettes of the mu-nu plane that start
    and end at x, all with the same orientation (first step +mu, then +nu,
    turning the same way around x), the "clover leaves";
  * F_munu(x) = (Q_munu(x) - Q_munu(x)^dag) / 8, anti-Hermitian, F_numu = -F_munu;
  * sigma_munu = (i/2) [gamma_mu, gamma_nu] in the chiral basis of dirac.py;
  * C(x) = c_sw (i/4) sum_{mu, nu} sigma_munu (x) F_munu(x), a Hermitian 12 x 12
    matrix per site that commutes with gamma5 (two 6 x 6 blocks), added to the
    site term: D = (4 + m0) + C(x) - 1/2 sum_mu (hops).
Links are periodic in every direction (the fermion boundary sign of t is not
part of a closed loop).  Component order 3 s + c as in dirac.py.
"""
from __future__ import annotations

import numpy as np

from .dirac import GAMMA, Lattice


def links(U, lat: Lattice, mu: int):
    """U_mu(x) as [V, 3, 3] matrices."""
    return np.moveaxis(U[mu].reshape(3, 3, lat.V), -1, 0)


def shift(M, lat: Lattice, mu: int, step: int):
    """M(x + step mu) for per-site matrices M[V, ...] (periodic, no sign)."""
    n, _ = lat.neighbour(np.arange(lat.V), mu, step)
    return M[n]


def dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def leaves(U, lat: Lattice, mu: int, nu: int):
    """Q_munu(x) = sum of the four plaquettes in the mu-nu plane at x, [V, 3, 3]."""
    Um, Un = links(U, lat, mu), links(U, lat, nu)
    Um_n = shift(Um, lat, nu, +1)                    # U_mu(x + nu)
    Un_m = shift(Un, lat, mu, +1)                    # U_nu(x + mu)
    Um_mm = shift(Um, lat, mu, -1)                   # U_mu(x - mu)
    Un_mm = shift(Un, lat, mu, -1)                   # U_nu(x - mu)
    Um_mm_n = shift(Um_mm, lat, nu, +1)              # U_mu(x - mu + nu)
    Um_nn = shift(Um, lat, nu, -1)                   # U_mu(x - nu)
    Un_nn = shift(Un, lat, nu, -1)                   # U_nu(x - nu)
    Um_mm_nn = shift(Um_mm, lat, nu, -1)             # U_mu(x - mu - nu)
    Un_mm_nn = shift(Un_mm, lat, nu, -1)             # U_nu(x - mu - nu)
    Un_nn_m = shift(Un_nn, lat, mu, +1)              # U_nu(x - nu + mu)
    p1 = Um @ Un_m @ dag(Um_n) @ dag(Un)
    p2 = Un @ dag(Um_mm_n) @ dag(Un_mm) @ Um_mm
    p3 = dag(Um_mm) @ dag(Un_mm_nn) @ Um_mm_nn @ Un_nn
    p4 = dag(Un_nn) @ Um_nn @ Un_nn_m @ dag(Um)
    return p1 + p2 + p3 + p4


def field_strength(U, lat: Lattice, mu: int, nu: int):
    """F_munu(x) = (Q_munu - Q_munu^dag) / 8, [V, 3, 3]."""
    Q = leaves(U, lat, mu, nu)
    return (Q - dag(Q)) / 8.0


def sigma(mu: int, nu: int):
    """sigma_munu = (i/2) [gamma_mu, gamma_nu] (4 x 4)."""
    return 0.5j * (GAMMA[mu] @ GAMMA[nu] - GAMMA[nu] @ GAMMA[mu])


def clover_matrix(U, lat: Lattice, csw: float):
    """C(x) = c_sw (i/4) sum_{mu, nu} sigma_munu (x) F_munu(x) as [V, 12, 12]
    (row and column index 3 s + c)."""
    C = np.zeros((lat.V, 12, 12), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            F = field_strength(U, lat, mu, nu)
            C += np.einsum("st,nab->nsatb", sigma(mu, nu), F).reshape(lat.V, 12, 12)
    return (csw * 0.25j) * C


def apply_clover(C, psi):
    """(C psi)(x) for psi[..., 12, V] and C[V, 12, 12]."""
    return np.einsum("nij,...jn->...in", C, psi)
