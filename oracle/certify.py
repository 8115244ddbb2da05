"""Certificates for computed eigenpairs of the Hermitian Q (the paper admits
that RQI with multigrid can miss eigenpairs, sec. 2.1; these checks tell
whether a returned set is the wanted one without a second eigensolver).

TEST INFRASTRUCTURE ONLY (see the package docstring).

  * residual bound: for a unit vector v, some eigenvalue of a Hermitian
    matrix lies within ||Q v - lambda v|| of its Rayleigh quotient lambda;
  * Kato-Temple bound: if the interval (lambda - delta, lambda + delta) with
    delta > eps holds a single eigenvalue mu, then
    |lambda - mu| <= eps^2 / delta (an error quadratic in the residual);
  * completeness: after deflating the found vectors V, the smallest |mu| of
    the operator restricted to the orthogonal complement of V must not lie
    below the largest |lambda| found (else a lower mode was missed).  The
    smallest |mu| is approached by inverse iteration on the complement from
    several random starts, each step a solve of Q by a dense or any
    converged solver passed in.  For a unit x in the complement,
    ||(1 - V V^dag) Q x|| >= min |mu| (the Rayleigh quotient of the squared
    restricted operator bounds its smallest eigenvalue from above, whatever
    the signs of the mu mixed in x), so a value below max |lambda| proves a
    missed mode; a value above it is evidence, not proof, that none was
    missed (the iteration may not have reached the smallest mode).
"""
from __future__ import annotations

import numpy as np

from .krylov import dot, norm


def residual_bound(op, lam, V):
    """eps_i = ||Q v_i - lambda_i v_i|| / ||v_i||: some eigenvalue of Q lies
    within eps_i of lambda_i."""
    QV = op.Q(V)
    return np.array([norm(QV[i] - lam[i] * V[i]) / norm(V[i]) for i in range(V.shape[0])])


def kato_temple(lam, eps, lower=None, upper=None):
    """Kato-Temple error bounds eps_i^2 / delta_i, with delta_i the distance
    from lambda_i to the nearest other computed eigenvalue (or to the given
    outer bounds lower/upper of the rest of the spectrum), minus its residual.
    Returns inf where delta_i <= eps_i (the bound does not apply)."""
    lam = np.asarray(lam, dtype=float)
    eps = np.asarray(eps, dtype=float)
    out = np.empty_like(lam)
    for i in range(len(lam)):
        others = np.delete(lam, i)
        cand = [np.abs(others - lam[i]).min()] if len(others) else []
        if lower is not None:
            cand.append(lam[i] - lower)
        if upper is not None:
            cand.append(upper - lam[i])
        delta = min(cand) - eps[i] if cand else np.inf
        out[i] = eps[i] ** 2 / delta if delta > eps[i] else np.inf
    return out


def project_out(V, x):
    """x minus its components along the orthonormal rows of V (twice)."""
    for _ in range(2):
        for v in V:
            x = x - dot(v, x) * v
    return x


def deflated_smallest(op, V, solve, n_start: int = 4, iters: int = 30, seed: int = 0, tol: float = 1e-8):
    """Smallest |mu| of Q restricted to the orthogonal complement of the
    orthonormal vectors V, by inverse iteration from n_start seeded random
    starts.  solve(b) must return Q^{-1} b (any converged solver); the
    iteration is x <- (1 - V V^dag) Q^{-1} x, normalised.  Returns
    (a, residual) for the best start: a = ||(1 - V V^dag) Q x||, an upper bound
    of the smallest |mu| that tends to it, and the eigen-residual of x."""
    rng = np.random.default_rng(seed)
    shape = V.shape[1:]
    best = (np.inf, np.inf)
    for _ in range(n_start):
        x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        x = project_out(V, x)
        x = x / norm(x)
        mu, res = np.inf, np.inf
        for _k in range(iters):
            y = project_out(V, solve(x))
            x = y / norm(y)
            Qx = project_out(V, op.Q(x))
            mu = dot(x, Qx).real
            res = norm(Qx - mu * x)
            if res <= tol * max(abs(mu), 1e-300):
                break
        a = norm(Qx)
        if a < best[0]:
            best = (a, res)
    return best


def missing_modes(lam_found, mu_deflated, tol: float):
    """True if the deflated spectrum has a mode below the largest |lambda|
    found (by more than tol): the set is not the lowest one."""
    return abs(mu_deflated) < np.max(np.abs(lam_found)) - tol
