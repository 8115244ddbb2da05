"""Rayleigh quotient iteration with multigrid (paper sec. 2.1, Alg. 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

What Alg. 1 computes: eigenpairs (lambda_i, v_i) of the Hermitian Q with the
smallest |lambda|.  Each unconverged approximation is improved by one step of
inverse iteration with a shift damped by its current residual, solved by the
multigrid-preconditioned FGMRES of sec. 2.2; after the step the vector is made
orthogonal to the approximations that precede it, normalised, put into the
interpolation P (P and Q_c are rebuilt), and its Rayleigh quotient and
residual are recomputed.  The start values are lambda_i = 0 and eps_i = 1, so
the first pass is plain inverse iteration; passes repeat until every residual
is at the tolerance.

Readings where the paper is silent:
  * the projection against earlier vectors is Gram-Schmidt applied twice;
  * when N_eig exceeds the number Nv of interpolation vectors, P is built from
    the Nv current approximations with the smallest |lambda| (ties: lower
    index), kept in index order; when N_eig < Nv, the remaining columns are the
    setup test vectors that follow;
  * the shifted systems are solved to a relative residual ``solve_tol``;
  * optional (``rayleigh_ritz``, not in the paper): after every pass the
    approximations are replaced by the Ritz vectors of their span, ordered by
    (|w|, w); this resolves pairs that inverse iteration alone cannot separate
    within a near-degenerate cluster;
  * results are returned sorted by (|lambda|, lambda).
"""
from __future__ import annotations

import numpy as np

from .krylov import dot, norm
from .mg import orthonormalise


def select_for_P(lam, n_eig: int, nv: int):
    """Indices of the current approximations that build P (index order)."""
    if n_eig <= nv:
        return list(range(n_eig))
    order = sorted(range(n_eig), key=lambda i: (abs(lam[i]), i))
    return sorted(order[:nv])


def rebuild_P(mg, v, lam, W_pad):
    nv = W_pad.shape[0]
    idx = select_for_P(lam, v.shape[0], nv)
    cols = [v[i] for i in idx]
    cols += [W_pad[k] for k in range(len(idx), nv)]
    mg.set_vectors(np.stack(cols))


def damped_shift(lam_i: float, eps_i: float) -> float:
    """The shift of Alg. 1: the Rayleigh quotient pulled towards zero by the
    residual, lambda * max(1 - eps, 0) (inverse iteration while eps >= 1)."""
    return lam_i * max(1.0 - eps_i, 0.0)


def project_out(x, basis):
    """x with its components along the orthonormal ``basis`` vectors removed
    (Gram-Schmidt applied twice)."""
    for _ in range(2):
        for b in basis:
            x = x - dot(b, x) * b
    return x


def rayleigh_pair(op, v):
    """(lambda, eps): the Rayleigh quotient of the unit vector v and the norm of
    its eigen-residual Q v - lambda v."""
    Qv = op.Q(v)
    lam = dot(v, Qv).real
    return lam, norm(Qv - lam * v)


def improve(mg, v, i, lam_i, eps_i, solve_tol):
    """The new unit vector for approximation i: the shifted solve started from
    v_i, made orthogonal to v_0 .. v_{i-1}.  Returns (vector, FGMRES info)."""
    x, info = mg.solve(damped_shift(lam_i, eps_i), v[i], solve_tol)
    x = project_out(x, v[:i])
    return x / norm(x), info


def wanted_converged(lam, eps, n_want: int, tol: float) -> bool:
    """The n_want approximations with the smallest |lambda| are at the tolerance."""
    idx = np.argsort(np.abs(lam), kind="stable")[:n_want]
    return bool(np.all(eps[idx] <= tol))


def rqi(mg, V0, tol: float, W_pad=None, solve_tol: float = 1e-8,
        max_sweeps: int = 30, callback=None, rayleigh_ritz: bool = False, n_want=None):
    """Alg. 1.  ``mg`` is a hierarchy with ``set_vectors``, ``solve`` and the
    field arguments; ``V0`` [n_eig, 12, V] are the start vectors; ``W_pad`` the
    setup test vectors (their count is Nv).  With ``n_want`` the passes stop
    once the n_want smallest |lambda| have converged (the other vectors are a
    guard band against missed modes); otherwise all must converge.  Returns
    (lambda, v, eps, info), all n_eig approximations sorted."""
    op = mg.op
    v = orthonormalise(V0)
    n_eig = v.shape[0]
    if W_pad is None:
        W_pad = v
    lam = np.zeros(n_eig)
    eps = np.ones(n_eig)
    rebuild_P(mg, v, lam, W_pad)
    solves = []
    sweeps = 0
    n_want = n_eig if n_want is None else int(n_want)
    while sweeps < max_sweeps and not wanted_converged(lam, eps, n_want, tol):
        for i in np.flatnonzero(eps > tol):
            v[i], info = improve(mg, v, i, lam[i], eps[i], solve_tol)
            solves.append(info["iters"])
            rebuild_P(mg, v, lam, W_pad)
            lam[i], eps[i] = rayleigh_pair(op, v[i])
            if callback is not None:
                callback(i, lam[i], eps[i])
        sweeps += 1
        if rayleigh_ritz:
            lam, v = rayleigh_ritz_step(op, v)
            eps = residuals(op, lam, v)
            rebuild_P(mg, v, lam, W_pad)
    order = sorted(range(n_eig), key=lambda i: (abs(lam[i]), lam[i]))
    info = {"sweeps": sweeps, "solve_iters": solves, "converged": wanted_converged(lam, eps, n_want, tol)}
    return lam[order], v[order], eps[order], info


def rayleigh_ritz(op, v):
    """Rayleigh-Ritz on span(v) (v orthonormal): H = V^dag Q V, H = C diag(w) C^dag,
    v <- V C, sorted by (|w|, w)."""
    Qv = op.Q(v)
    n = v.shape[0]
    H = np.array([[dot(v[i], Qv[j]) for j in range(n)] for i in range(n)])
    H = 0.5 * (H + H.conj().T)
    w, C = np.linalg.eigh(H)
    order = sorted(range(n), key=lambda i: (abs(w[i]), w[i]))
    w, C = w[order], C[:, order]
    return w, np.einsum("ij,i...->j...", C, v)


def rayleigh_ritz_step(op, v):
    """Rayleigh-Ritz after re-orthonormalising v (the approximations of one
    pass are orthogonal only to their predecessors at the time of each step)."""
    return rayleigh_ritz(op, orthonormalise(v))


def residuals(op, lam, v):
    """eps_i = ||Q v_i - lambda_i v_i|| for each pair."""
    Qv = op.Q(v)
    return np.array([norm(Qv[i] - lam[i] * v[i]) for i in range(v.shape[0])])
