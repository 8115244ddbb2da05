"""Rayleigh quotient iteration with multigrid (paper sec. 2.1, Alg. 1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Alg. 1 as the paper states it: start from orthonormal vectors with
lambda_i = 0 and eps_i = 1; while some eps_i exceeds the tolerance, visit every
unconverged i in order and
  * take the damped shift sigma = lambda_i * max(1 - eps_i, 0),
  * replace v_i by the multigrid-preconditioned solution of (Q - sigma) x = v_i,
  * remove the components along v_j, j < i, and normalise,
  * put the new v_i into the interpolation P (P and Q_c are rebuilt),
  * set lambda_i = <v_i|Q|v_i> and eps_i = ||Q v_i - lambda_i v_i||.

Readings where the paper is silent:
  * the projection against earlier vectors is Gram-Schmidt applied twice;
  * when N_eig exceeds the number Nv of interpolation vectors, P is built from
    the Nv current approximations with the smallest |lambda| (ties: lower
    index), kept in index order; when N_eig < Nv, the remaining columns are the
    setup test vectors that follow;
  * the shifted systems are solved to a relative residual ``solve_tol``;
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


def rqi(mg, V0, tol: float, W_pad=None, solve_tol: float = 1e-8,
        max_sweeps: int = 30, callback=None):
    """Alg. 1.  ``mg`` is a hierarchy with ``set_vectors``, ``solve`` and the
    field arguments; ``V0`` [n_eig, 12, V] are the start vectors; ``W_pad`` the
    setup test vectors (their count is Nv).  Returns (lambda, v, eps, info)."""
    op = mg.op
    v = orthonormalise(V0)
    n_eig = v.shape[0]
    if W_pad is None:
        W_pad = v
    lam = np.zeros(n_eig)
    eps = np.ones(n_eig)
    rebuild_P(mg, v, lam, W_pad)
    sweeps = 0
    solves = []
    while np.any(eps > tol) and sweeps < max_sweeps:
        for i in range(n_eig):
            if eps[i] <= tol:
                continue
            sigma = lam[i] * max(1.0 - eps[i], 0.0)
            x, info = mg.solve(sigma, v[i], solve_tol)
            solves.append(info["iters"])
            for _ in range(2):
                for j in range(i):
                    x = x - dot(v[j], x) * v[j]
            v[i] = x / norm(x)
            rebuild_P(mg, v, lam, W_pad)
            Qv = op.Q(v[i])
            lam[i] = dot(v[i], Qv).real
            eps[i] = norm(Qv - lam[i] * v[i])
            if callback is not None:
                callback(i, lam[i], eps[i])
        sweeps += 1
    order = sorted(range(n_eig), key=lambda i: (abs(lam[i]), lam[i]))
    info = {"sweeps": sweeps, "solve_iters": solves, "converged": bool(np.all(eps <= tol))}
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


def residuals(op, lam, v):
    """eps_i = ||Q v_i - lambda_i v_i|| for each pair."""
    Qv = op.Q(v)
    return np.array([norm(Qv[i] - lam[i] * v[i]) for i in range(v.shape[0])])
