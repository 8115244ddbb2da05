"""GMRES and flexible GMRES with zero initial guess (paper sec. 2 and 2.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper uses restarted GMRES as smoother and coarse-grid solver for Q and a
double-precision flexible GMRES, right-preconditioned by the multigrid cycle,
for every shifted inversion.  Both are written here as textbook Arnoldi with
modified Gram-Schmidt; the small least-squares problem is reduced by Givens
rotations column by column and solved by back substitution.
"""
from __future__ import annotations

import numpy as np


def dot(a, b):
    """<a, b> = sum conj(a) b with pairwise summation."""
    return np.sum(np.conj(a) * b)


def norm(a):
    return float(np.sqrt(np.sum(a.real * a.real + a.imag * a.imag)))


def _givens(a, b):
    """Rotation (c, s), c real, with [[c, s], [-conj(s), c]] [a, b]^T = [r, 0]^T."""
    if a == 0:
        return 0.0, 1.0 + 0j
    r = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    return abs(a) / r, (a / abs(a)) * np.conj(b) / r


class _Arnoldi:
    """Hessenberg matrix reduced by Givens rotations as columns arrive."""

    def __init__(self, m, beta):
        self.H = np.zeros((m + 1, m), dtype=np.complex128)
        self.cs = np.zeros(m)
        self.sn = np.zeros(m, dtype=np.complex128)
        self.g = np.zeros(m + 1, dtype=np.complex128)
        self.g[0] = beta

    def add_column(self, j, h):
        """h = [h_0j .. h_{j+1,j}]; returns |residual| after j + 1 steps."""
        H = self.H
        H[:j + 2, j] = h
        for i in range(j):
            a, b = H[i, j], H[i + 1, j]
            H[i, j] = self.cs[i] * a + self.sn[i] * b
            H[i + 1, j] = -np.conj(self.sn[i]) * a + self.cs[i] * b
        c, s = _givens(H[j, j], H[j + 1, j])
        self.cs[j], self.sn[j] = c, s
        H[j, j] = c * H[j, j] + s * H[j + 1, j]
        H[j + 1, j] = 0.0
        self.g[j + 1] = -np.conj(s) * self.g[j]
        self.g[j] = c * self.g[j]
        return abs(self.g[j + 1])

    def solve(self, k):
        """Back substitution R y = g on the leading k x k triangle."""
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (self.g[i] - self.H[i, i + 1:k] @ y[i + 1:k]) / self.H[i, i]
        return y


def gmres(apply_A, b, m: int, tol: float):
    """At most m Arnoldi steps of GMRES on A x = b from x0 = 0 (modified
    Gram-Schmidt, Givens rotations).

    Stops early when the residual estimate is <= tol * ||b|| (tol = 0:
    always m steps, unless the Krylov space becomes invariant).  Returns
    (x, steps, residual estimate)."""
    beta = norm(b)
    x = np.zeros_like(b)
    if beta == 0.0 or m == 0:
        return x, 0, beta
    arn = _Arnoldi(m, beta)
    Vs = [b / beta]
    k = 0
    res = beta
    for j in range(m):
        w = apply_A(Vs[j])
        h = np.zeros(j + 2, dtype=np.complex128)
        for i in range(j + 1):
            h[i] = dot(Vs[i], w)
            w = w - h[i] * Vs[i]
        h[j + 1] = norm(w)
        res = arn.add_column(j, h)
        k = j + 1
        if h[j + 1] == 0.0 or res <= tol * beta:
            break
        Vs.append(w / h[j + 1].real)
    y = arn.solve(k)
    for i in range(k):
        x = x + y[i] * Vs[i]
    return x, k, res


def fgmres(apply_A, apply_M, b, m: int, tol: float, max_restarts: int = 50):
    """Restarted flexible GMRES(m), right preconditioner ``apply_M`` (which may
    change from step to step), x0 = 0.  Converged when the true residual
    ||b - A x|| <= tol * ||b||.  Returns (x, info) with info a dict holding
    the iteration count, the final relative residual and a convergence flag."""
    bnorm = norm(b)
    x = np.zeros_like(b)
    info = {"iters": 0, "relres": 0.0, "converged": True}
    if bnorm == 0.0:
        return x, info
    r = b.copy()
    for _cycle in range(max_restarts + 1):
        beta = norm(r)
        if beta <= tol * bnorm:
            break
        arn = _Arnoldi(m, beta)
        Vs = [r / beta]
        Zs = []
        k = 0
        for j in range(m):
            z = apply_M(Vs[j])
            Zs.append(z)
            w = apply_A(z)
            h = np.zeros(j + 2, dtype=np.complex128)
            for i in range(j + 1):
                h[i] = dot(Vs[i], w)
                w = w - h[i] * Vs[i]
            h[j + 1] = norm(w)
            res = arn.add_column(j, h)
            k = j + 1
            info["iters"] += 1
            if h[j + 1] == 0.0 or res <= tol * bnorm:
                break
            Vs.append(w / h[j + 1].real)
        y = arn.solve(k)
        for i in range(k):
            x = x + y[i] * Zs[i]
        r = b - apply_A(x)
    relres = norm(r) / bnorm
    info["relres"] = relres
    info["converged"] = relres <= tol
    return x, info
