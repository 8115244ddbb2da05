"""Approximate low-mode averaging (paper sec. 3.2-3.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

With orthonormal approximate eigenvectors v~_i of Q (residuals eps_i) and the
projected matrix A_ij = <v~_i|Q|v~_j>:
  * the low-mode part of Q^{-1} is Q~_low^{-1} = sum_ij (A^{-1})_ij |v~_i><v~_j|
    (for exact eigenvectors A = diag(lambda) and it is sum_i |v_i><v_i| / lambda_i);
  * the rest, Q^{-1} - Q~_low^{-1} = Q^{-1} R~, with the oblique projector
    R~ = 1 - Q V~ A^{-1} V~^dag, is estimated stochastically from noise
    vectors eta: (Q^{-1} R~ eta) eta^dag averaged over the noise;
  * approximations with eps_i / |lambda~_i| > c are left out (the cutoff).
Observables per timeslice t of the lattice (t slowest in the site index):
  * the loop L(t) = sum_{x in t} tr Q^{-1}_{x,x}, split as L_low + L_high;
  * the connected low-mode correlator C_low(t) = (1/V) sum_{x, y, t0 : x_t = t0 + t, y_t = t0}
    tr[(Q~_low^{-1})_{x,y} (Q~_low^{-1})_{y,x}].
Both low-mode parts reduce to the per-timeslice overlaps
O(t)_{ji} = sum_{x in t} v~_j(x)^dag v~_i(x) (12 spin-colour components):
L_low(t) = tr[B O(t)] and C_low(t) = (1/V) sum_t0 tr[B O(t0) B O(t0 + t)] with B = A^{-1}.
"""
from __future__ import annotations

import numpy as np


def select(lam, eps, c: float):
    """Indices of the approximations kept by the cutoff eps / |lambda| <= c."""
    lam = np.asarray(lam, dtype=float)
    eps = np.asarray(eps, dtype=float)
    return [i for i in range(len(lam)) if eps[i] <= c * abs(lam[i])]


def projected_matrix(op, V):
    """A_ij = <v_i|Q|v_j> for fields V [n, 12, Vol]."""
    QV = op.Q(V)
    n = V.shape[0]
    return np.array([[np.vdot(V[i].ravel(), QV[j].ravel()) for j in range(n)] for i in range(n)])


def low_inverse_apply(V, A, x):
    """Q~_low^{-1} x = V A^{-1} V^dag x."""
    c = np.array([np.vdot(v.ravel(), x.ravel()) for v in V])
    return np.einsum("i,i...->...", np.linalg.solve(A, c), V)


def oblique_projector_apply(op, V, A, x):
    """R~ x = x - Q V A^{-1} V^dag x."""
    return x - op.Q(low_inverse_apply(V, A, x))


def slice_overlaps(V, T: int):
    """O[t, j, i] = sum over the sites of timeslice t of v_j^dag v_i (12 components)."""
    n = V.shape[0]
    Vt = V.reshape(n, 12, T, -1)                         # sites: t slowest
    return np.einsum("jctx,ictx->tji", np.conj(Vt), Vt)


def loop_low(V, A, T: int):
    """L_low(t) = tr[A^{-1} O(t)]."""
    B = np.linalg.inv(A)
    O = slice_overlaps(V, T)
    return np.einsum("ij,tji->t", B, O)


def connected_low(V, A, T: int, volume: int):
    """C_low(t) = (1/V) sum_t0 tr[B O(t0) B O(t0 + t)], B = A^{-1}."""
    B = np.linalg.inv(A)
    O = slice_overlaps(V, T)
    M = np.einsum("ij,tjk->tik", B, O)                  # B O(t)
    C = np.zeros(T, dtype=np.complex128)
    for t in range(T):
        for t0 in range(T):
            C[t] += np.trace(M[t0] @ M[(t0 + t) % T])
    return C / volume


def loop_high_sample(op, V, A, eta, s, T: int):
    """One noise sample of L_high(t): with eta a noise field and s = Q^{-1} R~ eta
    (the solution of Q s = R~ eta), the per-timeslice sums of eta^dag s."""
    return np.einsum("ctx,ctx->t", np.conj(eta.reshape(12, T, -1)), s.reshape(12, T, -1))


def loop_exact(Qinv_diag_blocks, T: int):
    """sum over the sites of timeslice t of tr Q^{-1}_{x,x}, from the 12 x 12
    diagonal blocks [Vol, 12, 12] of a dense inverse (small lattices)."""
    tr = np.einsum("xcc->x", Qinv_diag_blocks)
    return tr.reshape(T, -1).sum(axis=1)
