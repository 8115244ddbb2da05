"""Aggregation-based multigrid for the shifted Hermitian operator Q - sigma.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed (paper sec. 2):
  * aggregates: the lattice is cut into blocks of extent ``agg``; one coarse
    site per block;
  * interpolation P = diag(P1, P2) split by the gamma5 halves (spins {0,1} and
    {2,3}), so that gamma5 P = P gamma5^c (eq. gamma5 P = P gamma5^c).  For
    each aggregate A and half h, the Nv restrictions of the test vectors are
    orthonormalised (Gram-Schmidt applied twice, in vector order), hence
    P^dag P = 1 and R = P^dag;
  * coarse operator Q_c = P^dag Q P (sec. 2: the coarse-grid corrections of D
    and Q then coincide).  It couples an aggregate to itself and to its eight
    neighbours; it is computed by applying the split hops of Q to each column
    of P.  Because P^dag P = 1, (Q - sigma)_c = Q_c - sigma;
  * smoothers: the Schwarz alternating procedure on D_sigma = gamma5 (Q -
    sigma) = D - sigma gamma5 with right-hand side gamma5 r (red then black
    blocks, each block solved approximately by minimal-residual steps with
    Dirichlet boundary), or restarted GMRES on Q - sigma as in the paper;
  * the two-grid cycle of eq. E_2g: mu pre-smoothing steps, the coarse-grid
    correction P (Q_c - sigma)^{-1} P^dag r (coarse GMRES), nu post-smoothing
    steps;
  * the adaptive setup of sec. 2.1: smoother passes on random vectors, a first
    P, then repeated multigrid iterations on each test vector while keeping
    them orthonormal, rebuilding P and Q_c after each pass.

Layouts: a fine field is [..., 12, V] (component 3*s + c); P is stored as Nv
such fields, its restriction to (aggregate, half) being column (A, h, k).  A
coarse vector is [..., nA, 2*Nv] with index h*Nv + k inside an aggregate.  Q_c
is [nA, 9, 2Nv, 2Nv]: direction 0 is the aggregate itself, 1 + mu the
neighbour A + mu and 5 + mu the neighbour A - mu.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .dirac import Lattice, WilsonOp, gamma5
from .krylov import dot, fgmres, gmres, norm


@dataclass
class MGParams:
    smoother: str = "sap"        # "sap" (on D_sigma) or "gmres" (on Q - sigma)
    pre: int = 0                 # mu: pre-smoothing steps (SAP sweeps / GMRES calls)
    post: int = 3                # nu: post-smoothing steps
    n_mr: int = 4                # MR steps per SAP block solve
    m_smooth: int = 8            # GMRES smoother: Krylov steps per call
    coarse_m: int = 40           # coarse GMRES: restart length
    coarse_tol: float = 0.05     # coarse GMRES: relative residual target
    coarse_restarts: int = 4     # coarse GMRES: restarts after the first cycle
    fgmres_m: int = 10           # outer FGMRES restart length
    fgmres_restarts: int = 40
    n_init: int = 2              # setup: initial smoother passes
    n_setup: int = 4             # setup: multigrid passes
    coarse_direct: bool = False  # exact dense coarse solve (the two-grid method of eq. E_2g)


class Aggregation:
    """Blocks of extent ``agg`` = (ax, ay, az, at); block index of a site is
    bx + nbx*(by + nby*(bz + nbz*bt)) with b_mu = coordinate // a_mu."""

    def __init__(self, lat: Lattice, agg):
        self.lat = lat
        self.agg = tuple(int(a) for a in agg)
        for L, a in zip(lat.dims, self.agg):
            if a <= 0 or L % a:
                raise ValueError(f"aggregate extent {a} does not divide {L}")
        self.nb = tuple(L // a for L, a in zip(lat.dims, self.agg))
        self.nA = int(np.prod(self.nb))
        self.bvol = int(np.prod(self.agg))
        c = lat.coords(np.arange(lat.V))
        bc = [c[m] // self.agg[m] for m in range(4)]
        lc = [c[m] % self.agg[m] for m in range(4)]
        nb, a = self.nb, self.agg
        self.block = bc[0] + nb[0] * (bc[1] + nb[1] * (bc[2] + nb[2] * bc[3]))
        self.local = lc[0] + a[0] * (lc[1] + a[1] * (lc[2] + a[2] * lc[3]))
        self.sites = np.empty((self.nA, self.bvol), dtype=np.int64)
        self.sites[self.block, self.local] = np.arange(lat.V)
        A = np.arange(self.nA)
        ac = [A % nb[0], (A // nb[0]) % nb[1], (A // (nb[0] * nb[1])) % nb[2],
              A // (nb[0] * nb[1] * nb[2])]
        self.color = (ac[0] + ac[1] + ac[2] + ac[3]) % 2
        self.int_fwd = [lc[m] != a[m] - 1 for m in range(4)]
        self.int_bwd = [lc[m] != 0 for m in range(4)]
        self.cnbr = np.empty((self.nA, 9), dtype=np.int64)
        self.cnbr[:, 0] = A
        for m in range(4):
            up = list(ac); up[m] = (ac[m] + 1) % nb[m]
            dn = list(ac); dn[m] = (ac[m] - 1) % nb[m]
            self.cnbr[:, 1 + m] = up[0] + nb[0] * (up[1] + nb[1] * (up[2] + nb[2] * up[3]))
            self.cnbr[:, 5 + m] = dn[0] + nb[0] * (dn[1] + nb[1] * (dn[2] + nb[2] * dn[3]))

    # -- aggregate x half views -------------------------------------------------
    def to_blocks(self, f):
        """[..., 12, V] -> [..., nA, 2, 6*bvol] (aggregate, gamma5 half, local)."""
        lead = f.shape[:-2]
        g = f[..., self.sites]                               # [..., 12, nA, bvol]
        g = g.reshape(lead + (2, 6, self.nA, self.bvol))
        g = np.moveaxis(g, -2, -4)                           # [..., nA, 2, 6, bvol]
        return g.reshape(lead + (self.nA, 2, 6 * self.bvol))

    def from_blocks(self, g):
        lead = g.shape[:-3]
        g = g.reshape(lead + (self.nA, 2, 6, self.bvol))
        g = np.moveaxis(g, -4, -2)                           # [..., 2, 6, nA, bvol]
        g = g.reshape(lead + (12, self.nA, self.bvol))
        f = np.empty(lead + (12, self.lat.V), dtype=g.dtype)
        f[..., self.sites] = g
        return f


# ---------------------------------------------------------------------------
# interpolation, restriction, prolongation
# ---------------------------------------------------------------------------

def build_P(W, ag: Aggregation):
    """Columns of P from test vectors W[Nv, 12, V]: per aggregate and gamma5 half,
    Gram-Schmidt (applied twice) in vector order, then normalisation."""
    Wb = ag.to_blocks(np.asarray(W, dtype=np.complex128))    # [Nv, nA, 2, n]
    Nv = Wb.shape[0]
    Pb = np.empty_like(Wb)
    for k in range(Nv):
        w = Wb[k].copy()
        for _ in range(2):
            for j in range(k):
                w = w - np.sum(np.conj(Pb[j]) * w, axis=-1)[..., None] * Pb[j]
        nrm = np.sqrt(np.sum(np.abs(w) ** 2, axis=-1))
        if np.any(nrm < 1e-12):
            raise np.linalg.LinAlgError("test vectors are locally rank deficient")
        Pb[k] = w / nrm[..., None]
    return ag.from_blocks(Pb)


def restrict(P, ag: Aggregation, f):
    """P^dag f: [..., 12, V] -> [..., nA, 2*Nv]."""
    Pb = ag.to_blocks(P)                                     # [Nv, nA, 2, n]
    fb = ag.to_blocks(f)                                     # [..., nA, 2, n]
    c = np.stack([np.sum(np.conj(Pb[k]) * fb, axis=-1) for k in range(P.shape[0])],
                 axis=-1)                                    # [..., nA, 2, Nv]
    return c.reshape(c.shape[:-2] + (2 * P.shape[0],))


def prolong(P, ag: Aggregation, c):
    """P c: [..., nA, 2*Nv] -> [..., 12, V]."""
    Nv = P.shape[0]
    Pb = ag.to_blocks(P)                                     # [Nv, nA, 2, n]
    cc = c.reshape(c.shape[:-1] + (2, Nv))                   # [..., nA, 2, Nv]
    fb = np.zeros(c.shape[:-2] + Pb.shape[1:], dtype=np.complex128)
    for k in range(Nv):
        fb = fb + Pb[k] * cc[..., k][..., None]
    return ag.from_blocks(fb)


def half_columns(P):
    """The 2*Nv columns of P as separate fields [2Nv, 12, V]: column h*Nv + l
    is P_l with the other gamma5 half set to zero."""
    Nv = P.shape[0]
    cols = np.zeros((2 * Nv,) + P.shape[1:], dtype=np.complex128)
    cols[:Nv, :6] = P[:, :6]
    cols[Nv:, 6:] = P[:, 6:]
    return cols


def coarse_operator(op: WilsonOp, ag: Aggregation, P, chunk: int = 8):
    """Q_c = P^dag Q P as [nA, 9, 2Nv, 2Nv] by split hops (self, +mu, -mu)."""
    Nv = P.shape[0]
    n = 2 * Nv
    Qc = np.zeros((ag.nA, 9, n, n), dtype=np.complex128)
    cols_all = half_columns(P)
    for c0 in range(0, n, chunk):
        cols = cols_all[c0:c0 + chunk]
        parts = []
        self_part = op.site(cols)
        for mu in range(4):
            F = op.hop_f(cols, mu)
            B = op.hop_b(cols, mu)
            self_part = self_part - 0.5 * (F * ag.int_fwd[mu] + B * ag.int_bwd[mu])
            parts.append((1 + mu, -0.5 * F * (~ag.int_fwd[mu])))
            parts.append((5 + mu, -0.5 * B * (~ag.int_bwd[mu])))
        parts.append((0, self_part))
        for d, field in parts:
            r = restrict(P, ag, gamma5(field))               # [k, nA, 2Nv]
            Qc[:, d, :, c0:c0 + cols.shape[0]] = np.moveaxis(r, 0, -1)
    return Qc


def coarse_gamma5(Nv: int):
    """gamma5^c on one coarse site: +1 on the first gamma5 half, -1 on the second."""
    return np.concatenate([np.ones(Nv), -np.ones(Nv)])


def coarse_apply(Qc, ag: Aggregation, x, sigma: float = 0.0):
    """(Q_c - sigma) x for coarse vectors x[..., nA, 2Nv]."""
    y = -sigma * x
    for d in range(9):
        y = y + np.einsum("aij,...aj->...ai", Qc[:, d], x[..., ag.cnbr[:, d], :])
    return y


def dense_coarse(Qc, ag: Aggregation):
    n = Qc.shape[-1]
    M = np.zeros((ag.nA * n, ag.nA * n), dtype=np.complex128)
    for A in range(ag.nA):
        for d in range(9):
            B = ag.cnbr[A, d]
            M[A * n:(A + 1) * n, B * n:(B + 1) * n] += Qc[A, d]
    return M


# ---------------------------------------------------------------------------
# smoothers
# ---------------------------------------------------------------------------

def apply_Dsigma(op: WilsonOp, sigma, psi):
    """D_sigma psi = D psi - sigma gamma5 psi  ( = gamma5 (Q - sigma) psi )."""
    return op.D(psi) - sigma * gamma5(psi)


def apply_Dsigma_blocks(op: WilsonOp, ag: Aggregation, sigma, psi):
    """Block-diagonal part of D_sigma: hops that leave a block are dropped
    (Dirichlet block boundary)."""
    y = op.site(psi) - sigma * gamma5(psi)
    for mu in range(4):
        y = y - 0.5 * (op.hop_f(psi, mu) * ag.int_fwd[mu]
                       + op.hop_b(psi, mu) * ag.int_bwd[mu])
    return y


def block_dot(ag: Aggregation, a, b):
    """Per-block inner products <a|_B, b|_B> for fields [12, V] -> [nA]."""
    return np.sum(np.conj(a[:, ag.sites]) * b[:, ag.sites], axis=(0, 2))


def check_sap_colouring(ag: Aggregation):
    for n in ag.nb:
        if n != 1 and n % 2:
            raise ValueError("SAP needs 1 or an even number of blocks per direction")


def sap(op: WilsonOp, ag: Aggregation, sigma, r, n_sweeps: int, n_mr: int):
    """Multiplicative red/black SAP for D_sigma z = gamma5 r from z = 0.

    In each colour pass the residual is formed with the full operator; every
    block of that colour then takes n_mr minimal-residual steps on its
    Dirichlet block system and adds the correction."""
    check_sap_colouring(ag)
    b = gamma5(r)
    z = np.zeros_like(r)
    site_colour = ag.color[ag.block]
    for _ in range(n_sweeps):
        for col in (0, 1):
            mask = (site_colour == col)
            res = (b - apply_Dsigma(op, sigma, z)) * mask
            e = np.zeros_like(r)
            rho = res
            for _k in range(n_mr):
                p = apply_Dsigma_blocks(op, ag, sigma, rho)
                num = block_dot(ag, p, rho)
                den = block_dot(ag, p, p).real
                alpha = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
                a_site = alpha[ag.block]
                e = e + a_site * rho
                rho = rho - a_site * p
            z = z + e
    return z


def sap_exact(op: WilsonOp, ag: Aggregation, sigma, r, n_sweeps: int):
    """SAP as above but with exact (dense) block solves; small lattices only."""
    check_sap_colouring(ag)
    lat = op.lat
    b = gamma5(r)
    z = np.zeros_like(r)
    n = 12 * ag.bvol
    blocks = []
    for A in range(ag.nA):
        E = np.zeros((n, 12, lat.V), dtype=np.complex128)
        idx = ag.sites[A]
        for j in range(n):
            E[j, j // ag.bvol, idx[j % ag.bvol]] = 1.0
        cols = apply_Dsigma_blocks(op, ag, sigma, E)[:, :, idx].reshape(n, n).T
        blocks.append(cols)
    for _ in range(n_sweeps):
        for col in (0, 1):
            res = b - apply_Dsigma(op, sigma, z)
            for A in range(ag.nA):
                if ag.color[A] != col:
                    continue
                idx = ag.sites[A]
                rb = res[:, idx].reshape(n)
                eb = np.linalg.solve(blocks[A], rb).reshape(12, ag.bvol)
                z[:, idx] = z[:, idx] + eb
    return z


# ---------------------------------------------------------------------------
# two-level hierarchy, cycle, setup
# ---------------------------------------------------------------------------

class TwoLevel:
    """Two-grid method for Q - sigma (eq. E_2g with Q in place of D)."""

    def __init__(self, op: WilsonOp, agg, params: MGParams | None = None):
        self.op = op
        self.U, self.m0, self.lat = op.U, op.m0, op.lat
        self.ag = Aggregation(op.lat, agg)
        self.params = params or MGParams()
        self.P = None
        self.Qc = None
        self._Qc_dense = None

    def set_vectors(self, W):
        self.P = build_P(W, self.ag)
        self.Qc = coarse_operator(self.op, self.ag, self.P)
        self._Qc_dense = None

    def A(self, sigma, x):
        return self.op.Q(x) - sigma * x

    def smooth(self, sigma, r, steps):
        p = self.params
        if p.smoother == "sap":
            return sap(self.op, self.ag, sigma, r, steps, p.n_mr)
        z = np.zeros_like(r)
        for _ in range(steps):
            res = r - self.A(sigma, z)
            z = z + gmres(lambda v: self.A(sigma, v), res, p.m_smooth, 0.0)[0]
        return z

    def coarse_solve(self, sigma, c):
        """Restarted GMRES for (Q_c - sigma) e = c, run on the equivalent system
        gamma5^c (Q_c - sigma) e = gamma5^c c  ( = (D_c - sigma gamma5^c) e ):
        same solution, but the operator's field of values lies near the right
        half plane instead of straddling zero.  Stops when the residual of the
        equivalent system (equal in norm to that of the original one) is
        <= coarse_tol * ||c||, or after coarse_restarts + 1 cycles.  With
        ``coarse_direct`` the coarse system is solved exactly instead."""
        p = self.params
        if p.coarse_direct:
            # exact coarse-grid correction (Q_c - sigma)^{-1} c, dense LU
            if self._Qc_dense is None:
                self._Qc_dense = dense_coarse(self.Qc, self.ag)
            M = self._Qc_dense - sigma * np.eye(self._Qc_dense.shape[0])
            return np.linalg.solve(M, c.reshape(-1)).reshape(c.shape)
        g5c = coarse_gamma5(self.P.shape[0])

        def op(v):
            return g5c * coarse_apply(self.Qc, self.ag, v, sigma)

        rhs = g5c * c
        e = np.zeros_like(c)
        target = p.coarse_tol * norm(c)
        for _ in range(p.coarse_restarts + 1):
            res = rhs - op(e)
            if norm(res) <= target:
                break
            e = e + gmres(op, res, p.coarse_m, target / max(norm(res), 1e-300))[0]
        return e

    def cycle(self, sigma, r):
        """One application of the multigrid preconditioner B_sigma ~ (Q - sigma)^{-1}."""
        p = self.params
        z = np.zeros_like(r)
        if p.pre > 0:
            z = self.smooth(sigma, r, p.pre)
        rc = restrict(self.P, self.ag, r - self.A(sigma, z))
        z = z + prolong(self.P, self.ag, self.coarse_solve(sigma, rc))
        if p.post > 0:
            z = z + self.smooth(sigma, r - self.A(sigma, z), p.post)
        return z

    def solve(self, sigma, b, tol):
        p = self.params
        return fgmres(lambda v: self.A(sigma, v), lambda v: self.cycle(sigma, v), b,
                      p.fgmres_m, tol, p.fgmres_restarts)


def orthonormalise(W):
    """Gram-Schmidt (applied twice) in vector order over the whole lattice."""
    W = np.array(W, dtype=np.complex128, copy=True)
    for k in range(W.shape[0]):
        for _ in range(2):
            for j in range(k):
                W[k] = W[k] - dot(W[j], W[k]) * W[j]
        W[k] = W[k] / norm(W[k])
    return W


def setup(op: WilsonOp, agg, W0, params: MGParams | None = None):
    """Adaptive setup (sec. 2.1): returns the hierarchy and the test vectors."""
    mg = TwoLevel(op, agg, params)
    p = mg.params
    W = np.array(W0, dtype=np.complex128, copy=True)
    for _ in range(p.n_init):
        W = np.stack([mg.smooth(0.0, w, max(p.post, 1)) for w in W])
    W = orthonormalise(W)
    mg.set_vectors(W)
    for _ in range(p.n_setup):
        W = np.stack([mg.cycle(0.0, w) for w in W])
        W = orthonormalise(W)
        mg.set_vectors(W)
    return mg, W


# ---------------------------------------------------------------------------
# a third level: aggregation of the coarse lattice (the paper's hierarchy is
# two-level; the 32^3 x 64 workload adds one level below it)
# ---------------------------------------------------------------------------
#
# Level-1 vectors are [..., nA1, 2 Nv1] (sites of the coarse lattice, index
# h*Nv1 + k inside a site, h the gamma5^c half).  The level-1 sites are cut
# into blocks of extent agg2 of the coarse lattice; P2 holds Nv2 level-1
# vectors whose restriction to (level-2 aggregate A2, half h) are orthonormal
# columns, so gamma5^c P2 = P2 gamma5^c2 and P2^dag P2 = 1 as on the first
# level; Q_c2 = P2^dag Q_c P2 is again a nine-point stencil of dense blocks.

def coarse_lattice(ag: Aggregation) -> Lattice:
    """The lattice of aggregates (coarse sites; boundary signs live in Q_c)."""
    return Lattice(ag.nb, 1)


def coarse_to_blocks(ag2: Aggregation, v, Nv1: int):
    """[..., nA1, 2 Nv1] -> [..., nA2, 2, bvol2 * Nv1] (level-2 aggregate, half, local)."""
    lead = v.shape[:-2]
    g = v.reshape(lead + (v.shape[-2], 2, Nv1))[..., ag2.sites, :, :]      # [..., nA2, bvol2, 2, Nv1]
    g = np.moveaxis(g, -2, -3)                                              # [..., nA2, 2, bvol2, Nv1]
    return g.reshape(lead + (ag2.nA, 2, ag2.bvol * Nv1))


def coarse_from_blocks(ag2: Aggregation, g, Nv1: int):
    lead = g.shape[:-3]
    g = g.reshape(lead + (ag2.nA, 2, ag2.bvol, Nv1))
    g = np.moveaxis(g, -3, -2)                                              # [..., nA2, bvol2, 2, Nv1]
    v = np.empty(lead + (ag2.lat.V, 2, Nv1), dtype=g.dtype)
    v[..., ag2.sites, :, :] = g
    return v.reshape(lead + (ag2.lat.V, 2 * Nv1))


def local_gram_schmidt(Wb):
    """Per block and half, Gram-Schmidt (twice) in vector order and
    normalisation of Wb [Nv, ..., n] over its last axis."""
    Nv = Wb.shape[0]
    Pb = np.empty_like(Wb)
    for k in range(Nv):
        w = Wb[k].copy()
        for _ in range(2):
            for j in range(k):
                w = w - np.sum(np.conj(Pb[j]) * w, axis=-1)[..., None] * Pb[j]
        nrm = np.sqrt(np.sum(np.abs(w) ** 2, axis=-1))
        if np.any(nrm < 1e-12):
            raise np.linalg.LinAlgError("test vectors are locally rank deficient")
        Pb[k] = w / nrm[..., None]
    return Pb


def build_P2(W1, ag2: Aggregation, Nv1: int):
    """Level-2 interpolation from level-1 test vectors W1 [Nv2, nA1, 2 Nv1]."""
    Wb = coarse_to_blocks(ag2, np.asarray(W1, dtype=np.complex128), Nv1)
    return coarse_from_blocks(ag2, local_gram_schmidt(Wb), Nv1)


def restrict2(P2, ag2: Aggregation, v, Nv1: int):
    """P2^dag v: [..., nA1, 2 Nv1] -> [..., nA2, 2 Nv2]."""
    Pb = coarse_to_blocks(ag2, P2, Nv1)                 # [Nv2, nA2, 2, n]
    vb = coarse_to_blocks(ag2, v, Nv1)                  # [..., nA2, 2, n]
    c = np.einsum("kahn,...ahn->...ahk", np.conj(Pb), vb)
    return c.reshape(c.shape[:-2] + (2 * P2.shape[0],))


def prolong2(P2, ag2: Aggregation, c, Nv1: int):
    """P2 c: [..., nA2, 2 Nv2] -> [..., nA1, 2 Nv1]."""
    Nv2 = P2.shape[0]
    Pb = coarse_to_blocks(ag2, P2, Nv1)                 # [Nv2, nA2, 2, n]
    cb = c.reshape(c.shape[:-1] + (2, Nv2))             # [..., nA2, 2, Nv2]
    return coarse_from_blocks(ag2, np.einsum("kahn,...ahk->...ahn", Pb, cb), Nv1)


def coarse_half_columns(P2, Nv1: int):
    """The 2 Nv2 columns of P2 as level-1 vectors: column h*Nv2 + l is P2_l with
    the other gamma5^c half set to zero."""
    Nv2 = P2.shape[0]
    v = P2.reshape(Nv2, P2.shape[1], 2, Nv1)
    cols = np.zeros((2 * Nv2,) + v.shape[1:], dtype=np.complex128)
    cols[:Nv2, :, 0] = v[:, :, 0]
    cols[Nv2:, :, 1] = v[:, :, 1]
    return cols.reshape(2 * Nv2, P2.shape[1], 2 * Nv1)


def coarse_operator2(Qc, ag1: Aggregation, ag2: Aggregation, P2):
    """Q_c2 = P2^dag Q_c P2 as [nA2, 9, 2 Nv2, 2 Nv2]: each coupling term d of
    Q_c (source nb(A1, d), target A1) is assigned to the self block when both
    sites lie in one level-2 aggregate, else to the level-2 direction d."""
    Nv1 = Qc.shape[-1] // 2
    Nv2 = P2.shape[0]
    n = 2 * Nv2
    internal = [np.ones(ag1.nA, dtype=bool)]
    internal += [ag2.int_fwd[m] for m in range(4)] + [ag2.int_bwd[m] for m in range(4)]
    Qc2 = np.zeros((ag2.nA, 9, n, n), dtype=np.complex128)
    for j, x in enumerate(coarse_half_columns(P2, Nv1)):
        parts = np.zeros((9,) + x.shape, dtype=np.complex128)
        for d in range(9):
            term = np.einsum("aij,aj->ai", Qc[:, d], x[ag1.cnbr[:, d]])
            parts[0] += term * internal[d][:, None]
            if d > 0:
                parts[d] += term * (~internal[d])[:, None]
        Qc2[:, :, :, j] = np.moveaxis(restrict2(P2, ag2, parts, Nv1), 0, 1)
    return Qc2


@dataclass
class Level2Params:
    post: int = 2                # level-1 post-smoothing steps
    m_smooth: int = 4            # GMRES steps per level-1 smoothing step (on gamma5^c (Q_c - sigma))
    coarse_m: int = 40           # level-2 GMRES restart length
    coarse_tol: float = 0.05     # level-2 GMRES relative residual target
    coarse_restarts: int = 4
    coarse_direct: bool = False  # exact dense level-2 solve


class ThreeLevel(TwoLevel):
    """Three levels: the level-1 system (Q_c - sigma) e = c of the two-grid
    cycle is solved by FGMRES (restart coarse_m, relative coarse_tol) right-
    preconditioned by a level-1 two-grid cycle: the level-2 correction
    P2 (Q_c2 - sigma)^{-1} P2^dag r, then `post` smoothing steps of GMRES on
    the gamma5^c form of Q_c - sigma."""

    def __init__(self, op: WilsonOp, agg, agg2, params: MGParams | None = None,
                 params2: Level2Params | None = None):
        super().__init__(op, agg, params)
        self.agg2 = tuple(int(a) for a in agg2)
        self.ag2 = Aggregation(coarse_lattice(self.ag), self.agg2)
        self.params2 = params2 or Level2Params()
        self.P2 = None
        self.Qc2 = None
        self._Qc2_dense = None

    def set_vectors(self, W, W2=None):
        """P, Q_c from the fine test vectors W; P2, Q_c2 from the level-1 test
        vectors W2 [Nv2, nA1, 2 Nv1] (default: the restrictions P^dag W)."""
        super().set_vectors(W)
        if W2 is None:
            W2 = restrict(self.P, self.ag, np.asarray(W, dtype=np.complex128))
        self.set_level2(W2)

    def set_level2(self, W2):
        Nv1 = self.P.shape[0]
        self.P2 = build_P2(W2, self.ag2, Nv1)
        self.Qc2 = coarse_operator2(self.Qc, self.ag, self.ag2, self.P2)
        self._Qc2_dense = None

    def A1(self, sigma, v):
        return coarse_apply(self.Qc, self.ag, v, sigma)

    def solve2(self, sigma, c2):
        """(Q_c2 - sigma) e = c2: GMRES on the gamma5^c2 form, or exact."""
        p = self.params2
        if p.coarse_direct:
            if self._Qc2_dense is None:
                self._Qc2_dense = dense_coarse(self.Qc2, self.ag2)
            M = self._Qc2_dense - sigma * np.eye(self._Qc2_dense.shape[0])
            return np.linalg.solve(M, c2.reshape(-1)).reshape(c2.shape)
        g5 = coarse_gamma5(self.P2.shape[0])

        def op(v):
            return g5 * coarse_apply(self.Qc2, self.ag2, v, sigma)

        rhs = g5 * c2
        e = np.zeros_like(c2)
        target = p.coarse_tol * norm(c2)
        for _ in range(p.coarse_restarts + 1):
            res = rhs - op(e)
            if norm(res) <= target:
                break
            e = e + gmres(op, res, p.coarse_m, target / max(norm(res), 1e-300))[0]
        return e

    def smooth1(self, sigma, r, steps):
        """Level-1 smoother: each step m_smooth GMRES steps on
        gamma5^c (Q_c - sigma) for the current residual."""
        g5 = coarse_gamma5(self.P.shape[0])
        z = np.zeros_like(r)
        for _ in range(steps):
            res = g5 * (r - self.A1(sigma, z))
            z = z + gmres(lambda v: g5 * self.A1(sigma, v), res, self.params2.m_smooth, 0.0)[0]
        return z

    def cycle1(self, sigma, r):
        """Level-1 two-grid cycle B1 ~ (Q_c - sigma)^{-1}."""
        Nv1 = self.P.shape[0]
        z = prolong2(self.P2, self.ag2, self.solve2(sigma, restrict2(self.P2, self.ag2, r, Nv1)), Nv1)
        if self.params2.post > 0:
            z = z + self.smooth1(sigma, r - self.A1(sigma, z), self.params2.post)
        return z

    def coarse_solve(self, sigma, c):
        p = self.params
        if p.coarse_direct:
            return super().coarse_solve(sigma, c)
        x, _ = fgmres(lambda v: self.A1(sigma, v), lambda v: self.cycle1(sigma, v), c, p.coarse_m,
                      p.coarse_tol, p.coarse_restarts)
        return x
