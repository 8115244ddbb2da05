"""Wilson-Dirac operator D and its Hermitian form Q = gamma5 D (paper sec. 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions
  * gamma basis (chiral): gamma_k = [[0, i sigma_k], [-i sigma_k, 0]] for
    k = 1, 2, 3 (x, y, z) and gamma_4 = [[0, 1], [1, 0]] (t).  With it
    gamma5 = -gamma1 gamma2 gamma3 gamma4 = diag(1, 1, -1, -1), the
    representation the paper requires in sec. 2.
  * D psi(n) = (4 + m0) psi(n)
        - 1/2 sum_mu [ (1 - gamma_mu) U_mu(n) psi(n + mu)
                       + (1 + gamma_mu) U_mu(n - mu)^dag psi(n - mu) ],
    Wilson parameter r = 1; a hop in t across the boundary t = T-1 <-> 0 is
    multiplied by ``t_bc`` (-1 antiperiodic, +1 periodic).  The paper names the
    (clover-improved) Wilson operator without writing it; the benchmark
    workloads take c_sw = 0, and WilsonOp adds the clover term of clover.py
    for c_sw != 0.
  * fields are [..., 12, V] with component 3*s + c and canonical site order
    (x fastest); links are U[mu, 3*a + b, V].
"""
from __future__ import annotations

import numpy as np

SIGMA = [
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]


def _gamma_basis():
    z = np.zeros((2, 2), dtype=np.complex128)
    one = np.eye(2, dtype=np.complex128)
    g = []
    for k in range(3):
        g.append(np.block([[z, 1j * SIGMA[k]], [-1j * SIGMA[k], z]]))
    g.append(np.block([[z, one], [one, z]]))
    return g


GAMMA = _gamma_basis()                      # gamma_mu for mu = 0..3 (x, y, z, t)
GAMMA5 = -GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ID4 = np.eye(4, dtype=np.complex128)
G5DIAG = np.array([1.0, 1.0, -1.0, -1.0])   # gamma5 is diagonal in this basis


class Lattice:
    """Periodic 4D lattice with a sign on the t-boundary hop."""

    def __init__(self, dims, t_bc: int = -1):
        self.dims = tuple(int(d) for d in dims)
        X, Y, Z, T = self.dims
        self.V = X * Y * Z * T
        self.t_bc = int(t_bc)
        self._tables = None

    def coords(self, sites):
        X, Y, Z, T = self.dims
        sites = np.asarray(sites)
        return (sites % X, (sites // X) % Y, (sites // (X * Y)) % Z,
                sites // (X * Y * Z))

    def index(self, c):
        X, Y, Z, T = self.dims
        return c[0] + X * (c[1] + Y * (c[2] + Z * c[3]))

    def neighbour(self, sites, mu: int, step: int):
        """Neighbour index of ``sites`` in direction mu (step = +1 or -1) and the
        boundary sign carried by that hop."""
        c = list(self.coords(sites))
        L = self.dims[mu]
        new = c[mu] + step
        sign = np.ones(np.shape(sites))
        if mu == 3:
            crossing = (new < 0) | (new >= L)
            sign = np.where(crossing, float(self.t_bc), 1.0)
        c[mu] = new % L
        return self.index(c), sign

    def tables(self):
        """Full neighbour tables fwd[mu], bwd[mu] and their signs (cached)."""
        if self._tables is None:
            s = np.arange(self.V)
            fwd, fs, bwd, bs = [], [], [], []
            for mu in range(4):
                n, sg = self.neighbour(s, mu, +1)
                fwd.append(n); fs.append(sg)
                n, sg = self.neighbour(s, mu, -1)
                bwd.append(n); bs.append(sg)
            self._tables = (fwd, fs, bwd, bs)
        return self._tables


def spin_mul(M, psi):
    """Apply the 4x4 spin matrix M to psi[..., 4, 3, V]."""
    rows = []
    for s in range(4):
        acc = 0
        for t in range(4):
            if M[s, t] != 0:
                acc = acc + M[s, t] * psi[..., t, :, :]
        rows.append(acc * np.ones_like(psi[..., 0, :, :]))
    return np.stack(rows, axis=-3)


def colour_mul(Um, p):
    """out[..., s, a, n] = sum_b Um[a, b, n] p[..., s, b, n] for Um[3, 3, V]."""
    return np.stack([Um[a, 0] * p[..., 0, :] + Um[a, 1] * p[..., 1, :]
                     + Um[a, 2] * p[..., 2, :] for a in range(3)], axis=-2)


def colour_mul_dag(Um, p):
    """out[..., s, a, n] = sum_b conj(Um[b, a, n]) p[..., s, b, n] (U^dagger p)."""
    Uc = Um.conj()
    return np.stack([Uc[0, a] * p[..., 0, :] + Uc[1, a] * p[..., 1, :]
                     + Uc[2, a] * p[..., 2, :] for a in range(3)], axis=-2)


def _as_spin_colour(psi, V):
    return psi.reshape(psi.shape[:-2] + (4, 3, V))


def hop_forward(U, psi, lat: Lattice, mu: int):
    """F_mu psi(n) = (1 - gamma_mu) U_mu(n) psi(n + mu), BC sign included.
    psi: [..., 12, V]; returns [..., 12, V]."""
    V = lat.V
    fwd, fs, _, _ = lat.tables()
    p = _as_spin_colour(psi, V)[..., fwd[mu]] * fs[mu]
    Um = U[mu].reshape(3, 3, V)
    up = colour_mul(Um, p)
    return spin_mul(ID4 - GAMMA[mu], up).reshape(psi.shape)


def hop_backward(U, psi, lat: Lattice, mu: int):
    """B_mu psi(n) = (1 + gamma_mu) U_mu(n - mu)^dag psi(n - mu), BC sign included."""
    V = lat.V
    _, _, bwd, bs = lat.tables()
    p = _as_spin_colour(psi, V)[..., bwd[mu]] * bs[mu]
    Um = U[mu].reshape(3, 3, V)[:, :, bwd[mu]]
    up = colour_mul_dag(Um, p)
    return spin_mul(ID4 + GAMMA[mu], up).reshape(psi.shape)


def gamma5(psi):
    """gamma5 psi for psi[..., 12, V] (diag(1,1,-1,-1) on spin)."""
    out = psi.copy()
    out[..., 6:, :] *= -1.0
    return out


def apply_D(U, m0: float, psi, lat: Lattice):
    """Wilson-Dirac operator D psi (formula in the module docstring)."""
    y = (4.0 + m0) * psi
    for mu in range(4):
        y = y - 0.5 * (hop_forward(U, psi, lat, mu) + hop_backward(U, psi, lat, mu))
    return y


def apply_Q(U, m0: float, psi, lat: Lattice):
    """Hermitian Wilson-Dirac operator Q psi = gamma5 D psi (sec. 2)."""
    return gamma5(apply_D(U, m0, psi, lat))


def apply_Q_sites(U, m0: float, psi, lat: Lattice, sites):
    """(Q psi)(n) for the listed sites only, computed from the definition.

    Used to check large lattices one site at a time; needs no neighbour tables.
    Returns [12, len(sites)]."""
    sites = np.asarray(sites)
    ps = psi.reshape(4, 3, lat.V)
    y = (4.0 + m0) * ps[:, :, sites]
    for mu in range(4):
        nf, sf = lat.neighbour(sites, mu, +1)
        nb, sb = lat.neighbour(sites, mu, -1)
        Uf = U[mu].reshape(3, 3, lat.V)[:, :, sites]
        Ub = U[mu].reshape(3, 3, lat.V)[:, :, nb]
        fwd = colour_mul(Uf, ps[:, :, nf] * sf)
        bwd = colour_mul_dag(Ub, ps[:, :, nb] * sb)
        y = y - 0.5 * (spin_mul(ID4 - GAMMA[mu], fwd) + spin_mul(ID4 + GAMMA[mu], bwd))
    y = y * G5DIAG[:, None, None]
    return y.reshape(12, len(sites))


def dense_Q(U, m0: float, lat: Lattice, which: str = "Q"):
    """Dense matrix of Q (or D) on C^{12 V}; column j = Q e_j.  Small V only."""
    n = 12 * lat.V
    M = np.empty((n, n), dtype=np.complex128)
    op = apply_Q if which == "Q" else apply_D
    chunk = 768
    for j0 in range(0, n, chunk):
        k = min(chunk, n - j0)
        E = np.zeros((k, n), dtype=np.complex128)
        E[np.arange(k), j0 + np.arange(k)] = 1.0
        M[:, j0:j0 + k] = op(U, m0, E.reshape(k, 12, lat.V), lat).reshape(k, n).T
    return M


class WilsonOp:
    """D and Q for one gauge field, with each hop term held as a sparse matrix.

    The matrices are assembled entry by entry from the same formula as
    ``hop_forward``/``hop_backward``: for the forward hop in direction mu the
    entry at row (3s + a, n), column (3t + b, n + mu) is
    (1 - gamma_mu)[s, t] * U_mu(n)[a, b] * (boundary sign); the backward hop
    has (1 + gamma_mu)[s, t] * conj(U_mu(n - mu)[b, a]) at column (3t + b, n - mu).
    Vectors are flattened as index (3s + c) * V + n.  ``scipy.sparse`` only
    performs the matrix-vector products."""

    def __init__(self, U, m0: float, lat: Lattice, csw: float = 0.0):
        import scipy.sparse as sp
        self.U, self.m0, self.lat = U, float(m0), lat
        self.csw = float(csw)
        self.C = None
        if self.csw != 0.0:
            from .clover import clover_matrix
            self.C = clover_matrix(U, lat, self.csw)
        V = lat.V
        fwd, fs, bwd, bs = lat.tables()
        n = np.arange(V)
        self.F, self.B = [], []
        for mu in range(4):
            for kind in ("F", "B"):
                if kind == "F":
                    S = ID4 - GAMMA[mu]
                    nb, sg = fwd[mu], fs[mu]
                    Uab = lambda a, b: U[mu, 3 * a + b, :]
                else:
                    S = ID4 + GAMMA[mu]
                    nb, sg = bwd[mu], bs[mu]
                    Uab = lambda a, b: np.conj(U[mu, 3 * b + a, bwd[mu]])
                rows, cols, vals = [], [], []
                for s in range(4):
                    for t in range(4):
                        if S[s, t] == 0:
                            continue
                        for a in range(3):
                            for b in range(3):
                                rows.append((3 * s + a) * V + n)
                                cols.append((3 * t + b) * V + nb)
                                vals.append(S[s, t] * Uab(a, b) * sg)
                M = sp.csr_matrix((np.concatenate(vals),
                                   (np.concatenate(rows), np.concatenate(cols))),
                                  shape=(12 * V, 12 * V))
                (self.F if kind == "F" else self.B).append(M)
        self.g5 = np.repeat(G5DIAG, 3 * V)

    def _mv(self, M, psi):
        shp = psi.shape
        X = psi.reshape(-1, 12 * self.lat.V)
        return np.ascontiguousarray((M @ X.T).T).reshape(shp)

    def hop_f(self, psi, mu):
        return self._mv(self.F[mu], psi)

    def hop_b(self, psi, mu):
        return self._mv(self.B[mu], psi)

    def site(self, psi):
        """The site-local part of D: (4 + m0) psi, plus C psi with the clover term."""
        y = (4.0 + self.m0) * psi
        if self.C is not None:
            from .clover import apply_clover
            y = y + apply_clover(self.C, psi)
        return y

    def D(self, psi):
        y = self.site(psi)
        for mu in range(4):
            y = y - 0.5 * (self.hop_f(psi, mu) + self.hop_b(psi, mu))
        return y

    def Q(self, psi):
        return gamma5(self.D(psi))
