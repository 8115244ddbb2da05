"""Seeded synthetic inputs shared by the tests, the benchmark and the CPU oracle.

This module only draws random numbers and shapes them into inputs; it holds none
of the eigensolver's arithmetic (no Dirac operator, no multigrid, no Krylov or
Rayleigh-quotient step).  Both the HIP path and the oracle receive the arrays it
returns, so every random number the method uses is an input.

Layouts (canonical, shared with the C ABI):
  * site index  i = x + X*(y + Y*(z + Z*t)), x fastest;
  * gauge field U[mu, 3*a + b, i]  (mu = 0..3 for x, y, z, t), complex128, with
    U_mu(n) taking colour b at n + mu_hat to colour a at n;
  * spinor field psi[3*s + c, i]  (spin s = 0..3, colour c = 0..2), complex128;
    several spinors stack on a leading axis.

Gauge-field recipe: every link is U = exp(i * eps * H) with H a traceless
Hermitian Gaussian 3x3 matrix, H = (A + A^dagger)/2 - tr(.)/3 and
A = (N1 + i N2)/sqrt(2), N1, N2 standard normal.  The draws come from one
numpy PCG64 stream, as a C-ordered standard-normal array of shape
[V][4][3][3][2] (site, direction, row, column, re/im).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "gauge_field", "gaussian_spinors", "random_su3", "z2_spinors",
    "site_coords",
]


def volume(dims) -> int:
    X, Y, Z, T = (int(d) for d in dims)
    return X * Y * Z * T


def site_coords(dims):
    """Return (x, y, z, t) integer arrays of length V in canonical site order."""
    X, Y, Z, T = (int(d) for d in dims)
    i = np.arange(volume(dims))
    x = i % X
    y = (i // X) % Y
    z = (i // (X * Y)) % Z
    t = i // (X * Y * Z)
    return x, y, z, t


def _expi_hermitian(H: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*H) for a stack of Hermitian 3x3 matrices via eigh."""
    w, W = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ik,...k,...jk->...ij", W, ph, W.conj())


def gauge_field(dims, eps: float, seed: int, chunk: int = 1 << 18) -> np.ndarray:
    """SU(3) links U = exp(i*eps*H), H traceless Hermitian Gaussian.

    Returns complex128 array of shape [4, 9, V] (canonical layout).  The draw
    is made in site chunks from one generator, so the result does not depend
    on ``chunk``.
    """
    V = volume(dims)
    rng = np.random.default_rng(seed)
    out = np.empty((4, 9, V), dtype=np.complex128)
    for s0 in range(0, V, chunk):
        n = min(chunk, V - s0)
        g = rng.standard_normal((n, 4, 3, 3, 2))
        A = (g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0)
        H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
        tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
        H = H - tr[..., None, None] * np.eye(3)
        U = _expi_hermitian(H, eps)                     # [n, 4, 3, 3]
        # det U = exp(i eps tr H) = 1 up to rounding; remove the rounding drift.
        det = np.linalg.det(U)
        U = U / (det ** (1.0 / 3.0))[..., None, None]
        out[:, :, s0:s0 + n] = U.reshape(n, 4, 9).transpose(1, 2, 0)
    return out


def gaussian_spinors(n: int, dims, seed: int) -> np.ndarray:
    """n complex Gaussian spinor fields (N1 + i N2)/sqrt(2), shape [n, 12, V]."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 12, V, 2))
    return (g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0)


def z2_spinors(n: int, dims, seed: int) -> np.ndarray:
    """n spinor fields with entries drawn from (Z2 + i Z2)/sqrt(2), shape [n, 12, V]."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    b = rng.integers(0, 2, size=(n, 12, V, 2)) * 2 - 1
    return (b[..., 0] + 1j * b[..., 1]) / np.sqrt(2.0)


def random_su3(V: int, seed: int) -> np.ndarray:
    """V Haar-like random SU(3) matrices (QR of complex Gaussians), shape [V, 3, 3]."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((V, 3, 3, 2))
    Z = (g[..., 0] + 1j * g[..., 1]) / np.sqrt(2.0)
    Qm, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Qm = Qm * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Qm)
    return Qm / (det ** (1.0 / 3.0))[:, None, None]
