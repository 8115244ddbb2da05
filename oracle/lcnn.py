"""Gauge-equivariant convolutional network proposing multigrid test vectors.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no learned component: its setup (sec. 2.1) starts from random
vectors.  This module is the plain reference for an optional learned setup
that maps the gauge field and seeded noise fields to Nv test vectors, and for
the loss it is trained with.  Written with plain PyTorch CPU operations in
complex128 so that autograd supplies the weight gradients.

Layer (parallel-transport convolution): for output channel o,
    phi_out[o](x) = sum_i sum_{d in {-1,0,1}^4} W[o, i, d] T_d(x) phi_in[i](x + d),
W[o, i, d] a 4x4 complex matrix acting on spin, T_d(x) a 3x3 colour matrix: the
product of the links along the path from x to x + d that steps through the
directions mu = 0, 1, 2, 3 in that order; a step +mu from y contributes
U_mu(y), a step -mu contributes U_mu(y - mu)^dag, and a step across the t
boundary the boundary sign.  With W[0] = (4 + m0), W[+mu] = -(1 - gamma_mu)/2
and W[-mu] = -(1 + gamma_mu)/2 one layer is the Wilson-Dirac operator D.
Nonlinearity between layers (gauge invariant): for channel o,
    phi -> phi * relu(|phi(x)| + b[o]) / |phi(x)|,
|phi(x)| the spin-colour norm at site x, b real.  Channels 24 -> 16 -> 16 ->
16 -> 24; no nonlinearity after the last layer.

Loss: with X the network's outputs restricted to aggregate A and gamma5 half h
(a (6 |A|) x n_out matrix) and u_k the K target vectors (unit eigenvectors),
    L = (1/K) sum_k sum_{A,h} || (1 - Pi_{A,h}) u_k|_{A,h} ||^2,
Pi_{A,h} the orthogonal projector onto the span of the columns of X_{A,h}: the
part of each target that an interpolation built from X cannot represent.
"""
from __future__ import annotations

import itertools

import numpy as np
import torch

from .dirac import GAMMA, Lattice

OFFSETS = list(itertools.product((-1, 0, 1), repeat=4))     # 81 offsets d, index = position here
CHANNELS = (24, 16, 16, 16, 24)


def offset_index(d) -> int:
    return OFFSETS.index(tuple(d))


def transports(U: np.ndarray, lat: Lattice):
    """For every offset d: T_d as [3, 3, V] complex and the site index of x + d.

    U: links [4, 9, V] (component 3a + b), canonical site order."""
    V = lat.V
    fwd, fs, bwd, bs = lat.tables()
    Um = U.reshape(4, 3, 3, V)
    eye = np.broadcast_to(np.eye(3, dtype=np.complex128)[:, :, None], (3, 3, V))
    out = []
    for d in OFFSETS:
        pos = np.arange(V)
        T = eye.copy()
        for mu in range(4):
            if d[mu] == 0:
                continue
            if d[mu] > 0:
                step = Um[mu][:, :, pos] * fs[mu][pos]
                pos = fwd[mu][pos]
            else:
                nxt = bwd[mu][pos]
                step = np.conj(np.transpose(Um[mu][:, :, nxt], (1, 0, 2))) * bs[mu][pos]
                pos = nxt
            T = np.einsum("abn,bcn->acn", T, step)
        out.append((torch.from_numpy(np.ascontiguousarray(T)), torch.from_numpy(pos)))
    return out


def ptc_layer(trans, phi: torch.Tensor, W: torch.Tensor) -> torch.Tensor:
    """One parallel-transport convolution.

    trans: output of ``transports``; phi: [C_in, 4, 3, V] complex;
    W: [C_out, C_in, 81, 4, 4] complex.  Returns [C_out, 4, 3, V]."""
    out = None
    for k, (T, pos) in enumerate(trans):
        moved = torch.einsum("abn,itbn->itan", T, phi[..., pos])       # T_d(x) phi(x + d)
        term = torch.einsum("oist,itan->osan", W[:, :, k], moved)
        out = term if out is None else out + term
    return out


def mod_relu(phi: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """phi * relu(|phi(x)| + b[o]) / |phi(x)| per channel o and site x (0 where |phi(x)| = 0)."""
    nrm = torch.sqrt((phi.abs() ** 2).sum(dim=(1, 2)))                  # [C, V]
    scale = torch.relu(nrm + b[:, None]) / torch.where(nrm > 0, nrm, torch.ones_like(nrm))
    return phi * scale[:, None, None, :]


def forward(trans, phi0: torch.Tensor, weights, biases) -> torch.Tensor:
    """The network: ``weights`` a list of layer tensors [C_out, C_in, 81, 4, 4],
    ``biases`` a list (one shorter) of real [C_out] tensors.  phi0: [C_0, 12, V]
    fields (component 3s + c); returns [C_last, 12, V]."""
    V = phi0.shape[-1]
    phi = phi0.reshape(phi0.shape[0], 4, 3, V)
    for layer, W in enumerate(weights):
        phi = ptc_layer(trans, phi, W)
        if layer < len(weights) - 1:
            phi = mod_relu(phi, biases[layer])
    return phi.reshape(phi.shape[0], 12, V)


def wilson_weights(m0: float) -> torch.Tensor:
    """The 1 -> 1 layer weights that make one layer equal to D."""
    W = np.zeros((1, 1, len(OFFSETS), 4, 4), dtype=np.complex128)
    W[0, 0, offset_index((0, 0, 0, 0))] = (4.0 + m0) * np.eye(4)
    for mu in range(4):
        e = [0, 0, 0, 0]
        e[mu] = 1
        W[0, 0, offset_index(e)] = -0.5 * (np.eye(4) - GAMMA[mu])
        e[mu] = -1
        W[0, 0, offset_index(e)] = -0.5 * (np.eye(4) + GAMMA[mu])
    return torch.from_numpy(W)


def block_half_rows(lat: Lattice, agg):
    """Row indices (into a flattened [12 * V] field, index c * V + x for
    component c) of each aggregate and gamma5 half: a list of index arrays."""
    X, Y, Z, T = lat.dims
    s = np.arange(lat.V)
    c = lat.coords(s)
    nb = [lat.dims[m] // agg[m] for m in range(4)]
    blk = (c[0] // agg[0]) + nb[0] * ((c[1] // agg[1]) + nb[1] * ((c[2] // agg[2]) + nb[2] * (c[3] // agg[3])))
    rows = []
    for A in range(int(np.prod(nb))):
        sites = s[blk == A]
        for h in range(2):
            comps = range(6 * h, 6 * h + 6)                 # spins 2h, 2h+1, all colours
            rows.append(np.concatenate([k * lat.V + sites for k in comps]))
    return rows


def projection_loss(X: torch.Tensor, u: torch.Tensor, rows) -> torch.Tensor:
    """L = (1/K) sum_k sum_blocks ||(1 - Pi) u_k||^2 (module docstring).
    X: [n_out, 12, V]; u: [K, 12, V]; rows: ``block_half_rows``."""
    Xf = X.reshape(X.shape[0], -1)
    uf = u.reshape(u.shape[0], -1)
    total = torch.zeros((), dtype=torch.float64)
    for r in rows:
        idx = torch.from_numpy(r)
        M = Xf[:, idx].T                                    # (6|A|) x n_out
        B = uf[:, idx].T                                    # (6|A|) x K
        MH = M.conj().T
        coef = torch.linalg.solve(MH @ M, MH @ B)           # Pi B = M (M^dag M)^-1 M^dag B
        R = B - M @ coef
        total = total + (R.abs() ** 2).sum()
    return total / u.shape[0]
