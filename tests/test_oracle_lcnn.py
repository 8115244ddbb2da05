"""Pins of the oracle's gauge-equivariant network and its training loss against
what fixes them independently: the Wilson-Dirac operator (one layer with the
hopping weights is D), gauge covariance and translation equivariance (which a
wrong path order, a missing dagger or a misplaced boundary sign breaks), the
projector's two extreme cases, finite differences for the gradients, and the
nonlinearity's radial-shift properties."""
import numpy as np
import pytest
import torch

import lqsynth
from oracle import lcnn
from oracle.dirac import Lattice, apply_D


def _random_net(channels, seed):
    g = torch.Generator().manual_seed(seed)
    weights, biases = [], []
    for cin, cout in zip(channels[:-1], channels[1:]):
        scale = 1.0 / np.sqrt(cin * len(lcnn.OFFSETS) * 4)
        re = torch.randn((cout, cin, len(lcnn.OFFSETS), 4, 4), generator=g, dtype=torch.float64)
        im = torch.randn((cout, cin, len(lcnn.OFFSETS), 4, 4), generator=g, dtype=torch.float64)
        weights.append(torch.complex(re, im) * scale)
    for cout in channels[1:-1]:
        biases.append(-0.3 * torch.rand(cout, generator=g, dtype=torch.float64))   # some sites cut by relu
    return weights, biases


def _random_unitaries(V, seed):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((V, 3, 3)) + 1j * rng.standard_normal((V, 3, 3))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=1, axis2=2)
    return Q * (d / np.abs(d))[:, None, :]                 # Omega[x] unitary


@pytest.mark.parametrize("t_bc", [-1, 1])
def test_one_layer_with_hopping_weights_is_the_wilson_operator(t_bc):
    dims = (4, 2, 4, 6)
    lat = Lattice(dims, t_bc)
    U = lqsynth.gauge_field(dims, 0.4, 21)
    phi = lqsynth.gaussian_spinors(2, dims, 22)
    W = lcnn.wilson_weights(-0.27).expand(1, 1, -1, -1, -1)
    trans = lcnn.transports(U, lat)
    for k in range(2):
        y = lcnn.forward(trans, torch.from_numpy(phi[k:k + 1]), [W], []).numpy()[0]
        ref = apply_D(U, -0.27, phi[k], lat)
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("t_bc", [-1, 1])
def test_network_is_gauge_covariant(t_bc):
    # U_mu(x) -> O(x) U_mu(x) O(x + mu)^dag, phi(x) -> O(x) phi(x) must give
    # output(x) -> O(x) output(x): every path product T_d(x) -> O(x) T_d(x) O(x + d)^dag
    dims = (4, 4, 2, 4)
    lat = Lattice(dims, t_bc)
    V = lat.V
    U = lqsynth.gauge_field(dims, 0.5, 31)
    phi = lqsynth.gaussian_spinors(3, dims, 32)
    weights, biases = _random_net((3, 4, 4, 2), 33)
    out = lcnn.forward(lcnn.transports(U, lat), torch.from_numpy(phi), weights, biases).numpy()
    Om = _random_unitaries(V, 34)                            # [V, 3, 3]
    fwd, _, _, _ = lat.tables()
    Um = U.reshape(4, 3, 3, V)
    Ug = np.empty_like(Um)
    for mu in range(4):
        Ug[mu] = np.einsum("xab,bcx,xdc->adx", Om, Um[mu], Om[fwd[mu]].conj())
    def rot(f):                                              # f [C, 12, V] -> O(x) f(x) on colour
        g = f.reshape(f.shape[0], 4, 3, V)
        return np.einsum("xab,isbx->isax", Om, g).reshape(f.shape)
    out_g = lcnn.forward(lcnn.transports(Ug.reshape(4, 9, V), lat), torch.from_numpy(rot(phi)), weights,
                         biases).numpy()
    assert np.abs(out_g - rot(out)).max() <= 1e-12 * np.abs(out).max()


def test_network_is_translation_equivariant():
    dims = (4, 4, 2, 4)
    lat = Lattice(dims, 1)                                   # periodic: translations are symmetries
    U = lqsynth.gauge_field(dims, 0.5, 41)
    phi = lqsynth.gaussian_spinors(2, dims, 42)
    weights, biases = _random_net((2, 3, 2), 43)
    out = lcnn.forward(lcnn.transports(U, lat), torch.from_numpy(phi), weights, biases).numpy()
    s = np.arange(lat.V)
    c = lat.coords(s)
    a = (1, 3, 1, 2)
    shifted = lat.index([(c[m] + a[m]) % dims[m] for m in range(4)])   # f'(x) = f(x + a)
    out_s = lcnn.forward(lcnn.transports(U[..., shifted], lat), torch.from_numpy(phi[..., shifted]), weights,
                         biases).numpy()
    assert np.abs(out_s - out[..., shifted]).max() <= 1e-12 * np.abs(out).max()


def test_projection_loss_is_zero_on_the_span_and_one_off_it():
    dims, agg = (4, 4, 2, 4), (2, 2, 2, 2)
    lat = Lattice(dims, 1)
    rows = lcnn.block_half_rows(lat, agg)
    assert sorted(np.concatenate(rows).tolist()) == list(range(12 * lat.V))   # a partition
    X = lqsynth.gaussian_spinors(5, dims, 51)
    # targets in the span of the outputs on every block: loss 0
    u_in = X[:2] / np.linalg.norm(X[:2].reshape(2, -1), axis=1)[:, None, None]
    L0 = lcnn.projection_loss(torch.from_numpy(X), torch.from_numpy(u_in), rows).item()
    assert L0 < 1e-24
    # unit targets orthogonal to the outputs on every block: loss 1
    v = lqsynth.gaussian_spinors(3, dims, 52).reshape(3, -1)
    Xf = X.reshape(5, -1)
    for r in rows:
        Q, _ = np.linalg.qr(Xf[:, r].T)
        v[:, r] -= (v[:, r] @ Q.conj()) @ Q.T
    v /= np.linalg.norm(v, axis=1)[:, None]
    L1 = lcnn.projection_loss(torch.from_numpy(X), torch.from_numpy(v.reshape(3, 12, lat.V)), rows).item()
    assert abs(L1 - 1.0) < 1e-12


def test_loss_gradients_match_finite_differences():
    dims, agg = (4, 2, 2, 4), (2, 2, 2, 2)
    lat = Lattice(dims, -1)
    rows = lcnn.block_half_rows(lat, agg)
    trans = lcnn.transports(lqsynth.gauge_field(dims, 0.4, 61), lat)
    phi = torch.from_numpy(lqsynth.gaussian_spinors(2, dims, 62))
    u = lqsynth.gaussian_spinors(3, dims, 63)
    u = torch.from_numpy(u / np.linalg.norm(u.reshape(3, -1), axis=1)[:, None, None])
    weights, biases = _random_net((2, 3, 3), 64)
    params = [w.clone().requires_grad_(True) for w in weights] + [b.clone().requires_grad_(True) for b in biases]

    def loss(ps):
        return lcnn.projection_loss(lcnn.forward(trans, phi, ps[:2], ps[2:]), u, rows)

    L = loss(params)
    grads = torch.autograd.grad(L, params)
    g = torch.Generator().manual_seed(65)
    dirs = []
    for p in params:
        d = torch.randn(p.shape, generator=g, dtype=torch.float64)
        if p.is_complex():
            d = torch.complex(d, torch.randn(p.shape, generator=g, dtype=torch.float64))
        dirs.append(d)
    # dL = Re sum conj(grad) * dp for real L (PyTorch's convention for complex leaves)
    dl = sum(float(torch.real((gr.conj() * d).sum())) for gr, d in zip(grads, dirs))
    h = 1e-6
    with torch.no_grad():
        Lp = loss([p + h * d for p, d in zip(params, dirs)]).item()
        Lm = loss([p - h * d for p, d in zip(params, dirs)]).item()
    fd = (Lp - Lm) / (2 * h)
    assert abs(fd - dl) <= 1e-6 * max(abs(dl), 1e-3)


def test_mod_relu_is_a_radial_shift_with_a_cut():
    # Properties that fix the nonlinearity without restating it: per channel
    # and site it keeps the direction of the spinor (a non-negative real
    # factor), b = 0 is the identity, two shifts that cut nothing compose to
    # their sum, scaling the field and the bias together scales the output,
    # and a bias below minus the largest norm cuts every site to zero.  A norm
    # squared in place of the norm, a wrong division or a flipped sign of b
    # breaks one of them.
    g = torch.Generator().manual_seed(141)
    C, V = 3, 40
    phi = torch.complex(torch.randn((C, 4, 3, V), generator=g, dtype=torch.float64),
                        torch.randn((C, 4, 3, V), generator=g, dtype=torch.float64))
    nrm = torch.sqrt((phi.abs() ** 2).sum(dim=(1, 2)))                        # [C, V]
    rmin = float(nrm.min())
    b1 = -0.3 * rmin * torch.rand(C, generator=g, dtype=torch.float64)
    b2 = -0.3 * rmin * torch.rand(C, generator=g, dtype=torch.float64)
    out = lcnn.mod_relu(phi, b1)
    # direction kept: out = s phi with s real and >= 0
    s = (phi.conj() * out).sum(dim=(1, 2)) / nrm ** 2
    assert float(s.imag.abs().max()) < 1e-14 and float(s.real.min()) >= 0
    assert float((out - s[:, None, None, :] * phi).abs().max()) < 1e-13
    # the identity at b = 0
    assert float((lcnn.mod_relu(phi, torch.zeros(C, dtype=torch.float64)) - phi).abs().max()) < 1e-14
    # shifts that cut nothing compose
    two = lcnn.mod_relu(lcnn.mod_relu(phi, b1), b2)
    assert float((two - lcnn.mod_relu(phi, b1 + b2)).abs().max()) < 1e-13
    # joint scaling
    alpha = 2.7
    assert float((lcnn.mod_relu(alpha * phi, alpha * b1) - alpha * out).abs().max()) < 1e-13
    # the cut
    cut = lcnn.mod_relu(phi, -1.01 * float(nrm.max()) * torch.ones(C, dtype=torch.float64))
    assert float(cut.abs().max()) == 0.0
    # a partial cut: exactly the sites with |phi| below -b vanish, the others keep |phi| + b
    bm = -float(nrm.median()) * torch.ones(C, dtype=torch.float64)
    part = lcnn.mod_relu(phi, bm)
    pn = torch.sqrt((part.abs() ** 2).sum(dim=(1, 2)))
    kept = nrm > -bm[:, None]
    assert bool(torch.all(pn[~kept] == 0))
    assert float((pn[kept] - (nrm + bm[:, None])[kept]).abs().max()) < 1e-13
