"""The learned setup: a gauge-equivariant network of parallel-transport
convolutions proposes the multigrid test vectors from the gauge field (not
part of the paper; the plain adaptive setup of sec. 2.1 stays the fallback and
the reference).

Every numerical step is a library call (lq_ptc_forward / backward,
lq_mod_relu(_backward), lq_proj_loss, lq_adam_step, mg_setup, rqi_lowmodes);
this module only sequences them:
  * training: for each generated field, the K lowest eigenvectors of Q from
    rqi_lowmodes are the targets; one or more steps of forward, projection
    loss over the aggregates, backward and Adam update the weights;
  * inference: the network maps the plain setup's seeded Gaussian start
    vectors to test vectors, which mg_setup takes in their place (with fewer
    multigrid passes);
  * fallback: if the eigensolver started from the learned hierarchy does not
    reach the tolerance, the plain setup is run and the solve repeated.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from .lqmg import Context, MGParams

CHANNELS = (24, 16, 16, 16, 24)


@dataclass
class Network:
    weights: list            # [c_out, c_in, 81, 4, 4] complex128 on the device, per layer
    biases: list             # [c_out] float64 per hidden layer
    state: list = field(default_factory=list)   # Adam moments (m, v) per parameter
    step: int = 0

    def parameters(self):
        return list(self.weights) + list(self.biases)


def init_network(channels=CHANNELS, seed: int = 5000, scale: float = 1.0) -> Network:
    """Seeded initial weights (input generation: torch's generator on the
    device).  Each layer starts near an identity transport plus small
    couplings: the offset-0 spin matrix is the identity between channel i and
    output i mod c_out, the other entries are Gaussian with standard deviation
    scale / sqrt(81 c_in); biases start at zero (modReLU passes everything)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    Ws, bs = [], []
    for layer, (ci, co) in enumerate(zip(channels[:-1], channels[1:])):
        shape = (co, ci, 81, 4, 4)
        re = torch.randn(shape, generator=g, device="cuda", dtype=torch.float64)
        im = torch.randn(shape, generator=g, device="cuda", dtype=torch.float64)
        W = torch.complex(re, im) * (scale / np.sqrt(2 * 81 * ci))
        centre = 40                                    # offset (0, 0, 0, 0)
        for o in range(co):
            W[o, o % ci, centre] += torch.eye(4, dtype=torch.complex128, device="cuda")
        Ws.append(W.contiguous())
        if layer < len(channels) - 2:
            bs.append(torch.zeros(co, dtype=torch.float64, device="cuda"))
    net = Network(Ws, bs)
    for p in net.parameters():
        pr = torch.view_as_real(p) if p.is_complex() else p
        net.state.append((torch.zeros_like(pr), torch.zeros_like(pr)))
    return net


def gaussian_fields(n, V, seed):
    """n seeded complex Gaussian fields [n, 12, V] on the device (input generation)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    out = torch.empty((n, 12, V), dtype=torch.complex128, device="cuda")
    view = torch.view_as_real(out)
    for k in range(n):
        view[k].normal_(generator=g)
    out /= np.sqrt(2.0)
    return out


def eigen_targets(ctx: Context, U, m0, agg, tv0, k: int, tol: float = 1e-6, params: MGParams | None = None):
    """The k lowest eigenvectors of Q (unit, device [k, 12, V]) by the plain
    setup and rqi_lowmodes, and the solve's info."""
    p = params or MGParams(precision=1, rqi_block=16, fgmres_m=8, n_setup=3, coarse_m=40, coarse_restarts=1,
                           coarse_tol=0.3, rqi_start_passes=4, rqi_solve_restarts=0, rqi_guard=16,
                           rayleigh_ritz=1, rqi_max_sweeps=20)
    ctx.mg_setup(U, m0, agg, tv0, p)
    n_v0 = k + p.rqi_guard - min(tv0.shape[0], k + p.rqi_guard)
    V0 = gaussian_fields(n_v0, ctx.V, 7919) if n_v0 > 0 else None
    lam, V, res, info = ctx.rqi_lowmodes(k, tol, V0=V0)
    return V, info


def train_step(ctx: Context, U, net: Network, phi0, targets, agg, lr: float, bf16: bool = False):
    """One step: forward, loss, backward, Adam (bf16: the layers on the
    bfloat16 matrix cores).  Returns the loss before the update."""
    net.step += 1
    return ctx.lcnn_train_step(U, phi0, net.weights, net.biases, targets, agg, net.state, lr, net.step, bf16=bf16)


def propose(ctx: Context, U, net: Network, phi0, bf16: bool = False):
    """The network's test vectors for field U from the start vectors phi0
    (bf16: the layers on the bfloat16 matrix cores)."""
    return ctx.lcnn_forward(U, phi0, net.weights, net.biases, bf16=bf16)


def loss_of(ctx: Context, X, targets, agg):
    """Projection loss of given test vectors X against targets (no gradient)."""
    return ctx.proj_loss(X, targets, agg, grad=False)[0]


def setup_and_solve(ctx: Context, U, m0, agg, tv0, params: MGParams, n_eig: int, tol: float, V0=None):
    """mg_setup + rqi_lowmodes; returns (lambda, V, resid, info, setup_s, rqi_s)."""
    torch.cuda.synchronize()
    t0 = time.time()
    ctx.mg_setup(U, m0, agg, tv0, params)
    torch.cuda.synchronize()
    t1 = time.time()
    lam, V, res, info = ctx.rqi_lowmodes(n_eig, tol, V0=V0)
    torch.cuda.synchronize()
    return lam, V, res, info, t1 - t0, time.time() - t1


def learned_solve(ctx: Context, U, m0, agg, net: Network, phi0, params_learned: MGParams, params_plain: MGParams,
                  n_eig: int, tol: float, V0=None, nv: int | None = None, bf16: bool = False):
    """The learned setup with the plain one as fallback: the network's outputs
    (their first Nv) are the test vectors of a setup with params_learned; if
    the eigensolver then stops short of the tolerance (its residual stalled
    within the sweep limit), the plain setup from phi0 with params_plain is run
    and the solve repeated (bf16: the network's layers on the bfloat16 matrix
    cores).  Returns (lambda, V, resid, info) with info
    extended by 'learned' (bool: the learned hierarchy gave the result),
    'setup_s', 'rqi_s', 'network_s' and, after a fallback, 'fallback_s'."""
    torch.cuda.synchronize()
    t0 = time.time()
    X = propose(ctx, U, net, phi0, bf16=bf16)
    torch.cuda.synchronize()
    t_net = time.time() - t0
    nv = X.shape[0] if nv is None else nv
    lam, V, res, info, ts, tr = setup_and_solve(ctx, U, m0, agg, X[:nv].contiguous(), params_learned, n_eig, tol,
                                                V0)
    info = dict(info, learned=True, network_s=t_net, setup_s=ts, rqi_s=tr)
    if info["converged"]:
        return lam, V, res, info
    t1 = time.time()
    lam, V, res, info2, ts2, tr2 = setup_and_solve(ctx, U, m0, agg, phi0[:nv].contiguous(), params_plain, n_eig, tol,
                                                   V0)
    info = dict(info2, learned=False, network_s=t_net, setup_s=ts2, rqi_s=tr2, fallback_s=time.time() - t1,
                learned_attempt=info)
    return lam, V, res, info
