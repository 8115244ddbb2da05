"""The restarted Krylov eigensolver on the device (the kind of solver sec. 2.2
compares RQI with multigrid against): restarted Lanczos on Q^2 with a final
Rayleigh-Ritz step with Q.  Its result has a plain definition, the n_eig
eigenpairs of Q of smallest |lambda|, so every eigenvalue is checked against
the dense spectrum of the oracle's Q (each one to 1e-10 relative, so a missed
or duplicated mode fails), the residuals are recomputed with the oracle's Q,
and the vectors must be orthonormal."""
import json
import os

import numpy as np
import pytest

import lqsynth
from oracle.dirac import Lattice, WilsonOp, dense_Q

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.complex128)


def host(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def check_pairs(U, m0, dims, bc, lam, V, res, ref, res_tol):
    lam = np.asarray(lam)
    err = np.abs(lam - ref) / np.abs(ref)
    print("max rel eigenvalue error", err.max(), flush=True)
    assert np.all(err <= 1e-10), (np.flatnonzero(err > 1e-10), lam, ref)
    Vh = host(V)
    Qv = WilsonOp(U, m0, Lattice(dims, bc)).Q(Vh)
    r = np.array([np.linalg.norm(Qv[i] - lam[i] * Vh[i]) for i in range(len(lam))])
    assert np.all(r <= res_tol), r
    assert np.allclose(r, res, rtol=1e-3, atol=1e-14)          # the returned residuals are the true ones
    G = np.einsum("ian,jan->ij", Vh.conj(), Vh)
    assert np.abs(G - np.eye(len(lam))).max() < 1e-10


@pytest.mark.parametrize("name", ["tiny_periodic", "tiny_antiperiodic"])
def test_lanczos_lowest_eight_match_dense(name):
    from paper_1509_06865_amd import Context
    cfg = json.load(open(os.path.join(GOLDEN, "m0.json")))[name]
    dims, bc, m0 = tuple(cfg["dims"]), cfg["t_bc"], cfg["m0"]
    print(f"[lanczos] {name} {dims}, 8 lowest, n_kv 40", flush=True)
    U = lqsynth.gauge_field(dims, cfg["eps"], cfg["field_seed"])
    c = Context(dims, bc)
    v0 = dev(lqsynth.gaussian_spinors(1, dims, 901)[0])
    lam, V, res, info = c.lanczos_lowmodes(dev(U), m0, 8, v0, tol=1e-10, n_kv=40, n_guard=4)
    print(info, flush=True)
    assert info["converged"], info
    ev = np.linalg.eigvalsh(dense_Q(U, m0, Lattice(dims, bc)))
    ref = ev[np.argsort(np.abs(ev), kind="stable")][:8]
    check_pairs(U, m0, dims, bc, lam, V, res, ref, 1e-9)


def test_lanczos_lowest_twenty_match_dense_spectrum():
    # 8x8x4x4 (12,288 unknowns): the 20 lowest against the dense spectrum of the
    # oracle's Q (tests/golden/make_lowmodes.py)
    from paper_1509_06865_amd import Context
    g = json.load(open(os.path.join(GOLDEN, "lowmodes_8x8x4x4.json")))
    dims, bc, m0 = tuple(g["dims"]), g["t_bc"], g["m0"]
    print(f"[lanczos] {dims}, 20 lowest, n_kv 64", flush=True)
    U = lqsynth.gauge_field(dims, g["eps"], g["field_seed"])
    c = Context(dims, bc)
    v0 = dev(lqsynth.gaussian_spinors(1, dims, 902)[0])
    lam, V, res, info = c.lanczos_lowmodes(dev(U), m0, 20, v0, tol=1e-10, n_kv=64, n_guard=4)
    print(info, flush=True)
    assert info["converged"], info
    ref = np.array(g["lowest_by_abs"][:20])
    # the fixture orders equal |lambda| by lambda; the solver returns them in either order
    order = np.lexsort((np.asarray(lam), np.abs(lam)))
    check_pairs(U, m0, dims, bc, np.asarray(lam)[order], V[torch.from_numpy(order).cuda()], np.asarray(res)[order],
                ref, 2e-9)


def test_lanczos_argument_errors():
    from paper_1509_06865_amd import Context, LQError
    cfg = json.load(open(os.path.join(GOLDEN, "m0.json")))["tiny_periodic"]
    dims, bc, m0 = tuple(cfg["dims"]), cfg["t_bc"], cfg["m0"]
    U = dev(lqsynth.gauge_field(dims, cfg["eps"], cfg["field_seed"]))
    c = Context(dims, bc)
    v0 = dev(lqsynth.gaussian_spinors(1, dims, 903)[0])
    with pytest.raises(LQError):
        c.lanczos_lowmodes(U, m0, 8, v0, n_kv=20, n_guard=4)           # n_kv < n_eig + n_guard + 16
    with pytest.raises(LQError):
        c.lanczos_lowmodes(U, m0, 8, v0, n_kv=200)                     # above 191
    with pytest.raises(LQError):
        c.lanczos_lowmodes(U, m0, 8, torch.zeros_like(v0), n_kv=40)    # zero start vector
