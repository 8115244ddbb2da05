"""Pins of the oracle's third multigrid level (a level below the paper's two):
the level-2 interpolation P2 on the lattice of aggregates, Q_c2 = P2^dag Q_c P2,
the composite Galerkin identity Q_c2 = (P P2)^dag Q (P P2), and the
three-level cycle reducing to the exact two-level cycle when the level-1
system is solved exactly."""
import numpy as np
import pytest

import lqsynth
from oracle import mg as M
from oracle.dirac import Lattice, WilsonOp

DIMS, AGG1, AGG2, NV1, NV2 = (8, 8, 8, 8), (2, 2, 2, 2), (2, 2, 2, 2), 4, 3


@pytest.fixture(scope="module")
def three():
    lat = Lattice(DIMS, 1)
    U = lqsynth.gauge_field(DIMS, 0.3, 301)
    op = WilsonOp(U, -0.2, lat)
    W = lqsynth.gaussian_spinors(NV1, DIMS, 302)
    mg = M.ThreeLevel(op, AGG1, AGG2, M.MGParams(coarse_m=60, coarse_tol=1e-13, coarse_restarts=20),
                      M.Level2Params(coarse_direct=True))
    rng = np.random.default_rng(303)
    nA1 = 4 ** 4
    W2 = rng.standard_normal((NV2, nA1, 2 * NV1)) + 1j * rng.standard_normal((NV2, nA1, 2 * NV1))
    mg.set_vectors(W, W2)
    ag1, ag2 = mg.ag, mg.ag2
    n2 = ag2.nA * 2 * NV2
    E = np.eye(n2).reshape(n2, ag2.nA, 2 * NV2)
    P2d = M.prolong2(mg.P2, ag2, E, NV1).reshape(n2, -1).T          # [nA1 * 2Nv1, n2]
    return dict(op=op, mg=mg, ag1=ag1, ag2=ag2, W2=W2, P2d=P2d, lat=lat)


def test_level2_lattice_shape(three):
    assert three["ag1"].nb == (4, 4, 4, 4) and three["ag2"].nb == (2, 2, 2, 2)


def test_level2_interpolation_orthonormal_gamma5_split_and_local_qr(three):
    t = three
    P2d, ag2, mg = t["P2d"], t["ag2"], t["mg"]
    assert np.abs(P2d.conj().T @ P2d - np.eye(P2d.shape[1])).max() < 1e-13
    # gamma5^c P2 = P2 gamma5^c2 (the level-1 gamma5 is +1 on the first Nv1 entries of a site)
    g1 = np.tile(M.coarse_gamma5(NV1), ag2.lat.V)
    g2 = np.tile(M.coarse_gamma5(NV2), ag2.nA)
    assert np.abs(g1[:, None] * P2d - P2d * g2[None, :]).max() < 1e-14
    # per level-2 aggregate and half: the QR factor (positive diagonal) of the test vectors
    Wb = M.coarse_to_blocks(ag2, t["W2"], NV1)
    Pb = M.coarse_to_blocks(ag2, mg.P2, NV1)
    for A in range(ag2.nA):
        for h in range(2):
            Qm, Rm = np.linalg.qr(Wb[:, A, h, :].T)
            d = np.diag(Rm)
            assert np.abs(Pb[:, A, h, :].T - Qm * (d / np.abs(d))[None, :]).max() < 1e-12


def test_level2_restrict_prolong_are_the_dense_products(three):
    t = three
    rng = np.random.default_rng(4)
    v = rng.standard_normal((t["ag1"].nA, 2 * NV1)) + 1j * rng.standard_normal((t["ag1"].nA, 2 * NV1))
    c = M.restrict2(t["mg"].P2, t["ag2"], v, NV1)
    assert np.abs(c.ravel() - t["P2d"].conj().T @ v.ravel()).max() < 1e-13
    assert np.abs(M.prolong2(t["mg"].P2, t["ag2"], c, NV1).ravel() - t["P2d"] @ c.ravel()).max() < 1e-13


def test_level2_operator_is_the_galerkin_product(three):
    t = three
    mg = t["mg"]
    Q1 = M.dense_coarse(mg.Qc, t["ag1"])
    Q2 = M.dense_coarse(mg.Qc2, t["ag2"])
    ref = t["P2d"].conj().T @ Q1 @ t["P2d"]
    assert np.abs(Q2 - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(Q2 - Q2.conj().T).max() < 1e-12 * np.abs(Q2).max()


def test_composite_galerkin_identity_through_the_fine_operator(three):
    # Q_c2 = (P P2)^dag Q (P P2): each unit level-2 vector prolonged twice to a
    # fine field, Q applied on the fine lattice, restricted twice.  Checks the
    # direction bookkeeping of Q_c2 against the fine operator itself.
    t = three
    mg, ag1, ag2 = t["mg"], t["ag1"], t["ag2"]
    n2 = ag2.nA * 2 * NV2
    E = np.eye(n2).reshape(n2, ag2.nA, 2 * NV2)
    fine = M.prolong(mg.P, ag1, M.prolong2(mg.P2, ag2, E, NV1))        # [n2, 12, V]
    back = M.restrict2(mg.P2, ag2, M.restrict(mg.P, ag1, t["op"].Q(fine)), NV1)
    ref = back.reshape(n2, n2).T
    Q2 = M.dense_coarse(mg.Qc2, ag2)
    assert np.abs(Q2 - ref).max() < 1e-12 * np.abs(ref).max()


def test_level2_correction_annihilates_range_of_P2(three):
    # (1 - P2 (Q_c2 - s)^{-1} P2^dag (Q_c - s)) P2 = 0, the level-1 analogue of sec. 2's projector
    t = three
    mg = t["mg"]
    s = 0.013
    Q1 = M.dense_coarse(mg.Qc, t["ag1"]) - s * np.eye(t["P2d"].shape[0])
    Q2 = t["P2d"].conj().T @ Q1 @ t["P2d"]
    E = np.eye(t["P2d"].shape[0]) - t["P2d"] @ np.linalg.solve(Q2, t["P2d"].conj().T @ Q1)
    assert np.abs(E @ t["P2d"]).max() < 1e-10


def test_three_level_cycle_with_exact_level1_solve_is_the_exact_two_grid_cycle(three):
    # With the level-1 system solved to 1e-13 (FGMRES preconditioned by the
    # level-1 cycle) the three-level cycle equals the two-grid cycle of eq.
    # E_2g with an exact coarse solve.
    t = three
    mg = t["mg"]
    two = M.TwoLevel(t["op"], AGG1, M.MGParams(coarse_direct=True))
    two.P, two.Qc = mg.P, mg.Qc
    r = lqsynth.gaussian_spinors(1, DIMS, 305)[0]
    for s in (0.0, 0.02):
        z3 = mg.cycle(s, r)
        z2 = two.cycle(s, r)
        assert np.abs(z3 - z2).max() < 1e-9 * np.abs(z2).max()


def test_three_level_preconditioned_fgmres_solves_the_fine_system(three):
    t = three
    mg = M.ThreeLevel(t["op"], AGG1, AGG2, M.MGParams(coarse_m=30, coarse_tol=0.05, coarse_restarts=2),
                      M.Level2Params(coarse_tol=0.05, coarse_m=40))
    mg.set_vectors(lqsynth.gaussian_spinors(NV1, DIMS, 302), t["W2"])
    b = lqsynth.gaussian_spinors(1, DIMS, 306)[0]
    x, info = mg.solve(0.01, b, 1e-10)
    assert info["converged"]
    r = b - (t["op"].Q(x) - 0.01 * x)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
