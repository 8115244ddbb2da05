"""Pins of the oracle's multigrid pieces (paper sec. 2): the gamma5-split P,
the Galerkin coarse operator and its identities, the SAP smoother, GMRES /
FGMRES and the two-grid error propagator E_2g."""
import numpy as np
import pytest

import lqsynth
from oracle import mg as M
from oracle.dirac import Lattice, WilsonOp, dense_Q, gamma5
from oracle.krylov import fgmres, gmres, norm

DIMS = (4, 4, 4, 4)
AGG = (2, 2, 2, 2)
NV = 4


@pytest.fixture(scope="module")
def setup_small():
    lat = Lattice(DIMS, 1)
    U = lqsynth.gauge_field(DIMS, 0.4, 101)
    m0 = -0.3
    op = WilsonOp(U, m0, lat)
    ag = M.Aggregation(lat, AGG)
    W = lqsynth.gaussian_spinors(NV, DIMS, 7)
    P = M.build_P(W, ag)
    Qd = dense_Q(U, m0, lat)
    Dd = dense_Q(U, m0, lat, which="D")
    n = ag.nA * 2 * NV
    E = np.eye(n).reshape(n, ag.nA, 2 * NV)
    Pd = M.prolong(P, ag, E).reshape(n, -1).T          # [12V, n]
    return dict(lat=lat, U=U, m0=m0, op=op, ag=ag, W=W, P=P, Qd=Qd, Dd=Dd, Pd=Pd)


def test_interpolation_orthonormal_and_gamma5_split(setup_small):
    s = setup_small
    Pd, ag = s["Pd"], s["ag"]
    assert np.abs(Pd.conj().T @ Pd - np.eye(Pd.shape[1])).max() < 1e-13
    # gamma5 P = P gamma5^c (eq. gamma5 P = P gamma5^c)
    g5 = np.repeat([1.0, 1.0, -1.0, -1.0], 3 * s["lat"].V)
    g5c = np.tile(M.coarse_gamma5(NV), ag.nA)
    assert np.abs(g5[:, None] * Pd - Pd * g5c[None, :]).max() < 1e-14
    # each column lives on one aggregate
    for col in range(Pd.shape[1]):
        A = col // (2 * NV)
        nz = np.nonzero(np.abs(Pd[:, col].reshape(12, -1)).sum(0))[0]
        assert set(ag.block[nz]) <= {A}


def _local_qr(Wm):
    """Q factor of the thin QR of Wm with a positive real diagonal of R (unique
    for full column rank): LAPACK's QR with the phases moved from R to Q."""
    Qm, Rm = np.linalg.qr(Wm)
    d = np.diag(Rm)
    return Qm * (d / np.abs(d))[None, :]


def test_interpolation_is_the_local_qr_factor_of_the_test_vectors(setup_small):
    # sec. 2: P is block diagonal over aggregates and gamma5 halves with
    # orthonormal columns spanning the test vectors' restrictions; built by
    # Gram-Schmidt in vector order it is the QR factor of W_{A,h} with a
    # positive diagonal: span(P_{A,h}[:k]) = span(W_{A,h}[:k]) for every k.
    s = setup_small
    ag = s["ag"]
    Wb, Pb = ag.to_blocks(s["W"]), ag.to_blocks(s["P"])        # [Nv, nA, 2, n]
    for A in range(ag.nA):
        for h in range(2):
            Wm, Pm = Wb[:, A, h, :].T, Pb[:, A, h, :].T
            assert np.abs(Pm - _local_qr(Wm)).max() < 1e-12
            C = Pm.conj().T @ Wm                                  # coefficients of W in P
            assert np.abs(np.tril(C, -1)).max() < 1e-12         # nested spans
            assert np.all(np.diag(C).real > 0)
            assert np.abs(Wm - Pm @ C).max() < 1e-12            # W lies in span(P)


def test_interpolation_is_invariant_under_global_orthonormalisation(setup_small):
    # Gram-Schmidt over the whole lattice changes each test vector by earlier
    # ones with a positive diagonal, an upper-triangular change of basis that
    # leaves every local QR factor unchanged: P(W) = P(orthonormalise(W)).
    s = setup_small
    P2 = M.build_P(M.orthonormalise(s["W"]), s["ag"])
    assert np.abs(P2 - s["P"]).max() < 1e-12


def test_interpolation_rejects_locally_dependent_vectors(setup_small):
    s = setup_small
    W = s["W"].copy()
    # the third vector equals 2x the first on aggregate 0: dependent there only
    sites = s["ag"].sites[0]
    W[2][:, sites] = 2.0 * W[0][:, sites]
    with pytest.raises(np.linalg.LinAlgError):
        M.build_P(W, s["ag"])


def test_restrict_prolong_are_adjoint_dense_products(setup_small):
    s = setup_small
    f = lqsynth.gaussian_spinors(1, DIMS, 8)[0]
    c = M.restrict(s["P"], s["ag"], f).ravel()
    assert np.abs(c - s["Pd"].conj().T @ f.ravel()).max() < 1e-13
    rng = np.random.default_rng(9)
    cc = rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)
    g = M.prolong(s["P"], s["ag"], cc.reshape(s["ag"].nA, 2 * NV)).ravel()
    assert np.abs(g - s["Pd"] @ cc).max() < 1e-13


def test_coarse_operator_is_galerkin_product(setup_small):
    s = setup_small
    Qc = M.coarse_operator(s["op"], s["ag"], s["P"])
    Qcd = M.dense_coarse(Qc, s["ag"])
    ref = s["Pd"].conj().T @ s["Qd"] @ s["Pd"]
    assert np.abs(Qcd - ref).max() < 1e-13
    # Q_c Hermitian; backward blocks are the conjugate transposes of forward ones
    assert np.abs(Qcd - Qcd.conj().T).max() < 1e-13
    ag = s["ag"]
    for mu in range(4):
        back = Qc[ag.cnbr[:, 5 + mu], 1 + mu].conj().transpose(0, 2, 1)
        assert np.abs(Qc[:, 5 + mu] - back).max() < 1e-13
    # gamma5^c D_c Hermitian with D_c = P^dag D P, and gamma5^c D_c = Q_c
    Dc = s["Pd"].conj().T @ s["Dd"] @ s["Pd"]
    g5c = np.tile(M.coarse_gamma5(NV), ag.nA)
    assert np.abs(g5c[:, None] * Dc - Qcd).max() < 1e-13


def test_coarse_grid_corrections_for_D_and_Q_coincide(setup_small):
    s = setup_small
    Pd, Qd, Dd = s["Pd"], s["Qd"], s["Dd"]
    Qc = Pd.conj().T @ Qd @ Pd
    Dc = Pd.conj().T @ Dd @ Pd
    I = np.eye(Qd.shape[0])
    EQ = I - Pd @ np.linalg.solve(Qc, Pd.conj().T @ Qd)
    ED = I - Pd @ np.linalg.solve(Dc, Pd.conj().T @ Dd)
    assert np.abs(EQ - ED).max() < 1e-10
    assert np.abs(EQ @ Pd).max() < 1e-10          # annihilates range(P)
    assert np.abs(EQ @ EQ - EQ).max() < 1e-9     # projector


def _dense_block_schwarz(A, b, blocks_by_colour, sweeps):
    """Multiplicative Schwarz with exact block solves for a dense matrix A."""
    x = np.zeros_like(b)
    for _ in range(sweeps):
        for blocks in blocks_by_colour:
            r = b - A @ x
            for idx in blocks:
                x[idx] += np.linalg.solve(A[np.ix_(idx, idx)], r[idx])
    return x


def test_sap_exact_blocks_equal_schwarz_on_Q_minus_sigma(setup_small):
    # Reading of sec. 2: SAP on D_sigma = gamma5 (Q - sigma) with rhs gamma5 r
    # produces exactly the Schwarz iterates of Q - sigma when blocks are solved
    # exactly (gamma5 is site-local and cancels block by block).
    s = setup_small
    ag, lat = s["ag"], s["lat"]
    sigma = 0.07
    r = lqsynth.gaussian_spinors(1, DIMS, 10)[0]
    z = M.sap_exact(s["op"], ag, sigma, r, 2)
    A = s["Qd"] - sigma * np.eye(s["Qd"].shape[0])
    idx_of = []
    for col in (0, 1):
        blocks = []
        for Ab in range(ag.nA):
            if ag.color[Ab] == col:
                sites = ag.sites[Ab]
                blocks.append((np.arange(12)[:, None] * lat.V + sites[None, :]).ravel())
        idx_of.append(blocks)
    ref = _dense_block_schwarz(A, r.ravel(), idx_of, 2).reshape(12, lat.V)
    assert np.abs(z - ref).max() < 1e-11


def test_sap_mr_converges_to_exact_block_solves(setup_small):
    s = setup_small
    r = lqsynth.gaussian_spinors(1, DIMS, 11)[0]
    ex = M.sap_exact(s["op"], s["ag"], 0.0, r, 1)
    errs = [norm(M.sap(s["op"], s["ag"], 0.0, r, 1, k) - ex) / norm(ex) for k in (2, 8, 64)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-8


def test_mr_step_orthogonality(setup_small):
    # One MR step leaves a block residual orthogonal to D_B rho (the defining
    # property of the minimal-residual step size).
    s = setup_small
    ag, op = s["ag"], s["op"]
    rho = lqsynth.gaussian_spinors(1, DIMS, 12)[0]
    p = M.apply_Dsigma_blocks(op, ag, 0.05, rho)
    alpha = M.block_dot(ag, p, rho) / M.block_dot(ag, p, p).real
    new = rho - alpha[ag.block] * p
    assert np.abs(M.block_dot(ag, p, new)).max() < 1e-12


def test_gmres_full_space_is_exact(setup_small):
    rng = np.random.default_rng(3)
    n = 60
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, k, res = gmres(lambda v: A @ v, b, n, 0.0)
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-9
    x, k, res = gmres(lambda v: A @ v, b, 20, 0.0)
    assert abs(res - norm(b - A @ x)) < 1e-10 * norm(b)


def test_fgmres_multigrid_reaches_dense_solution(setup_small):
    s = setup_small
    p = M.MGParams(coarse_m=128, coarse_tol=1e-10, coarse_restarts=2, n_setup=2)
    mg, W = M.setup(s["op"], AGG, lqsynth.gaussian_spinors(8, DIMS, 13), p)
    b = lqsynth.gaussian_spinors(1, DIMS, 14)[0]
    sigma = 0.03
    x, info = mg.solve(sigma, b, 1e-10)
    ref = np.linalg.solve(s["Qd"] - sigma * np.eye(s["Qd"].shape[0]), b.ravel())
    assert info["converged"]
    assert norm(x.ravel() - ref) / norm(ref) < 1e-8
    assert info["iters"] < 60


def test_two_grid_error_propagator(setup_small):
    # eq. E_2g with mu = 0 and nu = 1 (Q in place of D): with an exact coarse
    # solve, I - B A = (I - S A)(I - P Q_c^{-1} P^dag A), S one SAP sweep.
    s = setup_small
    sigma = 0.05
    mg = M.TwoLevel(s["op"], AGG, M.MGParams(pre=0, post=1, n_mr=4, coarse_m=200,
                                             coarse_tol=1e-12, coarse_restarts=3))
    mg.set_vectors(s["W"])
    Pd = s["Pd"]
    A = s["Qd"] - sigma * np.eye(s["Qd"].shape[0])
    Ac = Pd.conj().T @ A @ Pd
    x = lqsynth.gaussian_spinors(1, DIMS, 15)[0].ravel()

    def S(v):
        return M.sap(s["op"], s["ag"], sigma, v.reshape(12, -1), 1, 4).ravel()

    Ax = A @ x
    lhs = x - mg.cycle(sigma, Ax.reshape(12, -1)).ravel()
    y = x - Pd @ np.linalg.solve(Ac, Pd.conj().T @ Ax)
    rhs = y - S(A @ y)
    assert norm(lhs - rhs) < 1e-9 * norm(x)
