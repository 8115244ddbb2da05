"""The C-ABI library loads and exports every function include/lqmg.h declares,
and its host-only dense helper is checked against numpy (no device call: this
runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lqmg.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?\**\s*\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "typedef")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("q_apply", "mg_setup", "mg_solve_shifted", "rqi_lowmodes"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1509_06865_amd import lqmg
    if not os.path.exists(lqmg.library_path()):
        pytest.fail("liblqmg.so is not built (python -m paper_1509_06865_amd.build)")
    lib = ctypes.CDLL(lqmg.library_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(lqmg.EXPORTED) == declared_functions()


def test_params_struct_matches_library_defaults():
    from paper_1509_06865_amd import lqmg
    lib = lqmg.load()
    p = lqmg._Params()
    assert lib.lq_params_default(ctypes.byref(p)) == 0
    assert p.rqi_block == 16 and p.fgmres_m == 10 and abs(p.rqi_solve_tol - 1e-6) < 1e-20
    assert p.rqi_deflate == 1 and p.rayleigh_ritz == 1
    assert p.rqi_stall_restarts == 0 and abs(p.rqi_stall_eps - 1e-4) < 1e-20
    assert lib.lq_params_default(None) == -1


def test_create_rejects_bad_arguments():
    from paper_1509_06865_amd import lqmg
    lib = lqmg.load()
    h = ctypes.c_void_p()
    bad = (ctypes.c_int * 4)(4, 4, 1, 4)
    assert lib.lq_create(ctypes.byref(h), bad, -1, None) == -1
    good = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert lib.lq_create(ctypes.byref(h), good, 0, None) == -1


def test_coarse_variant_switch_checks_its_argument():
    # host-only: forcing a coarse-apply kernel accepts -1 (tuned) and 0..7
    from paper_1509_06865_amd.lqmg import LQError, coarse_variant
    for v in (-2, 8, 100):
        with pytest.raises(LQError):
            coarse_variant(v)
    for v in range(8):
        coarse_variant(v)
    coarse_variant(-1)


@pytest.mark.parametrize("n,kind", [(1, "rand"), (7, "rand"), (64, "degen"), (132, "rand"), (132, "degen")])
def test_dense_hermitian_eigensolver_matches_numpy(n, kind):
    # the host eigensolver of the Rayleigh-Ritz step, against numpy's LAPACK,
    # on random spectra and on exactly degenerate ones (clusters of 4)
    from paper_1509_06865_amd.lqmg import herm_eigh
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    if kind == "rand":
        A = (X + X.conj().T) / 2
    else:
        Qm, _ = np.linalg.qr(X)
        lam = np.repeat(rng.standard_normal((n + 3) // 4), 4)[:n]
        A = (Qm * lam) @ Qm.conj().T
        A = (A + A.conj().T) / 2
    w, V = herm_eigh(A)
    ref = np.linalg.eigvalsh(A)
    scale = max(np.abs(ref).max(), 1.0)
    assert np.abs(w - ref).max() <= 1e-13 * scale
    assert np.abs(A @ V - V * w).max() <= 1e-13 * scale
    assert np.abs(V.conj().T @ V - np.eye(n)).max() <= 1e-13
