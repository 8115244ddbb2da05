"""CPU oracle for the RQI + aggregation-multigrid low-mode eigensolver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow FP64 implementation of
what the HIP library computes, written from the paper (Bali et al., "(Approximate)
Low-Mode Averaging with a new Multigrid Eigensolver", Lattice 2015, sec. 2 and
Alg. 1).  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it.  The product path never calls it, and it
shares no code with the HIP library: the only common inputs come from the
``lqsynth`` generators.

Modules
  dirac   lattice geometry, gamma basis, Wilson-Dirac D and Q = gamma5 D (sec. 2)
  clover  the clover term of the clover-improved operator (optional, c_sw != 0)
  krylov  GMRES and flexible GMRES with x0 = 0 (sec. 2 and 2.2)
  mg      aggregation, gamma5-split interpolation P, Galerkin Q_c = P^dag Q P,
          SAP and GMRES smoothers, the two-grid cycle E_2g, adaptive setup
  rqi     Rayleigh quotient iteration with multigrid (Alg. 1), Rayleigh-Ritz
  lcnn    gauge-equivariant network proposing test vectors and its training loss
          (not in the paper; the reference for an optional learned setup)
  certify residual and Kato-Temple bounds, deflated search for missed modes
  lma     approximate low-mode averaging (sec. 3): low-mode parts, oblique
          projector, stochastic high part

All inner products use numpy's pairwise summation (``np.sum`` over a
contiguous array), never a running sum.

Parity status: ``mg.setup`` has no unique result (random starts, a heuristic);
it is checked through invariants only ("parity unpinned" for the vectors
themselves).  Everything else is pinned by the tests in ``tests/test_oracle_*``.
"""
