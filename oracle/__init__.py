"""CPU oracle for the PDHG SDP method -- TEST INFRASTRUCTURE ONLY.

Plain float64 NumPy with a full eigendecomposition every iteration.  Only
the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the GPU library never does, and the
two share no code (only the seeded input generators in ``instances``).

Parity status per function (pins live in tests/test_oracle_*.py):
  svec/smat, Operators.apply/adjoint   pinned (adjointness, dense brute force)
  Operators.norm                       pinned (closed forms, dense SVD)
  proj_psd, aproj_psd                  pinned (cone invariants, Eckart-Young,
                                       2x2 and diagonal closed forms)
  proj_box, dual_resolvent             pinned (scalar prox by direct minimisation)
  pdhg_step, solve                     pinned (closed-form optima of K_n, C_n,
                                       bipartite graphs; brute-force max-cut and
                                       bisection brackets; KKT at convergence)
  residuals eps_p, eps_d (Sec. 2.2)    pinned (hand-derived one- and two-step
                                       values on 1 x 1 equality / inequality rows)
  rank test of Alg. 2                  pinned (odd cycles: rank-2 optimum, the
                                       rank path must end 1 -> 2 -> 4)
  certificate                          pinned (vanishes at closed-form optima,
                                       positive at perturbed points)
  maxcut_bracket                       pinned (exact values on K_n at the closed-
                                       form optimum, rescaled and feasible points)
  brute_force_maxcut / _min_bisection  pinned (K_n and C_n closed forms)
  hyperplane_round, gw_expected_cut    pinned (rank-one bipartite optimum rounds
                                       to the bipartition; every rounding at most
                                       the brute-force max-cut; the empirical
                                       mean of many trials matches the arccos
                                       expectation, which is >= 0.878 x SDP)
"""
from .sdp import *  # noqa: F401,F403
from .sdp import (CONVERGED, MAX_ITERS, NUMERICAL, RANK_LIMIT, TIME_LIMIT, Certificate, Operators,  # noqa
                  SolveResult, aproj_psd, brute_force_maxcut, brute_force_min_bisection,
                  certificate, dense_sym_from_coo, dual_resolvent, eig_desc, gw_expected_cut,
                  hyperplane_round, maxcut_bracket,
                  pdhg_step, proj_box, proj_psd, smat, solve, svec, svec_index)
