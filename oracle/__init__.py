"""Plain, slow, obviously correct CPU FP64 reference for the FETI solvers of
Medřický, Doškář, Pultarová and Zeman, "Comparison of FETI-based domain
decomposition methods for topology optimization problems" (arXiv 2111.11728).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link
or execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it. It shares no code with the
HIP path; both read their inputs from ``workloads``.

Modules:

* ``fem``       - SIMP law (Eq. 1), element stiffness, global assembly and direct
                  solve (Eq. 2), compliance and its gradient.
* ``topology``  - the partition into subdomains, the TFETI constraint matrix with
                  Dirichlet rows (Sec. 2.1, Eq. 4), the FETI-DP corner / remainder
                  split (Sec. 2.2, Eqs. 8-10), rigid-body modes, and the scaling
                  weights (Sec. 3.1, Eqs. 14-15).
* ``feti``      - the dual operators of TFETI (Sec. 2.1, Eq. 7) and FETI-DP
                  (Sec. 2.2, Eq. 12 with u_c condensed), the preconditioner
                  (Sec. 3.1, Eq. 13), the projector, recovery of u.
* ``krylov``    - projected PCG, full orthogonalisation (Sec. 3.2) and the
                  rank-revealing simultaneous FETI iteration (Sec. 3.3, Algorithm 1).

Parity status: every function is pinned by ``tests/test_oracle_*.py`` against
closed forms, the global direct solve, invariants of the method or brute force;
the rank-revealing decisions of Algorithm 1 are pinned only by the threshold
rule stated in ``krylov.pivoted_cholesky`` (the paper gives no tolerance), and
iteration counts against the paper are parity unpinned (its convergence plots
are not available as numbers).
"""
