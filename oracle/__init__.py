"""Plain FP64 CPU oracle for one time step of the second-order convex-splitting
scheme for Cahn-Hilliard-Hele-Shaw (Chen, Feng, Liu, Wang, Wise; arXiv 1611.02967).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library (different language, independently written stencils); the only
thing both sides share is the seeded input module ``workloads``.

Modules
-------
grid     discrete operators, inner products and norms of Appendix A
scheme   the scheme (2.4)-(2.7) as a nonlinear system N(u) = f, energies (2.8)-(2.9)
newton   the plain definition of the per-step result: Newton on the full system,
         Jacobian assembled cell by cell in index form, direct sparse/dense solve
fas      red-black full-approximation-scheme V-cycles (the solver of Section 5,
         whose details the paper omits; the reading used is stated in fas.py)

Every function cites the passage of the paper it follows.  No function here is
"parity unpinned": each is checked in ``tests/test_oracle_*.py`` against closed
forms, identities proved in the paper, or brute force.
"""
