"""Plain FP64 CPU oracle for adaptive spectral deferred correction (SDC).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` use it.  It
shares no code with the HIP library (no kernels, headers, helpers, tables or
constant generators); the only thing both sides consume is the seeded input
data produced by :mod:`workloads`, which holds none of the method's arithmetic.

Everything here is written for a reader to check against the paper by eye:
NumPy/SciPy in float64, no blocking, fusion or reordering beyond what the
paper's equations state.  Section/equation citations refer to Chegini,
Steinke, Weiser, "Efficient adaptivity for simulating cardiac
electrophysiology with spectral deferred correction methods" (arXiv
2311.07206).

Modules
-------
collocation  Radau-IIA nodes, integration matrix Q, LU-trick QI, explicit QE
             (Sec. 3.1, eq. "SDC Integration" and eq. (SDC)).
ionic        Aliev-Panfilov current and gating rate with derivatives (Sec. 5.1).
assembly     P1 lumped mass and stiffness on simplices (Sec. 2.2, eq. abstract
             monodomain).
pcg          Jacobi-preconditioned CG on a principal submatrix (Sec. 4.2).
sdc          IMEX SDC sweep with nested active-dof selection (eq. final-sdc,
             Sec. 4.2 index sets I_k).
collocation_newton  Dense Newton solve of the full collocation system (Sec. 3.1).
tlm          Tangent-linear model of the SDC step with frozen index sets.

Functions without an independent pin say "parity unpinned" in their docstring.
"""
