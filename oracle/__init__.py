"""Plain FP64 CPU oracle for the preconditioned FAS smoother (test
infrastructure only).

Only the tests, the package's ``smoke()`` check and the benchmark's CPU
baseline leg may import this package.  The GPU library never calls it and
shares no code with it; the two meet only through the seeded inputs of
``fas_inputs``.

Layout: numpy arrays ``U[k, j + 2, i + 2]`` with two ghost layers on every
side of the ``nj x ni`` interior (k = rho, rho*u, rho*v, rho*E).  The
block Gauss-Seidel sweeps run in a small C file (``sgs.c``) because they
are inherently cell-by-cell; everything else is vectorised numpy that
follows the paper's formulas in the order they are written.

Modules
-------
geometry   face vectors, volumes, agglomerated levels, ghost-cell geometry
gas        ideal-gas relations, fluxes, the flux Jacobian and its splitting
bc         ghost-cell boundary conditions
residual   JST residual, viscous terms, Baldwin-Lomax, the f^c / f^v split
precond    flux-vector-split blocks, SGS preconditioner
smoother   additive W / preconditioned additive RK low-storage stages
fas        full approximation scheme cycle, transfers, norms, dual time
"""
