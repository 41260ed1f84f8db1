"""Plain CPU FP64 oracle for the DG Shifted Boundary Method multigrid solver.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct reference
that the HIP path is checked against.  Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product library never
does, and it imports nothing from the product package.

Modules
-------
basis     -- Gauss-Lobatto-Legendre Lagrange basis and Gauss quadrature on [0,1]
geometry  -- level sets and closest-point projections (Sec. 4.2)
dg        -- levels, active cells, surrogate faces, shifts, the DG-SBM matrix
             and right-hand side by direct quadrature (Sec. 2.1-2.2)
mg        -- transfers, cell-wise red-black SSOR and the V-cycle (Sec. 3)
krylov    -- restarted flexible GMRES with modified Gram-Schmidt (Sec. 3)
mlp       -- reference forward/backward of the learned boundary-cell smoother
             correction (not part of the paper; see that module)
"""
