"""Plain, slow FP64 CPU oracle of the local p-multigrid vertex-patch smoother method.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import anything from here; the product path never
does.  It shares no code with the HIP library: every quantity is recomputed from its
definition with NumPy/SciPy, with assembled sparse matrices, dense patch matrices and
direct solves, and without sum factorization, coloring tricks or blocking.

Modules (each function cites the passage of the paper it follows):
  basis     -- Gauss-Legendre rules, Gauss-Lobatto nodes, 1D Lagrange basis
  mesh      -- structured hex/quad meshes, numbering and patch index sets by brute force
  assembly  -- element matrices by brute-force quadrature, global sparse operators
  transfer  -- h-embedding (mesh levels) and p-embedding (degree levels)
  smoother  -- local p-multigrid (Alg. 2 / Alg. 3) and the multiplicative patch smoother (Alg. 1)
  solver    -- h-multigrid V-cycle and the outer flexible CG

Pinned: every function is checked in tests/test_oracle_*.py against closed forms,
invariants, brute force or the paper's printed values.
"""
