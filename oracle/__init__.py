"""Plain, slow, FP64 CPU oracle for phi-function actions of Kronecker sums.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only the test-suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library
(no kernels, headers, helpers, tables or constant generators) and imports
nothing from the product package.

Modules
  phi_exact   -- definitions: dense Kronecker sum, the augmented-matrix
                 exponential (exact phi_k actions for tiny grids), scalar
                 phi_k, the eigendecomposition closed form for the Dirichlet
                 Laplacian, and the separable phi_0.
  quadrature  -- Gauss-Legendre and Clenshaw-Curtis rules on [0, 1].
  bounds      -- the a priori quadrature error bound (Thm 3.2) and the
                 parameter selection (Algorithms quaderr, quadnodes,
                 setup_quadrature), plus Corollary 3.3's closed forms.
  phiquad     -- the paper's algorithm itself (fixed-point and adaptive
                 quadrature with scaling and modified squaring), written in
                 the paper's order as a reference for sizes the exact
                 definitions cannot reach.
"""
