"""CPU FP64 oracle for the AM-AMG-preconditioned FGMRES solve of the Schwinger-model Wilson-Dirac system.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct NumPy/SciPy
implementation of what the GPU library computes.  Only the test suite, the package's
``smoke()`` check and the CPU-baseline leg of the benchmark may import it; the product
path never does.  It shares no code with the HIP library: the two meet only in the
seeded inputs of the ``synth`` module.

Modules (each function cites the passage of the paper it follows):

* ``dirac``      -- the Wilson-Dirac operator D (Schwinger Model subsection), sigma matrices,
                    boundary conditions, sigma3-hermiticity.
* ``wirebasket`` -- structured wirebaskets: vertex/edge/interior classes, owners, nodes
                    (SM-AMG for LQCD subsection, wirebasket figure).
* ``rng``        -- splitmix64 counter hash for the setup's random test vectors.
* ``amg``        -- local Schur-complement interpolation (block system, ideal presmoothing,
                    interpolation formula), normalisation, Galerkin coarse operator,
                    multicolour block Gauss-Seidel, dense coarsest solve, V-cycle
                    (two-level scheme algorithm, applied recursively).
* ``fgmres``     -- flexible GMRES(m) with classical Gram-Schmidt twice and Givens rotations.
* ``spectrum``   -- critical-mass estimate from the smallest real part of the spectrum.

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms, invariants and
brute-force dense solves.  Functions whose results have no such pin say so in their docstring.
"""
