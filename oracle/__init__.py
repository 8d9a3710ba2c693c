"""CPU FP64 oracle for the periodic linear-elastic voxel cell problem.

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that
the GPU path is checked against.  Only the test-suite, the smoke check and
the benchmark's CPU-baseline leg may import it; the product path (the HIP
library and its Python binding) never imports, links or calls anything
here, and this package imports nothing from the product.

What it computes (plain definitions, written out slowly):
  * ``fem``      P1 finite elements on the Kuhn subdivision of each voxel
                 (pixel: 2 triangles), the linear-elastic energy density of
                 Sec. 2.2 (eq. LinearElastEnergy) with the Lame parameters of
                 Sec. 6.3, explicit sparse assembly of the periodic stiffness
                 K and the load vectors, direct sparse solve, effective
                 stiffness (energy and mean-stress forms), Hill-Mandel gap,
                 and the closed-form derivative of C* with respect to the
                 per-voxel Young's modulus.
  * ``matfree``  the same operator applied matrix-free with numpy (for grids
                 too large to assemble), the translation-invariant reference
                 operator's Fourier symbol obtained numerically as the DFT of
                 its impulse response (Sec. 3.2: constant stencil functions
                 make the reference matrix circulant), and a textbook
                 preconditioned conjugate-gradient solve.
  * ``hyper``    the compressible neo-Hookean cell problem (Sec. 2.2, eq.
                 NeoHookeanEnergy) on the same mesh: energy, first Piola
                 stress, its derivative, explicit tangent assembly and
                 Newton's method (Sec. 4, nonlinear problems) with direct
                 sparse solves and an Armijo line search.
  * ``surrogate`` the stencil functions of the assembled K (Sec. 3.2), their
                 B-spline interpolants from every M-th node (Sec. 3.3), the
                 symmetric kernel-preserving surrogate matrix (Sec. 3.4) and
                 its constrained direct solve.
  * ``strainproj`` the strain-based Fourier projection variant: CG on
                 compatible strain fields with the FE-gradient projection
                 B (B^T D0 B)^-1 B^T D, a cross-check of the PCG iteration.

Every function states the passage or the standard mathematics it follows.
"""
from . import fem, hyper, matfree, strainproj, surrogate  # noqa: F401
