"""Plain FP64 CPU oracle for phase-field fracture with fixed-stress staggering.

TEST INFRASTRUCTURE ONLY.  This package exists to check the HIP path.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product path (``paper_2209_07969_amd``) never imports, links or calls it
and fails loudly when its HIP library is missing.

The oracle is written from the paper (Luo, "Fast staggered schemes for the
phase-field model of brittle fracture based on the fixed-stress concept"):

* ``constitutive`` - quadrature-point functions: the volumetric-deviatoric
  split (Section 2, energy split and stress equation), the spectral split
  (named in Section 2), the fixed-invariant predictor (Section 3.3, the
  half-step energy update; Section 3.5, the softening gate and the
  positive-increment rule).
* ``fem`` - Q1 geometry, shape functions and 2x2 Gauss quadrature.
* ``assembly`` - assembled sparse (CSR) residuals and Jacobians of the
  momentum balance and of the AT2 evolution equation (Section 3.2, weak
  forms; Section 3.4, augmented phase-field block).
* ``staggered`` - the standard scheme (Section 3.1) and the S1/S2/S3 schemes
  (Section 3.3-3.5), one load step at a time, with direct sparse solves; the
  literal readings of the trial solve (unfloored block, trial-only update).
* ``at1`` - AT1 with penalised irreversibility (Section 2, the evolution
  equation with the penalty; Section 3.2, F_d): residual, semismooth Newton
  matrix and solve.
* ``hex3d`` - the same model and staggered schemes on 3-D trilinear
  hexahedra (2x2x2 Gauss) with the full 3-D volumetric-deviatoric or
  spectral split.

Readings of passages that are silent or garbled are listed in the project's
design notes and repeated where they are used.
"""
from . import constitutive, fem, assembly, staggered, at1, hex3d  # noqa: F401
from .staggered import Oracle, StepStats  # noqa: F401
