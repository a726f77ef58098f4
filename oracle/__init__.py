"""Plain FP64 CPU oracle for the time-dependent SLDA (TDSLDA) step.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import anything from this package.
The product path (the HIP library and its Python binding) never imports,
calls or links it, and this package imports nothing from the product.

Everything here is written from the paper (W-SLDA Toolkit, arXiv 2602.08982)
in numpy / scipy, double precision, with no blocking, fusion or reordering
beyond what the paper's definitions and algorithms state:

  lattice      Sec. 3.1: periodic lattice, k-grid, spectral derivative,
               dense derivative matrices (Eqs. D1, D2).
  functional   Sec. 2.4-2.6: SLDA-type energy density, ASLDA constants,
               pairing field (Eq. Delta), regularisation (Eq. Creg), the
               A=1 simplification, energy terms (Sec. 3.2).
  bdg          Sec. 2.3: reduced 2x2 BdG operator (Eq. HpsiEpsi) applied
               spectrally and as a dense matrix; initial states.
  densities    Sec. 2.2-2.3: densities of the reduced problem, general
               (Eqs. na3D-jb3D) and spin-symmetric (Eqs. nab3D-jab3D).
  td           Sec. 3.3: shifted equation of motion (Eq. ABM-f), the
               AB3AM4 / AB4AM5 / AB5AM5 integrators (Alg. AB4AM5 and its
               analogues) and the Taylor start-up (Eq. Taylor-exp).
  q1d          Sec. 3.1 quasi-1D mode: plane waves in the two free
               directions, one 1D BdG problem per transverse momentum.
  uniform      Uniform-system solutions (continuum and lattice) used as
               pins and as the plane-wave starting point.
  static       Sec. 3.2 (Alg. MapK): the quasi-2D static self-consistent
               solve with linear and modified Broyden mixing.
  interp       Sec. 5.2: Fourier interpolation between lattices of a box.
  cnn          The warm-start network (forward, gradients, Adam).
  td.Friction  Sec. 5.2: quantum-friction (dissipative) mean fields.

Where the paper is silent or garbled, the reading taken is stated at the
function that takes it.
"""
