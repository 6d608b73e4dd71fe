"""Plain FP64 CPU oracle for the DISCOS slit-channel particle-grid core.

TEST INFRASTRUCTURE ONLY.  This package is a slow, obviously correct restatement
of the paper's definitions (Ladiges et al., "Modeling electrokinetic flows with
the discrete ion stochastic continuum overdamped solvent algorithm",
arXiv:2204.14167).  Only the tests, the smoke check of the package and the
CPU-baseline leg of the benchmark may import it.  The GPU library never calls it,
and it shares no code with the GPU library.

Geometry: periodic in x and y, walls at z = 0 and z = Lz (the paper confines its
channel in y; every channel formula here reads the paper's y as z).

Modules
  peskin        4-point Peskin kernel (App. B, eq peskin1d / pkernel)
  rng           Philox4x32-10 counter-based generator and Box-Muller normals
  electrostatics  S^es with images, Poisson with wall BCs, E = -grad phi, J^es,
                  P3M near-field correction with images (Sec. II.B.1)
  shortrange    wall 9-3 potential and the LJ / WCA pair force (Sec. II.B.2)
  mobility      fit function, wall mobility, dry-diffusion drift (Sec. II.C, III.A)
  dynamics      the dry time step (Sec. II.D, stages 1, 2 and the dry part of 4)
  stokes        MAC Stokes with no-slip walls, S^hy, J^hy, stochastic stress (Sec. II.A)
  adjoint       energy and electro-osmotic flux functionals and their gradients
"""
