"""CPU FP64 oracle for the shifted-Green-function periodic Dirichlet solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy/SciPy implementation of what the GPU library computes.  Only the test
suite, the smoke check of the entry module and the CPU-baseline leg of the
benchmark may import it; the product path (the HIP library and its Python
binding) never does, and shares no code, table or constant with it.

Modules (each function cites the passage of Bruno & Maas, "Shifted equivalent
sources and FFT acceleration for periodic scattering problems, including Wood
anomalies", that it follows):
  surface   - the profile f and its derivatives at the quadrature nodes
  greens    - windows, multipolar Green function, lattice sums, spectral
              series, Martensen-Kussmaul split and log-quadrature weights
  dense     - the dense direct Nystrom operator (1/2 I + D^dx) and the RHS
  rayleigh  - Rayleigh wavenumbers, completion set, Rayleigh coefficients,
              efficiencies and energy balance
  gmres     - unrestarted GMRES with Givens rotations
  accel     - the accelerated forward map (equivalent sources, FFT
              convolution, local corrections, plane-wave interpolation)

Readings of passages that are garbled or silent are listed in the design
notes and repeated next to the code that takes them.
"""
from . import surface, greens, dense, rayleigh, gmres  # noqa: F401
