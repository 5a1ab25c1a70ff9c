"""FP64 CPU oracle for the FC-SDNN hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call,
link or execute anything under this directory; only the tests, the smoke
check and the benchmark's CPU-baseline leg use it.  It shares no code,
header, table or constant generator with the HIP path; the only module both
sides use is the seeded input generator ``synth`` (geometry, states, random
weights), which contains none of the method's arithmetic.

Everything here is a plain, slow, readable FP64 transcription of the paper's
definitions (Bruno & Leibovici, "General-domain FC-based shock-dynamics
solver I"), vectorised over lines with numpy.  Each function cites the
section or equation it follows.  Where the paper leaves something open, the
reading taken is stated in the docstring.

Modules
  fcgram   FC-Gram continuation matrices and the FC derivative (Sec. 2.2)
  euler    fluxes, curvilinear right-hand side, viscous term (Secs. 2.1, 2.3, 3.3)
  rk       SSPRK(5,4) time stepping and the CFL step size (Sec. 4.1)
  av       proxy variable, network classifier, preliminary viscosity and the
           smoothing-blending operator (Secs. 5.1, 5.2)
  filter   spectral filter of FC expansions and the per-step state filter
           (Sec. 4.3.1)
  smear    localized discontinuity-smearing of the initial data (Sec. 4.3.2)
  interp   inter-patch interpolation of fringe values (Sec. 3.4.1)
  wall     no-slip adiabatic walls through a Neumann FC boundary value
  solver   multi-patch time stepping with fringe exchange and boundary
           overwrite (Secs. 3.4, 4.2, Algorithm 1)
  adjoint  hand-written discrete adjoints (reverse mode) of all of the above
"""
