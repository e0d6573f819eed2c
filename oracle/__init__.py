"""Plain, slow FP64 CPU oracle for the explicit finite-volume step of the 5-moment (1D1V)
and 14-moment (3V) maximum-entropy systems with the interpolative closure
(Boccelli, Kaufmann, Magin & McDonald, arXiv 2401.15233).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The HIP
product path never calls it, and this package imports nothing from the product: the two
share no kernels, headers, helpers, tables or constants.  The only common code is the
seeded input generator ``paper_2401_15233_amd.inputs``, which holds none of the method's
arithmetic.

Everything is NumPy float64, vectorised over cells, written from the paper's equations in
its own notation (Sections 2.3-2.4, 3, 5, Appendices A and B).  Library primitives used as
steps: ``numpy.linalg.inv`` (the matrix inverses that appear in the closure), ``einsum``
(the paper's index contractions), ``sqrt``/``exp``/``power`` from libm.

Modules
  moments     -- primitive <-> conserved maps (left-hand sides of the moment equations)
  closure     -- sigma mapping, sigma limiting and the interpolative closure (5 and 14 moments)
  wavespeeds  -- Baradaran 5-moment and the paper's approximate 14-moment wave speeds
  fluxes      -- physical fluxes, BGK sources, local collision time, HLL and Rusanov
  scheme      -- MUSCL with the common limiter, ghost cells, residual, CFL dt, integrators
  eigen       -- flux-Jacobian eigenvalues of the closed systems (diagnostic of the wave-speed fits)
"""

from . import moments, closure, wavespeeds, fluxes, scheme, eigen  # noqa: F401
