"""FP64 CPU oracle for the nodal DG shallow-water step.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy/SciPy implementation of what the GPU path computes, written from the
paper (Gandham, Medina & Warburton, "GPU accelerated discontinuous Galerkin
methods for shallow water equations"):

* ``refelem`` - reference triangle: Warp & Blend nodes, orthonormal basis,
  Dr, Ds, mass matrix, LIFT, cell-mean weights, P1 tools (Section 3).
* ``mesh``    - connectivity, affine geometry, CFL time step and multi-rate
  levels (Section 4, Eq. 4.1), TVB neighbour stencil (Section 5.3).
* ``swe``     - right-hand side with the well-balanced Lax-Friedrichs flux
  (Section 2, Eq. 2.3; Section 3, Eq. 3.2-3.3; Section 5.1, Eq. 5.1-5.2),
  positivity limiter (Algorithm 5.2), positivity-modified TVB limiter
  (Section 5.3, Eq. 5.3), Adams-Bashforth 3 and multi-rate AB3 with limiting
  (Algorithms 4.1 and 5.1), diagnostics.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run this package.  It shares no code with the HIP
library: the only common module is ``workloads`` (seeded inputs, no method
arithmetic).
"""
from . import refelem, mesh, swe  # noqa: F401
from .refelem import RefElement, reference_element  # noqa: F401
from .mesh import Mesh, build_mesh  # noqa: F401
from .swe import Params, Solver  # noqa: F401
