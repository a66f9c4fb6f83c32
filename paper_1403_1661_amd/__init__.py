"""MI355X (gfx950) nodal DG solver for the 2D shallow water equations.

The compute path lives in the HIP library ``libdgswe.so`` behind the C ABI of
``include/dgswe.h``; ``dgswe`` is its ctypes binding.  Importing this package
does not load the library; creating a ``Solver`` does, and fails loudly when
it has not been built.
"""
from .dgswe import DGError, Solver, default_params, load_library  # noqa: F401
