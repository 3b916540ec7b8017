"""MgNet-preconditioned flexible GMRES for the steady discrete-ordinates RTE on
MI355X (gfx950).  The solver lives in librte.so (HIP); this package is its
Python binding.  Importing it does not touch the GPU; the first call loads
the library and fails loudly if it has not been built."""
from ._lib import RteError, lib  # noqa: F401
from .api import Atfps, Model, Operator, Server, prof_enable, prof_query, prof_reset  # noqa: F401
