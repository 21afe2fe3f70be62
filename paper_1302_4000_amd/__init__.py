"""MI355X (gfx950) all-versus-all cRMSD.

The computation runs in ``libclusco.so`` (hand-written HIP kernels behind the
C ABI of ``include/clusco.h``); this package is its thin Python binding.
Importing the package does not load the library: the first call does, and
raises if it is not built.
"""
from .binding import (ClucsoError, PRECISION, crmsd_matrix, fixup_count, set_tolerance,  # noqa: F401
                      workspace_size)

__all__ = ["ClucsoError", "PRECISION", "crmsd_matrix", "fixup_count", "set_tolerance",
           "workspace_size"]
