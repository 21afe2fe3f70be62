"""MI355X (gfx950) all-versus-all cRMSD, dRMSD and contact map overlap.

The computation runs in ``libclusco.so`` (hand-written HIP kernels behind the
C ABI of ``include/clusco.h``); this package is its thin Python binding.
Importing the package does not load the library: the first call does, and
raises if it is not built.
"""
from .autograd import CRMSDCross, CRMSDMatrix, crmsd_cross_ad, crmsd_matrix_ad  # noqa: F401
from .binding import (Batch, ClucsoError, PRECISION, batched_workspace_size,  # noqa: F401
                      crmsd_backward, crmsd_batched, crmsd_cross, crmsd_cross_backward,
                      cmo_matrix, cmo_workspace_size, crmsd_matrix, crmsd_threshold,
                      drmsd_matrix, drmsd_workspace_size,
                      fixup_count, force_config, get_config, kmedoids, load_tuning,
                      set_tolerance, workspace_size)

__all__ = ["Batch", "CRMSDCross", "CRMSDMatrix", "ClucsoError", "PRECISION",
           "batched_workspace_size", "crmsd_backward", "crmsd_batched", "crmsd_cross",
           "crmsd_cross_ad", "crmsd_cross_backward", "crmsd_matrix", "crmsd_matrix_ad",
           "crmsd_threshold", "drmsd_matrix", "drmsd_workspace_size", "kmedoids",
           "cmo_matrix", "cmo_workspace_size",
           "fixup_count", "force_config", "get_config", "load_tuning", "set_tolerance",
           "workspace_size"]
