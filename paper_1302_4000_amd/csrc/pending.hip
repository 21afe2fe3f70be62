// Entry points whose kernels are not built yet: they validate nothing and
// report CLUSCO_ERR_UNSUPPORTED so that the exported symbol set matches the
// header.
#include "internal.h"

extern "C" {

size_t clusco_crmsd_batched_workspace_size(clusco_handle, int32_t, const int64_t *,
                                           const int64_t *, clusco_precision) { return 0; }
clusco_status clusco_crmsd_batched(clusco_handle, int32_t, const int64_t *, const int64_t *,
                                   const int64_t *, const int64_t *, const float *,
                                   clusco_precision, float *, void *, size_t, void *)
{ return CLUSCO_ERR_UNSUPPORTED; }
size_t clusco_crmsd_cross_workspace_size(clusco_handle, int64_t, int64_t, int64_t,
                                         clusco_precision) { return 0; }
clusco_status clusco_crmsd_cross(clusco_handle, const float *, int64_t, const float *, int64_t,
                                 int64_t, clusco_precision, float *, void *, size_t, void *)
{ return CLUSCO_ERR_UNSUPPORTED; }
size_t clusco_crmsd_backward_workspace_size(clusco_handle, int64_t, int64_t, clusco_precision)
{ return 0; }
clusco_status clusco_crmsd_backward(clusco_handle, const float *, int64_t, int64_t, const float *,
                                    const float *, clusco_precision, float *, void *, size_t,
                                    void *)
{ return CLUSCO_ERR_UNSUPPORTED; }
size_t clusco_crmsd_cross_backward_workspace_size(clusco_handle, int64_t, int64_t, int64_t,
                                                  clusco_precision) { return 0; }
clusco_status clusco_crmsd_cross_backward(clusco_handle, const float *, int64_t, const float *,
                                          int64_t, int64_t, const float *, const float *,
                                          clusco_precision, float *, float *, void *, size_t,
                                          void *)
{ return CLUSCO_ERR_UNSUPPORTED; }

} // extern "C"
