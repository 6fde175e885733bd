// Entry points whose implementation is not built yet: they validate nothing and report
// LS_ERR_UNSUPPORTED so a caller learns it explicitly instead of getting silent results.
#include "internal.h"

extern "C" {
ls_status ls_solve_gmres(ls_handle, const double *, double *, int32_t, int64_t, const ls_solve_opts *,
                         ls_solve_info *, hipStream_t) {
  return LS_ERR_UNSUPPORTED;
}
ls_status ls_grad_contrast(ls_handle, const double *, const double *, const double *, int32_t, int64_t, double *,
                           hipStream_t) {
  return LS_ERR_UNSUPPORTED;
}
}
