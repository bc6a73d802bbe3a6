// Interior-row kernels instantiated for double, on-the-fly method.
#include "hhg_interior.h"

namespace hhg {
template int launch_interior_v<double, METHOD_ONTHEFLY, false>(hhg_ctx *, const double *, const double *,
                                                 const double *, double *, hipStream_t);
template int launch_interior_v<double, METHOD_ONTHEFLY, true>(hhg_ctx *, const double *, const double *,
                                                const double *, double *, hipStream_t);
template int launch_interior_dot<double, METHOD_ONTHEFLY>(hhg_ctx *, const double *, const double *, double *, double *,
                                                  hipStream_t);
template int launch_interior_smooth<double, METHOD_ONTHEFLY>(hhg_ctx *, const double *, const double *, const double *,
                                                      const double *, double, double *, hipStream_t);
}  // namespace hhg
