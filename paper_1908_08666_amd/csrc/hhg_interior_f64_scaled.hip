// Interior-row kernels instantiated for double, scaled method.
#include "hhg_interior.h"

namespace hhg {
template int launch_interior_v<double, METHOD_SCALED, false>(hhg_ctx *, const double *, const double *,
                                                 const double *, double *, hipStream_t);
template int launch_interior_v<double, METHOD_SCALED, true>(hhg_ctx *, const double *, const double *,
                                                const double *, double *, hipStream_t);
template int launch_interior_dot<double, METHOD_SCALED>(hhg_ctx *, const double *, const double *, double *, double *,
                                                  hipStream_t);
template int launch_interior_smooth<double, METHOD_SCALED>(hhg_ctx *, const double *, const double *, const double *,
                                                      const double *, double, double *, hipStream_t);
}  // namespace hhg
