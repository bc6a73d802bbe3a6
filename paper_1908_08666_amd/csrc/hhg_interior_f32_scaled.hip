// Interior-row kernels instantiated for float, scaled method.
#include "hhg_interior.h"

namespace hhg {
template int launch_interior_v<float, METHOD_SCALED, false>(hhg_ctx *, const float *, const float *,
                                                 const float *, float *, hipStream_t);
template int launch_interior_v<float, METHOD_SCALED, true>(hhg_ctx *, const float *, const float *,
                                                const float *, float *, hipStream_t);
template int launch_interior_dot<float, METHOD_SCALED>(hhg_ctx *, const float *, const float *, float *, double *,
                                                  hipStream_t);
template int launch_interior_smooth<float, METHOD_SCALED>(hhg_ctx *, const float *, const float *, const float *,
                                                      const float *, float, float *, hipStream_t);
}  // namespace hhg
