// Interior-row kernels instantiated for float, on-the-fly method.
#include "hhg_interior.h"

namespace hhg {
template int launch_interior_v<float, METHOD_ONTHEFLY, false>(hhg_ctx *, const float *, const float *,
                                                 const float *, float *, hipStream_t);
template int launch_interior_v<float, METHOD_ONTHEFLY, true>(hhg_ctx *, const float *, const float *,
                                                const float *, float *, hipStream_t);
template int launch_interior_dot<float, METHOD_ONTHEFLY>(hhg_ctx *, const float *, const float *, float *, double *,
                                                  hipStream_t);
template int launch_interior_smooth<float, METHOD_ONTHEFLY>(hhg_ctx *, const float *, const float *, const float *,
                                                      const float *, float, float *, hipStream_t);
}  // namespace hhg
