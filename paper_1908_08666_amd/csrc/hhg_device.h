// Device helpers shared by the operator kernels.
#pragma once

#include "hhg_ctx.h"

namespace hhg {


template <typename T>
struct Node4 {
  T x0, x1, x2, k;
};
// LDS records: (x0, x1) and (x2, k) in two arrays, so that consecutive lanes
// read consecutive 2*sizeof(T) records without bank conflicts.
template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T a, b;
};

__device__ __forceinline__ int tri_root_dev(int p) {
  int s = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
  if ((s + 1) * (s + 2) / 2 <= p) ++s;
  if (s * (s + 1) / 2 > p) --s;
  return s;
}

// barycentric zero set of node (i, j, k) in a macro with n intervals
__device__ __forceinline__ int zero_set(int i, int j, int k, int n) {
  return ((n - i - j - k) == 0) | ((i == 0) << 1) | ((j == 0) << 2) | ((k == 0) << 3);
}

constexpr int METHOD_SCALED = 0;
constexpr int METHOD_ONTHEFLY = 1;

template <typename T>
__device__ __forceinline__ void sym_mv_acc(const T *S, T z0, T z1, T z2, T &y0, T &y1, T &y2) {
  // S = xx yy zz xy xz yz
  y0 = fma(S[0], z0, fma(S[3], z1, fma(S[4], z2, y0)));
  y1 = fma(S[3], z0, fma(S[1], z1, fma(S[5], z2, y1)));
  y2 = fma(S[4], z0, fma(S[5], z1, fma(S[2], z2, y2)));
}

template <typename T>
__device__ __forceinline__ void cross_acc(T w0, T w1, T w2, T d0, T d1, T d2, T &y0, T &y1, T &y2) {
  y0 = fma(w1, d2, fma(-w2, d1, y0));
  y1 = fma(w2, d0, fma(-w0, d2, y1));
  y2 = fma(w0, d1, fma(-w1, d0, y2));
}


// device copies of the per-macro constant tables for element type T
template <typename T>
const StencilConst<T> *sc_ptr(hhg_ctx *h);
template <>
inline const StencilConst<double> *sc_ptr<double>(hhg_ctx *h) { return h->d_sc64; }
template <>
inline const StencilConst<float> *sc_ptr<float>(hhg_ctx *h) { return h->d_sc32; }
template <typename T>
const ElemConst<T> *ec_ptr(hhg_ctx *h);
template <>
inline const ElemConst<double> *ec_ptr<double>(hhg_ctx *h) { return h->d_ec64; }
template <>
inline const ElemConst<float> *ec_ptr<float>(hhg_ctx *h) { return h->d_ec32; }

// Interior-row launch for element type T and method; defined (and
// explicitly instantiated) in one translation unit per (T, METHOD).
template <typename T, int METHOD, bool RESID>
int launch_interior_v(hhg_ctx *h, const T *x, const T *k, const T *f, T *y, hipStream_t st);
template <typename T, int METHOD>
int launch_interior_dot(hhg_ctx *h, const T *x, const T *k, T *y, double *part, hipStream_t st);
template <typename T, int METHOD>
int launch_interior_smooth(hhg_ctx *h, const T *x, const T *k, const T *f, const T *P, T omega,
                           T *xo, hipStream_t st);

}  // namespace hhg
