// Krylov solvers on top of the stencil-scaling operators.
//
//   CG_F64  preconditioned conjugate gradients in FP64.
//   IR_F32  iterative refinement: FP64 residual, norm and update; inner
//           preconditioned CG with FP32 vectors, coefficient and applies and
//           FP64-accumulated inner products.
//   FCG_F64 flexible CG in FP64 (Polak-Ribiere beta; equal to CG_F64 for a
//           fixed symmetric positive definite preconditioner).
// Preconditioners: inverse 3x3 diagonal blocks of the assembled operator
// (block Jacobi), or those blocks reshaped by a learned network.  All scalars of the iteration (alpha, beta, rho) stay on the
// device; the host reads the residual history every `check_every`
// iterations, and a block of iterations is captured once in a HIP graph and
// replayed.  Inner products run over the unknowns only: owner copies of
// non-Dirichlet nodes.  Reductions use a fixed grid and tree order, so the
// results are bitwise reproducible.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "hhg_ctx.h"

namespace hhg {

int apply_internal(hhg_ctx *h, int prec, int method, const void *f, const void *x, const void *k,
                   void *y, hipStream_t st);
int apply_dot_internal(hhg_ctx *h, int prec, int method, const void *x, const void *k, void *y,
                       double *part, hipStream_t st);
int64_t dot_parts(hhg_ctx *h);
int learned_precond(hhg_ctx *h, const double *k, double *P, uint16_t *feat, float *mout,
                    hipStream_t st);

namespace {

constexpr int RED_GRID = 512;       // blocks of every reduction kernel
constexpr int RED_TPB = 256;
constexpr int MAX_CHECK = 64;       // iterations per captured block

struct CGState {
  double rho;      // (r, z)
  double pq;       // (p, q)
  double rr;       // (r, r)
  double alpha;
  double beta;
  int32_t bad;     // breakdown seen
  int32_t bad_it;  // iteration of the current block in which it was first seen
  double hist[MAX_CHECK];  // (r, r) after each iteration of the current block
};

__device__ __forceinline__ bool unknown(const uint8_t *fl, int64_t s) { return (fl[s] & 3) == 2; }

__device__ __forceinline__ double block_sum(double v, double *sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += sh[q];
  __syncthreads();
  return t;
}

// partial sums of (a, b) and (c, d) over the unknowns
template <typename T>
__global__ __launch_bounds__(RED_TPB) void k_dot2(const T *__restrict__ a, const T *__restrict__ b,
                                                  const T *__restrict__ c, const T *__restrict__ d,
                                                  const uint8_t *__restrict__ fl, int64_t N,
                                                  double *__restrict__ part) {
  __shared__ double sh[RED_TPB / 64];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N;
       s += (int64_t)gridDim.x * blockDim.x) {
    if (!unknown(fl, s)) continue;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      s0 += (double)a[q * N + s] * (double)b[q * N + s];
      if (c) s1 += (double)c[q * N + s] * (double)d[q * N + s];
    }
  }
  s0 = block_sum(s0, sh);
  s1 = block_sum(s1, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = s0;
    part[3 * blockIdx.x + 1] = s1;
    part[3 * blockIdx.x + 2] = 0.0;
  }
}

// r -= alpha q, z = P r; partial sums of (r, z) and (r, r), and for the
// flexible variant (z, q).  The x update waits for k_pupdate, which reads p
// anyway, so x and p stream through HBM once per iteration.
template <typename T, bool FLEX>
__global__ __launch_bounds__(RED_TPB) void k_update(T *__restrict__ r, const T *__restrict__ q,
                                                    const T *__restrict__ P, T *__restrict__ z,
                                                    const uint8_t *__restrict__ fl, int64_t N,
                                                    const CGState *__restrict__ st,
                                                    double *__restrict__ part) {
  __shared__ double sh[RED_TPB / 64];
  const T alpha = (T)st->alpha;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N;
       s += (int64_t)gridDim.x * blockDim.x) {
    T rv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      rv[c] = fma(-alpha, q[c * N + s], r[c * N + s]);
      r[c * N + s] = rv[c];
    }
    const T Pxx = P[s], Pyy = P[N + s], Pzz = P[2 * N + s];
    const T Pxy = P[3 * N + s], Pxz = P[4 * N + s], Pyz = P[5 * N + s];
    const T z0 = Pxx * rv[0] + Pxy * rv[1] + Pxz * rv[2];
    const T z1 = Pxy * rv[0] + Pyy * rv[1] + Pyz * rv[2];
    const T z2 = Pxz * rv[0] + Pyz * rv[1] + Pzz * rv[2];
    z[s] = z0;
    z[N + s] = z1;
    z[2 * N + s] = z2;
    if (unknown(fl, s)) {
      s0 += (double)rv[0] * z0 + (double)rv[1] * z1 + (double)rv[2] * z2;
      s1 += (double)rv[0] * rv[0] + (double)rv[1] * rv[1] + (double)rv[2] * rv[2];
      if (FLEX)
        s2 += (double)z0 * q[s] + (double)z1 * q[N + s] + (double)z2 * q[2 * N + s];
    }
  }
  s0 = block_sum(s0, sh);
  s1 = block_sum(s1, sh);
  if (FLEX) s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = s0;
    part[3 * blockIdx.x + 1] = s1;
    part[3 * blockIdx.x + 2] = s2;
  }
}

// z = P r (also the start of an iteration), partial sums of (r, z), (r, r)
template <typename T>
__global__ __launch_bounds__(RED_TPB) void k_precond(const T *__restrict__ r, const T *__restrict__ P,
                                                     T *__restrict__ z, T *__restrict__ p,
                                                     const uint8_t *__restrict__ fl, int64_t N,
                                                     double *__restrict__ part) {
  __shared__ double sh[RED_TPB / 64];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N;
       s += (int64_t)gridDim.x * blockDim.x) {
    const T r0 = r[s], r1 = r[N + s], r2 = r[2 * N + s];
    const T Pxx = P[s], Pyy = P[N + s], Pzz = P[2 * N + s];
    const T Pxy = P[3 * N + s], Pxz = P[4 * N + s], Pyz = P[5 * N + s];
    const T z0 = Pxx * r0 + Pxy * r1 + Pxz * r2;
    const T z1 = Pxy * r0 + Pyy * r1 + Pyz * r2;
    const T z2 = Pxz * r0 + Pyz * r1 + Pzz * r2;
    z[s] = z0;
    z[N + s] = z1;
    z[2 * N + s] = z2;
    p[s] = z0;
    p[N + s] = z1;
    p[2 * N + s] = z2;
    if (unknown(fl, s)) {
      s0 += (double)r0 * z0 + (double)r1 * z1 + (double)r2 * z2;
      s1 += (double)r0 * r0 + (double)r1 * r1 + (double)r2 * r2;
    }
  }
  s0 = block_sum(s0, sh);
  s1 = block_sum(s1, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = s0;
    part[3 * blockIdx.x + 1] = s1;
    part[3 * blockIdx.x + 2] = 0.0;
  }
}

// x += alpha p (the iteration's step), then p = z + beta p
template <typename T>
__global__ __launch_bounds__(256) void k_pupdate(T *__restrict__ x, T *__restrict__ p,
                                                 const T *__restrict__ z, int64_t n3,
                                                 const CGState *__restrict__ st) {
  const T alpha = (T)st->alpha, beta = (T)st->beta;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n3;
       s += (int64_t)gridDim.x * blockDim.x) {
    const T pv = p[s];
    x[s] = fma(alpha, pv, x[s]);
    p[s] = fma(beta, pv, z[s]);
  }
}

enum { FIN_INIT = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_NORM = 3, FIN_BETA_FLEX = 4 };

// Deterministic final reduction of the block partials and the scalar step.
__global__ __launch_bounds__(RED_TPB) void k_finalize(const double *__restrict__ part, int nblk,
                                                      CGState *__restrict__ st, int mode, int hidx) {
  __shared__ double sh[RED_TPB / 64];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    s0 += part[3 * b];
    s1 += part[3 * b + 1];
    s2 += part[3 * b + 2];
  }
  s0 = block_sum(s0, sh);
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x != 0) return;
  if (mode == FIN_INIT) {
    st->rho = s0;
    st->rr = s1;
    st->bad = (!isfinite(s0) || !isfinite(s1) || s0 < 0.0) ? 1 : 0;
    st->bad_it = 0;
  } else if (mode == FIN_ALPHA) {
    st->pq = s0;
    if (!(s0 > 0.0) || !isfinite(s0)) {
      if (!st->bad) st->bad_it = hidx;
      st->bad = 1;
      st->alpha = 0.0;
    } else {
      st->alpha = st->rho / s0;
    }
  } else if (mode == FIN_BETA || mode == FIN_BETA_FLEX) {
    // Fletcher-Reeves (r+, z+)/(r, z), or Polak-Ribiere (z+, r+ - r)/(r, z)
    // with r+ - r = -alpha q
    const double num = mode == FIN_BETA ? s0 : -st->alpha * s2;
    st->beta = st->rho != 0.0 ? num / st->rho : 0.0;
    st->rho = s0;
    st->rr = s1;
    st->hist[hidx] = s1;
    if (!isfinite(s0) || !isfinite(s1)) {
      if (!st->bad) st->bad_it = hidx;
      st->bad = 1;
    }
  } else {
    st->rr = s0;
  }
}

__global__ void k_cast64to32(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    b[s] = (float)a[s];
}

__global__ void k_add32to64(double *__restrict__ x, const float *__restrict__ e, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    x[s] += (double)e[s];
}

template <typename T>
__global__ void k_fill(T *__restrict__ a, T v, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    a[s] = v;
}

// zero the Dirichlet entries of a vector field
template <typename T>
__global__ void k_zero_dirichlet(T *__restrict__ x, const uint8_t *__restrict__ fl, int64_t N) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N;
       s += (int64_t)gridDim.x * blockDim.x)
    if (fl[s] & 1) {
      x[s] = T(0);
      x[N + s] = T(0);
      x[2 * N + s] = T(0);
    }
}

// ----------------------------------------------------- diagonal blocks
__device__ __forceinline__ int plane_base_d(int n, int k) {
  const int a = n + 1, b = n + 1 - k;
  return a * (a + 1) * (a + 2) / 6 - b * (b + 1) * (b + 2) / 6;
}
__device__ __forceinline__ int tri_root_d(int p) {
  int s = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
  while ((s + 1) * (s + 2) / 2 <= p) ++s;
  while (s * (s + 1) / 2 > p) --s;
  return s;
}
__device__ __forceinline__ int zero_set_d(int i, int j, int k, int n) {
  return ((n - i - j - k) == 0) | ((i == 0) << 1) | ((j == 0) << 2) | ((k == 0) << 3);
}

// 3x3 diagonal block of every slot's row from its macro (xx yy zz xy xz yz):
// macro-interior rows of the scaled operator: -sum_d (khat_d Shat_d + A0_d)
// (the correction blocks sum to zero, Lemma); all other rows: the nodal
// diagonal sum_t (B0 + kbar^t B1)_{00} over the macro's elements at the node.
__global__ __launch_bounds__(256) void k_diag(const MacroInfo *__restrict__ minfo,
                                              const StencilConst<double> *__restrict__ scs,
                                              const ElemConst<double> *__restrict__ ecs,
                                              const double *__restrict__ kc, int method,
                                              int zerosum, int64_t N, double *__restrict__ D) {
  const int m = blockIdx.y;
  const MacroInfo mi = minfo[m];
  const int n = mi.n;
  const int ls = blockIdx.x * blockDim.x + threadIdx.x;
  if (ls >= (int)macro_nodes(n)) return;
  int lo = 0, hi = n;  // plane: largest k with plane_base(k) <= ls
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (plane_base_d(n, mid) <= ls) lo = mid; else hi = mid - 1;
  }
  const int k = lo;
  const int pos = ls - plane_base_d(n, k);
  const int s = tri_root_d(pos);
  const int i = pos - s * (s + 1) / 2, j = s - i;
  const int64_t slot = mi.off + ls;
  double d[6] = {0, 0, 0, 0, 0, 0};
  const int z = zero_set_d(i, j, k, n);
  const double *K = kc + mi.off;
  auto kat = [&](int dd, bool &ok) {
    const int a = i + DIR_I[dd], b = j + DIR_J[dd], c = k + DIR_K[dd];
    ok = a >= 0 && b >= 0 && c >= 0 && a + b + c <= n;
    return ok ? K[plane_base_d(n, c) + (a + b) * (a + b + 1) / 2 + a] : 0.0;
  };
  if (!((mi.dmask >> z) & 1u)) {
    double nk[NDIR];
    bool in[NDIR];
    for (int dd = 0; dd < NDIR; ++dd) nk[dd] = kat(dd, in[dd]);
    const double kc0 = K[ls];
    if (z != 0 && zerosum && method == HHG_METHOD_SCALED) {
      // zero-sum centre of an interface row: minus this macro's part of the
      // row's other blocks, nodal towards macro-boundary neighbours and
      // scaled towards macro-interior ones (the correction blocks are
      // antisymmetric and drop out of the symmetric part kept here; the
      // copies' partial centres sum to a symmetric block)
      bool onb[NDIR];
      for (int dd = 0; dd < NDIR; ++dd)
        onb[dd] = in[dd] && zero_set_d(i + DIR_I[dd], j + DIR_J[dd], k + DIR_K[dd], n) != 0;
      const ElemConst<double> &ec = ecs[m];
      const int ix[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
      for (int t = 0; t < NTET; ++t) {
        const int v1 = TET_V[t][0], v2 = TET_V[t][1], v3 = TET_V[t][2];
        if (!(in[v1] && in[v2] && in[v3])) continue;
        const double kb = 0.25 * (kc0 + nk[v1] + nk[v2] + nk[v3]);
        for (int c = 1; c < 4; ++c) {
          if (!onb[TET_V[t][c - 1]]) continue;
          const double *B1 = ec.b1[t][c];
          const double *B0 = ec.b0[t][c];
          for (int q = 0; q < 6; ++q) {
            const int a = 3 * ix[q][0] + ix[q][1], b = 3 * ix[q][1] + ix[q][0];
            d[q] -= 0.5 * ((B0[a] + kb * B1[a]) + (B0[b] + kb * B1[b]));
          }
        }
      }
      const StencilConst<double> &sc = scs[m];
      for (int dd = 0; dd < NDIR; ++dd) {
        if (!in[dd] || onb[dd]) continue;
        const int np = DIR_NT[dd] == 6 ? 3 : 2;
        double ring = 0.0;
        for (int q = 0; q < np; ++q) ring += nk[RING_V[dd][q]] + nk[RING_VM[dd][q]];
        const double wr = DIR_NT[dd] == 6 ? sc.w_ring6 : sc.w_ring4;
        const double kh = sc.w_end * (kc0 + nk[dd]) + wr * ring;
        for (int q = 0; q < 6; ++q) d[q] -= kh * sc.pr[dd >> 1].shat[q] + sc.pr[dd >> 1].a0[q];
      }
    } else if (z == 0 && method == HHG_METHOD_SCALED) {
      const StencilConst<double> &sc = scs[m];
      for (int dd = 0; dd < NDIR; ++dd) {
        const int np = DIR_NT[dd] == 6 ? 3 : 2;
        double ring = 0.0;
        for (int q = 0; q < np; ++q) ring += nk[RING_V[dd][q]] + nk[RING_VM[dd][q]];
        const double wr = DIR_NT[dd] == 6 ? sc.w_ring6 : sc.w_ring4;
        const double kh = sc.w_end * (kc0 + nk[dd]) + wr * ring;
        for (int q = 0; q < 6; ++q) d[q] -= kh * sc.pr[dd >> 1].shat[q] + sc.pr[dd >> 1].a0[q];
      }
    } else {
      const ElemConst<double> &ec = ecs[m];
      for (int t = 0; t < NTET; ++t) {
        const int v1 = TET_V[t][0], v2 = TET_V[t][1], v3 = TET_V[t][2];
        if (!(in[v1] && in[v2] && in[v3])) continue;
        const double kb = 0.25 * (kc0 + nk[v1] + nk[v2] + nk[v3]);
        const double *B1 = ec.b1[t][0];
        const double *B0 = ec.b0[t][0];
        const int ix[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
        for (int q = 0; q < 6; ++q) {
          const int a = 3 * ix[q][0] + ix[q][1], b = 3 * ix[q][1] + ix[q][0];
          d[q] += 0.5 * ((B0[a] + kb * B1[a]) + (B0[b] + kb * B1[b]));
        }
      }
    }
  }
  for (int q = 0; q < 6; ++q) D[q * N + slot] = d[q];
}

// Sum of the diagonal-block partials over the copies of interface nodes:
// one thread per (group, entry), so the grid must cover 6 * ng threads.
__global__ void k_group_sum6(const int64_t *__restrict__ ptr, const int64_t *__restrict__ slots,
                             int64_t ng, double *__restrict__ D, int64_t N) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = t / 6;
  const int c = (int)(t - 6 * g);
  if (g >= ng) return;
  double sum = 0.0;
  for (int64_t q = ptr[g]; q < ptr[g + 1]; ++q) sum += D[c * N + slots[q]];
  for (int64_t q = ptr[g]; q < ptr[g + 1]; ++q) D[c * N + slots[q]] = sum;
}

// P = D^{-1} (symmetric 3x3 by cofactors); zero block where D is zero
// (Dirichlet slots); identity when no preconditioner is wanted.
__global__ void k_invert(double *__restrict__ P, const uint8_t *__restrict__ fl, int64_t N, int ident) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N;
       s += (int64_t)gridDim.x * blockDim.x) {
    if (fl[s] & 1) {
      for (int q = 0; q < 6; ++q) P[q * N + s] = 0.0;
      continue;
    }
    if (ident) {
      P[s] = P[N + s] = P[2 * N + s] = 1.0;
      P[3 * N + s] = P[4 * N + s] = P[5 * N + s] = 0.0;
      continue;
    }
    const double a = P[s], b = P[N + s], c = P[2 * N + s];
    const double d = P[3 * N + s], e = P[4 * N + s], f = P[5 * N + s];
    // [[a d e] [d b f] [e f c]]
    const double A = b * c - f * f, B = e * f - d * c, C = d * f - b * e;
    const double det = a * A + d * B + e * C;
    const double r = 1.0 / det;
    P[s] = A * r;
    P[N + s] = (a * c - e * e) * r;
    P[2 * N + s] = (a * b - d * d) * r;
    P[3 * N + s] = B * r;
    P[4 * N + s] = C * r;
    P[5 * N + s] = (d * e - a * f) * r;
  }
}

}  // namespace

// Diagonal 3x3 blocks (xx yy zz xy xz yz, [6][n]) of the operator at every
// slot, summed over the copies of interface nodes; zero at Dirichlet slots.
int diag_blocks(hhg_ctx *h, const double *k, int method, double *D, hipStream_t st) {
  int maxn = 0;
  for (auto &mi : h->minfo) maxn = std::max(maxn, (int)macro_nodes(mi.n));
  const int64_t N = h->n_nodes;
  hipLaunchKernelGGL(k_diag, dim3((maxn + 255) / 256, h->n_macro), dim3(256), 0, st, h->d_minfo,
                     h->d_sc64, h->d_ec64, k, method, h->op.iface == HHG_IFACE_ZEROSUM ? 1 : 0, N, D);
  if (h->n_grp > 0)
    hipLaunchKernelGGL(k_group_sum6, dim3((unsigned)((6 * h->n_grp + 255) / 256)), dim3(256), 0, st,
                       h->d_grp_ptr, h->d_grp_slot, h->n_grp, D, N);
  HHG_HIP(hipGetLastError());
  return HHG_OK;
}

namespace {

// ------------------------------------------------------------ workspace
struct Layout {
  size_t off_r64, off_z64, off_p64, off_q64, off_P64, off_part, off_state;
  size_t off_feat, off_mlp;
  size_t off_k32, off_b32, off_e32, off_r32, off_z32, off_p32, off_q32, off_P32;
  size_t total;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

Layout layout_for(int64_t N, int solver, int precond) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  const size_t v64 = 3 * (size_t)N * 8, v32 = 3 * (size_t)N * 4;
  L.off_r64 = take(v64);
  L.off_P64 = take(6 * (size_t)N * 8);
  L.off_part = take(3 * RED_GRID * 8);
  L.off_state = take(sizeof(CGState));
  if (precond == HHG_PRECOND_LEARNED) {
    L.off_feat = take(16 * (size_t)N * 2);   // BF16 features
    L.off_mlp = take(9 * (size_t)N * 4);     // network outputs
  }
  if (solver != HHG_IR_F32) {
    L.off_z64 = take(v64);
    L.off_p64 = take(v64);
    L.off_q64 = take(v64);
  } else {
    L.off_k32 = take((size_t)N * 4);
    L.off_b32 = take(v32);
    L.off_e32 = take(v32);
    L.off_r32 = take(v32);
    L.off_z32 = take(v32);
    L.off_p32 = take(v32);
    L.off_q32 = take(v32);
    L.off_P32 = take(6 * (size_t)N * 4);
  }
  L.total = o;
  return L;
}

dim3 grid_for(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return dim3((unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), 4096));
}

struct Host {
  CGState *st = nullptr;  // pinned mirror of the device state
};

// One preconditioned CG run on A x = b (type T) from the given x to
// ||r|| <= tol_abs.  Returns HHG_OK / HHG_ENOCONV / HHG_EBREAKDOWN.
// Iterations run in blocks of `check` between host checks: `run` counts
// every iteration executed, `iters` the iterations until the recursive
// residual first met tol_abs (= run when it never did).
template <typename T>
int pcg(hhg_ctx *h, int method, bool flex, const T *b, const T *k, T *x, T *r, T *z, T *p, T *q,
        const T *P, double *part, CGState *dst, CGState *hst, double tol_abs, int maxit, int check,
        hipStream_t st, int &iters, int &run) {
  const int prec = sizeof(T) == 8 ? HHG_F64 : HHG_F32;
  const int64_t N = h->n_nodes;
  iters = 0;
  run = 0;
  int rc = apply_internal(h, prec, method, b, x, k, r, st);  // r = b - A x
  if (rc) return rc;
  // partial sums of (p, A p) from the apply itself (allocated here, before
  // any graph capture, and kept by the handle)
  const int64_t nparts = dot_parts(h);
  if (h->dotpart_cap < nparts) {
    if (h->d_dotpart) HHG_HIP(hipFree(h->d_dotpart));
    h->d_dotpart = nullptr;
    h->dotpart_cap = 0;
    HHG_HIP(hipMalloc((void **)&h->d_dotpart, 3 * (size_t)nparts * sizeof(double)));
    h->dotpart_cap = nparts;
  }
  {
    ProfScope ps(h, HHG_K_SOLVER_VECTOR, st);
    hipLaunchKernelGGL(k_precond<T>, dim3(RED_GRID), dim3(RED_TPB), 0, st, r, P, z, p, h->d_flags, N, part);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RED_TPB), 0, st, part, RED_GRID, dst, FIN_INIT, 0);
  }
  HHG_HIP(hipGetLastError());
  HHG_HIP(hipMemcpyAsync(hst, dst, sizeof(CGState), hipMemcpyDeviceToHost, st));
  HHG_HIP(hipStreamSynchronize(st));
  if (hst->bad) return fail(HHG_EBREAKDOWN, "non-finite initial residual");
  if (std::sqrt(hst->rr) <= tol_abs) return HHG_OK;

  auto body = [&](int nit) -> int {
    for (int it = 0; it < nit; ++it) {
      // q = A p with the partial sums of (p, q)
      int rc2 = apply_dot_internal(h, prec, method, p, k, q, h->d_dotpart, st);
      if (rc2) return rc2;
      ProfScope ps(h, HHG_K_SOLVER_VECTOR, st);
      hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RED_TPB), 0, st, h->d_dotpart, (int)nparts, dst,
                         FIN_ALPHA, it);
      if (flex)
        hipLaunchKernelGGL((k_update<T, true>), dim3(RED_GRID), dim3(RED_TPB), 0, st, r, q, P, z,
                           h->d_flags, N, dst, part);
      else
        hipLaunchKernelGGL((k_update<T, false>), dim3(RED_GRID), dim3(RED_TPB), 0, st, r, q, P, z,
                           h->d_flags, N, dst, part);
      hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RED_TPB), 0, st, part, RED_GRID, dst,
                         flex ? FIN_BETA_FLEX : FIN_BETA, it);
      hipLaunchKernelGGL(k_pupdate<T>, grid_for(3 * N), dim3(256), 0, st, x, p, z, 3 * N, dst);
    }
    HHG_HIP(hipGetLastError());
    return HHG_OK;
  };

  // capture one block of `check` iterations in a graph and replay it
  const bool use_graph = !h->prof_on && std::getenv("HHG_NO_GRAPH") == nullptr;
  hipGraphExec_t exec = nullptr;
  if (use_graph) {
    hipGraph_t graph = nullptr;
    HHG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    int brc = body(check);
    hipError_t ce = hipStreamEndCapture(st, &graph);
    if (brc) {
      if (graph) (void)hipGraphDestroy(graph);
      return brc;
    }
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
  }
  int status = HHG_ENOCONV;
  while (run < maxit) {
    const int nit = std::min(check, maxit - run);
    if (use_graph && nit == check) {
      hipError_t e = hipGraphLaunch(exec, st);
      if (e != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        return hip_fail(e, "hipGraphLaunch");
      }
    } else {
      int brc = body(nit);
      if (brc) {
        if (exec) (void)hipGraphExecDestroy(exec);
        return brc;
      }
    }
    HHG_HIP(hipMemcpyAsync(hst, dst, sizeof(CGState), hipMemcpyDeviceToHost, st));
    HHG_HIP(hipStreamSynchronize(st));
    // the first iteration of the block that met the tolerance, if it came
    // before a breakdown
    const int last = hst->bad ? std::min(hst->bad_it, nit) : nit;
    int first = -1;
    for (int it = 0; it < last; ++it)
      if (std::sqrt(hst->hist[it]) <= tol_abs) {
        first = it;
        break;
      }
    if (first >= 0) {
      iters = run + first + 1;
      run += nit;
      status = HHG_OK;
      break;
    }
    run += nit;
    iters = run;
    if (hst->bad) {
      status = HHG_EBREAKDOWN;
      set_error("CG breakdown: p^T A p <= 0 or non-finite value");
      break;
    }
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (status == HHG_ENOCONV) set_error("CG reached maxit");
  return status;
}

template <typename T>
T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

int dot_host(hhg_ctx *h, const double *a, const double *b, double *part, CGState *dst,
             CGState *hst, hipStream_t st, double &out) {
  hipLaunchKernelGGL(k_dot2<double>, dim3(RED_GRID), dim3(RED_TPB), 0, st, a, b,
                     (const double *)nullptr, (const double *)nullptr, h->d_flags, h->n_nodes, part);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RED_TPB), 0, st, part, RED_GRID, dst, FIN_NORM, 0);
  HHG_HIP(hipGetLastError());
  HHG_HIP(hipMemcpyAsync(hst, dst, sizeof(CGState), hipMemcpyDeviceToHost, st));
  HHG_HIP(hipStreamSynchronize(st));
  out = hst->rr;
  return HHG_OK;
}

int check_opts(hhg_ctx *h, const hhg_solve_opts *o) {
  if (!h || !o) return fail(HHG_EINVAL, "null argument");
  if (o->solver != HHG_CG_F64 && o->solver != HHG_IR_F32 && o->solver != HHG_FCG_F64)
    return fail(HHG_EINVAL, "unknown solver");
  if (o->precond != HHG_PRECOND_NONE && o->precond != HHG_PRECOND_BLOCK_JACOBI &&
      o->precond != HHG_PRECOND_LEARNED)
    return fail(HHG_EINVAL, "unknown preconditioner");
  if (o->precond == HHG_PRECOND_LEARNED && !h->model)
    return fail(HHG_EINVAL, "learned preconditioner requested but no model is attached");
  if (o->method != HHG_METHOD_SCALED && o->method != HHG_METHOD_ONTHEFLY)
    return fail(HHG_EINVAL, "unknown operator method");
  if (!(o->rtol > 0.0) || o->maxit < 1) return fail(HHG_EINVAL, "rtol must be > 0 and maxit >= 1");
  if (o->solver == HHG_IR_F32 && !(o->inner_rtol > 0.0 && o->inner_rtol < 1.0))
    return fail(HHG_EINVAL, "inner_rtol must lie in (0, 1)");
  return HHG_OK;
}

}  // namespace

namespace {
int solve_impl(hhg_ctx *h, const hhg_solve_opts *o, const double *b, const double *k, double *x,
               void *ws, hhg_solve_info *info, hipStream_t st);
}

// The solve runs on the handle's own stream (a graph cannot be captured on
// the legacy default stream), ordered after the caller's stream.
int solve_entry(hhg_ctx *h, const hhg_solve_opts *o, const double *b, const double *k, double *x,
                void *ws, hhg_solve_info *info, hipStream_t user) {
  int rc = check_opts(h, o);
  if (rc) return rc;
  if (!b || !k || !x || !ws || !info) return fail(HHG_EINVAL, "null pointer");
  if (((uintptr_t)ws & 255) || (((uintptr_t)b | (uintptr_t)k | (uintptr_t)x) & 15))
    return fail(HHG_EINVAL, "misaligned pointer");
  if ((rc = ensure_device(h))) return rc;
  HHG_HIP(hipEventRecord(h->ev_fork, user));
  HHG_HIP(hipStreamWaitEvent(h->solve_stream, h->ev_fork, 0));
  rc = solve_impl(h, o, b, k, x, ws, info, h->solve_stream);
  (void)hipStreamSynchronize(h->solve_stream);
  if (rc != HHG_OK && info->status == HHG_OK) info->status = rc;
  return rc;
}

namespace {
int solve_impl(hhg_ctx *h, const hhg_solve_opts *o, const double *b, const double *k, double *x,
               void *ws, hhg_solve_info *info, hipStream_t st) {
  int rc;
  std::memset(info, 0, sizeof(*info));
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t N = h->n_nodes;
  const Layout L = layout_for(N, o->solver, o->precond);
  const int check = std::max(1, std::min(o->check_every > 0 ? o->check_every : 8, MAX_CHECK));
  if (!h->h_state) HHG_HIP(hipHostMalloc((void **)&h->h_state, sizeof(CGState), hipHostMallocDefault));
  CGState *hst = static_cast<CGState *>(h->h_state);
  CGState *dst = at<CGState>(ws, L.off_state);
  double *part = at<double>(ws, L.off_part);
  double *r64 = at<double>(ws, L.off_r64);
  double *P64 = at<double>(ws, L.off_P64);

  // block-Jacobi preconditioner from the operator's diagonal blocks; the
  // learned one reshapes it by the network's 3x3 blocks
  {
    if ((rc = diag_blocks(h, k, o->method, P64, st))) return rc;
    hipLaunchKernelGGL(k_invert, grid_for(N), dim3(256), 0, st, P64, h->d_flags, N,
                       o->precond == HHG_PRECOND_NONE ? 1 : 0);
    HHG_HIP(hipGetLastError());
    if (o->precond == HHG_PRECOND_LEARNED &&
        (rc = learned_precond(h, k, P64, at<uint16_t>(ws, L.off_feat), at<float>(ws, L.off_mlp), st)))
      return rc;
    hipLaunchKernelGGL(k_zero_dirichlet<double>, grid_for(N), dim3(256), 0, st, x, h->d_flags, N);
    HHG_HIP(hipGetLastError());
  }
  double bb = 0.0;
  if ((rc = dot_host(h, b, b, part, dst, hst, st, bb))) return rc;
  const double bnorm = std::sqrt(bb);
  if (!std::isfinite(bnorm)) return fail(HHG_EBREAKDOWN, "non-finite right-hand side");
  int status = HHG_OK;
  int total = 0, total_run = 0;
  if (bnorm == 0.0) {
    hipLaunchKernelGGL(k_fill<double>, grid_for(3 * N), dim3(256), 0, st, x, 0.0, 3 * N);
    HHG_HIP(hipStreamSynchronize(st));
    info->status = HHG_OK;
    return HHG_OK;
  }

  if (o->solver != HHG_IR_F32) {
    double *z = at<double>(ws, L.off_z64), *p = at<double>(ws, L.off_p64), *q = at<double>(ws, L.off_q64);
    int outer = 0;
    status = HHG_ENOCONV;
    while (total_run < o->maxit) {
      int it = 0, itr = 0;
      ++outer;
      rc = pcg<double>(h, o->method, o->solver == HHG_FCG_F64, b, k, x, r64, z, p, q, P64, part, dst, hst, o->rtol * bnorm,
                       o->maxit - total_run, check, st, it, itr);
      total += it;
      total_run += itr;
      if (rc == HHG_EBREAKDOWN || (rc != HHG_OK && rc != HHG_ENOCONV)) {
        status = rc;
        break;
      }
      // true FP64 residual decides convergence (restart if the recursion drifted)
      if ((rc = apply_internal(h, HHG_F64, o->method, b, x, k, r64, st))) return rc;
      double rr = 0.0;
      if ((rc = dot_host(h, r64, r64, part, dst, hst, st, rr))) return rc;
      info->rel_residual = std::sqrt(rr) / bnorm;
      if (info->rel_residual <= o->rtol) {
        status = HHG_OK;
        break;
      }
      if (itr == 0) break;
    }
    info->outer_iterations = outer;
  } else {
    float *k32 = at<float>(ws, L.off_k32), *b32 = at<float>(ws, L.off_b32), *e32 = at<float>(ws, L.off_e32);
    float *r32 = at<float>(ws, L.off_r32), *z32 = at<float>(ws, L.off_z32), *p32 = at<float>(ws, L.off_p32);
    float *q32 = at<float>(ws, L.off_q32), *P32 = at<float>(ws, L.off_P32);
    hipLaunchKernelGGL(k_cast64to32, grid_for(N), dim3(256), 0, st, k, k32, N);
    hipLaunchKernelGGL(k_cast64to32, grid_for(6 * N), dim3(256), 0, st, P64, P32, 6 * N);
    HHG_HIP(hipGetLastError());
    int outer = 0;
    status = HHG_ENOCONV;
    while (true) {
      if ((rc = apply_internal(h, HHG_F64, o->method, b, x, k, r64, st))) return rc;  // FP64 residual
      double rr = 0.0;
      if ((rc = dot_host(h, r64, r64, part, dst, hst, st, rr))) return rc;
      info->rel_residual = std::sqrt(rr) / bnorm;
      if (!std::isfinite(info->rel_residual)) {
        status = HHG_EBREAKDOWN;
        set_error("non-finite residual");
        break;
      }
      if (info->rel_residual <= o->rtol) {
        status = HHG_OK;
        break;
      }
      if (total_run >= o->maxit) break;
      ++outer;
      hipLaunchKernelGGL(k_cast64to32, grid_for(3 * N), dim3(256), 0, st, r64, b32, 3 * N);
      hipLaunchKernelGGL(k_fill<float>, grid_for(3 * N), dim3(256), 0, st, e32, 0.0f, 3 * N);
      HHG_HIP(hipGetLastError());
      int it = 0, itr = 0;
      rc = pcg<float>(h, o->method, false, b32, k32, e32, r32, z32, p32, q32, P32, part, dst, hst,
                      o->inner_rtol * std::sqrt(rr), o->maxit - total_run, check, st, it, itr);
      total += it;
      total_run += itr;
      if (rc == HHG_EBREAKDOWN || (rc != HHG_OK && rc != HHG_ENOCONV)) {
        status = rc;
        break;
      }
      hipLaunchKernelGGL(k_add32to64, grid_for(3 * N), dim3(256), 0, st, x, e32, 3 * N);
      HHG_HIP(hipGetLastError());
    }
    info->outer_iterations = outer;
  }
  HHG_HIP(hipStreamSynchronize(st));
  info->iterations = total;
  info->iterations_run = total_run;
  info->status = status;
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (status == HHG_ENOCONV) set_error("maxit reached before rtol");
  return status;
}
}  // namespace

size_t workspace_bytes(hhg_ctx *h, int solver, int precond) {
  return layout_for(h->n_nodes, solver, precond).total;
}

}  // namespace hhg

extern "C" {

int hhg_workspace_bytes(hhg_handle h, const hhg_solve_opts *o, size_t *bytes) {
  if (!h || !o || !bytes) return hhg::fail(HHG_EINVAL, "null argument");
  if (o->solver != HHG_CG_F64 && o->solver != HHG_IR_F32 && o->solver != HHG_FCG_F64)
    return hhg::fail(HHG_EINVAL, "unknown solver");
  *bytes = hhg::workspace_bytes(h, o->solver, o->precond);
  return HHG_OK;
}

}  // extern "C"

namespace hhg {
namespace {
// Scratch of hhg_preconditioner_noalloc: one static array on every device
// the library runs on, held until the process ends.  Its device address is
// looked up once per device (with that device current) and used for every
// kernel argument; the array's name is a host-side stand-in.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_addr[MAX_DEVICES] = {};

int scratch_ptr(void **out) {
  int dev = 0;
  HHG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(HHG_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_addr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    scratch_addr[dev] = p;
  }
  *out = scratch_addr[dev];
  return HHG_OK;
}

// learned blocks: BF16 features [N][16] then FP32 network outputs [N][9]
size_t learned_scratch_bytes(int64_t N, size_t *feat_bytes) {
  const size_t fb = ((16 * (size_t)N * 2 + 255) / 256) * 256;
  if (feat_bytes) *feat_bytes = fb;
  return fb + 9 * (size_t)N * 4;
}
}  // namespace
}  // namespace hhg

extern "C" {

int hhg_preconditioner_noalloc(hhg_handle h, int32_t precond, int32_t method, const double *k,
                               double *P, void *stream) {
  using namespace hhg;
  if (!h || !k || !P) return fail(HHG_EINVAL, "null argument");
  if (((uintptr_t)k | (uintptr_t)P) & 7) return fail(HHG_EINVAL, "misaligned pointer");
  if (precond != HHG_PRECOND_NONE && precond != HHG_PRECOND_BLOCK_JACOBI &&
      precond != HHG_PRECOND_LEARNED)
    return fail(HHG_EINVAL, "unknown preconditioner");
  if (method != HHG_METHOD_SCALED && method != HHG_METHOD_ONTHEFLY)
    return fail(HHG_EINVAL, "unknown operator method");
  if (precond == HHG_PRECOND_LEARNED && !h->model)
    return fail(HHG_EINVAL, "learned preconditioner requested but no model is attached");
  const int64_t N = h->n_nodes;
  size_t fb = 0;
  if (precond == HHG_PRECOND_LEARNED && learned_scratch_bytes(N, &fb) > NOALLOC_SCRATCH_BYTES)
    return fail(HHG_EINVAL, "learned blocks of " + std::to_string(N) + " slots need " +
                                std::to_string(learned_scratch_bytes(N, nullptr)) +
                                " scratch bytes, more than the static 64 MiB");
  // the handle's tables are uploaded by its first device call, which
  // allocates: this entry point only runs on a handle that had one
  if (!h->on_device)
    return fail(HHG_EINVAL, "handle not yet on a device: call any device entry point on it first");
  int rc = ensure_device(h);   // on a device already: checks the current device only
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  void *s = nullptr;
  if (precond == HHG_PRECOND_LEARNED && (rc = scratch_ptr(&s))) return rc;
  if ((rc = diag_blocks(h, k, method, P, st))) return rc;
  hipLaunchKernelGGL(k_invert, grid_for(N), dim3(256), 0, st, P, h->d_flags, N,
                     precond == HHG_PRECOND_NONE ? 1 : 0);
  HHG_HIP(hipGetLastError());
  if (precond == HHG_PRECOND_LEARNED &&
      (rc = learned_precond(h, k, P, static_cast<uint16_t *>(s),
                            reinterpret_cast<float *>(static_cast<char *>(s) + fb), st)))
    return rc;
  HHG_HIP(hipStreamSynchronize(st));
  return HHG_OK;
}

int hhg_cg_solve(hhg_handle h, const hhg_solve_opts *o, const double *b, const double *k,
                 double *x, void *workspace, hhg_solve_info *info, void *stream) {
  return hhg::solve_entry(h, o, b, k, x, workspace, info, (hipStream_t)stream);
}

int hhg_preconditioner(hhg_handle h, int32_t precond, int32_t method, const double *k, double *P,
                       void *stream) {
  using namespace hhg;
  if (!h || !k || !P) return fail(HHG_EINVAL, "null argument");
  if (((uintptr_t)k | (uintptr_t)P) & 7) return fail(HHG_EINVAL, "misaligned pointer");
  if (precond != HHG_PRECOND_NONE && precond != HHG_PRECOND_BLOCK_JACOBI &&
      precond != HHG_PRECOND_LEARNED)
    return fail(HHG_EINVAL, "unknown preconditioner");
  if (method != HHG_METHOD_SCALED && method != HHG_METHOD_ONTHEFLY)
    return fail(HHG_EINVAL, "unknown operator method");
  if (precond == HHG_PRECOND_LEARNED && !h->model)
    return fail(HHG_EINVAL, "learned preconditioner requested but no model is attached");
  int rc = ensure_device(h);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int64_t N = h->n_nodes;
  if ((rc = diag_blocks(h, k, method, P, st))) return rc;
  hipLaunchKernelGGL(k_invert, grid_for(N), dim3(256), 0, st, P, h->d_flags, N,
                     precond == HHG_PRECOND_NONE ? 1 : 0);
  HHG_HIP(hipGetLastError());
  if (precond == HHG_PRECOND_LEARNED) {
    void *scratch = nullptr;
    const size_t fb = ((16 * (size_t)N * 2 + 255) / 256) * 256;
    HHG_HIP(hipMalloc(&scratch, fb + 9 * (size_t)N * 4));
    rc = learned_precond(h, k, P, static_cast<uint16_t *>(scratch),
                         reinterpret_cast<float *>(static_cast<char *>(scratch) + fb), st);
    hipError_t se = hipStreamSynchronize(st);
    (void)hipFree(scratch);
    if (rc) return rc;
    if (se != hipSuccess) return hip_fail(se, "hipStreamSynchronize");
    return HHG_OK;
  }
  HHG_HIP(hipStreamSynchronize(st));
  return HHG_OK;
}

}  // extern "C"
