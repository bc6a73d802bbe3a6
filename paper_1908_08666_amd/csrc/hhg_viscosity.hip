// Nodal viscosity of a generalized Newtonian fluid from a velocity field
// (Sec. 3 and the Carreau law eq. carreau of Sec. 5.2.2).
//
// Macro-interior node: gradient of the affine least-squares fit of u over
// the 15-node patch, grad u = sum_d W_d (u_{i+d} - u_i).  Node on a macro
// boundary: volume-weighted mean of the element gradients of all elements at
// the node, accumulated per macro and summed over the node's copies.  Then
// |eps|^2 = eps : eps and mu = eta_inf + (eta0 - eta_inf)(1 + kappa |eps|^2)^r.
#include <cmath>

#include "hhg_device.h"

namespace hhg {
namespace {

__device__ __forceinline__ int pbase(int n, int k) {
  const int a = n + 1, b = n + 1 - k;
  return a * (a + 1) * (a + 2) / 6 - b * (b + 1) * (b + 2) / 6;
}

__device__ __forceinline__ double carreau(const double G[3][3], const hhg_carreau &law) {
  double e2 = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const double e = 0.5 * (G[a][b] + G[b][a]);
      e2 += e * e;
    }
  return law.eta_inf + (law.eta0 - law.eta_inf) * pow(1.0 + law.kappa * e2, law.r);
}

__global__ __launch_bounds__(256) void k_visc(const MacroInfo *__restrict__ minfo,
                                              const StrainConst *__restrict__ stc,
                                              const double *__restrict__ u, int64_t N,
                                              hhg_carreau law, double *__restrict__ kout,
                                              double *__restrict__ S) {
  const int m = blockIdx.y;
  const MacroInfo mi = minfo[m];
  const int n = mi.n;
  const int ls = blockIdx.x * blockDim.x + threadIdx.x;
  if (ls >= (int)macro_nodes(n)) return;
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (pbase(n, mid) <= ls) lo = mid; else hi = mid - 1;
  }
  const int k = lo;
  const int pos = ls - pbase(n, k);
  const int s = tri_root_dev(pos);
  const int i = pos - s * (s + 1) / 2, j = s - i;
  const int64_t slot = mi.off + ls;
  const StrainConst &sc = stc[m];
  const double *U0 = u + mi.off, *U1 = U0 + N, *U2 = U1 + N;
  auto loc = [&](int d, bool &in) {
    const int a = i + DIR_I[d], b = j + DIR_J[d], c = k + DIR_K[d];
    in = a >= 0 && b >= 0 && c >= 0 && a + b + c <= n;
    return in ? pbase(n, c) + (a + b) * (a + b + 1) / 2 + a : 0;
  };
  const double c0 = U0[ls], c1 = U1[ls], c2 = U2[ls];
  double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  if (zero_set(i, j, k, n) == 0) {
    for (int d = 0; d < NDIR; ++d) {
      bool in;
      const int l = loc(d, in);
      const double du[3] = {U0[l] - c0, U1[l] - c1, U2[l] - c2};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) G[a][b] += du[a] * sc.w[d][b];
    }
    kout[slot] = carreau(G, law);
    return;
  }
  // macro-boundary node: this macro's share of sum_t |t| grad u_t and sum_t |t|
  int lv[NDIR];
  bool in[NDIR];
  for (int d = 0; d < NDIR; ++d) lv[d] = loc(d, in[d]);
  double vol = 0.0;
  for (int t = 0; t < NTET; ++t) {
    const int v1 = TET_V[t][0], v2 = TET_V[t][1], v3 = TET_V[t][2];
    if (!(in[v1] && in[v2] && in[v3])) continue;
    vol += sc.vol;
    const int ids[3] = {lv[v1], lv[v2], lv[v3]};
    for (int a = 0; a < 3; ++a) {
      const double *Ua = a == 0 ? U0 : (a == 1 ? U1 : U2);
      const double uc = a == 0 ? c0 : (a == 1 ? c1 : c2);
      for (int b = 0; b < 3; ++b) {
        double g = uc * sc.grad[t][0][b];
        for (int q = 0; q < 3; ++q) g += Ua[ids[q]] * sc.grad[t][q + 1][b];
        G[a][b] += sc.vol * g;
      }
    }
  }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) S[(3 * a + b) * N + slot] = G[a][b];
  S[9 * N + slot] = vol;
}

__global__ void k_group_sum10(const int64_t *__restrict__ ptr, const int64_t *__restrict__ slots,
                              int64_t ng, double *__restrict__ S, int64_t N) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = t / 10;
  const int c = (int)(t - 10 * g);
  if (g >= ng) return;
  double sum = 0.0;
  for (int64_t q = ptr[g]; q < ptr[g + 1]; ++q) sum += S[c * N + slots[q]];
  for (int64_t q = ptr[g]; q < ptr[g + 1]; ++q) S[c * N + slots[q]] = sum;
}

__global__ void k_visc_boundary(const uint8_t *__restrict__ fl, const double *__restrict__ S,
                                int64_t N, hhg_carreau law, double *__restrict__ kout) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N;
       s += (int64_t)gridDim.x * blockDim.x) {
    if (!(fl[s] & 4)) continue;
    const double v = S[9 * N + s];
    double G[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) G[a][b] = S[(3 * a + b) * N + s] / v;
    kout[s] = carreau(G, law);
  }
}

}  // namespace
}  // namespace hhg

extern "C" {

int hhg_viscosity_workspace_bytes(hhg_handle h, size_t *bytes) {
  if (!h || !bytes) return hhg::fail(HHG_EINVAL, "null argument");
  *bytes = 10 * (size_t)h->n_nodes * sizeof(double);
  return HHG_OK;
}

int hhg_nodal_viscosity(hhg_handle h, const double *u, const hhg_carreau *law, double *k,
                        void *workspace, void *stream) {
  using namespace hhg;
  if (!h || !u || !law || !k || !workspace) return fail(HHG_EINVAL, "null argument");
  if ((((uintptr_t)u | (uintptr_t)k | (uintptr_t)workspace) & 15))
    return fail(HHG_EINVAL, "misaligned pointer");
  if (!(law->eta0 >= law->eta_inf) || !(law->eta_inf > 0.0) || !(law->kappa >= 0.0) ||
      !std::isfinite(law->r))
    return fail(HHG_EINVAL, "Carreau parameters need eta0 >= eta_inf > 0, kappa >= 0");
  int rc = ensure_device(h);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int64_t N = h->n_nodes;
  double *S = static_cast<double *>(workspace);
  int maxn = 0;
  for (auto &mi : h->minfo) maxn = std::max(maxn, (int)macro_nodes(mi.n));
  hipLaunchKernelGGL(k_visc, dim3((maxn + 255) / 256, h->n_macro), dim3(256), 0, st, h->d_minfo,
                     h->d_stc, u, N, *law, k, S);
  if (h->n_agrp > 0)
    hipLaunchKernelGGL(k_group_sum10, dim3((unsigned)((10 * h->n_agrp + 255) / 256)), dim3(256), 0,
                       st, h->d_agrp_ptr, h->d_agrp_slot, h->n_agrp, S, N);
  hipLaunchKernelGGL(k_visc_boundary, dim3(2048), dim3(256), 0, st, h->d_flags, S, N, *law, k);
  HHG_HIP(hipGetLastError());
  return HHG_OK;
}

}  // extern "C"
