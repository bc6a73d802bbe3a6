// Nodal viscosity of a generalized Newtonian fluid from a velocity field
// (Sec. 3 and the Carreau law eq. carreau of Sec. 5.2.2).
//
// Macro-interior node: gradient of the affine least-squares fit of u over
// the 15-node patch, grad u = sum_d W_d (u_{i+d} - u_i).  Node on a macro
// boundary: least-squares fit onto quadratics over its patch in the whole
// mesh (weights built on the host, one thread per distinct node), or the
// volume-weighted mean of the element gradients of all elements at the node,
// accumulated per macro and summed over the node's copies.  Then
// |eps|^2 = eps : eps and mu = eta_inf + (eta0 - eta_inf)(1 + kappa |eps|^2)^r.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <unordered_map>
#include <vector>

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
                                              hhg_carreau law, int lsq, double *__restrict__ kout,
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
  if (lsq) return;                          // k_visc_lsq takes the macro-boundary nodes
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

// Macro-boundary nodes by least squares: one thread per distinct node,
// grad u = sum_e u(slot_e) w_e^T over its patch, the viscosity written to
// every copy.
__global__ void k_visc_lsq(const int64_t *__restrict__ ptr, const int64_t *__restrict__ pslot,
                           const double *__restrict__ w, const int64_t *__restrict__ optr,
                           const int64_t *__restrict__ oslot, int64_t nq,
                           const double *__restrict__ u, int64_t N, hhg_carreau law,
                           double *__restrict__ kout) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq;
       q += (int64_t)gridDim.x * blockDim.x) {
    double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int64_t e = ptr[q]; e < ptr[q + 1]; ++e) {
      const int64_t sl = pslot[e];
      const double uv[3] = {u[sl], u[N + sl], u[2 * N + sl]};
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) G[a][b] += uv[a] * w[3 * e + b];
    }
    const double mu = carreau(G, law);
    for (int64_t o = optr[q]; o < optr[q + 1]; ++o) kout[oslot[o]] = mu;
  }
}

// ---------------------------------------------------------------- host
// Relative size below which a singular value of the scaled design matrix
// counts as zero; the rank-deficient patches met here are exactly deficient,
// their null singular values at rounding level.
constexpr double RANK_TOL = 1e-6;

// Eigen-decomposition of a symmetric matrix (n <= 10) by cyclic Jacobi
// rotations: on return a holds the eigenvalues on its diagonal, v the
// eigenvectors in its columns.
void jacobi_eigen(int n, double a[10][10], double v[10][10]) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) v[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i) {
      diag += a[i][i] * a[i][i];
      for (int j = i + 1; j < n; ++j) off += a[i][j] * a[i][j];
    }
    if (off <= 1e-34 * diag) return;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        if (a[p][q] == 0.0) continue;
        const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {            // columns p, q
          const double akp = a[k][p], akq = a[k][q];
          a[k][p] = c * akp - sn * akq;
          a[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {            // rows p, q
          const double apk = a[p][k], aqk = a[q][k];
          a[p][k] = c * apk - sn * aqk;
          a[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = v[k][p], vkq = v[k][q];
          v[k][p] = c * vkp - sn * vkq;
          v[k][q] = sn * vkp + c * vkq;
        }
      }
  }
}

// Gradient weights at d[0] = 0 of the least-squares fit over the points d
// (already scaled to max |d| = 1) onto polynomials of the given degree:
// grad = sum_p W[p] u_p.  False when the gradient is not determined, i.e.
// a polynomial vanishing at every point has a non-zero gradient at d[0].
// The weights are those of the minimum-norm solution.
bool fit_weights(const std::vector<std::array<double, 3>> &d, int degree,
                 std::vector<std::array<double, 3>> &W) {
  const int nb = degree == 2 ? 10 : 4, P = (int)d.size();
  std::vector<std::array<double, 10>> A(P);
  for (int p = 0; p < P; ++p) {
    const double x = d[p][0], y = d[p][1], z = d[p][2];
    const double row[10] = {1.0, x, y, z, x * x, y * y, z * z, x * y, x * z, y * z};
    for (int c = 0; c < 10; ++c) A[p][c] = row[c];
  }
  double M[10][10], V[10][10];
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < nb; ++j) {
      double t = 0.0;
      for (int p = 0; p < P; ++p) t += A[p][i] * A[p][j];
      M[i][j] = t;
    }
  jacobi_eigen(nb, M, V);
  double lmax = 0.0;
  for (int i = 0; i < nb; ++i) lmax = std::max(lmax, M[i][i]);
  const double lcut = RANK_TOL * RANK_TOL * lmax;
  for (int k = 0; k < nb; ++k)
    if (M[k][k] <= lcut)
      for (int r = 1; r <= 3; ++r)
        if (std::fabs(V[r][k]) > RANK_TOL) return false;
  W.assign(P, {0.0, 0.0, 0.0});
  for (int k = 0; k < nb; ++k) {
    if (M[k][k] <= lcut) continue;
    for (int p = 0; p < P; ++p) {
      double av = 0.0;                           // (A v_k)_p
      for (int c = 0; c < nb; ++c) av += A[p][c] * V[c][k];
      for (int r = 0; r < 3; ++r) W[p][r] += V[r + 1][k] * av / M[k][k];
    }
  }
  return true;
}

template <typename T>
int upload_vec(T **dst, const std::vector<T> &src) {
  if (src.empty()) return HHG_OK;
  hipError_t e = hipMalloc((void **)dst, src.size() * sizeof(T));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  return HHG_OK;
}

// Patches and fit weights of all distinct macro-boundary nodes.
int build_lsq(hhg_ctx *h) {
  const int64_t N = h->n_nodes;
  // one canonical slot per node: the first slot of its copy group
  std::vector<int64_t> canon(N);
  for (int64_t s = 0; s < N; ++s) canon[s] = s;
  for (int64_t g = 0; g < h->n_agrp; ++g)
    for (int64_t q = h->agrp_ptr[g]; q < h->agrp_ptr[g + 1]; ++q)
      canon[h->agrp_slot[q]] = h->agrp_slot[h->agrp_ptr[g]];
  std::vector<int64_t> group_of(N, -1);
  for (int64_t g = 0; g < h->n_agrp; ++g)
    for (int64_t q = h->agrp_ptr[g]; q < h->agrp_ptr[g + 1]; ++q) group_of[h->agrp_slot[q]] = g;
  auto coords = [&](int m, int i, int j, int k) {
    const double *V = h->verts.data() + 12 * m;
    const int n = h->minfo[m].n;
    std::array<double, 3> x;
    for (int c = 0; c < 3; ++c)
      x[c] = V[c] + ((double)i * (V[3 + c] - V[c]) + (double)j * (V[6 + c] - V[c]) +
                     (double)k * (V[9 + c] - V[c])) / n;
    return x;
  };
  struct Node {
    int64_t slot;
    std::array<double, 3> x;
    std::vector<std::pair<int64_t, std::array<double, 3>>> nbr;
  };
  std::vector<Node> nodes;
  std::unordered_map<int64_t, int64_t> index;
  for (int m = 0; m < h->n_macro; ++m) {
    const int n = h->minfo[m].n;
    const int64_t off = h->minfo[m].off;
    for (int k = 0; k <= n; ++k)
      for (int s = 0; s + k <= n; ++s)
        for (int i = 0; i <= s; ++i) {
          const int j = s - i;
          if (!(i == 0 || j == 0 || k == 0 || i + j + k == n)) continue;   // macro-interior
          const int64_t c = canon[off + plane_base(n, k) + tri(s) + i];
          auto it = index.find(c);
          if (it == index.end()) {
            it = index.emplace(c, (int64_t)nodes.size()).first;
            nodes.push_back(Node{c, coords(m, i, j, k), {}});
          }
          Node &nd = nodes[it->second];
          for (int d = 0; d < NDIR; ++d) {
            const int a = i + DIR_I[d], b = j + DIR_J[d], cc = k + DIR_K[d];
            if (a < 0 || b < 0 || cc < 0 || a + b + cc > n) continue;
            const int64_t ns = canon[off + plane_base(n, cc) + tri(a + b) + a];
            nd.nbr.push_back({ns, coords(m, a, b, cc)});
          }
        }
  }
  // weights per node; patches of one shape (same scaled offsets in the same
  // order) share them
  std::vector<int64_t> ptr(1, 0), pslot, optr(1, 0), oslot;
  std::vector<double> w;
  struct Fit {
    bool affine;                               // the quadratic fit left the gradient open
    std::vector<std::array<double, 3>> W;
  };
  std::map<std::vector<int64_t>, Fit> cache;
  int64_t n_aff = 0;
  for (Node &nd : nodes) {
    std::sort(nd.nbr.begin(), nd.nbr.end(),
              [](const auto &a, const auto &b) { return a.first < b.first; });
    nd.nbr.erase(std::unique(nd.nbr.begin(), nd.nbr.end(),
                             [](const auto &a, const auto &b) { return a.first == b.first; }),
                 nd.nbr.end());
    std::vector<std::array<double, 3>> d(1, {0.0, 0.0, 0.0});
    std::vector<int64_t> sl(1, nd.slot);
    double hs = 0.0;
    for (auto &e : nd.nbr) {
      std::array<double, 3> t;
      for (int c = 0; c < 3; ++c) {
        t[c] = e.second[c] - nd.x[c];
        hs = std::max(hs, std::fabs(t[c]));
      }
      d.push_back(t);
      sl.push_back(e.first);
    }
    if (!(hs > 0.0)) return fail(HHG_EINVAL, "degenerate strain-rate patch");
    std::vector<int64_t> key;
    key.reserve(3 * d.size());
    for (auto &t : d)
      for (int c = 0; c < 3; ++c) {
        t[c] /= hs;
        key.push_back((int64_t)std::llround(t[c] * 1048576.0));
      }
    auto it = cache.find(key);
    if (it == cache.end()) {
      Fit f{false, {}};
      if (!fit_weights(d, 2, f.W)) {
        f.affine = true;
        if (!fit_weights(d, 1, f.W)) return fail(HHG_EINVAL, "strain-rate patch without an affine fit");
      }
      it = cache.emplace(key, std::move(f)).first;
    }
    const auto &W = it->second.W;
    n_aff += it->second.affine ? 1 : 0;
    for (size_t p = 0; p < d.size(); ++p) {
      pslot.push_back(sl[p]);
      for (int c = 0; c < 3; ++c) w.push_back(W[p][c] / hs);
    }
    ptr.push_back((int64_t)pslot.size());
    const int64_t g = group_of[nd.slot];
    if (g >= 0)
      for (int64_t q = h->agrp_ptr[g]; q < h->agrp_ptr[g + 1]; ++q) oslot.push_back(h->agrp_slot[q]);
    else
      oslot.push_back(nd.slot);
    optr.push_back((int64_t)oslot.size());
  }
  int rc;
  if ((rc = upload_vec(&h->d_lsq_ptr, ptr))) return rc;
  if ((rc = upload_vec(&h->d_lsq_slot, pslot))) return rc;
  if ((rc = upload_vec(&h->d_lsq_w, w))) return rc;
  if ((rc = upload_vec(&h->d_lsq_optr, optr))) return rc;
  if ((rc = upload_vec(&h->d_lsq_oslot, oslot))) return rc;
  h->n_lsq = (int64_t)nodes.size();
  h->n_lsq_affine = n_aff;
  h->lsq_built = true;
  return HHG_OK;
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
  if (law->boundary != HHG_STRAIN_LSQ && law->boundary != HHG_STRAIN_AVERAGE)
    return fail(HHG_EINVAL, "unknown strain-rate fit on macro boundaries");
  int rc = ensure_device(h);
  if (rc) return rc;
  const bool lsq = law->boundary == HHG_STRAIN_LSQ;
  if (lsq && !h->lsq_built && (rc = build_lsq(h))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int64_t N = h->n_nodes;
  double *S = static_cast<double *>(workspace);
  int maxn = 0;
  for (auto &mi : h->minfo) maxn = std::max(maxn, (int)macro_nodes(mi.n));
  hipLaunchKernelGGL(k_visc, dim3((maxn + 255) / 256, h->n_macro), dim3(256), 0, st, h->d_minfo,
                     h->d_stc, u, N, *law, lsq ? 1 : 0, k, S);
  if (lsq) {
    if (h->n_lsq > 0)
      hipLaunchKernelGGL(k_visc_lsq, dim3((unsigned)std::min<int64_t>((h->n_lsq + 255) / 256, 4096)),
                         dim3(256), 0, st, h->d_lsq_ptr, h->d_lsq_slot, h->d_lsq_w, h->d_lsq_optr,
                         h->d_lsq_oslot, h->n_lsq, u, N, *law, k);
  } else {
    if (h->n_agrp > 0)
      hipLaunchKernelGGL(k_group_sum10, dim3((unsigned)((10 * h->n_agrp + 255) / 256)), dim3(256), 0,
                         st, h->d_agrp_ptr, h->d_agrp_slot, h->n_agrp, S, N);
    hipLaunchKernelGGL(k_visc_boundary, dim3(2048), dim3(256), 0, st, h->d_flags, S, N, *law, k);
  }
  HHG_HIP(hipGetLastError());
  return HHG_OK;
}

}  // extern "C"
