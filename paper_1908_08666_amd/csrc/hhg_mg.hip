// Geometric multigrid on the hierarchy of uniform refinements (the paper's
// solver, Sec. 5 and 6): one library handle per level of the same macro mesh,
// P1 prolongation and its transpose between neighbouring levels, damped
// block-Jacobi smoothing with the scaled operator of every level (coefficient
// injected from the finest level), an exact solve on the coarsest level and
// CG preconditioned by one V-cycle.
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "hhg_device.h"

struct hhg_mg_s {
  std::vector<hhg_ctx *> lev;            // coarsest .. finest, owned
  int coarse_level = 0, fine_level = 0;
  int device = -1;
  int method = HHG_METHOD_SCALED;        // operator of the last coefficient setup
  const void *ready = nullptr;           // workspace of the last coefficient setup
  // restriction weights: 1 / (copies of the slot) at every level above the coarsest
  std::vector<double *> d_winv;          // [q], q >= 1
  // coarsest level: unknown nodes (owner slot, all copies)
  int n_cu = 0;
  std::vector<int64_t> cu_owner, cu_ptr, cu_slot;
  int64_t *d_cu_owner = nullptr, *d_cu_ptr = nullptr, *d_cu_slot = nullptr;
  // host copy of the coarsest operator's inverse is rebuilt per coefficient
  std::vector<double> dense;
  int smoother = HHG_PRECOND_BLOCK_JACOBI; // blocks of the smoother above the coarsest level
};

namespace hhg {

int apply_internal(hhg_ctx *h, int prec, int method, const void *f, const void *x, const void *k,
                   void *y, hipStream_t st);
int smooth_internal(hhg_ctx *h, int prec, int method, const void *f, const void *x, const void *k,
                    const void *P, double omega, void *r, void *xo, hipStream_t st);

namespace {

constexpr int MG_RED = 2048;             // blocks of the dot-product kernel (8 per CU)

dim3 grid1(int64_t n) { return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65535))); }

// (i, j, k) of the macro-local index q (slot order: planes k, rows s = i + j, i)
__device__ __forceinline__ void local_ijk(int64_t q, int n, int &i, int &j, int &k) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (plane_base(n, mid) <= q) lo = mid; else hi = mid - 1;
  }
  k = lo;
  const int p = (int)(q - plane_base(n, k));
  const int s = tri_root_dev(p);
  i = p - s * (s + 1) / 2;
  j = s - i;
}

__device__ __forceinline__ int64_t local_slot(int n, int i, int j, int k) {
  return plane_base(n, k) + (int64_t)(i + j) * (i + j + 1) / 2 + i;
}

// xf = P xc (or xf += P xc): a fine node that is a coarse node copies it, any
// other fine node is the midpoint of the coarse lattice edge (F - d)/2 --
// (F + d)/2, d the lattice direction with F's parity pattern.  Dirichlet
// slots stay zero.  Grid: (positions, macro).
template <bool ADD, typename T>
__global__ __launch_bounds__(256) void k_prolong(const MacroInfo *__restrict__ mc,
                                                 const MacroInfo *__restrict__ mf,
                                                 const uint8_t *__restrict__ flf,
                                                 const T *__restrict__ xc, T *__restrict__ xf,
                                                 int64_t Nc, int64_t Nf) {
  const int m = blockIdx.y;
  const int nf = mf[m].n, nc = mc[m].n;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= macro_nodes(nf)) return;
  const int64_t sf = mf[m].off + q;
  int I, J, K;
  local_ijk(q, nf, I, J, K);
  T v0 = T(0), v1 = T(0), v2 = T(0);
  if (!(flf[sf] & 1)) {
    const int pi = I & 1, pj = J & 1, pk = K & 1;
    const int64_t oc = mc[m].off;
    if (!(pi | pj | pk)) {
      const int64_t s = oc + local_slot(nc, I >> 1, J >> 1, K >> 1);
      v0 = xc[s];
      v1 = xc[Nc + s];
      v2 = xc[2 * Nc + s];
    } else {
      // lattice direction of the parity pattern: (1,0,0) (0,1,0) (0,0,1)
      // (1,-1,0) (1,0,-1) (0,1,-1) (1,-1,1)
      const int di = pi;
      const int dj = pj ? (pi ? -1 : 1) : 0;
      const int dk = pk ? ((pi ^ pj) ? -1 : 1) : 0;
      const int64_t sa = oc + local_slot(nc, (I - di) >> 1, (J - dj) >> 1, (K - dk) >> 1);
      const int64_t sb = oc + local_slot(nc, (I + di) >> 1, (J + dj) >> 1, (K + dk) >> 1);
      v0 = T(0.5) * (xc[sa] + xc[sb]);
      v1 = T(0.5) * (xc[Nc + sa] + xc[Nc + sb]);
      v2 = T(0.5) * (xc[2 * Nc + sa] + xc[2 * Nc + sb]);
    }
  }
  if (ADD) {
    xf[sf] += v0;
    xf[Nf + sf] += v1;
    xf[2 * Nf + sf] += v2;
  } else {
    xf[sf] = v0;
    xf[Nf + sf] = v1;
    xf[2 * Nf + sf] = v2;
  }
}

// Partial rc = P^T rf per coarse copy: the fine node at 2c with weight 1 and
// the fine midpoints 2c + d of the macro's coarse edges at c with weight 1/2,
// each divided by the number of copies of the fine node, so that the sum over
// the coarse copies (k_copy_sum3) counts every fine node once.  Dirichlet
// coarse slots get zero.
template <typename T>
__global__ __launch_bounds__(256) void k_restrict(const MacroInfo *__restrict__ mc,
                                                  const MacroInfo *__restrict__ mf,
                                                  const uint8_t *__restrict__ flc,
                                                  const double *__restrict__ winv,
                                                  const T *__restrict__ rf, T *__restrict__ rc,
                                                  int64_t Nc, int64_t Nf) {
  const int m = blockIdx.y;
  const int nf = mf[m].n, nc = mc[m].n;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= macro_nodes(nc)) return;
  const int64_t sc = mc[m].off + q;
  T s0 = T(0), s1 = T(0), s2 = T(0);
  if (!(flc[sc] & 1)) {
    int i, j, k;
    local_ijk(q, nc, i, j, k);
    const int64_t of = mf[m].off;
    {
      const int64_t s = of + local_slot(nf, 2 * i, 2 * j, 2 * k);
      const T w = (T)winv[s];
      s0 = w * rf[s];
      s1 = w * rf[Nf + s];
      s2 = w * rf[2 * Nf + s];
    }
#pragma unroll
    for (int d = 0; d < NDIR; ++d) {
      const int a = 2 * i + DIR_I[d], b = 2 * j + DIR_J[d], c = 2 * k + DIR_K[d];
      if (a < 0 || b < 0 || c < 0 || a + b + c > nf) continue;
      const int64_t s = of + local_slot(nf, a, b, c);
      const T w = (T)(0.5 * winv[s]);
      s0 = fma(w, rf[s], s0);
      s1 = fma(w, rf[Nf + s], s1);
      s2 = fma(w, rf[2 * Nf + s], s2);
    }
  }
  rc[sc] = s0;
  rc[Nc + sc] = s1;
  rc[2 * Nc + sc] = s2;
}

// Sum over the copies of every interface group, written to all copies.
template <typename T>
__global__ __launch_bounds__(256) void k_copy_sum3(const int64_t *__restrict__ ptr,
                                                   const int64_t *__restrict__ slots, int64_t ng,
                                                   T *__restrict__ v, int64_t N) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = ptr[g], b = ptr[g + 1];
    T s0 = T(0), s1 = T(0), s2 = T(0);
    for (int64_t q = a; q < b; ++q) {
      const int64_t s = slots[q];
      s0 += v[s];
      s1 += v[N + s];
      s2 += v[2 * N + s];
    }
    for (int64_t q = a; q < b; ++q) {
      const int64_t s = slots[q];
      v[s] = s0;
      v[N + s] = s1;
      v[2 * N + s] = s2;
    }
  }
}

// kc = fine coefficient at the coarse nodes (fine node 2c of the same macro)
__global__ __launch_bounds__(256) void k_inject(const MacroInfo *__restrict__ mc,
                                                const MacroInfo *__restrict__ mf,
                                                const double *__restrict__ kf, double *__restrict__ kc) {
  const int m = blockIdx.y;
  const int nc = mc[m].n, nf = mf[m].n;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= macro_nodes(nc)) return;
  int i, j, k;
  local_ijk(q, nc, i, j, k);
  kc[mc[m].off + q] = kf[mf[m].off + local_slot(nf, 2 * i, 2 * j, 2 * k)];
}

// x = omega P r (FIRST) or x += omega P r, P the inverse diagonal blocks
// (xx yy zz xy xz yz, zero at Dirichlet slots)
template <bool FIRST, typename T>
__global__ __launch_bounds__(256) void k_jacobi(const T *__restrict__ P, const T *__restrict__ r,
                                                T *__restrict__ x, T omega, int64_t N) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N;
       s += (int64_t)gridDim.x * blockDim.x) {
    const T r0 = r[s], r1 = r[N + s], r2 = r[2 * N + s];
    const T Pxx = P[s], Pyy = P[N + s], Pzz = P[2 * N + s];
    const T Pxy = P[3 * N + s], Pxz = P[4 * N + s], Pyz = P[5 * N + s];
    const T z0 = omega * (Pxx * r0 + Pxy * r1 + Pxz * r2);
    const T z1 = omega * (Pxy * r0 + Pyy * r1 + Pyz * r2);
    const T z2 = omega * (Pxz * r0 + Pyz * r1 + Pzz * r2);
    if (FIRST) {
      x[s] = z0;
      x[N + s] = z1;
      x[2 * N + s] = z2;
    } else {
      x[s] += z0;
      x[N + s] += z1;
      x[2 * N + s] += z2;
    }
  }
}

template <typename T>
__global__ void k_fill0(T *__restrict__ a, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    a[s] = T(0);
}

// b = a converted to the other precision
template <typename A, typename B>
__global__ void k_cast(const A *__restrict__ a, B *__restrict__ b, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    b[s] = (B)a[s];
}

// unit vector of unknown coarse DoF (u, c) at every copy of node u
__global__ void k_unit(const int64_t *__restrict__ ptr, const int64_t *__restrict__ slots, int u,
                       int c, double *__restrict__ e, int64_t N) {
  for (int64_t q = ptr[u] + threadIdx.x; q < ptr[u + 1]; q += blockDim.x) e[c * N + slots[q]] = 1.0;
}

// column col of the dense coarse operator: y at the owners of all unknown nodes
__global__ void k_column(const int64_t *__restrict__ owner, int nu, const double *__restrict__ y,
                         int64_t N, double *__restrict__ A, int col) {
  const int n3 = 3 * nu;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n3; r += gridDim.x * blockDim.x)
    A[(int64_t)col * n3 + r] = y[(r % 3) * N + owner[r / 3]];
}

constexpr int MG_MAX_CU = 512;           // unknown nodes of the coarsest level, at most

// x = A^{-1} b on the coarsest level: gather b at the owners into LDS, dense
// product with the inverse (column-major: entry (r, c) at c n3 + r), scatter
// to every copy.  One thread per row; the grid covers the 3 nu rows once.
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_solve(const int64_t *__restrict__ owner,
                                                      const int64_t *__restrict__ ptr,
                                                      const int64_t *__restrict__ slots, int nu,
                                                      const double *__restrict__ Ainv,
                                                      const T *__restrict__ b,
                                                      T *__restrict__ x, int64_t N) {
  __shared__ double bl[3 * MG_MAX_CU];
  const int n3 = 3 * nu;
  for (int c = threadIdx.x; c < n3; c += blockDim.x) bl[c] = (double)b[(c % 3) * N + owner[c / 3]];
  __syncthreads();
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n3) return;
  double s = 0.0;
  // the column loads are independent of the sum: unrolled, they are in
  // flight together instead of one memory latency per column
#pragma unroll 8
  for (int c = 0; c < n3; ++c) s = fma(Ainv[(int64_t)c * n3 + r], bl[c], s);
  const int u = r / 3, comp = r % 3;
  for (int64_t q = ptr[u]; q < ptr[u + 1]; ++q) x[comp * N + slots[q]] = (T)s;
}

// partial sums of (a, b) over unknown owner slots
__global__ __launch_bounds__(256) void k_dot(const double *__restrict__ a, const double *__restrict__ b,
                                             const uint8_t *__restrict__ fl, int64_t N,
                                             double *__restrict__ part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x)
    if ((fl[i] & 3) == 2) s += a[i] * b[i] + a[N + i] * b[N + i] + a[2 * N + i] * b[2 * N + i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// x += alpha p, r -= alpha q
__global__ void k_axpy2(double *__restrict__ x, const double *__restrict__ p, double *__restrict__ r,
                        const double *__restrict__ q, double alpha, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    x[s] = fma(alpha, p[s], x[s]);
    r[s] = fma(-alpha, q[s], r[s]);
  }
}

// p = z + beta p
__global__ void k_xpby(double *__restrict__ p, const double *__restrict__ z, double beta, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    p[s] = fma(beta, p[s], z[s]);
}

// ----------------------------------------------------------- workspace
struct MgWork {
  std::vector<double *> k, P, b, x, r, xs;   // per level (xs: second iterate of the smoother)
  std::vector<float *> k32, P32, b32, x32, r32, xs32;   // per level, for FP32 cycles
  double *Ainv = nullptr;                // (3 n_cu)^2, inverse of the coarsest operator
  double *pr = nullptr, *pz = nullptr, *pp = nullptr, *pq = nullptr;   // CG vectors (finest)
  double *part = nullptr;                // MG_RED partial sums
};

// the per-level arrays of one precision
template <typename T>
struct LevelArrays {
  const T *k, *P;
  T *b, *x, *r, *xs;
};
template <typename T>
LevelArrays<T> level_arrays(const MgWork &W, int q);
template <>
LevelArrays<double> level_arrays<double>(const MgWork &W, int q) {
  return {W.k[q], W.P[q], W.b[q], W.x[q], W.r[q], W.xs[q]};
}
template <>
LevelArrays<float> level_arrays<float>(const MgWork &W, int q) {
  return {W.k32[q], W.P32[q], W.b32[q], W.x32[q], W.r32[q], W.xs32[q]};
}
template <typename T>
constexpr int prec_of() {
  return sizeof(T) == 8 ? HHG_F64 : HHG_F32;
}

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t layout(const hhg_mg_s *mg, char *base, MgWork *w) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    double *p = base ? reinterpret_cast<double *>(base + off) : nullptr;
    off += al256(bytes);
    return p;
  };
  auto take32 = [&](size_t bytes) {
    float *p = base ? reinterpret_cast<float *>(base + off) : nullptr;
    off += al256(bytes);
    return p;
  };
  const int L = (int)mg->lev.size();
  MgWork tmp;
  MgWork &W = w ? *w : tmp;
  W.k.assign(L, nullptr);
  W.P.assign(L, nullptr);
  W.b.assign(L, nullptr);
  W.x.assign(L, nullptr);
  W.r.assign(L, nullptr);
  W.xs.assign(L, nullptr);
  W.k32.assign(L, nullptr);
  W.P32.assign(L, nullptr);
  W.b32.assign(L, nullptr);
  W.x32.assign(L, nullptr);
  W.r32.assign(L, nullptr);
  W.xs32.assign(L, nullptr);
  for (int q = 0; q < L; ++q) {
    const size_t N = (size_t)mg->lev[q]->n_nodes;
    W.k[q] = take(8 * N);
    W.P[q] = take(48 * N);
    W.b[q] = take(24 * N);
    W.x[q] = take(24 * N);
    W.r[q] = take(24 * N);
    W.xs[q] = take(24 * N);
    W.k32[q] = take32(4 * N);
    W.P32[q] = take32(24 * N);
    W.b32[q] = take32(12 * N);
    W.x32[q] = take32(12 * N);
    W.r32[q] = take32(12 * N);
    W.xs32[q] = take32(12 * N);
  }
  const size_t n3 = 3 * (size_t)mg->n_cu;
  W.Ainv = take(8 * n3 * n3);
  const size_t NF = (size_t)mg->lev.back()->n_nodes;
  W.pr = take(24 * NF);
  W.pz = take(24 * NF);
  W.pp = take(24 * NF);
  W.pq = take(24 * NF);
  W.part = take(8 * MG_RED);
  return off;
}

int check_mg(const hhg_mg_s *mg) {
  if (!mg || mg->lev.empty()) return fail(HHG_EINVAL, "null multigrid handle");
  int dev = -1;
  HHG_HIP(hipGetDevice(&dev));
  if (mg->device >= 0 && dev != mg->device)
    return fail(HHG_EINVAL, "multigrid handle used on another device than the one it was set up on");
  return HHG_OK;
}

// device copies of the level metadata (first device call)
int mg_device(hhg_mg_s *mg) {
  for (hhg_ctx *h : mg->lev) {
    const int rc = ensure_device(h);
    if (rc) return rc;
  }
  if (mg->device >= 0) return HHG_OK;
  HHG_HIP(hipGetDevice(&mg->device));
  for (size_t q = 1; q < mg->lev.size(); ++q) {
    hhg_ctx *h = mg->lev[q];
    std::vector<double> w((size_t)h->n_nodes, 1.0);
    for (size_t g = 0; g + 1 < h->agrp_ptr.size(); ++g) {
      const int64_t a = h->agrp_ptr[g], b = h->agrp_ptr[g + 1];
      for (int64_t s = a; s < b; ++s) w[h->agrp_slot[s]] = 1.0 / (double)(b - a);
    }
    double *d = nullptr;
    HHG_HIP(hipMalloc((void **)&d, w.size() * sizeof(double)));
    mg->d_winv[q] = d;
    HHG_HIP(hipMemcpy(d, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  auto up = [](int64_t **dst, const std::vector<int64_t> &v) -> int {
    HHG_HIP(hipMalloc((void **)dst, std::max<size_t>(1, v.size()) * sizeof(int64_t)));
    if (!v.empty()) HHG_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    return HHG_OK;
  };
  int rc;
  if ((rc = up(&mg->d_cu_owner, mg->cu_owner))) return rc;
  if ((rc = up(&mg->d_cu_ptr, mg->cu_ptr))) return rc;
  if ((rc = up(&mg->d_cu_slot, mg->cu_slot))) return rc;
  return HHG_OK;
}

dim3 macro_grid(const hhg_ctx *h) {
  int maxn = 0;
  for (const auto &mi : h->minfo) maxn = std::max<int>(maxn, (int)macro_nodes(mi.n));
  return dim3((unsigned)((maxn + 255) / 256), (unsigned)h->n_macro);
}

template <typename T>
int prolong(hhg_mg_s *mg, int q, const T *xc, T *xf, bool add, hipStream_t st) {
  hhg_ctx *c = mg->lev[q - 1], *f = mg->lev[q];
  if (add)
    hipLaunchKernelGGL((k_prolong<true, T>), macro_grid(f), dim3(256), 0, st, c->d_minfo, f->d_minfo,
                       f->d_flags, xc, xf, c->n_nodes, f->n_nodes);
  else
    hipLaunchKernelGGL((k_prolong<false, T>), macro_grid(f), dim3(256), 0, st, c->d_minfo, f->d_minfo,
                       f->d_flags, xc, xf, c->n_nodes, f->n_nodes);
  HHG_HIP(hipGetLastError());
  return HHG_OK;
}

template <typename T>
int restrict_(hhg_mg_s *mg, int q, const T *rf, T *rc, hipStream_t st) {
  hhg_ctx *c = mg->lev[q - 1], *f = mg->lev[q];
  hipLaunchKernelGGL(k_restrict<T>, macro_grid(c), dim3(256), 0, st, c->d_minfo, f->d_minfo, c->d_flags,
                     mg->d_winv[q], rf, rc, c->n_nodes, f->n_nodes);
  HHG_HIP(hipGetLastError());
  if (c->n_grp > 0) {
    hipLaunchKernelGGL(k_copy_sum3<T>, grid1(c->n_grp), dim3(256), 0, st, c->d_grp_ptr,
                       c->d_grp_slot, c->n_grp, rc, c->n_nodes);
    HHG_HIP(hipGetLastError());
  }
  return HHG_OK;
}

// x_q = V-cycle applied to b_q (levels q and below), in the precision T
// (operator, smoother and transfers in T; the coarse inverse is FP64).
// Level q of the finest F smooths nu1 + nu_inc (F - q) times before and
// nu2 + nu_inc (F - q) times after the coarse correction (Sec. 5.2.1: the
// variable V-cycle adds two steps per coarser level).
template <typename T>
int vcycle(hhg_mg_s *mg, const MgWork &W, const hhg_mg_opts &o, int q, const T *b, T *x,
           hipStream_t st) {
  hhg_ctx *h = mg->lev[q];
  const int64_t N = h->n_nodes;
  if (q == 0) {
    hipLaunchKernelGGL(k_fill0<T>, grid1(3 * N), dim3(256), 0, st, x, 3 * N);
    if (mg->n_cu > 0)
      hipLaunchKernelGGL(k_coarse_solve<T>, grid1(3 * mg->n_cu), dim3(256), 0, st, mg->d_cu_owner,
                         mg->d_cu_ptr, mg->d_cu_slot, mg->n_cu, W.Ainv, b, x, N);
    HHG_HIP(hipGetLastError());
    return HHG_OK;
  }
  int rc;
  const int extra = o.nu_inc * ((int)mg->lev.size() - 1 - q);
  const int nu1 = o.nu1 + extra, nu2 = o.nu2 + extra;
  const LevelArrays<T> A = level_arrays<T>(W, q), C = level_arrays<T>(W, q - 1);
  T *r = A.r;
  const T omega = (T)o.omega;
  // Every smoothing step after the first writes the other of two iterates
  // (x and the level's spare xs); start in the one that makes the last step
  // land in x.
  const int steps = (nu1 > 0 ? nu1 - 1 : 0) + nu2;
  T *cur = (steps % 2 == 0) ? x : A.xs, *oth = (steps % 2 == 0) ? A.xs : x;
  auto smooth = [&](bool first) -> int {
    if (first) {
      hipLaunchKernelGGL((k_jacobi<true, T>), grid1(N), dim3(256), 0, st, A.P, b, cur, omega, N);
      HHG_HIP(hipGetLastError());
      return HHG_OK;
    }
    const int rc2 = smooth_internal(h, prec_of<T>(), mg->method, b, cur, A.k, A.P, (double)omega, r,
                                    oth, st);
    std::swap(cur, oth);
    return rc2;
  };
  for (int s = 0; s < nu1; ++s)
    if ((rc = smooth(s == 0))) return rc;
  if (nu1 == 0) hipLaunchKernelGGL(k_fill0<T>, grid1(3 * N), dim3(256), 0, st, cur, 3 * N);
  if ((rc = apply_internal(h, prec_of<T>(), mg->method, b, cur, A.k, r, st))) return rc;
  if ((rc = restrict_<T>(mg, q, r, C.b, st))) return rc;
  if ((rc = vcycle<T>(mg, W, o, q - 1, C.b, C.x, st))) return rc;
  if ((rc = prolong<T>(mg, q, C.x, cur, true, st))) return rc;
  for (int s = 0; s < nu2; ++s)
    if ((rc = smooth(false))) return rc;
  return HHG_OK;
}

// z = V(r) on the finest level in the precision the options select: an FP32
// cycle runs on FP32 copies of r and z
int finest_cycle(hhg_mg_s *mg, const MgWork &W, const hhg_mg_opts &o, const double *r, double *z,
                 hipStream_t st) {
  const int F = (int)mg->lev.size() - 1;
  if (o.precision == HHG_F64) return vcycle<double>(mg, W, o, F, r, z, st);
  const int64_t n3 = 3 * mg->lev[F]->n_nodes;
  hipLaunchKernelGGL((k_cast<double, float>), grid1(n3), dim3(256), 0, st, r, W.b32[F], n3);
  HHG_HIP(hipGetLastError());
  const int rc = vcycle<float>(mg, W, o, F, W.b32[F], W.x32[F], st);
  if (rc) return rc;
  hipLaunchKernelGGL((k_cast<float, double>), grid1(n3), dim3(256), 0, st, W.x32[F], z, n3);
  HHG_HIP(hipGetLastError());
  return HHG_OK;
}

int dot(hhg_mg_s *mg, const MgWork &W, const double *a, const double *b, double *out,
        hipStream_t st) {
  hhg_ctx *h = mg->lev.back();
  hipLaunchKernelGGL(k_dot, dim3(MG_RED), dim3(256), 0, st, a, b, h->d_flags, h->n_nodes, W.part);
  HHG_HIP(hipGetLastError());
  double part[MG_RED];
  HHG_HIP(hipMemcpyAsync(part, W.part, sizeof(part), hipMemcpyDeviceToHost, st));
  HHG_HIP(hipStreamSynchronize(st));
  double s = 0.0;
  for (int q = 0; q < MG_RED; ++q) s += part[q];
  *out = s;
  return HHG_OK;
}

// Inverse of a dense matrix (column-major, n x n) in place by LU with
// partial pivoting; false if a pivot vanishes.  The coarsest operator is
// symmetric only under the symmetric interface rule.
bool dense_inverse(std::vector<double> &A, int n) {
  std::vector<double> LU(A);
  std::vector<int> piv(n);
  auto at = [&](int r, int c) -> double & { return LU[(size_t)c * n + r]; };
  double amax = 0.0;
  for (double v : A) amax = std::max(amax, std::fabs(v));
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(at(r, c)) > std::fabs(at(p, c))) p = r;
    if (!(std::fabs(at(p, c)) > 1e-14 * amax)) return false;
    piv[c] = p;
    if (p != c)
      for (int q = 0; q < n; ++q) std::swap(at(c, q), at(p, q));
    const double d = at(c, c);
    for (int r = c + 1; r < n; ++r) {
      const double l = at(r, c) / d;
      at(r, c) = l;
      if (l != 0.0)
        for (int q = c + 1; q < n; ++q) at(r, q) -= l * at(c, q);
    }
  }
  // solve LU x = P e_c column by column
  std::vector<double> y(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) y[i] = i == c ? 1.0 : 0.0;
    for (int i = 0; i < n; ++i) std::swap(y[i], y[piv[i]]);
    for (int i = 0; i < n; ++i) {
      double s = y[i];
      for (int q = 0; q < i; ++q) s -= at(i, q) * y[q];
      y[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = y[i];
      for (int q = i + 1; q < n; ++q) s -= at(i, q) * y[q];
      y[i] = s / at(i, i);
    }
    for (int i = 0; i < n; ++i) A[(size_t)c * n + i] = y[i];
  }
  return true;
}

int check_opts(const hhg_mg_opts *o) {
  if (!o) return fail(HHG_EINVAL, "null options");
  if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 < 1 || o->nu1 > 64 || o->nu2 > 64)
    return fail(HHG_EINVAL, "smoothing steps must be 0..64 each, at least one in total");
  if (!(o->omega > 0.0 && o->omega < 2.0)) return fail(HHG_EINVAL, "omega must lie in (0, 2)");
  if (o->nu_inc < 0 || o->nu_inc > 8) return fail(HHG_EINVAL, "nu_inc must be 0..8");
  if (o->method != HHG_MG_CG && o->method != HHG_MG_CYCLE)
    return fail(HHG_EINVAL, "unknown multigrid solve method");
  if (o->precision != HHG_F64 && o->precision != HHG_F32)
    return fail(HHG_EINVAL, "cycle precision must be HHG_F64 or HHG_F32");
  return HHG_OK;
}


// ------------------------------------------------ generalized Stokes (Sec. 5.2)
// The divergence pair B, B^T, the stabilization c_l(p, q) = -h^2/12 (grad p,
// grad q) and the lumped pressure mass of eqn. generalizedstokes, equal-order
// P1 velocity and pressure.  Every term is a sum over the elements at a node:
// on element t with volume |t| and constant gradients g_a of its vertices a,
// int psi = |t| / 4, so
//   (B u)_i       = -sum_t |t|/4 sum_a g_a . u_a
//   (B^T p)_{i,l} = -sum_t |t|/4 (g_i)_l sum_a p_a
//   (C p)_i       = -h^2/12 sum_t |t| sum_a (g_i . g_a) p_a
//   mass_i        =  sum_t |t| / 4,   C_ii = -h^2/12 sum_t |t| g_i . g_i.
// One thread per slot sums over the node's elements inside its macro (all
// 24 for a macro-interior node); the copy groups then add the other macros'
// shares.  Velocity entries of Dirichlet nodes are read as zero and B^T rows
// of Dirichlet nodes are zero, as for the velocity operator.
enum { SK_DIV = 0, SK_GRAD = 1, SK_STAB = 2, SK_MASS = 3, SK_CDIAG = 4 };

template <int MODE>
__global__ __launch_bounds__(256) void k_stokes_rows(const MacroInfo *__restrict__ minfo,
                                                     const StrainConst *__restrict__ stc,
                                                     const uint8_t *__restrict__ fl,
                                                     const double *__restrict__ in,
                                                     double *__restrict__ out, int64_t N, double cst) {
  const int m = blockIdx.y;
  const MacroInfo mi = minfo[m];
  const int n = mi.n;
  const int64_t ls = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ls >= macro_nodes(n)) return;
  int i, j, k;
  local_ijk(ls, n, i, j, k);
  const int64_t slot = mi.off + ls;
  const StrainConst &sc = stc[m];
  int64_t nb[NDIR];
  bool inb[NDIR];
#pragma unroll
  for (int d = 0; d < NDIR; ++d) {
    const int a = i + DIR_I[d], b = j + DIR_J[d], c = k + DIR_K[d];
    inb[d] = a >= 0 && b >= 0 && c >= 0 && a + b + c <= n;
    nb[d] = inb[d] ? mi.off + local_slot(n, a, b, c) : slot;
  }
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
  for (int t = 0; t < NTET; ++t) {
    const int v1 = TET_V[t][0], v2 = TET_V[t][1], v3 = TET_V[t][2];
    if (!(inb[v1] && inb[v2] && inb[v3])) continue;
    const int64_t vs[4] = {slot, nb[v1], nb[v2], nb[v3]};
    if constexpr (MODE == SK_DIV) {
      double s = 0.0;
      for (int a = 0; a < 4; ++a) {
        if (fl[vs[a]] & 1) continue;
        for (int c = 0; c < 3; ++c) s += sc.grad[t][a][c] * in[c * N + vs[a]];
      }
      acc0 -= 0.25 * sc.vol * s;
    } else if constexpr (MODE == SK_GRAD) {
      const double ps = in[vs[0]] + in[vs[1]] + in[vs[2]] + in[vs[3]];
      acc0 -= 0.25 * sc.vol * sc.grad[t][0][0] * ps;
      acc1 -= 0.25 * sc.vol * sc.grad[t][0][1] * ps;
      acc2 -= 0.25 * sc.vol * sc.grad[t][0][2] * ps;
    } else if constexpr (MODE == SK_STAB) {
      double s = 0.0;
      for (int a = 0; a < 4; ++a) {
        const double gg = sc.grad[t][0][0] * sc.grad[t][a][0] + sc.grad[t][0][1] * sc.grad[t][a][1] +
                          sc.grad[t][0][2] * sc.grad[t][a][2];
        s += gg * in[vs[a]];
      }
      acc0 += cst * sc.vol * s;
    } else if constexpr (MODE == SK_CDIAG) {
      acc0 += cst * sc.vol * (sc.grad[t][0][0] * sc.grad[t][0][0] + sc.grad[t][0][1] * sc.grad[t][0][1] +
                              sc.grad[t][0][2] * sc.grad[t][0][2]);
    } else {
      acc0 += 0.25 * sc.vol;
    }
  }
  if constexpr (MODE == SK_GRAD) {
    const bool dz = fl[slot] & 1;
    out[slot] = dz ? 0.0 : acc0;
    out[N + slot] = dz ? 0.0 : acc1;
    out[2 * N + slot] = dz ? 0.0 : acc2;
  } else {
    out[slot] = acc0;
  }
}

// scalar sum over the copies of every group, written to all copies
__global__ __launch_bounds__(256) void k_copy_sum1(const int64_t *__restrict__ ptr,
                                                   const int64_t *__restrict__ slots, int64_t ng,
                                                   double *__restrict__ v) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < ng;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = ptr[g], b = ptr[g + 1];
    double s = 0.0;
    for (int64_t q = a; q < b; ++q) s += v[slots[q]];
    for (int64_t q = a; q < b; ++q) v[slots[q]] = s;
  }
}

// partial sums of (a, b) over owner slots of scalar fields (pressure: every
// node); b null reads as ones
__global__ __launch_bounds__(256) void k_dot_owner(const double *__restrict__ a,
                                                   const double *__restrict__ b,
                                                   const uint8_t *__restrict__ fl, int64_t N,
                                                   double *__restrict__ part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x)
    if (fl[i] & 2) s += a[i] * (b ? b[i] : 1.0);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// per block: max over unknown owner nodes of |u_i - v_i| and of |u_i| (2-norms)
__global__ __launch_bounds__(256) void k_node_max2(const double *__restrict__ u,
                                                   const double *__restrict__ v,
                                                   const uint8_t *__restrict__ fl, int64_t N,
                                                   double *__restrict__ part) {
  __shared__ double sh[8];
  double dm = 0.0, um = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x)
    if ((fl[i] & 3) == 2) {
      const double d0 = u[i] - v[i], d1 = u[N + i] - v[N + i], d2 = u[2 * N + i] - v[2 * N + i];
      dm = fmax(dm, sqrt(d0 * d0 + d1 * d1 + d2 * d2));
      um = fmax(um, sqrt(u[i] * u[i] + u[N + i] * u[N + i] + u[2 * N + i] * u[2 * N + i]));
    }
  for (int off = 32; off > 0; off >>= 1) {
    dm = fmax(dm, __shfl_down(dm, off, 64));
    um = fmax(um, __shfl_down(um, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6] = dm;
    sh[4 + (threadIdx.x >> 6)] = um;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    part[2 * blockIdx.x + 1] = fmax(fmax(sh[4], sh[5]), fmax(sh[6], sh[7]));
  }
}

// p += omega_p (B u + C p - g) / S;  rp = B u + C p - g kept for the caller
__global__ void k_pressure_step(double *__restrict__ p, const double *__restrict__ rp,
                                const double *__restrict__ S, double omega_p, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    p[s] += omega_p * rp[s] / S[s];
}

// a += c b (n entries)
__global__ void k_axpy(double *__restrict__ a, const double *__restrict__ b, double c, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    a[s] = fma(c, b[s], a[s]);
}

// out = a + b - c (n entries; b or c may be null)
__global__ void k_add3(double *__restrict__ out, const double *__restrict__ a, const double *__restrict__ b,
                       const double *__restrict__ c, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    out[s] = a[s] + (b ? b[s] : 0.0) - (c ? c[s] : 0.0);
}

// S = mass / mu - diag(C): diagonal approximation of the pressure Schur
// complement B A(mu)^-1 B^T - C
__global__ void k_schur(double *__restrict__ S, const double *__restrict__ mass,
                        const double *__restrict__ mu, const double *__restrict__ cdiag, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    S[s] = mass[s] / mu[s] - cdiag[s];
}

int stokes_rows(hhg_ctx *h, int op, double hl, const double *in, double *out, hipStream_t st) {
  const double cst = -hl * hl / 12.0;
  const dim3 g = macro_grid(h);
  switch (op) {
    case SK_DIV:
      hipLaunchKernelGGL(k_stokes_rows<SK_DIV>, g, dim3(256), 0, st, h->d_minfo, h->d_stc, h->d_flags,
                         in, out, h->n_nodes, cst);
      break;
    case SK_GRAD:
      hipLaunchKernelGGL(k_stokes_rows<SK_GRAD>, g, dim3(256), 0, st, h->d_minfo, h->d_stc, h->d_flags,
                         in, out, h->n_nodes, cst);
      break;
    case SK_STAB:
      hipLaunchKernelGGL(k_stokes_rows<SK_STAB>, g, dim3(256), 0, st, h->d_minfo, h->d_stc,
                         h->d_flags, in, out, h->n_nodes, cst);
      break;
    case SK_CDIAG:
      hipLaunchKernelGGL(k_stokes_rows<SK_CDIAG>, g, dim3(256), 0, st, h->d_minfo, h->d_stc,
                         h->d_flags, in, out, h->n_nodes, cst);
      break;
    default:
      hipLaunchKernelGGL(k_stokes_rows<SK_MASS>, g, dim3(256), 0, st, h->d_minfo, h->d_stc,
                         h->d_flags, in, out, h->n_nodes, cst);
  }
  HHG_HIP(hipGetLastError());
  if (h->n_agrp > 0) {
    if (op == SK_GRAD)
      hipLaunchKernelGGL(k_copy_sum3<double>, grid1(h->n_agrp), dim3(256), 0, st, h->d_agrp_ptr,
                         h->d_agrp_slot, h->n_agrp, out, h->n_nodes);
    else
      hipLaunchKernelGGL(k_copy_sum1, grid1(h->n_agrp), dim3(256), 0, st, h->d_agrp_ptr,
                         h->d_agrp_slot, h->n_agrp, out);
    HHG_HIP(hipGetLastError());
  }
  return HHG_OK;
}

// Stokes workspace: vectors on the finest level
struct StokesWork {
  double *ru, *z, *gp, *rp, *bu, *S, *mass, *cdiag, *uprev, *visc, *part;
};
size_t stokes_layout(const hhg_ctx *h, char *base, StokesWork *w) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    double *p = base ? reinterpret_cast<double *>(base + off) : nullptr;
    off += al256(bytes);
    return p;
  };
  const size_t N = (size_t)h->n_nodes;
  StokesWork tmp;
  StokesWork &W = w ? *w : tmp;
  W.ru = take(24 * N);
  W.z = take(24 * N);
  W.gp = take(24 * N);
  W.rp = take(8 * N);
  W.bu = take(8 * N);
  W.S = take(8 * N);
  W.mass = take(8 * N);
  W.cdiag = take(8 * N);
  W.uprev = take(24 * N);
  W.visc = take(80 * N);
  W.part = take(16 * MG_RED);
  return off;
}

double host_sum(const double *part, int n, int stride = 1, int at = 0) {
  double s = 0.0;
  for (int q = 0; q < n; ++q) s += part[stride * q + at];
  return s;
}

// sum over owner slots of a b (scalar fields), synchronous
int dot_owner(hhg_ctx *h, const double *a, const double *b, double *part, hipStream_t st, double &out) {
  hipLaunchKernelGGL(k_dot_owner, dim3(MG_RED), dim3(256), 0, st, a, b, h->d_flags, h->n_nodes, part);
  HHG_HIP(hipGetLastError());
  std::vector<double> hp(MG_RED);
  HHG_HIP(hipMemcpyAsync(hp.data(), part, MG_RED * sizeof(double), hipMemcpyDeviceToHost, st));
  HHG_HIP(hipStreamSynchronize(st));
  out = host_sum(hp.data(), MG_RED);
  return HHG_OK;
}

// sum over unknown owner slots of a . b (velocity fields), synchronous
int dot_vel(hhg_ctx *h, const double *a, const double *b, double *part, hipStream_t st, double &out) {
  hipLaunchKernelGGL(k_dot, dim3(MG_RED), dim3(256), 0, st, a, b, h->d_flags, h->n_nodes, part);
  HHG_HIP(hipGetLastError());
  std::vector<double> hp(MG_RED);
  HHG_HIP(hipMemcpyAsync(hp.data(), part, MG_RED * sizeof(double), hipMemcpyDeviceToHost, st));
  HHG_HIP(hipStreamSynchronize(st));
  out = host_sum(hp.data(), MG_RED);
  return HHG_OK;
}

// a += c (n entries)
__global__ void k_add_const(double *__restrict__ a, double c, int64_t n) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    a[s] += c;
}

// Inexact Uzawa iteration on the finest level (see hhg_mg_stokes_solve):
//   u <- u + V(f - A u - B^T p)
//   p <- p + omega_p (B u + C p - g) / S,  S = mass / mu
//   p <- p - (mass . p) / (mass . 1)
// until the residual 2-norm of both blocks is <= tol_abs or maxit steps.
// On return S.ru and S.rp hold the residuals of the final iterate.
int uzawa(hhg_mg_s *mg, const MgWork &W, const StokesWork &S, const hhg_stokes_opts &o, double hl,
          const double *f, const double *g, double *u, double *p, int maxit, double tol_abs,
          hipStream_t st, int &iters, double &res) {
  const int F = (int)mg->lev.size() - 1;
  hhg_ctx *h = mg->lev[F];
  const int64_t N = h->n_nodes;
  hhg_mg_opts mo{};
  mo.nu1 = o.nu1;
  mo.nu2 = o.nu2;
  mo.nu_inc = o.nu_inc;
  mo.omega = o.omega;
  mo.method = HHG_MG_CYCLE;
  mo.precision = HHG_F64;
  int rc;
  double mtot = 0.0;
  if ((rc = dot_owner(h, S.mass, nullptr, S.part, st, mtot))) return rc;
  auto residuals = [&]() -> int {
    int r2 = stokes_rows(h, SK_GRAD, hl, p, S.gp, st);
    if (r2) return r2;
    if ((r2 = apply_internal(h, HHG_F64, mg->method, f, u, W.k[F], S.ru, st))) return r2;  // f - A u
    hipLaunchKernelGGL(k_axpy, grid1(3 * N), dim3(256), 0, st, S.ru, S.gp, -1.0, 3 * N);
    if ((r2 = stokes_rows(h, SK_DIV, hl, u, S.bu, st))) return r2;
    if ((r2 = stokes_rows(h, SK_STAB, hl, p, S.rp, st))) return r2;
    hipLaunchKernelGGL(k_add3, grid1(N), dim3(256), 0, st, S.rp, S.rp, S.bu, g, N);  // B u + C p - g
    HHG_HIP(hipGetLastError());
    double a = 0.0, b = 0.0;
    if ((r2 = dot_vel(h, S.ru, S.ru, S.part, st, a))) return r2;
    if ((r2 = dot_owner(h, S.rp, S.rp, S.part, st, b))) return r2;
    res = std::sqrt(a + b);
    return HHG_OK;
  };
  if ((rc = residuals())) return rc;
  iters = 0;
  while (iters < maxit && !(res <= tol_abs)) {
    if (!std::isfinite(res)) return fail(HHG_EBREAKDOWN, "non-finite Uzawa residual");
    ++iters;
    if ((rc = finest_cycle(mg, W, mo, S.ru, S.z, st))) return rc;     // z = V(f - A u - B^T p)
    hipLaunchKernelGGL(k_axpy, grid1(3 * N), dim3(256), 0, st, u, S.z, 1.0, 3 * N);
    if ((rc = stokes_rows(h, SK_DIV, hl, u, S.bu, st))) return rc;
    if ((rc = stokes_rows(h, SK_STAB, hl, p, S.rp, st))) return rc;
    hipLaunchKernelGGL(k_add3, grid1(N), dim3(256), 0, st, S.rp, S.rp, S.bu, g, N);
    hipLaunchKernelGGL(k_pressure_step, grid1(N), dim3(256), 0, st, p, S.rp, S.S, o.omega_p, N);
    HHG_HIP(hipGetLastError());
    double mp = 0.0;
    if ((rc = dot_owner(h, S.mass, p, S.part, st, mp))) return rc;
    hipLaunchKernelGGL(k_add_const, grid1(N), dim3(256), 0, st, p, -mp / mtot, N);
    HHG_HIP(hipGetLastError());
    if ((rc = residuals())) return rc;
  }
  if (!std::isfinite(res)) return fail(HHG_EBREAKDOWN, "non-finite Uzawa residual");
  return HHG_OK;
}

}  // namespace
}  // namespace hhg

using namespace hhg;

extern "C" {

int hhg_mg_create(const hhg_mesh_desc *mesh, const hhg_op_desc *op, int32_t coarse_level,
                  hhg_mg *out) {
  if (!mesh || !op || !out || !mesh->level || mesh->n_macro < 1)
    return fail(HHG_EINVAL, "null argument");
  *out = nullptr;
  if (mesh->coupling != HHG_CONFORMING) return fail(HHG_EINVAL, "multigrid needs a conforming mesh");
  const int L = mesh->level[0];
  for (int m = 1; m < mesh->n_macro; ++m)
    if (mesh->level[m] != L) return fail(HHG_EINVAL, "multigrid needs one common level");
  if (coarse_level < 2 || coarse_level > L) return fail(HHG_EINVAL, "coarse level must lie in 2..level");
  auto *mg = new hhg_mg_s();
  mg->coarse_level = coarse_level;
  mg->fine_level = L;
  std::vector<int32_t> lv((size_t)mesh->n_macro);
  for (int l = coarse_level; l <= L; ++l) {
    for (auto &v : lv) v = l;
    hhg_mesh_desc d = *mesh;
    d.level = lv.data();
    hhg_handle h = nullptr;
    const int rc = hhg_setup_macro(&d, op, &h);
    if (rc) {
      hhg_mg_destroy(mg);
      return rc;
    }
    mg->lev.push_back(h);
  }
  mg->d_winv.assign(mg->lev.size(), nullptr);
  // unknown nodes of the coarsest level with all their copies
  hhg_ctx *c = mg->lev[0];
  std::vector<int64_t> gid((size_t)c->n_nodes, -1);
  for (size_t g = 0; g + 1 < c->agrp_ptr.size(); ++g)
    for (int64_t s = c->agrp_ptr[g]; s < c->agrp_ptr[g + 1]; ++s) gid[c->agrp_slot[s]] = (int64_t)g;
  mg->cu_ptr.assign(1, 0);
  for (int64_t s = 0; s < c->n_nodes; ++s) {
    if ((c->flags[s] & 3) != 2) continue;            // owner copies of unknown nodes
    mg->cu_owner.push_back(s);
    if (gid[s] < 0) {
      mg->cu_slot.push_back(s);
    } else {
      for (int64_t q = c->agrp_ptr[gid[s]]; q < c->agrp_ptr[gid[s] + 1]; ++q)
        mg->cu_slot.push_back(c->agrp_slot[q]);
    }
    mg->cu_ptr.push_back((int64_t)mg->cu_slot.size());
  }
  mg->n_cu = (int)mg->cu_owner.size();
  if (mg->n_cu > MG_MAX_CU) {
    hhg_mg_destroy(mg);
    return fail(HHG_EINVAL, "coarse level too fine for the dense coarse solve (more than 512 unknown nodes)");
  }
  *out = mg;
  return HHG_OK;
}

int hhg_mg_destroy(hhg_mg mg) {
  if (!mg) return HHG_OK;
  for (double *d : mg->d_winv)
    if (d) (void)hipFree(d);
  if (mg->d_cu_owner) (void)hipFree(mg->d_cu_owner);
  if (mg->d_cu_ptr) (void)hipFree(mg->d_cu_ptr);
  if (mg->d_cu_slot) (void)hipFree(mg->d_cu_slot);
  for (hhg_ctx *h : mg->lev) hhg_destroy(h);
  delete mg;
  return HHG_OK;
}

int hhg_mg_set_smoother(hhg_mg mg, int32_t precond) {
  if (!mg) return fail(HHG_EINVAL, "null argument");
  if (precond != HHG_PRECOND_BLOCK_JACOBI && precond != HHG_PRECOND_LEARNED)
    return fail(HHG_EINVAL, "smoother must be block Jacobi or learned");
  if (precond == HHG_PRECOND_LEARNED)
    for (size_t q = 1; q < mg->lev.size(); ++q)
      if (!mg->lev[q]->model)
        return fail(HHG_EINVAL, "learned smoother: attach a model to every level above the coarsest");
  mg->smoother = precond;
  mg->ready = nullptr;                     // blocks change: a new coefficient setup is needed
  return HHG_OK;
}

int hhg_mg_level(hhg_mg mg, int32_t level, hhg_handle *out) {
  if (!mg || !out) return fail(HHG_EINVAL, "null argument");
  if (level < mg->coarse_level || level > mg->fine_level) return fail(HHG_EINVAL, "level out of range");
  *out = mg->lev[level - mg->coarse_level];
  return HHG_OK;
}

int hhg_mg_workspace_bytes(hhg_mg mg, size_t *bytes) {
  if (!mg || !bytes) return fail(HHG_EINVAL, "null argument");
  *bytes = layout(mg, nullptr, nullptr);
  return HHG_OK;
}

int hhg_mg_prolong(hhg_mg mg, int32_t fine_level, const double *xc, double *xf, void *stream) {
  int rc = check_mg(mg);
  if (rc) return rc;
  if (!xc || !xf) return fail(HHG_EINVAL, "null vector");
  if (fine_level <= mg->coarse_level || fine_level > mg->fine_level)
    return fail(HHG_EINVAL, "fine level out of range");
  if ((rc = mg_device(mg))) return rc;
  return prolong<double>(mg, fine_level - mg->coarse_level, xc, xf, false, (hipStream_t)stream);
}

int hhg_mg_restrict(hhg_mg mg, int32_t fine_level, const double *rf, double *rc_, void *stream) {
  int rc = check_mg(mg);
  if (rc) return rc;
  if (!rf || !rc_) return fail(HHG_EINVAL, "null vector");
  if (fine_level <= mg->coarse_level || fine_level > mg->fine_level)
    return fail(HHG_EINVAL, "fine level out of range");
  if ((rc = mg_device(mg))) return rc;
  return restrict_<double>(mg, fine_level - mg->coarse_level, rf, rc_, (hipStream_t)stream);
}

int hhg_mg_setup_coefficient(hhg_mg mg, int32_t method, const double *k, void *workspace,
                             void *stream) {
  int rc = check_mg(mg);
  if (rc) return rc;
  if (!k || !workspace) return fail(HHG_EINVAL, "null argument");
  if (method != HHG_METHOD_SCALED && method != HHG_METHOD_ONTHEFLY)
    return fail(HHG_EINVAL, "unknown operator method");
  mg->method = method;
  mg->ready = nullptr;
  if (((uintptr_t)k | (uintptr_t)workspace) & 255) return fail(HHG_EINVAL, "misaligned pointer");
  if ((rc = mg_device(mg))) return rc;
  hipStream_t st = (hipStream_t)stream;
  MgWork W;
  layout(mg, static_cast<char *>(workspace), &W);
  const int L = (int)mg->lev.size();
  HHG_HIP(hipMemcpyAsync(W.k[L - 1], k, 8 * (size_t)mg->lev[L - 1]->n_nodes, hipMemcpyDeviceToDevice, st));
  for (int q = L - 1; q > 0; --q) {
    hhg_ctx *c = mg->lev[q - 1], *f = mg->lev[q];
    hipLaunchKernelGGL(k_inject, macro_grid(c), dim3(256), 0, st, c->d_minfo, f->d_minfo, W.k[q],
                       W.k[q - 1]);
    HHG_HIP(hipGetLastError());
  }
  for (int q = 0; q < L; ++q) {
    // the coarsest level is solved exactly; its blocks stay block Jacobi
    const int pc = (mg->smoother == HHG_PRECOND_LEARNED && q > 0) ? HHG_PRECOND_LEARNED
                                                                 : HHG_PRECOND_BLOCK_JACOBI;
    if ((rc = hhg_preconditioner(mg->lev[q], pc, method, W.k[q], W.P[q], st))) return rc;
    // FP32 copies for FP32 cycles
    const int64_t N = mg->lev[q]->n_nodes;
    hipLaunchKernelGGL((k_cast<double, float>), grid1(N), dim3(256), 0, st, W.k[q], W.k32[q], N);
    hipLaunchKernelGGL((k_cast<double, float>), grid1(6 * N), dim3(256), 0, st, W.P[q], W.P32[q],
                       6 * N);
    HHG_HIP(hipGetLastError());
  }
  // dense coarsest operator, column by column, then its inverse on the host
  hhg_ctx *c = mg->lev[0];
  const int n3 = 3 * mg->n_cu;
  const int64_t N0 = c->n_nodes;
  for (int col = 0; col < n3; ++col) {
    hipLaunchKernelGGL(k_fill0<double>, grid1(3 * N0), dim3(256), 0, st, W.b[0], 3 * N0);
    hipLaunchKernelGGL(k_unit, dim3(1), dim3(64), 0, st, mg->d_cu_ptr, mg->d_cu_slot, col / 3, col % 3,
                       W.b[0], N0);
    HHG_HIP(hipGetLastError());
    if ((rc = apply_internal(c, HHG_F64, method, nullptr, W.b[0], W.k[0], W.x[0], st)))
      return rc;
    hipLaunchKernelGGL(k_column, grid1(n3), dim3(256), 0, st, mg->d_cu_owner, mg->n_cu, W.x[0], N0,
                       W.Ainv, col);
    HHG_HIP(hipGetLastError());
  }
  mg->dense.assign((size_t)n3 * n3, 0.0);
  if (n3 > 0) {
    HHG_HIP(hipMemcpyAsync(mg->dense.data(), W.Ainv, mg->dense.size() * 8, hipMemcpyDeviceToHost, st));
    HHG_HIP(hipStreamSynchronize(st));
    if (!dense_inverse(mg->dense, n3))
      return fail(HHG_EBREAKDOWN, "coarsest operator is singular");
    HHG_HIP(hipMemcpyAsync(W.Ainv, mg->dense.data(), mg->dense.size() * 8, hipMemcpyHostToDevice, st));
  }
  HHG_HIP(hipStreamSynchronize(st));
  mg->ready = workspace;
  return HHG_OK;
}

int hhg_mg_vcycle(hhg_mg mg, const hhg_mg_opts *o, const double *r, double *z, void *workspace,
                  void *stream) {
  int rc = check_mg(mg);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if (!r || !z || !workspace) return fail(HHG_EINVAL, "null argument");
  if (((uintptr_t)r | (uintptr_t)z) & 15 || (uintptr_t)workspace & 255)
    return fail(HHG_EINVAL, "misaligned pointer");
  if (r == z) return fail(HHG_EINVAL, "z must not alias r");
  if (workspace != mg->ready)
    return fail(HHG_EINVAL, "call hhg_mg_setup_coefficient with this workspace first");
  if ((rc = mg_device(mg))) return rc;
  MgWork W;
  layout(mg, static_cast<char *>(workspace), &W);
  return finest_cycle(mg, W, *o, r, z, (hipStream_t)stream);
}

int hhg_mg_solve(hhg_mg mg, const hhg_mg_opts *o, const double *b, double *x, void *workspace,
                 hhg_solve_info *info, void *stream) {
  int rc = check_mg(mg);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if (!b || !x || !workspace || !info) return fail(HHG_EINVAL, "null argument");
  if (((uintptr_t)b | (uintptr_t)x) & 15 || (uintptr_t)workspace & 255)
    return fail(HHG_EINVAL, "misaligned pointer");
  if (!(o->rtol > 0.0) || o->maxit < 1) return fail(HHG_EINVAL, "rtol must be > 0 and maxit >= 1");
  if (workspace != mg->ready)
    return fail(HHG_EINVAL, "call hhg_mg_setup_coefficient with this workspace first");
  if ((rc = mg_device(mg))) return rc;
  MgWork W;
  layout(mg, static_cast<char *>(workspace), &W);
  const int F = (int)mg->lev.size() - 1;
  hhg_ctx *h = mg->lev[F];
  const int64_t n3 = 3 * h->n_nodes;
  const auto t0 = std::chrono::steady_clock::now();
  *info = hhg_solve_info{};
  // the solve runs on the finest handle's own stream, after the caller's
  // queued work, and is complete on return
  HHG_HIP(hipStreamSynchronize((hipStream_t)stream));
  hipStream_t st = h->solve_stream;
  // one V-cycle (pr -> pz) captured in a HIP graph and replayed every
  // iteration (no timing events inside a graph)
  bool use_graph = std::getenv("HHG_NO_GRAPH") == nullptr;
  for (hhg_ctx *l : mg->lev) use_graph = use_graph && !l->prof_on;
  hipGraphExec_t exec = nullptr;
  if (use_graph) {
    hipGraph_t graph = nullptr;
    HHG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int crc = finest_cycle(mg, W, *o, W.pr, W.pz, st);
    const hipError_t ce = hipStreamEndCapture(st, &graph);
    if (crc) {
      if (graph) (void)hipGraphDestroy(graph);
      return crc;
    }
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
  }
  struct ExecGuard {
    hipGraphExec_t e;
    ~ExecGuard() {
      if (e) (void)hipGraphExecDestroy(e);
    }
  } guard{exec};
  auto cycle = [&]() -> int {
    if (exec) {
      HHG_HIP(hipGraphLaunch(exec, st));
      return HHG_OK;
    }
    return finest_cycle(mg, W, *o, W.pr, W.pz, st);
  };
  double bb = 0.0, rr = 0.0, rho = 0.0, pq = 0.0;
  if ((rc = dot(mg, W, b, b, &bb, st))) return rc;
  const double nb = std::sqrt(bb);
  if ((rc = apply_internal(h, HHG_F64, mg->method, b, x, W.k[F], W.pr, st))) return rc;
  if ((rc = dot(mg, W, W.pr, W.pr, &rr, st))) return rc;
  int it = 0, status = HHG_OK;
  if (nb == 0.0 || std::sqrt(rr) <= o->rtol * nb) goto done;
  if (o->method == HHG_MG_CYCLE) {
    // stationary iteration x += V(b - A x)
    while (true) {
      if (it >= o->maxit) {
        status = HHG_ENOCONV;
        break;
      }
      if ((rc = cycle())) return rc;
      hipLaunchKernelGGL(k_xpby, grid1(n3), dim3(256), 0, st, x, W.pz, 1.0, n3);
      HHG_HIP(hipGetLastError());
      ++it;
      if ((rc = apply_internal(h, HHG_F64, mg->method, b, x, W.k[F], W.pr, st))) return rc;
      if ((rc = dot(mg, W, W.pr, W.pr, &rr, st))) return rc;
      if (!std::isfinite(rr)) {
        status = HHG_EBREAKDOWN;
        break;
      }
      if (std::sqrt(rr) <= o->rtol * nb) break;
    }
    goto done;
  }
  if ((rc = cycle())) return rc;
  if ((rc = dot(mg, W, W.pr, W.pz, &rho, st))) return rc;
  HHG_HIP(hipMemcpyAsync(W.pp, W.pz, 8 * n3, hipMemcpyDeviceToDevice, st));
  while (true) {
    if (it >= o->maxit) {
      status = HHG_ENOCONV;
      break;
    }
    if ((rc = apply_internal(h, HHG_F64, mg->method, nullptr, W.pp, W.k[F], W.pq, st))) return rc;
    if ((rc = dot(mg, W, W.pp, W.pq, &pq, st))) return rc;
    if (!(pq > 0.0) || !std::isfinite(pq) || !std::isfinite(rho)) {
      status = HHG_EBREAKDOWN;
      break;
    }
    const double alpha = rho / pq;
    hipLaunchKernelGGL(k_axpy2, grid1(n3), dim3(256), 0, st, x, W.pp, W.pr, W.pq, alpha, n3);
    HHG_HIP(hipGetLastError());
    ++it;
    if ((rc = dot(mg, W, W.pr, W.pr, &rr, st))) return rc;
    if (std::sqrt(rr) <= o->rtol * nb) break;
    if ((rc = cycle())) return rc;
    double rho_new = 0.0;
    if ((rc = dot(mg, W, W.pr, W.pz, &rho_new, st))) return rc;
    hipLaunchKernelGGL(k_xpby, grid1(n3), dim3(256), 0, st, W.pp, W.pz, rho_new / rho, n3);
    HHG_HIP(hipGetLastError());
    rho = rho_new;
  }
done:
  // final residual recomputed from x
  if ((rc = apply_internal(h, HHG_F64, mg->method, b, x, W.k[F], W.pr, st))) return rc;
  if ((rc = dot(mg, W, W.pr, W.pr, &rr, st))) return rc;
  info->iterations = it;
  info->iterations_run = it;       // checked every iteration
  info->outer_iterations = 1;
  info->status = status;
  info->rel_residual = nb > 0.0 ? std::sqrt(rr) / nb : 0.0;
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (status == HHG_ENOCONV) return fail(HHG_ENOCONV, "multigrid solve reached maxit");
  if (status == HHG_EBREAKDOWN) return fail(HHG_EBREAKDOWN, "multigrid solve breakdown");
  return HHG_OK;
}

}  // extern "C"

extern "C" {

int hhg_stokes_rows(hhg_handle h, int32_t op, double hl, const double *in, double *out,
                    void *stream) {
  if (!h || !out || (op != HHG_STOKES_MASS && !in)) return fail(HHG_EINVAL, "null argument");
  if (op < HHG_STOKES_DIV || op > HHG_STOKES_MASS) return fail(HHG_EINVAL, "unknown Stokes term");
  if (op == HHG_STOKES_STAB && !(hl > 0.0)) return fail(HHG_EINVAL, "mesh width must be > 0");
  if (((uintptr_t)in | (uintptr_t)out) & 15) return fail(HHG_EINVAL, "misaligned pointer");
  if (in == out) return fail(HHG_EINVAL, "out must not alias in");
  int rc = ensure_device(h);
  if (rc) return rc;
  return stokes_rows(h, op, hl, in, out, (hipStream_t)stream);
}

int hhg_mg_stokes_workspace_bytes(hhg_mg mg, size_t *bytes) {
  const int rc = check_mg(mg);
  if (rc) return rc;
  if (!bytes) return fail(HHG_EINVAL, "null argument");
  *bytes = stokes_layout(mg->lev.back(), nullptr, nullptr);
  return HHG_OK;
}

namespace {
int check_stokes(hhg_mg mg, const hhg_stokes_opts *o, const double *f, const double *u,
                 const double *p, const double *mu, void *mgw, void *sw) {
  int rc = check_mg(mg);
  if (rc) return rc;
  if (!o || !f || !u || !p || !mu || !mgw || !sw) return fail(HHG_EINVAL, "null argument");
  if (((uintptr_t)f | (uintptr_t)u | (uintptr_t)p | (uintptr_t)mu) & 15 || ((uintptr_t)mgw | (uintptr_t)sw) & 255)
    return fail(HHG_EINVAL, "misaligned pointer");
  if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 < 1 || o->nu1 > 64 || o->nu2 > 64)
    return fail(HHG_EINVAL, "smoothing steps must be 0..64 each, at least one in total");
  if (!(o->omega > 0.0 && o->omega < 2.0)) return fail(HHG_EINVAL, "omega must lie in (0, 2)");
  if (!(o->omega_p > 0.0 && o->omega_p < 4.0)) return fail(HHG_EINVAL, "omega_p must lie in (0, 4)");
  if (o->nu_inc < 0 || o->nu_inc > 8) return fail(HHG_EINVAL, "nu_inc must be 0..8");
  if (!(o->rtol >= 0.0) || o->maxit < 0) return fail(HHG_EINVAL, "rtol must be >= 0 and maxit >= 0");
  return HHG_OK;
}
double mesh_width_of(const hhg_mg_s *mg, const hhg_stokes_opts *o) {
  return o->h > 0.0 ? o->h : 1.0 / (double)(1 << mg->fine_level);
}
}  // namespace

int hhg_mg_stokes_solve(hhg_mg mg, const hhg_stokes_opts *o, const double *f, const double *g,
                        const double *mu, double *u, double *p, void *mg_workspace,
                        void *stokes_workspace, hhg_solve_info *info, void *stream) {
  int rc = check_stokes(mg, o, f, u, p, mu, mg_workspace, stokes_workspace);
  if (rc) return rc;
  if (!info) return fail(HHG_EINVAL, "null argument");
  if ((uintptr_t)g & 15) return fail(HHG_EINVAL, "misaligned pointer");
  if (mg_workspace != mg->ready)
    return fail(HHG_EINVAL, "call hhg_mg_setup_coefficient with this workspace first");
  if ((rc = mg_device(mg))) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  *info = hhg_solve_info{};
  hipStream_t st = (hipStream_t)stream;
  MgWork W;
  layout(mg, static_cast<char *>(mg_workspace), &W);
  StokesWork S;
  stokes_layout(mg->lev.back(), static_cast<char *>(stokes_workspace), &S);
  hhg_ctx *h = mg->lev.back();
  const int64_t N = h->n_nodes;
  const double hl = mesh_width_of(mg, o);
  if ((rc = stokes_rows(h, SK_MASS, hl, nullptr, S.mass, st))) return rc;
  if ((rc = stokes_rows(h, SK_CDIAG, hl, nullptr, S.cdiag, st))) return rc;
  hipLaunchKernelGGL(k_schur, grid1(N), dim3(256), 0, st, S.S, S.mass, mu, S.cdiag, N);
  HHG_HIP(hipGetLastError());
  double ff = 0.0, gg = 0.0;
  if ((rc = dot_vel(h, f, f, S.part, st, ff))) return rc;
  if (g && (rc = dot_owner(h, g, g, S.part, st, gg))) return rc;
  const double nrm = std::sqrt(ff + gg);
  int it = 0;
  double res = 0.0;
  if ((rc = uzawa(mg, W, S, *o, hl, f, g, u, p, o->maxit, o->rtol * nrm, st, it, res))) return rc;
  HHG_HIP(hipStreamSynchronize(st));
  info->iterations = it;
  info->iterations_run = it;
  info->outer_iterations = 1;
  info->rel_residual = nrm > 0.0 ? res / nrm : res;
  info->status = info->rel_residual <= o->rtol ? HHG_OK : HHG_ENOCONV;
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info->status == HHG_ENOCONV) return fail(HHG_ENOCONV, "Stokes solve reached maxit");
  return HHG_OK;
}

int hhg_mg_stokes_picard(hhg_mg mg, const hhg_stokes_opts *o, const hhg_carreau *law,
                         int32_t method, int32_t max_picard, const double *f, double *u,
                         double *p, double *mu, void *mg_workspace, void *stokes_workspace,
                         hhg_picard_info *info, void *stream) {
  int rc = check_stokes(mg, o, f, u, p, mu, mg_workspace, stokes_workspace);
  if (rc) return rc;
  if (!law || !info) return fail(HHG_EINVAL, "null argument");
  if (method != HHG_METHOD_SCALED && method != HHG_METHOD_ONTHEFLY)
    return fail(HHG_EINVAL, "unknown operator method");
  if (max_picard < 1) return fail(HHG_EINVAL, "max_picard must be >= 1");
  if ((rc = mg_device(mg))) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  *info = hhg_picard_info{};
  hipStream_t st = (hipStream_t)stream;
  MgWork W;
  layout(mg, static_cast<char *>(mg_workspace), &W);
  StokesWork S;
  stokes_layout(mg->lev.back(), static_cast<char *>(stokes_workspace), &S);
  hhg_ctx *h = mg->lev.back();
  const int64_t N = h->n_nodes;
  const double hl = mesh_width_of(mg, o);
  // mu = mu(u) and the velocity multigrid of A(mu)
  auto viscosity = [&](bool setup) -> int {
    int r2 = hhg_nodal_viscosity(h, u, law, mu, S.visc, st);
    if (r2) return r2;
    if (!setup) return HHG_OK;
    if ((r2 = hhg_mg_setup_coefficient(mg, method, mu, mg_workspace, st))) return r2;
    hipLaunchKernelGGL(k_schur, grid1(N), dim3(256), 0, st, S.S, S.mass, mu, S.cdiag, N);
    HHG_HIP(hipGetLastError());
    return HHG_OK;
  };
  hipLaunchKernelGGL(k_fill0<double>, grid1(3 * N), dim3(256), 0, st, u, 3 * N);
  hipLaunchKernelGGL(k_fill0<double>, grid1(N), dim3(256), 0, st, p, N);
  HHG_HIP(hipGetLastError());
  if ((rc = stokes_rows(h, SK_MASS, hl, nullptr, S.mass, st))) return rc;
  if ((rc = stokes_rows(h, SK_CDIAG, hl, nullptr, S.cdiag, st))) return rc;
  if ((rc = viscosity(true))) return rc;
  double ff = 0.0;
  if ((rc = dot_vel(h, f, f, S.part, st, ff))) return rc;
  const double nrm = std::sqrt(ff);
  int status = HHG_ENOCONV;
  std::vector<double> hp(2 * MG_RED);
  for (int n = 0; n < max_picard; ++n) {
    HHG_HIP(hipMemcpyAsync(S.uprev, u, 24 * (size_t)N, hipMemcpyDeviceToDevice, st));
    int it = 0;
    double res = 0.0;
    if ((rc = uzawa(mg, W, S, *o, hl, f, nullptr, u, p, 1, 0.0, st, it, res))) return rc;
    if ((rc = viscosity(true))) return rc;
    info->picard = n + 1;
    hipLaunchKernelGGL(k_node_max2, dim3(MG_RED), dim3(256), 0, st, u, S.uprev, h->d_flags, N, S.part);
    HHG_HIP(hipGetLastError());
    HHG_HIP(hipMemcpyAsync(hp.data(), S.part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HHG_HIP(hipStreamSynchronize(st));
    double dm = 0.0, um = 0.0;
    for (int q = 0; q < MG_RED; ++q) {
      dm = std::max(dm, hp[2 * q]);
      um = std::max(um, hp[2 * q + 1]);
    }
    info->rel_change = um > 0.0 ? dm / um : 0.0;
    if (!std::isfinite(info->rel_change)) return fail(HHG_EBREAKDOWN, "non-finite fixed-point iterate");
    if (dm < 1e-3 * um) {
      status = HHG_OK;
      break;
    }
  }
  int it = 0;
  double res = 0.0;
  if ((rc = uzawa(mg, W, S, *o, hl, f, nullptr, u, p, o->maxit, o->rtol * nrm, st, it, res))) return rc;
  info->final_iterations = it;
  info->rel_residual = nrm > 0.0 ? res / nrm : res;
  if (info->rel_residual > o->rtol) status = HHG_ENOCONV;
  if ((rc = viscosity(false))) return rc;
  HHG_HIP(hipStreamSynchronize(st));
  info->status = status;
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (status == HHG_ENOCONV) return fail(HHG_ENOCONV, "fixed-point or final Stokes iteration reached its limit");
  return HHG_OK;
}

}  // extern "C"
