// The 2-D variant (Sec. 2 and Sec. 2.3): macro triangles refined uniformly,
// the vector operator 2 (mu0 + mu1 k)(eps, eps) + (lam0 + lam1 k)(div, div)
// applied matrix-free by physical stencil scaling (or its unphysical
// variant, or nodal integration).
//
// Layout: macro m owns the slots [off_m, off_m + (n+1)(n+2)/2); node (i, j),
// i + j <= n, of the index space x0 + (i/n)(x1 - x0) + (j/n)(x2 - x0) sits
// at slot off_m + j(n+1) - j(j-1)/2 + i (rows of constant j contiguous).
// Vectors are [2][n_slots] (x, y) and [n_slots] (k).  The six neighbour
// directions E, W, N, S, NW, SE and the six triangles around a node (each
// spanned by two consecutive directions E, N, NW, W, S, SE) are the same
// for every macro; their element matrices are per macro constants.
//
// Interior row i:  y_i = sum_d S_d (x_{i+d} - x_i),
//   S_d = A0_d + khat_d Shat_d + (k_p1(d) - k_p2(d)) c_d J,
// khat_d the patch mean (k_i + k_{i+d})/3 + (k_p1 + k_p2)/6 of the edge's
// two elements, Shat_d the sum of their symmetric parts, p1(d), p2(d) their
// third vertices, and c_d J = (1/3) times the antisymmetric part of the
// first element's block (eq. correction2d; the element t^m of the Lemma is
// the second element, so kbar^t - kbar^{t^m} = (k_p1 - k_p2) / 3).
// Rows of nodes on a macro boundary: partial rows per macro from its
// elements (nodal entries) and scaled entries towards its interior nodes,
// as in 3-D, summed over the node's copies by a group kernel.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <new>
#include <vector>

#include "hhg_ctx.h"

namespace hhg2 {

using hhg::fail;
using hhg::hip_fail;

constexpr int ND = 6;
// E, W, N, S, NW, SE; opposite directions in pairs (2p, 2p + 1)
constexpr int DI[ND] = {1, -1, 0, 0, -1, 1};
constexpr int DJ[ND] = {0, 0, 1, -1, 1, -1};
// the six triangles around a node, counter-clockwise: directions (a, b)
constexpr int TRI[ND][2] = {{0, 2}, {2, 4}, {4, 1}, {1, 3}, {3, 5}, {5, 0}};

template <typename T>
struct Const2D {
  T S[ND][3];          // Shat_d: xx, yy, xy
  T A0[ND][4];         // constant part of S_d, [l][m]
  T c[ND];             // correction: (R_d)[0][1] = c_d (k_p1 - k_p2), [1][0] = -that
  T E1[ND][3][4];      // triangle t around the node, vertex (centre, a, b): block [l][m]
  T E0[ND][3][4];
  int32_t p1[ND], p2[ND];   // third vertex directions of the two elements of edge d
};

struct Macro2D {
  int64_t off;
  int32_t n;
  uint32_t dmask;      // bit e: the macro edge opposite vertex e is Dirichlet; bit 3 + e:
                       // vertex e is (through another macro's edge, too)
};


__device__ __forceinline__ int slot_of(int i, int j, int n) { return j * (n + 1) - j * (j - 1) / 2 + i; }

// Dirichlet if on a macro edge marked in dmask (edge e opposite vertex e:
// e = 0: i + j = n, e = 1: i = 0, e = 2: j = 0) or a marked vertex
__host__ __device__ __forceinline__ bool is_dirichlet(int i, int j, int n, uint32_t dmask) {
  return (((dmask >> 0) & 1u) && i + j == n) || (((dmask >> 1) & 1u) && i == 0) ||
         (((dmask >> 2) & 1u) && j == 0) || (((dmask >> 3) & 1u) && i == 0 && j == 0) ||
         (((dmask >> 4) & 1u) && i == n && j == 0) || (((dmask >> 5) & 1u) && i == 0 && j == n);
}

constexpr int TPB2 = 256;          // threads per block: columns i0 - 1 .. i0 + TPB2 - 2
constexpr int OUT2 = TPB2 - 2;     // output columns per block
constexpr int STRIP = 8;           // rows per block

// third vertices of the two elements of edge d (the same on every macro;
// the host setup checks its element tables against them)
constexpr int P1[ND] = {2, 4, 0, 1, 2, 3};
constexpr int P2[ND] = {5, 3, 4, 5, 1, 0};

// Operator variant fixed at compile time: physical correction, unscaled
// part present, k-hat as the edge mean.
template <bool CORR, bool A0C, bool KEDGE>
struct Var {};

// Scaled entry of direction d applied to (e0, e1), accumulated into y.
template <typename T, bool CORR, bool A0C, bool KEDGE, int D>
__device__ __forceinline__ void scaled_entry(const T (&S)[ND][3], const T (&A)[ND][4], const T (&cc)[ND],
                                             const T (&nk)[ND], T ck, T e0, T e1, T &y0, T &y1) {
  const T kp1 = nk[P1[D]], kp2 = nk[P2[D]];
  const T kh = KEDGE ? T(0.5) * (ck + nk[D]) : fma(ck + nk[D], T(1.0 / 3.0), (kp1 + kp2) * T(1.0 / 6.0));
  const T s0 = fma(S[D][0], e0, S[D][2] * e1), s1 = fma(S[D][2], e0, S[D][1] * e1);
  y0 = fma(kh, s0, y0);
  y1 = fma(kh, s1, y1);
  if constexpr (A0C) {
    y0 = fma(A[D][0], e0, fma(A[D][2], e1, y0));
    y1 = fma(A[D][1], e0, fma(A[D][3], e1, y1));
  }
  if constexpr (CORR) {
    const T w = cc[D] * (kp1 - kp2);             // R[0][1] = w, R[1][0] = -w
    y0 = fma(-w, e1, y0);
    y1 = fma(w, e0, y1);
  }
}

template <typename T, bool CORR, bool A0C, bool KEDGE, int D = 0>
__device__ __forceinline__ void interior_row(const T (&S)[ND][3], const T (&A)[ND][4], const T (&cc)[ND],
                                             const T (&nx0)[ND], const T (&nx1)[ND], const T (&nk)[ND],
                                             T c0, T c1, T ck, T &y0, T &y1) {
  scaled_entry<T, CORR, A0C, KEDGE, D>(S, A, cc, nk, ck, nx0[D] - c0, nx1[D] - c1, y0, y1);
  if constexpr (D + 1 < ND)
    interior_row<T, CORR, A0C, KEDGE, D + 1>(S, A, cc, nx0, nx1, nk, c0, c1, ck, y0, y1);
}

// Row of a node on a macro boundary (or any row of the on-the-fly method):
// this macro's elements give nodal entries; under the symmetric and zero-sum
// rules the entries towards macro-interior neighbours are the scaled ones.
template <typename T, bool CORR, bool A0C, bool KEDGE>
__device__ __forceinline__ void boundary_row2d(const Const2D<T> &C, int scaled, int iface, int i, int j,
                                               int n, const T (&nx0)[ND], const T (&nx1)[ND],
                                               const T (&nk)[ND], T c0, T c1, T ck, T &y0, T &y1) {
  const auto &S = C.S;
  const auto &A = C.A0;
  const auto &cc = C.c;
  bool in[ND], nb_onb[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const int a = i + DI[d], b = j + DJ[d];
    in[d] = a >= 0 && b >= 0 && a + b <= n;
    nb_onb[d] = in[d] && (a == 0 || b == 0 || a + b == n);
  }
  const bool rowwise = !scaled || iface == HHG_IFACE_ROWWISE;
  const bool zs = !rowwise && iface == HHG_IFACE_ZEROSUM;
  y0 = T(0);
  y1 = T(0);
#pragma unroll
  for (int t = 0; t < ND; ++t) {
    const int da = TRI[t][0], db = TRI[t][1];
    if (!(in[da] && in[db])) continue;
    const T kb = (ck + nk[da] + nk[db]) * T(1.0 / 3.0);
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      T e0, e1;
      if (v == 0) {
        if (zs) continue;
        e0 = c0;
        e1 = c1;
      } else {
        const int d = v == 1 ? da : db;
        if (!rowwise && !nb_onb[d]) continue;   // scaled entry below
        e0 = zs ? nx0[d] - c0 : nx0[d];
        e1 = zs ? nx1[d] - c1 : nx1[d];
      }
      const T *B1 = C.E1[t][v], *B0 = C.E0[t][v];
      y0 = fma(kb, fma(B1[0], e0, B1[2] * e1), fma(B0[0], e0, fma(B0[2], e1, y0)));
      y1 = fma(kb, fma(B1[1], e0, B1[3] * e1), fma(B0[1], e0, fma(B0[3], e1, y1)));
    }
  }
  if (rowwise) return;
#define HHG2_SE(D)                                                                                    \
  if (in[D] && !nb_onb[D])                                                                            \
    scaled_entry<T, CORR, A0C, KEDGE, D>(S, A, cc, nk, ck, zs ? nx0[D] - c0 : nx0[D],                  \
                                         zs ? nx1[D] - c1 : nx1[D], y0, y1);
  HHG2_SE(0) HHG2_SE(1) HHG2_SE(2) HHG2_SE(3) HHG2_SE(4) HHG2_SE(5)
#undef HHG2_SE
}

// Macro-interior rows (i, j >= 1, i + j <= n - 1).  A block sweeps a strip
// of STRIP rows over OUT2 columns, RB rows at a time: the next RB rows of x
// and k (one halo column each side; Dirichlet x zeroed) are staged into a
// ring of RB + 2 rows in LDS, then the RB rows below them are computed from
// the ring, so every value is read from HBM about once.
// Grid: (column blocks, strips, macros).
constexpr int RB = 2;
constexpr int RING = RB + 2;

template <typename T, bool CORR, bool A0C, bool KEDGE>
__global__ __launch_bounds__(TPB2) void k_interior2d(const Macro2D *__restrict__ macros,
                                                     const Const2D<T> *__restrict__ cs,
                                                     const T *__restrict__ x, const T *__restrict__ kc,
                                                     T *__restrict__ y, int64_t N) {
  static_assert(STRIP % RB == 0, "whole batches per strip");
  __shared__ T rx0[RING][TPB2], rx1[RING][TPB2], rk[RING][TPB2];
  const Macro2D M = macros[blockIdx.z];
  const int n = M.n;
  const int i0 = blockIdx.x * OUT2, j0 = blockIdx.y * STRIP;
  if (i0 + j0 > n) return;                   // strip outside the triangle (block-uniform)
  const int t = threadIdx.x;
  const int i = i0 - 1 + t;                  // column of this thread
  const T *X0 = x + M.off, *X1 = X0 + N, *K = kc + M.off;
  const Const2D<T> &C = cs[blockIdx.z];
  // row j of this thread's column: global -> registers (nothing reads the
  // values until put(), so the loads stay in flight through the compute of
  // the rows below), then registers -> ring slot (j + RING) % RING
  struct V3 {
    T a, b, k;
  };
  auto fetch = [&](int j) {
    V3 v{T(0), T(0), T(0)};
    if (j >= 0 && j <= n && i >= 0 && i + j <= n) {
      const int s = slot_of(i, j, n);
      v.k = K[s];
      v.a = X0[s];
      v.b = X1[s];
    }
    return v;
  };
  auto put = [&](int j, const V3 &v) {
    const int r = (j + RING) % RING;
    const bool dz = j >= 0 && j <= n && i >= 0 && i + j <= n && is_dirichlet(i, j, n, M.dmask);
    rx0[r][t] = dz ? T(0) : v.a;
    rx1[r][t] = dz ? T(0) : v.b;
    rk[r][t] = v.k;
  };
  const int j1 = min(j0 + STRIP, n);
  {
    V3 v[RB + 2];
#pragma unroll
    for (int q = 0; q < RB + 2; ++q) v[q] = fetch(j0 - 1 + q);
#pragma unroll
    for (int q = 0; q < RB + 2; ++q) put(j0 - 1 + q, v[q]);
  }
  for (int jb = j0; jb < j1; jb += RB) {
    // the ring holds rows jb - 1 .. jb + RB; rows jb + RB + 1 .. jb + 2 RB
    // are fetched now and written after the compute
    const bool more = jb + RB < j1;
    V3 nv[RB];
    if (more)
#pragma unroll
      for (int q = 0; q < RB; ++q) nv[q] = fetch(jb + RB + 1 + q);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int j = jb + q;
      if (j >= 1 && j < j1 && t >= 1 && t <= OUT2 && i >= 1 && i + j <= n - 1) {
        const int rm = (j - 1 + RING) % RING, r0 = j % RING, rp = (j + 1) % RING;
        T nx0[ND], nx1[ND], nk[ND];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          const int r = DJ[d] > 0 ? rp : (DJ[d] < 0 ? rm : r0);
          const int c = t + DI[d];
          nx0[d] = rx0[r][c];
          nx1[d] = rx1[r][c];
          nk[d] = rk[r][c];
        }
        T y0 = T(0), y1 = T(0);
        interior_row<T, CORR, A0C, KEDGE>(C.S, C.A0, C.c, nx0, nx1, nk, rx0[r0][t], rx1[r0][t], rk[r0][t],
                                          y0, y1);
        const int64_t slot = M.off + slot_of(i, j, n);
        y[slot] = y0;
        y[N + slot] = y1;
      }
    }
    __syncthreads();
    if (more)
#pragma unroll
      for (int q = 0; q < RB; ++q) put(jb + RB + 1 + q, nv[q]);
  }
}

// Macro-boundary rows (and, for the on-the-fly method, the interior rows
// too): one thread per slot of the list, neighbours gathered from HBM.
// bpos: packed (macro << 40 | j << 20 | i) of every listed slot.
template <typename T, bool CORR, bool A0C, bool KEDGE>
__global__ __launch_bounds__(256) void k_rows2d(const Macro2D *__restrict__ macros,
                                                const Const2D<T> *__restrict__ cs,
                                                const int64_t *__restrict__ bpos, int64_t nb, int scaled,
                                                int iface, const T *__restrict__ x,
                                                const T *__restrict__ kc, T *__restrict__ y, int64_t N) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nb) return;
  const int64_t pk = bpos[q];
  const int m = (int)(pk >> 40), j = (int)((pk >> 20) & 0xFFFFF), i = (int)(pk & 0xFFFFF);
  const Macro2D M = macros[m];
  const int n = M.n;
  const int64_t slot = M.off + slot_of(i, j, n);
  if (is_dirichlet(i, j, n, M.dmask)) {
    y[slot] = T(0);
    y[N + slot] = T(0);
    return;
  }
  const T *X0 = x + M.off, *X1 = X0 + N, *K = kc + M.off;
  T nx0[ND], nx1[ND], nk[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const int a = i + DI[d], b = j + DJ[d];
    nx0[d] = nx1[d] = nk[d] = T(0);
    if (a >= 0 && b >= 0 && a + b <= n) {
      const int s = slot_of(a, b, n);
      nk[d] = K[s];
      if (!is_dirichlet(a, b, n, M.dmask)) {
        nx0[d] = X0[s];
        nx1[d] = X1[s];
      }
    }
  }
  const int ls = slot_of(i, j, n);
  T y0, y1;
  boundary_row2d<T, CORR, A0C, KEDGE>(cs[m], scaled, iface, i, j, n, nx0, nx1, nk, X0[ls], X1[ls], K[ls],
                                      y0, y1);
  y[slot] = y0;
  y[N + slot] = y1;
}

// sum of the partial rows over the copies of a node, written to every copy
template <typename T>
__global__ void k_group2d(const int64_t *__restrict__ ptr, const int64_t *__restrict__ slots,
                          int64_t ng, T *__restrict__ y, int64_t N) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  T s0 = T(0), s1 = T(0);
  for (int64_t q = ptr[g]; q < ptr[g + 1]; ++q) {
    s0 += y[slots[q]];
    s1 += y[N + slots[q]];
  }
  for (int64_t q = ptr[g]; q < ptr[g + 1]; ++q) {
    y[slots[q]] = s0;
    y[N + slots[q]] = s1;
  }
}

// ------------------------------------------------------------ host setup
// Element blocks of 2 mu (eps, eps) + lam (div, div) on the triangle with
// vertices X[0..2]: out[a][b][l*2+m] = int (D(phi_b e_l), D(phi_a e_m)).
void elem_blocks(const double X[3][2], double mu, double lam, double out[3][3][4]) {
  const double e1x = X[1][0] - X[0][0], e1y = X[1][1] - X[0][1];
  const double e2x = X[2][0] - X[0][0], e2y = X[2][1] - X[0][1];
  const double det = e1x * e2y - e1y * e2x;
  const double area = 0.5 * std::fabs(det);
  // rows of the inverse of [e1 e2] are the gradients of lambda_1, lambda_2
  double g[3][2];
  g[1][0] = e2y / det;
  g[1][1] = -e2x / det;
  g[2][0] = -e1y / det;
  g[2][1] = e1x / det;
  g[0][0] = -g[1][0] - g[2][0];
  g[0][1] = -g[1][1] - g[2][1];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int l = 0; l < 2; ++l)
        for (int mm = 0; mm < 2; ++mm) {
          // eps(phi e_c)_{pq} = (delta_cp g_q + delta_cq g_p) / 2
          double ee = 0.0;
          for (int p = 0; p < 2; ++p)
            for (int q = 0; q < 2; ++q) {
              const double eb = 0.5 * ((l == p ? g[b][q] : 0.0) + (l == q ? g[b][p] : 0.0));
              const double ea = 0.5 * ((mm == p ? g[a][q] : 0.0) + (mm == q ? g[a][p] : 0.0));
              ee += eb * ea;
            }
          out[a][b][2 * l + mm] = area * (2.0 * mu * ee + lam * g[b][l] * g[a][mm]);
        }
}

}  // namespace hhg2

struct hhg2d_ctx {
  int n_macro = 0, level = 0;
  int64_t n_slots = 0, n_unknown = 0;
  hhg_op_desc op{};
  std::vector<double> verts;
  std::vector<hhg2::Macro2D> macros;
  std::vector<hhg2::Const2D<double>> c64;
  std::vector<uint8_t> flags;
  std::vector<int64_t> gptr, gslot;
  bool on_device = false;
  int device = -1;
  hhg2::Macro2D *d_macros = nullptr;
  hhg2::Const2D<double> *d_c64 = nullptr;
  hhg2::Const2D<float> *d_c32 = nullptr;
  int64_t *d_gptr = nullptr, *d_gslot = nullptr;
  // row positions: the macro-boundary rows first (n_bpos of them), then the
  // macro-interior rows (n_apos in all), for the element-row kernel
  std::vector<int64_t> pos;
  int64_t n_bpos = 0, n_apos = 0;
  int64_t *d_pos = nullptr;
};

namespace hhg2 {

template <typename T>
int upload(T **dst, const T *src, size_t count) {
  if (count == 0) return HHG_OK;
  hipError_t e = hipMalloc((void **)dst, count * sizeof(T));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  e = hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  return HHG_OK;
}

int ensure_device(hhg2d_ctx *h) {
  int dev = 0;
  HHG_HIP(hipGetDevice(&dev));
  if (h->on_device) {
    if (dev != h->device) return fail(HHG_EINVAL, "handle used on a different device than its tables");
    return HHG_OK;
  }
  std::vector<Const2D<float>> c32(h->c64.size());
  for (size_t m = 0; m < h->c64.size(); ++m) {
    const Const2D<double> &a = h->c64[m];
    Const2D<float> &b = c32[m];
    for (int d = 0; d < ND; ++d) {
      for (int q = 0; q < 3; ++q) b.S[d][q] = (float)a.S[d][q];
      for (int q = 0; q < 4; ++q) b.A0[d][q] = (float)a.A0[d][q];
      b.c[d] = (float)a.c[d];
      b.p1[d] = a.p1[d];
      b.p2[d] = a.p2[d];
      for (int v = 0; v < 3; ++v)
        for (int q = 0; q < 4; ++q) {
          b.E1[d][v][q] = (float)a.E1[d][v][q];
          b.E0[d][v][q] = (float)a.E0[d][v][q];
        }
    }
  }
  int rc;
  if ((rc = upload(&h->d_macros, h->macros.data(), h->macros.size()))) return rc;
  if ((rc = upload(&h->d_c64, h->c64.data(), h->c64.size()))) return rc;
  if ((rc = upload(&h->d_c32, c32.data(), c32.size()))) return rc;
  if ((rc = upload(&h->d_gptr, h->gptr.data(), h->gptr.size()))) return rc;
  if ((rc = upload(&h->d_gslot, h->gslot.data(), h->gslot.size()))) return rc;
  if ((rc = upload(&h->d_pos, h->pos.data(), h->pos.size()))) return rc;
  h->on_device = true;
  h->device = dev;
  return HHG_OK;
}

void free_ctx(hhg2d_ctx *h) {
  if (!h) return;
  auto f = [](auto *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
  };
  f(h->d_macros);
  f(h->d_c64);
  f(h->d_c32);
  f(h->d_gptr);
  f(h->d_gslot);
  f(h->d_pos);
  delete h;
}

template <typename T>
int apply_t(hhg2d_ctx *h, int method, const T *x, const T *k, T *y, hipStream_t st) {
  const Const2D<T> *cs;
  if constexpr (sizeof(T) == 8) cs = h->d_c64; else cs = h->d_c32;
  const int scaled = method == HHG_METHOD_SCALED ? 1 : 0, iface = h->op.iface;
  const bool corr = h->op.corr == HHG_CORR_PHYSICAL, kedge = h->op.khat == HHG_KHAT_EDGE;
  const bool a0 = h->op.mu0 != 0.0 || h->op.lam0 != 0.0;
  const int n = 1 << h->level;
  const dim3 grid((unsigned)((n + 1 + OUT2 - 1) / OUT2), (unsigned)((n + 1 + STRIP - 1) / STRIP),
                  (unsigned)h->n_macro);
  // the on-the-fly method takes every row through the element path
  const int64_t nb = scaled ? h->n_bpos : h->n_apos;
  const dim3 g2((unsigned)((nb + 255) / 256));
#define HHG2_L(CR, A0, KE)                                                                              \
  do {                                                                                                  \
    if (scaled)                                                                                         \
      hipLaunchKernelGGL((k_interior2d<T, CR, A0, KE>), grid, dim3(TPB2), 0, st, h->d_macros, cs, x, k, y, \
                         h->n_slots);                                                                   \
    hipLaunchKernelGGL((k_rows2d<T, CR, A0, KE>), g2, dim3(256), 0, st, h->d_macros, cs, h->d_pos, nb,   \
                       scaled, iface, x, k, y, h->n_slots);                                             \
  } while (0)
  if (corr) {
    if (a0) { if (kedge) HHG2_L(true, true, true); else HHG2_L(true, true, false); }
    else { if (kedge) HHG2_L(true, false, true); else HHG2_L(true, false, false); }
  } else {
    if (a0) { if (kedge) HHG2_L(false, true, true); else HHG2_L(false, true, false); }
    else { if (kedge) HHG2_L(false, false, true); else HHG2_L(false, false, false); }
  }
#undef HHG2_L
  const int64_t ng = (int64_t)h->gptr.size() - 1;
  if (ng > 0)
    hipLaunchKernelGGL(k_group2d<T>, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, st, h->d_gptr,
                       h->d_gslot, ng, y, h->n_slots);
  HHG_HIP(hipGetLastError());
  return HHG_OK;
}

}  // namespace hhg2

extern "C" {

int hhg2d_setup(const hhg2d_mesh_desc *mesh, const hhg_op_desc *op, hhg2d_handle *out) {
  using namespace hhg2;
  if (!mesh || !op || !out) return fail(HHG_EINVAL, "null argument");
  *out = nullptr;
  if (mesh->n_macro < 1 || !mesh->verts) return fail(HHG_EINVAL, "empty mesh");
  if (mesh->level < 1 || mesh->level > 13) return fail(HHG_EINVAL, "level outside 1..13");
  if (mesh->dirichlet != HHG_DIRICHLET_OUTER && mesh->dirichlet != HHG_DIRICHLET_NONE)
    return fail(HHG_EINVAL, "unknown Dirichlet mode");
  if ((op->corr != HHG_CORR_PHYSICAL && op->corr != HHG_CORR_NONE) ||
      (op->khat != HHG_KHAT_PATCH && op->khat != HHG_KHAT_EDGE) ||
      (op->iface != HHG_IFACE_SYMMETRIC && op->iface != HHG_IFACE_ROWWISE && op->iface != HHG_IFACE_ZEROSUM))
    return fail(HHG_EINVAL, "unknown operator option");
  auto *h = new (std::nothrow) hhg2d_ctx();
  if (!h) return fail(HHG_EINVAL, "out of host memory");
  const int M = mesh->n_macro, n = 1 << mesh->level;
  h->n_macro = M;
  h->level = mesh->level;
  h->op = *op;
  h->verts.assign(mesh->verts, mesh->verts + 6 * M);
  const int64_t per = (int64_t)(n + 1) * (n + 2) / 2;
  h->n_slots = per * M;
  double scale = 1.0;
  for (double v : h->verts) scale = std::max(scale, std::fabs(v) + 1.0);
  const double q = scale * 1e-9 / n;
  auto key = [&](double x0, double x1) {
    return std::array<long long, 2>{std::llround(x0 / q), std::llround(x1 / q)};
  };
  // Dirichlet macro edges: met by one macro only
  std::map<std::array<long long, 4>, int> ecount;
  auto ekey = [&](int m, int a, int b) {
    const double *V = h->verts.data() + 6 * m;
    auto ka = key(V[2 * a], V[2 * a + 1]), kb = key(V[2 * b], V[2 * b + 1]);
    if (kb < ka) std::swap(ka, kb);
    return std::array<long long, 4>{ka[0], ka[1], kb[0], kb[1]};
  };
  for (int m = 0; m < M; ++m)
    for (int e = 0; e < 3; ++e) ecount[ekey(m, (e + 1) % 3, (e + 2) % 3)]++;
  // end points of Dirichlet edges: Dirichlet in every macro that has them
  std::map<std::array<long long, 2>, int> dvert;
  if (mesh->dirichlet == HHG_DIRICHLET_OUTER)
    for (int m = 0; m < M; ++m)
      for (int e = 0; e < 3; ++e)
        if (ecount[ekey(m, (e + 1) % 3, (e + 2) % 3)] == 1)
          for (int v : {(e + 1) % 3, (e + 2) % 3}) {
            const double *V = h->verts.data() + 6 * m;
            dvert[key(V[2 * v], V[2 * v + 1])] = 1;
          }
  h->macros.resize(M);
  h->c64.resize(M);
  std::map<std::array<long long, 2>, std::vector<int64_t>> copies;
  h->flags.assign(h->n_slots, 0);
  for (int m = 0; m < M; ++m) {
    Macro2D &mi = h->macros[m];
    mi.off = per * m;
    mi.n = n;
    mi.dmask = 0;
    const double *V = h->verts.data() + 6 * m;
    if (mesh->dirichlet == HHG_DIRICHLET_OUTER)
      for (int e = 0; e < 3; ++e) {
        if (ecount[ekey(m, (e + 1) % 3, (e + 2) % 3)] == 1) mi.dmask |= 1u << e;
        if (dvert.count(key(V[2 * e], V[2 * e + 1]))) mi.dmask |= 1u << (3 + e);
      }
    const double e1[2] = {(V[2] - V[0]) / n, (V[3] - V[1]) / n};
    const double e2[2] = {(V[4] - V[0]) / n, (V[5] - V[1]) / n};
    if (std::fabs(e1[0] * e2[1] - e1[1] * e2[0]) <= 0.0) {
      free_ctx(h);
      return fail(HHG_EINVAL, "degenerate macro triangle");
    }
    // constants: the six triangles around a node, vertices (0, da, db)
    Const2D<double> &C = h->c64[m];
    double B1[ND][3][3][4], B0[ND][3][3][4];
    for (int t = 0; t < ND; ++t) {
      double X[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
      for (int v = 1; v < 3; ++v) {
        const int d = TRI[t][v - 1];
        X[v][0] = DI[d] * e1[0] + DJ[d] * e2[0];
        X[v][1] = DI[d] * e1[1] + DJ[d] * e2[1];
      }
      elem_blocks(X, op->mu1, op->lam1, B1[t]);
      elem_blocks(X, op->mu0, op->lam0, B0[t]);
      for (int v = 0; v < 3; ++v)
        for (int c = 0; c < 4; ++c) {
          C.E1[t][v][c] = B1[t][0][v][c];
          C.E0[t][v][c] = B0[t][0][v][c];
        }
    }
    for (int d = 0; d < ND; ++d) {
      int ts[2], vs[2], cnt = 0;
      for (int t = 0; t < ND; ++t)
        for (int v = 1; v < 3; ++v)
          if (TRI[t][v - 1] == d) {
            ts[cnt] = t;
            vs[cnt] = v;
            ++cnt;
          }
      if (cnt != 2) {
        free_ctx(h);
        return fail(HHG_EINVAL, "lattice check: an edge without two elements");
      }
      const double *a = B1[ts[0]][0][vs[0]], *b = B1[ts[1]][0][vs[1]];
      C.S[d][0] = a[0] + b[0];
      C.S[d][1] = a[3] + b[3];
      C.S[d][2] = 0.5 * (a[1] + a[2]) + 0.5 * (b[1] + b[2]);
      for (int c = 0; c < 4; ++c) C.A0[d][c] = B0[ts[0]][0][vs[0]][c] + B0[ts[1]][0][vs[1]][c];
      // third vertices; (k_p1 - k_p2)/3 = kbar^t - kbar^{t^m} with t the first element
      C.p1[d] = TRI[ts[0]][2 - vs[0]];
      C.p2[d] = TRI[ts[1]][2 - vs[1]];
      if (C.p1[d] != P1[d] || C.p2[d] != P2[d]) {
        free_ctx(h);
        return fail(HHG_EINVAL, "lattice check: third vertices of an edge differ from the kernel's table");
      }
      // R = 1/2 (kbar^t - kbar^tm) asym(a_t) + 1/2 (kbar^tm - kbar^t) asym(a_tm),
      // asym(a_tm) = -asym(a_t): R = (k_p1 - k_p2)/3 asym(a_t); asym(a_t)[0][1] = (a[1] - a[2])/2
      C.c[d] = (a[1] - a[2]) / 6.0;
      if (std::fabs((a[1] - a[2]) + (b[1] - b[2])) > 1e-12 * (std::fabs(a[1]) + std::fabs(a[2]) + 1e-300)) {
        free_ctx(h);
        return fail(HHG_EINVAL, "lattice check: reflected elements of an edge do not mirror");
      }
    }
    for (int j = 0; j <= n; ++j)
      for (int i = 0; i + j <= n; ++i) {
        const int64_t s = mi.off + (int64_t)j * (n + 1) - (int64_t)j * (j - 1) / 2 + i;
        const bool onb = i == 0 || j == 0 || i + j == n;
        const bool dir = is_dirichlet(i, j, n, mi.dmask);
        h->flags[s] = (dir ? 1 : 0) | (onb ? 4 : 0);
        if (onb) {
          const double x0 = V[0] + i * e1[0] + j * e2[0], x1 = V[1] + i * e1[1] + j * e2[1];
          copies[key(x0, x1)].push_back(s);
        } else {
          h->flags[s] |= 2;
        }
      }
  }
  // copy groups (non-Dirichlet nodes with more than one copy) and owners
  h->gptr.assign(1, 0);
  int64_t unknown = 0;
  for (int64_t s = 0; s < h->n_slots; ++s)
    if ((h->flags[s] & 2) && !(h->flags[s] & 1)) ++unknown;
  for (auto &kv : copies) {
    auto &sl = kv.second;
    std::sort(sl.begin(), sl.end());
    const bool dir = h->flags[sl[0]] & 1;
    for (int64_t s : sl)
      if (((h->flags[s] & 1) != 0) != dir) {
        free_ctx(h);
        return fail(HHG_EINVAL, "copies of a node disagree on its Dirichlet status");
      }
    h->flags[sl[0]] |= 2;
    if (!dir) ++unknown;
    if (sl.size() > 1 && !dir) {
      for (int64_t s : sl) {
        h->flags[s] |= 8;
        h->gslot.push_back(s);
      }
      h->gptr.push_back((int64_t)h->gslot.size());
    }
  }
  h->n_unknown = unknown;
  for (int pass = 0; pass < 2; ++pass)
    for (int m = 0; m < M; ++m)
      for (int j = 0; j <= n; ++j)
        for (int i = 0; i + j <= n; ++i) {
          const bool onb = i == 0 || j == 0 || i + j == n;
          if (onb == (pass == 0)) h->pos.push_back(((int64_t)m << 40) | ((int64_t)j << 20) | i);
        }
  h->n_apos = (int64_t)h->pos.size();
  h->n_bpos = 0;
  for (int m = 0; m < M; ++m) h->n_bpos += 3 * (int64_t)n;
  *out = h;
  return HHG_OK;
}

int hhg2d_destroy(hhg2d_handle h) {
  hhg2::free_ctx(h);
  return HHG_OK;
}

int hhg2d_layout(hhg2d_handle h, int64_t *n_slots, int64_t *n_unknown) {
  if (!h || !n_slots || !n_unknown) return hhg::fail(HHG_EINVAL, "null argument");
  *n_slots = h->n_slots;
  *n_unknown = h->n_unknown;
  return HHG_OK;
}

int hhg2d_node_coords(hhg2d_handle h, double *xy) {
  if (!h || !xy) return hhg::fail(HHG_EINVAL, "null argument");
  const int n = 1 << h->level;
  const int64_t N = h->n_slots;
  for (int m = 0; m < h->n_macro; ++m) {
    const double *V = h->verts.data() + 6 * m;
    for (int j = 0; j <= n; ++j)
      for (int i = 0; i + j <= n; ++i) {
        const int64_t s = h->macros[m].off + (int64_t)j * (n + 1) - (int64_t)j * (j - 1) / 2 + i;
        for (int c = 0; c < 2; ++c)
          xy[c * N + s] = V[c] + ((double)i * (V[2 + c] - V[c]) + (double)j * (V[4 + c] - V[c])) / n;
      }
  }
  return HHG_OK;
}

int hhg2d_node_flags(hhg2d_handle h, uint8_t *flags) {
  if (!h || !flags) return hhg::fail(HHG_EINVAL, "null argument");
  std::copy(h->flags.begin(), h->flags.end(), flags);
  return HHG_OK;
}

int hhg2d_apply(hhg2d_handle h, int32_t prec, int32_t method, const void *x, const void *k, void *y,
                void *stream) {
  using namespace hhg2;
  if (!h || !x || !k || !y) return fail(HHG_EINVAL, "null argument");
  if (prec != HHG_F64 && prec != HHG_F32) return fail(HHG_EINVAL, "unknown precision");
  if (method != HHG_METHOD_SCALED && method != HHG_METHOD_ONTHEFLY)
    return fail(HHG_EINVAL, "unknown operator method");
  const uintptr_t al = prec == HHG_F64 ? 7 : 3;
  if (((uintptr_t)x | (uintptr_t)k | (uintptr_t)y) & al) return fail(HHG_EINVAL, "misaligned pointer");
  if (x == y || k == y) return fail(HHG_EINVAL, "y must not alias x or k");
  int rc = ensure_device(h);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  return prec == HHG_F64 ? apply_t<double>(h, method, static_cast<const double *>(x),
                                           static_cast<const double *>(k), static_cast<double *>(y), st)
                         : apply_t<float>(h, method, static_cast<const float *>(x),
                                          static_cast<const float *>(k), static_cast<float *>(y), st);
}

}  // extern "C"
