// Operator application kernels for gfx950.
//
// Interior rows (the hot path, Sec. 4: asymptotically all work is in macro
// interiors): for every macro-interior node i
//     y_i = sum_{d} S_{i,d} (x_{i+d} - x_i),
//     S_{i,d} = A0_d + khat_{i,d} Shat_d + sum_{v in H_d} (k_v - k_{v^m}) C^v_d,
// which is the Lemma (eqs. bilinearformscaling, patchmean, corrtermgeneral)
// in the ring form of Sec. 2.4 (eq. correctionterm3D), with the centre entry
// fixed by the zero row sum.  Opposite directions share Shat, so the
// symmetric part needs 7 instead of 14 block products.
//
// Work decomposition: a workgroup owns TPB consecutive positions of the
// in-plane layout (the same positions in every plane) and marches over a
// range of planes.  The positions +-1 and +-(s+1..s+2) around the chunk are
// staged, for planes k-1, k, k+1, in a rolling LDS buffer of (x0, x1, x2, k)
// records (two arrays of (x0, x1) and (x2, k) pairs), loaded with coalesced
// reads one plane ahead of the computation; Dirichlet values of x are zeroed while
// staging.  On-the-fly nodal integration (eq. nodalintegration) uses the same
// staging and loops over the 24 elements of the node.
#include <algorithm>

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

template <typename T, int METHOD, bool RESID, bool CORR, bool A0, int NW, int TPB>
__global__ __launch_bounds__(TPB) void k_interior(
    const MacroInfo *__restrict__ minfo, const StencilConst<T> *__restrict__ scs,
    const ElemConst<T> *__restrict__ ecs, const WorkItem *__restrict__ work,
    const T *__restrict__ x, const T *__restrict__ kc, const T *__restrict__ f,
    T *__restrict__ y, int64_t nn, int wl) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Pair<T> *bufA = reinterpret_cast<Pair<T> *>(smem_raw);   // 3 planes of (x0, x1)
  Pair<T> *bufB = bufA + 3 * wl;                             // 3 planes of (x2, k)

  const WorkItem w = work[blockIdx.x];
  if (w.macro < 0) return;                  // padding item of the XCD-aware order
  const MacroInfo mi = minfo[w.macro];
  const int n = mi.n;
  const int tid = threadIdx.x;
  const int p0 = w.chunk * TPB;
  const int p = p0 + tid;
  const int s = tri_root_dev(p);
  const int i = p - s * (s + 1) / 2;
  const int j = s - i;
  const int s_lo = tri_root_dev(p0);
  const int ws = max(0, p0 - s_lo - 1);

  // anti-diagonal / position of the window entries this thread stages
  int es[NW], ei[NW];
#pragma unroll
  for (int r = 0; r < NW; ++r) {
    const int q = ws + tid + r * TPB;
    const int sq = tri_root_dev(q);
    es[r] = sq;
    ei[r] = q - sq * (sq + 1) / 2;
  }

  const T *X0 = x + mi.off;
  const T *X1 = X0 + nn;
  const T *X2 = X1 + nn;
  const T *K = kc + mi.off;

  // plane kk of the window: global -> registers (Dirichlet values of x zeroed)
  Node4<T> pre[NW];
  auto fetch = [&](int kk) {
    const int ps = (int)tri(n + 1 - kk);
    const int64_t base = plane_base(n, kk);
#pragma unroll
    for (int r = 0; r < NW; ++r) {
      const int e = tid + r * TPB;
      const int q = ws + e;
      Node4<T> v;
      v.x0 = v.x1 = v.x2 = v.k = T(0);
      if (e < wl && q < ps) {
        const int64_t g = base + q;
        v.x0 = X0[g];
        v.x1 = X1[g];
        v.x2 = X2[g];
        v.k = K[g];
        const int z = zero_set(ei[r], es[r] - ei[r], kk, n);
        if ((mi.dmask >> z) & 1u) v.x0 = v.x1 = v.x2 = T(0);
      }
      pre[r] = v;
    }
  };
  // registers -> LDS slot of plane kk
  auto put = [&](int kk) {
    Pair<T> *da = bufA + (kk % 3) * wl;
    Pair<T> *db = bufB + (kk % 3) * wl;
#pragma unroll
    for (int r = 0; r < NW; ++r) {
      const int e = tid + r * TPB;
      if (e < wl) {
        da[e] = Pair<T>{pre[r].x0, pre[r].x1};
        db[e] = Pair<T>{pre[r].x2, pre[r].k};
      }
    }
  };

  fetch(w.ka - 1);
  put(w.ka - 1);
  fetch(w.ka);
  put(w.ka);
  fetch(w.ka + 1);
  put(w.ka + 1);
  __syncthreads();
  const int e0 = p - ws;
  const bool col_ok = (s >= 2) && (i >= 1) && (j >= 1);

  for (int kk = w.ka; kk < w.kb; ++kk) {
    // the plane needed by the next step is loaded while this one computes
    const bool more = kk + 2 <= w.kb;
    if (more) fetch(kk + 2);
    if (col_ok && s + kk <= n - 1) {
      const int om = ((kk + 2) % 3) * wl + e0;   // plane kk-1
      const int o0 = (kk % 3) * wl + e0;
      const int op = ((kk + 1) % 3) * wl + e0;
      auto rd = [&](int o) {
        const Pair<T> a = bufA[o], b = bufB[o];
        return Node4<T>{a.a, a.b, b.a, b.b};
      };
      const Node4<T> c = rd(o0);
      Node4<T> nb[NDIR];
#pragma unroll
      for (int d = 0; d < NDIR; ++d) {
        const int o = DIR_K[d] > 0 ? op : (DIR_K[d] < 0 ? om : o0);
        nb[d] = rd(o + dir_a(d) + dir_b(d) * s);
      }
      // LDS reads and the scalar loads of the stencil constants share one
      // wait counter: take all neighbour records before any constant load
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
      __builtin_amdgcn_sched_barrier(0);
      T y0 = T(0), y1 = T(0), y2 = T(0);
      if constexpr (METHOD == METHOD_SCALED) {
        const StencilConst<T> &sc = scs[w.macro];
#pragma unroll
        for (int pr = 0; pr < NPAIR; ++pr) {
          T z0 = T(0), z1 = T(0), z2 = T(0);
          T a0 = T(0), a1 = T(0), a2 = T(0);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int d = 2 * pr + h;
            const int np = DIR_NT[d] == 6 ? 3 : 2;
            const T dx0 = nb[d].x0 - c.x0, dx1 = nb[d].x1 - c.x1, dx2 = nb[d].x2 - c.x2;
            T ring = nb[RING_V[d][0]].k + nb[RING_VM[d][0]].k;
#pragma unroll
            for (int q = 1; q < np; ++q) ring += nb[RING_V[d][q]].k + nb[RING_VM[d][q]].k;
            const T wr = DIR_NT[d] == 6 ? sc.w_ring6 : sc.w_ring4;
            const T kh = fma(sc.w_end, c.k + nb[d].k, wr * ring);
            z0 = fma(kh, dx0, z0);
            z1 = fma(kh, dx1, z1);
            z2 = fma(kh, dx2, z2);
            if constexpr (A0) {
              a0 += dx0;
              a1 += dx1;
              a2 += dx2;
            }
            if constexpr (CORR) {
              T w0 = T(0), w1 = T(0), w2 = T(0);
#pragma unroll
              for (int q = 0; q < np; ++q) {
                const T dk = nb[RING_V[d][q]].k - nb[RING_VM[d][q]].k;
                w0 = fma(dk, sc.cax[d][q][0], w0);
                w1 = fma(dk, sc.cax[d][q][1], w1);
                w2 = fma(dk, sc.cax[d][q][2], w2);
              }
              cross_acc(w0, w1, w2, dx0, dx1, dx2, y0, y1, y2);
            }
          }
          sym_mv_acc(sc.shat[pr], z0, z1, z2, y0, y1, y2);
          if constexpr (A0) sym_mv_acc(sc.a0[pr], a0, a1, a2, y0, y1, y2);
        }
      } else {
        const ElemConst<T> &ec = ecs[w.macro];
#pragma unroll
        for (int t = 0; t < NTET; ++t) {
          const int v1 = TET_V[t][0], v2 = TET_V[t][1], v3 = TET_V[t][2];
          const T kb = T(0.25) * (c.k + nb[v1].k + nb[v2].k + nb[v3].k);
          T u0 = T(0), u1 = T(0), u2 = T(0);
          T q0 = T(0), q1 = T(0), q2 = T(0);
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) {
            const int v = TET_V[t][cc];
            const T d0 = nb[v].x0 - c.x0, d1 = nb[v].x1 - c.x1, d2 = nb[v].x2 - c.x2;
            const T *B = ec.b1[t][cc + 1];
            u0 = fma(B[0], d0, fma(B[1], d1, fma(B[2], d2, u0)));
            u1 = fma(B[3], d0, fma(B[4], d1, fma(B[5], d2, u1)));
            u2 = fma(B[6], d0, fma(B[7], d1, fma(B[8], d2, u2)));
            if constexpr (A0) {
              const T *C = ec.b0[t][cc + 1];
              q0 = fma(C[0], d0, fma(C[1], d1, fma(C[2], d2, q0)));
              q1 = fma(C[3], d0, fma(C[4], d1, fma(C[5], d2, q1)));
              q2 = fma(C[6], d0, fma(C[7], d1, fma(C[8], d2, q2)));
            }
          }
          y0 = fma(kb, u0, y0 + q0);
          y1 = fma(kb, u1, y1 + q1);
          y2 = fma(kb, u2, y2 + q2);
        }
      }
      const int64_t g = mi.off + plane_base(n, kk) + p;
      if constexpr (RESID) {
        y0 = f[g] - y0;
        y1 = f[g + nn] - y1;
        y2 = f[g + 2 * nn] - y2;
      }
      y[g] = y0;
      y[g + nn] = y1;
      y[g + 2 * nn] = y2;
    }
    __syncthreads();
    if (more) put(kk + 2);               // overwrites the slot of plane kk-1
    __syncthreads();
  }
}

// Rows of nodes on a macro boundary (Sec. 2.2).  Each copy of a node
// computes the partial row of its macro; copies are summed afterwards.
// ROWWISE: nodal integration for the whole row (also the on-the-fly method);
// otherwise scaled entries towards macro-interior neighbours and nodal
// entries towards macro-boundary neighbours and on the diagonal.  Every block
// holds nodes of one macro, so the macro's constants are uniform loads.
__device__ __forceinline__ int plane_base32(int n, int k) {
  const int a = n + 1, b = n + 1 - k;
  return a * (a + 1) * (a + 2) / 6 - b * (b + 1) * (b + 2) / 6;
}

template <typename T, bool RESID, bool ROWWISE, bool CORR>
__global__ __launch_bounds__(BOUNDARY_BLOCK) void k_boundary_rows(
    const MacroInfo *__restrict__ minfo, const StencilConst<T> *__restrict__ scs,
    const ElemConst<T> *__restrict__ ecs, const int32_t *__restrict__ bijk,
    const int32_t *__restrict__ bblk, const uint8_t *__restrict__ flags,
    const T *__restrict__ x, const T *__restrict__ kc, const T *__restrict__ f,
    T *__restrict__ y, int64_t nn) {
  const int m = bblk[blockIdx.x];
  const int packed = bijk[(int64_t)blockIdx.x * BOUNDARY_BLOCK + threadIdx.x];
  if (packed < 0) return;
  const MacroInfo mi = minfo[m];
  const int n = mi.n;
  const int i = packed & 1023, j = (packed >> 10) & 1023, k = (packed >> 20) & 1023;
  const T *X0 = x + mi.off;
  const T *X1 = X0 + nn;
  const T *X2 = X1 + nn;
  const T *KC = kc + mi.off;
  const int lslot = plane_base32(n, k) + (i + j) * (i + j + 1) / 2 + i;
  const int64_t slot = mi.off + lslot;
  // neighbour data (inside the macro, on its boundary, Dirichlet-masked x)
  bool in[NDIR], onb[NDIR];
  T nx0[NDIR], nx1[NDIR], nx2[NDIR], nk[NDIR];
#pragma unroll
  for (int d = 0; d < NDIR; ++d) {
    const int a = i + DIR_I[d], bb = j + DIR_J[d], cc = k + DIR_K[d];
    in[d] = a >= 0 && bb >= 0 && cc >= 0 && a + bb + cc <= n;
    onb[d] = false;
    nx0[d] = nx1[d] = nx2[d] = nk[d] = T(0);
    if (in[d]) {
      const int zz = zero_set(a, bb, cc, n);
      onb[d] = zz != 0;
      const int ls = plane_base32(n, cc) + (a + bb) * (a + bb + 1) / 2 + a;
      nk[d] = KC[ls];
      if (!((mi.dmask >> zz) & 1u)) {
        nx0[d] = X0[ls];
        nx1[d] = X1[ls];
        nx2[d] = X2[ls];
      }
    }
  }
  const T ci0 = X0[lslot], ci1 = X1[lslot], ci2 = X2[lslot];
  const T ck = KC[lslot];
  const ElemConst<T> &ec = ecs[m];
  T y0 = T(0), y1 = T(0), y2 = T(0);
#pragma unroll
  for (int t = 0; t < NTET; ++t) {
    const int v1 = TET_V[t][0], v2 = TET_V[t][1], v3 = TET_V[t][2];
    if (!(in[v1] && in[v2] && in[v3])) continue;
    const T kb = T(0.25) * (ck + nk[v1] + nk[v2] + nk[v3]);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      T d0, d1, d2;
      if (c == 0) {
        d0 = ci0; d1 = ci1; d2 = ci2;
      } else {
        const int v = TET_V[t][c - 1];
        if (!ROWWISE && !onb[v]) continue;   // scaled entry handled below
        d0 = nx0[v]; d1 = nx1[v]; d2 = nx2[v];
      }
      const T *B1 = ec.b1[t][c];
      const T *B0 = ec.b0[t][c];
      y0 += fma(kb, B1[0], B0[0]) * d0 + fma(kb, B1[1], B0[1]) * d1 + fma(kb, B1[2], B0[2]) * d2;
      y1 += fma(kb, B1[3], B0[3]) * d0 + fma(kb, B1[4], B0[4]) * d1 + fma(kb, B1[5], B0[5]) * d2;
      y2 += fma(kb, B1[6], B0[6]) * d0 + fma(kb, B1[7], B0[7]) * d1 + fma(kb, B1[8], B0[8]) * d2;
    }
  }
  if (!ROWWISE) {
    const StencilConst<T> &sc = scs[m];
#pragma unroll
    for (int d = 0; d < NDIR; ++d) {
      if (!in[d] || onb[d]) continue;
      const int np = DIR_NT[d] == 6 ? 3 : 2;
      T ring = T(0);
#pragma unroll
      for (int q = 0; q < np; ++q) ring += nk[RING_V[d][q]] + nk[RING_VM[d][q]];
      const T wr = DIR_NT[d] == 6 ? sc.w_ring6 : sc.w_ring4;
      const T kh = fma(sc.w_end, ck + nk[d], wr * ring);
      const T *S = sc.shat[d >> 1];
      const T *A = sc.a0[d >> 1];
      const T z0v = kh * nx0[d], z1v = kh * nx1[d], z2v = kh * nx2[d];
      sym_mv_acc(S, z0v, z1v, z2v, y0, y1, y2);
      sym_mv_acc(A, nx0[d], nx1[d], nx2[d], y0, y1, y2);
      if (CORR) {
        T w0 = T(0), w1 = T(0), w2 = T(0);
#pragma unroll
        for (int q = 0; q < np; ++q) {
          const T dk = nk[RING_V[d][q]] - nk[RING_VM[d][q]];
          w0 = fma(dk, sc.cax[d][q][0], w0);
          w1 = fma(dk, sc.cax[d][q][1], w1);
          w2 = fma(dk, sc.cax[d][q][2], w2);
        }
        cross_acc(w0, w1, w2, nx0[d], nx1[d], nx2[d], y0, y1, y2);
      }
    }
  }
  // a node with copies in other macros is completed by the group sum
  if (RESID && !(flags[slot] & 8)) {
    y0 = f[slot] - y0;
    y1 = f[slot + nn] - y1;
    y2 = f[slot + 2 * nn] - y2;
  }
  y[slot] = y0;
  y[slot + nn] = y1;
  y[slot + 2 * nn] = y2;
}

// Sum of the partial rows of all copies of an interface node; the total (or
// f minus it) is written to every copy, keeping the output consistent.
// Threads past the groups write the zero rows of the Dirichlet slots.
template <typename T, bool RESID>
__global__ __launch_bounds__(256) void k_finish(const int64_t *__restrict__ ptr,
                                                const int64_t *__restrict__ slots, int64_t ng,
                                                const int64_t *__restrict__ dslot, int64_t nd,
                                                const T *__restrict__ f, T *__restrict__ y,
                                                int64_t nn) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (item, component)
  const int64_t g = t / 3;
  const int c = (int)(t - 3 * g);
  if (g < ng) {
    const int64_t a = ptr[g], b = ptr[g + 1];
    T sum = T(0);
    for (int64_t q = a; q < b; ++q) sum += y[c * nn + slots[q]];
    if (RESID) sum = f[c * nn + slots[a]] - sum;
    for (int64_t q = a; q < b; ++q) y[c * nn + slots[q]] = sum;
  } else if (g - ng < nd) {
    y[c * nn + dslot[g - ng]] = T(0);
  }
}

// ------------------------------------------------------------ launchers
namespace {

template <typename T>
const StencilConst<T> *sc_ptr(hhg_ctx *h);
template <>
const StencilConst<double> *sc_ptr<double>(hhg_ctx *h) { return h->d_sc64; }
template <>
const StencilConst<float> *sc_ptr<float>(hhg_ctx *h) { return h->d_sc32; }
template <typename T>
const ElemConst<T> *ec_ptr(hhg_ctx *h);
template <>
const ElemConst<double> *ec_ptr<double>(hhg_ctx *h) { return h->d_ec64; }
template <>
const ElemConst<float> *ec_ptr<float>(hhg_ctx *h) { return h->d_ec32; }

template <typename T, int METHOD, bool RESID, bool CORR, bool A0, int NW, int TPB>
int launch_interior_nw(hhg_ctx *h, const T *x, const T *k, const T *f, T *y, hipStream_t st) {
  const int wl = h->wl_max;
  const size_t lds = 6 * (size_t)wl * sizeof(Pair<T>);
  auto kern = k_interior<T, METHOD, RESID, CORR, A0, NW, TPB>;
  if (lds > 65536) HHG_HIP(hipFuncSetAttribute((const void *)kern,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  ProfScope prof(h, METHOD == METHOD_SCALED ? HHG_K_INTERIOR_SCALED : HHG_K_INTERIOR_ONTHEFLY, st);
  hipLaunchKernelGGL(kern, dim3(h->n_work), dim3(TPB), lds, st, h->d_minfo, sc_ptr<T>(h),
                     ec_ptr<T>(h), h->d_work, x, k, f, y, h->n_nodes, wl);
  HHG_HIP(hipGetLastError());
  return HHG_OK;
}

// Positions per work item (= threads): 256 or 512; window entries per
// thread: up to 2 (levels <= 7 with 256, <= 8 with 512) or up to 6.
template <typename T, int METHOD, bool RESID, bool CORR, bool A0>
int launch_interior(hhg_ctx *h, const T *x, const T *k, const T *f, T *y, hipStream_t st) {
  if (h->n_work == 0) return HHG_OK;
  const int nw = (h->wl_max + h->chunk - 1) / h->chunk;
  if (h->chunk == 256) {
    if (nw <= 2) return launch_interior_nw<T, METHOD, RESID, CORR, A0, 2, 256>(h, x, k, f, y, st);
    if (nw <= 6) return launch_interior_nw<T, METHOD, RESID, CORR, A0, 6, 256>(h, x, k, f, y, st);
  } else if (h->chunk == 512) {
    if (nw <= 2) return launch_interior_nw<T, METHOD, RESID, CORR, A0, 2, 512>(h, x, k, f, y, st);
    if (nw <= 3) return launch_interior_nw<T, METHOD, RESID, CORR, A0, 3, 512>(h, x, k, f, y, st);
  }
  return fail(HHG_EINVAL, "interior window larger than supported");
}

template <typename T, int METHOD, bool RESID>
int launch_interior_v(hhg_ctx *h, const T *x, const T *k, const T *f, T *y, hipStream_t st) {
  const bool corr = METHOD == METHOD_SCALED && h->op.corr == HHG_CORR_PHYSICAL;
  const bool a0 = h->op.mu0 != 0.0 || h->op.lam0 != 0.0;
  if (corr && a0) return launch_interior<T, METHOD, RESID, true, true>(h, x, k, f, y, st);
  if (corr) return launch_interior<T, METHOD, RESID, true, false>(h, x, k, f, y, st);
  if (a0) return launch_interior<T, METHOD, RESID, false, true>(h, x, k, f, y, st);
  return launch_interior<T, METHOD, RESID, false, false>(h, x, k, f, y, st);
}

template <typename T, bool RESID>
int launch_boundary(hhg_ctx *h, int method, const T *x, const T *k, const T *f, T *y,
                    hipStream_t st) {
  const bool rowwise = method == METHOD_ONTHEFLY || h->op.iface == HHG_IFACE_ROWWISE;
  const bool corr = h->op.corr == HHG_CORR_PHYSICAL;
  if (!h->bblk.empty()) {
    const dim3 grid((unsigned)h->bblk.size());
#define HHG_LB(RW, CR)                                                                           \
  hipLaunchKernelGGL((k_boundary_rows<T, RESID, RW, CR>), grid, dim3(BOUNDARY_BLOCK), 0, st,    \
                     h->d_minfo, sc_ptr<T>(h), ec_ptr<T>(h), h->d_bijk, h->d_bblk, h->d_flags, x, \
                     k, f, y, h->n_nodes)
    ProfScope prof(h, HHG_K_BOUNDARY_ROWS, st);
    if (rowwise)
      HHG_LB(true, false);
    else if (corr)
      HHG_LB(false, true);
    else
      HHG_LB(false, false);
#undef HHG_LB
    HHG_HIP(hipGetLastError());
  }
  const int64_t nd = (int64_t)h->dslot.size();
  const int64_t total = 3 * (h->n_grp + nd);
  if (total > 0) {
    const dim3 g2((unsigned)((total + 255) / 256));
    ProfScope prof(h, HHG_K_GROUP_SUM, st);
    hipLaunchKernelGGL((k_finish<T, RESID>), g2, dim3(256), 0, st, h->d_grp_ptr, h->d_grp_slot,
                       h->n_grp, h->d_dslot, nd, f, y, h->n_nodes);
    HHG_HIP(hipGetLastError());
  }
  return HHG_OK;
}

// Interior rows run on the caller's stream, macro-boundary rows and the copy
// sums on the handle's side stream (they write disjoint slots), joined back
// before the call's work is complete on the caller's stream.
template <typename T>
int apply_t(hhg_ctx *h, int method, const T *f, const T *x, const T *k, T *y, hipStream_t st) {
  HHG_HIP(hipEventRecord(h->ev_fork, st));
  HHG_HIP(hipStreamWaitEvent(h->side, h->ev_fork, 0));
  int rc;
  if (f) {
    rc = method == METHOD_SCALED ? launch_interior_v<T, METHOD_SCALED, true>(h, x, k, f, y, st)
                                 : launch_interior_v<T, METHOD_ONTHEFLY, true>(h, x, k, f, y, st);
    if (!rc) rc = launch_boundary<T, true>(h, method, x, k, f, y, h->side);
  } else {
    rc = method == METHOD_SCALED ? launch_interior_v<T, METHOD_SCALED, false>(h, x, k, f, y, st)
                                 : launch_interior_v<T, METHOD_ONTHEFLY, false>(h, x, k, f, y, st);
    if (!rc) rc = launch_boundary<T, false>(h, method, x, k, f, y, h->side);
  }
  HHG_HIP(hipEventRecord(h->ev_join, h->side));
  HHG_HIP(hipStreamWaitEvent(st, h->ev_join, 0));
  return rc;
}

bool overlaps(const void *a, const void *b, size_t bytes) {
  const char *pa = (const char *)a, *pb = (const char *)b;
  return pa < pb + bytes && pb < pa + bytes;
}

}  // namespace

int apply_entry(hhg_ctx *h, int prec, int method, const void *f, const void *x, const void *k,
                void *y, void *stream) {
  if (!h) return fail(HHG_EINVAL, "null handle");
  if (!x || !k || !y) return fail(HHG_EINVAL, "null vector pointer");
  if (prec != HHG_F64 && prec != HHG_F32) return fail(HHG_EINVAL, "unknown precision");
  if (method != METHOD_SCALED && method != METHOD_ONTHEFLY) return fail(HHG_EINVAL, "unknown method");
  const uintptr_t al = (uintptr_t)x | (uintptr_t)k | (uintptr_t)y | (uintptr_t)f;
  if (al & 15) return fail(HHG_EINVAL, "vector pointers must be 16-byte aligned");
  const size_t vb = 3 * (size_t)h->n_nodes * (prec == HHG_F64 ? 8 : 4);
  if (overlaps(x, y, vb) || (f && overlaps(f, y, vb)))
    return fail(HHG_EINVAL, "output overlaps an input vector");
  int rc = ensure_device(h);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (prec == HHG_F64)
    return apply_t<double>(h, method, (const double *)f, (const double *)x, (const double *)k,
                           (double *)y, st);
  return apply_t<float>(h, method, (const float *)f, (const float *)x, (const float *)k,
                        (float *)y, st);
}

}  // namespace hhg

extern "C" {

int hhg_apply_scaled(hhg_handle h, int32_t prec, const void *x, const void *k, void *y,
                     void *stream) {
  return hhg::apply_entry(h, prec, hhg::METHOD_SCALED, nullptr, x, k, y, stream);
}

int hhg_apply_onthefly(hhg_handle h, int32_t prec, const void *x, const void *k, void *y,
                       void *stream) {
  return hhg::apply_entry(h, prec, hhg::METHOD_ONTHEFLY, nullptr, x, k, y, stream);
}

int hhg_residual(hhg_handle h, int32_t prec, int32_t method, const void *f, const void *x,
                 const void *k, void *r, void *stream) {
  if (!f) return hhg::fail(HHG_EINVAL, "null right-hand side");
  return hhg::apply_entry(h, prec, method, f, x, k, r, stream);
}

}  // extern "C"
