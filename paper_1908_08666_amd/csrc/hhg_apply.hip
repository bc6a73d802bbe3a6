// Operator application: macro-boundary rows, copy sums, launch sequence
// and the C ABI entry points.  The interior-row kernels (the hot path) live in
// hhg_interior.h and are compiled per element type and method.
#include <algorithm>

#include "hhg_device.h"

namespace hhg {

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

// One macro-boundary row of macro m at (i, j, k): the neighbours' positions
// are classified at run time (inside the macro, on its boundary) and
// Dirichlet values of x are masked.
template <typename T, bool RESID, bool ROWWISE, bool CORR, bool A0>
__device__ __forceinline__ void boundary_row(const MacroInfo &mi, const StencilConst<T> &sc,
                                             const ElemConst<T> &ec, int i, int j, int k,
                                             const uint8_t *__restrict__ flags,
                                             const T *__restrict__ x, const T *__restrict__ kc,
                                             const T *__restrict__ f, T *__restrict__ y,
                                             int64_t nn) {
  const int n = mi.n;
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
  T y0 = T(0), y1 = T(0), y2 = T(0);
#pragma unroll
  for (int t = 0; t < NTET; ++t) {
    const int v1 = TET_V[t][0], v2 = TET_V[t][1], v3 = TET_V[t][2];
    if (!(in[v1] && in[v2] && in[v3])) continue;
    const T kb = T(0.25) * (ck + nk[v1] + nk[v2] + nk[v3]);
    // this element's part of the row: kb (B1 x) + B0 x over its vertices
    T u0 = T(0), u1 = T(0), u2 = T(0), q0 = T(0), q1 = T(0), q2 = T(0);
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
      u0 = fma(B1[0], d0, fma(B1[1], d1, fma(B1[2], d2, u0)));
      u1 = fma(B1[3], d0, fma(B1[4], d1, fma(B1[5], d2, u1)));
      u2 = fma(B1[6], d0, fma(B1[7], d1, fma(B1[8], d2, u2)));
      if constexpr (A0) {
        const T *B0 = ec.b0[t][c];
        q0 = fma(B0[0], d0, fma(B0[1], d1, fma(B0[2], d2, q0)));
        q1 = fma(B0[3], d0, fma(B0[4], d1, fma(B0[5], d2, q1)));
        q2 = fma(B0[6], d0, fma(B0[7], d1, fma(B0[8], d2, q2)));
      }
    }
    y0 = fma(kb, u0, y0 + q0);
    y1 = fma(kb, u1, y1 + q1);
    y2 = fma(kb, u2, y2 + q2);
  }
  if (!ROWWISE) {
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
      const T z0v = kh * nx0[d], z1v = kh * nx1[d], z2v = kh * nx2[d];
      sym_mv_acc(S, z0v, z1v, z2v, y0, y1, y2);
      if constexpr (A0) sym_mv_acc(sc.a0[d >> 1], nx0[d], nx1[d], nx2[d], y0, y1, y2);
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

// Rows of nodes on a macro boundary (Sec. 2.2).  Each copy of a node
// computes the partial row of its macro; copies are summed afterwards.
// ROWWISE: nodal integration for the whole row (also the on-the-fly method);
// otherwise scaled entries towards macro-interior neighbours and nodal
// entries towards macro-boundary neighbours and on the diagonal.  Every block
// holds nodes of one macro (bblk), ordered by the boundary primitive they lie
// on, so that a wave rarely diverges; Dirichlet slots of the macro's boundary
// (flag bit 30 in bijk) get their zero rows here as well.
template <typename T, bool RESID, bool ROWWISE, bool CORR, bool A0>
__global__ __launch_bounds__(BOUNDARY_BLOCK) void k_boundary_rows(
    const MacroInfo *__restrict__ minfo, const StencilConst<T> *__restrict__ scs,
    const ElemConst<T> *__restrict__ ecs, const int32_t *__restrict__ bijk,
    const int32_t *__restrict__ bblk, const uint8_t *__restrict__ flags,
    const T *__restrict__ x, const T *__restrict__ kc, const T *__restrict__ f,
    T *__restrict__ y, int64_t nn) {
  // the macro's constants are staged in LDS and read from there by every
  // row (scalar loads of 15 KB of constants would not fit the scalar
  // registers); all lanes read the same address, so the reads broadcast
  __shared__ __align__(16) unsigned char cbuf[sizeof(ElemConst<T>) + sizeof(StencilConst<T>)];
  const int m = bblk[blockIdx.x];
  {
    static_assert(sizeof(ElemConst<T>) % 16 == 0 && sizeof(StencilConst<T>) % 4 == 0, "table sizes");
    const uint4 *ge = reinterpret_cast<const uint4 *>(ecs + m);
    const uint32_t *gs = reinterpret_cast<const uint32_t *>(scs + m);
    uint4 *le = reinterpret_cast<uint4 *>(cbuf);
    uint32_t *ls = reinterpret_cast<uint32_t *>(cbuf + sizeof(ElemConst<T>));
    for (int q = threadIdx.x; q < (int)(sizeof(ElemConst<T>) / 16); q += BOUNDARY_BLOCK) le[q] = ge[q];
    for (int q = threadIdx.x; q < (int)(sizeof(StencilConst<T>) / 4); q += BOUNDARY_BLOCK) ls[q] = gs[q];
  }
  __syncthreads();
  const int packed = bijk[(int64_t)blockIdx.x * BOUNDARY_BLOCK + threadIdx.x];
  if (packed < 0) return;
  const MacroInfo mi = minfo[m];
  const int i = packed & 1023, j = (packed >> 10) & 1023, k = (packed >> 20) & 1023;
  const ElemConst<T> &ec = *reinterpret_cast<const ElemConst<T> *>(cbuf);
  const StencilConst<T> &sc = *reinterpret_cast<const StencilConst<T> *>(cbuf + sizeof(ElemConst<T>));
  if (packed & (1 << 30)) {                // Dirichlet slot: its row is zero
    const int64_t slot = mi.off + plane_base32(mi.n, k) + (i + j) * (i + j + 1) / 2 + i;
    y[slot] = T(0);
    y[slot + nn] = T(0);
    y[slot + 2 * nn] = T(0);
    return;
  }
  boundary_row<T, RESID, ROWWISE, CORR, A0>(mi, sc, ec, i, j, k, flags, x, kc, f, y, nn);
}

// Sum of the partial rows of all copies of an interface node; the total (or
// f minus it) is written to every copy, keeping the output consistent.  One
// thread per group handles the three components (the copy list is read once).
template <typename T, bool RESID>
__global__ __launch_bounds__(256) void k_finish(const int64_t *__restrict__ ptr,
                                                const int64_t *__restrict__ slots, int64_t ng,
                                                const T *__restrict__ f, T *__restrict__ y,
                                                int64_t nn) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  const int64_t a = ptr[g], b = ptr[g + 1];
  T s0 = T(0), s1 = T(0), s2 = T(0);
  for (int64_t q = a; q < b; ++q) {
    const int64_t sl = slots[q];
    s0 += y[sl];
    s1 += y[nn + sl];
    s2 += y[2 * nn + sl];
  }
  if (RESID) {
    const int64_t s = slots[a];
    s0 = f[s] - s0;
    s1 = f[nn + s] - s1;
    s2 = f[2 * nn + s] - s2;
  }
  for (int64_t q = a; q < b; ++q) {
    const int64_t sl = slots[q];
    y[sl] = s0;
    y[nn + sl] = s1;
    y[2 * nn + sl] = s2;
  }
}

// ------------------------------------------------------------ launchers
namespace {

template <typename T, bool RESID>
int launch_boundary(hhg_ctx *h, int method, const T *x, const T *k, const T *f, T *y,
                    hipStream_t st) {
  const bool rowwise = method == METHOD_ONTHEFLY || h->op.iface == HHG_IFACE_ROWWISE;
  const bool corr = h->op.corr == HHG_CORR_PHYSICAL;
  if (!h->bblk.empty()) {
    const dim3 grid((unsigned)h->bblk.size());
#define HHG_LB(RW, CR, A0)                                                                       \
  hipLaunchKernelGGL((k_boundary_rows<T, RESID, RW, CR, A0>), grid, dim3(BOUNDARY_BLOCK), 0, st, \
                     h->d_minfo, sc_ptr<T>(h), ec_ptr<T>(h), h->d_bijk, h->d_bblk, h->d_flags, x, \
                     k, f, y, h->n_nodes)
    ProfScope prof(h, HHG_K_BOUNDARY_ROWS, st);
    const bool a0 = h->op.mu0 != 0.0 || h->op.lam0 != 0.0;
    if (rowwise) {
      if (a0) HHG_LB(true, false, true); else HHG_LB(true, false, false);
    } else if (corr) {
      if (a0) HHG_LB(false, true, true); else HHG_LB(false, true, false);
    } else {
      if (a0) HHG_LB(false, false, true); else HHG_LB(false, false, false);
    }
#undef HHG_LB
    HHG_HIP(hipGetLastError());
  }
  const int64_t total = h->n_grp;
  if (total > 0) {
    const dim3 g2((unsigned)((total + 255) / 256));
    ProfScope prof(h, HHG_K_GROUP_SUM, st);
    hipLaunchKernelGGL((k_finish<T, RESID>), g2, dim3(256), 0, st, h->d_grp_ptr, h->d_grp_slot,
                       h->n_grp, f, y, h->n_nodes);
    HHG_HIP(hipGetLastError());
  }
  return HHG_OK;
}

// Interior rows run on the caller's stream, macro-boundary rows and the copy
// sums on the handle's side stream (they write disjoint slots), joined back
// before the call's work is complete on the caller's stream.
template <typename T>
int apply_t(hhg_ctx *h, int method, const T *f, const T *x, const T *k, T *y, hipStream_t st) {
  if (h->serial_apply) {                    // one stream: clean per-kernel timings
    int rc = method == METHOD_SCALED
                 ? (f ? launch_interior_v<T, METHOD_SCALED, true>(h, x, k, f, y, st)
                      : launch_interior_v<T, METHOD_SCALED, false>(h, x, k, f, y, st))
                 : (f ? launch_interior_v<T, METHOD_ONTHEFLY, true>(h, x, k, f, y, st)
                      : launch_interior_v<T, METHOD_ONTHEFLY, false>(h, x, k, f, y, st));
    if (rc) return rc;
    return f ? launch_boundary<T, true>(h, method, x, k, f, y, st)
             : launch_boundary<T, false>(h, method, x, k, f, y, st);
  }
  // the small boundary launch goes first: queued behind the interior launch,
  // which fills every compute unit, it would only start as that one drains
  HHG_HIP(hipEventRecord(h->ev_fork, st));
  HHG_HIP(hipStreamWaitEvent(h->side, h->ev_fork, 0));
  int rc;
  if (f) {
    rc = launch_boundary<T, true>(h, method, x, k, f, y, h->side);
    if (!rc)
      rc = method == METHOD_SCALED ? launch_interior_v<T, METHOD_SCALED, true>(h, x, k, f, y, st)
                                   : launch_interior_v<T, METHOD_ONTHEFLY, true>(h, x, k, f, y, st);
  } else {
    rc = launch_boundary<T, false>(h, method, x, k, f, y, h->side);
    if (!rc)
      rc = method == METHOD_SCALED ? launch_interior_v<T, METHOD_SCALED, false>(h, x, k, f, y, st)
                                   : launch_interior_v<T, METHOD_ONTHEFLY, false>(h, x, k, f, y, st);
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

// Operator application for the solvers: no argument checks beyond the
// device upload (the caller owns consistent, aligned, non-overlapping data).
int apply_internal(hhg_ctx *h, int prec, int method, const void *f, const void *x, const void *k,
                   void *y, hipStream_t st) {
  int rc = ensure_device(h);
  if (rc) return rc;
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
