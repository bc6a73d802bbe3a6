// Interior-row kernels (the hot path) and their launchers.
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
#pragma once

#include "hhg_device.h"

namespace hhg {

// Row i of the operator applied to x for a macro-interior node from its
// 15-point neighbourhood: physical scaling (METHOD_SCALED) or nodal
// integration over the 24 elements (METHOD_ONTHEFLY).
template <typename T, int METHOD, bool CORR, bool A0>
__device__ __forceinline__ void node_rows(const Node4<T> &c, const Node4<T> (&nb)[NDIR],
                                          const StencilConst<T> &sc, const ElemConst<T> &ec,
                                          T &y0, T &y1, T &y2) {
  y0 = T(0);
  y1 = T(0);
  y2 = T(0);
  if constexpr (METHOD == METHOD_SCALED) {
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
            w0 = fma(dk, sc.pr[pr].cax[q][0], w0);
            w1 = fma(dk, sc.pr[pr].cax[q][1], w1);
            w2 = fma(dk, sc.pr[pr].cax[q][2], w2);
          }
          cross_acc(w0, w1, w2, dx0, dx1, dx2, y0, y1, y2);
        }
      }
      sym_mv_acc(sc.pr[pr].shat, z0, z1, z2, y0, y1, y2);
      if constexpr (A0) sym_mv_acc(sc.pr[pr].a0, a0, a1, a2, y0, y1, y2);
      // one pair's constants at a time: loaded all at once they would not
      // fit the scalar registers
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
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
}

// One work item (a slab of NSUB * TPB positions over planes [ka, kb) of one
// macro) computed by the whole workgroup, NSUB positions per thread (p0 + tid
// + u TPB); every thread must call it (barriers).
template <typename T, int METHOD, int OUT, bool CORR, bool A0, int NW, int TPB, int NSUB>
__device__ __forceinline__ void interior_item(
    const WorkItem w, unsigned char *smem_raw,
    const MacroInfo *__restrict__ minfo, const StencilConst<T> *__restrict__ scs,
    const ElemConst<T> *__restrict__ ecs,
    const T *__restrict__ x, const T *__restrict__ kc, const T *__restrict__ f,
    T *__restrict__ y, int64_t nn, int wl, double *__restrict__ part, int item,
    const T *__restrict__ P, T omega, T *__restrict__ xo) {
  static_assert(OUT >= 0 && OUT <= 3,
                "output: 0 apply, 1 residual, 2 apply and (x, y) partial sum, 3 smoothing step");
  Pair<T> *bufA = reinterpret_cast<Pair<T> *>(smem_raw);   // 3 planes of (x0, x1)
  Pair<T> *bufB = bufA + 3 * wl;                             // 3 planes of (x2, k)
  const MacroInfo mi = minfo[w.macro];
  const int n = mi.n;
  const int tid = threadIdx.x;
  const int p0 = w.chunk * (TPB * NSUB);
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

  // plane kk of the window: global -> registers.  Nothing here reads the
  // loaded values, so the loads stay in flight until put() (a select on
  // them at this point would make the wave wait for them at once).
  auto fetch = [&](int kk, Node4<T>(&dst)[NW]) {
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
      }
      dst[r] = v;
    }
  };
  // registers -> LDS slot of plane kk, Dirichlet values of x zeroed
  auto put = [&](int kk, const Node4<T>(&src)[NW]) {
    Pair<T> *da = bufA + (kk % 3) * wl;
    Pair<T> *db = bufB + (kk % 3) * wl;
#pragma unroll
    for (int r = 0; r < NW; ++r) {
      const int e = tid + r * TPB;
      if (e < wl) {
        const int z = zero_set(ei[r], es[r] - ei[r], kk, n);
        const bool dz = (mi.dmask >> z) & 1u;
        da[e] = Pair<T>{dz ? T(0) : src[r].x0, dz ? T(0) : src[r].x1};
        db[e] = Pair<T>{dz ? T(0) : src[r].x2, src[r].k};
      }
    }
  };

  double dot_acc = 0.0;                  // OUT == 2: this thread's rows of (x, A x)
  Node4<T> pre[NW];
  {
    // the first three planes in one round of loads
    Node4<T> pa[NW], pb[NW];
    fetch(w.ka - 1, pa);
    fetch(w.ka, pb);
    fetch(w.ka + 1, pre);
    put(w.ka - 1, pa);
    put(w.ka, pb);
    put(w.ka + 1, pre);
  }
  __syncthreads();
  // the positions of this thread: anti-diagonal, interior column
  int ps_[NSUB], ss_[NSUB];
  bool col_ok[NSUB];
#pragma unroll
  for (int u = 0; u < NSUB; ++u) {
    const int p = p0 + tid + u * TPB;
    const int sp = tri_root_dev(p);
    const int ip = p - sp * (sp + 1) / 2;
    ps_[u] = p;
    ss_[u] = sp;
    col_ok[u] = (sp >= 2) && (ip >= 1) && (sp - ip >= 1);
  }

  // Per plane: loads of plane kk+2 are issued first and land while plane kk
  // computes; the results of plane kk are stored only after plane kk+2 has
  // been written to LDS, so that waiting for those loads never waits for
  // stores issued a moment earlier (both share one counter).
  for (int kk = w.ka; kk < w.kb; ++kk) {
    const bool more = kk + 2 <= w.kb;
    if (more) fetch(kk + 2, pre);
    const int64_t gk = mi.off + plane_base(n, kk);
    T yv[NSUB][3];
    bool act[NSUB];
    // smoothing step: b and the node's block are loaded before the stencil,
    // so that their latency hides behind it (the kernel runs at two waves
    // per SIMD either way)
    T sb[NSUB][9];
#pragma unroll
    for (int u = 0; u < NSUB; ++u) {
      const int p = ps_[u], sp = ss_[u];
      act[u] = col_ok[u] && sp + kk <= n - 1;
      yv[u][0] = yv[u][1] = yv[u][2] = T(0);
      if constexpr (OUT == 3) {
        if (act[u]) {
          const int64_t g = gk + p;
#pragma unroll
          for (int c = 0; c < 3; ++c) sb[u][c] = f[g + c * nn];
#pragma unroll
          for (int c = 0; c < 6; ++c) sb[u][3 + c] = P[g + c * nn];
        }
      }
      if (act[u]) {
        const int e0 = p - ws;
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
          nb[d] = rd(o + dir_a(d) + dir_b(d) * sp);
        }
        // LDS reads and the scalar loads of the stencil constants share one
        // wait counter: take all neighbour records before any constant load
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
        __builtin_amdgcn_sched_barrier(0);
        T y0, y1, y2;
        node_rows<T, METHOD, CORR, A0>(c, nb, scs[w.macro], ecs[w.macro], y0, y1, y2);
        if constexpr (OUT == 2)
          dot_acc += (double)c.x0 * (double)y0 + (double)c.x1 * (double)y1 + (double)c.x2 * (double)y2;
        yv[u][0] = y0;
        yv[u][1] = y1;
        yv[u][2] = y2;
      }
    }
    __syncthreads();
    if (more) put(kk + 2, pre);          // overwrites the slot of plane kk-1
    // a residual reads f only now: loaded before the stencil, its three
    // values would stay live across it and cost a wave of occupancy
#pragma unroll
    for (int u = 0; u < NSUB; ++u)
      if (act[u]) {
        const int64_t g = gk + ps_[u];
        if constexpr (OUT == 3) {
          // damped block-Jacobi step x_out = x + omega P (f - A x) with the
          // node's 3x3 block P (xx yy zz xy xz yz); x of the node is still in
          // the LDS slot of plane kk
          const int o0 = (kk % 3) * wl + ps_[u] - ws;
          const Pair<T> xa = bufA[o0], xb = bufB[o0];
          const T r0 = sb[u][0] - yv[u][0], r1 = sb[u][1] - yv[u][1], r2 = sb[u][2] - yv[u][2];
          const T Pxx = sb[u][3], Pyy = sb[u][4], Pzz = sb[u][5];
          const T Pxy = sb[u][6], Pxz = sb[u][7], Pyz = sb[u][8];
          xo[g] = xa.a + omega * (Pxx * r0 + Pxy * r1 + Pxz * r2);
          xo[g + nn] = xa.b + omega * (Pxy * r0 + Pyy * r1 + Pyz * r2);
          xo[g + 2 * nn] = xb.a + omega * (Pxz * r0 + Pyz * r1 + Pzz * r2);
        } else if constexpr (OUT == 1) {
          y[g] = f[g] - yv[u][0];
          y[g + nn] = f[g + nn] - yv[u][1];
          y[g + 2 * nn] = f[g + 2 * nn] - yv[u][2];
        } else {
          y[g] = yv[u][0];
          y[g + nn] = yv[u][1];
          y[g + 2 * nn] = yv[u][2];
        }
      }
    __syncthreads();
  }
  if constexpr (OUT == 2) {
    // the item's partial sum, reduced in a fixed order (deterministic)
    __shared__ double red[TPB / 64];
    for (int off = 32; off > 0; off >>= 1) dot_acc += __shfl_down(dot_acc, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = dot_acc;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int q = 0; q < TPB / 64; ++q) s += red[q];
      part[3 * item] = s;
      part[3 * item + 1] = 0.0;
      part[3 * item + 2] = 0.0;
    }
    __syncthreads();
  }
}

// One workgroup per work item.
template <typename T, int METHOD, int OUT, bool CORR, bool A0, int NW, int TPB, int NSUB>
__global__ __launch_bounds__(TPB) void k_interior(
    const MacroInfo *__restrict__ minfo, const StencilConst<T> *__restrict__ scs,
    const ElemConst<T> *__restrict__ ecs, const WorkItem *__restrict__ work,
    const T *__restrict__ x, const T *__restrict__ kc, const T *__restrict__ f,
    T *__restrict__ y, int64_t nn, int wl, double *__restrict__ part, const T *__restrict__ P,
    T omega, T *__restrict__ xo) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const WorkItem w = work[blockIdx.x];
  if (w.macro < 0) {                        // padding item of the XCD-aware order
    if (OUT == 2 && threadIdx.x == 0) {
      part[3 * blockIdx.x] = 0.0;
      part[3 * blockIdx.x + 1] = 0.0;
      part[3 * blockIdx.x + 2] = 0.0;
    }
    return;
  }
  interior_item<T, METHOD, OUT, CORR, A0, NW, TPB, NSUB>(w, smem_raw, minfo, scs, ecs, x, kc, f,
                                                         y, nn, wl, part, blockIdx.x, P, omega, xo);
}

// Persistent form: a grid of resident workgroups walks the work list with a
// fixed stride (item q goes to workgroup q mod gridDim.x), so with a grid
// that is a multiple of the XCD count every item keeps the XCD that the
// list's order assigns it.  Every workgroup leaves after at most
// ceil(n_work / gridDim.x) items.
template <typename T, int METHOD, int OUT, bool CORR, bool A0, int NW, int TPB, int NSUB>
__global__ __launch_bounds__(TPB) void k_interior_persist(
    const MacroInfo *__restrict__ minfo, const StencilConst<T> *__restrict__ scs,
    const ElemConst<T> *__restrict__ ecs, const WorkItem *__restrict__ work, int n_work,
    const T *__restrict__ x, const T *__restrict__ kc, const T *__restrict__ f,
    T *__restrict__ y, int64_t nn, int wl, double *__restrict__ part, const T *__restrict__ P,
    T omega, T *__restrict__ xo) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  for (int q = blockIdx.x; q < n_work; q += gridDim.x) {
    const WorkItem w = work[q];
    if (w.macro >= 0)                       // block-uniform
      interior_item<T, METHOD, OUT, CORR, A0, NW, TPB, NSUB>(w, smem_raw, minfo, scs, ecs, x, kc,
                                                             f, y, nn, wl, part, q, P, omega, xo);
    else if (OUT == 2 && threadIdx.x == 0) {
      part[3 * q] = 0.0;
      part[3 * q + 1] = 0.0;
      part[3 * q + 2] = 0.0;
    }
    __syncthreads();
  }
}


template <typename T, int METHOD, int OUT, bool CORR, bool A0, int NW, int TPB, int NSUB>
int launch_interior_nw(hhg_ctx *h, const T *x, const T *k, const T *f, T *y, double *part,
                       hipStream_t st, const T *P, T omega, T *xo) {
  const int wl = h->wl_max;
  const size_t lds = 6 * (size_t)wl * sizeof(Pair<T>);
  ProfScope prof(h, METHOD == METHOD_SCALED ? HHG_K_INTERIOR_SCALED : HHG_K_INTERIOR_ONTHEFLY, st);
  if (h->persist_blocks > 0) {
    auto kern = k_interior_persist<T, METHOD, OUT, CORR, A0, NW, TPB, NSUB>;
    if (lds > 65536) HHG_HIP(hipFuncSetAttribute((const void *)kern,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(std::min(h->persist_blocks, h->n_work)), dim3(TPB), lds, st,
                       h->d_minfo, sc_ptr<T>(h), ec_ptr<T>(h), h->d_work, h->n_work, x, k, f, y,
                       h->n_nodes, wl, part, P, omega, xo);
  } else {
    auto kern = k_interior<T, METHOD, OUT, CORR, A0, NW, TPB, NSUB>;
    if (lds > 65536) HHG_HIP(hipFuncSetAttribute((const void *)kern,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3(h->n_work), dim3(TPB), lds, st, h->d_minfo, sc_ptr<T>(h),
                       ec_ptr<T>(h), h->d_work, x, k, f, y, h->n_nodes, wl, part, P, omega, xo);
  }
  HHG_HIP(hipGetLastError());
  return HHG_OK;
}

// Positions per work item (= threads): 256; window entries per thread: up
// to 2 (levels <= 7) or up to 6 (level 8).
template <typename T, int METHOD, int OUT, bool CORR, bool A0>
int launch_interior(hhg_ctx *h, const T *x, const T *k, const T *f, T *y, double *part,
                    hipStream_t st, const T *P, T omega, T *xo) {
  if (h->n_work == 0) return HHG_OK;
  const int nw = (h->wl_max + 255) / 256;
  if (nw <= 2)
    return launch_interior_nw<T, METHOD, OUT, CORR, A0, 2, 256, 1>(h, x, k, f, y, part, st, P, omega, xo);
  if (nw <= 6)
    return launch_interior_nw<T, METHOD, OUT, CORR, A0, 6, 256, 1>(h, x, k, f, y, part, st, P, omega, xo);
  return fail(HHG_EINVAL, "interior window larger than supported");
}

template <typename T, int METHOD, int OUT>
int launch_interior_o(hhg_ctx *h, const T *x, const T *k, const T *f, T *y, double *part,
                      hipStream_t st, const T *P = nullptr, T omega = T(0), T *xo = nullptr) {
  const bool corr = METHOD == METHOD_SCALED && h->op.corr == HHG_CORR_PHYSICAL;
  const bool a0 = h->op.mu0 != 0.0 || h->op.lam0 != 0.0;
  if (corr && a0) return launch_interior<T, METHOD, OUT, true, true>(h, x, k, f, y, part, st, P, omega, xo);
  if (corr) return launch_interior<T, METHOD, OUT, true, false>(h, x, k, f, y, part, st, P, omega, xo);
  if (a0) return launch_interior<T, METHOD, OUT, false, true>(h, x, k, f, y, part, st, P, omega, xo);
  return launch_interior<T, METHOD, OUT, false, false>(h, x, k, f, y, part, st, P, omega, xo);
}

template <typename T, int METHOD, bool RESID>
int launch_interior_v(hhg_ctx *h, const T *x, const T *k, const T *f, T *y, hipStream_t st) {
  return launch_interior_o<T, METHOD, RESID ? 1 : 0>(h, x, k, f, y, nullptr, st);
}

// y = A x on the macro-interior rows and, per work item q, the partial sum
// of (x, y) over its rows in part[3 q] (part[3 q + 1], part[3 q + 2] = 0):
// h->n_work items.
template <typename T, int METHOD>
int launch_interior_dot(hhg_ctx *h, const T *x, const T *k, T *y, double *part, hipStream_t st) {
  return launch_interior_o<T, METHOD, 2>(h, x, k, nullptr, y, part, st);
}

// One damped block-Jacobi step on the macro-interior rows:
// xo = x + omega P (f - A x), P the 3x3 blocks [6][n_nodes] (xx yy zz xy xz
// yz); xo must not alias x (other rows read x while it is written).
template <typename T, int METHOD>
int launch_interior_smooth(hhg_ctx *h, const T *x, const T *k, const T *f, const T *P, T omega,
                           T *xo, hipStream_t st) {
  return launch_interior_o<T, METHOD, 3>(h, x, k, f, nullptr, nullptr, st, P, omega, xo);
}


}  // namespace hhg
