// Operator application: macro-boundary rows, copy sums, launch sequence
// and the C ABI entry points.  The interior-row kernels (the hot path) live in
// hhg_interior.h and are compiled per element type and method.
#include <algorithm>

#include "hhg_device.h"

namespace hhg {

// Offset of plane k in a macro with n + 1 nodes per edge.
__device__ __forceinline__ int plane_base32(int n, int k) {
  const int a = n + 1, b = n + 1 - k;
  return a * (a + 1) * (a + 2) / 6 - b * (b + 1) * (b + 2) / 6;
}

// Neighbour data of one macro-boundary row at (i, j, k): which neighbours
// lie inside the macro and which on its boundary, their coefficients and
// their values of x (Dirichlet values masked), and the row's own values.
template <typename T>
struct BoundaryNbr {
  bool in[NDIR], onb[NDIR];
  T nx0[NDIR], nx1[NDIR], nx2[NDIR], nk[NDIR];
  T ci0, ci1, ci2, ck;
};

template <typename T>
__device__ __forceinline__ void boundary_gather(const MacroInfo &mi, int i, int j, int k,
                                                const T *__restrict__ x, const T *__restrict__ kc,
                                                int64_t nn, BoundaryNbr<T> &b) {
  const int n = mi.n;
  const T *X0 = x + mi.off;
  const T *X1 = X0 + nn;
  const T *X2 = X1 + nn;
  const T *KC = kc + mi.off;
#pragma unroll
  for (int d = 0; d < NDIR; ++d) {
    const int a = i + DIR_I[d], bb = j + DIR_J[d], cc = k + DIR_K[d];
    b.in[d] = a >= 0 && bb >= 0 && cc >= 0 && a + bb + cc <= n;
    b.onb[d] = false;
    b.nx0[d] = b.nx1[d] = b.nx2[d] = b.nk[d] = T(0);
    if (b.in[d]) {
      const int zz = zero_set(a, bb, cc, n);
      b.onb[d] = zz != 0;
      const int ls = plane_base32(n, cc) + (a + bb) * (a + bb + 1) / 2 + a;
      b.nk[d] = KC[ls];
      if (!((mi.dmask >> zz) & 1u)) {
        b.nx0[d] = X0[ls];
        b.nx1[d] = X1[ls];
        b.nx2[d] = X2[ls];
      }
    }
  }
  const int lslot = plane_base32(n, k) + (i + j) * (i + j + 1) / 2 + i;
  b.ci0 = X0[lslot];
  b.ci1 = X1[lslot];
  b.ci2 = X2[lslot];
  b.ck = KC[lslot];
}

// One macro-boundary row of macro m at (i, j, k) from its gathered
// neighbour data: the macro's partial row (or, for a node without copies in
// other macros and RESID, f minus the row) is written to the node's slot.
// ZS (zero-sum centre): every neighbour value enters as x_j - x_i and the
// nodal centre term is dropped, so the centre block becomes minus the sum of
// the row's other blocks.
template <typename T, bool RESID, bool ROWWISE, bool CORR, bool A0, bool ZS>
__device__ __forceinline__ double boundary_row(const MacroInfo &mi, const StencilConst<T> &sc,
                                             const ElemConst<T> &ec, int i, int j, int k,
                                             const BoundaryNbr<T> &b,
                                             const uint8_t *__restrict__ flags,
                                             const T *__restrict__ f, T *__restrict__ y,
                                             int64_t nn) {
  const int64_t slot = mi.off + plane_base32(mi.n, k) + (i + j) * (i + j + 1) / 2 + i;
  const bool *in = b.in, *onb = b.onb;
  const T *nx0 = b.nx0, *nx1 = b.nx1, *nx2 = b.nx2, *nk = b.nk;
  const T ci0 = b.ci0, ci1 = b.ci1, ci2 = b.ci2, ck = b.ck;
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
        if (ZS) continue;
        d0 = ci0; d1 = ci1; d2 = ci2;
      } else {
        const int v = TET_V[t][c - 1];
        if (!ROWWISE && !onb[v]) continue;   // scaled entry handled below
        d0 = nx0[v]; d1 = nx1[v]; d2 = nx2[v];
        if (ZS) {
          d0 -= ci0; d1 -= ci1; d2 -= ci2;
        }
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
      const T *S = sc.pr[d >> 1].shat;
      const T e0 = ZS ? nx0[d] - ci0 : nx0[d], e1 = ZS ? nx1[d] - ci1 : nx1[d],
              e2 = ZS ? nx2[d] - ci2 : nx2[d];
      const T z0v = kh * e0, z1v = kh * e1, z2v = kh * e2;
      sym_mv_acc(S, z0v, z1v, z2v, y0, y1, y2);
      if constexpr (A0) sym_mv_acc(sc.pr[d >> 1].a0, e0, e1, e2, y0, y1, y2);
      if (CORR) {
        T w0 = T(0), w1 = T(0), w2 = T(0);
#pragma unroll
        for (int q = 0; q < np; ++q) {
          const T dk = nk[RING_V[d][q]] - nk[RING_VM[d][q]];
          w0 = fma(dk, sc.pr[d >> 1].cax[q][0], w0);
          w1 = fma(dk, sc.pr[d >> 1].cax[q][1], w1);
          w2 = fma(dk, sc.pr[d >> 1].cax[q][2], w2);
        }
        cross_acc(w0, w1, w2, e0, e1, e2, y0, y1, y2);
      }
    }
  }
  // (x_i, this macro's part of the row): summed over the copies of a node
  // this gives (x_i, (A x)_i), since x is the same in every copy
  const double dot = (double)ci0 * (double)y0 + (double)ci1 * (double)y1 + (double)ci2 * (double)y2;
  // a node with copies in other macros is completed by the group sum
  if (RESID && !(flags[slot] & 8)) {
    y0 = f[slot] - y0;
    y1 = f[slot + nn] - y1;
    y2 = f[slot + 2 * nn] - y2;
  }
  y[slot] = y0;
  y[slot + nn] = y1;
  y[slot + 2 * nn] = y2;
  return dot;
}

// Partial sum of a block of BOUNDARY_BLOCK threads written to part[3 b]
// (part[3 b + 1], part[3 b + 2] = 0), reduced in a fixed order.
__device__ __forceinline__ void block_part(double v, double *__restrict__ part, int b) {
  __shared__ double red[BOUNDARY_BLOCK / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < BOUNDARY_BLOCK / 64; ++q) s += red[q];
    part[3 * b] = s;
    part[3 * b + 1] = 0.0;
    part[3 * b + 2] = 0.0;
  }
}

// Face coordinates: node (a, b) of layer l behind face f, and back.
__device__ __forceinline__ void face_to_ijk(int f, int n, int a, int b, int l, int &i, int &j,
                                            int &k) {
  switch (f) {
    case 0: i = a; j = b; k = n - a - b - l; break;
    case 1: i = l; j = a; k = b; break;
    case 2: i = a; j = l; k = b; break;
    default: i = a; j = b; k = l;
  }
}
__device__ __forceinline__ void ijk_to_face(int f, int n, int i, int j, int k, int &a, int &b,
                                            int &l) {
  switch (f) {
    case 0: a = i; b = j; l = n - i - j - k; break;
    case 1: a = j; b = k; l = i; break;
    case 2: a = i; b = k; l = j; break;
    default: a = i; b = j; l = k;
  }
}

// The macro's constants (element blocks and stencil table) copied straight
// into LDS by the loader, so staging costs no registers; all lanes later read
// the same addresses, so the reads broadcast.  The caller waits for vmcnt(0)
// and synchronizes before reading them.
template <typename T>
__device__ __forceinline__ void stage_constants(const StencilConst<T> *__restrict__ scs,
                                                const ElemConst<T> *__restrict__ ecs, int m,
                                                unsigned char *cbuf) {
  static_assert(sizeof(ElemConst<T>) % 16 == 0 && sizeof(StencilConst<T>) % 4 == 0, "table sizes");
  constexpr int EB = (int)sizeof(ElemConst<T>), SB = (int)sizeof(StencilConst<T>);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const char *ge = reinterpret_cast<const char *>(ecs + m);
  const char *gs = reinterpret_cast<const char *>(scs + m);
  for (int c = wave * 1024; c < EB; c += BOUNDARY_BLOCK * 16)      // wave-uniform
    if (c + lane * 16 < EB)
      __builtin_amdgcn_global_load_lds(ge + c + lane * 16,
                                       (__attribute__((address_space(3))) void *)(cbuf + c), 16, 0, 0);
  for (int c = wave * 256; c < SB; c += BOUNDARY_BLOCK * 4)
    if (c + lane * 4 < SB)
      __builtin_amdgcn_global_load_lds(gs + c + lane * 4,
                                       (__attribute__((address_space(3))) void *)(cbuf + EB + c), 4, 0, 0);
}

constexpr int FT_RPT = FT_W * FT_H / BOUNDARY_BLOCK;   // face-tile rows per thread

template <typename T>
constexpr int CONST_BYTES = (int)(sizeof(ElemConst<T>) + sizeof(StencilConst<T>));
template <typename T>
constexpr int TILE_BYTES = (int)(2 * 4 * FT_P * sizeof(T));

// Block of BOUNDARY_BLOCK listed macro-boundary rows (edges, vertices, faces
// without tiles, Dirichlet slots): every row gathers its neighbours from
// HBM.  The rows of a block belong to one macro (bblk) and are ordered by the
// boundary primitive they lie on, so that a wave rarely diverges; Dirichlet
// slots (bit 30 in bijk) get their zero rows.
template <typename T, bool RESID, bool ROWWISE, bool CORR, bool A0, bool ZS, bool DOT>
__device__ __forceinline__ void listed_rows(int blk, unsigned char *smem,
                                            const MacroInfo *__restrict__ minfo,
                                            const StencilConst<T> *__restrict__ scs,
                                            const ElemConst<T> *__restrict__ ecs,
                                            const int32_t *__restrict__ bijk,
                                            const int32_t *__restrict__ bblk,
                                            const uint8_t *__restrict__ flags,
                                            const T *__restrict__ x, const T *__restrict__ kc,
                                            const T *__restrict__ f, T *__restrict__ y,
                                            int64_t nn, double *__restrict__ part, int pb) {
  const int m = bblk[blk];
  const int packed = bijk[(int64_t)blk * BOUNDARY_BLOCK + threadIdx.x];
  const MacroInfo mi = minfo[m];
  const int i = packed & 1023, j = (packed >> 10) & 1023, k = (packed >> 20) & 1023;
  const bool live = packed >= 0 && !(packed & (1 << 30));
  if (!__syncthreads_or(live)) {           // a block of Dirichlet slots only
    if (packed >= 0) {
      const int64_t slot = mi.off + plane_base32(mi.n, k) + (i + j) * (i + j + 1) / 2 + i;
      y[slot] = T(0);
      y[slot + nn] = T(0);
      y[slot + 2 * nn] = T(0);
    }
    if (DOT && threadIdx.x == 0) {
      part[3 * pb] = 0.0;
      part[3 * pb + 1] = 0.0;
      part[3 * pb + 2] = 0.0;
    }
    return;
  }
  // the row's neighbour loads go out first, the constants' copies behind
  // them, so both are in flight together and one wait covers them
  BoundaryNbr<T> nb;
  if (live) boundary_gather(mi, i, j, k, x, kc, nn, nb);
  stage_constants(scs, ecs, m, smem);
  __builtin_amdgcn_s_waitcnt(0x0F70);      // vmcnt(0)
  __syncthreads();
  double dot = 0.0;
  if (packed >= 0) {
    if (packed & (1 << 30)) {              // Dirichlet slot: its row is zero
      const int64_t slot = mi.off + plane_base32(mi.n, k) + (i + j) * (i + j + 1) / 2 + i;
      y[slot] = T(0);
      y[slot + nn] = T(0);
      y[slot + 2 * nn] = T(0);
    } else {
      const ElemConst<T> &ec = *reinterpret_cast<const ElemConst<T> *>(smem);
      const StencilConst<T> &sc =
          *reinterpret_cast<const StencilConst<T> *>(smem + sizeof(ElemConst<T>));
      dot = boundary_row<T, RESID, ROWWISE, CORR, A0, ZS>(mi, sc, ec, i, j, k, nb, flags, f, y, nn);
    }
  }
  if constexpr (DOT) block_part(dot, part, pb);
}

// Displacement (da, db, dl) in face coordinates of lattice direction d for
// face FACE (see face_to_ijk).
template <int FACE>
__host__ __device__ constexpr int face_da(int d) {
  return FACE == 1 ? DIR_J[d] : DIR_I[d];
}
template <int FACE>
__host__ __device__ constexpr int face_db(int d) {
  return FACE == 0 || FACE == 3 ? DIR_J[d] : DIR_K[d];
}
template <int FACE>
__host__ __device__ constexpr int face_dl(int d) {
  return FACE == 0 ? -(DIR_I[d] + DIR_J[d] + DIR_K[d])
                   : (FACE == 1 ? DIR_I[d] : (FACE == 2 ? DIR_J[d] : DIR_K[d]));
}

// One FaceTile of deep rows of a macro face (face coordinates a, b >= 2 and
// n - a - b >= 2): the tile's nodes and a halo of one, in the face layer and
// in the first layer behind it, are staged in LDS (each value is loaded once
// per tile instead of once per neighbouring row; Dirichlet values of x are
// masked), then every thread computes FT_RPT rows from there.  For a deep row
// the neighbours in the face layer lie on the face, those in the first
// layer inside the macro and those in front of the face outside it, so with
// the face fixed at compile time every neighbour's role and LDS offset is a
// constant and the row needs no branches.
template <typename T, bool RESID, bool ROWWISE, bool CORR, bool A0, bool ZS, bool DOT, int FACE>
__device__ __forceinline__ void face_rows(const FaceTile &ft, unsigned char *smem,
                                          const MacroInfo *__restrict__ minfo,
                                          const StencilConst<T> *__restrict__ scs,
                                          const ElemConst<T> *__restrict__ ecs,
                                          const uint8_t *__restrict__ flags,
                                          const T *__restrict__ x, const T *__restrict__ kc,
                                          const T *__restrict__ f, T *__restrict__ y,
                                          int64_t nn, double *__restrict__ part, int pb) {
  static_assert(FT_RPT * BOUNDARY_BLOCK == FT_W * FT_H && FT_H % FT_RPT == 0, "whole rows per thread");
  T(*tile)[4][FT_P] = reinterpret_cast<T(*)[4][FT_P]>(smem + CONST_BYTES<T>);  // [layer][x0 x1 x2 k]
  const int m = ft.macro;
  const MacroInfo mi = minfo[m];
  const int n = mi.n;
  const int a0 = ft.a0, b0 = ft.b0;
  const int tid = threadIdx.x;
  // staging loads: entry q of 2 * FT_P is (layer, halo row, halo column)
  constexpr int NR = (2 * FT_P + BOUNDARY_BLOCK - 1) / BOUNDARY_BLOCK;
  T v[NR][4];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int q = r * BOUNDARY_BLOCK + tid;
    const int l = q / FT_P, p = q - l * FT_P;
    const int a = a0 - 1 + p % (FT_W + 2), b = b0 - 1 + p / (FT_W + 2);
    v[r][0] = v[r][1] = v[r][2] = v[r][3] = T(0);
    if (q < 2 * FT_P && a >= 0 && b >= 0 && a + b + l <= n) {
      int i, j, k;
      face_to_ijk(FACE, n, a, b, l, i, j, k);
      const int64_t ls = mi.off + plane_base32(n, k) + (i + j) * (i + j + 1) / 2 + i;
      v[r][3] = kc[ls];
      if (!((mi.dmask >> zero_set(i, j, k, n)) & 1u)) {
        v[r][0] = x[ls];
        v[r][1] = x[nn + ls];
        v[r][2] = x[2 * nn + ls];
      }
    }
  }
  stage_constants(scs, ecs, m, smem);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int q = r * BOUNDARY_BLOCK + tid;
    if (q < 2 * FT_P) {
      const int l = q / FT_P, p = q - l * FT_P;
#pragma unroll
      for (int c = 0; c < 4; ++c) tile[l][c][p] = v[r][c];
    }
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);      // vmcnt(0)
  __syncthreads();
  double dot = 0.0;
#pragma unroll 1
  for (int r = 0; r < FT_RPT; ++r) {       // rows b0 + tid / FT_W + r * FT_H / FT_RPT
    // the constants' LDS base is made opaque in every iteration, so that
    // their reads are not hoisted out of the loop into registers
    int coff = 0;
    asm volatile("" : "+v"(coff));
    const unsigned char *cb = smem + coff;
    const ElemConst<T> &ec = *reinterpret_cast<const ElemConst<T> *>(cb);
    const StencilConst<T> &sc = *reinterpret_cast<const StencilConst<T> *>(cb + sizeof(ElemConst<T>));
    const int a = a0 + tid % FT_W, b = b0 + tid / FT_W + r * (FT_H / FT_RPT);
    if (a + b > n - 2) continue;           // a, b >= 2 by construction
    int i, j, k;
    face_to_ijk(FACE, n, a, b, 0, i, j, k);
    const int pc = (a - a0 + 1) + (b - b0 + 1) * (FT_W + 2);
    BoundaryNbr<T> nb;
#pragma unroll
    for (int d = 0; d < NDIR; ++d) {
      const int dl = face_dl<FACE>(d);
      nb.in[d] = dl >= 0;
      nb.onb[d] = dl == 0;
      nb.nx0[d] = nb.nx1[d] = nb.nx2[d] = nb.nk[d] = T(0);
      if (dl >= 0) {
        const int p = pc + face_da<FACE>(d) + face_db<FACE>(d) * (FT_W + 2);
        nb.nx0[d] = tile[dl][0][p];
        nb.nx1[d] = tile[dl][1][p];
        nb.nx2[d] = tile[dl][2][p];
        nb.nk[d] = tile[dl][3][p];
      }
    }
    nb.ci0 = tile[0][0][pc];
    nb.ci1 = tile[0][1][pc];
    nb.ci2 = tile[0][2][pc];
    nb.ck = tile[0][3][pc];
    dot += boundary_row<T, RESID, ROWWISE, CORR, A0, ZS>(mi, sc, ec, i, j, k, nb, flags, f, y, nn);
  }
  if constexpr (DOT) block_part(dot, part, pb);
}

// Rows of nodes on a macro boundary (Sec. 2.2).  Each copy of a node
// computes the partial row of its macro; copies are summed afterwards.
// ROWWISE: nodal integration for the whole row (also the on-the-fly method);
// otherwise scaled entries towards macro-interior neighbours and nodal
// entries towards macro-boundary neighbours, with the nodal diagonal or (ZS)
// the zero-sum centre.  One launch
// covers all of them: the first nft blocks are face tiles, the rest blocks
// of listed rows, so that the whole boundary is queued at once.
template <typename T, bool RESID, bool ROWWISE, bool CORR, bool A0, bool ZS, bool DOT>
__global__ __launch_bounds__(BOUNDARY_BLOCK) void k_boundary_rows(
    const MacroInfo *__restrict__ minfo, const StencilConst<T> *__restrict__ scs,
    const ElemConst<T> *__restrict__ ecs, const FaceTile *__restrict__ tiles, int nft,
    const int32_t *__restrict__ bijk, const int32_t *__restrict__ bblk,
    const uint8_t *__restrict__ flags, const T *__restrict__ x, const T *__restrict__ kc,
    const T *__restrict__ f, T *__restrict__ y, int64_t nn, double *__restrict__ part) {
  __shared__ __align__(16) unsigned char smem[CONST_BYTES<T> + TILE_BYTES<T>];
  if ((int)blockIdx.x < nft) {
    const FaceTile ft = tiles[blockIdx.x];
    switch (__builtin_amdgcn_readfirstlane(ft.face)) {
#define HHG_FR(F)                                                                                 \
  face_rows<T, RESID, ROWWISE, CORR, A0, ZS, DOT, F>(ft, smem, minfo, scs, ecs, flags, x, kc, f, y, nn, \
                                                    part, (int)blockIdx.x);                            \
  break
      case 0: HHG_FR(0);
      case 1: HHG_FR(1);
      case 2: HHG_FR(2);
      default: HHG_FR(3);
#undef HHG_FR
    }
  } else
    listed_rows<T, RESID, ROWWISE, CORR, A0, ZS, DOT>((int)blockIdx.x - nft, smem, minfo, scs, ecs, bijk,
                                                      bblk, flags, x, kc, f, y, nn, part, (int)blockIdx.x);
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

// Boundary part of a damped block-Jacobi step: xo = x + omega P r on the
// macro-boundary slots (r complete there after the copy-group sum).
template <typename T>
__global__ __launch_bounds__(256) void k_bjacobi(const int64_t *__restrict__ bnd, int64_t nb,
                                                 const T *__restrict__ P, const T *__restrict__ r,
                                                 const T *__restrict__ x, T *__restrict__ xo,
                                                 T omega, int64_t nn) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nb) return;
  const int64_t s = bnd[q];
  const T r0 = r[s], r1 = r[nn + s], r2 = r[2 * nn + s];
  const T Pxx = P[s], Pyy = P[nn + s], Pzz = P[2 * nn + s];
  const T Pxy = P[3 * nn + s], Pxz = P[4 * nn + s], Pyz = P[5 * nn + s];
  xo[s] = x[s] + omega * (Pxx * r0 + Pxy * r1 + Pxz * r2);
  xo[nn + s] = x[nn + s] + omega * (Pxy * r0 + Pyy * r1 + Pyz * r2);
  xo[2 * nn + s] = x[2 * nn + s] + omega * (Pxz * r0 + Pyz * r1 + Pzz * r2);
}

// ------------------------------------------------------------ launchers
namespace {

template <typename T, bool RESID, bool DOT = false>
int launch_boundary(hhg_ctx *h, int method, const T *x, const T *k, const T *f, T *y,
                    hipStream_t st, double *part = nullptr) {
  static_assert(!(DOT && RESID), "partial sums of (x, A x) only for the plain apply");
  const bool rowwise = method == METHOD_ONTHEFLY || h->op.iface == HHG_IFACE_ROWWISE;
  const bool zs = !rowwise && h->op.iface == HHG_IFACE_ZEROSUM;
  const bool corr = h->op.corr == HHG_CORR_PHYSICAL;
  const int nft = (int)h->ftile.size();
  const int nblk = nft + (int)h->bblk.size();
  if (nblk > 0) {
    const dim3 grid((unsigned)nblk);
#define HHG_LB(RW, CR, A0, ZS)                                                                       \
  hipLaunchKernelGGL((k_boundary_rows<T, RESID, RW, CR, A0, ZS, DOT>), grid, dim3(BOUNDARY_BLOCK), 0,  \
                     st, h->d_minfo, sc_ptr<T>(h), ec_ptr<T>(h), h->d_ftile, nft, h->d_bijk,          \
                     h->d_bblk, h->d_flags, x, k, f, y, h->n_nodes, part)
#define HHG_LB2(CR, A0) \
  if (zs) HHG_LB(false, CR, A0, true); else HHG_LB(false, CR, A0, false)
    ProfScope prof(h, HHG_K_BOUNDARY_ROWS, st);
    const bool a0 = h->op.mu0 != 0.0 || h->op.lam0 != 0.0;
    if (rowwise) {
      if (a0) HHG_LB(true, false, true, false); else HHG_LB(true, false, false, false);
    } else if (corr) {
      if (a0) { HHG_LB2(true, true); } else { HHG_LB2(true, false); }
    } else {
      if (a0) { HHG_LB2(false, true); } else { HHG_LB2(false, false); }
    }
#undef HHG_LB2
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
  hipStream_t sb = h->side, si = st;
  int rc;
  if (f) {
    rc = launch_boundary<T, true>(h, method, x, k, f, y, sb);
    if (!rc)
      rc = method == METHOD_SCALED ? launch_interior_v<T, METHOD_SCALED, true>(h, x, k, f, y, si)
                                   : launch_interior_v<T, METHOD_ONTHEFLY, true>(h, x, k, f, y, si);
  } else {
    rc = launch_boundary<T, false>(h, method, x, k, f, y, sb);
    if (!rc)
      rc = method == METHOD_SCALED ? launch_interior_v<T, METHOD_SCALED, false>(h, x, k, f, y, si)
                                   : launch_interior_v<T, METHOD_ONTHEFLY, false>(h, x, k, f, y, si);
  }
  HHG_HIP(hipEventRecord(h->ev_join, h->side));
  HHG_HIP(hipStreamWaitEvent(st, h->ev_join, 0));
  return rc;
}

// y = A x and the partial sums of (x, y): the interior kernel writes one per
// work item to part[0 .. n_work), the boundary-row kernel one per block to
// part[n_work .. n_work + boundary blocks); summed in index order they give
// (x, A x) over the owner copies of all nodes (each copy of an interface node
// contributes x_i times its partial row).  Same streams as apply_t.
template <typename T>
int apply_dot_t(hhg_ctx *h, int method, const T *x, const T *k, T *y, double *part, hipStream_t st) {
  double *pb = part + 3 * (int64_t)h->n_work;
  auto interior = [&](hipStream_t s) {
    return method == METHOD_SCALED ? launch_interior_dot<T, METHOD_SCALED>(h, x, k, y, part, s)
                                   : launch_interior_dot<T, METHOD_ONTHEFLY>(h, x, k, y, part, s);
  };
  if (h->serial_apply) {
    int rc = interior(st);
    if (rc) return rc;
    return launch_boundary<T, false, true>(h, method, x, k, nullptr, y, st, pb);
  }
  HHG_HIP(hipEventRecord(h->ev_fork, st));
  HHG_HIP(hipStreamWaitEvent(h->side, h->ev_fork, 0));
  int rc = launch_boundary<T, false, true>(h, method, x, k, nullptr, y, h->side, pb);
  if (!rc) rc = interior(st);
  HHG_HIP(hipEventRecord(h->ev_join, h->side));
  HHG_HIP(hipStreamWaitEvent(st, h->ev_join, 0));
  return rc;
}

// One damped block-Jacobi step xo = x + omega P (f - A x) (xo must not alias
// x): the interior kernel applies the step to the macro-interior rows in its
// epilogue, so their residual never goes to memory; the boundary rows and the
// copy sums write the residual of the macro-boundary rows to r as in a
// residual apply (same streams as apply_t), and k_bjacobi completes the step
// there.
template <typename T>
int smooth_t(hhg_ctx *h, int method, const T *f, const T *x, const T *k, const T *P, T omega,
             T *r, T *xo, hipStream_t st) {
  auto interior = [&](hipStream_t s) {
    return method == METHOD_SCALED
               ? launch_interior_smooth<T, METHOD_SCALED>(h, x, k, f, P, omega, xo, s)
               : launch_interior_smooth<T, METHOD_ONTHEFLY>(h, x, k, f, P, omega, xo, s);
  };
  int rc;
  if (h->serial_apply) {
    if ((rc = interior(st))) return rc;
    if ((rc = launch_boundary<T, true>(h, method, x, k, f, r, st))) return rc;
  } else {
    HHG_HIP(hipEventRecord(h->ev_fork, st));
    HHG_HIP(hipStreamWaitEvent(h->side, h->ev_fork, 0));
    rc = launch_boundary<T, true>(h, method, x, k, f, r, h->side);
    if (!rc) rc = interior(st);
    HHG_HIP(hipEventRecord(h->ev_join, h->side));
    HHG_HIP(hipStreamWaitEvent(st, h->ev_join, 0));
    if (rc) return rc;
  }
  if (h->n_bnd > 0) {
    hipLaunchKernelGGL(k_bjacobi<T>, dim3((unsigned)((h->n_bnd + 255) / 256)), dim3(256), 0, st,
                       h->d_bnd, h->n_bnd, P, r, x, xo, omega, h->n_nodes);
    HHG_HIP(hipGetLastError());
  }
  return HHG_OK;
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

// Number of partial sums apply_dot_internal writes (3 doubles each).
int64_t dot_parts(hhg_ctx *h) { return (int64_t)h->n_work + (int64_t)h->ftile.size() + (int64_t)h->bblk.size(); }

// y = A x with the partial sums of (x, y) (see apply_dot_t); part holds
// 3 dot_parts(h) doubles.
int apply_dot_internal(hhg_ctx *h, int prec, int method, const void *x, const void *k, void *y,
                       double *part, hipStream_t st) {
  int rc = ensure_device(h);
  if (rc) return rc;
  if (prec == HHG_F64)
    return apply_dot_t<double>(h, method, (const double *)x, (const double *)k, (double *)y, part, st);
  return apply_dot_t<float>(h, method, (const float *)x, (const float *)k, (float *)y, part, st);
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

// One damped block-Jacobi smoothing step for the multigrid (see smooth_t).
int smooth_internal(hhg_ctx *h, int prec, int method, const void *f, const void *x, const void *k,
                    const void *P, double omega, void *r, void *xo, hipStream_t st) {
  int rc = ensure_device(h);
  if (rc) return rc;
  if (prec == HHG_F64)
    return smooth_t<double>(h, method, (const double *)f, (const double *)x, (const double *)k,
                            (const double *)P, omega, (double *)r, (double *)xo, st);
  return smooth_t<float>(h, method, (const float *)f, (const float *)x, (const float *)k,
                         (const float *)P, (float)omega, (float *)r, (float *)xo, st);
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
