// Internal definitions shared by the host setup and the HIP kernels.
//
// Lattice: inside a macro the uniform refinement is the lattice triangulation
// whose elements are v0, v0+s1, v0+s1+s2, v0+s1+s2+s3 for the steps
// (1,0,0), (-1,1,0), (0,-1,1) of index space taken in any order (the same
// micro-mesh as Bey's regular refinement, Sec. 2).  Every macro-interior node
// has the same 14 neighbours and 24 elements (Fig. subtypes_and_stencil).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/hhg.h"

namespace hhg {

constexpr int NDIR = 14;
constexpr int NPAIR = 7;     // direction 2p and 2p+1 are opposite
constexpr int NTET = 24;     // elements around an interior node
constexpr int MIN_LEVEL = 2;
constexpr int MAX_LEVEL = 8;   // the largest level the test suite checks (one macro: 2.86 M nodes)

// Direction order: me mw mse mnw tc bc ts bn mn ms tw be tse bnw (names of
// the paper's stencil figure).  Offsets in (i, j, k).
constexpr int DIR_I[NDIR] = {1, -1, 1, -1, 0, 0, 0, 0, 0, 0, -1, 1, 1, -1};
constexpr int DIR_J[NDIR] = {0, 0, -1, 1, 0, 0, -1, 1, 1, -1, 0, 0, -1, 1};
constexpr int DIR_K[NDIR] = {0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 1, -1, 1, -1};
// Number of elements around the edge (node, node + d): 6 or 4.
constexpr int DIR_NT[NDIR] = {6, 6, 6, 6, 6, 6, 6, 6, 4, 4, 4, 4, 4, 4};

// Slot layout inside a plane k: position T(i+j) + i, T(m) = m(m+1)/2.  A
// neighbour (i+di, j+dj, k+dk) of a node at position p on anti-diagonal
// s = i+j is at position p + DIR_A + DIR_B * s of plane k+dk.
__host__ __device__ constexpr int dir_b(int d) { return DIR_I[d] + DIR_J[d]; }
__host__ __device__ constexpr int dir_a(int d) { return (dir_b(d) == 1 ? 1 : 0) + DIR_I[d]; }

// Correction pairs of every direction: ring nodes v and their reflection
// v^m = d - v through the edge midpoint, as direction indices; 3 pairs for
// 6-element edges, 2 for 4-element edges (third entry unused).  The host
// setup re-derives this table from the element list and refuses to run if
// it differs.
constexpr int RING_V[NDIR][3] = {
    {2, 4, 7}, {3, 5, 6}, {0, 5, 6}, {1, 4, 7}, {0, 3, 6}, {1, 2, 7}, {1, 2, 4},
    {0, 3, 5}, {0, 4, -1}, {1, 5, -1}, {1, 3, -1}, {0, 2, -1}, {0, 2, -1}, {1, 3, -1}};
constexpr int RING_VM[NDIR][3] = {
    {8, 11, 12}, {9, 10, 13}, {9, 12, 11}, {8, 13, 10}, {10, 12, 8}, {11, 13, 9},
    {12, 10, 9}, {13, 11, 8}, {3, 7, -1}, {2, 6, -1}, {4, 6, -1}, {5, 7, -1}, {6, 4, -1},
    {7, 5, -1}};

// The 24 elements around a node: the three vertices other than the node,
// as direction indices.
constexpr int TET_V[NTET][3] = {
    {1, 10, 3}, {1, 10, 6}, {1, 13, 3}, {1, 13, 5}, {1, 9, 6},  {1, 9, 5},
    {10, 3, 4}, {10, 6, 4}, {13, 3, 7}, {13, 5, 7}, {3, 4, 8},  {3, 7, 8},
    {9, 6, 2},  {9, 5, 2},  {6, 4, 12}, {6, 2, 12}, {5, 7, 11}, {5, 2, 11},
    {4, 8, 0},  {4, 12, 0}, {7, 8, 0},  {7, 11, 0}, {2, 12, 0}, {2, 11, 0}};

__host__ __device__ constexpr int64_t tri(int64_t m) { return m * (m + 1) / 2; }
__host__ __device__ constexpr int64_t tet_num(int64_t m) { return m * (m + 1) * (m + 2) / 6; }
// Slots of a macro with n intervals per edge, and of the planes below k.
__host__ __device__ constexpr int64_t macro_nodes(int n) { return tet_num(n + 1); }
__host__ __device__ constexpr int64_t plane_base(int n, int k) {
  return tet_num(n + 1) - tet_num(n + 1 - k);
}

// Per-macro geometry and bookkeeping, uniform within a workgroup.
struct MacroInfo {
  int64_t off;      // first global slot
  int32_t n;        // intervals per edge
  int32_t level;
  uint32_t dmask;   // bit z set: primitive with barycentric zero set z is Dirichlet
  int32_t pad;
};

// Stencil constants of the scaled operator for one macro (type T).
// Blocks use the convention y_m = sum_l B[m][l] x_l.
// Pair-major: the constants of directions 2p and 2p+1 are contiguous, so
// a kernel that works through the pairs in order loads them pair by pair.
// Opposite directions share the reference stencil and the correction axes:
// the point reflection through the node maps the edge patch of d onto that
// of -d and ring pair q of d (RING_V/RING_VM) onto ring pair q of -d, and
// element blocks are quadratic in the gradients, hence unchanged (the host
// setup checks both identities).
template <typename T>
struct StencilPair {
  T shat[6];            // reference stencil of the scaled form (symmetric):
                        // xx yy zz xy xz yz
  T cax[3][3];          // axial vectors of the correction blocks C^v_d,
                        // ring pair q (third unused on 4-element edges)
  T a0[6];              // constant (unscaled) part, symmetric
};
template <typename T>
struct StencilConst {
  StencilPair<T> pr[NPAIR];
  T w_end;              // k-hat weight of the two edge end points
  T w_ring6, w_ring4;   // k-hat weight of a ring node (6- / 4-element edge)
  int32_t has_a0;
  int32_t pad;
};

// Element blocks for on-the-fly integration and interface rows: for each of
// the 24 elements, B^t_{0,b} for its vertices b = node itself, TET_V[t][0..2].
template <typename T>
struct ElemConst {
  T b1[NTET][4][9];     // k-scaled form
  T b0[NTET][4][9];     // constant form
};

// Constants of the nodal strain-rate estimate for one macro: least-squares
// weights of the 14 neighbour differences (affine fit on the 15-node patch)
// and the P1 gradients of the 24 elements around a node (vertex 0 = node,
// 1..3 = TET_V), all micro elements having the same volume.
struct StrainConst {
  double w[NDIR][3];
  double grad[NTET][4][3];
  double vol;
};

// Interior work item: macro, chunk of plane positions, plane range [ka, kb).
struct WorkItem {
  int32_t macro, chunk, ka, kb;
};

constexpr int BOUNDARY_BLOCK = 256;  // threads per block of the boundary-row kernel

// A tile of rows inside one face of a macro, in the face's own coordinates
// (a, b) with the face layer l = 0 and the macro's layers l = 1, 2, ... behind
// it; face f is the one whose nodes have barycentric coordinate f equal to
// zero (0: i + j + k = n, 1: i = 0, 2: j = 0, 3: k = 0).  Rows a0 <= a <
// a0 + FT_W, b0 <= b < b0 + FT_H with a, b >= 2 and a + b <= n - 2 (the
// face's deep rows, two or more nodes away from its edges).
struct FaceTile {
  int32_t macro, face, a0, b0;
};
constexpr int FT_W = 32, FT_H = 8;             // rows per tile: FT_W * FT_H = BOUNDARY_BLOCK
constexpr int FT_P = (FT_W + 2) * (FT_H + 2);  // tile positions with their halo, per layer
constexpr int NXCD = 8;              // accelerator complex dies of an MI355X

}  // namespace hhg
