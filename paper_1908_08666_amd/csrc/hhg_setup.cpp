// Host-side setup of the stencil-scaling library (all FP64).
//
// For every macro-tet this builds, once (Sec. 2.4: the reference stencil and
// the correction stencils are stored per macro and only the scaling is
// recomputed):
//   * the reference stencil Shat_d of the k-scaled form, the constant part
//     A0_d, the correction blocks C^v_d of the Lemma in the ring form of
//     Sec. 2.4 and the k-hat weights of eq. patchmean;
//   * the element blocks of the 24 elements around a node (nodal
//     integration on the fly, eq. nodalintegration, and macro-boundary rows);
//   * Dirichlet masks, interface copy groups and the interior work list.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <unordered_map>

#include "hhg_ctx.h"

namespace hhg {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}
int hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return HHG_EHIP;
}

namespace {

using Vec3 = std::array<double, 3>;
using Mat3 = std::array<std::array<double, 3>, 3>;

double det3(const Mat3 &M) {
  return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
         M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
         M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

// Gradients of the barycentric basis of element P[0..3] and its volume.
void p1_grads(const Vec3 P[4], Vec3 g[4], double &vol) {
  Mat3 M;  // columns P[a] - P[0]
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) M[r][c] = P[c + 1][r] - P[0][r];
  const double d = det3(M);
  // inverse via cofactors; row a of M^{-1} is grad lambda_{a+1}
  Mat3 inv;
  inv[0][0] = (M[1][1] * M[2][2] - M[1][2] * M[2][1]) / d;
  inv[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) / d;
  inv[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) / d;
  inv[1][0] = (M[1][2] * M[2][0] - M[1][0] * M[2][2]) / d;
  inv[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) / d;
  inv[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) / d;
  inv[2][0] = (M[1][0] * M[2][1] - M[1][1] * M[2][0]) / d;
  inv[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) / d;
  inv[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) / d;
  for (int a = 0; a < 3; ++a) g[a + 1] = {inv[a][0], inv[a][1], inv[a][2]};
  for (int c = 0; c < 3; ++c) g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
  vol = std::fabs(d) / 6.0;
}

// Block of 2 mu (eps, eps) + lam (div, div) coupling trial node b (gradient
// gb) into test node a (gradient ga): B[m][l] with y_m = sum_l B[m][l] x_l.
// 2 eps(phi_b e_l) : eps(phi_a e_m) = (ga.gb) delta_ml + gb_m ga_l and
// div(phi_b e_l) div(phi_a e_m) = gb_l ga_m.
Mat3 form_block(const Vec3 &ga, const Vec3 &gb, double vol, double mu, double lam) {
  const double dot = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
  Mat3 B;
  for (int m = 0; m < 3; ++m)
    for (int l = 0; l < 3; ++l)
      B[m][l] = vol * (mu * ((m == l ? dot : 0.0) + gb[m] * ga[l]) + lam * ga[m] * gb[l]);
  return B;
}

int dir_index(int i, int j, int k) {
  for (int d = 0; d < NDIR; ++d)
    if (DIR_I[d] == i && DIR_J[d] == j && DIR_K[d] == k) return d;
  return -1;
}

// Re-derive the element list around a node and the reflection pairs of every
// edge from the lattice definition and compare with the compiled tables.
bool verify_lattice_tables(std::string &why) {
  const int steps[3][3] = {{1, 0, 0}, {-1, 1, 0}, {0, -1, 1}};
  const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  std::set<std::array<int, 3>> found;
  for (int a = -3; a <= 3; ++a)
    for (int b = -3; b <= 3; ++b)
      for (int c = -3; c <= 3; ++c)
        for (const auto &p : perms) {
          int v[4][3] = {{a, b, c}};
          for (int s = 0; s < 3; ++s)
            for (int q = 0; q < 3; ++q) v[s + 1][q] = v[s][q] + steps[p[s]][q];
          int has0 = -1;
          for (int s = 0; s < 4; ++s)
            if (v[s][0] == 0 && v[s][1] == 0 && v[s][2] == 0) has0 = s;
          if (has0 < 0) continue;
          std::array<int, 3> key;
          int w = 0;
          bool ok = true;
          for (int s = 0; s < 4; ++s) {
            if (s == has0) continue;
            int d = dir_index(v[s][0], v[s][1], v[s][2]);
            if (d < 0) ok = false;
            key[w++] = d;
          }
          if (!ok) { why = "lattice element with a vertex outside the 14 neighbours"; return false; }
          std::sort(key.begin(), key.end());
          found.insert(key);
        }
  std::set<std::array<int, 3>> table;
  for (int t = 0; t < NTET; ++t) {
    std::array<int, 3> key = {TET_V[t][0], TET_V[t][1], TET_V[t][2]};
    std::sort(key.begin(), key.end());
    table.insert(key);
  }
  if (found != table) { why = "element table differs from the lattice"; return false; }
  for (int d = 0; d < NDIR; ++d) {
    std::set<int> ring;
    int nt = 0;
    for (int t = 0; t < NTET; ++t) {
      bool has = false;
      for (int c = 0; c < 3; ++c) has |= TET_V[t][c] == d;
      if (!has) continue;
      ++nt;
      for (int c = 0; c < 3; ++c)
        if (TET_V[t][c] != d) ring.insert(TET_V[t][c]);
    }
    if (nt != DIR_NT[d]) { why = "edge element count mismatch"; return false; }
    std::set<int> covered;
    const int np = nt == 6 ? 3 : 2;
    for (int p = 0; p < np; ++p) {
      const int v = RING_V[d][p], vm = RING_VM[d][p];
      if (!ring.count(v) || !ring.count(vm)) { why = "ring pair not on the ring"; return false; }
      if (DIR_I[v] + DIR_I[vm] != DIR_I[d] || DIR_J[v] + DIR_J[vm] != DIR_J[d] ||
          DIR_K[v] + DIR_K[vm] != DIR_K[d]) {
        why = "ring pair is not a reflection through the edge midpoint";
        return false;
      }
      covered.insert(v);
      covered.insert(vm);
    }
    if (covered != ring) { why = "ring pairs do not cover the ring"; return false; }
  }
  return true;
}

struct MacroTables {
  StencilConst<double> sc;
  ElemConst<double> ec;
  StrainConst st;
};

// Least-squares weights of the affine fit on the 15-node patch: with
// d = x_{i+d} - x_i and M = sum_d d d^T, grad u = sum_d M^{-1} d (u_{i+d} - u_i)
// (the neighbour offsets are symmetric, so the constant decouples).
int build_strain_tables(const Vec3 e[3], StrainConst &st) {
  Mat3 M{};
  Vec3 dv[NDIR];
  for (int d = 0; d < NDIR; ++d) {
    for (int c = 0; c < 3; ++c) dv[d][c] = DIR_I[d] * e[0][c] + DIR_J[d] * e[1][c] + DIR_K[d] * e[2][c];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) M[a][b] += dv[d][a] * dv[d][b];
  }
  const double det = det3(M);
  if (!(std::fabs(det) > 0.0)) return fail(HHG_EINVAL, "singular least-squares patch");
  Mat3 Mi;
  Mi[0][0] = (M[1][1] * M[2][2] - M[1][2] * M[2][1]) / det;
  Mi[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) / det;
  Mi[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) / det;
  Mi[1][0] = (M[1][2] * M[2][0] - M[1][0] * M[2][2]) / det;
  Mi[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) / det;
  Mi[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) / det;
  Mi[2][0] = (M[1][0] * M[2][1] - M[1][1] * M[2][0]) / det;
  Mi[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) / det;
  Mi[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) / det;
  for (int d = 0; d < NDIR; ++d)
    for (int a = 0; a < 3; ++a)
      st.w[d][a] = Mi[a][0] * dv[d][0] + Mi[a][1] * dv[d][1] + Mi[a][2] * dv[d][2];
  return HHG_OK;
}

int build_macro_tables(const double *V, int n, const hhg_op_desc &op, MacroTables &out) {
  Vec3 e[3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) e[a][c] = (V[3 * (a + 1) + c] - V[c]) / n;
  auto phys = [&](int d) {
    Vec3 p;
    for (int c = 0; c < 3; ++c) p[c] = DIR_I[d] * e[0][c] + DIR_J[d] * e[1][c] + DIR_K[d] * e[2][c];
    return p;
  };
  // element blocks around the origin
  Mat3 B1[NTET][4], B0[NTET][4];
  for (int t = 0; t < NTET; ++t) {
    Vec3 P[4] = {{0, 0, 0}, phys(TET_V[t][0]), phys(TET_V[t][1]), phys(TET_V[t][2])};
    Vec3 g[4];
    double vol;
    p1_grads(P, g, vol);
    out.st.vol = vol;
    for (int c = 0; c < 4; ++c)
      for (int q = 0; q < 3; ++q) out.st.grad[t][c][q] = g[c][q];
    for (int c = 0; c < 4; ++c) {
      B1[t][c] = form_block(g[0], g[c], vol, op.mu1, op.lam1);
      B0[t][c] = form_block(g[0], g[c], vol, op.mu0, op.lam0);
      for (int m = 0; m < 3; ++m)
        for (int l = 0; l < 3; ++l) {
          out.ec.b1[t][c][3 * m + l] = B1[t][c][m][l];
          out.ec.b0[t][c][3 * m + l] = B0[t][c][m][l];
        }
    }
  }
  {
    int rc = build_strain_tables(e, out.st);
    if (rc) return rc;
  }
  // per direction: sums over the elements of the edge (origin, d)
  Mat3 Ssym[NDIR], A0[NDIR];
  double scale = 0.0;
  for (int d = 0; d < NDIR; ++d) {
    Ssym[d] = Mat3{};
    A0[d] = Mat3{};
    for (int t = 0; t < NTET; ++t)
      for (int c = 0; c < 3; ++c)
        if (TET_V[t][c] == d)
          for (int m = 0; m < 3; ++m)
            for (int l = 0; l < 3; ++l) {
              Ssym[d][m][l] += 0.5 * (B1[t][c + 1][m][l] + B1[t][c + 1][l][m]);
              A0[d][m][l] += B0[t][c + 1][m][l];
              scale = std::max(scale, std::fabs(B1[t][c + 1][m][l]) + std::fabs(B0[t][c + 1][m][l]));
            }
  }
  const double tol = 1e-11 * (scale > 0 ? scale : 1.0);
  StencilConst<double> &sc = out.sc;
  std::memset(&sc, 0, sizeof(sc));
  bool any_a0 = false;
  for (int p = 0; p < NPAIR; ++p) {
    const int d = 2 * p, db = 2 * p + 1;
    for (int m = 0; m < 3; ++m)
      for (int l = 0; l < 3; ++l) {
        if (std::fabs(Ssym[d][m][l] - Ssym[db][m][l]) > tol ||
            std::fabs(A0[d][m][l] - A0[db][m][l]) > tol ||
            std::fabs(A0[d][m][l] - A0[d][l][m]) > tol)
          return fail(HHG_EINVAL, "reference stencil is not symmetric under d -> -d");
        any_a0 |= A0[d][m][l] != 0.0;
      }
    const int ix[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    for (int q = 0; q < 6; ++q) {
      sc.pr[p].shat[q] = Ssym[d][ix[q][0]][ix[q][1]];
      sc.pr[p].a0[q] = 0.5 * (A0[d][ix[q][0]][ix[q][1]] + A0[d][ix[q][1]][ix[q][0]]);
    }
  }
  sc.has_a0 = any_a0 ? 1 : 0;
  // correction blocks C^v_d = 1/4 (antisym of the two elements containing v)
  if (op.corr == HHG_CORR_PHYSICAL) {
    double cax[NDIR][3][3] = {};
    for (int d = 0; d < NDIR; ++d) {
      const int np = DIR_NT[d] == 6 ? 3 : 2;
      for (int q = 0; q < np; ++q) {
        const int v = RING_V[d][q];
        Mat3 C{};
        int cnt = 0;
        for (int t = 0; t < NTET; ++t) {
          int cd = -1;
          bool hv = false;
          for (int c = 0; c < 3; ++c) {
            if (TET_V[t][c] == d) cd = c;
            if (TET_V[t][c] == v) hv = true;
          }
          if (cd < 0 || !hv) continue;
          ++cnt;
          for (int m = 0; m < 3; ++m)
            for (int l = 0; l < 3; ++l)
              C[m][l] += 0.25 * 0.5 * (B1[t][cd + 1][m][l] - B1[t][cd + 1][l][m]);
        }
        if (cnt != 2) return fail(HHG_EINVAL, "ring node not in exactly two edge elements");
        // y = C x = c cross x with c = (C[2][1], C[0][2], C[1][0])
        cax[d][q][0] = C[2][1];
        cax[d][q][1] = C[0][2];
        cax[d][q][2] = C[1][0];
      }
    }
    double cscale = 0.0;
    for (int d = 0; d < NDIR; ++d)
      for (int q = 0; q < 3; ++q)
        for (int c = 0; c < 3; ++c) cscale = std::max(cscale, std::fabs(cax[d][q][c]));
    for (int p = 0; p < NPAIR; ++p)
      for (int q = 0; q < 3; ++q)
        for (int c = 0; c < 3; ++c) {
          if (std::fabs(cax[2 * p][q][c] - cax[2 * p + 1][q][c]) > 1e-12 * (cscale > 0 ? cscale : 1.0))
            return fail(HHG_EINVAL, "correction blocks differ between d and -d");
          sc.pr[p].cax[q][c] = cax[2 * p][q][c];
        }
  }
  // k-hat weights: ring node v is in 2 of the |T_d| elements, each element
  // mean weighs its vertices 1/4 (eq. nodalquad), the patch mean 1/|T_d|
  if (op.khat == HHG_KHAT_PATCH) {
    sc.w_end = 0.25;
    sc.w_ring6 = 2.0 / (4.0 * 6.0);
    sc.w_ring4 = 2.0 / (4.0 * 4.0);
  } else {
    sc.w_end = 0.5;
    sc.w_ring6 = 0.0;
    sc.w_ring4 = 0.0;
  }
  return HHG_OK;
}

int64_t tri_root(int64_t p) {  // largest s with s(s+1)/2 <= p
  int64_t s = (int64_t)((std::sqrt(8.0 * (double)p + 1.0) - 1.0) / 2.0);
  while (tri(s + 1) <= p) ++s;
  while (tri(s) > p) --s;
  return s;
}

template <typename TO>
void convert(const StencilConst<double> &a, StencilConst<TO> &b) {
  for (int p = 0; p < NPAIR; ++p) {
    for (int q = 0; q < 6; ++q) {
      b.pr[p].shat[q] = (TO)a.pr[p].shat[q];
      b.pr[p].a0[q] = (TO)a.pr[p].a0[q];
    }
    for (int q = 0; q < 3; ++q)
      for (int c = 0; c < 3; ++c) b.pr[p].cax[q][c] = (TO)a.pr[p].cax[q][c];
  }
  b.w_end = (TO)a.w_end;
  b.w_ring6 = (TO)a.w_ring6;
  b.w_ring4 = (TO)a.w_ring4;
  b.has_a0 = a.has_a0;
  b.pad = 0;
}

template <typename TO>
void convert(const ElemConst<double> &a, ElemConst<TO> &b) {
  for (int t = 0; t < NTET; ++t)
    for (int c = 0; c < 4; ++c)
      for (int q = 0; q < 9; ++q) {
        b.b1[t][c][q] = (TO)a.b1[t][c][q];
        b.b0[t][c][q] = (TO)a.b0[t][c][q];
      }
}

template <typename T>
int upload(T **dst, const T *src, size_t count) {
  if (count == 0) return HHG_OK;
  hipError_t e = hipMalloc((void **)dst, count * sizeof(T));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  e = hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  return HHG_OK;
}

struct KeyHash {
  size_t operator()(const std::array<int64_t, 6> &k) const {
    uint64_t h = 1469598103934665603ull;
    for (int64_t v : k) {
      h ^= (uint64_t)v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    }
    return (size_t)h;
  }
};

template <typename P>
void dfree(P *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void free_ctx(hhg_ctx *h) {
  if (!h) return;
  free_graphs(h);
  dfree(h->d_minfo);
  dfree(h->d_sc64);
  dfree(h->d_sc32);
  dfree(h->d_ec64);
  dfree(h->d_ec32);
  dfree(h->d_work);
  dfree(h->d_bijk);
  dfree(h->d_bblk);
  dfree(h->d_ftile);
  dfree(h->d_dslot);
  dfree(h->d_bnd);
  dfree(h->d_grp_ptr);
  dfree(h->d_grp_slot);
  dfree(h->d_flags);
  dfree(h->d_agrp_ptr);
  dfree(h->d_agrp_slot);
  dfree(h->d_stc);
  dfree(h->d_dotpart);
  dfree(h->d_lsq_ptr);
  dfree(h->d_lsq_slot);
  dfree(h->d_lsq_w);
  dfree(h->d_lsq_optr);
  dfree(h->d_lsq_oslot);
  for (auto &r : h->prof_pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->side) (void)hipStreamDestroy(h->side);
  if (h->solve_stream) (void)hipStreamDestroy(h->solve_stream);
  if (h->h_state) (void)hipHostFree(h->h_state);
  delete h;
}

int setup_impl(const hhg_mesh_desc *mesh, const hhg_op_desc *op, hhg_ctx *h) {
  const int M = mesh->n_macro;
  h->n_macro = M;
  h->coupling = mesh->coupling;
  h->dirichlet = mesh->dirichlet;
  h->op = *op;
  h->verts.assign(mesh->verts, mesh->verts + 12 * (size_t)M);

  std::string why;
  if (!verify_lattice_tables(why)) return fail(HHG_EINVAL, "internal lattice table check: " + why);

  // ---------------------------------------------------------------- macros
  h->minfo.resize(M);
  h->sc64.resize(M);
  h->ec64.resize(M);
  h->stc.resize(M);
  int64_t off = 0;
  double gscale = 0.0;
  for (int m = 0; m < 12 * M; ++m) gscale = std::max(gscale, std::fabs(mesh->verts[m]));
  for (int m = 0; m < M; ++m) {
    const int L = mesh->level[m];
    if (L < MIN_LEVEL || L > MAX_LEVEL)
      return fail(HHG_EINVAL, "level of macro " + std::to_string(m) + " outside 2..8");
    if (mesh->coupling == HHG_CONFORMING && L != mesh->level[0])
      return fail(HHG_EINVAL, "conforming macros need one common level");
    const double *V = mesh->verts + 12 * m;
    Mat3 E;
    double emax = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        E[r][c] = V[3 * (c + 1) + r] - V[r];
        emax = std::max(emax, std::fabs(E[r][c]));
      }
    if (!(std::fabs(det3(E)) > 1e-12 * emax * emax * emax) || !std::isfinite(det3(E)))
      return fail(HHG_EINVAL, "degenerate macro " + std::to_string(m));
    const int n = 1 << L;
    h->minfo[m].off = off;
    h->minfo[m].n = n;
    h->minfo[m].level = L;
    h->minfo[m].dmask = 0;
    h->minfo[m].pad = 0;
    off += macro_nodes(n);
    h->max_level = std::max(h->max_level, L);
    MacroTables tabs;
    int rc = build_macro_tables(V, n, *op, tabs);
    if (rc) return rc;
    h->sc64[m] = tabs.sc;
    h->ec64[m] = tabs.ec;
    h->stc[m] = tabs.st;
  }
  h->n_nodes = off;

  // ------------------------------------------------ global macro vertices
  std::vector<int64_t> gv(4 * (size_t)M);
  if (mesh->coupling == HHG_CONFORMING) {
    std::vector<std::array<double, 3>> uniq;
    const double tol = 1e-10 * (gscale + 1.0);
    for (int q = 0; q < 4 * M; ++q) {
      const double *p = mesh->verts + 3 * q;
      int64_t id = -1;
      for (size_t u = 0; u < uniq.size(); ++u)
        if (std::fabs(uniq[u][0] - p[0]) < tol && std::fabs(uniq[u][1] - p[1]) < tol &&
            std::fabs(uniq[u][2] - p[2]) < tol) {
          id = (int64_t)u;
          break;
        }
      if (id < 0) {
        id = (int64_t)uniq.size();
        uniq.push_back({p[0], p[1], p[2]});
      }
      gv[q] = id;
    }
  } else {
    for (int q = 0; q < 4 * M; ++q) gv[q] = q;
  }

  // faces: count owners; Dirichlet primitives are the faces with one owner
  // and the edges / vertices of those faces
  std::map<std::array<int64_t, 3>, int> face_cnt;
  for (int m = 0; m < M; ++m)
    for (int a = 0; a < 4; ++a) {
      std::array<int64_t, 3> f;
      int w = 0;
      for (int b = 0; b < 4; ++b)
        if (b != a) f[w++] = gv[4 * m + b];
      std::sort(f.begin(), f.end());
      face_cnt[f]++;
    }
  std::set<std::vector<int64_t>> dir_prims;
  if (mesh->dirichlet == HHG_DIRICHLET_OUTER) {
    for (const auto &fc : face_cnt) {
      if (fc.second != 1) continue;
      const auto &f = fc.first;
      dir_prims.insert({f[0], f[1], f[2]});
      for (int a = 0; a < 3; ++a) {
        dir_prims.insert({f[a]});
        for (int b = a + 1; b < 3; ++b) dir_prims.insert({f[a], f[b]});
      }
    }
  }
  for (int m = 0; m < M; ++m) {
    uint32_t mask = 0;
    for (int z = 1; z < 15; ++z) {  // zero sets of size 1..3
      std::vector<int64_t> prim;
      for (int a = 0; a < 4; ++a)
        if (!(z & (1 << a))) prim.push_back(gv[4 * m + a]);
      std::sort(prim.begin(), prim.end());
      if (dir_prims.count(prim)) mask |= 1u << z;
    }
    h->minfo[m].dmask = mask;
  }

  // -------------------------------------------- slots: flags and groups
  h->flags.assign((size_t)h->n_nodes, 0);
  std::vector<int2> bslot;          // all boundary slots (macro, packed i | j<<10 | k<<20)
  std::unordered_map<std::array<int64_t, 6>, std::vector<int64_t>, KeyHash> groups;
  for (int m = 0; m < M; ++m) {
    const int n = h->minfo[m].n;
    const uint32_t mask = h->minfo[m].dmask;
    for (int k = 0; k <= n; ++k)
      for (int s = 0; s + k <= n; ++s)
        for (int i = 0; i <= s; ++i) {
          const int j = s - i;
          const int lam[4] = {n - s - k, i, j, k};
          int z = 0;
          for (int a = 0; a < 4; ++a) z |= (lam[a] == 0) << a;
          if (z == 0) continue;
          const int64_t slot = h->minfo[m].off + plane_base(n, k) + tri(s) + i;
          uint8_t fl = 4;
          if (mask & (1u << z)) fl |= 1;
          h->flags[slot] = fl;
          bslot.push_back(make_int2(m, i | (j << 10) | (k << 20)));
          if (mesh->coupling == HHG_CONFORMING) {
            std::array<std::pair<int64_t, int64_t>, 3> kp;
            int w = 0;
            for (int a = 0; a < 4; ++a)
              if (lam[a] > 0) kp[w++] = {gv[4 * m + a], lam[a]};
            for (; w < 3; ++w) kp[w] = {-1, 0};
            std::sort(kp.begin(), kp.end());
            std::array<int64_t, 6> key;
            for (int q = 0; q < 3; ++q) {
              key[2 * q] = kp[q].first;
              key[2 * q + 1] = kp[q].second;
            }
            groups[key].push_back(slot);
          }
        }
  }
  // owners: every interior slot, the first copy of every boundary node
  for (int m = 0; m < M; ++m) {
    const int n = h->minfo[m].n;
    for (int k = 1; k <= n; ++k)
      for (int s = 2; s + k <= n - 1; ++s)
        for (int i = 1; i <= s - 1; ++i) h->flags[h->minfo[m].off + plane_base(n, k) + tri(s) + i] = 2;
  }
  std::vector<int64_t> gptr{0}, gslot;
  if (mesh->coupling == HHG_CONFORMING) {
    std::vector<std::vector<int64_t>> multi;
    for (auto &g : groups) {
      auto &sl = g.second;
      std::sort(sl.begin(), sl.end());
      h->flags[sl[0]] |= 2;
      // Dirichlet rows are written as zero by every copy; no sum needed
      if (sl.size() > 1 && !(h->flags[sl[0]] & 1)) {
        for (int64_t q : sl) h->flags[q] |= 8;   // completed by the copy-group sum
        multi.push_back(sl);
      }
    }
    std::vector<std::vector<int64_t>> all;
    for (auto &g : groups)
      if (g.second.size() > 1) all.push_back(g.second);
    std::sort(all.begin(), all.end());
    h->agrp_ptr.assign(1, 0);
    for (auto &sl : all) {
      for (int64_t q : sl) h->agrp_slot.push_back(q);
      h->agrp_ptr.push_back((int64_t)h->agrp_slot.size());
    }
    std::sort(multi.begin(), multi.end());
    for (auto &sl : multi) {
      for (int64_t s : sl) gslot.push_back(s);
      gptr.push_back((int64_t)gslot.size());
    }
  } else {
    for (auto &b : bslot) {
      const int m = b.x, n = h->minfo[m].n;
      const int i = b.y & 1023, j = (b.y >> 10) & 1023, k = (b.y >> 20) & 1023;
      h->flags[h->minfo[m].off + plane_base(n, k) + tri(i + j) + i] |= 2;
    }
  }
  h->n_grp = (int64_t)gptr.size() - 1;
  if (h->agrp_ptr.empty()) h->agrp_ptr.assign(1, 0);
  h->n_agrp = (int64_t)h->agrp_ptr.size() - 1;
  // boundary-row kernel input: non-Dirichlet boundary slots grouped by macro,
  // each macro padded to whole blocks so that a block sees a single macro
  std::vector<int32_t> bijk, bblk;
  std::vector<int64_t> dslot;
  std::vector<FaceTile> ftile;
  {
    size_t q = 0;
    for (int m = 0; m < M; ++m) {
      // rows inside a non-Dirichlet face are computed in face tiles, whose
      // two layers are staged in LDS once for all rows of the tile
      bool tiled[4];
      const int nm = h->minfo[m].n;
      for (int f = 0; f < 4; ++f) {
        tiled[f] = nm >= 6 && !((h->minfo[m].dmask >> (1u << f)) & 1u);
        if (!tiled[f]) continue;
        for (int b0 = 2; b0 <= nm - 4; b0 += FT_H)
          for (int a0 = 2; a0 + b0 <= nm - 2; a0 += FT_W) ftile.push_back({m, f, a0, b0});
      }
      size_t cnt = 0;
      // rows of one boundary primitive (face, edge, vertex) together, so that
      // the waves of the boundary-row kernel rarely diverge; then the
      // macro's Dirichlet slots (bit 30), whose rows the kernel sets to zero
      std::vector<std::pair<int, int32_t>> rows;
      std::vector<int32_t> drows;
      const int n = h->minfo[m].n;
      for (; q < bslot.size() && bslot[q].x == m; ++q) {
        const int i = bslot[q].y & 1023, j = (bslot[q].y >> 10) & 1023, k = (bslot[q].y >> 20) & 1023;
        const int64_t slot = h->minfo[m].off + plane_base(n, k) + tri(i + j) + i;
        if (h->flags[slot] & 1) {
          dslot.push_back(slot);
          drows.push_back(bslot[q].y | (1 << 30));
          continue;
        }
        const int z = ((n - i - j - k) == 0) | ((i == 0) << 1) | ((j == 0) << 2) | ((k == 0) << 3);
        if ((z & (z - 1)) == 0 && tiled[__builtin_ctz(z)]) {
          // deep rows of a tiled face (face coordinates a, b, n - a - b >= 2)
          const int f = __builtin_ctz(z);
          const int fa = f == 1 ? j : i, fb = (f == 0 || f == 3) ? j : k;
          if (fa >= 2 && fb >= 2 && n - fa - fb >= 2) continue;   // in a face tile
        }
        rows.push_back({z, bslot[q].y});
      }
      std::stable_sort(rows.begin(), rows.end(),
                       [](const std::pair<int, int32_t> &a, const std::pair<int, int32_t> &b) {
                         return a.first < b.first;
                       });
      for (auto &r : rows) bijk.push_back(r.second);
      for (int32_t v : drows) bijk.push_back(v);
      cnt = rows.size() + drows.size();
      const size_t pad = (BOUNDARY_BLOCK - cnt % BOUNDARY_BLOCK) % BOUNDARY_BLOCK;
      for (size_t r = 0; r < pad; ++r) bijk.push_back(-1);
      for (size_t r = 0; r < (cnt + pad) / BOUNDARY_BLOCK; ++r) bblk.push_back(m);
    }
  }
  int64_t nu = 0;
  for (uint8_t f : h->flags) nu += ((f & 2) && !(f & 1)) ? 1 : 0;
  h->n_unknown = nu;

  // --------------------------------------------------- interior work list
  const char *env = std::getenv("HHG_PLANES_PER_ITEM");
  if (env) h->planes_per_item = std::max(1, std::atoi(env));
  const char *envs = std::getenv("HHG_SERIAL_APPLY");
  h->serial_apply = envs && std::atoi(envs) == 1;
  {
    std::vector<int> all(M);
    for (int m = 0; m < M; ++m) all[m] = m;
    build_work(h, all, nullptr, h->work, h->wl_max);
  }
  h->n_work = (int)h->work.size();

  h->bijk = std::move(bijk);
  h->bblk = std::move(bblk);
  h->ftile = std::move(ftile);
  h->dslot = std::move(dslot);
  // every macro-boundary slot: the rows that the boundary-row kernel and the
  // copy-group sum complete, for the boundary part of a smoothing step
  h->bnd.clear();
  for (int64_t s = 0; s < h->n_nodes; ++s)
    if (h->flags[(size_t)s] & 4) h->bnd.push_back(s);
  h->n_bnd = (int64_t)h->bnd.size();
  h->grp_ptr = std::move(gptr);
  h->grp_slot = std::move(gslot);
  return HHG_OK;
}

}  // namespace

namespace {
// Workgroups an interior launch keeps resident on an MI355X: 256 compute
// units, three FP64 interior workgroups each (LDS and registers).
constexpr int RESIDENT_ITEMS = 768;
// Cost of one plane step of a chunk in units of one wave's row: the waves
// whose lowest anti-diagonal still has an interior row in plane k, plus the
// step's staging and barrier.
constexpr int STEP_OVERHEAD = 2;
int64_t step_cost(int n, int64_t p0, int CH, int k) {
  const int64_t npos = tri(n - 1);
  int64_t c = STEP_OVERHEAD;
  for (int64_t q = p0; q < std::min<int64_t>(p0 + CH, npos); q += 64)
    if (tri_root(q) + k <= n - 1) ++c;
  return c;
}
}  // namespace

void build_work(const hhg_ctx *h, const std::vector<int> &macros, const int *slab,
                std::vector<WorkItem> &out, int &wl_max) {
  const int CH = h->chunk;
  std::vector<WorkItem> natural;
  wl_max = 0;
  struct Column {
    int m, c, kmax, depth;
    std::vector<int64_t> cost;   // per plane 1..kmax (balanced columns)
  };
  std::vector<Column> cols;
  int64_t total_cost = 0;
  for (int m : macros) {
    const int n = h->minfo[m].n;
    const int lev = h->minfo[m].level;
    const int sl = (slab && slab[lev] != 0) ? slab[lev] : default_slab(h, lev);
    const int depth = sl == SLAB_BALANCED ? 0 : std::max(1, sl);
    const int64_t npos = tri(n - 1);  // interior positions live below T(n-1)
    const int nchunk = (int)((npos + CH - 1) / CH);
    for (int c = 0; c < nchunk; ++c) {
      const int64_t p0 = (int64_t)c * CH;
      const int64_t s_lo = tri_root(p0);
      const int64_t s_hi = std::min<int64_t>(tri_root(p0 + CH - 1), n - 2);
      const int64_t ws = std::max<int64_t>(0, p0 - s_lo - 1);
      wl_max = std::max<int>(wl_max, (int)(p0 + CH - 1 + s_hi + 2 - ws + 1));
      Column col{m, c, (int)(n - 1 - std::max<int64_t>(2, s_lo)), depth, {}};
      if (depth == 0) {
        col.cost.resize(col.kmax);
        for (int k = 1; k <= col.kmax; ++k) {
          col.cost[k - 1] = step_cost(n, p0, CH, k);
          total_cost += col.cost[k - 1];
        }
      }
      cols.push_back(std::move(col));
    }
  }
  // fixed depth: slabs of `depth` planes, plane range by plane range (all
  // chunks of a macro at the lowest planes first); balanced: every column
  // cut into consecutive segments of about total / RESIDENT_ITEMS cost
  const double target = std::max(1.0, (double)total_cost / RESIDENT_ITEMS);
  size_t q0 = 0;
  while (q0 < cols.size()) {
    size_t q1 = q0;
    while (q1 < cols.size() && cols[q1].m == cols[q0].m) ++q1;
    int kmax_all = 0;
    for (size_t q = q0; q < q1; ++q) kmax_all = std::max(kmax_all, cols[q].kmax);
    for (size_t q = q0; q < q1; ++q) {
      const Column &col = cols[q];
      if (col.depth != 0) continue;
      int ka = 1;
      double acc = 0.0;
      for (int k = 1; k <= col.kmax; ++k) {
        acc += (double)col.cost[k - 1];
        if (acc >= target || k == col.kmax) {
          natural.push_back({col.m, col.c, ka, k + 1});
          ka = k + 1;
          acc = 0.0;
        }
      }
    }
    for (int ka = 1; ka <= kmax_all; ka += 1)
      for (size_t q = q0; q < q1; ++q) {
        const Column &col = cols[q];
        if (col.depth == 0 || (ka - 1) % col.depth != 0) continue;
        if (ka <= col.kmax) natural.push_back({col.m, col.c, ka, std::min(ka + col.depth, col.kmax + 1)});
      }
    q0 = q1;
  }
  // workgroup g runs on XCD g % NXCD: give every XCD a contiguous stretch of
  // the natural order so that neighbouring chunks share its L2
  const size_t per = (natural.size() + NXCD - 1) / NXCD;
  out.assign(per * NXCD, WorkItem{-1, 0, 0, 0});
  for (size_t q = 0; q < natural.size(); ++q) {
    const size_t x = q / per, r = q % per;
    out[r * NXCD + x] = natural[q];
  }
}

// Upload the constant tables to the current device at the first device call.
int ensure_device(hhg_ctx *h) {
  int dev = 0;
  HHG_HIP(hipGetDevice(&dev));
  if (h->on_device) {
    if (dev != h->device) return fail(HHG_EINVAL, "handle used on a different device than its tables");
    return HHG_OK;
  }
  const int M = h->n_macro;
  h->device = dev;
  std::vector<StencilConst<float>> sc32(M);
  std::vector<ElemConst<float>> ec32(M);
  for (int m = 0; m < M; ++m) {
    convert(h->sc64[m], sc32[m]);
    convert(h->ec64[m], ec32[m]);
  }
  int rc;
  if ((rc = upload(&h->d_minfo, h->minfo.data(), M))) return rc;
  if ((rc = upload(&h->d_sc64, h->sc64.data(), M))) return rc;
  if ((rc = upload(&h->d_sc32, sc32.data(), M))) return rc;
  if ((rc = upload(&h->d_ec64, h->ec64.data(), M))) return rc;
  if ((rc = upload(&h->d_ec32, ec32.data(), M))) return rc;
  if ((rc = upload(&h->d_work, h->work.data(), h->work.size()))) return rc;
  if ((rc = upload(&h->d_bijk, h->bijk.data(), h->bijk.size()))) return rc;
  if ((rc = upload(&h->d_bblk, h->bblk.data(), h->bblk.size()))) return rc;
  if ((rc = upload(&h->d_ftile, h->ftile.data(), h->ftile.size()))) return rc;
  if ((rc = upload(&h->d_dslot, h->dslot.data(), h->dslot.size()))) return rc;
  if ((rc = upload(&h->d_bnd, h->bnd.data(), h->bnd.size()))) return rc;
  if ((rc = upload(&h->d_grp_ptr, h->grp_ptr.data(), h->grp_ptr.size()))) return rc;
  if ((rc = upload(&h->d_grp_slot, h->grp_slot.data(), h->grp_slot.size()))) return rc;
  if ((rc = upload(&h->d_flags, h->flags.data(), h->flags.size()))) return rc;
  if ((rc = upload(&h->d_agrp_ptr, h->agrp_ptr.data(), h->agrp_ptr.size()))) return rc;
  if ((rc = upload(&h->d_agrp_slot, h->agrp_slot.data(), h->agrp_slot.size()))) return rc;
  if ((rc = upload(&h->d_stc, h->stc.data(), h->stc.size()))) return rc;
  HHG_HIP(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
  HHG_HIP(hipStreamCreateWithFlags(&h->solve_stream, hipStreamNonBlocking));
  // The fork and join events only order the library's own streams on this
  // device; the host never waits on them.  The kernels' own dispatch fences
  // already make their writes visible across the XCDs, so the events skip
  // the system-scope fence (its L2 write-back cost ~3 us per apply).
  const unsigned evf = hipEventDisableTiming | hipEventDisableSystemFence;
  HHG_HIP(hipEventCreateWithFlags(&h->ev_fork, evf));
  HHG_HIP(hipEventCreateWithFlags(&h->ev_join, evf));
  h->on_device = true;
  h->device = dev;
  return HHG_OK;
}

}  // namespace hhg

extern "C" {

int hhg_setup_macro(const hhg_mesh_desc *mesh, const hhg_op_desc *op, hhg_handle *out) {
  using namespace hhg;
  if (!mesh || !op || !out) return fail(HHG_EINVAL, "null argument");
  *out = nullptr;
  if (mesh->n_macro < 1 || !mesh->verts || !mesh->level) return fail(HHG_EINVAL, "empty mesh");
  if (mesh->coupling != HHG_CONFORMING && mesh->coupling != HHG_INDEPENDENT)
    return fail(HHG_EINVAL, "unknown coupling");
  if (mesh->dirichlet != HHG_DIRICHLET_OUTER && mesh->dirichlet != HHG_DIRICHLET_NONE)
    return fail(HHG_EINVAL, "unknown dirichlet mode");
  if ((op->corr != HHG_CORR_PHYSICAL && op->corr != HHG_CORR_NONE) ||
      (op->khat != HHG_KHAT_PATCH && op->khat != HHG_KHAT_EDGE) ||
      (op->iface != HHG_IFACE_SYMMETRIC && op->iface != HHG_IFACE_ROWWISE &&
       op->iface != HHG_IFACE_ZEROSUM))
    return fail(HHG_EINVAL, "unknown operator variant");
  if (!std::isfinite(op->mu0) || !std::isfinite(op->mu1) || !std::isfinite(op->lam0) ||
      !std::isfinite(op->lam1))
    return fail(HHG_EINVAL, "non-finite form weight");
  hhg_ctx *h = nullptr;
  try {
    h = new hhg_ctx();
    int rc = setup_impl(mesh, op, h);
    if (rc) {
      free_ctx(h);
      return rc;
    }
  } catch (const std::bad_alloc &) {
    free_ctx(h);
    return fail(HHG_ENOMEM, "host allocation failed");
  } catch (...) {
    free_ctx(h);
    return fail(HHG_EINVAL, "unexpected exception in setup");
  }
  set_error("");
  *out = h;
  return HHG_OK;
}

int hhg_destroy(hhg_handle h) {
  hhg::free_ctx(h);
  return HHG_OK;
}

int hhg_layout(hhg_handle h, int64_t *n_nodes, int64_t *n_unknown, int64_t *macro_offset) {
  if (!h) return hhg::fail(HHG_EINVAL, "null handle");
  if (n_nodes) *n_nodes = h->n_nodes;
  if (n_unknown) *n_unknown = h->n_unknown;
  if (macro_offset) {
    for (int m = 0; m < h->n_macro; ++m) macro_offset[m] = h->minfo[m].off;
    macro_offset[h->n_macro] = h->n_nodes;
  }
  return HHG_OK;
}

int hhg_node_coords(hhg_handle h, double *xyz) {
  using namespace hhg;
  if (!h || !xyz) return fail(HHG_EINVAL, "null argument");
  const int64_t N = h->n_nodes;
  for (int m = 0; m < h->n_macro; ++m) {
    const int n = h->minfo[m].n;
    const double *V = h->verts.data() + 12 * m;
    for (int k = 0; k <= n; ++k)
      for (int s = 0; s + k <= n; ++s)
        for (int i = 0; i <= s; ++i) {
          const int j = s - i;
          const int64_t slot = h->minfo[m].off + plane_base(n, k) + tri(s) + i;
          for (int c = 0; c < 3; ++c)
            xyz[c * N + slot] = V[c] + ((double)i * (V[3 + c] - V[c]) + (double)j * (V[6 + c] - V[c]) +
                                        (double)k * (V[9 + c] - V[c])) / n;
        }
  }
  return HHG_OK;
}

int hhg_node_flags(hhg_handle h, uint8_t *flags) {
  if (!h || !flags) return hhg::fail(HHG_EINVAL, "null argument");
  std::memcpy(flags, h->flags.data(), h->flags.size());
  return HHG_OK;
}

const char *hhg_last_error(void) { return hhg::g_last_error.c_str(); }

}  // extern "C"
