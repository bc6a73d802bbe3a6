"""The 2-D variant of the method (paper Sec. 2 and Sec. 2.3): macro triangles
refined uniformly, the P1 vector forms in two dimensions, nodal integration
and physical stencil scaling with the 2-D correction.  TEST INFRASTRUCTURE
ONLY (tests, smoke check, CPU baseline); no code shared with the HIP library.

* Refinement: each triangle splits into its four children through the edge
  midpoints (the 2-D counterpart of the refinement of Sec. 2), carried out in
  integer index space where a macro's vertices x0, x1, x2 sit at (0,0),
  (n,0), (0,n), n = 2^level; node (i, j) lies at x0 + (i/n)(x1-x0) +
  (j/n)(x2-x0).
* Forms: 2 mu (eps(u), eps(v)) + lam (div u, div v) with
  (a^t_ij)_{lm} = int_t (D(phi_j e_l), D(phi_i e_m)), as in 3-D; the operator
  is A0 + k A1 with A0 from (mu0, lam0) and A1 from (mu1, lam1).
* Nodal integration: element t contributes A0^t + kbar^t A1^t, kbar^t the
  vertex mean (eq. nodalquad).
* Physical scaling (Lemma), macro-interior row i, j != i:
  S_ij = sum_{t in T_ij} A0^t_ij + khat_ij a^{s;t}_ij
         + 1/2 (kbar^t - kbar^{t^m}) a^{a;t}_ij,
  khat_ij the mean of kbar^t over the edge patch (eq. patchmean), t^m the
  element reflected through the midpoint of edge ij (found geometrically);
  in 2-D every interior edge has two elements, t and t^m of each other.  The
  centre entry is minus the sum of the others.  corr="none" drops the
  correction (unphysical scaling).
* Rows of nodes on a macro boundary: iface="symmetric" (nodal entries
  between two macro-boundary nodes and on the diagonal, scaled entries
  towards macro-interior neighbours), "rowwise" (the whole nodal row) or
  "zerosum" (the symmetric rule's off-diagonal entries, the centre minus
  their sum), as in 3-D (Sec. 2.2).
* Dirichlet: homogeneous on every macro edge owned by a single macro
  (dirichlet="outer"); rows and columns of those nodes are removed.

Parity: pinned by tests (mesh counts and areas, element-matrix null space
and symmetry, the closed form eq. correction2d of the correction with its
orientation sign and the factor its derivation implies, scaled = nodal for
constant k and on interior rows for affine k, O(h^2) against O(h)
consistency, symmetry, SPD, planted mistakes).
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp


# ------------------------------------------------------------------ mesh
def red_children(t: np.ndarray) -> np.ndarray:
    """One uniform refinement step: (T, 3, 2) integer triangles (even
    coordinates) -> (4T, 3, 2): the three corner triangles and the middle
    one through the edge midpoints."""
    x0, x1, x2 = t[:, 0], t[:, 1], t[:, 2]
    m01, m02, m12 = (x0 + x1) // 2, (x0 + x2) // 2, (x1 + x2) // 2
    kids = [(x0, m01, m02), (m01, x1, m12), (m02, m12, x2), (m12, m02, m01)]
    return np.concatenate([np.stack(k, axis=1) for k in kids], axis=0)


@functools.lru_cache(maxsize=16)
def reference_refinement(level: int):
    """(ij (N, 2) node index pairs, tris (n^2, 3) local node ids) of the
    refined reference triangle."""
    n = 1 << level
    t = np.array([[[0, 0], [n, 0], [0, n]]], dtype=np.int64)
    for _ in range(level):
        t = red_children(t)
    flat = t.reshape(-1, 2)
    key = flat[:, 0] * (n + 1) + flat[:, 1]
    ukey, inv = np.unique(key, return_inverse=True)
    ij = np.column_stack([ukey // (n + 1), ukey % (n + 1)])
    return ij, inv.reshape(-1, 3).astype(np.int64)


class Mesh2D:
    """Conforming macro triangulation with its uniform refinement.

    verts (M, 3, 2); level (common); dirichlet "outer" or "none".
    Attributes as the 3-D MacroMesh: n_nodes, xy, gid, local_ij, local_tris,
    local_xy, on_macro_boundary, interface, dirichlet, unknown.
    """

    def __init__(self, verts, level, dirichlet="outer"):
        verts = np.asarray(verts, dtype=np.float64)
        if verts.ndim != 3 or verts.shape[1:] != (3, 2):
            raise ValueError("verts must be (M,3,2)")
        self.verts = verts
        self.n_macro = verts.shape[0]
        self.level = int(level)
        n = 1 << self.level
        ij, tris = reference_refinement(self.level)
        self.local_ij, self.local_tris, self.local_xy, self.on_macro_boundary = [], [], [], []
        for m in range(self.n_macro):
            x0 = verts[m, 0]
            E = verts[m, 1:] - x0
            self.local_ij.append(ij)
            self.local_tris.append(tris)
            self.local_xy.append(x0 + (ij / n) @ E)
            self.on_macro_boundary.append((ij[:, 0] == 0) | (ij[:, 1] == 0) | (ij.sum(1) == n))
        # global numbering by coordinates (rounded to a fraction of h)
        scale = (np.abs(verts).max() + 1.0) * 1e-9 / n
        keys, gid = {}, []
        for m in range(self.n_macro):
            g = np.empty(len(ij), dtype=np.int64)
            for a, x in enumerate(self.local_xy[m]):
                kk = (int(round(x[0] / scale)), int(round(x[1] / scale)))
                g[a] = keys.setdefault(kk, len(keys))
            gid.append(g)
        self.gid = gid
        self.n_nodes = len(keys)
        self.xy = np.zeros((self.n_nodes, 2))
        for m in range(self.n_macro):
            self.xy[gid[m]] = self.local_xy[m]
        self.interface = np.zeros(self.n_nodes, dtype=bool)
        for m in range(self.n_macro):
            self.interface[gid[m][self.on_macro_boundary[m]]] = True
        self.dirichlet = np.zeros(self.n_nodes, dtype=bool)
        if dirichlet == "outer":
            # a macro edge met by one macro only lies on the domain boundary
            count = {}
            ekeys = []
            for m in range(self.n_macro):
                for a, b in ((0, 1), (1, 2), (2, 0)):
                    k2 = tuple(sorted((tuple(np.round(verts[m, a], 9)), tuple(np.round(verts[m, b], 9)))))
                    count[k2] = count.get(k2, 0) + 1
                    ekeys.append((m, a, b, k2))
            for m, a, b, k2 in ekeys:
                if count[k2] != 1:
                    continue
                bi, bj = ij[:, 0], ij[:, 1]
                bc = np.column_stack([n - bi - bj, bi, bj])      # barycentric x n
                c = 3 - a - b                                    # opposite vertex
                on = bc[:, c] == 0
                self.dirichlet[gid[m][on]] = True
        elif dirichlet != "none":
            raise ValueError(dirichlet)
        self.unknown = np.nonzero(~self.dirichlet)[0]


# ------------------------------------------------------------------ forms
def p1_gradients(X: np.ndarray):
    """Gradients of the barycentric basis on triangles X (T, 3, 2):
    (grad (T, 3, 2), area (T,))."""
    X = np.asarray(X, dtype=np.float64)
    M = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))
    Minv = np.linalg.inv(M)
    g = np.empty(X.shape)
    g[:, 1:, :] = Minv
    g[:, 0, :] = -Minv.sum(axis=1)
    return g, np.abs(np.linalg.det(M)) / 2.0


def form_tensor(X: np.ndarray, mu: float, lam: float) -> np.ndarray:
    """(a^t_ij)_{lm} of 2 mu (eps, eps) + lam (div, div): [t, i, j, l, m]."""
    g, area = p1_gradients(X)
    eye = np.eye(2)
    grad_u = np.einsum("lp,taq->talpq", eye, g)              # d_q (phi_a e_l)_p
    E = 0.5 * (grad_u + np.swapaxes(grad_u, -1, -2))
    out = np.zeros((X.shape[0], 3, 3, 2, 2))
    if mu != 0.0:
        out += 2.0 * mu * area[:, None, None, None, None] * np.einsum("tjlpq,timpq->tijlm", E, E)
    if lam != 0.0:
        out += lam * area[:, None, None, None, None] * np.einsum("tjl,tim->tijlm", g, g)
    return out


def sym_part(a):
    return 0.5 * (a + np.swapaxes(a, -1, -2))


def antisym_part(a):
    return 0.5 * (a - np.swapaxes(a, -1, -2))


# ------------------------------------------------------------------ operators
def _op(op):
    o = dict(mu0=0.0, lam0=0.0, mu1=0.0, lam1=0.0)
    o.update(op)
    return o


def _to_csr(mesh, R, C, V):
    n = mesh.n_nodes
    if not R:
        return sp.csr_matrix((2 * n, 2 * n))
    gi, gj, B = np.concatenate(R), np.concatenate(C), np.concatenate(V)
    # y_{i,m} = sum_j sum_l B_ij[l][m] x_{j,l}
    rows = (2 * gi[:, None, None] + np.arange(2)[None, None, :]).repeat(2, axis=1)
    cols = (2 * gj[:, None, None] + np.arange(2)[None, :, None]).repeat(2, axis=2)
    return sp.csr_matrix((B.ravel(), (rows.ravel(), cols.ravel())), shape=(2 * n, 2 * n))


def nodal_matrix(mesh: Mesh2D, k, op) -> sp.csr_matrix:
    o = _op(op)
    k = np.asarray(k, dtype=np.float64)
    R, C, V = [], [], []
    for m in range(mesh.n_macro):
        tris = mesh.local_tris[m]
        X = mesh.local_xy[m][tris]
        a = form_tensor(X, o["mu0"], o["lam0"])
        a1 = form_tensor(X, o["mu1"], o["lam1"])
        kbar = k[mesh.gid[m][tris]].mean(axis=1)
        blk = a + kbar[:, None, None, None, None] * a1
        g = mesh.gid[m][tris]
        for i in range(3):
            for j in range(3):
                R.append(g[:, i])
                C.append(g[:, j])
                V.append(blk[:, i, j])
    return _to_csr(mesh, R, C, V)


def scaled_matrix(mesh: Mesh2D, k, op, corr="physical", iface="symmetric", return_parts=False):
    """Physically (or unphysically) scaled operator, unreduced."""
    o = _op(op)
    if corr not in ("physical", "none") or iface not in ("symmetric", "rowwise", "zerosum"):
        raise ValueError((corr, iface))
    k = np.asarray(k, dtype=np.float64)
    R, C, V, parts = [], [], [], []
    for m in range(mesh.n_macro):
        tris = mesh.local_tris[m]
        xy = mesh.local_xy[m]
        gid = mesh.gid[m]
        onb = mesh.on_macro_boundary[m]
        X = xy[tris]
        a0 = form_tensor(X, o["mu0"], o["lam0"])
        a1 = form_tensor(X, o["mu1"], o["lam1"])
        kbar = k[gid[tris]].mean(axis=1)
        # element lookup by its sorted vertex set, for the reflections
        lookup = {tuple(sorted(t)): q for q, t in enumerate(tris.tolist())}
        key = {tuple(np.round(p, 12)): a for a, p in enumerate(xy)}
        edges = {}
        for q, t in enumerate(tris):
            for ia in range(3):
                for ja in range(3):
                    if ia != ja:
                        edges.setdefault((t[ia], t[ja]), []).append((q, ia, ja))
        diag = {}
        for (i, j), lst in edges.items():
            nodal = sum(a0[q, ia, ja] + kbar[q] * a1[q, ia, ja] for q, ia, ja in lst)
            use_scaled = (not onb[i]) or (iface != "rowwise" and not onb[j])
            if use_scaled:
                if len(lst) != 2:
                    raise RuntimeError("scaled entry on an incomplete edge patch")
                khat = np.mean([kbar[q] for q, _, _ in lst])
                val = sum(a0[q, ia, ja] + khat * sym_part(a1[q, ia, ja]) for q, ia, ja in lst)
                parts_R = np.zeros((2, 2))
                if corr == "physical":
                    for q, ia, ja in lst:
                        # t^m: the other vertex reflected through the edge midpoint
                        other = [v for v in tris[q] if v != i and v != j][0]
                        pm = xy[i] + xy[j] - xy[other]
                        vm = key[tuple(np.round(pm, 12))]
                        qm = lookup[tuple(sorted((i, j, vm)))]
                        parts_R += 0.5 * (kbar[q] - kbar[qm]) * antisym_part(a1[q, ia, ja])
                    val = val + parts_R
                if return_parts and not onb[i]:
                    parts.append(dict(macro=m, i=i, j=j, R=parts_R, khat=khat,
                                      others=[[v for v in tris[q] if v != i and v != j][0]
                                              for q, _, _ in lst]))
            else:
                val = nodal
            R.append(np.array([gid[i]]))
            C.append(np.array([gid[j]]))
            V.append(val[None])
            if (not onb[i]) or iface == "zerosum":
                diag[i] = diag.get(i, 0.0) - val
        for i in range(len(xy)):
            if onb[i] and iface != "zerosum":
                d = np.zeros((2, 2))
                for q, t in enumerate(tris):
                    for ia in range(3):
                        if t[ia] == i:
                            d = d + a0[q, ia, ia] + kbar[q] * a1[q, ia, ia]
                diag[i] = d
        for i, d in diag.items():
            R.append(np.array([gid[i]]))
            C.append(np.array([gid[i]]))
            V.append(np.asarray(d)[None])
    A = _to_csr(mesh, R, C, V)
    return (A, parts) if return_parts else A


def reduce_dirichlet(mesh: Mesh2D, A: sp.spmatrix) -> sp.csr_matrix:
    dof = unknown_dofs(mesh)
    return A.tocsr()[dof][:, dof]


def unknown_dofs(mesh: Mesh2D) -> np.ndarray:
    u = mesh.unknown
    return (2 * u[:, None] + np.arange(2)[None]).ravel()


def apply(mesh: Mesh2D, k, op, x, method="scaled", **kw) -> np.ndarray:
    """y = A x with Dirichlet rows zero and Dirichlet entries of x read as 0:
    x, y (n_nodes, 2)."""
    A = scaled_matrix(mesh, k, op, **kw) if method == "scaled" else nodal_matrix(mesh, k, op)
    xx = np.array(x, dtype=np.float64).reshape(-1, 2)
    xx[mesh.dirichlet] = 0.0
    y = (A @ xx.ravel()).reshape(-1, 2)
    y[mesh.dirichlet] = 0.0
    return y
