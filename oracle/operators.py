"""Nodal integration and physical / unphysical stencil scaling (paper Sec. 2).

All operators are returned as SciPy CSR matrices over all unique micro nodes,
with row/column index 3*node + component and entries

    A[3i+m, 3j+l] = (a_ij)_{lm},

the paper's convention in which a_h(v, w) = sum v^(j)_l w^(i)_m (a_ij)_{lm}.
The operator description ``op`` is a dict with the constant (unscaled) and the
k-scaled weights of 2 mu (eps, eps) + lam (div, div):

    op = dict(mu0=..., lam0=..., mu1=..., lam1=...)

so the coefficient of the paper's problem is mu(x) = mu0 + mu1 k(x),
lam(x) = lam0 + lam1 k(x) with one nodal scalar field k.

Methods
-------
``nodal``   a_h of eq. nodalintegration with kbar^t the vertex mean of eq.
            nodalquad (the constant part is integrated exactly).
``scaled``  hat a_h of the Lemma: for a macro-interior row i and j != i,
            S_ij = A0_ij + khat_ij Shat_ij + R_ij with khat the patch mean of
            eq. patchmean, Shat_ij = sum_t a^{s;t}_ij and
            R_ij = 1/2 sum_t (kbar^t - kbar^{t^m}) a^{a;t}_ij (eq.
            corrtermgeneral), t^m the element reflected through the midpoint
            of edge ij; the centre entry is minus the sum of the others.
            ``corr='none'`` drops R (unphysical scaling, eq.
            stencilscalingwithoutcorr); ``khat='edge'`` uses (k_i + k_j)/2
            (Remark after the Lemma).
Rows of nodes on a macro boundary follow Sec. 2.2: ``iface='symmetric'`` uses
nodal entries when both x_i and x_j lie on dT of the macro and the scaled entry
otherwise (diagonal nodal); ``iface='rowwise'`` uses the nodal row for every
node on a macro boundary; ``iface='zerosum'`` takes the off-diagonal entries
of the symmetric rule and sets the centre of every row to minus the sum of
the others, as the Lemma does for macro-interior rows (not in the paper: the
interface rows then keep translations in their kernel, and since the
off-diagonal entries are those of a symmetric matrix and their block row sums
are symmetric 3x3 blocks, the matrix stays symmetric).

Parity: pinned by tests against what the paper fixes (equal to nodal
integration for constant and for affine k on macro-interior rows, unphysical
differs for non-constant affine k, symmetry, zero row sums, rigid-body kernel,
O(h^2) vs O(h) consistency for smooth k).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .forms import form_tensor, sym_part, antisym_part, p1_gradients
from .mesh import MacroMesh


def _check_op(op):
    out = dict(mu0=0.0, lam0=0.0, mu1=0.0, lam1=0.0)
    for key, val in op.items():
        if key not in out:
            raise KeyError(key)
        out[key] = float(val)
    return out


def _tets_touching(mesh: MacroMesh, m: int, rows_mask):
    tets = mesh.local_tets[m]
    if rows_mask is None:
        return np.arange(tets.shape[0]), None
    local_rows = rows_mask[mesh.gid[m]]
    sel = np.nonzero(local_rows[tets].any(axis=1))[0]
    return sel, local_rows


def _emit(blocks, gi, gj, rows_out, cols_out, vals_out):
    """Append 3x3 blocks [l, m] for (row node gi, column node gj)."""
    if blocks.shape[0] == 0:
        return
    l, mm = np.meshgrid(np.arange(3), np.arange(3), indexing="ij")
    rows_out.append((3 * gi[:, None, None] + mm[None]).ravel())
    cols_out.append((3 * gj[:, None, None] + l[None]).ravel())
    vals_out.append(blocks.ravel())


def nodal_matrix(mesh: MacroMesh, k, op, rows=None) -> sp.csr_matrix:
    """Nodal integration a_h (eq. nodalintegration), unreduced (no Dirichlet).

    Entry (i, j): sum over macros T and elements t of T containing i and j of
    a0^t_ij + kbar^t a1^t_ij, kbar^t the mean of k over the 4 vertices.
    ``rows`` restricts the computed rows to the given node ids.
    """
    op = _check_op(op)
    k = np.asarray(k, dtype=np.float64)
    rows_mask = _rows_mask(mesh, rows)
    R, C, V = [], [], []
    for m in range(mesh.n_macro):
        sel, local_rows = _tets_touching(mesh, m, rows_mask)
        tets = mesh.local_tets[m][sel]
        if tets.shape[0] == 0:
            continue
        X = mesh.local_xyz[m][tets]
        a0 = form_tensor(X, op["mu0"], op["lam0"])
        a1 = form_tensor(X, op["mu1"], op["lam1"])
        g = mesh.gid[m][tets]
        kbar = k[g].mean(axis=1)
        blk = a0 + kbar[:, None, None, None, None] * a1       # [t, i, j, l, m]
        for a in range(4):
            for b in range(4):
                keep = slice(None) if local_rows is None else local_rows[tets[:, a]]
                _emit(blk[keep, a, b], g[keep, a], g[keep, b], R, C, V)
    return _to_csr(mesh, R, C, V)


def _rows_mask(mesh, rows):
    if rows is None:
        return None
    mask = np.zeros(mesh.n_nodes, dtype=bool)
    mask[np.asarray(rows, dtype=np.int64)] = True
    return mask


def _to_csr(mesh, R, C, V):
    N = 3 * mesh.n_nodes
    if not R:
        return sp.csr_matrix((N, N))
    A = sp.coo_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))),
                      shape=(N, N)).tocsr()
    A.sum_duplicates()
    return A


def _set_keys(verts: np.ndarray, N: int) -> np.ndarray:
    """Exact key of a 4-vertex set: sorted ids (a<b<c<d) packed as the complex
    number (a N + b) + i (c N + d); exact in float64 while N^2 < 2^53, and
    complex arrays sort lexicographically (real part, then imaginary)."""
    v = np.sort(verts, axis=1).astype(np.float64)
    return (v[:, 0] * N + v[:, 1]) + 1j * (v[:, 2] * N + v[:, 3])


def _tet_lookup(tets: np.ndarray, N: int):
    """Sorted element keys for membership queries of vertex sets."""
    if float(N) * N >= 2.0 ** 53:
        raise ValueError("macro too large for exact element keys")
    key = _set_keys(tets, N)
    order = np.argsort(key, kind="stable")
    return key[order], order, N


def _find_tets(lookup, query: np.ndarray) -> np.ndarray:
    """Element id of each queried vertex set, -1 if it is not an element."""
    skey, order, N = lookup
    q = _set_keys(query, N)
    pos = np.minimum(np.searchsorted(skey, q), skey.shape[0] - 1)
    hit = skey[pos] == q
    return np.where(hit, order[pos], -1)


def scaled_matrix(mesh: MacroMesh, k, op, rows=None, corr="physical",
                  khat="patch", iface="symmetric", return_parts=False):
    """Physical (or unphysical) stencil scaling hat a_h, unreduced.

    For every macro T, every node i of T and every neighbour j of i in T, the
    elements T_ij of T containing edge ij are collected.  Macro-interior rows
    use the Lemma; rows on dT use the chosen interface rule.  With
    ``return_parts`` the per-edge pieces (khat, Shat, R, nodal block) of
    macro-interior rows are also returned for inspection by tests.
    """
    op = _check_op(op)
    if corr not in ("physical", "none"):
        raise ValueError(corr)
    if khat not in ("patch", "edge"):
        raise ValueError(khat)
    if iface not in ("symmetric", "rowwise", "zerosum"):
        raise ValueError(iface)
    k = np.asarray(k, dtype=np.float64)
    rows_mask = _rows_mask(mesh, rows)
    R, C, V = [], [], []
    parts = []
    for m in range(mesh.n_macro):
        n = 1 << int(mesh.levels[m])
        sel, local_rows = _tets_touching(mesh, m, rows_mask)
        all_tets = mesh.local_tets[m]
        tets = all_tets[sel]
        if tets.shape[0] == 0:
            continue
        ijk = mesh.local_ijk[m]
        gid = mesh.gid[m]
        onb = mesh.on_macro_boundary[m]
        N = ijk.shape[0]
        X = mesh.local_xyz[m][tets]
        a0 = form_tensor(X, op["mu0"], op["lam0"])
        a1 = form_tensor(X, op["mu1"], op["lam1"])
        kbar = k[gid[tets]].mean(axis=1)

        # dense lookup of index triples -> local node id (for reflections)
        cube = np.full((n + 1,) * 3, -1, dtype=np.int64)
        cube[ijk[:, 0], ijk[:, 1], ijk[:, 2]] = np.arange(N)
        lookup = _tet_lookup(all_tets, N)

        # all (element, test vertex a, trial vertex b), a != b
        T = tets.shape[0]
        ta, aa, bb = [], [], []
        for a in range(4):
            for b in range(4):
                if a != b:
                    ta.append(np.arange(T))
                    aa.append(np.full(T, a))
                    bb.append(np.full(T, b))
        ta = np.concatenate(ta)
        aa = np.concatenate(aa)
        bb = np.concatenate(bb)
        i_loc = tets[ta, aa]
        j_loc = tets[ta, bb]
        if local_rows is not None:
            keep = local_rows[i_loc]
            ta, aa, bb, i_loc, j_loc = ta[keep], aa[keep], bb[keep], i_loc[keep], j_loc[keep]

        blk1 = a1[ta, aa, bb]                           # (P, 3, 3) [l, m]
        blk0 = a0[ta, aa, bb]
        kb = kbar[ta]

        # reflected element t^m: vertices x_i + x_j - v
        refl_ijk = ijk[i_loc][:, None, :] + ijk[j_loc][:, None, :] - ijk[tets[ta]]
        inside = np.all((refl_ijk >= 0) & (refl_ijk.sum(axis=2, keepdims=True) <= n), axis=2).all(axis=1)
        refl_ijk_c = np.clip(refl_ijk, 0, n)
        refl_nodes = cube[refl_ijk_c[..., 0], refl_ijk_c[..., 1], refl_ijk_c[..., 2]]
        refl_nodes = np.where(inside[:, None], refl_nodes, -1)
        tm = np.full(ta.shape[0], -1, dtype=np.int64)
        ok = inside & np.all(refl_nodes >= 0, axis=1)
        if np.any(ok):
            tm[ok] = _find_tets(lookup, refl_nodes[ok])
        kb_m = np.where(tm >= 0, k[gid[np.maximum(refl_nodes, 0)]].mean(axis=1), np.nan)

        # group by directed edge (i, j)
        ekey = i_loc * N + j_loc
        uk, grp = np.unique(ekey, return_inverse=True)
        G = uk.shape[0]
        ei, ej = uk // N, uk % N
        cnt = np.bincount(grp, minlength=G).astype(np.float64)

        def gsum(vals):
            flat = vals.reshape(vals.shape[0], -1)
            out = np.stack([np.bincount(grp, weights=flat[:, c], minlength=G)
                            for c in range(flat.shape[1])], axis=1)
            return out.reshape((G,) + vals.shape[1:])

        khat_patch = gsum(kb) / cnt
        Shat = gsum(sym_part(blk1))
        Rcorr = 0.5 * gsum((kb - kb_m)[:, None, None] * antisym_part(blk1))
        A0sum = gsum(blk0)
        nodal = gsum(blk0 + kb[:, None, None] * blk1)
        complete = gsum((tm >= 0).astype(np.float64)) == cnt

        kh = khat_patch if khat == "patch" else 0.5 * (k[gid[ei]] + k[gid[ej]])
        scaled = A0sum + kh[:, None, None] * Shat
        if corr == "physical":
            scaled = scaled + Rcorr

        i_int = ~onb[ei]
        j_int = ~onb[ej]
        use_scaled = i_int | ((iface != "rowwise") & j_int)
        if np.any(use_scaled & ~complete):
            raise RuntimeError("scaled entry requested on an incomplete edge patch")
        value = np.where(use_scaled[:, None, None], scaled, nodal)
        _emit(value, gid[ei], gid[ej], R, C, V)

        # centre entries: minus the sum of the row's other entries from this
        # macro (macro-interior rows; every row under the zero-sum rule)
        diag = np.zeros((N, 3, 3))
        rows_int = i_int | (iface == "zerosum")
        np.add.at(diag, ei[rows_int], -value[rows_int])
        # nodes on dT (symmetric and row-wise rules): nodal diagonal from this
        # macro's elements
        dsel = []
        for a in range(4):
            il = tets[:, a]
            keep = onb[il]
            if local_rows is not None:
                keep &= local_rows[il]
            if iface == "zerosum":
                keep = np.zeros_like(keep)
            dsel.append((il[keep], a0[keep, a, a] + kbar[keep, None, None] * a1[keep, a, a]))
        for il, blk in dsel:
            np.add.at(diag, il, blk)
        touched = np.unique(ei)
        if local_rows is not None:
            touched = touched[local_rows[touched]]
        bnd_rows = np.unique(np.concatenate([d[0] for d in dsel])) if dsel else np.zeros(0, np.int64)
        dn = np.union1d(touched, bnd_rows)
        _emit(diag[dn], gid[dn], gid[dn], R, C, V)

        if return_parts:
            sel_int = i_int
            parts.append(dict(macro=m, i=ei[sel_int], j=ej[sel_int], khat=kh[sel_int],
                              Shat=Shat[sel_int], R=Rcorr[sel_int], nodal=nodal[sel_int],
                              A0=A0sum[sel_int], count=cnt[sel_int]))
    A = _to_csr(mesh, R, C, V)
    return (A, parts) if return_parts else A


def mass_matrix(mesh: MacroMesh) -> sp.csr_matrix:
    """Scalar P1 mass matrix (n_nodes x n_nodes): the element integral of
    phi_a phi_b is |t| (1 + delta_ab) / 20."""
    R, C, V = [], [], []
    for m in range(mesh.n_macro):
        tets = mesh.local_tets[m]
        _, vol = p1_gradients(mesh.local_xyz[m][tets])
        g = mesh.gid[m][tets]
        for a in range(4):
            for b in range(4):
                R.append(g[:, a])
                C.append(g[:, b])
                V.append(vol * ((2.0 if a == b else 1.0) / 20.0))
    n = mesh.n_nodes
    return sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))), shape=(n, n))


def operator_matrix(mesh, k, op, method="scaled", **kw):
    if method == "scaled":
        return scaled_matrix(mesh, k, op, **kw)
    if method == "nodal":
        return nodal_matrix(mesh, k, op, rows=kw.get("rows"))
    raise ValueError(method)


def reduce_dirichlet(mesh: MacroMesh, A: sp.spmatrix) -> sp.csr_matrix:
    """Principal submatrix on the unknown (non-Dirichlet) DoFs."""
    u = mesh.unknown
    dof = (3 * u[:, None] + np.arange(3)[None]).ravel()
    return A.tocsr()[dof][:, dof]


def unknown_dofs(mesh: MacroMesh) -> np.ndarray:
    u = mesh.unknown
    return (3 * u[:, None] + np.arange(3)[None]).ravel()


def apply(mesh: MacroMesh, k, op, x, method="scaled", rows=None, **kw) -> np.ndarray:
    """y = A x with homogeneous Dirichlet nodes eliminated.

    ``x`` is (n_nodes, 3); Dirichlet entries of x are treated as zero and
    Dirichlet rows of y are zero.  With ``rows`` only those rows are computed
    (the others are returned as NaN).
    """
    x = np.array(x, dtype=np.float64).reshape(mesh.n_nodes, 3)
    x[mesh.dirichlet] = 0.0
    A = operator_matrix(mesh, k, op, method=method, rows=rows, **kw)
    y = (A @ x.ravel()).reshape(mesh.n_nodes, 3)
    y[mesh.dirichlet] = 0.0
    if rows is not None:
        out = np.full_like(y, np.nan)
        out[rows] = y[rows]
        return out
    return y
