"""Geometric multigrid over the uniform refinement hierarchy (test infrastructure).

The paper solves its systems with multigrid V-cycles on the hierarchy of
uniformly refined macro meshes (Sec. 5 and 6: V(3,3) cycles, scaled stencils
on every level).  This module states the plain definitions the GPU hierarchy
is checked against:

* ``prolongation``   P1 interpolation from level l to level l + 1 of the same
                     macro mesh: a fine node that is a coarse node keeps its
                     value, every other fine node is the midpoint of one coarse
                     lattice edge and takes the mean of its two end values
                     (the refinement of Sec. 2 halves every edge).
* ``inject``         a nodal coefficient restricted to the coarse nodes.
* ``Hierarchy``      the Dirichlet-reduced operators of every level (scaled
                     stencils rediscretised on each level with the injected
                     coefficient), the reduced transfers P and R = P^T and the
                     inverse 3x3 diagonal blocks.
* ``vcycle``         one V(nu1, nu2) cycle: damped block-Jacobi smoothing,
                     residual restriction, coarse correction, smoothing; an
                     exact solve on the coarsest level; optionally the
                     variable cycle (more smoothing on coarser levels).
* ``mg_pcg``         conjugate gradients preconditioned by one V-cycle.

Reading: the paper smooths with a hybrid Gauss-Seidel; here the smoother is
damped block Jacobi (x += omega D^-1 (b - A x) with the 3x3 node blocks D), the
parallel smoother the GPU hierarchy uses.  Equal pre- and post-smoothing
with a symmetric smoother keeps the V-cycle symmetric, so it can precondition
CG.

Parity: pinned by tests.  P reproduces affine fields exactly and its rows
sum to one; for a constant coefficient the rediscretised coarse operator
equals the Galerkin product P^T A_fine P (nested P1 spaces, exact element
integrals); the V-cycle contracts at a level-independent rate; MG-PCG and
the sparse direct solve agree.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import operators as O
from .mesh import MacroMesh
from .solvers import block_jacobi_inverse

# one lattice direction per parity pattern of a fine index triple: the fine
# node F with that pattern is the midpoint of (F - d) / 2 and (F + d) / 2
_PARITY_DIR = {
    (1, 0, 0): (1, 0, 0), (0, 1, 0): (0, 1, 0), (0, 0, 1): (0, 0, 1),
    (1, 1, 0): (1, -1, 0), (1, 0, 1): (1, 0, -1), (0, 1, 1): (0, 1, -1),
    (1, 1, 1): (1, -1, 1),
}


def _local_index(ijk: np.ndarray, n: int) -> np.ndarray:
    """Dense lookup (i, j, k) -> macro-local node number."""
    look = np.full((n + 1) ** 3, -1, dtype=np.int64)
    look[(ijk[:, 0] * (n + 1) + ijk[:, 1]) * (n + 1) + ijk[:, 2]] = np.arange(ijk.shape[0])
    return look


def prolongation(coarse: MacroMesh, fine: MacroMesh) -> sp.csr_matrix:
    """Node-level P1 interpolation matrix (fine nodes x coarse nodes)."""
    if coarse.n_macro != fine.n_macro or np.any(fine.levels != coarse.levels + 1):
        raise ValueError("fine must be the next level of the same macro mesh")
    rows, cols, vals = [], [], []
    for m in range(coarse.n_macro):
        nc = 1 << int(coarse.levels[m])
        look = _local_index(coarse.local_ijk[m], nc)
        F = fine.local_ijk[m]
        par = F & 1
        gf = fine.gid[m]
        gc = coarse.gid[m]
        even = ~par.any(axis=1)
        e_idx = np.nonzero(even)[0]
        c = F[e_idx] // 2
        rows.append(gf[e_idx])
        cols.append(gc[look[(c[:, 0] * (nc + 1) + c[:, 1]) * (nc + 1) + c[:, 2]]])
        vals.append(np.ones(e_idx.shape[0]))
        for pat, d in _PARITY_DIR.items():
            sel = np.nonzero(np.all(par == np.array(pat), axis=1))[0]
            if sel.size == 0:
                continue
            d = np.array(d)
            for end in (F[sel] - d, F[sel] + d):
                ab = end // 2
                li = look[(ab[:, 0] * (nc + 1) + ab[:, 1]) * (nc + 1) + ab[:, 2]]
                if np.any(li < 0):
                    raise AssertionError("edge end outside the coarse macro")
                rows.append(gf[sel])
                cols.append(gc[li])
                vals.append(np.full(sel.size, 0.5))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    # a node shared by several macros is listed once per macro with equal
    # weights: keep one copy of every (row, column) entry
    key = r * coarse.n_nodes + c
    _, first = np.unique(key, return_index=True)
    return sp.csr_matrix((v[first], (r[first], c[first])), shape=(fine.n_nodes, coarse.n_nodes))


def inject(coarse: MacroMesh, fine: MacroMesh, k_fine: np.ndarray) -> np.ndarray:
    """Nodal values of the fine coefficient at the coarse nodes."""
    kc = np.empty(coarse.n_nodes)
    for m in range(coarse.n_macro):
        nf = 1 << int(fine.levels[m])
        look = _local_index(fine.local_ijk[m], nf)
        F = 2 * coarse.local_ijk[m]
        kc[coarse.gid[m]] = k_fine[fine.gid[m][look[(F[:, 0] * (nf + 1) + F[:, 1]) * (nf + 1) + F[:, 2]]]]
    return kc


def reduced_prolongation(coarse: MacroMesh, fine: MacroMesh) -> sp.csr_matrix:
    """P on the unknown DoFs (3 components per node, Dirichlet rows and
    columns removed: Dirichlet values are zero on every level)."""
    P = sp.kron(prolongation(coarse, fine), sp.identity(3), format="csr")
    return P[O.unknown_dofs(fine)][:, O.unknown_dofs(coarse)].tocsr()


class Hierarchy:
    """Levels coarse..fine of one macro mesh with the operators of each.

    ``k_fine`` is the nodal coefficient on the finest level; coarser levels
    use its injection.  ``op`` and the keywords go to the scaled operator."""

    def __init__(self, verts, coarse_level: int, fine_level: int, k_fine, op, method="scaled",
                 dirichlet="outer", **kw):
        self.meshes = [MacroMesh(verts, l, dirichlet=dirichlet)
                       for l in range(coarse_level, fine_level + 1)]
        ks = [np.asarray(k_fine, dtype=np.float64)]
        for q in range(len(self.meshes) - 1, 0, -1):
            ks.append(inject(self.meshes[q - 1], self.meshes[q], ks[-1]))
        self.k = ks[::-1]
        self.A = [O.reduce_dirichlet(m, O.operator_matrix(m, kk, op, method=method, **kw)).tocsr()
                  for m, kk in zip(self.meshes, self.k)]
        self.P = [reduced_prolongation(self.meshes[q], self.meshes[q + 1])
                  for q in range(len(self.meshes) - 1)]
        self.Dinv = [block_jacobi_inverse(A) for A in self.A]
        self._coarse_lu = spla.splu(self.A[0].tocsc())


def vcycle(H: Hierarchy, b: np.ndarray, level: int | None = None, nu1=3, nu2=3,
           omega=0.7, nu_inc=0) -> np.ndarray:
    """One V(nu1, nu2) cycle for A_level e = b from e = 0.  With nu_inc > 0
    the variable V-cycle of Sec. 5.2.1: a level that lies j levels below the
    finest smooths nu1 + j nu_inc times before and nu2 + j nu_inc times
    after its coarse correction."""
    finest = len(H.A) - 1
    q = finest if level is None else level
    if q == 0:
        return H._coarse_lu.solve(b)
    A, Dinv, P = H.A[q], H.Dinv[q], H.P[q - 1]
    pre = nu1 + nu_inc * (finest - q)
    post = nu2 + nu_inc * (finest - q)
    x = np.zeros_like(b)
    for _ in range(pre):
        x = x + omega * (Dinv @ (b - A @ x))
    r = b - A @ x
    x = x + P @ vcycle(H, P.T @ r, q - 1, nu1, nu2, omega, nu_inc)
    for _ in range(post):
        x = x + omega * (Dinv @ (b - A @ x))
    return x


def mg_pcg(H: Hierarchy, b: np.ndarray, rtol=1e-8, maxiter=200, **cyc):
    """CG preconditioned by one V-cycle; stops at ||b - A x|| <= rtol ||b||.
    Returns (x, iterations)."""
    A = H.A[-1]
    x = np.zeros_like(b)
    r = b.copy()
    z = vcycle(H, r, **cyc)
    p = z.copy()
    rz = r @ z
    nb = np.linalg.norm(b)
    for it in range(1, maxiter + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= rtol * nb:
            return x, it
        z = vcycle(H, r, **cyc)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    raise RuntimeError("mg_pcg did not converge")
