"""Reference solves of A x = b on the unknowns (test infrastructure).

The systems are those of the operators in ``operators`` after homogeneous
Dirichlet reduction (Sec. 2).  ``direct_solve`` is the plain definition
x = A^{-1} b by sparse LU; ``block_jacobi_cg`` is textbook preconditioned CG
with the inverse 3x3 diagonal blocks, used as the CPU timing baseline of the
solvers.

Parity: pinned by tests (manufactured solutions x* with b = A x* are
recovered; CG and LU agree; the block-Jacobi preconditioner is SPD).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import operators as O
from .mesh import MacroMesh


def reduced_system(mesh: MacroMesh, k, op, method="scaled", **kw):
    """(A_uu, dof index) of the Dirichlet-reduced operator."""
    A = O.operator_matrix(mesh, k, op, method=method, **kw)
    dof = O.unknown_dofs(mesh)
    return A.tocsr()[dof][:, dof].tocsc(), dof


def direct_solve(A: sp.spmatrix, b: np.ndarray) -> np.ndarray:
    return spla.spsolve(A.tocsc(), b)


def block_jacobi_inverse(A: sp.spmatrix) -> sp.csr_matrix:
    """Inverse of the 3x3 diagonal blocks (nodes are consecutive dof triples)."""
    A = A.tocsr()
    n = A.shape[0] // 3
    blocks = np.zeros((n, 3, 3))
    for a in range(3):
        for c in range(3):
            blocks[:, a, c] = A[np.arange(n) * 3 + a, np.arange(n) * 3 + c].A1
    inv = np.linalg.inv(blocks)
    rows = (np.arange(n)[:, None, None] * 3 + np.arange(3)[None, :, None]).repeat(3, axis=2)
    cols = (np.arange(n)[:, None, None] * 3 + np.arange(3)[None, None, :]).repeat(3, axis=1)
    return sp.csr_matrix((inv.ravel(), (rows.ravel(), cols.ravel())), shape=A.shape)


def block_jacobi_cg(A, b, rtol=1e-8, maxiter=100000):
    """Preconditioned CG to ||b - A x|| <= rtol ||b||; returns (x, iterations)."""
    M = block_jacobi_inverse(A)
    it = [0]

    def cb(_):
        it[0] += 1

    x, info = spla.cg(A, b, rtol=rtol, atol=0.0, maxiter=maxiter, M=M, callback=cb)
    if info != 0:
        raise RuntimeError(f"cg did not converge ({info})")
    return x, it[0]
