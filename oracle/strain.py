"""Nodal strain rate and generalized-Newtonian viscosity (paper Sec. 3 and
Sec. 5.2.2).  Test infrastructure only.

Macro-interior node i: the velocity is projected locally onto affine
functions by least squares over the 15 nodes of the patch (eq.
minimization_problem with m = 1; on the symmetric interior patch this equals
the quadratic fit's gradient, Sec. 3), and |D(u)|^2 is evaluated from the
fitted gradient with D = eps: |eps|^2 = eps : eps.

Node on a macro boundary (face, edge or vertex of a macro), ``boundary=
"quadratic"`` (default): least squares over the node's patch in the whole
mesh (the node and every node that shares an element with it, in any
macro) onto quadratic polynomials (eq. minimization_problem with m = 2, as
Sec. 3 asks on the lower-dimensional primitives), the gradient taken at the
node.  Where the patch has too few points for a unique quadratic but every
least-squares quadratic has the same gradient at the node (the quadratics
vanishing on the patch have zero gradient there, e.g. on a macro edge
whose patch lies in two planes through the edge), that gradient is used.
Where the gradient is not determined either (on the domain boundary the
patch has a single layer of nodes on one side, which cannot tell the
normal slope from the normal curvature) the affine fit (m = 1) over the
same patch is used.  ``boundary="average"``: the volume-weighted
average of the element gradients over all elements at the node, the local
averaging the paper names as the alternative in Sec. 3.

Viscosity: Carreau law eq. carreau, mu = eta_inf + (eta0 - eta_inf)
(1 + kappa |eps|^2)^r.

Parity: pinned by tests (exact gradients for affine fields everywhere and for
quadratic fields at every node whose patch determines a quadratic, the
quadratic and affine fits agreeing on the symmetric macro-interior patch as
Sec. 3 argues, O(h^2) agreement with the analytic strain of a smooth field,
values and limits of the law).
"""
from __future__ import annotations

import numpy as np

from .forms import p1_gradients
from .mesh import MacroMesh


def carreau(eps2, eta0, eta_inf, kappa, r):
    """Eq. carreau: eta_inf + (eta0 - eta_inf) (1 + kappa |eps|^2)^r."""
    return eta_inf + (eta0 - eta_inf) * (1.0 + kappa * np.asarray(eps2)) ** r


# relative size below which a singular value of the scaled quadratic design
# matrix counts as zero (the rank-deficient patches are exactly deficient)
RANK_TOL = 1e-6


def patches(mesh: MacroMesh):
    """Neighbours of every node in the whole mesh: (ptr, nbr) in CSR form,
    nbr[ptr[i]:ptr[i+1]] the sorted global ids sharing an element with i."""
    pairs = []
    for m in range(mesh.n_macro):
        t = mesh.gid[m][mesh.local_tets[m]]
        pairs += [t[:, [a, b]] for a in range(4) for b in range(4) if a != b]
    pairs = np.unique(np.concatenate(pairs), axis=0)
    ptr = np.searchsorted(pairs[:, 0], np.arange(mesh.n_nodes + 1))
    return ptr, pairs[:, 1]


def fit_gradient(X: np.ndarray, U: np.ndarray, degree: int):
    """Least-squares fit of the columns of U (P, 3) at the points X (P, 3),
    centred at X[0], onto polynomials of the given degree (1 or 2).  Returns
    (gradient at X[0] as (3, 3) [component, direction], determined?): the
    gradient is determined when every least-squares polynomial has the same
    gradient at X[0], i.e. the polynomials vanishing at all the points
    (the null space of the design matrix) have zero gradient there; it is
    then that of the minimum-norm solution."""
    d = X - X[0]
    h = np.abs(d).max()
    d = d / h
    cols = [np.ones(len(X)), d[:, 0], d[:, 1], d[:, 2]]
    if degree == 2:
        cols += [d[:, 0] ** 2, d[:, 1] ** 2, d[:, 2] ** 2,
                 d[:, 0] * d[:, 1], d[:, 0] * d[:, 2], d[:, 1] * d[:, 2]]
    A = np.column_stack(cols)
    _, sv, Vt = np.linalg.svd(A, full_matrices=True)
    rank = int(np.sum(sv > RANK_TOL * sv[0]))
    null = Vt[rank:]
    if null.size and np.abs(null[:, 1:4]).max() > RANK_TOL:
        return None, False
    coef = np.linalg.pinv(A, rcond=RANK_TOL) @ U
    return coef[1:4].T / h, True


def boundary_fit_degrees(mesh: MacroMesh) -> np.ndarray:
    """Degree of the fit (2, or 1 where the patch does not determine a
    quadratic) at every node on a macro boundary; 0 elsewhere."""
    ptr, nbr = patches(mesh)
    deg = np.zeros(mesh.n_nodes, dtype=np.int64)
    for i in np.nonzero(mesh.interface)[0]:
        pts = np.concatenate([[i], nbr[ptr[i]:ptr[i + 1]]])
        _, ok = fit_gradient(mesh.xyz[pts], np.zeros((len(pts), 3)), 2)
        deg[i] = 2 if ok else 1
    return deg


def nodal_gradients(mesh: MacroMesh, u: np.ndarray, boundary: str = "quadratic") -> np.ndarray:
    """(n_nodes, 3, 3) array G[i, c, d] ~ d u_c / d x_d at every node."""
    if boundary not in ("quadratic", "average"):
        raise ValueError(boundary)
    u = np.asarray(u, dtype=np.float64).reshape(mesh.n_nodes, 3)
    G = np.full((mesh.n_nodes, 3, 3), np.nan)
    iface = mesh.interface
    if boundary == "quadratic":
        ptr, nbr = patches(mesh)
        for i in np.nonzero(iface)[0]:
            pts = np.concatenate([[i], nbr[ptr[i]:ptr[i + 1]]])
            g, ok = fit_gradient(mesh.xyz[pts], u[pts], 2)
            if not ok:
                g, ok = fit_gradient(mesh.xyz[pts], u[pts], 1)
                assert ok, "patch does not determine an affine function"
            G[i] = g
    else:
        # element gradients and volumes, accumulated for macro-boundary nodes
        SG = np.zeros((mesh.n_nodes, 3, 3))
        SV = np.zeros(mesh.n_nodes)
        for m in range(mesh.n_macro):
            tets = mesh.local_tets[m]
            gid = mesh.gid[m]
            g, vol = p1_gradients(mesh.local_xyz[m][tets])
            ut = u[gid[tets]]                                   # (T, 4, 3)
            Gt = np.einsum("tac,tad->tcd", ut, g)               # element gradient
            for a in range(4):
                np.add.at(SG, gid[tets[:, a]], vol[:, None, None] * Gt)
                np.add.at(SV, gid[tets[:, a]], vol)
        G[iface] = SG[iface] / SV[iface, None, None]
    # affine least squares on the 15-node patch of macro-interior nodes
    for m in range(mesh.n_macro):
        tets = mesh.local_tets[m]
        gid = mesh.gid[m]
        inner = np.nonzero(~mesh.on_macro_boundary[m])[0]
        if inner.size == 0:
            continue
        # neighbours via elements
        pairs = np.concatenate([tets[:, [a, b]] for a in range(4) for b in range(4) if a != b])
        pairs = np.unique(pairs, axis=0)
        keep = np.isin(pairs[:, 0], inner)
        pairs = pairs[keep]
        order = np.argsort(pairs[:, 0], kind="stable")
        pairs = pairs[order]
        starts = np.searchsorted(pairs[:, 0], inner)
        xyz = mesh.local_xyz[m]
        for idx, i in enumerate(inner):
            nbr = pairs[starts[idx]:starts[idx] + 14, 1]
            assert nbr.shape[0] == 14 and np.all(pairs[starts[idx]:starts[idx] + 14, 0] == i)
            pts = np.concatenate([[i], nbr])
            Amat = np.column_stack([np.ones(15), xyz[pts] - xyz[i]])
            coef, *_ = np.linalg.lstsq(Amat, u[gid[pts]], rcond=None)   # (4, 3)
            G[gid[i]] = coef[1:].T
    return G


def strain_rate_squared(G: np.ndarray) -> np.ndarray:
    """|eps(u)|^2 = eps : eps with eps = (G + G^T)/2."""
    E = 0.5 * (G + np.swapaxes(G, -1, -2))
    return np.einsum("ncd,ncd->n", E, E)


def nodal_viscosity(mesh: MacroMesh, u, eta0, eta_inf, kappa, r, boundary="quadratic"):
    return carreau(strain_rate_squared(nodal_gradients(mesh, u, boundary)), eta0, eta_inf, kappa, r)
