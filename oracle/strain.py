"""Nodal strain rate and generalized-Newtonian viscosity (paper Sec. 3 and
Sec. 5.2.2).  Test infrastructure only.

Macro-interior node i: the velocity is projected locally onto affine
functions by least squares over the 15 nodes of the patch (eq.
minimization_problem with m = 1; on the symmetric interior patch this equals
the quadratic fit's gradient, Sec. 3), and |D(u)|^2 is evaluated from the
fitted gradient with D = eps: |eps|^2 = eps : eps.

Node on a macro boundary: the paper fits quadratics on the lower-dimensional
primitives without fixing the patch; this build uses the volume-weighted
average of the element gradients over all elements (of all macros) at the
node -- the local averaging the paper mentions as the alternative in Sec. 3.

Viscosity: Carreau law eq. carreau, mu = eta_inf + (eta0 - eta_inf)
(1 + kappa |eps|^2)^r.

Parity: pinned by tests (exact gradients for affine fields everywhere and for
quadratic fields at interior nodes, O(h^2) agreement with the analytic strain
of a smooth field, limits and monotonicity of the law).
"""
from __future__ import annotations

import numpy as np

from .forms import p1_gradients
from .mesh import MacroMesh


def carreau(eps2, eta0, eta_inf, kappa, r):
    """Eq. carreau: eta_inf + (eta0 - eta_inf) (1 + kappa |eps|^2)^r."""
    return eta_inf + (eta0 - eta_inf) * (1.0 + kappa * np.asarray(eps2)) ** r


def nodal_gradients(mesh: MacroMesh, u: np.ndarray) -> np.ndarray:
    """(n_nodes, 3, 3) array G[i, c, d] ~ d u_c / d x_d at every node."""
    u = np.asarray(u, dtype=np.float64).reshape(mesh.n_nodes, 3)
    G = np.full((mesh.n_nodes, 3, 3), np.nan)
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
    iface = mesh.interface
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


def nodal_viscosity(mesh: MacroMesh, u, eta0, eta_inf, kappa, r):
    return carreau(strain_rate_squared(nodal_gradients(mesh, u)), eta0, eta_inf, kappa, r)
