"""Generalized Stokes system on the macro mesh (paper Sec. 5.2): the P1
divergence pair B, B^T, the pressure stabilization c_l and the saddle-point
operator.  TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline); no
code shared with the HIP library.

With velocity u = sum_j u_j phi_j (components l) and pressure
p = sum_q p_q psi_q, both equal-order P1 (Sec. 5.2, eqn. generalizedstokes
with the stress 2 mu eps(u) - p I):

* a(u, v)     = 2 (mu eps(u), eps(v))                    (the velocity block A)
* b(v, p)     = -(div v, p)                              B[q, (j, l)] = -int d_l phi_j psi_q
* c_l(p, q)   = -h_l^2 / 12 (grad p, grad q)             (stabilization, Sec. 5.2)

and the discrete system [[A, B^T], [B, C]] [u; p] = [f; 0].  On an element
t all P1 gradients are constant and int_t psi_q = |t| / 4, so every entry is
a sum of element contributions written out below.  Rows of Dirichlet velocity
nodes are removed (principal submatrix), the pressure lives on every node.

Parity: pinned by tests (hand-computed element matrices of the unit
tetrahedron, B of a constant or rigid rotation field vanishes, B of u = x
sums to -3 |Omega|, B^T of a constant pressure vanishes at interior velocity
nodes, C is symmetric, negative semidefinite with zero row sums and maps
affine pressures to zero at interior nodes, and the exact Stokes solution
of a manufactured divergence-free flow is approached at the expected rate).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import operators as O
from .forms import p1_gradients
from .mesh import MacroMesh
from .multigrid import vcycle


def _elements(mesh: MacroMesh):
    """All elements of the mesh as (global node ids (T,4), gradients (T,4,3),
    volumes (T,))."""
    G, Gr, V = [], [], []
    for m in range(mesh.n_macro):
        tets = mesh.local_tets[m]
        g, vol = p1_gradients(mesh.local_xyz[m][tets])
        G.append(mesh.gid[m][tets])
        Gr.append(g)
        V.append(vol)
    return np.concatenate(G), np.concatenate(Gr), np.concatenate(V)


def divergence_matrix(mesh: MacroMesh) -> sp.csr_matrix:
    """B (n_nodes x 3 n_nodes): B[q, 3 j + l] = -sum_t |t| / 4 (grad phi_j)_l
    over the elements t holding both q and j."""
    gid, g, vol = _elements(mesh)
    rows, cols, vals = [], [], []
    for a in range(4):            # test node q = vertex a
        for b in range(4):        # trial node j = vertex b
            for l in range(3):
                rows.append(gid[:, a])
                cols.append(3 * gid[:, b] + l)
                vals.append(-0.25 * vol * g[:, b, l])
    n = mesh.n_nodes
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, 3 * n))


def stabilization_matrix(mesh: MacroMesh, h: float) -> sp.csr_matrix:
    """C (n_nodes x n_nodes) of c_l(p, q) = -h^2/12 (grad p, grad q):
    C[q, r] = -h^2/12 sum_t |t| grad psi_q . grad psi_r."""
    gid, g, vol = _elements(mesh)
    rows, cols, vals = [], [], []
    for a in range(4):
        for b in range(4):
            rows.append(gid[:, a])
            cols.append(gid[:, b])
            vals.append(-(h * h / 12.0) * vol * np.einsum("tc,tc->t", g[:, a], g[:, b]))
    n = mesh.n_nodes
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def mesh_width(level: int) -> float:
    """h_l of the unit-cube meshes: the cube edge (one macro edge of the
    6-macro cube) over 2^level intervals."""
    return 1.0 / (1 << int(level))


def saddle_matrix(mesh: MacroMesh, A: sp.spmatrix, h: float):
    """K = [[A_uu, B_u^T], [B_u, C]] on the unknown velocity DoFs (Dirichlet
    nodes removed) and all pressure nodes, with the velocity operator A
    (3 n x 3 n, e.g. the oracle's scaled or nodal matrix of 2 mu (eps, eps),
    or already reduced to the unknown DoFs).  Returns (K, velocity dofs)."""
    u = mesh.unknown
    dof = (3 * u[:, None] + np.arange(3)[None]).ravel()
    B = divergence_matrix(mesh)[:, dof]
    C = stabilization_matrix(mesh, h)
    Auu = A.tocsr() if A.shape[0] == dof.size else A.tocsr()[dof][:, dof]
    K = sp.bmat([[Auu, B.T], [B, C]], format="csr")
    return K, dof


def solve_saddle(K: sp.spmatrix, rhs: np.ndarray, n_u: int, mass: np.ndarray | None = None):
    """Direct solve of K z = rhs with the pressure fixed by a zero mean: the
    constant pressure spans the kernel when every boundary node is
    Dirichlet, so the system is bordered by the constraint
    sum_q mass_q p_q = 0 (mass: lumped pressure mass, ones if None)."""
    n = K.shape[0]
    n_p = n - n_u
    w = np.ones(n_p) if mass is None else np.asarray(mass, dtype=np.float64)
    e = np.zeros(n)
    e[n_u:] = w
    Kb = sp.bmat([[K, sp.csr_matrix(e[:, None])], [sp.csr_matrix(e[None, :]), None]], format="csc")
    z = sp.linalg.spsolve(Kb, np.concatenate([rhs, [0.0]]))
    return z[:n]


def lumped_mass(mesh: MacroMesh) -> np.ndarray:
    """int psi_q over the domain: sum_t |t| / 4."""
    gid, _, vol = _elements(mesh)
    out = np.zeros(mesh.n_nodes)
    for a in range(4):
        np.add.at(out, gid[:, a], 0.25 * vol)
    return out


def schur_diag(mesh: MacroMesh, mu: np.ndarray, h: float) -> np.ndarray:
    """Diagonal approximation of the pressure Schur complement
    B A^-1 B^T - C: the lumped pressure mass weighted by 1/mu at the node
    (B A^-1 B^T of the viscous operator is spectrally close to the
    1/mu-weighted mass) plus the diagonal of -C."""
    C = stabilization_matrix(mesh, h)
    return lumped_mass(mesh) / np.asarray(mu, dtype=np.float64) - C.diagonal()


def inexact_uzawa(H, mesh: MacroMesh, mu, f, g=None, h=None, u0=None, p0=None, omega_p=1.0,
                  rtol=1e-8, maxit=500, cycles=1, nu1=3, nu2=3, omega=0.7, nu_inc=0):
    """Inexact Uzawa iteration for [[A, B^T], [B, C]] [u; p] = [f; g] on the
    finest level of the velocity hierarchy H (operator A = H.A[-1] on the
    unknown velocity DoFs, pressure on every node):

        u <- u + V(f - A u - B^T p)        (``cycles`` V(nu1, nu2) cycles of H)
        p <- p + omega_p S^-1 (B u + C p - g),  S = diag(mass / mu - C)
        p <- p - (mass . p) / (mass . 1)   (zero mean; the constant pressure
                                            is in the kernel)

    Stops when the residual norm of both blocks is <= rtol times that of the
    right-hand side.  Returns (u, p, iterations, residual history)."""
    A = H.A[-1]
    dof = O.unknown_dofs(mesh)
    B = divergence_matrix(mesh)[:, dof].tocsr()
    h = mesh_width(int(mesh.levels[0])) if h is None else h
    C = stabilization_matrix(mesh, h)
    m = lumped_mass(mesh)
    S = schur_diag(mesh, mu, h)
    g = np.zeros(mesh.n_nodes) if g is None else g
    u = np.zeros(dof.size) if u0 is None else np.array(u0, dtype=np.float64)
    p = np.zeros(mesh.n_nodes) if p0 is None else np.array(p0, dtype=np.float64)
    nrm = np.sqrt(f @ f + g @ g)
    hist = []
    for it in range(1, maxit + 1):
        for _ in range(cycles):
            u = u + vcycle(H, f - A @ u - B.T @ p, nu1=nu1, nu2=nu2, omega=omega, nu_inc=nu_inc)
        p = p + omega_p * (B @ u + C @ p - g) / S
        p = p - (m @ p) / m.sum()
        ru = f - A @ u - B.T @ p
        rp = g - B @ u - C @ p
        hist.append(np.sqrt(ru @ ru + rp @ rp) / nrm)
        if hist[-1] <= rtol:
            return u, p, it, hist
    return u, p, maxit, hist


def picard(verts, coarse_level: int, level: int, f: np.ndarray, law: dict, method="scaled",
           max_picard=100, rtol=1e-3, maxit=500, **uz):
    """Fixed-point iteration of Sec. 5.2.2 (eq. fixpointsystem, Alg.
    fixedpoint_mg) for the Carreau fluid with the operator 2 (mu eps, eps):
    u = 0, p = 0, mu = mu(u); repeat one inexact Uzawa step with A(mu), then
    mu = mu(u), until max_i |u_i - u_i^prev| < 1e-3 max_i |u_i| (node-wise
    2-norms over unknown nodes); then Uzawa steps to relative residual rtol
    and a last mu = mu(u).  f: (n_nodes, 3) right-hand side vector.  Returns
    (u (n_nodes, 3), p, mu, picard steps, final steps, rel. change)."""
    from . import strain as SR
    from .multigrid import Hierarchy
    mesh = MacroMesh(verts, level)
    dof = O.unknown_dofs(mesh)
    fu = np.asarray(f, dtype=np.float64).ravel()[dof]
    u = np.zeros((mesh.n_nodes, 3))
    p = np.zeros(mesh.n_nodes)
    unk = mesh.unknown
    mu = SR.nodal_viscosity(mesh, u, **law)
    H = Hierarchy(verts, coarse_level, level, mu, dict(mu1=1.0), method=method)
    change = np.inf
    steps = 0
    for steps in range(1, max_picard + 1):
        uprev = u.copy()
        ud, p, _, _ = inexact_uzawa(H, mesh, mu, fu, u0=u.ravel()[dof], p0=p, maxit=1, rtol=0.0, **uz)
        u = np.zeros(3 * mesh.n_nodes)
        u[dof] = ud
        u = u.reshape(-1, 3)
        mu = SR.nodal_viscosity(mesh, u, **law)
        H = Hierarchy(verts, coarse_level, level, mu, dict(mu1=1.0), method=method)
        change = (np.linalg.norm(u[unk] - uprev[unk], axis=1).max() /
                  np.linalg.norm(u[unk], axis=1).max())
        if change < 1e-3:
            break
    ud, p, final, hist = inexact_uzawa(H, mesh, mu, fu, u0=u.ravel()[dof], p0=p, rtol=rtol,
                                       maxit=maxit, **uz)
    u = np.zeros(3 * mesh.n_nodes)
    u[dof] = ud
    u = u.reshape(-1, 3)
    mu = SR.nodal_viscosity(mesh, u, **law)
    return u, p, mu, steps, final, change
