"""Pins of the Stokes oracle (Sec. 5.2): the divergence pair and the
pressure stabilization against hand-computed element matrices of the unit
tetrahedron, their kernels and identities, and convergence of the
stabilized equal-order discretization to a manufactured Stokes flow."""
import numpy as np
import pytest

import workloads as W
from oracle import operators as O
from oracle import stokes as ST
from oracle.mesh import MacroMesh


def _unit_tet_nodes(mesh):
    """Global node ids of the unit tet's vertices 0, e_x, e_y, e_z."""
    want = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)
    return np.array([int(np.argmin(np.linalg.norm(mesh.xyz - w, axis=1))) for w in want])


def test_unit_tet_by_hand():
    """One element, vol 1/6, gradients of 1 - x - y - z, x, y, z:
    (-1,-1,-1), e_x, e_y, e_z.  B[q, (j, l)] = -(1/6)(1/4) (grad phi_j)_l for
    every q; C[q, r] = -(h^2/12)(1/6) grad phi_q . grad phi_r with
    grad phi_0 . grad phi_0 = 3, grad phi_0 . grad phi_a = -1,
    grad phi_a . grad phi_b = delta_ab."""
    mesh = MacroMesh(W.unit_tet(), 0)
    v = _unit_tet_nodes(mesh)
    B = ST.divergence_matrix(mesh).toarray()
    grads = np.array([[-1.0, -1.0, -1.0], [1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
    for q in range(4):
        for j in range(4):
            for l in range(3):
                assert abs(B[v[q], 3 * v[j] + l] - (-grads[j, l] / 24.0)) <= 1e-15
    h = 0.5
    C = ST.stabilization_matrix(mesh, h).toarray()
    dots = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]], dtype=float)
    np.testing.assert_allclose(C[np.ix_(v, v)], -(h * h / 12.0) / 6.0 * dots, rtol=0, atol=1e-16)
    np.testing.assert_allclose(ST.lumped_mass(mesh)[v], 1.0 / 24.0, rtol=0, atol=1e-17)


@pytest.fixture(scope="module")
def cube():
    return MacroMesh(W.kuhn6(), 3)


def test_divergence_kernel_and_value(cube):
    """B u = 0 for translations and rotations (div = 0 everywhere); for
    u = x the divergence is 3, so B u = -3 int psi_q, summing to -3 |Omega|."""
    B = ST.divergence_matrix(cube)
    x = cube.xyz
    for u in (np.tile([1.0, -2.0, 0.5], (cube.n_nodes, 1)),
              np.cross(np.array([0.3, -1.0, 2.0]), x)):
        assert np.abs(B @ u.ravel()).max() <= 1e-14
    Bu = B @ x.ravel()
    np.testing.assert_allclose(Bu, -3.0 * ST.lumped_mass(cube), rtol=1e-12)
    assert abs(Bu.sum() + 3.0) <= 1e-12


def test_gradient_of_constant_pressure(cube):
    """(B^T 1)_(j,l) = -int d_l phi_j = -int_boundary phi_j n_l: zero at every
    node off the boundary, and B^T of an affine p is -grad p times the mass."""
    B = ST.divergence_matrix(cube)
    g = (B.T @ np.ones(cube.n_nodes)).reshape(-1, 3)
    inner = ~np.isclose(cube.xyz, 0).any(1) & ~np.isclose(cube.xyz, 1).any(1)
    assert np.abs(g[inner]).max() <= 1e-14 and np.abs(g[~inner]).max() > 1e-3
    p = cube.xyz @ np.array([1.0, 2.0, -3.0])
    gp = (B.T @ p).reshape(-1, 3)
    # -(div v, p) = (v, grad p) - boundary term: at interior nodes
    # -int p d_l phi_j = int d_l p phi_j = (grad p)_l int phi_j
    np.testing.assert_allclose(gp[inner], np.outer(ST.lumped_mass(cube)[inner], [1.0, 2.0, -3.0]),
                               rtol=1e-12)


def test_stabilization_properties(cube):
    h = ST.mesh_width(3)
    C = ST.stabilization_matrix(cube, h)
    assert abs(C - C.T).max() <= 1e-18
    assert np.abs(C @ np.ones(cube.n_nodes)).max() <= 1e-17
    ev = np.linalg.eigvalsh(C.toarray())
    assert ev.max() <= 1e-15 and ev.min() < 0
    inner = ~np.isclose(cube.xyz, 0).any(1) & ~np.isclose(cube.xyz, 1).any(1)
    p = cube.xyz @ np.array([0.7, -1.1, 0.4]) + 2.0
    assert np.abs((C @ p)[inner]).max() <= 1e-17
    # scaling in h: C(2h) = 4 C(h)
    assert abs(ST.stabilization_matrix(cube, 2 * h) - 4 * C).max() <= 1e-16


def _manufactured(x):
    """Divergence-free velocity u = curl(psi e_z) with
    psi = sin(pi x)^2 sin(pi y)^2 (zero on x, y in {0, 1}), times
    sin(pi z) (zero at z in {0, 1}) for the z-direction; pressure
    p = cos(pi x) cos(pi y) cos(pi z); mu = 1.  Returns u, p and
    f = -div(2 eps(u)) + grad p = -Delta u + grad p."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    s, c, pi = np.sin, np.cos, np.pi
    u = np.column_stack([
        2 * pi * s(pi * X) ** 2 * s(pi * Y) * c(pi * Y) * s(pi * Z),
        -2 * pi * s(pi * X) * c(pi * X) * s(pi * Y) ** 2 * s(pi * Z),
        np.zeros_like(X)])
    p = c(pi * X) * c(pi * Y) * c(pi * Z)
    return u, p


def _force(x, hstep=1e-4):
    """f = -Delta u + grad p by central differences of the closed forms."""
    f = np.zeros_like(x)
    u0, _ = _manufactured(x)
    for d in range(3):
        e = np.zeros(3)
        e[d] = hstep
        up, pp = _manufactured(x + e)
        um, pm = _manufactured(x - e)
        f -= (up - 2 * u0 + um) / hstep ** 2
        f[:, d] += (pp - pm) / (2 * hstep)
    return f


def test_manufactured_flow_converges():
    """Stabilized P1-P1 Stokes with mu = 1 on the 6-macro cube (the operator
    2 (eps, eps) through the oracle's scaled matrix with k = 1): the velocity
    error at the nodes falls by about 4 per refinement."""
    errs = []
    for L in (2, 3):
        mesh = MacroMesh(W.kuhn6(), L)
        A = O.operator_matrix(mesh, np.ones(mesh.n_nodes), dict(mu1=1.0))
        K, dof = ST.saddle_matrix(mesh, A, ST.mesh_width(L))
        # consistent P1 load of the interpolated force, lumped
        m = ST.lumped_mass(mesh)
        f = (_force(mesh.xyz) * m[:, None]).ravel()[dof]
        rhs = np.concatenate([f, np.zeros(mesh.n_nodes)])
        z = ST.solve_saddle(K, rhs, dof.size, m)
        u_ex, _ = _manufactured(mesh.xyz)
        err = np.abs(z[:dof.size] - u_ex.ravel()[dof]).max()
        errs.append(err)
    assert errs[1] < errs[0] / 2.5, errs


def _shear_force(mesh, amp=100.0):
    """Body force (amp sin(pi y), 0, amp sin(pi x)) times the lumped mass:
    not a gradient, so it drives a flow."""
    x = mesh.xyz
    f = np.column_stack([amp * np.sin(np.pi * x[:, 1]), np.zeros(mesh.n_nodes),
                         amp * np.sin(np.pi * x[:, 0])])
    f = f * ST.lumped_mass(mesh)[:, None]
    f[mesh.dirichlet] = 0.0
    return f


def test_inexact_uzawa_reaches_direct_solution():
    """The Uzawa iteration converges to the bordered direct solve of the
    same saddle-point system (constant viscosity 2 on the 6-macro cube)."""
    from oracle import multigrid as MG
    L = 3
    mesh = MacroMesh(W.kuhn6(), L)
    mu = 2.0 * np.ones(mesh.n_nodes)
    H = MG.Hierarchy(W.kuhn6(), 2, L, mu, dict(mu1=1.0))
    dof = O.unknown_dofs(mesh)
    f = _shear_force(mesh).ravel()[dof]
    u, p, it, hist = ST.inexact_uzawa(H, mesh, mu, f, rtol=1e-10, maxit=400)
    assert hist[-1] <= 1e-10 and it < 400
    K, _ = ST.saddle_matrix(mesh, H.A[-1], ST.mesh_width(L))
    z = ST.solve_saddle(K, np.concatenate([f, np.zeros(mesh.n_nodes)]), dof.size,
                        ST.lumped_mass(mesh))
    assert np.abs(u - z[:dof.size]).max() <= 1e-8 * np.abs(z[:dof.size]).max()
    assert np.abs(p - z[dof.size:]).max() <= 1e-7 * np.abs(z[dof.size:]).max()


def test_picard_newtonian_is_one_linear_solve():
    """With r = 0 the Carreau law is the constant eta0: the fixed point is
    reached after the first change test that sees no change, and the result
    is the linear Stokes solution with viscosity eta0."""
    L = 3
    mesh = MacroMesh(W.kuhn6(), L)
    f = _shear_force(mesh)
    law = dict(eta0=3.0, eta_inf=1.0, kappa=5.0, r=0.0)
    u, p, mu, steps, final, change = ST.picard(W.kuhn6(), 2, L, f, law, rtol=1e-10, maxit=600)
    assert np.all(mu == 3.0)
    from oracle import multigrid as MG
    H = MG.Hierarchy(W.kuhn6(), 2, L, mu, dict(mu1=1.0))
    dof = O.unknown_dofs(mesh)
    K, _ = ST.saddle_matrix(mesh, H.A[-1], ST.mesh_width(L))
    z = ST.solve_saddle(K, np.concatenate([f.ravel()[dof], np.zeros(mesh.n_nodes)]), dof.size,
                        ST.lumped_mass(mesh))
    assert np.abs(u.ravel()[dof] - z[:dof.size]).max() <= 1e-7 * np.abs(z[:dof.size]).max()


def test_picard_carreau_fixed_point():
    """Shear-thinning Carreau fluid: the returned velocity solves the
    Stokes system with the viscosity of the previous fixed-point step to the
    final tolerance, and that viscosity reproduces itself within the
    fixed-point tolerance (mu(u) changes by well under a percent)."""
    from oracle import strain as SR
    L = 3
    mesh = MacroMesh(W.kuhn6(), L)
    f = _shear_force(mesh)
    law = dict(eta0=1.0, eta_inf=1e-3, kappa=1.0, r=-0.25)
    u, p, mu, steps, final, change = ST.picard(W.kuhn6(), 2, L, f, law, rtol=1e-8, maxit=800)
    assert change < 1e-3 and steps < 60
    assert mu.min() < 0.9 * mu.max()                 # shear thinning visible
    mu2 = SR.nodal_viscosity(mesh, u, **law)
    np.testing.assert_allclose(mu2, mu, rtol=1e-12)
