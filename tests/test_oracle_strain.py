"""Pins of the oracle's nodal strain rate and Carreau law (Sec. 3, eq. carreau)."""
import numpy as np
import pytest

import workloads as W
from oracle import strain as ST
from oracle.mesh import MacroMesh


@pytest.fixture(scope="module")
def mesh():
    return MacroMesh(W.cube24(), 2)


def test_affine_field_exact_everywhere(mesh):
    rng = np.random.default_rng(0)
    A = rng.normal(size=(3, 3))
    c = rng.normal(size=3)
    u = mesh.xyz @ A.T + c
    G = ST.nodal_gradients(mesh, u)
    np.testing.assert_allclose(G, np.broadcast_to(A, G.shape), atol=1e-12)


def test_quadratic_field_exact_in_macro_interiors():
    """Sec. 3: on the symmetric interior patch the affine fit has the gradient
    of the quadratic fit, i.e. the exact gradient of a quadratic field."""
    mesh = MacroMesh(W.unit_tet(), 3)
    x = mesh.xyz
    u = np.column_stack([x[:, 0] ** 2 + 3 * x[:, 1] * x[:, 2], x[:, 1] ** 2 - x[:, 0] * x[:, 2],
                         2 * x[:, 2] ** 2 + x[:, 0] * x[:, 1]])
    gx = np.zeros((mesh.n_nodes, 3, 3))
    gx[:, 0] = np.column_stack([2 * x[:, 0], 3 * x[:, 2], 3 * x[:, 1]])
    gx[:, 1] = np.column_stack([-x[:, 2], 2 * x[:, 1], -x[:, 0]])
    gx[:, 2] = np.column_stack([x[:, 1], x[:, 0], 4 * x[:, 2]])
    G = ST.nodal_gradients(mesh, u)
    inner = ~mesh.interface
    np.testing.assert_allclose(G[inner], gx[inner], atol=1e-12)
    # one macro: every boundary node is on the domain boundary, where the
    # one-sided patch only allows the affine fit
    assert np.abs(G[~inner] - gx[~inner]).max() > 1e-3


def test_smooth_field_converges():
    """Interior least-squares gradients of a smooth field converge at second
    order (the fit is exact for quadratics)."""
    def field(x):
        return np.column_stack([np.sin(x[:, 0] + 2 * x[:, 1]), np.cos(x[:, 2] - x[:, 0]),
                                np.sin(x[:, 1] * x[:, 2])])

    def grad(x):
        g = np.zeros((x.shape[0], 3, 3))
        c0 = np.cos(x[:, 0] + 2 * x[:, 1])
        s1 = np.sin(x[:, 2] - x[:, 0])
        c2 = np.cos(x[:, 1] * x[:, 2])
        g[:, 0, 0], g[:, 0, 1] = c0, 2 * c0
        g[:, 1, 0], g[:, 1, 2] = s1, -s1
        g[:, 2, 1], g[:, 2, 2] = x[:, 2] * c2, x[:, 1] * c2
        return g

    errs = []
    for L in (3, 4):
        mesh = MacroMesh(W.kuhn6(), L)
        G = ST.nodal_gradients(mesh, field(mesh.xyz))
        inner = ~mesh.interface
        errs.append(np.abs(G[inner] - grad(mesh.xyz)[inner]).max())
    assert errs[0] / errs[1] > 3.0


def test_carreau_law():
    eps2 = np.array([0.0, 1e-3, 1.0, 1e3, 1e12])
    mu = ST.carreau(eps2, 1.0, 1e-3, 1.0, -0.25)
    assert mu[0] == 1.0
    assert np.all(np.diff(mu) < 0)
    assert abs(mu[-1] - 1e-3) < 1e-3
    # shear thinning reduces to the Newtonian case for r = 0
    assert np.all(ST.carreau(eps2, 2.0, 1e-3, 5.0, 0.0) == 2.0)


def test_carreau_values_by_hand():
    """Eq. carreau at points where 1 + kappa |eps|^2 is a perfect power, so the
    value follows by hand: 16^(-1/4) = 1/2 and 81^(-1/4) = 1/3 with the
    library's default constants (eta0 1, eta_inf 1e-3, kappa 1, r -1/4); and the
    paper's dimensionless blood constants (Sec. 5.2.2: eta0 140.764, eta_inf
    1, kappa 212.2, r -0.325) at 1 + kappa |eps|^2 = 2^(40/13), where the
    power is 2^(-1) exactly."""
    law = dict(eta0=1.0, eta_inf=1e-3, kappa=1.0, r=-0.25)
    got = ST.carreau(np.array([0.0, 15.0, 80.0]), **law)
    assert got[0] == 1.0
    assert abs(got[1] - (1e-3 + 0.999 / 2)) <= 1e-15        # 0.5005
    assert abs(got[2] - (1e-3 + 0.999 / 3)) <= 1e-15        # 0.334
    paper = dict(eta0=140.764, eta_inf=1.0, kappa=212.2, r=-0.325)
    eps2 = (2.0 ** (40.0 / 13.0) - 1.0) / 212.2             # (1 + kappa eps2)^r = 2^(-1)
    assert abs(ST.carreau(eps2, **paper) - (1.0 + 139.764 / 2)) <= 1e-12   # 70.882
    assert ST.carreau(0.0, **paper) == 140.764


def test_strain_rate_scale_by_hand():
    """Simple shear u = (g y, 0, 0) has eps = g/2 (e_x e_y^T + e_y e_x^T), so
    eps : eps = g^2 / 2; uniaxial stretch u = (a x, 0, 0) has eps : eps = a^2."""
    g, a = 3.0, 5.0
    G = np.zeros((2, 3, 3))
    G[0, 0, 1] = g
    G[1, 0, 0] = a
    np.testing.assert_array_equal(ST.strain_rate_squared(G), [g * g / 2, a * a])


def test_viscosity_of_simple_shear_by_hand(mesh):
    """Affine simple shear with shear rate sqrt(30): eps : eps = 15 at every
    node (the fit is exact for affine fields), so the viscosity is 0.5005."""
    g = np.sqrt(30.0)
    u = np.column_stack([g * mesh.xyz[:, 1], np.zeros(mesh.n_nodes), np.zeros(mesh.n_nodes)])
    mu = ST.nodal_viscosity(mesh, u, 1.0, 1e-3, 1.0, -0.25)
    np.testing.assert_allclose(mu, 0.5005, rtol=0, atol=1e-13)


def test_seeded_velocity_gradient_converges():
    """The seeded velocity field of the Carreau workloads: interior
    least-squares gradients approach its analytic gradient at second order."""
    errs = []
    for L in (5, 6):                      # wave numbers up to 3: h = 1/32, 1/64 resolve them
        mesh = MacroMesh(W.unit_tet(), L)
        u = W.velocity_field(mesh.xyz, W.rng_for(3, 0), 0.1)
        gx = W.velocity_gradient(mesh.xyz, W.rng_for(3, 0), 0.1)
        G = ST.nodal_gradients(mesh, u)
        inner = ~mesh.interface
        errs.append(np.abs(G[inner] - gx[inner]).max() / np.abs(gx[inner]).max())
    assert errs[1] < 0.05 and errs[0] / errs[1] > 3.5, errs


def test_strain_rate_of_rotation_is_zero():
    G = np.zeros((4, 3, 3))
    G[:, 0, 1], G[:, 1, 0] = 1.0, -1.0
    assert np.all(ST.strain_rate_squared(G) == 0)


def _quadratic(x):
    u = np.column_stack([x[:, 0] ** 2 + 3 * x[:, 1] * x[:, 2], x[:, 1] ** 2 - x[:, 0] * x[:, 2],
                         2 * x[:, 2] ** 2 + x[:, 0] * x[:, 1]])
    g = np.zeros((x.shape[0], 3, 3))
    g[:, 0] = np.column_stack([2 * x[:, 0], 3 * x[:, 2], 3 * x[:, 1]])
    g[:, 1] = np.column_stack([-x[:, 2], 2 * x[:, 1], -x[:, 0]])
    g[:, 2] = np.column_stack([x[:, 1], x[:, 0], 4 * x[:, 2]])
    return u, g


@pytest.mark.parametrize("name,verts,L", [("kuhn6", W.kuhn6(), 3), ("cube24", W.cube24(), 2),
                                          ("cube24", W.cube24(), 3)])
def test_quadratic_fit_exact_on_macro_boundaries(name, verts, L):
    """Sec. 3: the quadratic fit on the lower-dimensional primitives gives the
    exact gradient of a quadratic field at every node off the domain
    boundary (faces, edges, vertices of macros; on the 24-macro mesh their
    patches are not point symmetric, and some edge patches determine only the
    gradient, not the whole quadratic); the domain boundary falls back to
    the affine fit; the element average is not exact there."""
    mesh = MacroMesh(verts, L)
    u, g = _quadratic(mesh.xyz - 0.3)
    G = ST.nodal_gradients(mesh, u)
    off = ~mesh.dirichlet
    np.testing.assert_allclose(G[off], g[off], atol=1e-12)
    deg = ST.boundary_fit_degrees(mesh)
    assert np.all(deg[mesh.interface & off] == 2)
    assert np.all(deg[mesh.dirichlet] == 1)
    if name == "cube24":
        Ga = ST.nodal_gradients(mesh, u, "average")
        assert np.abs(Ga[mesh.interface & off] - g[mesh.interface & off]).max() > 1e-3


def test_quadratic_and_affine_fits_agree_on_interior_patch():
    """Sec. 3: on the point-symmetric 15-node patch of a macro-interior node
    the quadratic and affine least-squares fits have the same gradient at the
    node, for any data."""
    mesh = MacroMesh(W.unit_tet(), 4)
    ptr, nbr = ST.patches(mesh)
    rng = np.random.default_rng(7)
    inner = np.nonzero(~mesh.interface)[0]
    for i in inner[::37]:
        pts = np.concatenate([[i], nbr[ptr[i]:ptr[i + 1]]])
        assert len(pts) == 15
        U = rng.normal(size=(15, 3))
        g2, ok2 = ST.fit_gradient(mesh.xyz[pts], U, 2)
        g1, ok1 = ST.fit_gradient(mesh.xyz[pts], U, 1)
        assert ok1 and ok2
        np.testing.assert_allclose(g2, g1, atol=1e-10 * np.abs(g1).max())


def test_quadratic_fit_converges_on_macro_boundaries():
    """Off the domain boundary the fitted gradient of a smooth field
    converges at second order on macro-boundary nodes too."""
    def field(x):
        return np.column_stack([np.sin(x[:, 0] + 2 * x[:, 1]), np.cos(x[:, 2] - x[:, 0]),
                                np.sin(x[:, 1] * x[:, 2])])

    def grad(x):
        g = np.zeros((x.shape[0], 3, 3))
        c0 = np.cos(x[:, 0] + 2 * x[:, 1])
        s1 = np.sin(x[:, 2] - x[:, 0])
        c2 = np.cos(x[:, 1] * x[:, 2])
        g[:, 0, 0], g[:, 0, 1] = c0, 2 * c0
        g[:, 1, 0], g[:, 1, 2] = s1, -s1
        g[:, 2, 1], g[:, 2, 2] = x[:, 2] * c2, x[:, 1] * c2
        return g

    errs = []
    for L in (3, 4):
        mesh = MacroMesh(W.cube24(), L)
        sel = mesh.interface & ~mesh.dirichlet
        G = ST.nodal_gradients(mesh, field(mesh.xyz))
        errs.append(np.abs(G[sel] - grad(mesh.xyz)[sel]).max())
    assert errs[0] / errs[1] > 3.3


def test_planted_fit_mistakes_are_caught(monkeypatch):
    """A dropped cross term or an unscaled gradient in the quadratic fit
    breaks the exactness pin on the macro boundaries."""
    mesh = MacroMesh(W.cube24(), 2)
    u, g = _quadratic(mesh.xyz)
    sel = mesh.interface & ~mesh.dirichlet
    orig = ST.fit_gradient

    def no_cross(X, U, degree):
        if degree != 2:
            return orig(X, U, degree)
        d = (X - X[0]) / np.abs(X - X[0]).max()
        A = np.column_stack([np.ones(len(X)), d, d ** 2, d[:, 0] * d[:, 1], d[:, 0] * d[:, 2]])
        coef = np.linalg.lstsq(A, U, rcond=None)[0]
        return coef[1:4].T / np.abs(X - X[0]).max(), True

    def unscaled(X, U, degree):
        G, ok = orig(X, U, degree)
        return (None if G is None else G * np.abs(X - X[0]).max()), ok

    for bad in (no_cross, unscaled):
        monkeypatch.setattr(ST, "fit_gradient", bad)
        G = ST.nodal_gradients(mesh, u)
        monkeypatch.undo()
        assert np.abs(G[sel] - g[sel]).max() > 1e-3
