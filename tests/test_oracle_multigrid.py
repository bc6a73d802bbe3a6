"""Pins of the multigrid oracle (oracle/multigrid.py) against facts that do
not depend on it: P1 interpolation reproduces affine fields, the Galerkin
identity of nested P1 spaces with a constant coefficient, the injection of an
analytic coefficient, and the textbook behaviour of a V-cycle (symmetric,
contracting at a rate that does not grow with the level, and CG with it as
preconditioner reaching the sparse direct solution)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import multigrid as MG
from oracle import operators as O
from oracle.mesh import MacroMesh

MU, LAM = W.eform_weights()
EFORM = dict(mu1=MU, lam1=LAM)
LAME1 = dict(mu0=1.0, lam1=1.0)


def _distorted_tet():
    rng = np.random.default_rng(5)
    return W.unit_tet() + rng.normal(scale=0.08, size=(1, 4, 3))


@pytest.mark.parametrize("name", ["kuhn6", "cube24", "distorted"])
def test_prolongation_reproduces_affine_fields(name):
    V = {"kuhn6": W.kuhn6(), "cube24": W.cube24(), "distorted": _distorted_tet()}[name]
    for lev in (2, 3):
        c, f = MacroMesh(V, lev), MacroMesh(V, lev + 1)
        P = MG.prolongation(c, f)
        for A, c0 in (((0.3, -1.2, 2.0), 0.7), ((0.0, 0.0, 0.0), 1.0), ((1.5, 0.25, -0.5), -2.0)):
            u = lambda X: X @ np.array(A) + c0   # noqa: E731
            assert np.abs(P @ u(c.xyz) - u(f.xyz)).max() < 1e-12
        assert np.abs(P.sum(axis=1).A1 - 1.0).max() < 1e-15
        assert P.nnz <= 2 * f.n_nodes


@pytest.mark.parametrize("name,op", [("kuhn6", EFORM), ("kuhn6", LAME1), ("cube24", dict(mu1=1.0))])
def test_galerkin_identity_for_constant_coefficient(name, op):
    """Nested P1 spaces and exact element integrals: the level-l operator is
    P^T A_(l+1) P when the coefficient is constant."""
    V = {"kuhn6": W.kuhn6(), "cube24": W.cube24()}[name]
    c, f = MacroMesh(V, 2), MacroMesh(V, 3)
    Ac = O.reduce_dirichlet(c, O.operator_matrix(c, np.full(c.n_nodes, 2.5), op))
    Af = O.reduce_dirichlet(f, O.operator_matrix(f, np.full(f.n_nodes, 2.5), op))
    P = MG.reduced_prolongation(c, f)
    G = (P.T @ Af @ P).tocsr()
    assert abs(G - Ac).max() <= 1e-13 * abs(Ac).max()


def test_injection_of_an_analytic_coefficient():
    c, f = MacroMesh(W.kuhn6(), 2), MacroMesh(W.kuhn6(), 3)
    g = lambda X: np.exp(np.sin(3 * X[:, 0]) * X[:, 1] + X[:, 2])   # noqa: E731
    assert np.array_equal(MG.inject(c, f, g(f.xyz)), g(c.xyz))


@pytest.fixture(scope="module")
def hierarchies():
    out = {}
    for L in (3, 4):
        fm = MacroMesh(W.kuhn6(), L)
        k = W.exp_fourier_coefficient(fm.xyz, W.rng_for(2, 0), 16, 1.0)
        out[L] = MG.Hierarchy(W.kuhn6(), 2, L, k, EFORM)
    return out


def test_vcycle_is_symmetric(hierarchies):
    H = hierarchies[3]
    n = H.A[-1].shape[0]
    r1 = W.uniform_vector(n, W.rng_for(9, 1))
    r2 = W.uniform_vector(n, W.rng_for(9, 2))
    a = MG.vcycle(H, r1) @ r2
    b = r1 @ MG.vcycle(H, r2)
    assert abs(a - b) <= 1e-10 * abs(a)


def test_vcycle_contracts_independently_of_the_level(hierarchies):
    rates = {}
    for L, H in hierarchies.items():
        A = H.A[-1]
        b = W.uniform_vector(A.shape[0], W.rng_for(9, L))
        x = np.zeros_like(b)
        res = [np.linalg.norm(b)]
        for _ in range(8):
            x = x + MG.vcycle(H, b - A @ x)
            res.append(np.linalg.norm(b - A @ x))
        rates[L] = (res[-1] / res[2]) ** (1 / 6)
    assert rates[3] < 0.6 and rates[4] < 0.6, rates
    assert rates[4] < rates[3] + 0.15, rates


def test_variable_vcycle(hierarchies):
    """The variable V-cycle (Sec. 5.2.1: more smoothing on coarser levels)
    stays symmetric, adds smoothing only below the finest level (on a
    two-level hierarchy, whose coarse level is solved exactly, it is the
    fixed cycle), and contracts at least as fast as the fixed cycle with the
    same finest-level smoothing."""
    H = hierarchies[4]
    A = H.A[-1]
    n = A.shape[0]
    r1 = W.uniform_vector(n, W.rng_for(9, 3))
    r2 = W.uniform_vector(n, W.rng_for(9, 4))
    a = MG.vcycle(H, r1, nu_inc=2) @ r2
    b = r1 @ MG.vcycle(H, r2, nu_inc=2)
    assert abs(a - b) <= 1e-10 * abs(a)
    assert np.array_equal(MG.vcycle(H, r1, nu_inc=0), MG.vcycle(H, r1))
    assert np.abs(MG.vcycle(H, r1, nu_inc=2) - MG.vcycle(H, r1)).max() > 1e-8 * np.abs(MG.vcycle(H, r1)).max()
    two = MG.Hierarchy(W.kuhn6(), 3, 4, H.k[-1], EFORM)
    assert np.array_equal(MG.vcycle(two, r1, nu_inc=2), MG.vcycle(two, r1))
    rates = {}
    for inc in (0, 2):
        x = np.zeros(n)
        res = [np.linalg.norm(r1)]
        for _ in range(6):
            x = x + MG.vcycle(H, r1 - A @ x, nu_inc=inc)
            res.append(np.linalg.norm(r1 - A @ x))
        rates[inc] = (res[-1] / res[2]) ** 0.25
    assert rates[2] <= rates[0], rates


def test_mg_pcg_matches_direct_solve(hierarchies):
    for L, H in hierarchies.items():
        A = H.A[-1]
        b = W.uniform_vector(A.shape[0], W.rng_for(9, 10 + L))
        x, it = MG.mg_pcg(H, b, rtol=1e-10)
        xs = spla.spsolve(A.tocsc(), b)
        assert np.linalg.norm(x - xs) <= 1e-7 * np.linalg.norm(xs)
        assert it <= 25, it
