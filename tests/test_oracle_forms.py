"""Pins of the oracle's local stiffness tensors (Sec. 2 and Sec. 2.4)."""
import numpy as np
import pytest

from oracle.forms import form_tensor, p1_gradients, antisym_part, sym_part


@pytest.fixture(scope="module")
def elements():
    rng = np.random.default_rng(11)
    X = rng.normal(size=(64, 4, 3))
    # drop nearly degenerate draws
    _, vol = p1_gradients(X)
    return X[vol > 1e-2]


def _as_matrix(a):
    """[t, i, j, l, m] -> (T, 12, 12) with row 3i+m, column 3j+l."""
    T = a.shape[0]
    return np.transpose(a, (0, 1, 4, 2, 3)).reshape(T, 12, 12)


@pytest.mark.parametrize("mu,lam", [(1.0, 0.0), (0.0, 1.0), (0.37, 0.79)])
def test_block_row_sums_vanish(elements, mu, lam):
    a = form_tensor(elements, mu, lam)
    assert np.abs(a.sum(axis=2)).max() < 1e-12 * np.abs(a).max()


@pytest.mark.parametrize("mu,lam", [(1.0, 0.0), (0.0, 1.0), (0.37, 0.79)])
def test_symmetric_form(elements, mu, lam):
    A = _as_matrix(form_tensor(elements, mu, lam))
    assert np.abs(A - np.transpose(A, (0, 2, 1))).max() < 1e-12 * np.abs(A).max()


def test_rigid_body_modes_in_kernel(elements):
    """eps(w x x) = 0 and div(w x x) = 0 for every rotation vector w."""
    A = _as_matrix(form_tensor(elements, 0.6, 1.3))
    rng = np.random.default_rng(5)
    for _ in range(4):
        w = rng.normal(size=3)
        c = rng.normal(size=3)
        u = np.cross(w, elements) + c               # (T, 4, 3)
        r = np.einsum("tab,tb->ta", A, u.reshape(-1, 12))
        assert np.abs(r).max() < 1e-11 * np.abs(A).max() * np.abs(u).max()


def test_energy_of_affine_field(elements):
    """For u = G x the discrete energy equals the exact integral
    |t| (2 mu eps(G):eps(G) + lam tr(G)^2) (P1 reproduces affine fields)."""
    mu, lam = 0.45, 1.7
    A = _as_matrix(form_tensor(elements, mu, lam))
    _, vol = p1_gradients(elements)
    rng = np.random.default_rng(9)
    G = rng.normal(size=(3, 3))
    u = np.einsum("cd,tad->tac", G, elements).reshape(-1, 12)
    energy = np.einsum("ta,tab,tb->t", u, A, u)
    eps = 0.5 * (G + G.T)
    exact = vol * (2 * mu * np.sum(eps * eps) + lam * np.trace(G) ** 2)
    assert np.allclose(energy, exact, rtol=1e-11)


def test_point_reflection_relation(elements):
    """Reflected element t^m through the midpoint of edge ij: its tensor for
    (i, j) is the transpose, so symmetric parts agree and antisymmetric parts
    change sign (Sec. 2, proof of the Lemma)."""
    a = form_tensor(elements, 0.8, 0.3)
    # reflect through midpoint of vertices 0 and 1: v -> x0 + x1 - v; the
    # reflected element has vertex 0 <-> 1 swapped in role
    Xm = elements[:, 0:1] + elements[:, 1:2] - elements
    am = form_tensor(Xm, 0.8, 0.3)
    # in t^m node i sits at the image of j, i.e. local index 1, and j at 0
    np.testing.assert_allclose(sym_part(am[:, 1, 0]), sym_part(a[:, 0, 1]), atol=1e-12)
    np.testing.assert_allclose(antisym_part(am[:, 1, 0]), -antisym_part(a[:, 0, 1]), atol=1e-12)


def test_antisymmetric_closed_form_3d(elements):
    """Eq. localcorr3d (Sec. 2.4): for the 2 (eps, eps) form the antisymmetric
    part of a_ij is the cross-product matrix of (x_p - x_q)/12 for a positively
    oriented (x_j - x_i, x_p - x_i, x_q - x_i); the (eps, eps) form gives half
    of it and (div, div) the same values with flipped sign."""
    X = elements
    a2 = form_tensor(X, 1.0, 0.0)
    ae = form_tensor(X, 0.5, 0.0)     # 2 * 0.5 (eps, eps) = (eps, eps)
    ad = form_tensor(X, 0.0, 1.0)
    for (i, j, p, q) in [(0, 1, 2, 3), (1, 3, 0, 2), (2, 0, 3, 1), (3, 2, 1, 0)]:
        A = antisym_part(a2[:, i, j])
        d = (X[:, p] - X[:, q]) / 12.0
        orient = np.sign(np.einsum("ti,ti->t", np.cross(X[:, j] - X[:, i], X[:, p] - X[:, i]),
                                   X[:, q] - X[:, i]))
        d = orient[:, None] * d
        Z = np.zeros(X.shape[0])
        closed = np.stack([np.stack([Z, -d[:, 2], d[:, 1]], 1),
                           np.stack([d[:, 2], Z, -d[:, 0]], 1),
                           np.stack([-d[:, 1], d[:, 0], Z], 1)], 1)   # [l, m]
        np.testing.assert_allclose(A, closed, atol=1e-12)
        np.testing.assert_allclose(antisym_part(ae[:, i, j]), 0.5 * closed, atol=1e-12)
        np.testing.assert_allclose(antisym_part(ad[:, i, j]), -closed, atol=1e-12)
