"""Pins of the 2-D oracle (paper Sec. 2, Sec. 2.3): mesh, element matrices,
the closed form eq. correction2d and the scaled operator."""
import numpy as np
import pytest

import workloads as W
from oracle import twod as T

MU, LAM = W.eform_weights()
EFORM = dict(mu1=MU, lam1=LAM)
MIXED = dict(mu0=1.0, lam1=1.0)


@pytest.fixture(scope="module", params=["triangle", "square", "cross"])
def mesh(request):
    return T.Mesh2D(W.twod_mesh(request.param), 3)


def _interior_dofs(mesh):
    nodes = np.nonzero(~mesh.interface)[0]
    return (2 * nodes[:, None] + np.arange(2)).ravel()


def test_refinement_counts_and_area():
    """Uniform refinement: n^2 congruent triangles covering the macro, (n+1)(n+2)/2
    nodes, 6 neighbours and 6 triangles at an interior node, 2 triangles at
    an interior edge."""
    for L in (1, 2, 4):
        n = 1 << L
        ij, tris = T.reference_refinement(L)
        assert len(ij) == (n + 1) * (n + 2) // 2 and len(tris) == n * n
        X = ij[tris].astype(float)
        e1, e2 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]
        area = 0.5 * np.abs(e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
        assert np.allclose(area, 0.5) and abs(area.sum() - n * n / 2) < 1e-12
        inner = np.nonzero((ij[:, 0] > 0) & (ij[:, 1] > 0) & (ij.sum(1) < n))[0]
        for a in inner:
            touching = tris[np.any(tris == a, axis=1)]
            assert len(touching) == 6 and len(np.unique(touching)) == 7
        edges = np.sort(np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [0, 2]]]), axis=1)
        _, cnt = np.unique(edges, axis=0, return_counts=True)
        assert set(cnt.tolist()) <= {1, 2} and (cnt == 1).sum() == 3 * n


def test_conforming_meshes():
    sq = T.Mesh2D(W.twod_mesh("square"), 3)
    assert sq.n_nodes == 9 * 9 and sq.dirichlet.sum() == 4 * 8
    # four macros with (9 * 10 / 2) nodes each, sharing 4 half-diagonals of
    # 9 nodes (the centre counted once)
    cr = T.Mesh2D(W.twod_mesh("cross"), 3)
    assert cr.n_nodes == 4 * 45 - 4 * 9 + 1 and cr.dirichlet.sum() == 4 * 8


def test_element_matrices(mesh):
    """Zero block-row sums, a_ij = a_ji^T, rigid motions (translations and the
    rotation (-y, x)) in the kernel of the eps form, and the energy of an
    affine displacement."""
    X = mesh.local_xy[0][mesh.local_tris[0]][:5]
    a = T.form_tensor(X, 1.0, 0.7)
    assert np.abs(a.sum(axis=2)).max() < 1e-14
    assert np.abs(a - np.swapaxes(np.swapaxes(a, 1, 2), -1, -2)).max() < 1e-14
    e = T.form_tensor(X, 1.0, 0.0)
    for u in (lambda x: np.array([1.0, 0.0]), lambda x: np.array([0.0, 1.0]),
              lambda x: np.array([-x[1], x[0]])):
        U = np.array([[u(x) for x in tri] for tri in X])          # (t, vertex, comp)
        r = np.einsum("tijlm,tjl->tim", e, U)
        assert np.abs(r).max() < 1e-13
    G = np.array([[0.3, -0.2], [0.5, 0.1]])
    U = np.einsum("cd,tvd->tvc", G, X)
    _, area = T.p1_gradients(X)
    eps = 0.5 * (G + G.T)
    energy = np.einsum("tim,tijlm,tjl->t", U, a, U)
    want = area * (2.0 * np.sum(eps * eps) + 0.7 * np.trace(G) ** 2)
    assert np.allclose(energy, want, rtol=1e-12)


def test_correction_closed_form():
    """Eq. correction2d: R_ij = c (k_pt - k_ptm) J with J antisymmetric, the
    same for every edge; c = 1/12 for 2 (eps, eps) (the paper's value, which
    is twice that of the (eps, eps) form its derivation names: the gamma of
    eq. antisymmetric2d is a difference of the two off-diagonal entries), and
    the sign flipped for (div, div).  In the [trial][test] component
    convention R[1][0] = -s c (k_pt - k_ptm), s the orientation of
    (x_j - x_i, x_pt - x_i)."""
    mesh = T.Mesh2D(W.twod_mesh("square"), 3)
    rng = np.random.default_rng(1)
    k = rng.uniform(1.0, 2.0, mesh.n_nodes)
    for op, c in ((dict(mu1=1.0), 1.0 / 12), (dict(mu1=0.5), 1.0 / 24), (dict(lam1=1.0), -1.0 / 12)):
        _, parts = T.scaled_matrix(mesh, k, op, return_parts=True)
        assert parts
        for pr in parts:
            g, xy = mesh.gid[pr["macro"]], mesh.local_xy[pr["macro"]]
            i, j = pr["i"], pr["j"]
            pt, ptm = pr["others"]
            u, v = xy[j] - xy[i], xy[pt] - xy[i]
            s = np.sign(u[0] * v[1] - u[1] * v[0])
            want = -s * c * (k[g[pt]] - k[g[ptm]])
            assert abs(pr["R"][1, 0] - want) < 1e-14 and abs(pr["R"][0, 1] + want) < 1e-14
            assert abs(pr["R"][0, 0]) < 1e-15 and abs(pr["R"][1, 1]) < 1e-15


@pytest.mark.parametrize("op", [EFORM, MIXED], ids=["eform", "mixed"])
def test_physical_scaling_equals_nodal_integration(mesh, op):
    """In 2-D every edge patch is one element and its reflection, so the
    Lemma's scaled entries reproduce nodal integration for any k (not only
    affine k), on every row under the row-wise rule and on macro-interior
    rows under the others; the unphysical scaling does not."""
    rng = np.random.default_rng(3)
    k = np.exp(rng.uniform(-1, 1, mesh.n_nodes))
    An = T.nodal_matrix(mesh, k, op)
    scale = abs(An).max()
    assert abs(T.scaled_matrix(mesh, k, op, iface="rowwise") - An).max() < 1e-13 * scale
    rows = _interior_dofs(mesh)
    for iface in ("symmetric", "zerosum"):
        D = (T.scaled_matrix(mesh, k, op, iface=iface) - An).tocsr()[rows]
        assert abs(D).max() < 1e-13 * scale
    Du = (T.scaled_matrix(mesh, k, op, corr="none") - An).tocsr()[rows]
    assert abs(Du).max() > 1e-3 * scale


def test_unphysical_scaling_is_first_order():
    """Smooth k: the unphysical stencil departs from nodal integration like
    O(h) relative to the entries (it discretizes another operator)."""
    errs = []
    for L in (3, 4):
        mesh = T.Mesh2D(W.twod_mesh("square"), L)
        k = 2.0 + np.sin(3 * mesh.xy[:, 0]) * np.cos(2 * mesh.xy[:, 1])
        An = T.nodal_matrix(mesh, k, EFORM)
        rows = _interior_dofs(mesh)
        D = (T.scaled_matrix(mesh, k, EFORM, corr="none") - An).tocsr()[rows]
        errs.append(abs(D).max() / abs(An).max())
    assert 1.6 < errs[0] / errs[1] < 2.5


def test_symmetry_spd_and_translations(mesh):
    rng = np.random.default_rng(5)
    k = np.exp(rng.uniform(-1, 1, mesh.n_nodes))
    for iface in ("symmetric", "zerosum"):
        A = T.scaled_matrix(mesh, k, EFORM, iface=iface)
        assert abs(A - A.T).max() < 1e-14 * abs(A).max()
        Ar = T.reduce_dirichlet(mesh, A).toarray()
        if Ar.shape[0]:
            assert np.linalg.eigvalsh(Ar).min() > 0
    Az = T.scaled_matrix(mesh, k, EFORM, iface="zerosum")
    for c in range(2):
        t = np.zeros((mesh.n_nodes, 2))
        t[:, c] = 1.0
        assert np.abs(Az @ t.ravel()).max() < 1e-13 * abs(Az).max()


def test_planted_mistakes_are_caught(monkeypatch):
    """A flipped correction, a correction without its factor 1/2 and a
    transposed component convention each break the equality with nodal
    integration on interior rows."""
    mesh = T.Mesh2D(W.twod_mesh("triangle"), 3)
    k = 2.0 + np.sin(3 * mesh.xy[:, 0])
    An = T.nodal_matrix(mesh, k, EFORM)
    rows = _interior_dofs(mesh)
    orig = T.antisym_part
    for bad_part in (lambda a: -orig(a), lambda a: 2.0 * orig(a)):
        monkeypatch.setattr(T, "antisym_part", bad_part)
        bad = (T.scaled_matrix(mesh, k, EFORM) - An).tocsr()[rows]
        monkeypatch.undo()
        assert abs(bad).max() > 1e-4 * abs(An).max()
    orig_form = T.form_tensor
    monkeypatch.setattr(T, "form_tensor", lambda X, mu, lam: np.swapaxes(orig_form(X, mu, lam), -1, -2))
    At = T.nodal_matrix(mesh, k, EFORM)
    monkeypatch.undo()
    assert abs((At - An).tocsr()[rows]).max() > 1e-4 * abs(An).max()
