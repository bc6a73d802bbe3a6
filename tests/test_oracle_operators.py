"""Pins of the oracle's nodal-integration and stencil-scaling operators against
what the paper fixes (Sec. 2, Lemma and Sec. 2.2) and against the algebra of
the 3-D correction (Sec. 2.4)."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import operators as O
from oracle.forms import antisym_part
from oracle.mesh import MacroMesh

MU, LAM = W.eform_weights()
EFORM = dict(mu1=MU, lam1=LAM)
MIXED = dict(mu0=1.0, lam1=1.0)          # mu = 1 unscaled, lambda = k scaled


def _interior_dofs(mesh):
    nodes = np.nonzero(~mesh.interface)[0]
    return (3 * nodes[:, None] + np.arange(3)).ravel()


def _rel(A, B, rows=None):
    D = (A - B).tocsr()
    if rows is not None:
        D = D[rows]
    return abs(D).max() / abs(B).max()


MESHES = [("unit", W.unit_tet(), 3), ("kuhn6", W.kuhn6(), 2), ("cube24", W.cube24(), 2)]


@pytest.fixture(scope="module", params=MESHES, ids=[m[0] for m in MESHES])
def mesh(request):
    _, verts, L = request.param
    return MacroMesh(verts, L)


@pytest.mark.parametrize("op", [EFORM, MIXED], ids=["eform", "mixed"])
def test_constant_coefficient_equal(mesh, op):
    """k constant: scaled form equals nodal integration (Sec. 2.2)."""
    k = np.full(mesh.n_nodes, 1.7)
    An = O.nodal_matrix(mesh, k, op)
    for iface in ("symmetric", "rowwise"):
        As = O.scaled_matrix(mesh, k, op, iface=iface)
        assert _rel(As, An) < 1e-13


@pytest.mark.parametrize("op", [EFORM, MIXED], ids=["eform", "mixed"])
def test_affine_coefficient_interior_rows_equal(mesh, op):
    """k globally affine: physical scaling equals nodal integration on every
    macro-interior row (Lemma; Sec. 2.2), for both k-hat rules (the edge mean
    equals the patch mean for affine k)."""
    k = W.affine_coefficient(mesh.xyz)
    An = O.nodal_matrix(mesh, k, op)
    rows = _interior_dofs(mesh)
    for khat in ("patch", "edge"):
        As = O.scaled_matrix(mesh, k, op, khat=khat)
        assert _rel(As, An, rows) < 1e-13


def test_unphysical_differs_for_affine(mesh):
    """Without R the scaled form differs from a_h for non-constant affine k."""
    k = W.affine_coefficient(mesh.xyz)
    An = O.nodal_matrix(mesh, k, EFORM)
    Au = O.scaled_matrix(mesh, k, EFORM, corr="none")
    assert _rel(Au, An, _interior_dofs(mesh)) > 1e-4


def test_symmetry_and_translations(mesh):
    """Symmetric interface rule gives a symmetric matrix; macro-interior rows
    have zero block-row sums so translations lie in their kernel (Lemma)."""
    k = W.sine_coefficient(mesh.xyz) + 0.3 * np.cos(7 * mesh.xyz[:, 0])
    As = O.scaled_matrix(mesh, k, EFORM)
    assert abs(As - As.T).max() < 1e-14 * abs(As).max()
    rows = _interior_dofs(mesh)
    for c in range(3):
        t = np.zeros((mesh.n_nodes, 3))
        t[:, c] = 1.0
        assert np.abs((As @ t.ravel())[rows]).max() < 1e-13 * abs(As).max()


def test_rowwise_is_nodal_on_interface_rows(mesh):
    k = W.sine_coefficient(mesh.xyz) + 1.0
    An = O.nodal_matrix(mesh, k, EFORM).tocsr()
    Ar = O.scaled_matrix(mesh, k, EFORM, iface="rowwise").tocsr()
    Asym = O.scaled_matrix(mesh, k, EFORM).tocsr()
    inodes = np.nonzero(mesh.interface)[0]
    rows = (3 * inodes[:, None] + np.arange(3)).ravel()
    assert abs(Ar[rows] - An[rows]).max() < 1e-14 * abs(An).max()
    irows = _interior_dofs(mesh)
    assert abs(Ar[irows] - Asym[irows]).max() < 1e-14 * abs(An).max()


def test_nodal_properties(mesh):
    """a_h: symmetric, rigid-body modes in the Neumann kernel, linear in k,
    SPD after Dirichlet reduction."""
    rng = np.random.default_rng(2)
    k = np.exp(rng.uniform(-1, 1, mesh.n_nodes))
    An = O.nodal_matrix(mesh, k, EFORM)
    assert abs(An - An.T).max() < 1e-14 * abs(An).max()
    for w in np.eye(3):
        u = np.cross(w, mesh.xyz)
        assert np.abs(An @ u.ravel()).max() < 1e-12 * abs(An).max()
    assert _rel(O.nodal_matrix(mesh, 3.0 * k, EFORM), 3.0 * An) < 1e-14
    Ar = O.reduce_dirichlet(mesh, An).toarray()
    if Ar.shape[0]:
        assert np.linalg.eigvalsh(Ar).min() > 0


def test_scaled_spd_after_dirichlet():
    mesh = MacroMesh(W.kuhn6(), 2)
    k = np.exp(W.fourier_field(mesh.xyz, W.rng_for(2), 16, 1.0))
    As = O.reduce_dirichlet(mesh, O.scaled_matrix(mesh, k, EFORM)).toarray()
    assert np.abs(As - As.T).max() < 1e-14 * np.abs(As).max()
    assert np.linalg.eigvalsh(As).min() > 0


def test_antisymmetric_blocks_match_nodal():
    """R_ij equals the block-antisymmetric part of the nodal entry, since the
    reflected pairs t, t^m cover T_ij: antisym(S_ij) = antisym(a_h,ij) on
    macro-interior rows for any k."""
    mesh = MacroMesh(W.unit_tet(), 3)
    rng = np.random.default_rng(4)
    k = rng.uniform(0.5, 2.0, mesh.n_nodes)
    _, parts = O.scaled_matrix(mesh, k, EFORM, return_parts=True)
    p = parts[0]
    np.testing.assert_allclose(p["R"], antisym_part(p["nodal"]), atol=1e-14)


def test_ring_form_equals_lemma():
    """Sec. 2.4 rewrites R_ij through ring nodes: with H_ij one node of each
    pair (v, v^m = x_i + x_j - v) around the edge, R_ij = sum_v (k_v - k_v^m)
    C^v with C^v a quarter of the antisymmetric parts of the two elements of
    T_ij containing v.  Checked against the oracle's literal Lemma for random
    nodal k; also 3 terms on 6-element edges and 2 on 4-element edges."""
    from oracle.forms import form_tensor
    mesh = MacroMesh(W.unit_tet(), 3)
    rng = np.random.default_rng(8)
    k = rng.uniform(0.5, 2.0, mesh.n_nodes)
    _, parts = O.scaled_matrix(mesh, k, EFORM, return_parts=True)
    p = parts[0]
    tets = mesh.local_tets[0]
    ijk = mesh.local_ijk[0]
    lut = {tuple(v): a for a, v in enumerate(ijk)}
    checked = 0
    for e in range(0, p["i"].shape[0], 11):
        i, j = p["i"][e], p["j"][e]
        T_ij = tets[np.all(np.isin(tets, [i, j]).sum(1, keepdims=True) == 2, axis=1)]
        a1 = form_tensor(mesh.local_xyz[0][T_ij], MU, LAM)
        ring = sorted({v for t in T_ij for v in t if v not in (i, j)})
        half = []
        for v in ring:
            vm = lut[tuple(ijk[i] + ijk[j] - ijk[v])]
            if vm in ring and vm not in half and v not in half:
                half.append(v)
        assert len(half) == (3 if T_ij.shape[0] == 6 else 2)
        R = np.zeros((3, 3))
        for v in half:
            vm = lut[tuple(ijk[i] + ijk[j] - ijk[v])]
            C = np.zeros((3, 3))
            for t, blk in zip(T_ij, a1):
                if v in t:
                    a_loc = list(t).index(i)
                    b_loc = list(t).index(j)
                    C += 0.25 * antisym_part(blk[a_loc, b_loc])
            R += (k[v] - k[vm]) * C
        np.testing.assert_allclose(R, p["R"][e], atol=1e-14)
        checked += 1
    assert checked > 30


def _max_rel_entry_error(L, corr):
    mesh = MacroMesh(W.unit_tet(), L)
    x = mesh.xyz      # smooth, gradient-dominated coefficient
    k = np.exp(0.8 * x[:, 0] - 0.5 * x[:, 1] + 0.3 * x[:, 2] + 0.4 * x[:, 0] * x[:, 1])
    An = O.nodal_matrix(mesh, k, EFORM)
    As = O.scaled_matrix(mesh, k, EFORM, corr=corr)
    return _rel(As, An, _interior_dofs(mesh))


@pytest.mark.slow
def test_consistency_orders():
    """Smooth k: physical scaling approaches nodal integration like O(h^2), the
    unphysical one only like O(h) (Lemma: exact for linear k on each patch;
    Sec. 2.1: the unphysical form discretizes a different PDE)."""
    e3, e4 = _max_rel_entry_error(3, "physical"), _max_rel_entry_error(4, "physical")
    u3, u4 = _max_rel_entry_error(3, "none"), _max_rel_entry_error(4, "none")
    assert e3 / e4 > 3.0
    assert u3 / u4 < 2.5
    assert u4 > 3 * e4


def test_planted_mistakes_are_caught(monkeypatch):
    """Mutations of the oracle that a careless implementation could contain
    must break the affine-coefficient pin."""
    mesh = MacroMesh(W.unit_tet(), 3)
    k = W.affine_coefficient(mesh.xyz)
    An = O.nodal_matrix(mesh, k, EFORM)
    rows = _interior_dofs(mesh)
    import oracle.operators as mod
    # (1) wrong sign of the antisymmetric part
    monkeypatch.setattr(mod, "antisym_part", lambda a: -antisym_part(a))
    assert _rel(O.scaled_matrix(mesh, k, EFORM), An, rows) > 1e-4
    monkeypatch.undo()
    # (2) transposed component convention of the scaled part
    orig = mod.form_tensor
    monkeypatch.setattr(mod, "form_tensor", lambda X, mu, lam: np.swapaxes(orig(X, mu, lam), -1, -2))
    An_t = O.nodal_matrix(mesh, k, EFORM)
    monkeypatch.undo()
    assert _rel(An_t, An, rows) > 1e-4
    # (3) dropping the correction
    assert _rel(O.scaled_matrix(mesh, k, EFORM, corr="none"), An, rows) > 1e-4


def test_apply_handles_dirichlet():
    mesh = MacroMesh(W.unit_tet(), 3)
    rng = np.random.default_rng(1)
    k = W.sine_coefficient(mesh.xyz)
    x = rng.uniform(-1, 1, (mesh.n_nodes, 3))
    y = O.apply(mesh, k, MIXED, x)
    assert np.all(y[mesh.dirichlet] == 0)
    xd = x.copy()
    xd[mesh.dirichlet] = 0
    Ar = O.reduce_dirichlet(mesh, O.scaled_matrix(mesh, k, MIXED))
    u = mesh.unknown
    np.testing.assert_allclose(y[u].ravel(), Ar @ xd[u].ravel(), rtol=1e-13, atol=1e-14)
    # row sampling gives the same rows
    rows = u[::5]
    ys = O.apply(mesh, k, MIXED, x, rows=rows)
    np.testing.assert_allclose(ys[rows], y[rows], rtol=1e-13, atol=1e-15)
