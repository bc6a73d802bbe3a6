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


def test_zerosum_rule(mesh):
    """Zero-sum interface rule: the symmetric rule's off-diagonal entries, a
    centre of minus the row's other entries on every row.  Symmetric,
    translations in the kernel of every row (interface rows included), equal
    to the symmetric rule on macro-interior rows and to nodal integration for
    constant k."""
    k = W.sine_coefficient(mesh.xyz) + 0.3 * np.cos(7 * mesh.xyz[:, 0])
    Az = O.scaled_matrix(mesh, k, EFORM, iface="zerosum").tocsr()
    As = O.scaled_matrix(mesh, k, EFORM).tocsr()
    scale = abs(As).max()
    assert abs(Az - Az.T).max() < 1e-14 * scale
    for c in range(3):
        t = np.zeros((mesh.n_nodes, 3))
        t[:, c] = 1.0
        assert np.abs(Az @ t.ravel()).max() < 1e-13 * scale
    irows = _interior_dofs(mesh)
    assert abs(Az[irows] - As[irows]).max() < 1e-14 * scale
    # off the 3x3 diagonal blocks the two rules agree entry by entry
    n = mesh.n_nodes
    blockdiag = sp.kron(sp.identity(n), np.ones((3, 3))).tocsr()
    D = (Az - As).tocsr()
    assert abs(D - D.multiply(blockdiag)).max() < 1e-15 * scale
    if mesh.interface.any():
        assert abs(D).max() > 1e-6 * scale        # the centre does change
    kc = np.full(mesh.n_nodes, 1.7)
    assert _rel(O.scaled_matrix(mesh, kc, EFORM, iface="zerosum"), O.nodal_matrix(mesh, kc, EFORM)) < 1e-13


def test_zerosum_spd_after_dirichlet():
    mesh = MacroMesh(W.kuhn6(), 2)
    k = np.exp(W.fourier_field(mesh.xyz, W.rng_for(2), 16, 1.0))
    Az = O.reduce_dirichlet(mesh, O.scaled_matrix(mesh, k, EFORM, iface="zerosum")).toarray()
    assert np.abs(Az - Az.T).max() < 1e-14 * np.abs(Az).max()
    assert np.linalg.eigvalsh(Az).min() > 0


def test_mass_matrix_closed_form():
    """P1 mass: total |Omega|, symmetric, and on the Kuhn lattice an interior
    row is h^3 (2/5 at the node, 1/20 towards the 8 neighbours along the
    six-element edges, 1/30 towards the 6 along the four-element edges)."""
    L = 3
    mesh = MacroMesh(W.kuhn6(), L)
    Mm = O.mass_matrix(mesh)
    assert abs(Mm.sum() - 1.0) < 1e-13
    assert abs(Mm - Mm.T).max() < 1e-17
    h3 = 1.0 / 8 ** L
    i = int(np.argmin(np.linalg.norm(mesh.xyz - 0.5, axis=1)))
    row = Mm[i].toarray().ravel()
    nb = np.flatnonzero(row)
    vals = np.sort(row[nb] / h3)
    assert np.allclose(vals, np.sort([0.4] + [1 / 20] * 8 + [1 / 30] * 6), rtol=1e-12, atol=0)


def _elastostatics_error(level, iface, m=8):
    """Discrete L2 nodal error of the direct solution of the elastostatics
    problem of Sec. 5.1.2 (E = cos(m pi xyz) + 2, manufactured u*) on the
    6-macro cube: load M I_h f, Dirichlet data u*."""
    import scipy.sparse.linalg as spla
    mesh = MacroMesh(W.kuhn6(), level)
    x = mesh.xyz
    k = W.elastostatics_modulus(x, m)
    us = W.elastostatics_solution(x)
    b = (O.mass_matrix(mesh) @ W.elastostatics_force(x, m)).ravel()
    A = O.scaled_matrix(mesh, k, EFORM, iface=iface).tocsr()
    unk = np.zeros(mesh.n_nodes, bool)
    unk[mesh.unknown] = True
    du = (3 * np.flatnonzero(unk)[:, None] + np.arange(3)).ravel()
    db = (3 * np.flatnonzero(~unk)[:, None] + np.arange(3)).ravel()
    g = us.ravel()
    Arows = A[du]
    w = spla.spsolve(Arows[:, du].tocsc(), b[du] - Arows[:, db] @ g[db])
    return np.sqrt(np.sum((w - g[du]) ** 2) / 8 ** level)


def test_zerosum_restores_second_order():
    """With the nodal centre on interface rows (the paper's symmetric rule)
    the elastostatics error for m = 8 falls at first order or below; the
    zero-sum centre brings back the second order that physical scaling
    reaches with the row-wise rule (Sec. 5.1.2)."""
    e = {r: [_elastostatics_error(L, r) for L in (3, 4)] for r in ("symmetric", "zerosum", "rowwise")}
    eoc = {r: np.log2(v[0] / v[1]) for r, v in e.items()}
    assert eoc["zerosum"] > 1.8 and eoc["rowwise"] > 1.8
    assert eoc["symmetric"] < 1.0
    assert abs(e["zerosum"][1] / e["rowwise"][1] - 1) < 0.1
