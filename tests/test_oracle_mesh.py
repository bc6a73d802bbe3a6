"""Pins of the oracle's micro-mesh (Bey refinement, Sec. 2) against counts and
structure the paper states and against an independent lattice construction."""
import itertools
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle.mesh import MacroMesh, reference_refinement, bey_children
from oracle.forms import p1_gradients

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")))


@pytest.mark.parametrize("level", range(0, 6))
def test_counts(level):
    n = 1 << level
    ijk, tets = reference_refinement(level)
    assert ijk.shape[0] == (n + 1) * (n + 2) * (n + 3) // 6
    assert tets.shape[0] == n ** 3
    bc = np.column_stack([n - ijk.sum(1), ijk])
    interior = np.all(bc > 0, axis=1).sum()
    assert interior == max(n - 1, 0) * max(n - 2, 0) * max(n - 3, 0) // 6


def test_paper_printed_sizes():
    """Sec. 5.1.1 sizes at the benchmark level (129 points per macro edge)."""
    ijk, _ = reference_refinement(7)
    nodes = ijk.shape[0]
    n = 128
    interior = (n - 1) * (n - 2) * (n - 3) // 6
    g = GOLD
    assert abs(3 * nodes / g["dofs_per_macro_L5"]["value"] - 1) < g["dofs_per_macro_L5"]["rel_tol"]
    assert abs(3 * nodes * 8 / 2**20 / g["vector_storage_MiB"]["value"] - 1) < 0.01
    assert abs(nodes * 8 / 2**20 / g["coefficient_storage_MiB"]["value"] - 1) < 0.01
    assert 500 * 3 * interior == g["inner_loop_executions"]["value"]


def test_volumes_partition_random_macro():
    rng = np.random.default_rng(3)
    V = rng.normal(size=(1, 4, 3))
    m = MacroMesh(V, 3, dirichlet="none")
    X = m.local_xyz[0][m.local_tets[0]]
    _, vol = p1_gradients(X)
    M = (V[0, 1:] - V[0, 0]).T
    total = abs(np.linalg.det(M)) / 6
    assert np.isclose(vol.sum(), total, rtol=1e-12)
    assert np.allclose(vol, total / 8**3, rtol=1e-10)   # all children equal volume


def _freudenthal(level):
    """Independent lattice triangulation: v0 + partial sums of a permutation
    of the steps (1,0,0), (-1,1,0), (0,-1,1), kept if inside the simplex."""
    n = 1 << level
    steps = np.array([[1, 0, 0], [-1, 1, 0], [0, -1, 1]])
    out = set()
    pts = [(i, j, k) for i in range(n + 1) for j in range(n + 1) for k in range(n + 1) if i + j + k <= n]
    ok = lambda p: min(p) >= 0 and sum(p) <= n  # noqa: E731
    for p in pts:
        for perm in itertools.permutations(range(3)):
            v = [np.array(p)]
            for s in perm:
                v.append(v[-1] + steps[s])
            if all(ok(tuple(q)) for q in v):
                out.add(frozenset(tuple(q) for q in v))
    return out


@pytest.mark.parametrize("level", [1, 2, 3])
def test_bey_equals_freudenthal_lattice(level):
    ijk, tets = reference_refinement(level)
    bey = {frozenset(tuple(ijk[v]) for v in t) for t in tets}
    assert bey == _freudenthal(level)


def test_interior_neighbourhood_structure():
    """Every macro-interior node: 24 elements, 14 neighbours; 8 edges with 6
    elements and 6 edges with 4 (Sec. 2, Sec. 2.4, Sec. 4.1.1)."""
    level = 4
    n = 1 << level
    ijk, tets = reference_refinement(level)
    bc = np.column_stack([n - ijk.sum(1), ijk])
    interior = np.nonzero(np.all(bc > 0, axis=1))[0]
    offsets_seen = set()
    for i in interior[::7]:
        ts = tets[np.any(tets == i, axis=1)]
        assert ts.shape[0] == 24
        nb = {}
        for t in ts:
            for v in t:
                if v != i:
                    nb[v] = nb.get(v, 0) + 1
        assert len(nb) + 1 == GOLD["stencil_points"]["value"]
        cnt = sorted(nb.values())
        assert cnt.count(GOLD["elements_per_red_edge"]["value"]) == GOLD["red_edges_per_stencil"]["value"]
        assert cnt.count(GOLD["elements_per_other_edge"]["value"]) == GOLD["other_edges_per_stencil"]["value"]
        offsets_seen |= {tuple(ijk[v] - ijk[i]) for v in nb}
    assert len(offsets_seen) == 14            # the same stencil at every node


def test_three_congruence_classes():
    """Up to translation and point reflection the elements fall into three
    classes with eight elements of each class at an interior node (Sec. 2.4)."""
    level = 3
    n = 1 << level
    ijk, tets = reference_refinement(level)

    def shape(t, sign):
        p = sign * ijk[t]
        p = p - p.min(axis=0)
        return tuple(sorted(map(tuple, p)))

    classes = {}
    for t in tets:
        a, b = shape(t, 1), shape(t, -1)
        key = min(a, b)
        classes[key] = classes.get(key, 0) + 1
    assert len(classes) == GOLD["congruence_classes"]["value"]
    bc = np.column_stack([n - ijk.sum(1), ijk])
    i = np.nonzero(np.all(bc > 1, axis=1))[0][0]
    ts = tets[np.any(tets == i, axis=1)]
    per = {}
    for t in ts:
        key = min(shape(t, 1), shape(t, -1))
        per[key] = per.get(key, 0) + 1
    assert sorted(per.values()) == [GOLD["elements_per_class_at_node"]["value"]] * 3


def test_conforming_meshes_node_counts():
    for L in (1, 2, 3):
        n = 1 << L
        m = MacroMesh(W.kuhn6(), L)
        assert m.n_nodes == (n + 1) ** 3
        assert m.dirichlet.sum() == (n + 1) ** 3 - (n - 1) ** 3
        m = MacroMesh(W.cube24(), L)
        # 15 macro vertices, 50 macro edges, 60 macro faces, 24 macro cells
        expect = 15 + 50 * (n - 1) + 60 * (n - 1) * (n - 2) // 2 + 24 * (n - 1) * (n - 2) * (n - 3) // 6
        assert m.n_nodes == expect
        # outer boundary of the cube: 6 faces of a grid with 2n intervals per side
        # in the face-centre split; count boundary nodes geometrically
        on_bnd = np.any((np.abs(m.xyz) < 1e-12) | (np.abs(m.xyz - 1) < 1e-12), axis=1)
        assert np.array_equal(on_bnd, m.dirichlet)


def test_independent_macros_do_not_share():
    V = np.concatenate([W.unit_tet(), W.unit_tet()])
    m = MacroMesh(V, [2, 3], coupling="independent")
    assert m.n_nodes == 35 + 165
    assert m.dirichlet.sum() == (35 - 1) + (165 - 35)   # all but interior nodes


def test_bey_children_even_coordinates():
    t = np.array([[[0, 0, 0], [4, 0, 0], [0, 4, 0], [0, 0, 4]]])
    c = bey_children(t)
    assert c.shape == (8, 4, 3)
    assert np.all(c % 2 == 0)
