"""Hierarchical hybrid grid: macro-tets refined uniformly (paper Sec. 2).

The macro triangulation T_H is refined ``level`` times by Bey's regular
refinement of a tetrahedron into 8 children (the refinement the paper cites in
Sec. 2 for its grid hierarchy).  Refinement is carried out in the integer index
space of a macro, where the macro's vertices x0..x3 sit at (0,0,0), (n,0,0),
(0,n,0), (0,0,n) with n = 2**level, so node (i, j, k) lies at

    x = x0 + (i/n)(x1 - x0) + (j/n)(x2 - x0) + (k/n)(x3 - x0).

The barycentric coordinates of that node are (n-i-j-k, i, j, k)/n; a node lies
on the macro boundary dT iff one of them is zero.

Parity: pinned by tests (node and element counts, volume partition, the
15-point neighbourhood with 24 elements at a macro-interior node and 6 / 4
elements per interior edge quoted in Sec. 2 and Sec. 2.4, and agreement with an
independently built Freudenthal (Kuhn) lattice triangulation).
"""
from __future__ import annotations

import functools

import numpy as np
from scipy.spatial import cKDTree


def bey_children(t: np.ndarray) -> np.ndarray:
    """One step of Bey's regular refinement.

    ``t`` has shape (T, 4, 3) (integer vertex coordinates with even
    differences); returns the (8T, 4, 3) children.  With midpoints x_ab of the
    edges, the children are the four corner tets (x0,x01,x02,x03),
    (x01,x1,x12,x13), (x02,x12,x2,x23), (x03,x13,x23,x3) and the four tets of
    the inner octahedron cut along its diagonal x02-x13: (x01,x02,x03,x13),
    (x01,x02,x12,x13), (x02,x03,x13,x23), (x02,x12,x13,x23).
    """
    x0, x1, x2, x3 = t[:, 0], t[:, 1], t[:, 2], t[:, 3]
    m = lambda a, b: (a + b) // 2  # noqa: E731
    x01, x02, x03 = m(x0, x1), m(x0, x2), m(x0, x3)
    x12, x13, x23 = m(x1, x2), m(x1, x3), m(x2, x3)
    kids = [
        (x0, x01, x02, x03),
        (x01, x1, x12, x13),
        (x02, x12, x2, x23),
        (x03, x13, x23, x3),
        (x01, x02, x03, x13),
        (x01, x02, x12, x13),
        (x02, x03, x13, x23),
        (x02, x12, x13, x23),
    ]
    return np.concatenate([np.stack(k, axis=1) for k in kids], axis=0)


@functools.lru_cache(maxsize=16)
def reference_refinement(level: int):
    """Bey-refined reference macro in index space.

    Returns ``ijk`` (N, 3) int64 node index triples (lexicographic in (i,j,k))
    and ``tets`` (n^3, 4) local node ids, vertex order as produced by Bey's
    children (so every element keeps a well-defined local numbering).
    """
    if level < 0:
        raise ValueError("level must be >= 0")
    n = 1 << level
    t = np.array([[[0, 0, 0], [n, 0, 0], [0, n, 0], [0, 0, n]]], dtype=np.int64)
    for _ in range(level):
        t = bey_children(t)
    flat = t.reshape(-1, 3)
    key = flat[:, 0] * (n + 1) ** 2 + flat[:, 1] * (n + 1) + flat[:, 2]
    ukey, inv = np.unique(key, return_inverse=True)
    ijk = np.column_stack([ukey // (n + 1) ** 2, (ukey // (n + 1)) % (n + 1), ukey % (n + 1)])
    tets = inv.reshape(-1, 4).astype(np.int64)
    ijk.setflags(write=False)
    tets.setflags(write=False)
    return ijk, tets


def barycentric_index(ijk: np.ndarray, n: int) -> np.ndarray:
    """(N,4) integer barycentric coordinates times n: (n-i-j-k, i, j, k)."""
    return np.column_stack([n - ijk.sum(1), ijk[:, 0], ijk[:, 1], ijk[:, 2]])


class MacroMesh:
    """Macro triangulation with its uniform micro refinement.

    Parameters
    ----------
    verts : (M, 4, 3) macro vertex coordinates; the vertex order fixes each
            macro's index space.
    levels : int or (M,) ints; conforming meshes need one common level.
    coupling : 'conforming' (macros share faces/edges/vertices, matched by
               coordinates) or 'independent' (each macro its own problem).
    dirichlet : 'outer' (homogeneous Dirichlet on every macro face that belongs
                to a single macro) or 'none'.

    Attributes
    ----------
    n_nodes : number of unique micro nodes.
    xyz : (n_nodes, 3) coordinates.
    gid : list of (N_m,) arrays mapping macro-local node -> unique node.
    local_ijk, local_tets : per macro, index triples and element connectivity.
    on_macro_boundary : list of (N_m,) bool, node on dT of that macro.
    interface : (n_nodes,) bool, node lies on dT of at least one macro.
    dirichlet : (n_nodes,) bool.
    """

    def __init__(self, verts, levels, coupling="conforming", dirichlet="outer"):
        verts = np.asarray(verts, dtype=np.float64)
        if verts.ndim != 3 or verts.shape[1:] != (4, 3):
            raise ValueError("verts must be (M,4,3)")
        self.verts = verts
        self.n_macro = verts.shape[0]
        lv = np.broadcast_to(np.asarray(levels, dtype=np.int64), (self.n_macro,)).copy()
        self.levels = lv
        if coupling not in ("conforming", "independent"):
            raise ValueError(coupling)
        if coupling == "conforming" and len(set(lv.tolist())) != 1:
            raise ValueError("conforming macros need one common level")
        self.coupling = coupling

        self.local_ijk, self.local_tets, self.local_xyz = [], [], []
        self.on_macro_boundary, self.bary = [], []
        for m in range(self.n_macro):
            n = 1 << int(lv[m])
            ijk, tets = reference_refinement(int(lv[m]))
            x0 = verts[m, 0]
            E = verts[m, 1:] - x0                      # rows x1-x0, x2-x0, x3-x0
            xyz = x0 + (ijk.astype(np.float64) / n) @ E
            bc = barycentric_index(ijk, n)
            self.local_ijk.append(ijk)
            self.local_tets.append(tets)
            self.local_xyz.append(xyz)
            self.bary.append(bc)
            self.on_macro_boundary.append(np.any(bc == 0, axis=1))

        self._number_nodes()
        self._classify_dirichlet(dirichlet)

    # ------------------------------------------------------------ numbering
    def _number_nodes(self):
        counts = [x.shape[0] for x in self.local_xyz]
        starts = np.concatenate([[0], np.cumsum(counts)])
        total = int(starts[-1])
        parent = np.arange(total)
        if self.coupling == "conforming" and self.n_macro > 1:
            # only macro-boundary nodes can be shared between macros
            cand = np.concatenate([starts[m] + np.nonzero(self.on_macro_boundary[m])[0]
                                   for m in range(self.n_macro)])
            pts = np.concatenate(self.local_xyz)[cand]
            h = 1.0 / (1 << int(self.levels[0]))
            scale = np.max(np.abs(self.verts)) + 1.0
            tree = cKDTree(pts)
            pairs = tree.query_pairs(r=1e-9 * h * scale, output_type="ndarray")
            # union-find over candidate pairs
            def find(a):
                while parent[a] != a:
                    parent[a] = parent[parent[a]]
                    a = parent[a]
                return a
            for a, b in pairs:
                ra, rb = find(cand[a]), find(cand[b])
                if ra != rb:
                    lo, hi = min(ra, rb), max(ra, rb)
                    parent[hi] = lo
            while True:                       # pointer jumping to the roots
                nxt = parent[parent]
                if np.array_equal(nxt, parent):
                    break
                parent = nxt
        roots, flat_gid = np.unique(parent, return_inverse=True)
        # order unique nodes by first occurrence
        first = np.full(roots.shape[0], total, dtype=np.int64)
        np.minimum.at(first, flat_gid, np.arange(total))
        order = np.argsort(first, kind="stable")
        rank = np.empty_like(order)
        rank[order] = np.arange(order.shape[0])
        flat_gid = rank[flat_gid]
        self.n_nodes = int(roots.shape[0])
        self.gid = [flat_gid[starts[m]:starts[m + 1]] for m in range(self.n_macro)]
        self.xyz = np.zeros((self.n_nodes, 3))
        for m in range(self.n_macro):
            self.xyz[self.gid[m]] = self.local_xyz[m]
        self.interface = np.zeros(self.n_nodes, dtype=bool)
        for m in range(self.n_macro):
            self.interface[self.gid[m][self.on_macro_boundary[m]]] = True

    # ------------------------------------------------------------ Dirichlet
    def _classify_dirichlet(self, mode):
        self.dirichlet = np.zeros(self.n_nodes, dtype=bool)
        if mode == "none":
            return
        if mode != "outer":
            raise ValueError(mode)
        # macro faces: face opposite vertex a has barycentric coordinate a = 0
        keys = {}
        scale = np.max(np.abs(self.verts)) + 1.0
        for m in range(self.n_macro):
            for a in range(4):
                fv = np.delete(self.verts[m], a, axis=0)
                key = tuple(sorted(tuple(np.round(v / scale, 10)) for v in fv))
                if self.coupling == "independent":
                    key = (m,) + key
                keys.setdefault(key, []).append((m, a))
        for owners in keys.values():
            if len(owners) == 1:
                m, a = owners[0]
                on_face = self.bary[m][:, a] == 0
                self.dirichlet[self.gid[m][on_face]] = True

    # ------------------------------------------------------------ helpers
    @property
    def unknown(self) -> np.ndarray:
        """Indices of non-Dirichlet nodes (the unknowns), ascending."""
        return np.nonzero(~self.dirichlet)[0]

    def tet_coords(self, m: int, tets: np.ndarray | None = None) -> np.ndarray:
        t = self.local_tets[m] if tets is None else tets
        return self.local_xyz[m][t]
