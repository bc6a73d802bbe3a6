"""Test helpers: map library slots to oracle nodes and compare results."""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from oracle.mesh import MacroMesh


def slot_to_node(lib_mesh, orc: MacroMesh) -> np.ndarray:
    """Oracle node id of every library slot, matched by coordinates (for
    independent macros additionally by macro)."""
    xyz = lib_mesh.coords().T
    if orc.coupling == "independent":
        out = np.empty(lib_mesh.n_nodes, dtype=np.int64)
        off = lib_mesh.macro_offset
        for m in range(orc.n_macro):
            tree = cKDTree(orc.local_xyz[m])
            d, idx = tree.query(xyz[off[m]:off[m + 1]])
            assert d.max() < 1e-9
            out[off[m]:off[m + 1]] = orc.gid[m][idx]
        return out
    tree = cKDTree(orc.xyz)
    d, idx = tree.query(xyz)
    assert d.max() < 1e-9, d.max()
    return idx


def scatter(values: np.ndarray, s2n: np.ndarray) -> np.ndarray:
    """Node-indexed (n_nodes, c) array -> slot-indexed SoA (c, n_slots)."""
    v = values[s2n]
    return np.ascontiguousarray(v.T) if v.ndim == 2 else np.ascontiguousarray(v)


def gather_consistent(y_soa: np.ndarray, s2n: np.ndarray, n_nodes: int) -> np.ndarray:
    """Slot SoA (3, n_slots) -> node array (n_nodes, 3), asserting that all
    copies of a node carry identical values."""
    out = np.full((n_nodes, 3), np.nan)
    out[s2n] = y_soa.T
    again = out[s2n]
    assert np.array_equal(again, y_soa.T), "copies of an interface node differ"
    return out


def rel_err(a: np.ndarray, b: np.ndarray) -> float:
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
