"""C-ABI library: loads, exports what include/hhg.h declares, host-side setup
(layout, coordinates, Dirichlet and copy bookkeeping) and argument checks.
No device compute here."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle.mesh import MacroMesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hhg.h")

pytestmark = pytest.mark.skipif(
    not os.path.exists(os.path.join(ROOT, "paper_1908_08666_amd", "libhhg.so")),
    reason="libhhg.so not built")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(hhg(?:2d)?_\w+)\s*\(", text, re.M)))


def test_exports_every_declared_symbol():
    from paper_1908_08666_amd import _lib as L
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 9
    for name in names:
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, f"binding lacks {name}"


def _mesh(verts, level, **kw):
    from paper_1908_08666_amd import Mesh
    mu, lam = W.eform_weights()
    return Mesh(verts, level, mu1=mu, lam1=lam, **kw)


@pytest.mark.parametrize("name,verts,L", [("unit", W.unit_tet(), 4), ("kuhn6", W.kuhn6(), 3),
                                          ("cube24", W.cube24(), 2)])
def test_layout_matches_oracle(name, verts, L):
    from tests.helpers import slot_to_node
    m = _mesh(verts, L)
    orc = MacroMesh(verts, L)
    n = 1 << L
    assert m.n_nodes == len(verts) * (n + 1) * (n + 2) * (n + 3) // 6
    s2n = slot_to_node(m, orc)
    assert set(s2n.tolist()) == set(range(orc.n_nodes))
    fl = m.flags()
    # Dirichlet flags agree with the oracle's outer-boundary nodes
    assert np.array_equal((fl & 1).astype(bool), orc.dirichlet[s2n])
    # exactly one owner copy per distinct node
    owners = s2n[(fl & 2) > 0]
    assert np.array_equal(np.sort(owners), np.arange(orc.n_nodes))
    assert m.n_unknown == int((~orc.dirichlet).sum())
    # slots completed by a copy-group sum: shared non-Dirichlet nodes
    counts = np.bincount(s2n, minlength=orc.n_nodes)
    assert np.array_equal(((fl & 8) > 0), (counts[s2n] > 1) & ~orc.dirichlet[s2n])


def test_independent_levels_layout():
    from paper_1908_08666_amd import Mesh
    V = np.concatenate([W.unit_tet()] * 3)
    m = Mesh(V, [2, 4, 3], mu1=1.0, coupling="independent")
    sizes = np.diff(m.macro_offset)
    assert sizes.tolist() == [35, 969, 165]
    fl = m.flags()
    assert ((fl & 8) == 0).all() and ((fl & 2) > 0).all()


def test_node_index_formula():
    """Slot of node (i, j, k) is P(k) + (i+j)(i+j+1)/2 + i (include/hhg.h)."""
    m = _mesh(W.unit_tet(), 3)
    xyz = m.coords()
    n = 8
    for (i, j, k) in [(0, 0, 0), (1, 2, 3), (8, 0, 0), (0, 8, 0), (0, 0, 8), (2, 2, 2)]:
        P = sum((n + 1 - q) * (n + 2 - q) // 2 for q in range(k))
        s = i + j
        slot = P + s * (s + 1) // 2 + i
        np.testing.assert_allclose(xyz[:, slot], [i / n, j / n, k / n], atol=1e-15)


@pytest.mark.parametrize("bad", ["level_low", "level_high", "mixed", "degenerate", "enum", "nan"])
def test_setup_rejects_bad_input(bad):
    from paper_1908_08666_amd import Mesh, _lib as L
    verts, lv, kw = W.kuhn6(), 3, dict(mu1=1.0)
    if bad == "level_low":
        lv = 1
    elif bad == "level_high":
        lv = 9                      # above the largest level (8)
    elif bad == "mixed":
        lv = [3, 3, 3, 3, 3, 4]
    elif bad == "degenerate":
        verts = W.unit_tet().copy()
        verts[0, 3] = verts[0, 1] + verts[0, 2]
    elif bad == "nan":
        kw = dict(mu1=float("nan"))
    if bad == "enum":
        md = L.MeshDesc(1, W.unit_tet().ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        np.array([3], np.int32).ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 7, 0)
        od = L.OpDesc(0, 0, 1, 0, 0, 0, 0)
        h = ctypes.c_void_p()
        assert L.lib().hhg_setup_macro(ctypes.byref(md), ctypes.byref(od), ctypes.byref(h)) == L.HHG_EINVAL
        return
    with pytest.raises(L.HHGError) as e:
        Mesh(verts, lv, **kw)
    assert e.value.code == L.HHG_EINVAL


def test_null_arguments():
    from paper_1908_08666_amd import _lib as L
    lib = L.lib()
    assert lib.hhg_setup_macro(None, None, None) == L.HHG_EINVAL
    assert lib.hhg_layout(None, None, None, None) == L.HHG_EINVAL
    assert lib.hhg_apply_scaled(None, 0, None, None, None, None) == L.HHG_EINVAL
    assert lib.hhg_residual(None, 0, 0, None, None, None, None, None) == L.HHG_EINVAL
    assert lib.hhg_destroy(None) == L.HHG_OK
    assert b"null" in lib.hhg_last_error()


_STRUCTS = {"hhg_mesh_desc": "MeshDesc", "hhg_op_desc": "OpDesc", "hhg_solve_opts": "SolveOpts",
            "hhg_solve_info": "SolveInfo", "hhg_carreau": "Carreau", "hhg_tune_report": "TuneReport",
            "hhg_train_opts": "TrainOpts", "hhg_mg_opts": "MgOpts", "hhg_stokes_opts": "StokesOpts",
            "hhg_picard_info": "PicardInfo", "hhg2d_mesh_desc": "MeshDesc2D"}


def declared_structs():
    """Field names, in order, of every typedef struct in the header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(hhg(?:2d)?_\w+)\s*;", text, re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            # "int32_t nu1, nu2" / "const double *xyz" / "int64_t counts[6]"
            first, *rest = [d.strip() for d in decl.split(",")]
            names = [re.findall(r"(\w+)\s*(?:\[[^\]]*\])?$", first)[0]]
            names += [re.findall(r"(\w+)\s*(?:\[[^\]]*\])?$", d.lstrip("*").strip())[0] for d in rest]
            fields += names
        out[name] = fields
    return out


def test_bindings_mirror_the_header_structs():
    """Every option/descriptor struct of the header has a ctypes mirror with
    the same fields in the same order (a missing or reordered field shifts
    every later one)."""
    from paper_1908_08666_amd import _lib as L
    structs = declared_structs()
    assert set(_STRUCTS) <= set(structs), sorted(structs)
    for cname, pyname in _STRUCTS.items():
        py = [f[0] for f in getattr(L, pyname)._fields_]
        assert py == structs[cname], (cname, py, structs[cname])


@pytest.mark.parametrize("name,level", [("triangle", 3), ("square", 4), ("cross", 3)])
def test_twod_layout_matches_oracle(name, level):
    """2-D handle (host setup only): slot count, coordinates, Dirichlet flags,
    one owner per distinct node and the unknown count against the 2-D
    oracle's mesh."""
    from scipy.spatial import cKDTree
    from oracle import twod as T2
    from paper_1908_08666_amd.twod import Mesh2D
    mu, lam = W.eform_weights()
    m = Mesh2D(W.twod_mesh(name), level, mu1=mu, lam1=lam)
    orc = T2.Mesh2D(W.twod_mesh(name), level)
    n = 1 << level
    assert m.n_nodes == len(W.twod_mesh(name)) * (n + 1) * (n + 2) // 2
    d, s2n = cKDTree(orc.xy).query(m.coords().T)
    assert d.max() < 1e-12
    fl = m.flags()
    assert np.array_equal((fl & 1).astype(bool), orc.dirichlet[s2n])
    assert np.array_equal(np.sort(s2n[(fl & 2) > 0]), np.arange(orc.n_nodes))
    assert m.n_unknown == int((~orc.dirichlet).sum())
    shared = np.bincount(s2n, minlength=orc.n_nodes) > 1
    assert np.array_equal((fl & 8) > 0, shared[s2n] & ~orc.dirichlet[s2n])
    m.close()


def test_twod_rejects_bad_setup():
    from paper_1908_08666_amd import _lib as L
    from paper_1908_08666_amd.twod import Mesh2D
    with pytest.raises(L.HHGError):
        Mesh2D(W.twod_mesh("square"), 14, mu1=1.0)
    with pytest.raises(L.HHGError):
        Mesh2D(np.array([[[0.0, 0.0], [1.0, 0.0], [2.0, 0.0]]]), 3, mu1=1.0)    # degenerate
