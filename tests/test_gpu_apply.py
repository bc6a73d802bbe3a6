"""GPU parity of the operator applications against the CPU oracle.

Every case builds the same macro mesh in the HIP library and in the oracle,
draws seeded nodal inputs, applies the operator on the GPU through the C ABI
and compares with the oracle's sparse apply element by element.  Tolerances:
relative 2-norm error <= 1e-12 in FP64 and <= 1e-5 in FP32 (FP32 inputs are
the FP32-rounded FP64 inputs, fed to the oracle as well).
"""
import numpy as np
import pytest

import workloads as W
from oracle import operators as O
from oracle.mesh import MacroMesh
from tests.helpers import slot_to_node, scatter, gather_consistent, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MU, LAM = W.eform_weights()
EFORM = dict(mu1=MU, lam1=LAM)
LAME1 = dict(mu0=1.0, lam1=1.0)       # mu = 1 (unscaled), lambda = k
EPS = dict(mu1=1.0)                   # 2 nu (eps, eps), nu = k
TOL = {torch.float64: 1e-12, torch.float32: 1e-5}

_cache = {}


def setup_case(verts, levels, op, coupling="conforming", dirichlet="outer", **variant):
    from paper_1908_08666_amd import Mesh
    key = (verts.tobytes(), tuple(np.atleast_1d(levels)), tuple(sorted(op.items())), coupling,
           dirichlet, tuple(sorted(variant.items())))
    if key not in _cache:
        lib = Mesh(verts, levels, coupling=coupling, dirichlet=dirichlet, **op, **variant)
        orc = MacroMesh(verts, levels, coupling=coupling, dirichlet=dirichlet)
        _cache[key] = (lib, orc, slot_to_node(lib, orc))
    return _cache[key]


def run_apply(lib, s2n, x_nodes, k_nodes, dtype, method="scaled", f_nodes=None):
    dev = "cuda"
    x = torch.from_numpy(scatter(x_nodes, s2n)).to(dev, dtype)
    k = torch.from_numpy(scatter(k_nodes, s2n)).to(dev, dtype)
    if f_nodes is not None:
        f = torch.from_numpy(scatter(f_nodes, s2n)).to(dev, dtype)
        y = lib.residual(f, x, k, method=method)
    elif method == "scaled":
        y = lib.apply_scaled(x, k)
    else:
        y = lib.apply_onthefly(x, k)
    torch.cuda.synchronize()
    return y.double().cpu().numpy()


def oracle_apply(orc, k, op, x, method, dtype, **variant):
    if dtype == torch.float32:
        x = x.astype(np.float32).astype(np.float64)
        k = k.astype(np.float32).astype(np.float64)
    return O.apply(orc, k, op, x, method="scaled" if method == "scaled" else "nodal", **variant)


def check(lib, orc, s2n, k, op, x, dtype, method="scaled", **variant):
    y = gather_consistent(run_apply(lib, s2n, x, k, dtype, method), s2n, orc.n_nodes)
    ref = oracle_apply(orc, k, op, x, method, dtype, **variant)
    u = orc.unknown
    assert np.all(y[orc.dirichlet] == 0)
    err = rel_err(y[u], ref[u])
    print(f"  {method} {dtype} rel err {err:.3e}", flush=True)
    assert err <= TOL[dtype], err
    return err


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("method", ["scaled", "onthefly"])
def test_unit_tet_level4_ten_inputs(dtype, method):
    """Single reference macro at level 4 (969 nodes), mu = 1, lambda = k with
    k = 1 + 0.5 sin sin sin; ten seeded inputs x ~ U(-1, 1)."""
    lib, orc, s2n = setup_case(W.unit_tet(), 4, LAME1)
    k = W.sine_coefficient(orc.xyz)
    for seed in range(10):
        x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(1, 100 + seed)).reshape(-1, 3)
        check(lib, orc, s2n, k, LAME1, x, dtype, method)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("iface", ["symmetric", "rowwise", "zerosum"])
def test_kuhn6_multi_macro(dtype, iface):
    """Six conforming macros (cube), interface rows summed over copies."""
    lib, orc, s2n = setup_case(W.kuhn6(), 3, EFORM, iface=iface)
    k = W.exp_fourier_coefficient(orc.xyz, W.rng_for(2, 0), 16, 1.0)
    x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(2, 1)).reshape(-1, 3)
    check(lib, orc, s2n, k, EFORM, x, dtype, "scaled", iface=iface)
    check(lib, orc, s2n, k, EFORM, x, dtype, "onthefly")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_cube24_eps_operator(dtype):
    """24 congruent macros around the cube centre, 2 nu (eps, eps)."""
    lib, orc, s2n = setup_case(W.cube24(), 3, EPS)
    k = W.exp_fourier_coefficient(orc.xyz, W.rng_for(3, 0), 8, 1.5)
    x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(3, 1)).reshape(-1, 3)
    check(lib, orc, s2n, k, EPS, x, dtype, "scaled")
    check(lib, orc, s2n, k, EPS, x, dtype, "onthefly")


def test_cube24_zerosum_rule():
    """Zero-sum interface centre on 24 macros (edges shared by up to six
    macros, the cube centre by all 24), with an unscaled part of the form."""
    lib, orc, s2n = setup_case(W.cube24(), 3, LAME1, iface="zerosum")
    k = W.exp_fourier_coefficient(orc.xyz, W.rng_for(3, 2), 8, 1.5)
    x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(3, 3)).reshape(-1, 3)
    check(lib, orc, s2n, k, LAME1, x, torch.float64, "scaled", iface="zerosum")


@pytest.mark.parametrize("op,dtype", [("lame1", torch.float64), ("lame1", torch.float32),
                                      ("eform", torch.float64)])
def test_unit_tet_level6_all_faces_tiled(op, dtype):
    """One macro at level 6 (47,905 nodes) without Dirichlet nodes: all four
    faces are macro-boundary faces, each cut into several 32 x 8 tiles of
    deep rows in both face directions, with the rim of each face, the edges
    and the vertices on the listed-row path.  Full scaled and on-the-fly
    applies against the oracle, with (mu = 1) and without (E-form) an
    unscaled part of the form."""
    opd = {"lame1": LAME1, "eform": EFORM}[op]
    lib, orc, s2n = setup_case(W.unit_tet(), 6, opd, dirichlet="none")
    k = W.sine_coefficient(orc.xyz) + 0.2
    x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(1, 600)).reshape(-1, 3)
    check(lib, orc, s2n, k, opd, x, dtype, "scaled")
    check(lib, orc, s2n, k, opd, x, dtype, "onthefly")


@pytest.mark.parametrize("variant", [dict(corr="none"), dict(khat="edge")])
def test_variants(variant):
    lib, orc, s2n = setup_case(W.kuhn6(), 3, EFORM, **variant)
    k = W.exp_fourier_coefficient(orc.xyz, W.rng_for(2, 2), 16, 1.0)
    x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(2, 3)).reshape(-1, 3)
    check(lib, orc, s2n, k, EFORM, x, torch.float64, "scaled", **variant)


def test_residual_and_neumann():
    """r = f - A x, also for a pure Neumann operator (no Dirichlet nodes: the
    outer faces become macro-boundary rows)."""
    for dirichlet in ("outer", "none"):
        lib, orc, s2n = setup_case(W.kuhn6(), 3, LAME1, dirichlet=dirichlet)
        k = W.sine_coefficient(orc.xyz) + 0.2
        x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(2, 4)).reshape(-1, 3)
        f = W.uniform_vector(3 * orc.n_nodes, W.rng_for(2, 5)).reshape(-1, 3)
        for method in ("scaled", "onthefly"):
            r = gather_consistent(run_apply(lib, s2n, x, k, torch.float64, method, f_nodes=f),
                                  s2n, orc.n_nodes)
            ref = f - O.apply(orc, k, LAME1, x, method="scaled" if method == "scaled" else "nodal")
            ref[orc.dirichlet] = 0
            u = orc.unknown
            assert rel_err(r[u], ref[u]) < 1e-12
            assert np.all(r[orc.dirichlet] == 0)


def test_independent_uneven_levels():
    """Independent macros of levels 2..5 (the minimum level has one interior
    node per macro) in one launch."""
    rng = np.random.default_rng(7)
    V = np.concatenate([W.unit_tet(), W.unit_tet() * 2.0, W.kuhn6()[:2]])
    V = V + rng.normal(scale=0.05, size=V.shape)
    levels = [2, 3, 4, 5]
    lib, orc, s2n = setup_case(V, levels, EFORM, coupling="independent")
    k = np.exp(0.5 * np.sin(3 * orc.xyz).sum(1))
    x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(4, 9)).reshape(-1, 3)
    for dtype in (torch.float64, torch.float32):
        check(lib, orc, s2n, k, EFORM, x, dtype, "scaled")
        check(lib, orc, s2n, k, EFORM, x, dtype, "onthefly")


def test_dirichlet_entries_of_x_ignored():
    lib, orc, s2n = setup_case(W.unit_tet(), 4, LAME1)
    k = W.sine_coefficient(orc.xyz)
    x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(1, 50)).reshape(-1, 3)
    x2 = x.copy()
    x2[orc.dirichlet] = 1e6
    a = run_apply(lib, s2n, x, k, torch.float64)
    b = run_apply(lib, s2n, x2, k, torch.float64)
    assert np.array_equal(a, b)


def test_bitwise_reproducible():
    lib, orc, s2n = setup_case(W.kuhn6(), 3, EFORM)
    k = W.exp_fourier_coefficient(orc.xyz, W.rng_for(2, 0), 16, 1.0)
    x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(2, 1)).reshape(-1, 3)
    a = run_apply(lib, s2n, x, k, torch.float64)
    b = run_apply(lib, s2n, x, k, torch.float64)
    assert np.array_equal(a, b)


def test_full_size_kuhn6_level7_sampled_rows():
    """The benchmarked workload: 6 macros at level 7 (2,146,689 nodes),
    k = exp(g), E-form.  2000 sampled rows (interior, face, edge and vertex
    rows included) are recomputed by the oracle one by one."""
    lib, orc, s2n = setup_case(W.kuhn6(), 7, EFORM)
    k = W.exp_fourier_coefficient(orc.xyz, W.rng_for(2, 0), 16, 1.0)
    x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(2, 1)).reshape(-1, 3)
    rng = np.random.default_rng(11)
    u = orc.unknown
    iface = u[orc.interface[u]]
    rows = np.unique(np.concatenate([rng.choice(u, 1500, replace=False),
                                     rng.choice(iface, 500, replace=False)]))
    for dtype in (torch.float64, torch.float32):
        y = gather_consistent(run_apply(lib, s2n, x, k, dtype), s2n, orc.n_nodes)
        ref = oracle_apply(orc, k, EFORM, x, "scaled", dtype, rows=rows)
        err = rel_err(y[rows], ref[rows])
        print(f"  level-7 sampled rows {dtype}: {err:.3e}", flush=True)
        assert err <= TOL[dtype]


def test_full_size_cube24_level7_sampled_rows():
    """24 macros at level 7 (8,787,480 slots): the largest single-mesh case.
    Sampled unknown rows, half of them on macro interfaces where up to 24
    copies meet, recomputed by the oracle one by one."""
    lib, orc, s2n = setup_case(W.cube24(), 7, dict(mu1=1.0))
    k = W.exp_fourier_coefficient(orc.xyz, W.rng_for(3, 0), 8, 1.5)
    x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(3, 1)).reshape(-1, 3)
    rng = np.random.default_rng(12)
    u = orc.unknown
    iface = u[orc.interface[u]]
    rows = np.unique(np.concatenate([rng.choice(u, 400, replace=False),
                                     rng.choice(iface, 400, replace=False)]))
    y = gather_consistent(run_apply(lib, s2n, x, k, torch.float64), s2n, orc.n_nodes)
    ref = oracle_apply(orc, k, dict(mu1=1.0), x, "scaled", torch.float64, rows=rows)
    err = rel_err(y[rows], ref[rows])
    print(f"  cube24 level-7 sampled rows: {err:.3e}", flush=True)
    assert err <= TOL[torch.float64]


def test_unit_tet_level8_sampled_rows():
    """The largest level the library accepts: one macro at level 8 (257
    points per edge, 2,862,209 nodes; the window of a 256-position chunk
    needs up to 6 entries per thread).  Sampled rows of the scaled and the
    on-the-fly operator in FP64 and FP32 against the oracle."""
    lib, orc, s2n = setup_case(W.unit_tet(), 8, EFORM)
    k = W.exp_fourier_coefficient(orc.xyz, W.rng_for(2, 0), 16, 1.0)
    x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(2, 1)).reshape(-1, 3)
    rows = np.unique(np.random.default_rng(13).choice(orc.unknown, 1000, replace=False))
    for method in ("scaled", "onthefly"):
        ref = oracle_apply(orc, k, EFORM, x, method, torch.float64, rows=rows)
        ref32 = oracle_apply(orc, k, EFORM, x, method, torch.float32, rows=rows)
        for dtype, want in ((torch.float64, ref), (torch.float32, ref32)):
            y = gather_consistent(run_apply(lib, s2n, x, k, dtype, method), s2n, orc.n_nodes)
            err = rel_err(y[rows], want[rows])
            print(f"  level-8 sampled rows {method} {dtype}: {err:.3e}", flush=True)
            assert err <= TOL[dtype]


@pytest.mark.parametrize("env", [dict(HHG_PLANES_PER_ITEM="1"), dict(HHG_PLANES_PER_ITEM="2"),
                                 dict(HHG_PLANES_PER_ITEM="7"), dict(HHG_SERIAL_APPLY="1")])
def test_environment_switches_bitwise(env, monkeypatch):
    """The slab depth override and the one-stream apply (read when a handle
    is set up) move rows between workgroups and streams only: the apply of
    both operators is bitwise the default handle's, which the oracle checks."""
    from paper_1908_08666_amd import Mesh
    orc = MacroMesh(W.kuhn6(), 5)
    k = W.exp_fourier_coefficient(orc.xyz, W.rng_for(2, 0), 16, 1.0)
    x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(2, 1)).reshape(-1, 3)
    base = Mesh(W.kuhn6(), 5, **EFORM)
    for name, val in env.items():
        monkeypatch.setenv(name, val)
    other = Mesh(W.kuhn6(), 5, **EFORM)
    for name in env:
        monkeypatch.delenv(name)
    s2n = slot_to_node(base, orc)
    for method in ("scaled", "onthefly"):
        for dtype in (torch.float64, torch.float32):
            a = run_apply(base, s2n, x, k, dtype, method)
            b = run_apply(other, s2n, x, k, dtype, method)
            assert np.array_equal(a, b), (env, method, dtype)
    y = gather_consistent(run_apply(other, s2n, x, k, torch.float64), s2n, orc.n_nodes)
    ref = oracle_apply(orc, k, EFORM, x, "scaled", torch.float64)
    assert rel_err(y[orc.unknown], ref[orc.unknown]) <= TOL[torch.float64]
