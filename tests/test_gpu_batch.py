"""Batched independent problems of uneven level in one interior launch:
parity with the CPU oracle, invariance of the results under the tuning
(slab depth per level, per-item or persistent grid) and HIP-graph replay.

The workload is the batched one: independent unit macro-tets, levels drawn
uniformly from 3..6, each with its own seeded coefficient k = exp(g_p),
E-form elasticity, homogeneous Dirichlet data on every macro boundary (so
every unknown row is a macro-interior row)."""
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
TOL = {torch.float64: 1e-12, torch.float32: 1e-5}

_cache = {}


def batch_case(n_problems, levels):
    from paper_1908_08666_amd import Mesh
    key = (n_problems, tuple(levels))
    if key not in _cache:
        V = np.repeat(W.unit_tet(), n_problems, axis=0)
        lib = Mesh(V, levels, coupling="independent", **EFORM)
        orc = MacroMesh(V, levels, coupling="independent")
        s2n = slot_to_node(lib, orc)
        k = np.empty(orc.n_nodes)
        for m, km in enumerate(W.batch_coefficients(orc.local_xyz)):
            k[orc.gid[m]] = km
        x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(4, 3)).reshape(-1, 3)
        _cache[key] = (lib, orc, s2n, k, x)
    return _cache[key]


def gpu_apply(lib, s2n, x, k, dtype):
    xt = torch.from_numpy(scatter(x, s2n)).to("cuda", dtype)
    kt = torch.from_numpy(scatter(k, s2n)).to("cuda", dtype)
    return xt, kt


def oracle_ref(orc, k, x, dtype, rows=None):
    if dtype == torch.float32:
        x = x.astype(np.float32).astype(np.float64)
        k = k.astype(np.float32).astype(np.float64)
    return O.apply(orc, k, EFORM, x, rows=rows)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_uneven_levels_parity_and_tuning_invariance(dtype):
    """12 problems of levels 3..5 (full oracle) and every tuning shape."""
    levels = [3, 4, 5, 4, 3, 5, 5, 3, 4, 4, 5, 3]
    lib, orc, s2n, k, x = batch_case(len(levels), levels)
    xt, kt = gpu_apply(lib, s2n, x, k, dtype)
    lib.set_tuning()                                   # defaults
    y0 = lib.apply_scaled(xt, kt)
    torch.cuda.synchronize()
    y_nodes = gather_consistent(y0.double().cpu().numpy(), s2n, orc.n_nodes)
    ref = oracle_ref(orc, k, x, dtype)
    u = orc.unknown
    err = rel_err(y_nodes[u], ref[u])
    print(f"  batch of 12, {dtype}: rel err {err:.3e}", flush=True)
    assert err <= TOL[dtype]
    assert np.all(y_nodes[orc.dirichlet] == 0)
    # tuning moves rows between workgroups only: bitwise identical results
    for slabs, grid in (([1, 1, 1], 0), ([2, 8, 32], 0), ([64, 64, 64], 0), ([4, 4, 4], 256),
                        ([1, 2, 4], 8), ([8, 1, 16], 1024), ([-1, -1, -1], 0), ([-1, 2, -1], 16)):
        lib.set_tuning(levels=[3, 4, 5], slabs=slabs, persist_blocks=grid)
        y1 = lib.apply_scaled(xt, kt)
        torch.cuda.synchronize()
        assert torch.equal(y0, y1), (slabs, grid)
    y_auto, rep = lib.autotune(xt, kt, reps=3)
    torch.cuda.synchronize()
    print(f"  autotune: {rep}", flush=True)
    assert [lv["level"] for lv in rep["levels"]] == [3, 4, 5]
    assert torch.equal(y0, y_auto)
    assert torch.equal(y0, lib.apply_scaled(xt, kt))
    lib.set_tuning()


def test_batch256_full_size_sampled_rows():
    """The full batched workload: 256 problems, levels uniform in 3..6
    (about 3.5 M slots), after autotuning in FP32; sampled rows of every
    level recomputed by the oracle, FP64 and FP32."""
    levels = W.batch_levels(256)
    lib, orc, s2n, k, x = batch_case(256, levels.tolist())
    rng = np.random.default_rng(21)
    u = orc.unknown
    rows = np.unique(rng.choice(u, 1200, replace=False))
    x32, k32 = gpu_apply(lib, s2n, x, k, torch.float32)
    _, rep = lib.autotune(x32, k32, reps=3)
    print(f"  autotune: {rep}", flush=True)
    assert sorted(lv["level"] for lv in rep["levels"]) == sorted(set(levels.tolist()))
    for dtype in (torch.float64, torch.float32):
        xt, kt = gpu_apply(lib, s2n, x, k, dtype)
        y = lib.apply_scaled(xt, kt)
        torch.cuda.synchronize()
        y = gather_consistent(y.double().cpu().numpy(), s2n, orc.n_nodes)
        ref = oracle_ref(orc, k, x, dtype, rows=rows)
        err = rel_err(y[rows], ref[rows])
        print(f"  batch256 sampled rows {dtype}: {err:.3e}", flush=True)
        assert err <= TOL[dtype]
    lib.set_tuning()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_graph_replay_matches_eager(dtype):
    """Captured applies replayed several times, with eager library and torch
    work between the replays; every replay equals the eager result."""
    levels = [3, 4, 5, 4, 3, 5, 5, 3, 4, 4, 5, 3]
    lib, orc, s2n, k, x = batch_case(len(levels), levels)
    xt, kt = gpu_apply(lib, s2n, x, k, dtype)
    ref = lib.apply_scaled(xt, kt)
    torch.cuda.synchronize()
    y = torch.full_like(xt, float("nan"))
    gid = lib.graph_create(xt, kt, y, count=3)
    try:
        other = torch.empty_like(xt)
        for rep in range(4):
            y.fill_(float("nan"))
            torch.cuda.synchronize()
            lib.graph_launch(gid)
            torch.cuda.synchronize()
            assert torch.equal(y, ref), rep
            # eager work between replays
            lib.apply_scaled(xt * 2, kt, other)
            torch.cuda.synchronize()
            assert torch.allclose(other, 2 * ref, rtol=1e-5 if dtype == torch.float32 else 1e-12,
                                  atol=1e-5 if dtype == torch.float32 else 1e-12)
    finally:
        lib.graph_destroy(gid)
    from paper_1908_08666_amd._lib import HHGError
    with pytest.raises(HHGError):
        lib.graph_launch(gid)
