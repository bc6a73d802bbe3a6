"""GPU parity of the multigrid hierarchy (hhg_mg_*) against the oracle.

Transfers are compared node by node with the oracle's P and P^T; one V-cycle
with the oracle's V-cycle (same smoother, exact coarse solves); the
V-cycle-preconditioned CG with the sparse direct solution.  Tolerances:
prolongation 1e-15 (two terms per node), restriction 1e-13 (sums in another
order), V-cycle 1e-10 relative (the coarse solves are exact up to rounding
by different factorizations, amplified by the smoothing on the way up).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import multigrid as MG
from oracle import operators as O
from oracle.mesh import MacroMesh
from tests.helpers import slot_to_node, scatter, gather_consistent, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MU, LAM = W.eform_weights()
EFORM = dict(mu1=MU, lam1=LAM)

_cache = {}


def hierarchy(name, level, coarse=2, op=None, **variant):
    from paper_1908_08666_amd import Multigrid
    op = EFORM if op is None else op
    V = {"kuhn6": W.kuhn6(), "cube24": W.cube24()}[name]
    key = (name, level, coarse, tuple(sorted(op.items())), tuple(sorted(variant.items())))
    if key not in _cache:
        mg = Multigrid(V, level, coarse, **op, **variant)
        orcs = [MacroMesh(V, lev) for lev in range(coarse, level + 1)]
        s2n = [slot_to_node(m, o) for m, o in zip(mg.meshes, orcs)]
        _cache[key] = (mg, orcs, s2n, V)
    return _cache[key]


def consistent_random(orc, s2n, seed):
    x = W.uniform_vector(3 * orc.n_nodes, W.rng_for(7, seed)).reshape(-1, 3)
    x[orc.dirichlet] = 0.0
    return x, torch.from_numpy(scatter(x, s2n)).cuda()


def dof_vec(nodes, orc):
    return nodes[orc.unknown].ravel()


def node_vec(dofs, orc):
    out = np.zeros((orc.n_nodes, 3))
    out[orc.unknown] = dofs.reshape(-1, 3)
    return out


@pytest.mark.parametrize("name", ["kuhn6", "cube24"])
def test_transfers_match_oracle(name):
    mg, orcs, s2n, _ = hierarchy(name, 4 if name == "kuhn6" else 3)
    for q in range(1, len(orcs)):
        c, f = orcs[q - 1], orcs[q]
        lev = mg.coarse_level + q
        P = MG.prolongation(c, f)
        xc, xc_d = consistent_random(c, s2n[q - 1], 10 + q)
        xf = gather_consistent(mg.prolong(lev, xc_d).cpu().numpy(), s2n[q], f.n_nodes)
        ref = P @ xc
        u = f.unknown
        assert np.all(xf[f.dirichlet] == 0)
        assert rel_err(xf[u], ref[u]) <= 1e-15
        rf, rf_d = consistent_random(f, s2n[q], 20 + q)
        rc = gather_consistent(mg.restrict(lev, rf_d).cpu().numpy(), s2n[q - 1], c.n_nodes)
        refc = P.T @ rf
        uc = c.unknown
        assert np.all(rc[c.dirichlet] == 0)
        err = rel_err(rc[uc], refc[uc])
        print(f"  {name} level {lev}: restriction rel err {err:.2e}", flush=True)
        assert err <= 1e-13


@pytest.mark.parametrize("name,level", [("kuhn6", 4), ("cube24", 3)])
def test_vcycle_matches_oracle(name, level):
    mg, orcs, s2n, V = hierarchy(name, level)
    f = orcs[-1]
    k = W.exp_fourier_coefficient(f.xyz, W.rng_for(2, 0), 16, 1.0)
    H = MG.Hierarchy(V, mg.coarse_level, level, k, EFORM)
    mg.setup_coefficient(torch.from_numpy(scatter(k, s2n[-1])).cuda())
    # smoothing-step counts of both parities (the fused steps alternate
    # between two iterates), no pre- or no post-smoothing, variable cycles
    for seed, (nu1, nu2, omega, inc) in enumerate([(3, 3, 0.7, 0), (1, 2, 0.6, 0), (3, 3, 0.7, 2),
                                                   (0, 2, 0.7, 0), (2, 0, 0.7, 1)]):
        r, r_d = consistent_random(f, s2n[-1], 30 + seed)
        z = gather_consistent(mg.vcycle(r_d, nu1=nu1, nu2=nu2, omega=omega, nu_inc=inc).cpu().numpy(),
                              s2n[-1], f.n_nodes)
        ref = node_vec(MG.vcycle(H, dof_vec(r, f), nu1=nu1, nu2=nu2, omega=omega, nu_inc=inc), f)
        u = f.unknown
        assert np.all(z[f.dirichlet] == 0)
        err = rel_err(z[u], ref[u])
        print(f"  {name} level {level} V({nu1},{nu2}) omega {omega} +{inc} per coarser level: "
              f"rel err {err:.2e}", flush=True)
        assert err <= 1e-10


def test_mg_pcg_solves_and_is_level_robust():
    """Kuhn cube at levels 4 and 5 (coarsest level 2): V-cycle CG reaches
    1e-10 in a level-independent number of iterations; the level-4 solution
    matches the sparse direct solve of the oracle's operator."""
    its = {}
    for level in (4, 5):
        mg, orcs, s2n, V = hierarchy("kuhn6", level)
        f = orcs[-1]
        k = W.exp_fourier_coefficient(f.xyz, W.rng_for(2, 0), 16, 1.0)
        mg.setup_coefficient(torch.from_numpy(scatter(k, s2n[-1])).cuda())
        b, b_d = consistent_random(f, s2n[-1], 40 + level)
        x_d, info = mg.solve(b_d, rtol=1e-10, maxit=60)
        print(f"  level {level}: {info['iterations']} iterations, rel residual "
              f"{info['rel_residual']:.2e}", flush=True)
        assert info["status"] == "HHG_OK" and info["rel_residual"] <= 1e-10
        its[level] = info["iterations"]
        if level == 4:
            x = gather_consistent(x_d.cpu().numpy(), s2n[-1], f.n_nodes)
            A = O.reduce_dirichlet(f, O.operator_matrix(f, k, EFORM)).tocsc()
            xs = node_vec(spla.spsolve(A, dof_vec(b, f)), f)
            assert rel_err(x[f.unknown], xs[f.unknown]) <= 1e-8
    assert its[5] <= its[4] + 3, its
    assert its[5] <= 25, its


def test_invalid_arguments_rejected():
    from paper_1908_08666_amd import Multigrid
    from paper_1908_08666_amd._lib import HHGError
    with pytest.raises(HHGError):
        Multigrid(W.kuhn6(), 4, 5, **EFORM)          # coarse level above the finest
    with pytest.raises(HHGError):
        Multigrid(W.cube24(), 4, 3, **EFORM)         # coarse level too fine for the dense solve
    mg, orcs, s2n, _ = hierarchy("kuhn6", 4)
    r = torch.zeros((3, mg.meshes[-1].n_nodes), dtype=torch.float64, device="cuda")
    with pytest.raises(HHGError):
        mg.vcycle(r, nu1=0, nu2=0)
    with pytest.raises(HHGError):
        mg.vcycle(r, omega=2.5)
    with pytest.raises(HHGError):
        mg.vcycle(r, nu_inc=9)
    import ctypes
    from paper_1908_08666_amd import _lib as L
    o = L.MgOpts(3, 3, 0.7, 1e-8, 10, L.HHG_MG_CG, 7)      # unknown cycle precision
    z = torch.empty_like(r)
    ws = mg._workspace(r.device)
    assert mg._lib.hhg_mg_vcycle(mg._mg, ctypes.byref(o), ctypes.c_void_p(r.data_ptr()),
                                 ctypes.c_void_p(z.data_ptr()), ws, None) == L.HHG_EINVAL
    assert b"precision" in mg._lib.hhg_last_error()


def test_graph_replayed_cycles_match_eager_cycles(monkeypatch):
    """hhg_mg_solve replays one captured V-cycle per iteration; without the
    graph (HHG_NO_GRAPH) the same kernels run eagerly.  Both solves must give
    the same iterates bit for bit, with eager work between the runs."""
    mg, orcs, s2n, _ = hierarchy("kuhn6", 4)
    f = orcs[-1]
    k = W.exp_fourier_coefficient(f.xyz, W.rng_for(2, 3), 16, 1.0)
    mg.setup_coefficient(torch.from_numpy(scatter(k, s2n[-1])).cuda())
    b, b_d = consistent_random(f, s2n[-1], 77)
    runs = []
    for eager in (False, True, False):
        if eager:
            monkeypatch.setenv("HHG_NO_GRAPH", "1")
        else:
            monkeypatch.delenv("HHG_NO_GRAPH", raising=False)
        x_d, info = mg.solve(b_d, rtol=1e-9, maxit=60)
        runs.append((x_d.cpu().numpy(), info["iterations"]))
        _ = mg.vcycle(b_d)          # eager work between the solves
        torch.cuda.synchronize()
    for x, it in runs[1:]:
        assert it == runs[0][1]
        assert np.array_equal(x, runs[0][0])


def test_cycles_need_the_workspace_of_the_coefficient_setup():
    from paper_1908_08666_amd._lib import HHGError
    mg, orcs, s2n, _ = hierarchy("kuhn6", 4)
    f = orcs[-1]
    k = torch.from_numpy(scatter(W.exp_fourier_coefficient(f.xyz, W.rng_for(2, 0), 16, 1.0),
                                 s2n[-1])).cuda()
    mg.setup_coefficient(k)
    r = torch.ones((3, mg.meshes[-1].n_nodes), dtype=torch.float64, device="cuda")
    mg.vcycle(r)                      # the workspace of the setup: accepted
    old = mg._ws                      # kept alive, so the fresh workspace gets another address
    mg._ws = None                     # a fresh workspace without coefficient setup
    with pytest.raises(HHGError):
        mg.vcycle(r)
    with pytest.raises(HHGError):
        mg.solve(r)
    assert mg._ws.data_ptr() != old.data_ptr()
    mg.setup_coefficient(k)           # set up again on the new workspace
    mg.vcycle(r)


@pytest.mark.parametrize("method,iface,corr", [("onthefly", "symmetric", "physical"),
                                               ("scaled", "rowwise", "physical"),
                                               ("scaled", "symmetric", "none"),
                                               ("scaled", "zerosum", "physical")])
def test_vcycle_variants_match_oracle(method, iface, corr):
    """V-cycles for the nodal-integration operator, the row-wise interface
    rule (a non-symmetric matrix: the coarse solve pivots), the unphysical
    scaling and the zero-sum interface centre (whose smoother blocks are the
    zero-sum centres) against the oracle's cycle of the same operator; for
    the row-wise rule also the V-cycle iteration, for the zero-sum rule
    V-cycle CG, against the direct solve."""
    mg, orcs, s2n, V = hierarchy("kuhn6", 4, iface=iface, corr=corr)
    f = orcs[-1]
    k = W.exp_fourier_coefficient(f.xyz, W.rng_for(2, 5), 16, 1.0)
    H = MG.Hierarchy(V, mg.coarse_level, 4, k, EFORM,
                     method="nodal" if method == "onthefly" else "scaled",
                     **({} if method == "onthefly" else dict(iface=iface, corr=corr)))
    mg.setup_coefficient(torch.from_numpy(scatter(k, s2n[-1])).cuda(), method=method)
    r, r_d = consistent_random(f, s2n[-1], 60)
    z = gather_consistent(mg.vcycle(r_d).cpu().numpy(), s2n[-1], f.n_nodes)
    ref = node_vec(MG.vcycle(H, dof_vec(r, f)), f)
    err = rel_err(z[f.unknown], ref[f.unknown])
    print(f"  {method} {iface} {corr}: V-cycle rel err {err:.2e}", flush=True)
    assert err <= 1e-10
    if iface in ("rowwise", "zerosum"):
        x_d, info = mg.solve(r_d, rtol=1e-11, maxit=80, method="cycle" if iface == "rowwise" else "cg")
        assert info["status"] == "HHG_OK"
        x = gather_consistent(x_d.cpu().numpy(), s2n[-1], f.n_nodes)
        xs = node_vec(spla.spsolve(H.A[-1].tocsc(), dof_vec(r, f)), f)
        assert rel_err(x[f.unknown], xs[f.unknown]) <= 1e-8



@pytest.mark.parametrize("name,level,method,iface", [("kuhn6", 4, "scaled", "symmetric"),
                                                      ("cube24", 3, "scaled", "symmetric"),
                                                      ("kuhn6", 4, "onthefly", "symmetric"),
                                                      ("kuhn6", 4, "scaled", "rowwise")])
def test_fp32_vcycle_matches_oracle(name, level, method, iface):
    """An FP32 cycle (operator, smoother, transfers in FP32, coarse inverse
    FP64) against the oracle's FP64 cycle of the same operator.  Bound: FP32
    rounding (6e-8) of each apply, amplified by the cancellation in the
    residuals and by the smoothing steps of the levels (measured 1.1e-7 on
    the Kuhn cube at level 4); 2e-6 relative leaves room while a wrong term
    in any kernel, or an FP32 coarse inverse, gives far more."""
    mg, orcs, s2n, V = hierarchy(name, level, iface=iface)
    f = orcs[-1]
    k = W.exp_fourier_coefficient(f.xyz, W.rng_for(2, 0), 16, 1.0)
    H = MG.Hierarchy(V, mg.coarse_level, level, k, EFORM,
                     method="nodal" if method == "onthefly" else "scaled",
                     **({} if method == "onthefly" else dict(iface=iface)))
    mg.setup_coefficient(torch.from_numpy(scatter(k, s2n[-1])).cuda(), method=method)
    r, r_d = consistent_random(f, s2n[-1], 31)
    z = gather_consistent(mg.vcycle(r_d, precision="f32").cpu().numpy(), s2n[-1], f.n_nodes)
    ref = node_vec(MG.vcycle(H, dof_vec(r, f)), f)
    assert np.all(z[f.dirichlet] == 0)
    err = rel_err(z[f.unknown], ref[f.unknown])
    print(f"  {name} level {level} {method} {iface}: FP32 V(3,3) rel err {err:.2e}", flush=True)
    assert err <= 2e-6


@pytest.mark.parametrize("method", ["cg", "cycle"])
def test_fp32_cycles_reach_fp64_accuracy(method):
    """With FP32 cycles the outer iteration keeps its FP64 residuals, so the
    solve still reaches 1e-10 and the direct solution, in about as many
    iterations as with FP64 cycles."""
    mg, orcs, s2n, V = hierarchy("kuhn6", 4)
    f = orcs[-1]
    k = W.exp_fourier_coefficient(f.xyz, W.rng_for(2, 0), 16, 1.0)
    mg.setup_coefficient(torch.from_numpy(scatter(k, s2n[-1])).cuda())
    b, b_d = consistent_random(f, s2n[-1], 44)
    its = {}
    for prec in ("f64", "f32"):
        x_d, info = mg.solve(b_d, rtol=1e-10, maxit=80, method=method, precision=prec)
        print(f"  {method} {prec}: {info['iterations']} iterations, rel residual "
              f"{info['rel_residual']:.2e}", flush=True)
        assert info["status"] == "HHG_OK" and info["rel_residual"] <= 1e-10
        its[prec] = info["iterations"]
    x = gather_consistent(x_d.cpu().numpy(), s2n[-1], f.n_nodes)
    A = O.reduce_dirichlet(f, O.operator_matrix(f, k, EFORM)).tocsc()
    xs = node_vec(spla.spsolve(A, dof_vec(b, f)), f)
    assert rel_err(x[f.unknown], xs[f.unknown]) <= 1e-8
    assert its["f32"] <= its["f64"] + 2, its


def test_full_size_cycle_properties():
    """The hierarchy of the level-7 benchmark (6-macro cube, levels 2..7),
    where the oracle cannot run, checked through properties that hold at any
    size: the FP64 cycle is linear; under the symmetric interface rule with
    nu1 = nu2 it is a symmetric positive definite operator (the V-cycle of a
    symmetric smoother with P^T restriction and an exact coarse solve); the
    FP32 cycle stays within FP32 rounding of it; and the CG it preconditions
    reaches 1e-8 in a level-robust number of iterations, with the residual
    recomputed by an independent apply of a separate level-7 handle."""
    from paper_1908_08666_amd import Mesh, Multigrid
    level = 7
    mg = Multigrid(W.kuhn6(), level, 2, **EFORM)
    mesh = Mesh(W.kuhn6(), level, **EFORM)
    try:
        f = mg.meshes[-1]
        fl = torch.from_numpy(f.flags()).cuda()
        own = (fl & 3) == 2
        xyz = f.coords().T
        k = torch.from_numpy(W.exp_fourier_coefficient(xyz, W.rng_for(2, 0), 16, 1.0)).cuda()
        mg.setup_coefficient(k)

        v = torch.from_numpy(W.consistent_uniform(xyz, (f.flags() & 2) > 0, W.rng_for(8, 1), 6)).cuda()
        v[:, (fl & 1) > 0] = 0.0
        r1, r2 = v[:3].contiguous(), v[3:].contiguous()

        def dot(a, b):
            return float((a[:, own] * b[:, own]).sum())

        z1, z2 = mg.vcycle(r1), mg.vcycle(r2)
        z12 = mg.vcycle(r1 + 2.0 * r2)
        lin = float(torch.linalg.norm(z12 - z1 - 2.0 * z2) / torch.linalg.norm(z12))
        sym = abs(dot(r1, z2) - dot(r2, z1)) / abs(dot(r1, z2))
        print(f"  level 7 V(3,3): linearity {lin:.2e}, symmetry {sym:.2e}", flush=True)
        assert lin <= 1e-12
        assert sym <= 1e-10
        assert dot(r1, z1) > 0 and dot(r2, z2) > 0
        z32 = mg.vcycle(r1, precision="f32")
        d32 = float(torch.linalg.norm(z32 - z1) / torch.linalg.norm(z1))
        print(f"  level 7 FP32 cycle vs FP64 cycle: {d32:.2e}", flush=True)
        assert d32 <= 2e-6          # FP32 rounding through the cycle (measured 1.7e-7)
        b = r1
        for prec in ("f64", "f32"):
            x, info = mg.solve(b, rtol=1e-8, maxit=40, precision=prec)
            res = mesh.residual(b, x, k)
            rel = float(torch.linalg.norm(res[:, own]) / torch.linalg.norm(b[:, own]))
            print(f"  level 7 MG-PCG {prec}: {info['iterations']} iterations, independent residual "
                  f"{rel:.2e}", flush=True)
            assert info["status"] == "HHG_OK" and info["iterations"] <= 20
            assert rel <= 1.01e-8
    finally:
        mg.close()
        mesh.close()
