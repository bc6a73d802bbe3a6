"""GPU parity of the generalized Stokes terms and solvers (Sec. 5.2)
against the oracle: the divergence pair, the stabilization and the lumped
mass entry by entry; inexact Uzawa iterates step by step and its converged
solution against the bordered direct solve; the Carreau fixed-point
iteration against the oracle's."""
import numpy as np
import pytest

import workloads as W
from oracle import multigrid as MG
from oracle import operators as O
from oracle import stokes as ST
from oracle.mesh import MacroMesh
from tests.helpers import slot_to_node, scatter, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pressure_gather(v, s2n, n):
    out = np.full(n, np.nan)
    out[s2n] = v
    assert np.array_equal(out[s2n], v), "copies of a pressure node differ"
    return out


def _vel_gather(v, s2n, n):
    out = np.full((n, 3), np.nan)
    out[s2n] = v.T
    assert np.array_equal(out[s2n], v.T), "copies of a velocity node differ"
    return out


@pytest.mark.parametrize("name,level", [("kuhn6", 3), ("cube24", 2), ("kuhn6", 5)])
def test_terms_match_oracle(name, level):
    from paper_1908_08666_amd import Mesh
    V = W.kuhn6() if name == "kuhn6" else W.cube24()
    lib = Mesh(V, level, mu1=1.0)
    orc = MacroMesh(V, level)
    s2n = slot_to_node(lib, orc)
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, (orc.n_nodes, 3))
    p = rng.uniform(-1, 1, orc.n_nodes)
    dof = O.unknown_dofs(orc)
    B = ST.divergence_matrix(orc)
    h = ST.mesh_width(level)
    ut = torch.from_numpy(scatter(u, s2n)).cuda()
    pt = torch.from_numpy(scatter(p, s2n)).cuda()
    # B u with Dirichlet velocities read as zero
    uz = u.copy()
    uz[orc.dirichlet] = 0.0
    want = B @ uz.ravel()
    got = _pressure_gather(lib.stokes_rows("div", ut).cpu().numpy(), s2n, orc.n_nodes)
    assert rel_err(got, want) <= 1e-13
    # B^T p on unknown rows, zero at Dirichlet nodes
    want = np.zeros(3 * orc.n_nodes)
    want[dof] = B[:, dof].T @ p
    got = _vel_gather(lib.stokes_rows("grad", pt).cpu().numpy(), s2n, orc.n_nodes)
    assert rel_err(got.ravel(), want) <= 1e-13
    assert np.all(got[orc.dirichlet] == 0)
    want = ST.stabilization_matrix(orc, h) @ p
    got = _pressure_gather(lib.stokes_rows("stab", pt, hl=h).cpu().numpy(), s2n, orc.n_nodes)
    assert rel_err(got, want) <= 1e-13
    got = _pressure_gather(lib.stokes_rows("mass").cpu().numpy(), s2n, orc.n_nodes)
    assert rel_err(got, ST.lumped_mass(orc)) <= 1e-14
    torch.cuda.synchronize()


def _shear_force(mesh, amp=100.0):
    x = mesh.xyz
    f = np.column_stack([amp * np.sin(np.pi * x[:, 1]), np.zeros(mesh.n_nodes),
                         amp * np.sin(np.pi * x[:, 0])])
    f = f * ST.lumped_mass(mesh)[:, None]
    f[mesh.dirichlet] = 0.0
    return f


def _setup(level, coarse=2):
    from paper_1908_08666_amd import Multigrid
    mg = Multigrid(W.kuhn6(), level, coarse, mu1=1.0)
    orc = MacroMesh(W.kuhn6(), level)
    s2n = slot_to_node(mg.meshes[-1], orc)
    return mg, orc, s2n


def test_uzawa_matches_oracle():
    """Five inexact Uzawa steps (same V(3,3) cycle, same pressure step) agree
    with the oracle's, then the solve to 1e-9 meets the direct solution."""
    L = 4
    mg, orc, s2n = _setup(L)
    mu = 0.5 + W.exp_fourier_coefficient(orc.xyz, W.rng_for(6, 0), 8, 0.5)
    f = _shear_force(orc)
    mut = torch.from_numpy(scatter(mu, s2n)).cuda()
    ft = torch.from_numpy(scatter(f, s2n)).cuda()
    mg.setup_coefficient(mut)
    u, p, info = mg.stokes_solve(ft, mut, rtol=0.0, maxit=5, raise_on_status=False)
    torch.cuda.synchronize()
    assert info["iterations"] == 5 and info["status"] == "HHG_ENOCONV"
    H = MG.Hierarchy(W.kuhn6(), 2, L, mu, dict(mu1=1.0))
    dof = O.unknown_dofs(orc)
    uo, po, it, hist = ST.inexact_uzawa(H, orc, mu, f.ravel()[dof], rtol=0.0, maxit=5)
    ug = _vel_gather(u.cpu().numpy(), s2n, orc.n_nodes).ravel()[dof]
    pg = _pressure_gather(p.cpu().numpy(), s2n, orc.n_nodes)
    print(f"  5 Uzawa steps: u {rel_err(ug, uo):.2e}, p {rel_err(pg, po):.2e}; "
          f"residual {info['rel_residual']:.3e} vs {hist[-1]:.3e}", flush=True)
    assert rel_err(ug, uo) <= 1e-9 and rel_err(pg, po) <= 1e-9
    assert abs(info["rel_residual"] - hist[-1]) <= 1e-9 * hist[-1]
    u, p, info = mg.stokes_solve(ft, mut, u=u, p=p, rtol=1e-9, maxit=800)
    torch.cuda.synchronize()
    K, _ = ST.saddle_matrix(orc, H.A[-1], ST.mesh_width(L))
    z = ST.solve_saddle(K, np.concatenate([f.ravel()[dof], np.zeros(orc.n_nodes)]), dof.size,
                        ST.lumped_mass(orc))
    ug = _vel_gather(u.cpu().numpy(), s2n, orc.n_nodes).ravel()[dof]
    pg = _pressure_gather(p.cpu().numpy(), s2n, orc.n_nodes)
    print(f"  Uzawa to 1e-9 in {info['iterations']} steps: u {rel_err(ug, z[:dof.size]):.2e}, "
          f"p {rel_err(pg, z[dof.size:]):.2e}", flush=True)
    assert info["status"] == "HHG_OK"
    assert rel_err(ug, z[:dof.size]) <= 1e-6 and rel_err(pg, z[dof.size:]) <= 1e-5


def test_uzawa_with_the_papers_cycle_settings():
    """The paper's settings of Sec. 5.2.1: variable V(3,3) cycles (two more
    smoothing steps per coarser level) and pressure relaxation 0.3.  Five
    steps agree with the oracle's, and the solve converges to 1e-8."""
    L = 4
    mg, orc, s2n = _setup(L)
    mu = 0.5 + W.exp_fourier_coefficient(orc.xyz, W.rng_for(6, 0), 8, 0.5)
    f = _shear_force(orc)
    mut = torch.from_numpy(scatter(mu, s2n)).cuda()
    ft = torch.from_numpy(scatter(f, s2n)).cuda()
    mg.setup_coefficient(mut)
    u, p, info = mg.stokes_solve(ft, mut, rtol=0.0, maxit=5, omega_p=0.3, nu_inc=2,
                                 raise_on_status=False)
    torch.cuda.synchronize()
    H = MG.Hierarchy(W.kuhn6(), 2, L, mu, dict(mu1=1.0))
    dof = O.unknown_dofs(orc)
    uo, po, it, hist = ST.inexact_uzawa(H, orc, mu, f.ravel()[dof], rtol=0.0, maxit=5, omega_p=0.3,
                                        nu_inc=2)
    ug = _vel_gather(u.cpu().numpy(), s2n, orc.n_nodes).ravel()[dof]
    pg = _pressure_gather(p.cpu().numpy(), s2n, orc.n_nodes)
    print(f"  5 Uzawa steps, variable cycle, omega_p 0.3: u {rel_err(ug, uo):.2e}, "
          f"p {rel_err(pg, po):.2e}", flush=True)
    assert rel_err(ug, uo) <= 1e-9 and rel_err(pg, po) <= 1e-9
    assert abs(info["rel_residual"] - hist[-1]) <= 1e-9 * hist[-1]
    steps = {}
    for name, kw in (("fixed, omega_p 1", dict()), ("variable, omega_p 0.3", dict(omega_p=0.3, nu_inc=2)),
                     ("variable, omega_p 1", dict(nu_inc=2))):
        _, _, inf = mg.stokes_solve(ft, mut, rtol=1e-8, maxit=800, **kw)
        torch.cuda.synchronize()
        steps[name] = inf["iterations"]
    print(f"  Uzawa steps to 1e-8: {steps}", flush=True)


@pytest.mark.parametrize("method", ["scaled", "onthefly"])
def test_picard_matches_oracle(method):
    """Carreau fixed-point iteration (Alg. fixedpoint_mg) on the 6-macro cube
    at level 3: same number of fixed-point steps as the oracle, same final
    velocity, pressure and viscosity within the accumulated rounding."""
    L = 3
    mg, orc, s2n = _setup(L)
    f = _shear_force(orc)
    law = dict(eta0=1.0, eta_inf=1e-3, kappa=1.0, r=-0.25)
    ft = torch.from_numpy(scatter(f, s2n)).cuda()
    u, p, mu, info = mg.stokes_picard(ft, **law, method=method, rtol=1e-6, maxit=800)
    torch.cuda.synchronize()
    uo, po, muo, steps, final, change = ST.picard(W.kuhn6(), 2, L, f, law,
                                                  method="scaled" if method == "scaled" else "nodal",
                                                  rtol=1e-6, maxit=800)
    ug = _vel_gather(u.cpu().numpy(), s2n, orc.n_nodes)
    pg = _pressure_gather(p.cpu().numpy(), s2n, orc.n_nodes)
    mug = _pressure_gather(mu.cpu().numpy(), s2n, orc.n_nodes)
    unk = orc.unknown
    print(f"  Picard {method}: steps {info['picard']} vs {steps}, final {info['final_iterations']} vs "
          f"{final}; u {rel_err(ug[unk], uo[unk]):.2e}, p {rel_err(pg, po):.2e}, "
          f"mu {rel_err(mug, muo):.2e}; contrast {mug.max() / mug.min():.2f}", flush=True)
    assert info["status"] == "HHG_OK" and info["picard"] == steps
    assert abs(info["final_iterations"] - final) <= 1
    assert rel_err(ug[unk], uo[unk]) <= 1e-6 and rel_err(pg, po) <= 1e-6
    assert rel_err(mug, muo) <= 1e-8


def test_physical_scaling_follows_nodal_integration_in_the_carreau_flow():
    """Fig. stokes_profile: in the shear-thinning flow the viscosity and the
    velocity of physical scaling follow those of nodal integration, while the
    unphysical scaling departs from them (paper's Carreau parameters, force
    1000 sin(2 pi x) e_z in the no-slip cube, level 4, line y = z = 1/2)."""
    from paper_1908_08666_amd import carreau_profile as CP
    res = CP.profiles(4)
    for name, r in res["runs"].items():
        print(f"  {name}: Picard {r['picard']} + {r['final_iterations']}, {r['status']}, "
              f"viscosity {r['mu_range'][0]:.2f}..{r['mu_range'][1]:.2f}", flush=True)
        assert r["status"] == "HHG_OK"
    ph, un = res["physical_vs_nodal"], res["unphysical_vs_nodal"]
    print(f"  deviation from nodal integration: physical mu {ph['mu']:.2e} speed {ph['speed']:.2e}; "
          f"unphysical mu {un['mu']:.2e} speed {un['speed']:.2e}", flush=True)
    assert res["runs"]["nodal"]["mu_range"][1] / res["runs"]["nodal"]["mu_range"][0] > 5.0
    assert ph["mu"] < 0.25 * un["mu"] and ph["speed"] < 0.25 * un["speed"]
    assert ph["mu_l2"] < 0.25 * un["mu_l2"] and ph["speed_l2"] < 0.1 * un["speed_l2"]
