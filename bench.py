"""Benchmark of the physical stencil-scaling apply on one MI355X.

Workload (one "step" = one application y = A_s(k) x of the whole operator:
macro-interior rows, macro-boundary rows and the copy-group sum): the unit
cube cut into 6 macro-tets along its main diagonal, every macro refined to
level 7 (129 points per macro edge, 2,146,689 distinct nodes, 6,145,149
unknowns after homogeneous Dirichlet conditions on the cube boundary),
E-form elasticity with nu = 0.34 scaled by k = exp(g), g a seeded 16-mode
Fourier field of amplitude 1, x ~ U(-1, 1).  Synthetic data; FP64.

Inputs rotate over 5 buffer sets (5 x 123 MB) so that consecutive steps do
not hit the 256 MB Infinity Cache.  The timed region is bracketed by
torch.cuda.synchronize() and HIP events on the launch stream and runs with
the library's per-kernel events off; a second loop of the same steps with
them on gives the kernels' average durations for the roofline line (and its
own step time, profiled_loop_ms_per_step).

Prints ONE JSON line.  Options: --gpus (must be 1), --steps, --warmup,
--level, --no-cpu-baseline, --extra (also time FP32, on-the-fly and the
residual).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6     # 256 CUs x 2.4 GHz x 64 FP64 FMA lanes per clock x 2
FP32_VECTOR_PEAK_TFLOPS = 157.3    # published; twice the FP64 rate only with packed FP32
BYTES_PER_INTERIOR_NODE = {"f64": 56.0, "f32": 28.0}   # x (3) + k (1) read, y (3) written
# Operations per updated node: the interior kernel's own count, 311 fused
# multiply-adds (2 each), 150 additions and 14 multiplications of the ring
# form with opposite directions sharing the reference stencil; and the
# paper's count for the same update (Table tab:operations: 855 = 242 + 123 +
# 135 additions, 220 + 135 multiplications for the residual, less the 3
# subtractions of the right-hand side an apply does not perform), reported
# beside it as the paper-equivalent rate.
FLOP_PER_INTERIOR_NODE = 786.0
PAPER_FLOP_PER_INTERIOR_NODE = 852.0
# The paper's apply benchmark (Sec. 5.1.1, Fig. performancebars): FP64
# residual updates of 3 DoF on a SuperMUC-NG node (2 x Xeon Platinum 8174,
# 48 cores, 3.1 GHz nominal), 48 ranks x 3 level-7 macros (the paper's L = 5)
PAPER_APPLY = dict(hardware="SuperMUC-NG node: 2 x Intel Xeon Platinum 8174, 48 cores, 3.1 GHz",
                   ns_per_update=dict(physical_scaling=222, nodal_integration=393, stored_stencils=275),
                   MDoF_s_node=dict(physical_scaling=round(48 * 3 / 222e-9 / 1e6, 1),
                                    nodal_integration=round(48 * 3 / 393e-9 / 1e6, 1),
                                    stored_stencils=round(48 * 3 / 275e-9 / 1e6, 1)),
                   source="Sec. 5.1.1, Fig. performancebars (time per update); node rates derived "
                          "as 48 ranks x 3 DoF per update time")
N_SETS = 5


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_interior_f64_kuhn6_level7_traffic.md")


def traffic_record():
    """Counter-measured HBM bytes per interior-kernel launch (FETCH_SIZE and
    WRITE_SIZE passes scaled by a plain copy), valid only while the kernel
    sources are the ones the counters were taken on."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_RECORD).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    h = hashlib.sha256()
    try:
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as fh:
                h.update(fh.read())
    except OSError:
        return None
    return rec if h.hexdigest() == rec["source_sha256"] else None


def consistent_random(mesh, rng, shape_first):
    """U(-1,1) values per distinct node, copied to every copy slot."""
    import workloads as W
    return W.consistent_uniform(mesh.coords().T, (mesh.flags() & 2) > 0, rng, shape_first)


def cpu_baseline(level=6, runs=10, seed=0, cg_level=5):
    """The CPU oracle's apply on the host: the scaled operator of the same
    workload (6 Kuhn macros, E-form, k = exp(16-mode field)) assembled by the
    oracle from the Lemma at a level the host assembles in about a minute,
    reduced to the unknown DoFs, then y = A x timed as a CSR product: SciPy
    on one core and the oracle's plain OpenMP loop on every core the
    process may use.  Median of ``runs`` products each."""
    import numpy as np
    import workloads as W
    from oracle import cspmv
    from oracle import operators as O
    from oracle.mesh import MacroMesh
    mu, lam = W.eform_weights()
    orc = MacroMesh(W.kuhn6(), level)
    k = W.exp_fourier_coefficient(orc.xyz, W.rng_for(2, 0), 16, 1.0)
    t0 = time.perf_counter()
    A = O.reduce_dirichlet(orc, O.operator_matrix(orc, k, dict(mu1=mu, lam1=lam))).tocsr()
    t_asm = time.perf_counter() - t0
    x = np.random.default_rng(seed).uniform(-1.0, 1.0, A.shape[0])
    t_sp, t_omp = [], []
    y = np.empty(A.shape[0])
    for _ in range(runs):
        t0 = time.perf_counter()
        A @ x
        t_sp.append(time.perf_counter() - t0)
    for _ in range(runs):
        t0 = time.perf_counter()
        _, used = cspmv.spmv(A, x, y)
        t_omp.append(time.perf_counter() - t0)
    dofs = A.shape[0]
    cores = len(os.sched_getaffinity(0))
    # block-Jacobi PCG to 1e-8 with SciPy on one core (the oracle's solver),
    # on the same workload at a level that solves in seconds
    from oracle import solvers as OS
    orc_cg = MacroMesh(W.kuhn6(), cg_level)
    k_cg = W.exp_fourier_coefficient(orc_cg.xyz, W.rng_for(2, 0), 16, 1.0)
    A_cg = O.reduce_dirichlet(orc_cg, O.operator_matrix(orc_cg, k_cg, dict(mu1=mu, lam1=lam))).tocsr()
    b_cg = np.random.default_rng(seed + 1).uniform(-1.0, 1.0, A_cg.shape[0])
    t0 = time.perf_counter()
    _, cg_it = OS.block_jacobi_cg(A_cg, b_cg, rtol=1e-8)
    t_cg = time.perf_counter() - t0
    return dict(value=round(dofs / float(np.median(t_omp)) / 1e6, 2), unit="MDoF/s", cores=int(used),
                kind="oracle", host_cores=cores,
                scipy_1core=dict(value=round(dofs / float(np.median(t_sp)) / 1e6, 2), unit="MDoF/s",
                                 cores=1),
                runs=runs, assembly_seconds=round(t_asm, 1), nnz=int(A.nnz), dofs=int(dofs),
                cg=dict(level=cg_level, dofs=int(A_cg.shape[0]), iterations=int(cg_it),
                        seconds=round(t_cg, 3), cores=1, rtol=1e-8,
                        note="SciPy cg with the block-Jacobi preconditioner of the oracle's assembled "
                             "operator (the oracle's solver), one core"),
                sample=f"the same workload at level {level} (unknown DoFs {dofs}, {A.nnz} nonzeros, "
                       f"CSR {A.nnz * 12 / 1e6:.0f} MB): the oracle's assembled scaled operator, "
                       f"y = A x as a plain OpenMP CSR loop over {used} threads (value) and SciPy on "
                       f"one core; median of {runs} products each")


def mg_solve(verts, level, op, k, b, coarse=2, rtol=1e-8, maxit=100, precision="f64"):
    """V(3,3)-cycle preconditioned CG on the hierarchy coarse..level (damped
    block Jacobi, omega 0.7, exact coarsest solve; cycles in FP64 or FP32,
    CG in FP64): coefficient setup time (injection, inverse blocks of every
    level, coarse inverse) and solve time of a second, warm run."""
    import torch
    from paper_1908_08666_amd import Multigrid
    mgh = Multigrid(verts, level, coarse, **op)
    try:
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mgh.setup_coefficient(k)
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            x = torch.zeros_like(b)
            t0 = time.perf_counter()
            x, info = mgh.solve(b, x=x, rtol=rtol, maxit=maxit, precision=precision,
                                raise_on_status=False)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
    finally:
        mgh.close()
    return dict(iterations=info["iterations"], seconds=round(wall, 4),
                setup_seconds=round(t_setup, 4), rel_residual=info["rel_residual"],
                status=info["status"], levels=[coarse, level], cycle="V(3,3)", omega=0.7,
                cycle_precision=precision)


def carreau_workload(level, dev, solve=True, maxit=60000):
    """Generalized-Newtonian eps-operator on the 24-macro cube: Carreau
    viscosity of a seeded smooth velocity field (viscosity contrast of order
    1e2), then FP64 CG vs FP32 + FP64 refinement to 1e-8."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1908_08666_amd import Mesh
    law = dict(W.CARREAU_DEFAULT)
    mesh = Mesh(W.cube24(), level, mu1=1.0)
    xyz = mesh.coords().T
    # velocity concentrated around a seeded centre: amplitude 1e3 gives a
    # viscosity contrast of order 1e2 across the cube
    u = torch.from_numpy(np.ascontiguousarray(
        W.localized_velocity_field(xyz, W.rng_for(3, 0), 1e3).T)).to(dev)
    ws = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k = mesh.nodal_viscosity(u, **law)      # the first call builds the boundary fit tables
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    reps = 10
    for _ in range(reps):
        k = mesh.nodal_viscosity(u, k=k, **law)
    torch.cuda.synchronize()
    t_visc = (time.perf_counter() - t0) / reps
    out = dict(level=level, macros=mesh.n_macro, unknown_dofs=3 * mesh.n_unknown,
               viscosity_ms=round(t_visc * 1e3, 3), viscosity_first_call_ms=round(t_first * 1e3, 1),
               viscosity_min=float(k.min()), viscosity_max=float(k.max()),
               contrast=float(k.max() / k.min()))
    if solve:
        b = torch.from_numpy(consistent_random(mesh, W.rng_for(3, 99), 3)).to(dev, torch.float64)
        fl = torch.from_numpy(mesh.flags()).to(dev)
        b[:, (fl & 1) > 0] = 0.0
        for name, opts in (("cg64", dict(solver="cg64")), ("ir32", dict(solver="ir32", inner_rtol=1e-2))):
            nb = mesh.workspace_bytes(**opts)
            if ws is None or ws.numel() < nb + 256:
                ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
            for rep in range(2):
                x = torch.zeros_like(b)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = mesh.solve(b, k, x=x, workspace=ws, rtol=1e-8, check_every=16,
                                     maxit=maxit, raise_on_status=False, **opts)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
            out[name] = dict(iterations=info["iterations"], outer=info["outer_iterations"],
                             seconds=round(wall, 4), rel_residual=info["rel_residual"],
                             status=info["status"])
        ws = None
        torch.cuda.empty_cache()
        out["mg_pcg64"] = mg_solve(W.cube24(), level, dict(mu1=1.0), k, b)
        out["mg_pcg64_f32cycle"] = mg_solve(W.cube24(), level, dict(mu1=1.0), k, b, precision="f32")
    return out


def learned_workload(dev, level=6, n_records=20000, epochs=100, batch=2048, lr=3e-3):
    """Learned block smoother on the 24-macro Carreau eps-operator: records
    from the plain solver, training on the device, then FP64 solves to 1e-8
    with block Jacobi (PCG, FCG) and with the learned blocks (FCG), and the
    FP32 + refinement solver with either preconditioner."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1908_08666_amd import Mesh
    from paper_1908_08666_amd import learned as LG
    mesh = Mesh(W.cube24(), level, mu1=1.0)
    xyz = mesh.coords().T
    owner = (mesh.flags() & 2) > 0
    u = torch.from_numpy(np.ascontiguousarray(
        W.localized_velocity_field(xyz, W.rng_for(5, 0), 1e6).T)).to(dev)
    k = mesh.nodal_viscosity(u, **W.CARREAU_DEFAULT)
    b = torch.from_numpy(W.consistent_uniform(xyz, owner, W.rng_for(5, 1))).to(dev)
    fl = torch.from_numpy(mesh.flags()).to(dev)
    b[:, (fl & 1) > 0] = 0.0
    noise = torch.from_numpy(W.consistent_uniform(xyz, owner, W.rng_for(5, 2))).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec, xs = LG.solver_pairs(mesh, k, b, noise, n_records, seed=3)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    perm = torch.randperm(n_records, generator=torch.Generator().manual_seed(0)).to(dev)
    rec = rec[perm].contiguous()
    net = LG.SmootherNet(W.smoother_init_weights(W.rng_for(5, 4)))
    held = rec[-2000:]
    l0, _ = net.loss_grad(held, held.shape[0])
    t0 = time.perf_counter()
    hist = net.train(rec[:-2000], n_records - 2000, epochs=epochs, batch=batch, lr=lr)
    t_train = time.perf_counter() - t0
    l1, _ = net.loss_grad(held, held.shape[0])
    LG.attach(mesh, net)
    out = dict(level=level, macros=mesh.n_macro, unknown_dofs=3 * mesh.n_unknown,
               viscosity_min=float(k.min()), viscosity_max=float(k.max()),
               contrast=float(k.max() / k.min()), records=n_records, epochs=epochs, batch=batch,
               pairs_seconds=round(t_pairs, 3), train_seconds=round(t_train, 3),
               train_loss_first_last=[float(hist[0]), float(hist[-1])],
               heldout_loss_block_jacobi=round(l0, 5), heldout_loss_learned=round(l1, 5))
    ws = None
    xn = float(torch.linalg.norm(xs))
    for name, opts in (("pcg64_block_jacobi", dict(solver="cg64", precond="block_jacobi")),
                       ("fcg64_block_jacobi", dict(solver="fcg64", precond="block_jacobi")),
                       ("fcg64_learned", dict(solver="fcg64", precond="learned")),
                       ("ir32_block_jacobi", dict(solver="ir32", precond="block_jacobi", inner_rtol=1e-2)),
                       ("ir32_learned", dict(solver="ir32", precond="learned", inner_rtol=1e-2))):
        nb = mesh.workspace_bytes(**opts)
        if ws is None or ws.numel() < nb + 256:
            ws = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        for rep in range(2):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = mesh.solve(b, k, x=x, workspace=ws, rtol=1e-8, check_every=16, maxit=60000,
                                 raise_on_status=False, **opts)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        out[name] = dict(iterations=info["iterations"], outer=info["outer_iterations"],
                         seconds=round(wall, 4), rel_residual=info["rel_residual"],
                         status=info["status"],
                         rel_error_vs_tight_fp64_solution=float(torch.linalg.norm(x - xs)) / xn)
    LG.attach(mesh, None)
    return out


def twod_workload(dev, level=12, steps=50):
    """2-D apply (macro triangles, Sec. 2.3): the unit square as two macros
    at the given level, E-form elasticity with an exp-Fourier coefficient;
    scaled apply in FP64 and FP32 over 3 rotating input sets, HBM resident."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1908_08666_amd.twod import Mesh2D
    mu, lam = W.eform_weights()
    mesh = Mesh2D(W.twod_mesh("square"), level, mu1=mu, lam1=lam)
    xy = mesh.coords().T
    xyz = np.column_stack([xy, np.zeros(len(xy))])
    out = dict(level=level, macros=2, slots=mesh.n_nodes, unknown_dofs=2 * mesh.n_unknown,
               bytes_per_row=dict(f64=40, f32=20))
    for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
        sets = []
        for s in range(3):
            rng = W.rng_for(6, s)
            k = torch.from_numpy(W.exp_fourier_coefficient(xyz, rng, 16, 1.0)).to(dev, dt)
            x = torch.from_numpy(rng.uniform(-1, 1, (2, mesh.n_nodes))).to(dev, dt)
            sets.append((x, k, torch.empty_like(x)))
        for q in range(6):
            mesh.apply_scaled(*sets[q % 3])
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for q in range(steps):
            mesh.apply_scaled(*sets[q % 3])
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        b = out["bytes_per_row"][name] * mesh.n_nodes
        out[name] = dict(ms_per_apply=round(ms, 5), MDoF_s=round(2 * mesh.n_unknown / (ms * 1e-3) / 1e6, 1),
                         GB_s=round(b / (ms * 1e-3) / 1e9, 1), hbm_frac=round(b / (ms * 1e-3) / 8e12, 3))
        sets = None
    mesh.close()
    return out


def batch_workload(dev, launches=20, count=10):
    """256 independent single-macro elasticity problems, levels uniform in
    3..6, each with its own coefficient field: FP32 apply over the whole
    batch in one interior launch, tuned by the library's autotuner and
    replayed from a HIP graph of `count` applies; FP64 apply of the same
    inputs as the per-problem accuracy check."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1908_08666_amd import Mesh
    mu, lam = W.eform_weights()
    levels = W.batch_levels(256)
    mesh = Mesh(np.repeat(W.unit_tet(), 256, axis=0), levels, coupling="independent",
                mu1=mu, lam1=lam)
    off = mesh.macro_offset
    xyz = mesh.coords().T
    k_np = np.concatenate(W.batch_coefficients([xyz[off[m]:off[m + 1]] for m in range(256)]))
    x_np = W.uniform_vector(3 * mesh.n_nodes, W.rng_for(4, 3)).reshape(3, -1)
    x32 = torch.from_numpy(x_np).to(dev, torch.float32)
    k32 = torch.from_numpy(k_np).to(dev, torch.float32)
    y32 = torch.empty_like(x32)
    _, rep = mesh.autotune(x32, k32, y32, reps=5)
    gid = mesh.graph_create(x32, k32, y32, count=count)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        mesh.graph_launch(gid, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(launches):
        mesh.graph_launch(gid, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_per_apply = e0.elapsed_time(e1) / (launches * count)
    mesh.graph_destroy(gid)
    dofs = 3 * mesh.n_unknown
    # the graph replays one input set (x, k, y), which fits the 256 MB
    # Infinity Cache; direct applies rotating over enough sets to exceed it
    # twice over give the rate with inputs streamed from HBM
    set_bytes = 2 * x32.numel() * 4 + k32.numel() * 4
    n_sets = max(3, -(-512 * 2**20 // set_bytes))
    rot = [(torch.from_numpy(W.uniform_vector(3 * mesh.n_nodes, W.rng_for(4, 10 + s)).reshape(3, -1))
            .to(dev, torch.float32), k32.clone(), torch.empty_like(x32)) for s in range(n_sets)]
    for s in range(2 * n_sets):
        mesh.apply_scaled(*rot[s % n_sets], stream=stream)
    torch.cuda.synchronize()
    n_rot = n_sets * max(1, (10 * launches) // n_sets)
    e0.record(stream)
    for s in range(n_rot):
        mesh.apply_scaled(*rot[s % n_sets], stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_rot = e0.elapsed_time(e1) / n_rot
    rot = None
    # accuracy: FP32 result against the FP64 apply, per problem
    y64 = mesh.apply_scaled(x32.double(), k32.double())
    torch.cuda.synchronize()
    a, b = y32.double().cpu().numpy(), y64.cpu().numpy()
    errs = [np.linalg.norm(a[:, off[m]:off[m + 1]] - b[:, off[m]:off[m + 1]]) /
            np.linalg.norm(b[:, off[m]:off[m + 1]]) for m in range(256)]
    per_level = []
    for q, lv in enumerate(rep["levels"]):
        per_level.append(dict(level=lv["level"], problems=lv["macros"], rows=lv["rows"],
                              slab=lv["slab"], interior_ms_alone=round(lv["ms"], 5),
                              MDoF_s_alone=round(3 * lv["rows"] / (lv["ms"] * 1e-3) / 1e6, 1)))
    return dict(problems=256, slots=mesh.n_nodes, unknown_dofs=dofs, dtype="f32",
                applies_per_graph=count, ms_per_apply=round(ms_per_apply, 5),
                MDoF_s=round(dofs / (ms_per_apply * 1e-3) / 1e6, 1),
                MDoF_s_note="graph of applies on one input set (Infinity-Cache resident)",
                ms_per_apply_hbm=round(ms_rot, 5),
                MDoF_s_hbm=round(dofs / (ms_rot * 1e-3) / 1e6, 1),
                MDoF_s_hbm_note=f"direct applies rotating over {n_sets} input sets of "
                                f"{set_bytes / 1e6:.0f} MB (HBM resident)",
                interior_GBs=round(28.0 * mesh.n_unknown / (rep["ms_total"] * 1e-3) / 1e9, 1),
                persist_blocks=rep["persist_blocks"], tuning_candidates=rep["candidates"],
                per_level=per_level,
                max_rel_err_vs_f64_per_problem=float(max(errs)))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--level", type=int, default=7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-level", type=int, default=6)
    ap.add_argument("--extra", action="store_true")
    ap.add_argument("--quick", action="store_true",
                    help="only the headline apply (and the CPU baseline); the other workloads are "
                         "run by default")
    ap.add_argument("--solve", action="store_true", help="also time CG / IR solves to 1e-8")
    ap.add_argument("--carreau-level", type=int, default=7)
    ap.add_argument("--carreau", action="store_true",
                    help="also run the 24-macro Carreau eps-operator workload (viscosity + solves)")
    ap.add_argument("--batch", action="store_true",
                    help="also run 256 independent uneven-level problems in one tuned, graph-replayed launch")
    ap.add_argument("--learned", action="store_true",
                    help="also train the learned block smoother and compare FCG solves (24 macros, level 6)")
    ap.add_argument("--twod", action="store_true", help="2-D apply on the square (two macro triangles)")
    ap.add_argument("--carreau-profile", action="store_true",
                    help="physical / nodal / unphysical scaling in the Carreau fixed-point flow")
    ap.add_argument("--carreau-profile-level", type=int, default=5)
    ap.add_argument("--elastostatics-finest", type=int, default=7,
                    help="finest level of the elastostatics benchmark (8 is the paper's finest)")
    ap.add_argument("--elastostatics-variants", default="",
                    help="comma-separated subset of the elastostatics variants (default all)")
    ap.add_argument("--elastostatics", action="store_true",
                    help="also run the paper's manufactured-solution benchmark (V-cycles, levels 3..7)")
    ap.add_argument("--elastostatics-m", default="1,8",
                    help="frequencies m of the modulus cos(m pi xyz) + 2 (the paper: 1,2,3,8)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB FP64 buffer 10 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if not args.quick:
        args.extra = args.solve = args.batch = args.learned = args.carreau = args.elastostatics = True
        args.carreau_profile = args.twod = True
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); sharding the macros "
              f"across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    from paper_1908_08666_amd import Mesh

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": nbytes, "bytes_written": nbytes,
                                               "launches": 10}}), flush=True)
        return
    mu, lam = W.eform_weights()
    mesh = Mesh(W.kuhn6(), args.level, mu1=mu, lam1=lam)
    n = 1 << args.level
    N = mesh.n_nodes
    dofs = 3 * mesh.n_unknown
    interior_rows = mesh.n_macro * (n - 1) * (n - 2) * (n - 3) // 6
    xyz = mesh.coords().T
    k_np = W.exp_fourier_coefficient(xyz, W.rng_for(2, 0), 16, 1.0)

    def make_sets(dtype):
        sets = []
        for s in range(N_SETS):
            x = torch.from_numpy(consistent_random(mesh, W.rng_for(2, 10 + s), 3)).to(dev, dtype)
            k = torch.from_numpy(k_np).to(dev, dtype)
            y = torch.empty_like(x)
            sets.append((x, k, y))
        return sets

    stream = torch.cuda.current_stream()

    def timed(fn, sets, steps, warmup, profile=True):
        for w in range(warmup):
            fn(*sets[w % N_SETS])
        torch.cuda.synchronize()
        if profile:
            mesh.profile_enable(True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for s in range(steps):
            fn(*sets[s % N_SETS])
        e1.record(stream)
        torch.cuda.synchronize()
        total_ms = e0.elapsed_time(e1)
        prof = mesh.profile_read() if profile else {}
        if profile:
            mesh.profile_enable(False)
        return total_ms, prof

    sets64 = make_sets(torch.float64)
    # the headline loop runs without the library's per-kernel events (they add
    # two event records per kernel to every step); a second loop over the
    # same workload, with the events on, gives the per-kernel durations
    total_ms, _ = timed(lambda x, k, y: mesh.apply_scaled(x, k, y), sets64, args.steps,
                        args.warmup, profile=False)
    prof_ms, prof = timed(lambda x, k, y: mesh.apply_scaled(x, k, y), sets64, args.steps,
                          args.warmup)
    ms_per_step = total_ms / args.steps
    value = dofs / (ms_per_step * 1e-3) / 1e6

    nl, int_ms = prof["interior_scaled"]
    avg_int_ms = int_ms / max(nl, 1)
    alg_bytes = BYTES_PER_INTERIOR_NODE["f64"] * interior_rows
    achieved = alg_bytes / (avg_int_ms * 1e-3) / 1e9
    rec = traffic_record() if args.level == 7 else None
    traffic = rec["traffic_bytes_per_launch"] if rec else None
    # 786 FLOP per 56 B is 14.0 FLOP/B, above the FP64 ridge of 78.6 TF / 8 TB/s
    # = 9.8 FLOP/B: the apply is bound by FP64 vector arithmetic on this chip
    flops = FLOP_PER_INTERIOR_NODE * interior_rows
    tflops = flops / (avg_int_ms * 1e-3) / 1e12
    roofline = dict(bound="alu", achieved=round(tflops, 2), peak=FP64_VECTOR_PEAK_TFLOPS,
                    unit="TFLOP/s", frac=round(tflops / FP64_VECTOR_PEAK_TFLOPS, 4), traffic=traffic,
                    traffic_unit="HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    traffic_over_algorithmic=round(traffic / alg_bytes, 3) if traffic else None,
                    kernel="k_interior<double, scaled>",
                    avg_kernel_ms=round(avg_int_ms, 5),
                    profiled_loop_ms_per_step=round(prof_ms / args.steps, 5),
                    flop_per_launch=int(flops), units_per_launch=interior_rows,
                    flop_per_unit=FLOP_PER_INTERIOR_NODE,
                    paper_flop_per_unit=PAPER_FLOP_PER_INTERIOR_NODE,
                    paper_equivalent_tflops=round(PAPER_FLOP_PER_INTERIOR_NODE * interior_rows /
                                                  (avg_int_ms * 1e-3) / 1e12, 2),
                    hbm=dict(achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=round(achieved / HBM_PEAK_GBS, 4), bytes_per_launch=int(alg_bytes),
                             bytes_per_unit=56))
    kernels = {name: dict(launches=c, avg_ms=round(ms / c, 5) if c else None)
               for name, (c, ms) in prof.items()}

    extra = {}
    if args.extra:
        sets64 = None
        torch.cuda.empty_cache()
        sets64 = make_sets(torch.float64)
        t_fly, p_fly = timed(lambda x, k, y: mesh.apply_onthefly(x, k, y), sets64,
                             max(args.steps // 4, 5), 5)
        extra["onthefly_f64_MDoF_s"] = round(dofs / (t_fly / max(args.steps // 4, 5) * 1e-3) / 1e6, 1)
        c, ms = p_fly["interior_onthefly"]
        extra["onthefly_f64_interior_avg_ms"] = round(ms / max(c, 1), 5)
        t_res, _ = timed(lambda x, k, y: mesh.residual(x, x, k, y), sets64, max(args.steps // 4, 5),
                         5, profile=False)
        extra["residual_f64_MDoF_s"] = round(dofs / (t_res / max(args.steps // 4, 5) * 1e-3) / 1e6, 1)
        sets64 = None
        torch.cuda.empty_cache()
        sets32 = make_sets(torch.float32)
        t32, p32 = timed(lambda x, k, y: mesh.apply_scaled(x, k, y), sets32, args.steps, args.warmup)
        extra["scaled_f32_MDoF_s"] = round(dofs / (t32 / args.steps * 1e-3) / 1e6, 1)
        c, ms = p32["interior_scaled"]
        a32 = BYTES_PER_INTERIOR_NODE["f32"] * interior_rows / (ms / max(c, 1) * 1e-3) / 1e9
        extra["scaled_f32_interior_avg_ms"] = round(ms / max(c, 1), 5)
        extra["scaled_f32_interior_GBs"] = round(a32, 1)
        extra["scaled_f32_interior_TFLOPs"] = round(
            FLOP_PER_INTERIOR_NODE * interior_rows / (ms / max(c, 1) * 1e-3) / 1e12, 2)

    if args.solve:
        sets64 = sets32 = None
        torch.cuda.empty_cache()
        b = torch.from_numpy(consistent_random(mesh, W.rng_for(2, 99), 3)).to(dev, torch.float64)
        fl = torch.from_numpy(mesh.flags()).to(dev)
        b[:, (fl & 1) > 0] = 0.0
        k64 = torch.from_numpy(k_np).to(dev, torch.float64)
        solves = {}
        ws = None
        for name, opts in (("cg64", dict(solver="cg64")),
                           ("ir32_inner1e-2", dict(solver="ir32", inner_rtol=1e-2)),
                           ("ir32_inner1e-3", dict(solver="ir32", inner_rtol=1e-3)),
                           ("ir32_inner1e-4", dict(solver="ir32", inner_rtol=1e-4))):
            nbytes = mesh.workspace_bytes(**opts)
            if ws is None or ws.numel() < nbytes + 256:
                ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
            for rep in range(2):          # second run reuses the warmed state
                x = torch.zeros_like(b)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, info = mesh.solve(b, k64, x=x, workspace=ws, rtol=1e-8, check_every=16, **opts)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
            solves[name] = dict(iterations=info["iterations"], outer=info["outer_iterations"],
                                seconds=round(wall, 4), rel_residual=info["rel_residual"],
                                status=info["status"])
        ws = None
        torch.cuda.empty_cache()
        solves["mg_pcg64"] = mg_solve(W.kuhn6(), args.level, dict(mu1=mu, lam1=lam), k64, b)
        solves["mg_pcg64_f32cycle"] = mg_solve(W.kuhn6(), args.level, dict(mu1=mu, lam1=lam), k64, b,
                                               precision="f32")
        # the same solver at the CPU baseline's CG level, for a like-for-like time
        m5 = Mesh(W.kuhn6(), 5, mu1=mu, lam1=lam)
        k5 = torch.from_numpy(W.exp_fourier_coefficient(m5.coords().T, W.rng_for(2, 0), 16, 1.0)).to(dev)
        b5 = torch.from_numpy(consistent_random(m5, W.rng_for(2, 98), 3)).to(dev, torch.float64)
        b5[:, (torch.from_numpy(m5.flags()).to(dev) & 1) > 0] = 0.0
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info5 = m5.solve(b5, k5, rtol=1e-8, check_every=16, solver="cg64")
            torch.cuda.synchronize()
            wall5 = time.perf_counter() - t0
        solves["cg64_level5"] = dict(iterations=info5["iterations"], seconds=round(wall5, 4),
                                     status=info5["status"], dofs=3 * m5.n_unknown)
        m5 = None
        extra["solve_to_1e-8"] = solves

    if args.batch:
        sets64 = sets32 = None
        torch.cuda.empty_cache()
        extra["batch256_independent"] = batch_workload(dev)

    if args.learned:
        sets64 = sets32 = None
        torch.cuda.empty_cache()
        extra["learned_smoother_cube24"] = learned_workload(dev)

    if args.carreau:
        sets64 = sets32 = None
        torch.cuda.empty_cache()
        extra["carreau_cube24"] = carreau_workload(args.carreau_level, dev)

    if args.twod:
        torch.cuda.empty_cache()
        extra["twod_square"] = twod_workload(dev)

    if args.carreau_profile:
        torch.cuda.empty_cache()
        from paper_1908_08666_amd import carreau_profile as CPR
        extra["carreau_profile_kuhn6"] = CPR.profiles(args.carreau_profile_level, dev=dev)

    if args.elastostatics:
        sets64 = sets32 = None
        torch.cuda.empty_cache()
        from paper_1908_08666_amd import elastostatics as ELS
        variants = {
            "physical": dict(corr="physical", op_method="scaled", iface="rowwise", method="cycle"),
            "nodal": dict(corr="physical", op_method="onthefly", iface="rowwise", method="cycle"),
            "unphysical": dict(corr="none", op_method="scaled", iface="rowwise", method="cycle"),
            "physical_symmetric_rule": dict(corr="physical", op_method="scaled", iface="symmetric",
                                            method="cg"),
            "physical_zerosum_rule": dict(corr="physical", op_method="scaled", iface="zerosum",
                                          method="cg"),
            "physical_f32_cycles": dict(corr="physical", op_method="scaled", iface="rowwise",
                                        method="cycle", precision="f32"),
            "physical_variable_cycles": dict(corr="physical", op_method="scaled", iface="rowwise",
                                             method="cycle", nu_inc=2),
        }
        if args.elastostatics_variants:
            variants = {k: v for k, v in variants.items() if k in args.elastostatics_variants.split(",")}
        fin = args.elastostatics_finest
        lv = list(range(3, fin + 1))
        extra["elastostatics_kuhn6"] = dict(
            levels=lv, finest=fin, paper_levels=[q - 2 for q in lv],
            load="consistent mass matrix times the interpolated body force",
            results=ELS.benchmark(lv, fin, ms=tuple(int(m) for m in args.elastostatics_m.split(",")),
                                  variants=variants, dev=dev))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_level)

    out = {
        "metric": "scaled-stencil apply MDoF/s + %HBM peak; CG time to 1e-8 (FP64 vs FP32+IR vs learned)",
        "value": round(value, 1),
        "unit": "MDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"elasticity E-form (nu=0.34), unit cube as 6 macro-tets at level "
                               f"{args.level}, k=exp(16-mode Fourier field, amplitude 1), "
                               f"physical stencil scaling apply",
                   "level": args.level, "macros": mesh.n_macro, "distinct_nodes_unknown": mesh.n_unknown,
                   "dofs_per_step": dofs, "slots": N, "interior_rows": interior_rows,
                   "buffer_sets": N_SETS},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "paper": PAPER_APPLY,
        "kernels": kernels,
    }
    if extra:
        out["extra"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
