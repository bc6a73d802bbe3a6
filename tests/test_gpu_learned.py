"""GPU parity of the learned 3x3 block smoother against the CPU oracle:
features (within one BF16 unit), MFMA inference (bound derived from the BF16 rounding of
the hidden layer), training records, loss and gradient, Adam steps,
preconditioner blocks, FCG, and what training gains over block Jacobi."""
import numpy as np
import pytest

import workloads as W
from oracle import learned as LN
from oracle import operators as O
from oracle import solvers as S
from oracle.mesh import MacroMesh
from tests.helpers import slot_to_node, scatter, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MU, LAM = W.eform_weights()
EFORM = dict(mu1=MU, lam1=LAM)


def _u16_to_bf16_values(a):
    return (a.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _case(verts, level, op, kseed):
    from paper_1908_08666_amd import Mesh
    lib = Mesh(verts, level, **op)
    orc = MacroMesh(verts, level)
    s2n = slot_to_node(lib, orc)
    k = W.exp_fourier_coefficient(orc.xyz, W.rng_for(5, kseed), 8, 1.5)
    return lib, orc, s2n, k


def _slot_to_local(lib, orc):
    """(macro, oracle local index) of every library slot, by coordinates."""
    from scipy.spatial import cKDTree
    xyz = lib.coords().T
    off = lib.macro_offset
    out = []
    for m in range(orc.n_macro):
        d, idx = cKDTree(orc.local_xyz[m]).query(xyz[off[m]:off[m + 1]])
        assert d.max() < 1e-9
        out.append(idx)
    return out


def _random_weights(seed, scale2=0.2):
    rng = np.random.default_rng(seed)
    w = LN.init_params(rng)
    w[LN.N_IN * LN.N_HID:] = rng.normal(scale=scale2, size=LN.N_PARAM - LN.N_IN * LN.N_HID)
    return w.astype(np.float32).astype(np.float64)


def _forward_bound(w, F):
    """Per-output bound on |GPU - oracle|: one BF16 ulp on every hidden unit
    (a hidden value whose FP32 and FP64 pre-activations round differently)
    plus FP32 accumulation; and the tight FP32-only part."""
    o, (z1, h, W1r, W2r) = LN.forward(w, F)
    ulp = np.where(h > 0, 2.0 ** (np.floor(np.log2(np.where(h > 0, h, 1.0))) - 7), 0.0)
    mag = np.abs(h) @ np.abs(W2r) + np.abs(LN.unpack(w)[3])
    flip = ulp @ np.abs(W2r)
    tight = 1e-5 * (mag + 1e-30)
    return o, flip + tight, tight


def _features_agree(Fg, Fo):
    """GPU features against the oracle's: the kernel sums the patch left to
    right, the oracle takes the correctly rounded sum, so a BF16 rounding may
    move by one unit; almost every feature is bit-exact."""
    assert np.all(np.abs(Fg - Fo) <= LN.bf16_ulp(Fo))
    assert np.mean(Fg == Fo) >= 0.99


@pytest.mark.parametrize("name", ["kuhn6", "cube24"])
def test_features_match_oracle(name):
    from paper_1908_08666_amd import learned as LG
    verts = W.kuhn6() if name == "kuhn6" else W.cube24()
    lib, orc, s2n, k = _case(verts, 3 if name == "kuhn6" else 2, EFORM, 1)
    kt = torch.from_numpy(scatter(k, s2n)).cuda()
    F = LG.features(lib, kt)
    torch.cuda.synchronize()
    Fg = _u16_to_bf16_values(F.cpu().numpy().view(np.uint16))
    loc = _slot_to_local(lib, orc)
    off = lib.macro_offset
    for m in range(orc.n_macro):
        Fo = LN.macro_features(orc, m, k)
        _features_agree(Fg[off[m]:off[m + 1]], Fo[loc[m]])


def test_mfma_forward_matches_oracle():
    from paper_1908_08666_amd import learned as LG
    lib, orc, s2n, k = _case(W.kuhn6(), 4, EFORM, 2)
    # the oracle's features of every slot, handed to the kernel as BF16 bits
    loc = _slot_to_local(lib, orc)
    off = lib.macro_offset
    Fv = np.concatenate([LN.macro_features(orc, m, k)[loc[m]] for m in range(orc.n_macro)])
    bits = (Fv.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    assert off[-1] == Fv.shape[0] and np.array_equal(_u16_to_bf16_values(bits), Fv)
    F = torch.from_numpy(bits.view(np.int16).copy()).cuda()
    w = _random_weights(11)
    net = LG.SmootherNet(w)
    out = net.forward(F).cpu().numpy().astype(np.float64)
    o, bound, tight = _forward_bound(w, Fv)
    err = np.abs(out - o)
    frac_tight = np.mean(err <= tight)
    print(f"  forward: max err {err.max():.3e}, within FP32 bound {frac_tight:.5f}", flush=True)
    assert np.all(err <= bound)
    assert frac_tight >= 0.99
    # ragged tail: a record count that is not a multiple of 16
    n = 16 * 37 + 5
    out2 = net.forward(F, n=n).cpu().numpy()
    assert np.array_equal(out2, out[:n].astype(np.float32))


def _records_from_oracle(Fv, r, e, S6):
    """Host-built training records (same byte layout as the library's)."""
    n = Fv.shape[0]
    rec = np.zeros((n, 128), dtype=np.uint8)
    f32 = Fv.astype(np.float32).view(np.uint32)
    rec.view(np.uint16)[:, :16] = (f32 >> 16).astype(np.uint16)
    vals = np.concatenate([r, e, S6], axis=1).astype(np.float32)
    rec.view(np.float32)[:, 8:20] = vals
    return rec


def _oracle_inputs_from_records(rec):
    Fv = _u16_to_bf16_values(rec.view(np.uint16)[:, :16])
    v = rec.view(np.float32)[:, 8:20].astype(np.float64)
    return Fv, v[:, 0:3], v[:, 3:6], v[:, 6:12]


def test_collect_records_match_oracle():
    from paper_1908_08666_amd import learned as LG
    lib, orc, s2n, k = _case(W.kuhn6(), 3, EFORM, 3)
    rng = np.random.default_rng(4)
    r = rng.uniform(-1, 1, size=(orc.n_nodes, 3))
    e = rng.uniform(-1, 1, size=(orc.n_nodes, 3))
    fl = lib.flags()
    cand = np.nonzero((fl & 3) == 2)[0]
    slots = np.sort(rng.choice(cand, 150, replace=False))
    kt = torch.from_numpy(scatter(k, s2n)).cuda()
    rec = LG.collect(lib, kt, torch.from_numpy(scatter(r, s2n)).cuda(),
                     torch.from_numpy(scatter(e, s2n)).cuda(), torch.from_numpy(slots).cuda())
    rec = rec.cpu().numpy()
    Fg, rg, eg, Sg = _oracle_inputs_from_records(rec)
    A = O.operator_matrix(orc, k, EFORM)
    nodes = s2n[slots]
    D = LN.diag_blocks(A, nodes)
    # features: the copy that the slot belongs to
    off = lib.macro_offset
    loc = _slot_to_local(lib, orc)
    Fo = np.empty((slots.size, 16))
    for q, s in enumerate(slots):
        m = int(np.searchsorted(off, s, side="right") - 1)
        Fo[q] = LN.macro_features(orc, m, k)[loc[m][s - off[m]]]
    _, ro, eo, So = LN.make_samples(Fo, r[nodes], e[nodes], D)
    assert np.all(np.abs(Fg - Fo) <= LN.bf16_ulp(Fo))
    for got, want in ((rg, ro), (eg, eo), (Sg, So)):
        assert np.allclose(got, want, rtol=2e-7, atol=2e-7 * np.abs(want).max())


def _synthetic_records(n, seed):
    rng = np.random.default_rng(seed)
    Fv = LN.bf16_round(rng.uniform(0.0, 2.0, size=(n, 16)))
    r = rng.normal(size=(n, 3))
    e = rng.normal(size=(n, 3))
    A = rng.normal(size=(n, 3, 3)) * 0.5
    Sm = np.einsum("nab,ncb->nac", A, A) + np.eye(3)
    S6 = np.stack([Sm[:, 0, 0], Sm[:, 1, 1], Sm[:, 2, 2], Sm[:, 0, 1], Sm[:, 0, 2], Sm[:, 1, 2]], 1)
    return _records_from_oracle(Fv, r, e, S6)


def test_loss_and_gradient_match_oracle():
    from paper_1908_08666_amd import learned as LG
    rec = _synthetic_records(3000, 5)
    w = _random_weights(12)
    net = LG.SmootherNet(w)
    loss, g = net.loss_grad(torch.from_numpy(rec).cuda(), rec.shape[0])
    lo, go = LN.loss_and_grad(w, *_oracle_inputs_from_records(rec))
    print(f"  loss {loss:.6e} vs {lo:.6e}; grad rel err {rel_err(g, go):.3e}", flush=True)
    assert abs(loss - lo) <= 1e-5 * lo
    assert rel_err(g.astype(np.float64), go) <= 1e-4


def test_adam_steps_match_oracle():
    from paper_1908_08666_amd import learned as LG
    rec = _synthetic_records(1000, 6)
    w = _random_weights(13)
    net = LG.SmootherNet(w)
    lr = 1e-3
    net.train(torch.from_numpy(rec).cuda(), rec.shape[0], epochs=2, batch=500, lr=lr)
    wg = net.get_weights().astype(np.float64)
    wo = w.copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    inputs = _oracle_inputs_from_records(rec)
    t = 0
    for _ in range(2):
        for a in (0, 500):
            t += 1
            _, g = LN.loss_and_grad(wo, *[x[a:a + 500] for x in inputs])
            wo, m, v = LN.adam_step(wo, g, m, v, t, lr)
    d = np.abs(wg - wo)
    print(f"  adam: max |dw| {d.max():.3e} (lr {lr})", flush=True)
    # every step moves a weight by at most lr; the FP32 and FP64 paths agree
    # unless a gradient entry is near zero (its sign then decides the step)
    assert np.mean(d <= 1e-3 * lr) >= 0.98
    assert d.max() <= 4 * lr


def _solve_setup(level=3):
    from paper_1908_08666_amd import Mesh
    lib, orc, s2n, k = _case(W.kuhn6(), level, EFORM, 7)
    kt = torch.from_numpy(scatter(k, s2n)).cuda()
    b_nodes = np.random.default_rng(8).uniform(-1, 1, size=(orc.n_nodes, 3))
    b_nodes[orc.dirichlet] = 0
    bt = torch.from_numpy(scatter(b_nodes, s2n)).cuda()
    return lib, orc, s2n, k, kt, b_nodes, bt


def test_zero_model_is_block_jacobi_and_fcg_matches_cg():
    from paper_1908_08666_amd import learned as LG
    lib, orc, s2n, k, kt, b_nodes, bt = _solve_setup()
    net = LG.SmootherNet()                       # all parameters zero
    LG.attach(lib, net)
    Pl = LG.preconditioner(lib, kt, "learned")
    Pb = LG.preconditioner(lib, kt, "block_jacobi")
    assert torch.equal(Pl, Pb)
    x1, i1 = lib.solve(bt, kt, precond="block_jacobi", solver="cg64", rtol=1e-10, check_every=1)
    x2, i2 = lib.solve(bt, kt, precond="learned", solver="cg64", rtol=1e-10, check_every=1)
    assert torch.equal(x1, x2) and i1["iterations"] == i2["iterations"]
    x3, i3 = lib.solve(bt, kt, precond="block_jacobi", solver="fcg64", rtol=1e-10, check_every=1)
    print(f"  CG {i1['iterations']} vs FCG {i3['iterations']} iterations", flush=True)
    assert abs(i1["iterations"] - i3["iterations"]) <= 2
    assert rel_err(x3.cpu().numpy(), x1.cpu().numpy()) <= 1e-8
    # and the oracle agrees on the solution
    Auu, dof = S.reduced_system(orc, k, EFORM)
    xs = S.direct_solve(Auu, b_nodes.ravel()[dof])
    xg = np.zeros((orc.n_nodes, 3))
    xg[s2n] = x3.cpu().numpy().T
    assert rel_err(xg.ravel()[dof], xs) <= 1e-8
    LG.attach(lib, None)


def test_learned_blocks_match_oracle():
    from paper_1908_08666_amd import learned as LG
    lib, orc, s2n, k, kt, b_nodes, bt = _solve_setup()
    w = _random_weights(14, scale2=0.05)
    net = LG.SmootherNet(w)
    LG.attach(lib, net)
    P = LG.preconditioner(lib, kt, "learned").cpu().numpy()
    A = O.operator_matrix(orc, k, EFORM)
    Po = LN.learned_blocks(orc, k, w, A)
    u = orc.unknown
    fl = lib.flags()
    slots = np.nonzero((fl & 1) == 0)[0]
    Pg = LN.sym6_to_mat(P[:, slots].T)
    err = np.abs(Pg - Po[s2n[slots]]).max() / np.abs(Po[u]).max()
    print(f"  learned blocks max rel err {err:.3e}", flush=True)
    assert err <= 1e-3                            # BF16 hidden-unit flips, see forward bound
    assert np.all(P[:, (fl & 1) > 0] == 0)
    # solve with them converges to the oracle's solution
    x, info = lib.solve(bt, kt, precond="learned", solver="fcg64", rtol=1e-10, check_every=4)
    Auu, dof = S.reduced_system(orc, k, EFORM)
    xs = S.direct_solve(Auu, b_nodes.ravel()[dof])
    xg = np.zeros((orc.n_nodes, 3))
    xg[s2n] = x.cpu().numpy().T
    assert rel_err(xg.ravel()[dof], xs) <= 1e-8
    LG.attach(lib, None)


@pytest.fixture(scope="module")
def trained():
    """Records of rough errors (start vector x* + noise, iterates 0..2 of the
    plain solver) on a Carreau-viscosity eps-operator (cube24, level 4,
    viscosity contrast near 1e3), and a network trained on 12,000 of them;
    the held-out loss of the zero network (block Jacobi) and of the trained
    one on the other 2,000."""
    from paper_1908_08666_amd import Mesh
    from paper_1908_08666_amd import learned as LG
    mesh = Mesh(W.cube24(), 4, mu1=1.0)
    xyz = mesh.coords().T
    u = torch.from_numpy(np.ascontiguousarray(
        W.localized_velocity_field(xyz, W.rng_for(5, 0), 1e6).T)).cuda()
    k = mesh.nodal_viscosity(u, **W.CARREAU_DEFAULT)
    owner = (mesh.flags() & 2) > 0
    b = torch.from_numpy(W.consistent_uniform(xyz, owner, W.rng_for(5, 1))).cuda()
    fl = torch.from_numpy(mesh.flags()).cuda()
    b[:, (fl & 1) > 0] = 0
    x0 = torch.from_numpy(W.consistent_uniform(xyz, owner, W.rng_for(5, 2))).cuda()
    rec, xs = LG.solver_pairs(mesh, k, b, x0, 14000, seed=3)
    perm = torch.randperm(rec.shape[0], generator=torch.Generator().manual_seed(0)).cuda()
    rec = rec[perm].contiguous()
    train, held = rec[:12000], rec[12000:]
    net = LG.SmootherNet(W.smoother_init_weights(W.rng_for(5, 4)))
    l0, _ = net.loss_grad(held, held.shape[0])
    hist = net.train(train, train.shape[0], epochs=100, batch=1000, lr=3e-3)
    l1, _ = net.loss_grad(held, held.shape[0])
    print(f"  contrast {float(k.max() / k.min()):.1f}; held-out loss: block Jacobi {l0:.4f} -> "
          f"learned {l1:.4f}; train {hist[0]:.4f} -> {hist[-1]:.4f}", flush=True)
    return dict(mesh=mesh, k=k, b=b, xs=xs, net=net, l0=l0, l1=l1, hist=hist)


def test_training_gain_over_block_jacobi(trained):
    """Training lowers the held-out one-step smoothing error below block
    Jacobi's (the zero network); FCG with the learned blocks reaches 1e-8.
    Both iteration counts are printed: among block-diagonal preconditioners
    block Jacobi minimises Kaporin's condition number, so the learned blocks
    are not asserted to beat it in CG."""
    from paper_1908_08666_amd import learned as LG
    t = trained
    mesh, k, b = t["mesh"], t["k"], t["b"]
    assert t["hist"][-1] < t["hist"][0]
    assert t["l1"] < t["l0"]
    LG.attach(mesh, t["net"])
    _, ib = mesh.solve(b, k, precond="block_jacobi", solver="cg64", rtol=1e-8, check_every=8)
    xl, il = mesh.solve(b, k, precond="learned", solver="fcg64", rtol=1e-8, check_every=8)
    print(f"  iterations to 1e-8: block Jacobi PCG {ib['iterations']}, learned FCG "
          f"{il['iterations']}", flush=True)
    assert il["status"] == "HHG_OK" and il["rel_residual"] <= 1e-8
    assert rel_err(xl.cpu().numpy(), t["xs"].cpu().numpy()) <= 1e-6
    LG.attach(mesh, None)


@pytest.mark.xfail(strict=True, reason="measured negative result: the pointwise 3x3 learned blocks "
                   "lower the held-out one-step error by about 1 %, not 5 %, and do not cut CG "
                   "iterations below block Jacobi's")
def test_training_gain_reaches_five_percent(trained):
    """The gain the learned smoother was meant to show: held-out one-step
    error 5 % below block Jacobi's and fewer FCG iterations than block-Jacobi
    PCG.  Expected to fail (strict): if it ever passes, the recorded negative
    result is out of date."""
    t = trained
    from paper_1908_08666_amd import learned as LG
    mesh, k, b = t["mesh"], t["k"], t["b"]
    assert t["l1"] < 0.95 * t["l0"]
    LG.attach(mesh, t["net"])
    try:
        _, ib = mesh.solve(b, k, precond="block_jacobi", solver="cg64", rtol=1e-8, check_every=8)
        _, il = mesh.solve(b, k, precond="learned", solver="fcg64", rtol=1e-8, check_every=8)
    finally:
        LG.attach(mesh, None)
    assert il["iterations"] < ib["iterations"]


def test_learned_blocks_as_multigrid_smoother(trained):
    """The learned blocks where a pointwise block smoother has headroom: as
    the damped smoother of the V(3,3) cycle on every level above the
    coarsest, against damped block Jacobi in the same cycle, by MG-PCG
    iterations to 1e-8 on the Carreau operator of the training records
    (cube24 level 4, contrast near 1e3).  Measured outcome, asserted as such:
    block Jacobi converges in a dozen iterations; the learned blocks, larger
    than D^-1 in some directions, make the smoother lose its contraction,
    and MG-PCG needs more than twice as many iterations (omega 0.5) or
    converges far more slowly (omega 0.7)."""
    from paper_1908_08666_amd import Multigrid
    t = trained
    k, b = t["k"], t["b"]
    mg = Multigrid(W.cube24(), 4, 2, mu1=1.0)
    try:
        res = {}
        for sm in ("block_jacobi", "learned"):
            mg.set_smoother(sm, t["net"] if sm == "learned" else None)
            mg.setup_coefficient(k)
            for om in (0.5, 0.7):
                _, info = mg.solve(b, rtol=1e-8, maxit=300, method="cg", omega=om, raise_on_status=False)
                res[(sm, om)] = (info["iterations"], info["status"])
        print("  MG-PCG iterations to 1e-8: " + ", ".join(f"{sm} omega {om}: {it} ({st})"
                                                       for (sm, om), (it, st) in res.items()), flush=True)
        for om in (0.5, 0.7):
            it_bj, st_bj = res[("block_jacobi", om)]
            it_l, st_l = res[("learned", om)]
            assert st_bj == "HHG_OK" and it_bj <= 15
            assert it_l > 2 * it_bj or st_l != "HHG_OK"
        # block Jacobi again after the learned blocks: the option is reversible
        mg.set_smoother("block_jacobi")
        mg.setup_coefficient(k)
        _, info = mg.solve(b, rtol=1e-8, maxit=300, method="cg")
        assert (info["iterations"], info["status"]) == res[("block_jacobi", 0.7)]
    finally:
        mg.close()
