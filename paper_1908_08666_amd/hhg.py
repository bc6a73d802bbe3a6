"""Python binding of the C ABI: a macro mesh handle plus operator calls.

Only argument marshalling happens here; every step of an operator
application runs in the HIP kernels of libhhg.so.  Device vectors are torch
tensors on a ROCm device (SoA [3, n_nodes] for vector fields, [n_nodes] for the
coefficient), float64 or float32.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as L


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _prec_of(t):
    import torch
    if t.dtype == torch.float64:
        return L.HHG_F64
    if t.dtype == torch.float32:
        return L.HHG_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev_ptr(t, shape, dtype):
    if not t.is_cuda:
        raise ValueError("device tensor required")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"shape {tuple(t.shape)} != {tuple(shape)}")
    if t.dtype != dtype:
        raise TypeError(f"dtype {t.dtype} != {dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _descriptors(verts, levels, mu0, lam0, mu1, lam1, coupling, dirichlet, corr, khat, iface):
    """hhg_mesh_desc / hhg_op_desc, plus the arrays they point to."""
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    M = verts.shape[0]
    lv = np.ascontiguousarray(np.broadcast_to(np.asarray(levels, dtype=np.int32), (M,)))
    md = L.MeshDesc(M, verts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    lv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    {"conforming": L.HHG_CONFORMING, "independent": L.HHG_INDEPENDENT}[coupling],
                    {"outer": L.HHG_DIRICHLET_OUTER, "none": L.HHG_DIRICHLET_NONE}[dirichlet])
    od = L.OpDesc(mu0, lam0, mu1, lam1,
                  {"physical": L.HHG_CORR_PHYSICAL, "none": L.HHG_CORR_NONE}[corr],
                  {"patch": L.HHG_KHAT_PATCH, "edge": L.HHG_KHAT_EDGE}[khat],
                  {"symmetric": L.HHG_IFACE_SYMMETRIC, "rowwise": L.HHG_IFACE_ROWWISE,
                   "zerosum": L.HHG_IFACE_ZEROSUM}[iface])
    return md, od, (verts, lv)


def _strain_fit(boundary):
    return {"lsq": L.HHG_STRAIN_LSQ, "average": L.HHG_STRAIN_AVERAGE}[boundary]


class Mesh:
    """Handle of a macro mesh with its operator (``hhg_setup_macro``).

    Parameters mirror ``hhg_mesh_desc`` / ``hhg_op_desc``: ``verts`` (M,4,3),
    ``levels`` int or (M,), weights of 2 (mu0 + mu1 k)(eps, eps) +
    (lam0 + lam1 k)(div, div), and the variant flags.
    """

    def __init__(self, verts, levels, mu0=0.0, lam0=0.0, mu1=0.0, lam1=0.0,
                 coupling="conforming", dirichlet="outer", corr="physical",
                 khat="patch", iface="symmetric"):
        md, od, keep = _descriptors(verts, levels, mu0, lam0, mu1, lam1, coupling, dirichlet, corr,
                                    khat, iface)
        h = ctypes.c_void_p()
        self._lib = L.lib()
        L.check(self._lib.hhg_setup_macro(ctypes.byref(md), ctypes.byref(od), ctypes.byref(h)))
        self._owner = None
        self._init_from(h, keep[1])

    @classmethod
    def _borrowed(cls, h, levels, owner):
        """A Mesh view of a handle owned by ``owner`` (never destroyed here)."""
        self = cls.__new__(cls)
        self._lib = L.lib()
        self._owner = owner
        self._init_from(h, levels)
        return self

    def _init_from(self, h, levels):
        self._h = h
        M = len(levels)
        self.n_macro = M
        self.levels = np.asarray(levels, dtype=np.int32).copy()
        nn = ctypes.c_int64()
        nu = ctypes.c_int64()
        off = np.zeros(M + 1, dtype=np.int64)
        L.check(self._lib.hhg_layout(h, ctypes.byref(nn), ctypes.byref(nu),
                                     off.ctypes.data_as(L._I64P)))
        self.n_nodes = int(nn.value)
        self.n_unknown = int(nu.value)
        self.macro_offset = off

    # --------------------------------------------------------------- host
    def coords(self) -> np.ndarray:
        out = np.zeros((3, self.n_nodes), dtype=np.float64)
        L.check(self._lib.hhg_node_coords(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def flags(self) -> np.ndarray:
        out = np.zeros(self.n_nodes, dtype=np.uint8)
        L.check(self._lib.hhg_node_flags(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
        return out

    # ------------------------------------------------------------- device
    def _vec_args(self, x, k, y):
        prec = _prec_of(x)
        dt = x.dtype
        N = self.n_nodes
        return (prec, _dev_ptr(x, (3, N), dt), _dev_ptr(k, (N,), dt), _dev_ptr(y, (3, N), dt))

    def apply_scaled(self, x, k, y=None, stream=None):
        """y = A_s(k) x (``hhg_apply_scaled``)."""
        import torch
        if y is None:
            y = torch.empty_like(x)
        prec, px, pk, py = self._vec_args(x, k, y)
        L.check(self._lib.hhg_apply_scaled(self._h, prec, px, pk, py, _stream_ptr(stream)))
        return y

    def apply_onthefly(self, x, k, y=None, stream=None):
        """y = A_n(k) x (``hhg_apply_onthefly``)."""
        import torch
        if y is None:
            y = torch.empty_like(x)
        prec, px, pk, py = self._vec_args(x, k, y)
        L.check(self._lib.hhg_apply_onthefly(self._h, prec, px, pk, py, _stream_ptr(stream)))
        return y

    def residual(self, f, x, k, r=None, method="scaled", stream=None):
        """r = f - A x (``hhg_residual``)."""
        import torch
        if r is None:
            r = torch.empty_like(x)
        prec, px, pk, pr = self._vec_args(x, k, r)
        pf = _dev_ptr(f, (3, self.n_nodes), x.dtype)
        m = {"scaled": L.HHG_METHOD_SCALED, "onthefly": L.HHG_METHOD_ONTHEFLY}[method]
        L.check(self._lib.hhg_residual(self._h, prec, m, pf, px, pk, pr, _stream_ptr(stream)))
        return r

    # ------------------------------------------------------------ solvers
    def solve_opts(self, solver="cg64", precond="block_jacobi", method="scaled", rtol=1e-8,
                   maxit=20000, inner_rtol=1e-3, check_every=8):
        return L.SolveOpts({"cg64": L.HHG_CG_F64, "ir32": L.HHG_IR_F32, "fcg64": L.HHG_FCG_F64}[solver],
                           {"none": L.HHG_PRECOND_NONE, "block_jacobi": L.HHG_PRECOND_BLOCK_JACOBI,
                            "learned": L.HHG_PRECOND_LEARNED}[precond],
                           {"scaled": L.HHG_METHOD_SCALED, "onthefly": L.HHG_METHOD_ONTHEFLY}[method],
                           int(maxit), float(rtol), float(inner_rtol), int(check_every), 0)

    def workspace_bytes(self, **opts) -> int:
        o = self.solve_opts(**opts)
        n = ctypes.c_size_t()
        L.check(self._lib.hhg_workspace_bytes(self._h, ctypes.byref(o), ctypes.byref(n)))
        return int(n.value)

    def solve(self, b, k, x=None, workspace=None, stream=None, raise_on_status=True, **opts):
        """Solve A x = b (``hhg_cg_solve``); returns (x, info dict).  b, k, x
        are float64 device tensors; x (start vector) defaults to zero."""
        import torch
        N = self.n_nodes
        if x is None:
            x = torch.zeros((3, N), dtype=torch.float64, device=b.device)
        o = self.solve_opts(**opts)
        nbytes = ctypes.c_size_t()
        L.check(self._lib.hhg_workspace_bytes(self._h, ctypes.byref(o), ctypes.byref(nbytes)))
        if workspace is None or workspace.numel() < nbytes.value:
            workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=b.device)
        base = workspace.data_ptr()
        ws = ctypes.c_void_p(base + ((-base) % 256))
        info = L.SolveInfo()
        rc = self._lib.hhg_cg_solve(self._h, ctypes.byref(o), _dev_ptr(b, (3, N), torch.float64),
                                    _dev_ptr(k, (N,), torch.float64), _dev_ptr(x, (3, N), torch.float64),
                                    ws, ctypes.byref(info), _stream_ptr(stream))
        out = dict(iterations=info.iterations, iterations_run=info.iterations_run,
                   outer_iterations=info.outer_iterations,
                   status=L.STATUS_NAMES.get(info.status if rc == L.HHG_OK or info.status else rc, rc),
                   code=rc, rel_residual=info.rel_residual, seconds=info.seconds,
                   message=(self._lib.hhg_last_error() or b"").decode())
        if rc not in (L.HHG_OK,) and raise_on_status:
            L.check(rc)
        return x, out

    # ------------------------------------------------------- viscosity
    def nodal_viscosity(self, u, eta0=1.0, eta_inf=1e-3, kappa=1.0, r=-0.25, k=None,
                        workspace=None, stream=None, boundary="lsq"):
        """Carreau viscosity at the nodes from velocity u (``hhg_nodal_viscosity``);
        boundary: "lsq" (least-squares fit on macro-boundary nodes) or
        "average" (volume-weighted element gradients there)."""
        import torch
        N = self.n_nodes
        if k is None:
            k = torch.empty(N, dtype=torch.float64, device=u.device)
        nb = ctypes.c_size_t()
        L.check(self._lib.hhg_viscosity_workspace_bytes(self._h, ctypes.byref(nb)))
        if workspace is None or workspace.numel() * workspace.element_size() < nb.value:
            workspace = torch.empty(int(nb.value) // 8 + 2, dtype=torch.float64, device=u.device)
        law = L.Carreau(eta0, eta_inf, kappa, r, _strain_fit(boundary))
        L.check(self._lib.hhg_nodal_viscosity(self._h, _dev_ptr(u, (3, N), torch.float64),
                                              ctypes.byref(law), _dev_ptr(k, (N,), torch.float64),
                                              ctypes.c_void_p(workspace.data_ptr()),
                                              _stream_ptr(stream)))
        return k

    # ------------------------------------------------------------ batching
    def autotune(self, x, k, y=None, method="scaled", reps=5, stream=None):
        """Pick slab depth per level and the launch grid (``hhg_autotune``);
        returns (y = A x, report dict)."""
        import torch
        if y is None:
            y = torch.empty_like(x)
        prec, px, pk, py = self._vec_args(x, k, y)
        rep = L.TuneReport()
        m = {"scaled": L.HHG_METHOD_SCALED, "onthefly": L.HHG_METHOD_ONTHEFLY}[method]
        L.check(self._lib.hhg_autotune(self._h, prec, m, px, pk, py, int(reps), ctypes.byref(rep),
                                       _stream_ptr(stream)))
        levels = []
        for q in range(rep.n_levels):
            levels.append(dict(level=rep.level[q], slab=rep.slab[q], macros=rep.macros[q],
                               rows=int(rep.rows[q]), ms=rep.ms[q]))
        return y, dict(levels=levels, persist_blocks=rep.persist_blocks, ms_total=rep.ms_total,
                       candidates=rep.candidates)

    def set_tuning(self, levels=None, slabs=None, persist_blocks=0):
        """Adopt slab depths per level and a grid without timing (``hhg_set_tuning``)."""
        rep = L.TuneReport()
        levels = list(levels or [])
        slabs = list(slabs or [])
        if len(levels) != len(slabs) or len(levels) > 8:
            raise ValueError("levels and slabs: equal length, at most 8")
        rep.n_levels = len(levels)
        for q, (lv, sb) in enumerate(zip(levels, slabs)):
            rep.level[q] = int(lv)
            rep.slab[q] = int(sb)
        rep.persist_blocks = int(persist_blocks)
        L.check(self._lib.hhg_set_tuning(self._h, ctypes.byref(rep)))

    def graph_create(self, x, k, y, method="scaled", count=1):
        """Capture ``count`` applies y = A x in a HIP graph (``hhg_graph_create``)."""
        prec, px, pk, py = self._vec_args(x, k, y)
        m = {"scaled": L.HHG_METHOD_SCALED, "onthefly": L.HHG_METHOD_ONTHEFLY}[method]
        gid = ctypes.c_int32()
        L.check(self._lib.hhg_graph_create(self._h, prec, m, px, pk, py, int(count), ctypes.byref(gid)))
        return int(gid.value)

    def graph_launch(self, graph_id, stream=None):
        L.check(self._lib.hhg_graph_launch(self._h, int(graph_id), _stream_ptr(stream)))

    def graph_destroy(self, graph_id):
        L.check(self._lib.hhg_graph_destroy(self._h, int(graph_id)))

    def stokes_rows(self, op, x=None, hl=0.0, out=None, stream=None):
        """One term of the generalized Stokes system (``hhg_stokes_rows``):
        op "div" (x [3, n] -> [n]), "grad" ([n] -> [3, n]), "stab" ([n] -> [n],
        mesh width hl) or "mass" (-> [n])."""
        import torch
        code = {"div": L.HHG_STOKES_DIV, "grad": L.HHG_STOKES_GRAD, "stab": L.HHG_STOKES_STAB,
                "mass": L.HHG_STOKES_MASS}[op]
        N = self.n_nodes
        in_shape = (3, N) if op == "div" else (N,)
        out_shape = (3, N) if op == "grad" else (N,)
        dev = x.device if x is not None else torch.device("cuda")
        if out is None:
            out = torch.empty(out_shape, dtype=torch.float64, device=dev)
        px = _dev_ptr(x, in_shape, torch.float64) if x is not None else ctypes.c_void_p(0)
        L.check(self._lib.hhg_stokes_rows(self._h, code, float(hl), px,
                                          _dev_ptr(out, out_shape, torch.float64), _stream_ptr(stream)))
        return out

    # ------------------------------------------------------------ tracing
    def profile_enable(self, on=True):
        L.check(self._lib.hhg_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """{kernel name: (launches, total ms)} since profiling was enabled."""
        out = {}
        for kid, name in L.KERNEL_NAMES.items():
            n = ctypes.c_int64()
            ms = ctypes.c_double()
            L.check(self._lib.hhg_profile_read(self._h, kid, ctypes.byref(n), ctypes.byref(ms)))
            out[name] = (int(n.value), float(ms.value))
        return out

    def close(self):
        if getattr(self, "_h", None):
            if getattr(self, "_owner", None) is None:
                self._lib.hhg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Multigrid:
    """Geometric multigrid hierarchy (``hhg_mg_create``): levels
    ``coarse_level..level`` of one conforming macro mesh with the scaled
    operator, P1 transfers, damped block-Jacobi V-cycles and V-cycle
    preconditioned CG.  ``meshes[q]`` is a Mesh view of level
    ``coarse_level + q`` (slot layout of the vectors on that level)."""

    def __init__(self, verts, level, coarse_level=2, mu0=0.0, lam0=0.0, mu1=0.0, lam1=0.0,
                 dirichlet="outer", corr="physical", khat="patch", iface="symmetric"):
        md, od, _keep = _descriptors(verts, level, mu0, lam0, mu1, lam1, "conforming", dirichlet,
                                     corr, khat, iface)
        self._lib = L.lib()
        mg = ctypes.c_void_p()
        L.check(self._lib.hhg_mg_create(ctypes.byref(md), ctypes.byref(od), int(coarse_level),
                                        ctypes.byref(mg)))
        self._mg = mg
        self.coarse_level = int(coarse_level)
        self.level = int(level)
        M = np.asarray(verts).shape[0]
        self.meshes = []
        for lev in range(self.coarse_level, self.level + 1):
            h = ctypes.c_void_p()
            L.check(self._lib.hhg_mg_level(mg, lev, ctypes.byref(h)))
            self.meshes.append(Mesh._borrowed(h, [lev] * M, self))
        self._ws = None

    def mesh(self, level) -> "Mesh":
        return self.meshes[level - self.coarse_level]

    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t()
        L.check(self._lib.hhg_mg_workspace_bytes(self._mg, ctypes.byref(n)))
        return int(n.value)

    def _workspace(self, device):
        import torch
        nb = self.workspace_bytes()
        if self._ws is None or self._ws.numel() < nb + 256 or self._ws.device != device:
            self._ws = torch.empty(nb + 256, dtype=torch.uint8, device=device)
        base = self._ws.data_ptr()
        return ctypes.c_void_p(base + ((-base) % 256))

    @staticmethod
    def _opts(nu1, nu2, omega, rtol=1e-8, maxit=100, method="cg", precision="f64", nu_inc=0):
        m = {"cg": L.HHG_MG_CG, "cycle": L.HHG_MG_CYCLE}[method]
        p = {"f64": L.HHG_F64, "f32": L.HHG_F32}[precision]
        return L.MgOpts(int(nu1), int(nu2), float(omega), float(rtol), int(maxit), m, p, int(nu_inc))

    def prolong(self, fine_level, xc, xf=None, stream=None):
        """xf = P xc (``hhg_mg_prolong``)."""
        import torch
        c, f = self.mesh(fine_level - 1), self.mesh(fine_level)
        if xf is None:
            xf = torch.empty((3, f.n_nodes), dtype=torch.float64, device=xc.device)
        L.check(self._lib.hhg_mg_prolong(self._mg, int(fine_level),
                                          _dev_ptr(xc, (3, c.n_nodes), torch.float64),
                                          _dev_ptr(xf, (3, f.n_nodes), torch.float64),
                                          _stream_ptr(stream)))
        return xf

    def restrict(self, fine_level, rf, rc=None, stream=None):
        """rc = P^T rf (``hhg_mg_restrict``)."""
        import torch
        c, f = self.mesh(fine_level - 1), self.mesh(fine_level)
        if rc is None:
            rc = torch.empty((3, c.n_nodes), dtype=torch.float64, device=rf.device)
        L.check(self._lib.hhg_mg_restrict(self._mg, int(fine_level),
                                           _dev_ptr(rf, (3, f.n_nodes), torch.float64),
                                           _dev_ptr(rc, (3, c.n_nodes), torch.float64),
                                           _stream_ptr(stream)))
        return rc

    def set_smoother(self, smoother="block_jacobi", net=None):
        """Blocks of the damped smoother above the coarsest level
        (``hhg_mg_set_smoother``): "block_jacobi", or "learned" with the
        network ``net`` (a learned.SmootherNet) attached to those levels."""
        from . import learned as LG
        for q, mesh in enumerate(self.meshes):
            LG.attach(mesh, net if (smoother == "learned" and q > 0) else None)
        pc = {"block_jacobi": L.HHG_PRECOND_BLOCK_JACOBI, "learned": L.HHG_PRECOND_LEARNED}[smoother]
        L.check(self._lib.hhg_mg_set_smoother(self._mg, pc))

    def setup_coefficient(self, k, method="scaled", stream=None):
        """Inject k (finest level, float64) and build every level's blocks
        and the coarse inverse for the scaled or the nodal-integration
        ("onthefly") operator (``hhg_mg_setup_coefficient``)."""
        import torch
        f = self.meshes[-1]
        ws = self._workspace(k.device)
        m = {"scaled": L.HHG_METHOD_SCALED, "onthefly": L.HHG_METHOD_ONTHEFLY}[method]
        L.check(self._lib.hhg_mg_setup_coefficient(self._mg, m, _dev_ptr(k, (f.n_nodes,), torch.float64),
                                                    ws, _stream_ptr(stream)))

    def vcycle(self, r, z=None, nu1=3, nu2=3, omega=0.7, precision="f64", stream=None, nu_inc=0):
        """z = V(r) on the finest level (``hhg_mg_vcycle``); precision "f32"
        runs the cycle in FP32 on rounded copies of r and z; nu_inc extra
        smoothing steps per coarser level (the variable V-cycle: 2)."""
        import torch
        f = self.meshes[-1]
        if z is None:
            z = torch.empty_like(r)
        o = self._opts(nu1, nu2, omega, precision=precision, nu_inc=nu_inc)
        L.check(self._lib.hhg_mg_vcycle(self._mg, ctypes.byref(o), _dev_ptr(r, (3, f.n_nodes), torch.float64),
                                        _dev_ptr(z, (3, f.n_nodes), torch.float64),
                                        self._workspace(r.device), _stream_ptr(stream)))
        return z

    def solve(self, b, x=None, nu1=3, nu2=3, omega=0.7, rtol=1e-8, maxit=100, method="cg",
              precision="f64", stream=None, raise_on_status=True, nu_inc=0):
        """A x = b by V-cycle-preconditioned CG (method "cg") or the V-cycle
        iteration (method "cycle") (``hhg_mg_solve``); call setup_coefficient
        first.  precision "f32" runs the V-cycles in FP32 (the outer
        iteration stays FP64).  Returns (x, info dict)."""
        import torch
        f = self.meshes[-1]
        if x is None:
            x = torch.zeros((3, f.n_nodes), dtype=torch.float64, device=b.device)
        o = self._opts(nu1, nu2, omega, rtol, maxit, method, precision, nu_inc)
        info = L.SolveInfo()
        rc = self._lib.hhg_mg_solve(self._mg, ctypes.byref(o), _dev_ptr(b, (3, f.n_nodes), torch.float64),
                                    _dev_ptr(x, (3, f.n_nodes), torch.float64), self._workspace(b.device),
                                    ctypes.byref(info), _stream_ptr(stream))
        out = dict(iterations=info.iterations, status=L.STATUS_NAMES.get(info.status, info.status),
                   code=rc, rel_residual=info.rel_residual, seconds=info.seconds,
                   message=(self._lib.hhg_last_error() or b"").decode())
        if rc != L.HHG_OK and raise_on_status:
            L.check(rc)
        return x, out

    # ------------------------------------------------ generalized Stokes
    def _stokes_workspace(self, device):
        import torch
        n = ctypes.c_size_t()
        L.check(self._lib.hhg_mg_stokes_workspace_bytes(self._mg, ctypes.byref(n)))
        nb = int(n.value)
        ws = getattr(self, "_sws", None)
        if ws is None or ws.numel() < nb + 256 or ws.device != device:
            self._sws = torch.empty(nb + 256, dtype=torch.uint8, device=device)
        base = self._sws.data_ptr()
        return ctypes.c_void_p(base + ((-base) % 256))

    @staticmethod
    def _stokes_opts(nu1, nu2, omega, omega_p, h, rtol, maxit, nu_inc=0):
        return L.StokesOpts(int(nu1), int(nu2), float(omega), float(omega_p), float(h), float(rtol),
                            int(maxit), int(nu_inc))

    def stokes_solve(self, f, mu, u=None, p=None, g=None, nu1=3, nu2=3, omega=0.7, omega_p=1.0,
                     h=0.0, rtol=1e-8, maxit=500, stream=None, raise_on_status=True, nu_inc=0):
        """Inexact Uzawa for the generalized Stokes system on the finest
        level (``hhg_mg_stokes_solve``); call setup_coefficient(mu) first.
        nu_inc: extra velocity smoothing steps per coarser level.
        Returns (u, p, info dict)."""
        import torch
        fm = self.meshes[-1]
        N = fm.n_nodes
        if u is None:
            u = torch.zeros((3, N), dtype=torch.float64, device=f.device)
        if p is None:
            p = torch.zeros((N,), dtype=torch.float64, device=f.device)
        o = self._stokes_opts(nu1, nu2, omega, omega_p, h, rtol, maxit, nu_inc)
        info = L.SolveInfo()
        gp = _dev_ptr(g, (N,), torch.float64) if g is not None else ctypes.c_void_p(0)
        rc = self._lib.hhg_mg_stokes_solve(self._mg, ctypes.byref(o), _dev_ptr(f, (3, N), torch.float64), gp,
                                           _dev_ptr(mu, (N,), torch.float64), _dev_ptr(u, (3, N), torch.float64),
                                           _dev_ptr(p, (N,), torch.float64), self._workspace(f.device),
                                           self._stokes_workspace(f.device), ctypes.byref(info),
                                           _stream_ptr(stream))
        out = dict(iterations=info.iterations, status=L.STATUS_NAMES.get(info.status, info.status),
                   code=rc, rel_residual=info.rel_residual, seconds=info.seconds)
        if rc != L.HHG_OK and raise_on_status:
            L.check(rc)
        return u, p, out

    def stokes_picard(self, f, eta0, eta_inf, kappa, r, method="scaled", max_picard=100, nu1=3, nu2=3,
                      omega=0.7, omega_p=1.0, h=0.0, rtol=1e-3, maxit=500, stream=None,
                      raise_on_status=True, boundary="lsq", nu_inc=0):
        """Fixed-point iteration for the Carreau fluid (``hhg_mg_stokes_picard``);
        boundary: the strain-rate fit on macro-boundary nodes ("lsq" or
        "average").  Returns (u, p, mu, info dict)."""
        import torch
        fm = self.meshes[-1]
        N = fm.n_nodes
        u = torch.empty((3, N), dtype=torch.float64, device=f.device)
        p = torch.empty((N,), dtype=torch.float64, device=f.device)
        mu = torch.empty((N,), dtype=torch.float64, device=f.device)
        o = self._stokes_opts(nu1, nu2, omega, omega_p, h, rtol, maxit, nu_inc)
        law = L.Carreau(float(eta0), float(eta_inf), float(kappa), float(r), _strain_fit(boundary))
        m = {"scaled": L.HHG_METHOD_SCALED, "onthefly": L.HHG_METHOD_ONTHEFLY}[method]
        info = L.PicardInfo()
        rc = self._lib.hhg_mg_stokes_picard(self._mg, ctypes.byref(o), ctypes.byref(law), m, int(max_picard),
                                            _dev_ptr(f, (3, N), torch.float64), _dev_ptr(u, (3, N), torch.float64),
                                            _dev_ptr(p, (N,), torch.float64), _dev_ptr(mu, (N,), torch.float64),
                                            self._workspace(f.device), self._stokes_workspace(f.device),
                                            ctypes.byref(info), _stream_ptr(stream))
        out = dict(picard=info.picard, final_iterations=info.final_iterations,
                   status=L.STATUS_NAMES.get(info.status, info.status), code=rc, rel_change=info.rel_change,
                   rel_residual=info.rel_residual, seconds=info.seconds)
        if rc != L.HHG_OK and raise_on_status:
            L.check(rc)
        return u, p, mu, out

    def close(self):
        for m in getattr(self, "meshes", []):
            m._h = None
        self.meshes = []
        if getattr(self, "_mg", None):
            self._lib.hhg_mg_destroy(self._mg)
            self._mg = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
