"""Binding of the learned 3x3 block smoother (``hhg_mlp_*``, ``hhg_learn_*``).

Argument marshalling only: features, inference, training-record collection,
gradients and Adam training all run in the library's kernels.  Device
buffers are torch tensors.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as L
from .hhg import Mesh, _stream_ptr, _dev_ptr

N_PARAM = L.HHG_MLP_NPARAM
RECORD_BYTES = L.HHG_SAMPLE_BYTES


class SmootherNet:
    """Handle of the network (16 -> 64 -> 9) on the current device; starts
    with all parameters zero (block Jacobi)."""

    def __init__(self, weights=None):
        self._lib = L.lib()
        h = ctypes.c_void_p()
        L.check(self._lib.hhg_mlp_create(ctypes.byref(h)))
        self._h = h
        if weights is not None:
            self.set_weights(weights)

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.shape != (N_PARAM,):
            raise ValueError(f"expected {N_PARAM} parameters")
        L.check(self._lib.hhg_mlp_set_weights(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_weights(self) -> np.ndarray:
        w = np.zeros(N_PARAM, dtype=np.float32)
        L.check(self._lib.hhg_mlp_get_weights(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return w

    def forward(self, feat, stride=16, n=None, out=None, stream=None):
        """Outputs [n, 9] float32 of feature records (uint16 BF16 patterns,
        record q at q * stride)."""
        import torch
        if n is None:
            n = feat.numel() // stride
        if out is None:
            out = torch.empty((n, 9), dtype=torch.float32, device=feat.device)
        L.check(self._lib.hhg_mlp_forward(self._h, ctypes.c_void_p(feat.data_ptr()), int(stride), int(n),
                                          ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def loss_grad(self, records, n, stream=None):
        loss = ctypes.c_double()
        g = np.zeros(N_PARAM, dtype=np.float32)
        L.check(self._lib.hhg_mlp_loss_grad(self._h, ctypes.c_void_p(records.data_ptr()), int(n),
                                            ctypes.byref(loss),
                                            g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                            _stream_ptr(stream)))
        return float(loss.value), g

    def train(self, records, n, epochs=100, batch=2048, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              stream=None):
        """Adam on the device; returns the per-epoch mean loss (numpy)."""
        o = L.TrainOpts(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps))
        hist = np.zeros(int(epochs), dtype=np.float32)
        L.check(self._lib.hhg_mlp_train(self._h, ctypes.c_void_p(records.data_ptr()), int(n),
                                        ctypes.byref(o),
                                        hist.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                        _stream_ptr(stream)))
        return hist

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hhg_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def features(mesh: Mesh, k, out=None, stream=None):
    """BF16 features [n_nodes, 16] (uint16 patterns as int16 tensor) of every slot."""
    import torch
    if out is None:
        out = torch.empty((mesh.n_nodes, 16), dtype=torch.int16, device=k.device)
    L.check(mesh._lib.hhg_learn_features(mesh._h, _dev_ptr(k, (mesh.n_nodes,), torch.float64),
                                         ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def collect(mesh: Mesh, k, r, e, slots, method="scaled", stream=None):
    """Training records (uint8 tensor [n, 128]) of the given slots from the
    residual r and error e of a solver iterate."""
    import torch
    N = mesh.n_nodes
    n = int(slots.numel())
    rec = torch.empty((n, RECORD_BYTES), dtype=torch.uint8, device=k.device)
    m = {"scaled": L.HHG_METHOD_SCALED, "onthefly": L.HHG_METHOD_ONTHEFLY}[method]
    L.check(mesh._lib.hhg_learn_collect(mesh._h, m, _dev_ptr(k, (N,), torch.float64),
                                        _dev_ptr(r, (3, N), torch.float64), _dev_ptr(e, (3, N), torch.float64),
                                        _dev_ptr(slots, (n,), torch.int64), n,
                                        ctypes.c_void_p(rec.data_ptr()), _stream_ptr(stream)))
    return rec


def attach(mesh: Mesh, net: SmootherNet | None):
    """Use ``net`` for precond="learned" solves of ``mesh`` (None detaches)."""
    L.check(mesh._lib.hhg_set_learned_model(mesh._h, net._h if net is not None else None))
    mesh._learned = net


def preconditioner(mesh: Mesh, k, precond="learned", method="scaled", stream=None, P=None,
                   noalloc=False):
    """Preconditioner blocks [6, n_nodes] (xx yy zz xy xz yz) a solve would
    use; noalloc=True calls the allocation-free entry point (P may then be
    passed in, so that nothing is allocated on this path either)."""
    import torch
    N = mesh.n_nodes
    if P is None:
        P = torch.empty((6, N), dtype=torch.float64, device=k.device)
    pc = {"none": L.HHG_PRECOND_NONE, "block_jacobi": L.HHG_PRECOND_BLOCK_JACOBI,
          "learned": L.HHG_PRECOND_LEARNED}[precond]
    m = {"scaled": L.HHG_METHOD_SCALED, "onthefly": L.HHG_METHOD_ONTHEFLY}[method]
    fn = mesh._lib.hhg_preconditioner_noalloc if noalloc else mesh._lib.hhg_preconditioner
    L.check(fn(mesh._h, pc, m, _dev_ptr(k, (N,), torch.float64), _dev_ptr(P, (6, N), torch.float64),
               _stream_ptr(stream)))
    return P


def solver_pairs(mesh: Mesh, k, b, noise, n_records, iters=(0, 1, 2), seed=0,
                 method="scaled", workspace=None):
    """Training records from the plain solver (FP64 block-Jacobi CG): its
    solution x* to rtol 1e-11, the start vector x0 = x* + max|x*| noise
    (``noise`` a consistent vector, e.g. U(-1, 1) per node), so that the
    error starts rough, the iterates x_j after j = ``iters`` iterations from
    x0, and at random unknown nodes of each iterate the record of
    r = b - A x_j, e = x* - x_j.  Returns (records uint8 [n, 128], x*)."""
    import torch
    dev = b.device
    xs, info = mesh.solve(b, k, x=torch.zeros_like(b), workspace=workspace, rtol=1e-11,
                          check_every=16, method=method)
    fl = torch.from_numpy(mesh.flags()).to(dev)
    x0 = xs + float(xs.abs().max()) * noise
    x0[:, (fl & 1) > 0] = 0.0
    cand = torch.nonzero((fl & 3) == 2).flatten()
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    per = [n_records // len(iters) + (1 if q < n_records % len(iters) else 0) for q in range(len(iters))]
    out = []
    for j, cnt in zip(iters, per):
        x = x0.clone()
        if j > 0:
            x, _ = mesh.solve(b, k, x=x, workspace=workspace, rtol=1e-300, maxit=int(j), check_every=1,
                              method=method, raise_on_status=False)
        r = mesh.residual(b, x, k, method=method)
        e = xs - x
        pick = cand[torch.randperm(cand.numel(), generator=g)[:cnt].to(dev)]
        out.append(collect(mesh, k, r, e, pick.contiguous(), method=method))
    return torch.cat(out), xs
