"""Python-side names of the C ABI (include/qiral.h), taking torch tensors.

Canonical fields are contiguous complex128 CUDA tensors shaped
(nrhs, Lt, Lz, Ly, Lx, 3, 4) (colour, spin); canonical links are contiguous
complex128 CUDA tensors shaped (Lt, Lz, Ly, Lx, 4, 3, 3).  Packed fields are
uint8 CUDA tensors of qiral_field_bytes() bytes.  These wrappers check tensor
types and sizes, pass raw pointers and the current torch stream, and raise
QiralError on a non-OK status; they compute nothing themselves.
"""
import ctypes

import torch

from . import _lib as L


def _stream(stream=None):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _need_cuda(t, name, dtype=None, nbytes=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, not {t.dtype}")
    if nbytes is not None and t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{name} holds {t.numel() * t.element_size()} bytes, needs {nbytes}")
    return ctypes.c_void_p(t.data_ptr())


def _volume(dims):
    v = 1
    for d in dims:
        v *= int(d)
    return v


def qiral_field_bytes(dims, subset, prec, nrhs=1):
    return int(L.load().qiral_field_bytes(L.dims_arg(dims), subset, prec, nrhs))


def qiral_gauge_bytes(dims, prec, recon=None):
    if recon is None:
        recon = L.RECON18 if prec == L.F64 else L.RECON12
    return int(L.load().qiral_gauge_bytes(L.dims_arg(dims), prec, recon))


def _bytes_tensor(n, device="cuda"):
    """A device buffer of n bytes (uint8; torch's allocations are 512-byte aligned)."""
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


def qiral_lattice_create(dims, kappa, gauge_canon, gauge_f64, gauge_f32=None, gauge_f16=None, mu=0.0, stream=None):
    """Create a handle whose packed links live in the given uint8 CUDA tensors
    (sized by qiral_gauge_bytes); they must outlive the handle."""
    lib = L.load()
    ptr = _need_cuda(gauge_canon, "gauge_canon", torch.complex128, _volume(dims) * 4 * 9 * 16)
    g64 = _need_cuda(gauge_f64, "gauge_f64", nbytes=qiral_gauge_bytes(dims, L.F64))
    g32 = ctypes.c_void_p(None) if gauge_f32 is None else \
        _need_cuda(gauge_f32, "gauge_f32", nbytes=qiral_gauge_bytes(dims, L.F32))
    g16 = ctypes.c_void_p(None) if gauge_f16 is None else \
        _need_cuda(gauge_f16, "gauge_f16", nbytes=qiral_gauge_bytes(dims, L.F16S))
    h = ctypes.c_void_p()
    L.check(lib.qiral_lattice_create(ctypes.byref(h), L.dims_arg(dims), float(kappa), float(mu), ptr, g64, g32, g16,
                                     _stream(stream)), "qiral_lattice_create")
    return h.value


def qiral_lattice_destroy(handle):
    L.check(L.load().qiral_lattice_destroy(ctypes.c_void_p(handle)), "qiral_lattice_destroy")


def qiral_field_import(handle, dims, dst, src_canon, subset, prec, nrhs=1, stream=None):
    need = qiral_field_bytes(dims, subset, prec, nrhs)
    d = _need_cuda(dst, "dst", nbytes=need)
    s = _need_cuda(src_canon, "src_canon", torch.complex128, _volume(dims) * 12 * 16 * nrhs)
    L.check(L.load().qiral_field_import(ctypes.c_void_p(handle), d, s, subset, prec, nrhs, _stream(stream)),
            "qiral_field_import")


def qiral_field_export(handle, dims, dst_canon, src, subset, prec, nrhs=1, stream=None):
    need = qiral_field_bytes(dims, subset, prec, nrhs)
    d = _need_cuda(dst_canon, "dst_canon", torch.complex128, _volume(dims) * 12 * 16 * nrhs)
    s = _need_cuda(src, "src", nbytes=need)
    L.check(L.load().qiral_field_export(ctypes.c_void_p(handle), d, s, subset, prec, nrhs, _stream(stream)),
            "qiral_field_export")


def qiral_dslash_eo(handle, dims, out, inp, out_parity, dagger, prec, nrhs=1, stream=None):
    need = qiral_field_bytes(dims, L.EVEN, prec, nrhs)
    o = _need_cuda(out, "out", nbytes=need)
    i = _need_cuda(inp, "in", nbytes=need)
    L.check(L.load().qiral_dslash_eo(ctypes.c_void_p(handle), o, i, int(out_parity), int(dagger), prec, nrhs,
                                     _stream(stream)), "qiral_dslash_eo")


def qiral_apply_M(handle, dims, out, inp, tmp, op, prec, nrhs=1, stream=None):
    subset = L.FULL if op in (L.OP_D, L.OP_DDAG) else L.ODD
    need = qiral_field_bytes(dims, subset, prec, nrhs)
    o = _need_cuda(out, "out", nbytes=need)
    i = _need_cuda(inp, "in", nbytes=need)
    t = ctypes.c_void_p(None) if tmp is None else _need_cuda(tmp, "tmp", nbytes=qiral_field_bytes(dims, L.EVEN, prec, nrhs))
    L.check(L.load().qiral_apply_M(ctypes.c_void_p(handle), o, i, t, int(op), prec, nrhs, _stream(stream)),
            "qiral_apply_M")


def qiral_tune(handle, dims, prec, inp, out, nrhs=1, stream=None):
    """Autotune the hop launch shape on two caller half-fields; returns (waves per
    site block, rhs per lane, microseconds)."""
    need = qiral_field_bytes(dims, L.EVEN, prec, nrhs)
    i = _need_cuda(inp, "in", nbytes=need)
    o = _need_cuda(out, "out", nbytes=need)
    t, nr, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    L.check(L.load().qiral_tune(ctypes.c_void_p(handle), int(prec), int(nrhs), i, o, ctypes.byref(t),
                                ctypes.byref(nr), ctypes.byref(us), _stream(stream)), "qiral_tune")
    return t.value, nr.value, us.value


def solve_params(solver=L.CGNR_EO, tol=1e-10, maxiter=10000, inner_prec=L.F64, delta=0.01, restart=20, precond=None,
                 fallback_cg=1, x0_is_guess=0, use_graph=0, check_every=0, system=L.SYSTEM_DEFAULT):
    return L.SolveParams(solver, tol, maxiter, inner_prec, delta, restart, precond, fallback_cg, x0_is_guess,
                         use_graph, check_every, system)


def qiral_solve_workspace_bytes(handle, params, nrhs=1):
    return int(L.load().qiral_solve_workspace_bytes(ctypes.c_void_p(handle), ctypes.byref(params), int(nrhs)))


def qiral_solve_batch_workspace_bytes(handles, params):
    n = len(handles)
    hp = (ctypes.c_void_p * n)(*handles)
    return int(L.load().qiral_solve_batch_workspace_bytes(hp, n, ctypes.byref(params)))


def _ws_arg(ws):
    if ws is None:
        return ctypes.c_void_p(None), 0
    return _need_cuda(ws, "ws"), ws.numel() * ws.element_size()


def qiral_solve(handle, dims, x_canon, b_canon, nrhs, params, ws="auto", stream=None):
    """ws: a uint8 CUDA tensor of at least qiral_solve_workspace_bytes bytes, None
    (passes NULL), or "auto" (a torch tensor of the queried size for this call)."""
    n = _volume(dims) * 12 * 16 * nrhs
    x = _need_cuda(x_canon, "x_canon", torch.complex128, n)
    b = _need_cuda(b_canon, "b_canon", torch.complex128, n)
    if isinstance(ws, str):
        need = qiral_solve_workspace_bytes(handle, params, nrhs)
        ws = _bytes_tensor(need) if need else None
    wp, wn = _ws_arg(ws)
    infos = (L.SolveInfo * nrhs)()
    st = L.load().qiral_solve(ctypes.c_void_p(handle), x, b, nrhs, ctypes.byref(params), wp, wn, infos,
                              _stream(stream))
    if st not in (L.OK, L.ERR_NOT_CONVERGED):
        L.check(st, "qiral_solve")
    return st, [i.as_dict() for i in infos]


def qiral_solve_static(handle, dims, x_canon, b_canon, nrhs, params, stream=None):
    """qiral_solve in the library's static device workspace (no allocation)."""
    n = _volume(dims) * 12 * 16 * nrhs
    x = _need_cuda(x_canon, "x_canon", torch.complex128, n)
    b = _need_cuda(b_canon, "b_canon", torch.complex128, n)
    infos = (L.SolveInfo * nrhs)()
    st = L.load().qiral_solve_static(ctypes.c_void_p(handle), x, b, nrhs, ctypes.byref(params), infos,
                                     _stream(stream))
    if st not in (L.OK, L.ERR_NOT_CONVERGED):
        L.check(st, "qiral_solve_static")
    return st, [i.as_dict() for i in infos]


def qiral_solve_batch(handles, dims_list, xs, bs, params, ws="auto", stream=None):
    n = len(handles)
    hp = (ctypes.c_void_p * n)(*handles)
    xp = (ctypes.c_void_p * n)(*[_need_cuda(x, "x", torch.complex128, _volume(d) * 192).value
                                 for x, d in zip(xs, dims_list)])
    bp = (ctypes.c_void_p * n)(*[_need_cuda(b, "b", torch.complex128, _volume(d) * 192).value
                                 for b, d in zip(bs, dims_list)])
    if isinstance(ws, str):
        need = qiral_solve_batch_workspace_bytes(handles, params)
        ws = _bytes_tensor(need) if need else None
    wp, wn = _ws_arg(ws)
    infos = (L.SolveInfo * n)()
    st = L.load().qiral_solve_batch(hp, xp, bp, n, ctypes.byref(params), wp, wn, infos, _stream(stream))
    if st not in (L.OK, L.ERR_NOT_CONVERGED):
        L.check(st, "qiral_solve_batch")
    return st, [i.as_dict() for i in infos]


class Lattice:
    """A lattice handle: dims, kappa, twisted mass mu and packed links on the
    current CUDA device."""

    def __init__(self, dims, kappa, gauge, lo_precs=L.LINKS_F32 | L.LINKS_F16, device="cuda", mu=0.0):
        self.dims = tuple(int(d) for d in dims)
        self.kappa = float(kappa)
        self.mu = float(mu)
        g = gauge if isinstance(gauge, torch.Tensor) else torch.from_numpy(gauge)
        g = g.to(device=device, dtype=torch.complex128).contiguous()
        # the packed link stores: device memory this object owns for the handle's lifetime
        self.gauge_f64 = _bytes_tensor(qiral_gauge_bytes(self.dims, L.F64), device)
        self.gauge_f32 = _bytes_tensor(qiral_gauge_bytes(self.dims, L.F32), device) if lo_precs & L.LINKS_F32 else None
        self.gauge_f16 = _bytes_tensor(qiral_gauge_bytes(self.dims, L.F16S), device) if lo_precs & L.LINKS_F16 else None
        self.handle = qiral_lattice_create(self.dims, self.kappa, g, self.gauge_f64, self.gauge_f32, self.gauge_f16,
                                           mu=self.mu)
        self.ws = None

    def close(self):
        if self.handle:
            qiral_lattice_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def field(self, subset, prec, nrhs=1):
        n = qiral_field_bytes(self.dims, subset, prec, nrhs)
        return torch.zeros(n, dtype=torch.uint8, device="cuda")

    def canon(self, nrhs=1):
        lx, ly, lz, lt = self.dims
        return torch.zeros((nrhs, lt, lz, ly, lx, 3, 4), dtype=torch.complex128, device="cuda")

    def import_field(self, canon, subset, prec):
        canon = canon.contiguous()
        nrhs = canon.shape[0]
        dst = self.field(subset, prec, nrhs)
        qiral_field_import(self.handle, self.dims, dst, canon, subset, prec, nrhs)
        return dst

    def export_field(self, packed, subset, prec, nrhs=1, out=None):
        out = self.canon(nrhs) if out is None else out
        qiral_field_export(self.handle, self.dims, out, packed, subset, prec, nrhs)
        return out

    def dslash_eo(self, out, inp, out_parity, dagger, prec, nrhs=1):
        qiral_dslash_eo(self.handle, self.dims, out, inp, out_parity, dagger, prec, nrhs)

    def apply_M(self, out, inp, tmp, op, prec, nrhs=1):
        qiral_apply_M(self.handle, self.dims, out, inp, tmp, op, prec, nrhs)

    def tune(self, prec, nrhs=1):
        a, b = self.field(L.EVEN, prec, nrhs), self.field(L.EVEN, prec, nrhs)
        return qiral_tune(self.handle, self.dims, prec, a, b, nrhs)

    def workspace(self, params, nrhs=1):
        """The solver workspace for these parameters, kept and grown on demand."""
        need = qiral_solve_workspace_bytes(self.handle, params, nrhs)
        if self.ws is None or self.ws.numel() < need:
            self.ws = None
            self.ws = _bytes_tensor(need)
        return self.ws

    def solve(self, b_canon, x_canon=None, **kw):
        b_canon = b_canon.contiguous()
        nrhs = b_canon.shape[0]
        x = self.canon(nrhs) if x_canon is None else x_canon
        prm = solve_params(**kw)
        st, info = qiral_solve(self.handle, self.dims, x, b_canon, nrhs, prm, ws=self.workspace(prm, nrhs))
        return x, st, info


class Network:
    """The learned preconditioner of a lattice (qiral_nn_*): weights as a complex64
    numpy array of shape (2, 9, hidden, 4, 4) view of layers [9][H][1] and [9][1][H]."""

    def __init__(self, lattice, hidden=8):
        import numpy as np
        self.lat = lattice
        self.hidden = hidden
        h = ctypes.c_void_p()
        nbytes = int(L.load().qiral_nn_bytes(ctypes.c_void_p(lattice.handle), int(hidden)))
        self.mem = _bytes_tensor(nbytes)   # the network's device memory, owned here
        L.check(L.load().qiral_nn_create(ctypes.byref(h), ctypes.c_void_p(lattice.handle), int(hidden),
                                         _need_cuda(self.mem, "mem"), nbytes, _stream()), "qiral_nn_create")
        self.handle = h.value
        self.nw = int(L.load().qiral_nn_num_weights(ctypes.c_void_p(self.handle)))
        self._np = np

    def close(self):
        if self.handle:
            L.check(L.load().qiral_nn_destroy(ctypes.c_void_p(self.handle)), "qiral_nn_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_weights(self):
        """(w1 [9][H][1][4][4], w2 [9][1][H][4][4]) complex64."""
        np = self._np
        buf = np.zeros(2 * self.nw, dtype=np.float32)
        L.check(L.load().qiral_nn_get_weights(ctypes.c_void_p(self.handle), buf.ctypes.data_as(ctypes.c_void_p),
                                              self.nw, _stream()), "qiral_nn_get_weights")
        c = buf.view(np.complex64)
        H = self.hidden
        n1 = 9 * H * 16
        return c[:n1].reshape(9, H, 1, 4, 4).copy(), c[n1:].reshape(9, 1, H, 4, 4).copy()

    def set_weights(self, w1, w2):
        np = self._np
        c = np.concatenate([np.asarray(w1, np.complex64).ravel(), np.asarray(w2, np.complex64).ravel()])
        assert c.size == self.nw
        buf = np.ascontiguousarray(c).view(np.float32)
        L.check(L.load().qiral_nn_set_weights(ctypes.c_void_p(self.handle), buf.ctypes.data_as(ctypes.c_void_p),
                                              self.nw, _stream()), "qiral_nn_set_weights")

    def apply(self, out, inp, adjoint=False):
        fn = L.load().qiral_nn_apply_adjoint if adjoint else L.load().qiral_nn_apply
        L.check(fn(ctypes.c_void_p(self.handle), _need_cuda(out, "out"), _need_cuda(inp, "in"), _stream()),
                "qiral_nn_apply")

    def sample(self, out, seed, step):
        n2 = ctypes.c_double()
        L.check(L.load().qiral_nn_sample(ctypes.c_void_p(self.handle), _need_cuda(out, "out"), int(seed), int(step),
                                         ctypes.byref(n2), _stream()), "qiral_nn_sample")
        return n2.value

    def grad(self, src, target):
        np = self._np
        loss = ctypes.c_double()
        g = np.zeros(2 * self.nw, dtype=np.float64)
        L.check(L.load().qiral_nn_grad(ctypes.c_void_p(self.handle), _need_cuda(src, "src"),
                                       _need_cuda(target, "target"), ctypes.byref(loss),
                                       g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream()),
                "qiral_nn_grad")
        return loss.value, g

    def train(self, steps, lr=1e-3, seed=1):
        np = self._np
        hist = np.zeros(max(steps, 1), dtype=np.float64)
        L.check(L.load().qiral_nn_train(ctypes.c_void_p(self.handle), int(steps), float(lr), int(seed),
                                        hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream()),
                "qiral_nn_train")
        return hist[:steps]
