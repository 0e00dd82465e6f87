"""Thin ctypes binding of the C ABI in include/sbp.h.

Every ``sbp_*`` function here marshals its arguments and calls the function
of the same name in libsbp.so; all numerical work happens in the HIP
library.  PyTorch is used only to allocate device memory (the workspace, the
receiver buffer, device-side states) and to supply the current HIP stream.
If libsbp.so is missing the import of this module's ``lib()`` raises: there is
no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbp.so")

SBP_OK, SBP_EINVAL, SBP_ENOMEM, SBP_EHIP, SBP_ESTATE, SBP_EUNSTABLE = 0, -1, -2, -3, -4, -5
SBP_F32, SBP_F64 = 32, 64
SBP_SAT_CHARACTERISTIC, SBP_SAT_TRACTION = 0, 1
SBP_STF_RICKER, SBP_STF_EXPT = 0, 1

_lib = None


class SBPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("sbp error %d: %s" % (code, msg))
        self.code = code


def lib():
    """Load libsbp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsbp.so not found at %s; run __graft_entry__.build() first" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        c_int, c_double, c_void_p, c_size_t = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
        P = ctypes.POINTER
        sig = {
            "sbp_workspace_bytes": [c_int, c_int, c_int, c_int, c_int, P(c_size_t)],
            "sbp_init_grid": [P(c_void_p), c_int, c_int, c_int, c_void_p, c_int, c_int, c_void_p, c_int,
                              c_void_p, c_size_t, c_void_p],
            "sbp_set_material": [c_void_p, c_void_p, c_void_p, c_void_p],
            "sbp_add_source": [c_void_p, c_void_p, c_void_p, c_int, c_double, c_double],
            "sbp_add_source_at": [c_void_p, c_void_p, c_void_p, c_int, c_double, c_double],
            "sbp_locate": [c_void_p, c_void_p, c_void_p],
            "sbp_set_graphs": [c_void_p, c_int],
            "sbp_checkpoint_id": [c_void_p, P(ctypes.c_longlong)],
            "sbp_fill_scratch": [c_void_p, c_double],
            "sbp_clear_sources": [c_void_p],
            "sbp_set_state": [c_void_p, c_void_p, c_int, c_double],
            "sbp_get_state": [c_void_p, c_void_p, c_int, P(c_double)],
            "sbp_record": [c_void_p, c_int, c_void_p, c_void_p, c_int],
            "sbp_step": [c_void_p, c_int, c_double],
            "sbp_rhs": [c_void_p, c_void_p, c_double],
            "sbp_energy": [c_void_p, P(c_double)],
            "sbp_set_launch": [c_void_p, c_int, c_int],
            "sbp_time": [c_void_p, P(c_double), P(ctypes.c_longlong)],
            "sbp_set_profiling": [c_void_p, c_int],
            "sbp_set_addressing": [c_void_p, c_int],
            "sbp_step_batch": [c_void_p, c_int, c_int, P(c_double)],
            "sbp_autotune": [c_void_p, c_int, P(c_int), P(c_int), P(c_double)],
            "sbp_autotune_batch": [c_void_p, c_int, c_int, P(c_int), P(c_double)],
            "sbp_profile": [c_void_p, P(c_double), P(c_double), P(ctypes.c_longlong), P(ctypes.c_longlong)],
            "sbp_destroy": [c_void_p],
            "sbp_adjoint_bytes": [c_void_p, c_int, c_int, P(c_size_t)],
            "sbp_adjoint_rhs": [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t],
            "sbp_gradient": [c_void_p, c_int, c_double, c_void_p, c_int, c_void_p, c_size_t, c_void_p, c_void_p],
            "sbp_step_checkpointed": [c_void_p, c_int, c_double, c_int, c_void_p, c_size_t],
            "sbp_gradient_from_checkpoints": [c_void_p, c_void_p, c_void_p, c_size_t, c_void_p, c_void_p],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = c_int
        L.sbp_last_error.argtypes = []
        L.sbp_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != SBP_OK:
        raise SBPError(rc, lib().sbp_last_error().decode())
    return rc


def _host_f64(a, n):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


# ---- functions with the names of the C ABI ----------------------------------

def sbp_workspace_bytes(nq, nr, ns, order, dtype):
    b = ctypes.c_size_t(0)
    _check(lib().sbp_workspace_bytes(nq, nr, ns, order, dtype, ctypes.byref(b)))
    return b.value


def sbp_init_grid(nq, nr, ns, xyz, order, dtype, gamma, sat_variant, workspace_ptr, workspace_bytes,
                  stream_ptr):
    h = ctypes.c_void_p()
    x = None if xyz is None else _host_f64(xyz, 3 * nq * nr * ns)
    g = _host_f64(gamma, 6)
    _check(lib().sbp_init_grid(ctypes.byref(h), nq, nr, ns, None if x is None else x.ctypes.data, order, dtype,
                               g.ctypes.data, sat_variant, workspace_ptr, workspace_bytes, stream_ptr))
    return h


def sbp_set_material(h, rho, cp, cs, n):
    r, p, s = (_host_f64(a, n) for a in (rho, cp, cs))
    _check(lib().sbp_set_material(h, r.ctypes.data, p.ctypes.data, s.ctypes.data))


def sbp_add_source(h, xi, M, stf, param, t0):
    x = _host_f64(xi, 3)
    m = _host_f64(M, 6)
    _check(lib().sbp_add_source(h, x.ctypes.data, m.ctypes.data, stf, float(param), float(t0)))


def sbp_add_source_at(h, x, M, stf, param, t0):
    p = _host_f64(x, 3)
    m = _host_f64(M, 6)
    _check(lib().sbp_add_source_at(h, p.ctypes.data, m.ctypes.data, stf, float(param), float(t0)))


def sbp_locate(h, x):
    p = _host_f64(x, 3)
    xi = np.zeros(3)
    _check(lib().sbp_locate(h, p.ctypes.data, xi.ctypes.data))
    return xi


def sbp_set_graphs(h, on):
    _check(lib().sbp_set_graphs(h, 1 if on else 0))


def sbp_fill_scratch(h, value):
    _check(lib().sbp_fill_scratch(h, float(value)))


def sbp_checkpoint_id(h):
    n = ctypes.c_longlong(0)
    _check(lib().sbp_checkpoint_id(h, ctypes.byref(n)))
    return n.value


def sbp_clear_sources(h):
    _check(lib().sbp_clear_sources(h))


def sbp_set_state(h, ptr, is_device, t):
    _check(lib().sbp_set_state(h, ptr, int(is_device), float(t)))


def sbp_get_state(h, ptr, is_device):
    t = ctypes.c_double(0)
    _check(lib().sbp_get_state(h, ptr, int(is_device), ctypes.byref(t)))
    return t.value


def sbp_record(h, nrec, ijk, out_ptr, max_steps):
    a = None
    if nrec:
        a = np.ascontiguousarray(np.asarray(ijk, dtype=np.int32).reshape(-1))
        if a.size != 3 * nrec:
            raise ValueError("ijk must hold 3 * nrec ints")
    _check(lib().sbp_record(h, nrec, None if a is None else a.ctypes.data, out_ptr, max_steps))


def sbp_step(h, nsteps, dt):
    _check(lib().sbp_step(h, int(nsteps), float(dt)))


def sbp_rhs(h, out_ptr, t):
    _check(lib().sbp_rhs(h, out_ptr, float(t)))


def sbp_energy(h):
    e = ctypes.c_double(0)
    _check(lib().sbp_energy(h, ctypes.byref(e)))
    return e.value


def sbp_set_launch(h, ty, zchunk):
    _check(lib().sbp_set_launch(h, int(ty), int(zchunk)))


def sbp_step_batch(handles, nsteps, dts):
    """Advance several handles (same dtype and stream) by nsteps steps of
    their own dt in shared launches; synchronises the stream."""
    n = len(handles)
    arr = (ctypes.c_void_p * n)(*handles)
    d = (ctypes.c_double * n)(*[float(x) for x in dts])
    _check(lib().sbp_step_batch(arr, n, int(nsteps), d))


def sbp_autotune(h, reps=5):
    """Time the candidate launch shapes and keep the fastest; returns
    (ty, zchunk, ms per right-hand-side evaluation)."""
    ty, zc, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(lib().sbp_autotune(h, int(reps), ctypes.byref(ty), ctypes.byref(zc), ctypes.byref(ms)))
    return ty.value, zc.value, ms.value


def sbp_autotune_batch(handles, reps=3):
    """Time batched right-hand-side launches for a few s-chunk lengths and
    keep the fastest for later sbp_step_batch calls of these handles;
    returns (chunk length, ms per batched stage launch)."""
    n = len(handles)
    arr = (ctypes.c_void_p * n)(*handles)
    L, ms = ctypes.c_int(), ctypes.c_double()
    _check(lib().sbp_autotune_batch(arr, n, int(reps), ctypes.byref(L), ctypes.byref(ms)))
    return L.value, ms.value


def sbp_set_addressing(h, plain):
    _check(lib().sbp_set_addressing(h, int(plain)))


def sbp_set_profiling(h, on):
    _check(lib().sbp_set_profiling(h, 1 if on else 0))


def sbp_profile(h):
    """(stage_ms, edge_ms, nstages, stage_nodes): average launch durations of
    the stage and edge kernels since profiling was switched on."""
    a, b = ctypes.c_double(), ctypes.c_double()
    n, m = ctypes.c_longlong(), ctypes.c_longlong()
    _check(lib().sbp_profile(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n), ctypes.byref(m)))
    return a.value, b.value, n.value, m.value


def sbp_time(h):
    t = ctypes.c_double(0)
    n = ctypes.c_longlong(0)
    _check(lib().sbp_time(h, ctypes.byref(t), ctypes.byref(n)))
    return t.value, n.value


def sbp_destroy(h):
    _check(lib().sbp_destroy(h))


def sbp_adjoint_bytes(h, nsteps, every):
    n = ctypes.c_size_t(0)
    _check(lib().sbp_adjoint_bytes(h, int(nsteps), int(every), ctypes.byref(n)))
    return n.value


def sbp_adjoint_rhs(h, lam_ptr, out_ptr, ws_ptr, ws_bytes):
    _check(lib().sbp_adjoint_rhs(h, lam_ptr, out_ptr, ws_ptr, int(ws_bytes)))


def sbp_step_checkpointed(h, nsteps, dt, every, ws_ptr, ws_bytes):
    _check(lib().sbp_step_checkpointed(h, int(nsteps), float(dt), int(every), ws_ptr, int(ws_bytes)))


def sbp_gradient_from_checkpoints(h, res_ptr, ws_ptr, ws_bytes, grad_ptr, qbar_ptr=None):
    _check(lib().sbp_gradient_from_checkpoints(h, res_ptr, ws_ptr, int(ws_bytes), grad_ptr, qbar_ptr))


def sbp_gradient(h, nsteps, dt, res_ptr, every, ws_ptr, ws_bytes, grad_ptr, qbar_ptr=None):
    _check(lib().sbp_gradient(h, int(nsteps), float(dt), res_ptr, int(every), ws_ptr, int(ws_bytes), grad_ptr,
                              qbar_ptr))


# ---- convenience wrapper -----------------------------------------------------

class Solver:
    """One curvilinear block on one GPU.

    xyz: (3, ns, nr, nq) node coordinates (numpy, float64) or None for the
    unit cube together with shape=(ns, nr, nq).  The workspace, the receiver
    buffer and device-side states are torch tensors on `device`.
    """

    def __init__(self, xyz=None, order=6, dtype="f32", gamma=(0, 0, 0, 0, 0, 1),
                 sat_variant=SBP_SAT_CHARACTERISTIC, shape=None, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        if xyz is not None:
            xyz = np.asarray(xyz, dtype=np.float64)
            shape = xyz.shape[1:]
        if shape is None:
            raise ValueError("give xyz or shape")
        self.shape = tuple(int(s) for s in shape)
        ns, nr, nq = self.shape
        self.n = nq * nr * ns
        self.code = SBP_F32 if dtype in ("f32", "float32", 32) else SBP_F64
        self.tdtype = torch.float32 if self.code == SBP_F32 else torch.float64
        self.device = torch.device(device)
        nbytes = sbp_workspace_bytes(nq, nr, ns, order, self.code)
        # 256-byte alignment: over-allocate and offset
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.ws_bytes = nbytes
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = sbp_init_grid(nq, nr, ns, xyz, order, self.code, gamma, sat_variant, self.ws_ptr, nbytes,
                               self.stream.cuda_stream)
        self.order = order
        self.traces = None

    def set_material(self, rho, cp, cs):
        b = lambda a: np.broadcast_to(np.asarray(a, dtype=np.float64), self.shape)
        sbp_set_material(self.h, b(rho), b(cp), b(cs), self.n)

    def add_source(self, xi, M, stf=SBP_STF_RICKER, param=2.0, t0=0.0):
        sbp_add_source(self.h, xi, M, stf, param, t0)

    def add_source_at(self, x, M, stf=SBP_STF_RICKER, param=2.0, t0=0.0):
        sbp_add_source_at(self.h, x, M, stf, param, t0)

    def locate(self, x):
        return sbp_locate(self.h, x)

    def set_graphs(self, on=True):
        sbp_set_graphs(self.h, on)

    def fill_scratch(self, value):
        sbp_fill_scratch(self.h, value)

    def checkpoint_id(self):
        return sbp_checkpoint_id(self.h)

    def set_state(self, Q, t=0.0):
        torch = self.torch
        if isinstance(Q, torch.Tensor) and Q.is_cuda:
            Qd = Q.to(self.tdtype).contiguous()
            if Qd.numel() != 9 * self.n:
                raise ValueError("state must hold 9 * n values")
            sbp_set_state(self.h, Qd.data_ptr(), 1, t)
            self.stream.synchronize()
        else:
            Qh = np.ascontiguousarray(np.asarray(Q, dtype=np.float32 if self.code == SBP_F32 else np.float64))
            if Qh.size != 9 * self.n:
                raise ValueError("state must hold 9 * n values")
            sbp_set_state(self.h, Qh.ctypes.data, 0, t)

    def get_state(self):
        out = self.torch.empty((9,) + self.shape, dtype=self.tdtype, device=self.device)
        sbp_get_state(self.h, out.data_ptr(), 1)
        return out

    def record(self, ijk, max_steps):
        ijk = np.asarray(ijk, dtype=np.int32).reshape(-1, 3)
        self.traces = self.torch.zeros((max_steps, ijk.shape[0], 3), dtype=self.tdtype, device=self.device)
        sbp_record(self.h, ijk.shape[0], ijk, self.traces.data_ptr(), max_steps)
        return self.traces

    def step(self, nsteps, dt):
        sbp_step(self.h, nsteps, dt)

    def rhs(self, t=0.0):
        out = self.torch.empty((9,) + self.shape, dtype=self.tdtype, device=self.device)
        sbp_rhs(self.h, out.data_ptr(), t)
        return out

    def energy(self):
        return sbp_energy(self.h)

    def set_launch(self, ty=8, zchunk=0):
        sbp_set_launch(self.h, ty, zchunk)

    def set_addressing(self, plain):
        sbp_set_addressing(self.h, plain)

    def autotune(self, reps=5):
        return sbp_autotune(self.h, reps)

    def set_profiling(self, on=True):
        sbp_set_profiling(self.h, on)

    def profile(self):
        return sbp_profile(self.h)

    def time(self):
        return sbp_time(self.h)

    def _adjoint_ws(self, nbytes):
        """A 256-byte aligned device buffer of at least nbytes (kept and reused)."""
        if getattr(self, "_adj", None) is None or self._adj_bytes < nbytes:
            self._adj = None
            self._adj = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
            self._adj_bytes = nbytes
        return (self._adj.data_ptr() + 255) // 256 * 256

    def adjoint_rhs(self, lam):
        """L^T lam for a (9, ns, nr, nq) device tensor lam."""
        lam = lam.to(device=self.device, dtype=self.tdtype).contiguous()
        if lam.numel() != 9 * self.n:
            raise ValueError("lam must hold 9 * n values")
        nbytes = sbp_adjoint_bytes(self.h, 0, 1)
        ws = self._adjoint_ws(nbytes)
        out = self.torch.empty((9,) + self.shape, dtype=self.tdtype, device=self.device)
        sbp_adjoint_rhs(self.h, lam.data_ptr(), out.data_ptr(), ws, nbytes)
        return out

    def step_checkpointed(self, nsteps, dt, every=100):
        """step() that keeps checkpoints for gradient_from_checkpoints()."""
        nbytes = sbp_adjoint_bytes(self.h, nsteps, every)
        ws = self._adjoint_ws(nbytes)
        sbp_step_checkpointed(self.h, nsteps, dt, every, ws, nbytes)
        self._ck = (nsteps, every, ws, nbytes)

    def gradient_from_checkpoints(self, residual, want_qbar=False):
        """The gradient of the last step_checkpointed() run (see gradient())."""
        nsteps, every, ws, nbytes = self._ck
        res = residual.to(device=self.device, dtype=self.tdtype).contiguous()
        if self.traces is None or res.numel() != nsteps * self.traces.shape[1] * 3:
            raise ValueError("residual must have shape (nsteps, nrec, 3) for the receivers of record()")
        grad = self.torch.empty((3,) + self.shape, dtype=self.tdtype, device=self.device)
        qbar = self.torch.empty((9,) + self.shape, dtype=self.tdtype, device=self.device) if want_qbar else None
        sbp_gradient_from_checkpoints(self.h, res.data_ptr(), ws, nbytes, grad.data_ptr(),
                                      qbar.data_ptr() if want_qbar else None)
        return (grad, qbar) if want_qbar else grad

    def gradient(self, nsteps, dt, residual, every=100, want_qbar=False):
        """d chi / d (rho, lambda, mu) as a (3, ns, nr, nq) tensor (and d chi /
        d Q0 if want_qbar) for the residual d chi / d traces of shape
        (nsteps, nrec, 3), from the current state; the receivers are those of
        the last record() call."""
        res = residual.to(device=self.device, dtype=self.tdtype).contiguous()
        if self.traces is None or res.numel() != nsteps * self.traces.shape[1] * 3:
            raise ValueError("residual must have shape (nsteps, nrec, 3) for the receivers of record()")
        nbytes = sbp_adjoint_bytes(self.h, nsteps, every)
        ws = self._adjoint_ws(nbytes)
        grad = self.torch.empty((3,) + self.shape, dtype=self.tdtype, device=self.device)
        qbar = self.torch.empty((9,) + self.shape, dtype=self.tdtype, device=self.device) if want_qbar else None
        sbp_gradient(self.h, nsteps, dt, res.data_ptr(), every, ws, nbytes, grad.data_ptr(),
                     qbar.data_ptr() if want_qbar else None)
        return (grad, qbar) if want_qbar else grad

    def close(self):
        if getattr(self, "h", None) is not None:
            sbp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
