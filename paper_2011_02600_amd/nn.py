"""Surrogate of the solver: a spectral neural operator from a material field
to receiver traces, built on the kernels of include/sbp_nn.h.

Thin ctypes binding (``sbp_nn_*``, argument marshalling only) and the network
``SpectralOperator``, whose forward pass, backward pass and Adam steps are
sequences of those kernels on torch-allocated device buffers.  Architecture
(Fourier-neural-operator style, with a truncated orthonormal cosine basis in
place of the Fourier basis, so that all transforms are real GEMMs):

    h0 = w_lift x + b_lift                               (1 -> C channels)
    h_{l+1} = act(T^T(R_l T(h_l)) + W_l h_l + b_l)       l = 0..L-1 (act: GELU,
                                                         none on the last layer)
    traces[r, t] = sum_c h_L[c, pos_r] D[r, c, t] + b_out[r, t]

T maps a grid function on n^3 points to its m^3 lowest cosine modes
(B^T along each axis, B[i, k] = sqrt((2 - [k = 0]) / n) cos(pi k (i + 1/2) / n)),
T^T maps back; R_l holds one C x C matrix per mode.  Every contraction runs
in the BF16 matrix-core GEMM with FP32 accumulation.
"""
import ctypes
import math

import numpy as np

from . import sbp as _sbp

_nn = None


class NNError(RuntimeError):
    pass


def lib():
    global _nn
    if _nn is None:
        L = _sbp.lib()
        c_int, c_ll, c_float, c_void_p = ctypes.c_int, ctypes.c_longlong, ctypes.c_float, ctypes.c_void_p
        P = ctypes.POINTER
        sig = {
            "sbp_nn_gemm": [c_int, c_int, c_int, c_int, c_float, c_void_p, c_ll, c_ll, c_ll, c_void_p, c_ll, c_ll, c_ll,
                            c_float, c_void_p, c_ll, c_ll, c_ll, c_void_p],
            "sbp_nn_bias_act": [c_int, c_int, c_ll, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p],
            "sbp_nn_act_bwd": [c_ll, c_void_p, c_void_p, c_void_p, c_int, c_void_p],
            "sbp_nn_channel_sum": [c_int, c_int, c_ll, c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p],
            "sbp_nn_lift": [c_int, c_int, c_ll, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p],
            "sbp_nn_gather": [c_int, c_int, c_ll, c_int, c_void_p, c_void_p, c_void_p, c_void_p],
            "sbp_nn_scatter": [c_int, c_int, c_ll, c_int, c_void_p, c_void_p, c_void_p, c_void_p],
            "sbp_nn_add_rows": [c_int, c_ll, c_void_p, c_void_p, c_void_p],
            "sbp_nn_sum_rows": [c_int, c_ll, c_void_p, c_void_p, c_int, c_void_p],
            "sbp_nn_mse": [c_ll, c_void_p, c_void_p, c_void_p, c_float, c_void_p, P(ctypes.c_double), c_void_p],
            "sbp_nn_mse_noalloc": [c_ll, c_void_p, c_void_p, c_void_p, c_float, P(ctypes.c_double), c_void_p],
            "sbp_nn_adam": [c_ll, c_void_p, c_void_p, c_void_p, c_void_p, c_float, c_float, c_float, c_float, c_int,
                            c_void_p],
            "sbp_nn_axpy": [c_ll, c_float, c_void_p, c_void_p, c_void_p],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = c_int
        L.sbp_nn_last_error.argtypes = []
        L.sbp_nn_last_error.restype = ctypes.c_char_p
        _nn = L
    return _nn


def _ck(rc):
    if rc != 0:
        raise NNError("sbp_nn error %d: %s" % (rc, lib().sbp_nn_last_error().decode()))


def _p(t):
    return None if t is None else t.data_ptr()


_gemm_log = None


def gemm_profile(on):
    """Start (True) or stop (False) recording every gemm call: its flops
    (2 M N K per batch entry), its algorithmic bytes (A, B and C once, C
    twice when accumulated, 4 bytes each) and a pair of events on its
    stream.  Returns the records of the stopped recording."""
    global _gemm_log
    out = _gemm_log
    _gemm_log = [] if on else None
    return out


def gemm_profile_summary(records):
    """Totals of gemm_profile records (after a synchronisation): calls,
    flops, bytes, milliseconds."""
    ms = sum(e0.elapsed_time(e1) for (_, _, e0, e1) in records)
    return {"calls": len(records), "flops": float(sum(r[0] for r in records)),
            "bytes": float(sum(r[1] for r in records)), "ms": ms}


def gemm(A, B, C, M, N, K, sA, sB, sC, batch=1, alpha=1.0, beta=0.0, stream=None, offs=(0, 0, 0)):
    """C[b] = alpha A[b] B[b] + beta C[b]; sA = (sAb, sAm, sAk), sB = (sBb, sBk,
    sBn), sC = (sCb, sCm, sCn) element strides; offs: element offsets into
    the three tensors."""
    es = 4
    rec = _gemm_log is not None
    if rec:
        import torch
        st = torch.cuda.ExternalStream(stream) if stream else torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
    _ck(lib().sbp_nn_gemm(batch, M, N, K, alpha, A.data_ptr() + es * offs[0], *sA, B.data_ptr() + es * offs[1], *sB,
                          beta, C.data_ptr() + es * offs[2], *sC, stream))
    if rec:
        e1.record(st)
        nbytes = es * batch * (M * K + K * N + M * N * (2 if beta != 0.0 else 1))
        _gemm_log.append((2.0 * batch * M * N * K, nbytes, e0, e1))


def cosine_basis(n, m):
    """B[i, k] = sqrt((2 - [k = 0]) / n) cos(pi k (i + 1/2) / n), n x m (float64)."""
    i = np.arange(n)[:, None] + 0.5
    k = np.arange(m)[None, :]
    return np.sqrt((2.0 - (k == 0)) / n) * np.cos(np.pi * k * i / n)


class SpectralOperator:
    """The surrogate network on one GPU.  x: (S, n, n, n) material field;
    output (S, R, T) traces at the receiver positions `pos` (flat indices
    z n^2 + y n + x of the grid)."""

    def __init__(self, n, modes, width, layers, pos, T, device="cuda:0", seed=0, stream=None):
        import torch
        self.torch = torch
        self.n, self.m, self.C, self.L, self.T = n, modes, width, layers, T
        self.P = n ** 3
        self.R = len(pos)
        self.dev = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev).cuda_stream
        self.pos = torch.tensor(np.asarray(pos, dtype=np.int32), device=self.dev)
        self.B = torch.tensor(cosine_basis(n, modes), dtype=torch.float32, device=self.dev)  # n x m
        rng = np.random.default_rng(seed)
        C, m3 = width, modes ** 3
        f32 = lambda a: torch.tensor(np.asarray(a, dtype=np.float32), device=self.dev)
        p = {"w_lift": f32(rng.standard_normal(C)), "b_lift": f32(0.1 * rng.standard_normal(C))}
        for l in range(layers):
            p["R%d" % l] = f32(rng.standard_normal((m3, C, C)) / C)
            p["W%d" % l] = f32(rng.standard_normal((C, C)) / math.sqrt(C))
            p["b%d" % l] = f32(np.zeros(C))
        p["D"] = f32(rng.standard_normal((self.R, C, T)) / math.sqrt(C))
        p["b_out"] = f32(np.zeros((self.R, T)))
        self.params = p
        self.grads = {k: torch.zeros_like(v) for k, v in p.items()}
        self.adam_m = {k: torch.zeros_like(v) for k, v in p.items()}
        self.adam_v = {k: torch.zeros_like(v) for k, v in p.items()}
        self.step_count = 0
        self._part = torch.zeros(256, dtype=torch.float64, device=self.dev)
        self._cpart = torch.zeros(64 * width, dtype=torch.float64, device=self.dev)  # channel sums
        self._bufs = {}

    # ---- buffers --------------------------------------------------------------
    def _buf(self, name, shape):
        t = self._bufs.get(name)
        if t is None or tuple(t.shape) != tuple(shape):
            t = self.torch.empty(shape, dtype=self.torch.float32, device=self.dev)
            self._bufs[name] = t
        return t

    # ---- separable transforms (each a GEMM per axis) ---------------------------
    def _fwd_T(self, X, S, out, tag):
        """out (S*C, m^3) = T applied to X (S*C, n^3): x, then y, then z."""
        n, m, SC = self.n, self.m, S * self.C
        t1 = self._buf(tag + "t1", (SC, n, n, m))
        t2 = self._buf(tag + "t2", (SC, n, m, m))
        st = self.stream
        # x: (SC n n, n) @ B (n, m)
        gemm(X, self.B, t1, SC * n * n, m, n, (0, n, 1), (0, m, 1), (0, m, 1), stream=st)
        # y: per (sc, z): B^T (m, n) @ t1 (n, m)
        gemm(self.B, t1, t2, m, m, n, (0, 1, m), (n * m, m, 1), (m * m, m, 1), batch=SC * n, stream=st)
        # z: per sc: B^T (m, n) @ t2 (n, m m)
        gemm(self.B, t2, out, m, m * m, n, (0, 1, m), (n * m * m, m * m, 1), (m ** 3, m * m, 1), batch=SC, stream=st)

    def _inv_T(self, Y, S, out, tag, beta=0.0):
        """out (S*C, n^3) (+)= T^T applied to Y (S*C, m^3): z, then y, then x."""
        n, m, SC = self.n, self.m, S * self.C
        t2 = self._buf(tag + "i2", (SC, n, m, m))
        t1 = self._buf(tag + "i1", (SC, n, n, m))
        st = self.stream
        # z: per sc: B (n, m) @ Y (m, m m)
        gemm(self.B, Y, t2, n, m * m, m, (0, m, 1), (m ** 3, m * m, 1), (n * m * m, m * m, 1), batch=SC, stream=st)
        # y: per (sc, z): B (n, m) @ t2 (m, m)
        gemm(self.B, t2, t1, n, m, m, (0, m, 1), (m * m, m, 1), (n * m, m, 1), batch=SC * n, stream=st)
        # x: (SC n n, m) @ B^T (m, n)
        gemm(t1, self.B, out, SC * n * n, n, m, (0, m, 1), (0, 1, m), (0, n, 1), beta=beta, stream=st)

    def _mix(self, Rw, Xh, S, out, transpose=False, beta=0.0):
        """out[s, co, q] = sum_ci R[q, co, ci] Xh[s, ci, q] (transpose: R^T)."""
        C, m3 = self.C, self.m ** 3
        sR = (C * C, 1, C) if transpose else (C * C, C, 1)
        gemm(Rw, Xh, out, C, S, C, sR, (1, m3, C * m3), (1, m3, C * m3), batch=m3, beta=beta, stream=self.stream)

    # ---- forward -------------------------------------------------------------
    def forward(self, x, keep=True):
        """x: (S, n, n, n) float32 device tensor -> (S, R, T) traces."""
        S, C, P, L = x.shape[0], self.C, self.P, self.L
        p, st, lb = self.params, self.stream, lib()
        self.S = S
        self.x = x
        h = self._buf("h0", (S, C, P))
        _ck(lb.sbp_nn_lift(S, C, P, _p(x), _p(p["w_lift"]), _p(p["b_lift"]), _p(h), st))
        self.hs, self.zs, self.xh = [h], [], []
        for l in range(L):
            xh = self._buf("xh%d" % l, (S, C, self.m ** 3))
            self._fwd_T(h, S, xh, "f")
            yh = self._buf("yh", (S, C, self.m ** 3))
            self._mix(p["R%d" % l], xh, S, yh)
            k = self._buf("k", (S, C, P))
            self._inv_T(yh, S, k, "f")
            u = self._buf("u", (S, C, P))
            gemm(p["W%d" % l], h, u, C, P, C, (0, C, 1), (C * P, P, 1), (C * P, P, 1), batch=S, stream=st)
            z = self._buf("z%d" % l, (S, C, P))
            hn = self._buf("h%d" % (l + 1), (S, C, P))
            act = 1 if l < L - 1 else 0
            _ck(lb.sbp_nn_bias_act(S, C, P, _p(k), _p(u), _p(p["b%d" % l]), _p(z), _p(hn), act, st))
            self.xh.append(xh)
            self.zs.append(z)
            self.hs.append(hn)
            h = hn
        f = self._buf("feat", (S, self.R, C))
        _ck(lb.sbp_nn_gather(S, C, P, self.R, _p(self.pos), _p(h), _p(f), st))
        y = self._buf("y", (S, self.R, self.T))
        R, T = self.R, self.T
        # per receiver r: y[:, r, :] (S x T) = f[:, r, :] (S x C) @ D[r] (C x T)
        gemm(f, p["D"], y, S, T, C, (C, R * C, 1), (C * T, T, 1), (T, R * T, 1), batch=R, stream=st)
        _ck(lb.sbp_nn_add_rows(S, self.R * self.T, _p(p["b_out"]), _p(y), st))
        return y

    # ---- loss and backward ---------------------------------------------------
    def loss(self, y, target, scale=1.0):
        """1/2 sum (y - target)^2 * scale; leaves dy = scale (y - target)."""
        dy = self._buf("dy", tuple(y.shape))
        loss = ctypes.c_double(0)
        _ck(lib().sbp_nn_mse(y.numel(), _p(y), _p(target), _p(dy), scale, _p(self._part), ctypes.byref(loss),
                             self.stream))
        return loss.value * scale, dy

    def backward(self, dy):
        """Gradients of the loss with respect to every parameter (into
        self.grads) for the output gradient dy (S, R, T)."""
        S, C, P, L, R, T = self.S, self.C, self.P, self.L, self.R, self.T
        p, g, st, lb = self.params, self.grads, self.stream, lib()
        # head: y = F D + b_out
        f = self._bufs["feat"]
        gemm(f, dy, g["D"], C, T, S, (C, 1, R * C), (T, R * T, 1), (C * T, T, 1), batch=R, stream=st)
        _ck(lb.sbp_nn_sum_rows(S, R * T, _p(dy), _p(g["b_out"]), 0, st))
        df = self._buf("dfeat", (S, R, C))
        gemm(dy, p["D"], df, S, C, T, (T, R * T, 1), (C * T, 1, T), (C, R * C, 1), batch=R, stream=st)
        dh = self._buf("dh", (S, C, P))
        dh.zero_()
        _ck(lb.sbp_nn_scatter(S, C, P, R, _p(self.pos), _p(df), _p(dh), st))
        for l in range(L - 1, -1, -1):
            act = 1 if l < L - 1 else 0
            dz = self._buf("dz", (S, C, P))
            _ck(lb.sbp_nn_act_bwd(S * C * P, _p(self.zs[l]), _p(dh), _p(dz), act, st))
            _ck(lb.sbp_nn_channel_sum(S, C, P, _p(dz), None, _p(g["b%d" % l]), 0, _p(self._cpart), st))
            h = self.hs[l]
            # pointwise path u = W h: dW = sum_s dz_s h_s^T, dh = W^T dz
            self._weight_grad(dz, h, g["W%d" % l])
            dhn = self._buf("dhn", (S, C, P))
            gemm(p["W%d" % l], dz, dhn, C, P, C, (0, 1, C), (C * P, P, 1), (C * P, P, 1), batch=S, stream=st)
            # spectral path k = T^T(R T(h)): dY = T(dz), dR_q = dY_q X_q^T, dX = R^T dY, dh += T^T(dX)
            dyh = self._buf("dyh", (S, C, self.m ** 3))
            self._fwd_T(dz, S, dyh, "b")
            m3 = self.m ** 3
            gemm(dyh, self.xh[l], g["R%d" % l], C, C, S, (1, m3, C * m3), (1, C * m3, m3), (C * C, C, 1), batch=m3,
                 stream=st)
            dxh = self._buf("dxh", (S, C, m3))
            self._mix(p["R%d" % l], dyh, S, dxh, transpose=True)
            self._inv_T(dxh, S, dhn, "b", beta=1.0)
            dh, self._bufs["dh"], self._bufs["dhn"] = dhn, dhn, dh
        # lift: h0 = w x + b
        _ck(lb.sbp_nn_channel_sum(S, C, P, _p(dh), _p(self.x), _p(g["w_lift"]), 0, _p(self._cpart), st))
        _ck(lb.sbp_nn_channel_sum(S, C, P, _p(dh), None, _p(g["b_lift"]), 0, _p(self._cpart), st))

    def _weight_grad(self, dz, h, out):
        """out (C x C) = sum_s dz_s h_s^T: the long contraction over the grid is
        split into chunks (one GEMM batch entry, i.e. one thread block, each)
        whose partial products are summed afterwards; chunks of 512 points
        when the grid has at least 128 of them, so that a call fills the
        GPU, else one chunk."""
        S, C, P = self.S, self.C, self.P
        PC = 512 if P % 512 == 0 and P // 512 >= 128 else P
        nch = P // PC
        parts = self._buf("wparts", (S * nch, C, C))
        for s in range(S):
            gemm(dz, h, parts, C, C, PC, (PC, P, 1), (PC, 1, P), (C * C, C, 1), batch=nch, stream=self.stream,
                 offs=(s * C * P, s * C * P, s * nch * C * C))
        _ck(lib().sbp_nn_sum_rows(S * nch, C * C, _p(parts), _p(out), 0, self.stream))

    def adam_step(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        for k, v in self.params.items():
            _ck(lib().sbp_nn_adam(v.numel(), _p(v), _p(self.grads[k]), _p(self.adam_m[k]), _p(self.adam_v[k]), lr,
                                  b1, b2, eps, self.step_count, self.stream))

    def state_numpy(self):
        return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in self.params.items()}

    def load_numpy(self, state):
        for k, v in state.items():
            self.params[k].copy_(self.torch.tensor(np.asarray(v, dtype=np.float32)))
