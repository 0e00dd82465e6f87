"""Reference of the surrogate network (oracle side; test infrastructure only):
the spectral neural operator of the library's surrogate written out in
float64 numpy, forward pass and hand-derived backward pass, to check the
GPU kernels against.  Not part of the paper's method.

    h0 = w_lift x + b_lift
    z_l = T^T(R_l T(h_l)) + W_l h_l + b_l,   h_{l+1} = gelu(z_l)  (l < L-1),
                                             h_L = z_{L-1}
    y[s, r, t] = sum_c h_L[s, c, pos_r] D[r, c, t] + b_out[r, t]

T: the m^3 lowest modes of the orthonormal cosine basis
B[i, k] = sqrt((2 - [k = 0]) / n) cos(pi k (i + 1/2) / n) along each axis;
gelu(z) = z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).  The backward pass is
pinned by central finite differences (tests/test_oracle_fno.py).
"""
import numpy as np

S2PI = np.sqrt(2.0 / np.pi)


def cosine_basis(n, m):
    i = np.arange(n)[:, None] + 0.5
    k = np.arange(m)[None, :]
    return np.sqrt((2.0 - (k == 0)) / n) * np.cos(np.pi * k * i / n)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(S2PI * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    u = S2PI * (z + 0.044715 * z ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * S2PI * (1.0 + 3 * 0.044715 * z * z)


def T(B, h):
    """(S, C, n, n, n) -> (S, C, m, m, m)."""
    return np.einsum("zc,yb,xa,sqzyx->sqcba", B, B, B, h, optimize=True)


def Tt(B, y):
    """(S, C, m, m, m) -> (S, C, n, n, n)."""
    return np.einsum("zc,yb,xa,sqcba->sqzyx", B, B, B, y, optimize=True)


def init_params(n, m, C, L, R, Tn, seed=0):
    rng = np.random.default_rng(seed)
    p = {"w_lift": rng.standard_normal(C), "b_lift": 0.1 * rng.standard_normal(C)}
    for l in range(L):
        p["R%d" % l] = rng.standard_normal((m ** 3, C, C)) / C
        p["W%d" % l] = rng.standard_normal((C, C)) / np.sqrt(C)
        p["b%d" % l] = 0.1 * rng.standard_normal(C)
    p["D"] = rng.standard_normal((R, C, Tn)) / np.sqrt(C)
    p["b_out"] = 0.1 * rng.standard_normal((R, Tn))
    return p


def forward(p, x, pos, m, L):
    """x: (S, n, n, n); pos: flat receiver indices.  Returns (y, cache)."""
    S, n = x.shape[0], x.shape[1]
    C = p["w_lift"].shape[0]
    B = cosine_basis(n, m)
    h = p["w_lift"][None, :, None, None, None] * x[:, None] + p["b_lift"][None, :, None, None, None]
    hs, zs, xhs = [h], [], []
    for l in range(L):
        xh = T(B, h).reshape(S, C, m ** 3)
        yh = np.einsum("qoi,siq->soq", p["R%d" % l], xh)
        k = Tt(B, yh.reshape(S, C, m, m, m))
        u = np.einsum("oi,sizyx->sozyx", p["W%d" % l], h)
        z = k + u + p["b%d" % l][None, :, None, None, None]
        h = gelu(z) if l < L - 1 else z
        xhs.append(xh)
        zs.append(z)
        hs.append(h)
    f = h.reshape(S, C, -1)[:, :, pos].transpose(0, 2, 1)  # (S, R, C)
    y = np.einsum("src,rct->srt", f, p["D"]) + p["b_out"][None]
    return y, dict(x=x, hs=hs, zs=zs, xhs=xhs, f=f, B=B, m=m, L=L, pos=pos)


def backward(p, dy, cache):
    """Gradients of a scalar loss with d loss / d y = dy."""
    x, hs, zs, xhs, f, B, m, L, pos = (cache[k] for k in ("x", "hs", "zs", "xhs", "f", "B", "m", "L", "pos"))
    S, n = x.shape[0], x.shape[1]
    C = p["w_lift"].shape[0]
    g = {}
    g["D"] = np.einsum("src,srt->rct", f, dy)
    g["b_out"] = dy.sum(axis=0)
    df = np.einsum("srt,rct->src", dy, p["D"])  # (S, R, C)
    dh = np.zeros_like(hs[-1]).reshape(S, C, -1)
    for r, q in enumerate(pos):
        dh[:, :, q] += df[:, r, :]
    dh = dh.reshape(hs[-1].shape)
    for l in range(L - 1, -1, -1):
        dz = dh * gelu_grad(zs[l]) if l < L - 1 else dh
        g["b%d" % l] = dz.sum(axis=(0, 2, 3, 4))
        h = hs[l]
        g["W%d" % l] = np.einsum("sozyx,sizyx->oi", dz, h)
        dh = np.einsum("oi,sozyx->sizyx", p["W%d" % l], dz)
        dyh = T(B, dz).reshape(S, C, m ** 3)
        g["R%d" % l] = np.einsum("soq,siq->qoi", dyh, xhs[l])
        dxh = np.einsum("qoi,soq->siq", p["R%d" % l], dyh)
        dh = dh + Tt(B, dxh.reshape(S, C, m, m, m))
    g["w_lift"] = np.einsum("sczyx,szyx->c", dh, x)
    g["b_lift"] = dh.sum(axis=(0, 2, 3, 4))
    return g
