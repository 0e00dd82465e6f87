"""Pins of the surrogate reference network (oracle/fno.py): the hand-derived
backward pass against central finite differences of the forward pass (every
parameter block and the input), the cosine basis orthonormality, and the
transform pair (T^T T is the projection onto the kept modes)."""
import numpy as np
import pytest

from oracle import fno


def small(seed=0, L=3):
    n, m, C, R, Tn, S = 6, 3, 4, 3, 5, 2
    rng = np.random.default_rng(seed)
    p = fno.init_params(n, m, C, L, R, Tn, seed)
    x = rng.standard_normal((S, n, n, n))
    pos = np.array([5, 100, 213])
    return p, x, pos, m, L


def test_basis_orthonormal_and_projection():
    B = fno.cosine_basis(10, 4)
    assert np.allclose(B.T @ B, np.eye(4), atol=1e-14)
    # full basis: T^T T = I; truncated: a projection (idempotent)
    Bf = fno.cosine_basis(6, 6)
    h = np.random.default_rng(1).standard_normal((1, 1, 6, 6, 6))
    assert np.allclose(fno.Tt(Bf, fno.T(Bf, h)), h, atol=1e-12)
    Bt = fno.cosine_basis(6, 3)
    ph = fno.Tt(Bt, fno.T(Bt, h))
    assert np.allclose(fno.Tt(Bt, fno.T(Bt, ph)), ph, atol=1e-12)


@pytest.mark.parametrize("L", [1, 3])
def test_backward_matches_finite_differences(L):
    p, x, pos, m, L = small(L=L)
    rng = np.random.default_rng(7)
    target = rng.standard_normal((x.shape[0], len(pos), p["D"].shape[2]))

    def loss(pp, xx):
        y, _ = fno.forward(pp, xx, pos, m, L)
        return 0.5 * np.sum((y - target) ** 2)

    y, cache = fno.forward(p, x, pos, m, L)
    g = fno.backward(p, y - target, cache)
    eps = 1e-6
    for k in p:
        d = rng.standard_normal(p[k].shape)
        pp = dict(p)
        pp[k] = p[k] + eps * d
        fp = loss(pp, x)
        pp[k] = p[k] - eps * d
        fm = loss(pp, x)
        fd = (fp - fm) / (2 * eps)
        ad = float(np.sum(g[k] * d))
        assert ad == pytest.approx(fd, rel=1e-6, abs=1e-9), k


def test_gelu_grad_matches_finite_differences():
    z = np.linspace(-4, 4, 41)
    eps = 1e-6
    fd = (fno.gelu(z + eps) - fno.gelu(z - eps)) / (2 * eps)
    assert np.allclose(fno.gelu_grad(z), fd, atol=1e-8)
