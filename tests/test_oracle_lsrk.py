"""Pins of the oracle's low-storage Runge-Kutta scheme: the eight classical
order-4 conditions of the equivalent Butcher tableau (textbook), the stage
times, and the observed order on y' = i w y."""
from fractions import Fraction as Fr

import numpy as np

from oracle import lsrk


def butcher_from_2n():
    """Expand the 2N-storage recursion symbolically: each register is a
    vector of coefficients of dt * f_j, j = 0..4 (f_j = RHS at stage j)."""
    s = lsrk.NSTAGE
    dQ = [Fr(0)] * s
    Q = [Fr(0)] * s
    a = []
    for k in range(s):
        a.append(list(Q))  # stage k reads Q = y0 + sum_j a[k][j] dt f_j
        dQ = [lsrk.A[k] * x for x in dQ]
        dQ[k] += 1
        Q = [qq + lsrk.B[k] * d for qq, d in zip(Q, dQ)]
    return a, Q


def test_order_conditions():
    a, b = butcher_from_2n()
    A = np.array([[float(x) for x in row] for row in a])
    bb = np.array([float(x) for x in b])
    c = A.sum(axis=1)
    conds = [
        (bb.sum(), 1.0),
        (bb @ c, 1 / 2),
        (bb @ c ** 2, 1 / 3),
        (bb @ (A @ c), 1 / 6),
        (bb @ c ** 3, 1 / 4),
        (bb @ (c * (A @ c)), 1 / 8),
        (bb @ (A @ c ** 2), 1 / 12),
        (bb @ (A @ (A @ c)), 1 / 24),
    ]
    for got, want in conds:
        assert abs(got - want) < 1e-11
    # the tableau is explicit and the stored stage times are its row sums
    assert np.allclose(np.triu(A), 0.0)
    assert np.allclose(c, lsrk.C_F, atol=1e-11)
    # not fifth order (the method is exactly fourth order)
    assert abs(bb @ c ** 4 - 1 / 5) > 1e-6


def test_observed_order_four():
    w = 1.3
    errs = []
    for n in (20, 40, 80):
        dt = 2.0 / n
        y = np.array([1.0 + 0j])
        d = np.zeros_like(y)
        t = 0.0
        for _ in range(n):
            lsrk.step(y, d, t, dt, lambda yy, tt: 1j * w * yy)
            t += dt
        errs.append(abs(y[0] - np.exp(1j * w * 2.0)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.8) and np.all(rates < 4.3)


def test_imaginary_axis_stability_limit():
    """Stability polynomial R(z) = sum_k b^T A^k ... evaluated directly:
    |R(i y)| <= 1 up to |y| ~ 3.3 (used for the CFL choice), > 1 beyond 3.5."""
    def amp(y):
        u = np.array([1.0 + 0j])
        d = np.zeros_like(u)
        lsrk.step(u, d, 0.0, 1.0, lambda yy, tt: 1j * y * yy)
        return abs(u[0])
    assert all(amp(y) <= 1.0 + 1e-12 for y in np.linspace(0, 3.3, 200))
    assert amp(3.5) > 1.0
