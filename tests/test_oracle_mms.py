"""Manufactured-solution convergence of the oracle (a priori estimate,
Theorem theo:error_estimate): the fully discrete error converges at the
global rate p + 1 for interior order 2p or 2p + 1, p = order // 2, since the
boundary closures are accurate to order p (Sec. 6.1 and Sec. 7 claim 4th
order global accuracy for interior order 6).

The exact field Q_e is a product of sines in physical space and time.  The
forcing is the continuous residual dQ_e/dt - P (div sigma_e, sym grad v_e)
evaluated analytically at the nodes, and the boundary penalties act on
Q - Q_e (the SAT terms are linear, so this imposes the boundary data of Q_e).
"""
import numpy as np
import pytest

import workloads as W
from oracle import elastic as E
from oracle import lsrk

TW = 2 * np.pi


def mms_fields(seed):
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.5, 1.5, size=9)
    ph = rng.uniform(0, TW, size=(9, 4))

    def Q(X, t, deriv=None):
        """Fields (deriv=None), their x/y/z derivative (deriv=0/1/2) or time
        derivative (deriv='t') at coordinates X (3, ...)."""
        out = []
        for f in range(9):
            fac = [np.sin(TW * X[c] + ph[f, c]) for c in range(3)]
            ft = np.cos(TW * t + ph[f, 3])
            if deriv == "t":
                ft = -TW * np.sin(TW * t + ph[f, 3])
            elif deriv is not None:
                fac[deriv] = TW * np.cos(TW * X[deriv] + ph[f, deriv])
            out.append(amp[f] * fac[0] * fac[1] * fac[2] * ft)
        return np.array(out)
    return Q


def forcing(Qe, X, t, rho, lam, mu):
    d = [Qe(X, t, c) for c in range(3)]  # d[c][field]
    res = Qe(X, t, "t")
    # div sigma rows
    S = [[3, 6, 7], [6, 4, 8], [7, 8, 5]]
    for i in range(3):
        res[i] -= sum(d[c][S[i][c]] for c in range(3)) / rho
    g = lambda c, i: d[c][i]  # dv_i/dx_c
    div = g(0, 0) + g(1, 1) + g(2, 2)
    res[3] -= lam * div + 2 * mu * g(0, 0)
    res[4] -= lam * div + 2 * mu * g(1, 1)
    res[5] -= lam * div + 2 * mu * g(2, 2)
    res[6] -= mu * (g(1, 0) + g(0, 1))
    res[7] -= mu * (g(2, 0) + g(0, 2))
    res[8] -= mu * (g(2, 1) + g(1, 2))
    return res


def mms_error(order, n, warped, gamma, T=0.05, cfl=0.25):
    X = W.warped_mesh(n, n, n, seed=9, amp=0.03) if warped else W.unit_cube(n, n, n)
    blk = E.Block(X, order)
    rho, cp, cs = 1.3, 2.0, 1.1
    blk.set_material(rho, cp, cs)
    mu = rho * cs ** 2
    lam = rho * cp ** 2 - 2 * mu
    Qe = mms_fields(4)
    nsteps = int(np.ceil(T / (cfl * (1.0 / (n - 1)) / cp)))
    dt = T / nsteps

    def f(Q, t):
        return E.volume_rhs(blk, Q) + E.sat_rhs(blk, Q - Qe(X, t), gamma) + forcing(Qe, X, t, rho, lam, mu)
    Q = Qe(X, 0.0)
    dQ = np.zeros_like(Q)
    t = 0.0
    for k in range(nsteps):
        lsrk.step(Q, dQ, t, dt, f)
        t = (k + 1) * dt
    err = Q - Qe(X, T)
    w = blk.norm_weights() * blk.J
    return np.sqrt(np.sum(w * (err ** 2).sum(axis=0)))


@pytest.mark.parametrize("order,sizes,warped", [
    (2, (9, 17, 33), False),
    (4, (9, 17, 33), False),
    (4, (9, 17, 33), True),
    (3, (9, 17, 33), False),
    (3, (9, 17, 33), True),
    (5, (13, 19, 25, 37), False),
    (5, (13, 19, 25, 37), True),
    (7, (15, 21, 29, 41), False),
    (8, (17, 23, 31, 41), False),
    (6, (13, 19, 25, 37), False),
    (6, (13, 19, 25, 37), True),
])
def test_mms_rate(order, sizes, warped):
    gamma = (1.0, 0.0, -1.0, 0.5, 0.0, 1.0)
    errs = [mms_error(order, n, warped, gamma) for n in sizes]
    hs = [1.0 / (n - 1) for n in sizes]
    rates = [np.log(errs[i] / errs[i + 1]) / np.log(hs[i] / hs[i + 1]) for i in range(len(errs) - 1)]
    p = order // 2
    assert rates[-1] > p + 1 - 0.3, (errs, rates)
