"""Pins of the oracle's SBP operators against what the paper fixes:
the dual-pair identity (eq. upw_SBP), the upwind dissipation property
(Definition in Sec. 4.1), the accuracy conditions (eq. acc), the interior
stencils (Table tab:upwind) and the numerical dispersion relation
(eq. dispersion_relation_upwind / _traditional, Sec. 6.2)."""
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import sbp_operators as sbp

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_table(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tok = line.split()
            out[int(tok[0])] = [int(t) for t in tok[1:3]] + [Fr(t) for t in tok[3:]] \
                if name == "tab_upwind.txt" else [int(tok[1])] + [Fr(t) for t in tok[2:]]
    return out


UPW = read_table("tab_upwind.txt")
TRAD = read_table("tab_traditional.txt")


def sizes(order):
    m = sbp.closure(order)["m"]
    return [2 * m, 2 * m + 1, 2 * m + 4, 3 * m + 7]


@pytest.mark.parametrize("order", sorted(UPW))
def test_table_consistency_and_order(order):
    """Every row of tab:upwind is consistent (sum alpha = 0, sum j alpha = 1)
    and exact for polynomials up to its order; the order-8 row is so only
    with alpha_4 = -1/28 (reading of the printed +1/28)."""
    r, q, *al = UPW[order]
    js = range(-r, q + 1)
    assert len(al) == r + q + 1
    assert sum(al) == 0
    assert sum(j * a for j, a in zip(js, al)) == 1
    for k in range(2, order + 1):
        assert sum(Fr(j) ** k * a for j, a in zip(js, al)) == 0, k
    # the next moment does not vanish: the order is exactly `order`
    assert sum(Fr(j) ** (order + 1) * a for j, a in zip(js, al)) != 0
    if order == 8:
        printed = list(al)
        printed[4 + r] = Fr(1, 28)
        assert sum(printed) != 0


def test_oracle_table_is_the_golden_table():
    for order, (r, q, *al) in UPW.items():
        rr, coeffs = sbp.UPWIND_ALPHA[order]
        assert rr == r and coeffs == al


@pytest.mark.parametrize("order", sbp.CLOSED_ORDERS)
def test_interior_rows_are_table_stencils(order):
    r, q, *al = UPW[order]
    for N in sizes(order):
        e = sbp.operators_exact(order, N)
        m = sbp.closure(order)["m"]
        h = e["h"]
        for i in range(m, N - m):
            row_p = {j - i: e["Dp"][i][j] * h for j in range(N) if e["Dp"][i][j] != 0}
            row_m = {j - i: e["Dm"][i][j] * h for j in range(N) if e["Dm"][i][j] != 0}
            assert row_p == {j: a for j, a in zip(range(-r, q + 1), al) if a != 0}
            # backward stencil beta_j = -alpha_{-j} (Sec. 6.2)
            assert row_m == {-j: -a for j, a in zip(range(-r, q + 1), al) if a != 0}


@pytest.mark.parametrize("order", sbp.CLOSED_ORDERS)
def test_dual_pair_sbp_identity_exact(order):
    """(D+ f)^T H g + f^T H (D- g) = f_N g_N - f_0 g_0 for all f, g, i.e.
    D+^T H + H D- = B entrywise, in exact arithmetic (eq. upw_SBP)."""
    for N in sizes(order):
        e = sbp.operators_exact(order, N)
        H, Dp, Dm = e["Hdiag"], e["Dp"], e["Dm"]
        for i in range(N):
            for j in range(N):
                lhs = Dp[j][i] * H[j] + H[i] * Dm[i][j]
                rhs = Fr(-1) if i == j == 0 else (Fr(1) if i == j == N - 1 else Fr(0))
                assert lhs == rhs, (order, N, i, j)
        assert all(x > 0 for x in H)


@pytest.mark.parametrize("order", sbp.CLOSED_ORDERS)
def test_upwind_dissipation_symmetric_nsd(order):
    """H (D+ - D-) is symmetric negative semi-definite (the upwind property
    of the dual pair, Definition in Sec. 4.1), and not zero."""
    for N in sizes(order):
        e = sbp.operators_exact(order, N)
        H = e["Hdiag"]
        S = [[H[i] * (e["Dp"][i][j] - e["Dm"][i][j]) for j in range(N)] for i in range(N)]
        assert all(S[i][j] == S[j][i] for i in range(N) for j in range(N))
        ev = np.linalg.eigvalsh(np.array(S, dtype=float))
        assert ev.max() < 1e-12 * abs(ev.min())
        assert ev.min() < -1e-3


@pytest.mark.parametrize("order", sbp.CLOSED_ORDERS)
def test_accuracy_conditions(order):
    """D x^k = k x^{k-1} on every row for k <= p (boundary order p for
    interior order 2p) and on interior rows for k <= 2p (eq. acc); the
    boundary rows are not exact at k = p + 1 (order is exactly p there)."""
    p = order // 2
    m = sbp.closure(order)["m"]
    for N in sizes(order):
        e = sbp.operators_exact(order, N)
        x = [Fr(i, N - 1) for i in range(N)]
        for D in (e["Dp"], e["Dm"]):
            for k in range(0, 2 * p + 2):
                res = [sum(D[i][j] * x[j] ** k for j in range(N)) - (k * x[i] ** (k - 1) if k else 0)
                       for i in range(N)]
                if k <= p:
                    assert all(v == 0 for v in res), (order, N, k)
                if k <= 2 * p:
                    assert all(v == 0 for v in res[m:N - m]), (order, N, k)
                if k == p + 1:
                    assert any(v != 0 for v in res[:m])


@pytest.mark.parametrize("order", sbp.CLOSED_ORDERS)
def test_norm_is_a_quadrature(order):
    """A diagonal SBP norm integrates polynomials up to degree 2p - 1 exactly."""
    p = order // 2
    N = 3 * sbp.closure(order)["m"] + 5
    e = sbp.operators_exact(order, N)
    x = [Fr(i, N - 1) for i in range(N)]
    for k in range(0, 2 * p):
        assert sum(hh * xx ** k for hh, xx in zip(e["Hdiag"], x)) == Fr(1, k + 1)


@pytest.mark.parametrize("order", sbp.CLOSED_ORDERS)
def test_right_closure_is_mirror_of_left(order):
    """D+ at the right end is the negated flip of D- at the left end."""
    N = 3 * sbp.closure(order)["m"] + 2
    e = sbp.operators_exact(order, N)
    for i in range(N):
        for j in range(N):
            assert e["Dp"][N - 1 - i][N - 1 - j] == -e["Dm"][i][j]


def symbol(al, r, k):
    return sum(float(a) * np.exp(1j * (j - r) * k) for j, a in enumerate(al))


@pytest.mark.parametrize("order", sorted(UPW))
def test_dispersion_relation_from_periodic_scheme(order):
    """The 1D scheme rho v_t = D+ sigma, sigma_t / mu = D- v (eq. 1D_wave_disc)
    with the interior stencils on a periodic grid has frequencies equal to
    eq. dispersion_relation_upwind: omega~ = c |sum alpha_j e^{i j k~}|."""
    r, q, *al = UPW[order]
    n = 64
    Dp = np.zeros((n, n))
    Dm = np.zeros((n, n))
    for i in range(n):
        for j, a in zip(range(-r, q + 1), al):
            Dp[i, (i + j) % n] += float(a)
            Dm[i, (i - j) % n] += -float(a)
    L = np.block([[np.zeros((n, n)), Dp], [Dm, np.zeros((n, n))]])  # rho = mu = 1, h = 1
    ev = np.linalg.eigvals(L)
    assert np.abs(ev.real).max() < 1e-10
    ks = 2 * np.pi * np.arange(n) / n
    pred = np.abs(np.array([symbol(al, r, k) for k in ks]))
    got = np.sort(np.abs(ev.imag))
    want = np.sort(np.concatenate([pred, pred]))
    assert np.allclose(got, want, atol=1e-10)


def test_dispersion_closed_forms_and_claims():
    """omega~(pi) = 4, 8/3, 32/15 for orders 2, 4, 6; omega~ ~ k~ for small k~;
    traditional stencils vanish at pi; even orders 2 and 4 have a
    non-decreasing relation on [0, pi], order 6 nearly so (reading of the
    paper's 'gtrsim 0'), odd orders 3, 5, 7, 9 and order 8 have a clearly
    negative slope somewhere (spurious modes, Sec. 6.2 observations)."""
    k = np.linspace(0, np.pi, 4001)
    for order, val in ((2, 4.0), (4, 8 / 3), (6, 32 / 15)):
        r, q, *al = UPW[order]
        assert abs(abs(symbol(al, r, np.pi)) - val) < 1e-13
    for order, (r, q, *al) in UPW.items():
        w = np.abs(np.array([symbol(al, r, kk) for kk in k]))
        ks = k[k < 0.05]
        assert np.all(np.abs(w[: len(ks)] - ks) <= 5 * ks ** (order + 1) + 1e-14)
        slope = np.diff(w) / np.diff(k)
        if order in (2, 4):
            assert slope.min() > -1e-9
        elif order == 6:
            assert slope.min() > -0.2
        else:
            assert slope.min() < -0.2, order
    for order, (q, *g) in TRAD.items():
        w = np.abs(sum(2 * float(gj) * np.sin((j + 1) * k) for j, gj in enumerate(g)))
        assert w[-1] < 1e-12
        assert abs(sum(2 * (j + 1) * gj for j, gj in enumerate(g)) - 1) == 0


def one_d_elastic(order, N, gamma, Z=1.0):
    """1D elastic operator (rho = mu = 1) with the characteristic penalties."""
    o = sbp.operators(order, N)
    L = np.zeros((2 * N, 2 * N))
    L[:N, N:] = o["Dm"]
    L[N:, :N] = o["Dp"]
    for idx, eps in ((0, -1.0), (N - 1, 1.0)):
        k = 1.0 / o["H"][idx]
        L[idx, idx] += -k * 0.5 * (1 - gamma) * Z
        L[idx, N + idx] += -k * 0.5 * eps * (1 + gamma)
        L[N + idx, idx] += -eps * k * 0.5 * (1 - gamma)
        L[N + idx, N + idx] += -eps * k * 0.5 * eps * (1 + gamma) / Z
    return L, o["h"]


@pytest.mark.parametrize("order", sbp.CLOSED_ORDERS)
@pytest.mark.parametrize("gamma", [-1.0, 0.0, 0.5, 1.0])
def test_one_d_stability_and_spectral_radius(order, gamma):
    """Semi-discrete 1D operator with SATs has no growing modes (energy
    estimate, Theorem for general boundary conditions) and a spectral radius
    close to the interior maximum of |alpha^| (closures do not stiffen the
    scheme)."""
    L, h = one_d_elastic(order, 61, gamma)
    ev = np.linalg.eigvals(L)
    assert ev.real.max() < 1e-9
    r, q, *al = UPW[order]
    kk = np.linspace(0, np.pi, 2001)
    inter = np.abs(np.array([symbol(al, r, x) for x in kk])).max()
    assert np.abs(ev).max() * h < 1.2 * inter
