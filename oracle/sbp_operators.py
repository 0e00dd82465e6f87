"""Upwind diagonal-norm dual-pair SBP operators, built in exact rational
arithmetic (oracle side; test infrastructure only).

What the paper fixes (Sec. 4.1):
  * the dual-pair identity (D+ f)^T H g + f^T H (D- g) = f_N g_N - f_0 g_0
    (eq. upw_SBP), i.e. H D+ + (H D-)^T = B with B = diag(-1, 0, ..., 0, 1);
  * the upwind property: H (D+ - D-) symmetric negative semi-definite
    (Definition following eq. upw_SBP);
  * accuracy D x^k = k x^{k-1} (eq. acc): order 2p in the interior and p at
    the boundary closures for interior order 2p (interior order 2p + 1: p at
    the boundary);
  * the interior forward stencil alpha_j (Table tab:upwind) and the backward
    one beta_j = -alpha_{-j} (Sec. 6.2).

What it does not give: the boundary closures and the norm H (they live in
Mattsson 2017, which is not reproduced in the paper).  The oracle therefore
constructs its own closures:

  H D+- = A + B/2 +- S/2,
  S = -kappa Dp^T Dp      (Dp: undivided P-th difference, P = q, the forward
                           stencil's reach; kappa matches the interior of S
                           to twice the symmetric part of alpha),
  A skew-symmetric, Toeplitz with the antisymmetric part of alpha except for a
  free m x m block at the left end (and its antipersymmetric image at the
  right end), H = h diag(w_0..w_{m-1}, 1, ..., 1, w_{m-1}..w_0).

The accuracy conditions on the first m = order rows are linear in (w, free
block of A); they are solved exactly.  For orders 2 and 4 the solution is
unique.  For orders 3, 5, 6, 7 and 8 entries of the free block stay free
(one, two, one, four, three) and are fixed (FREE_ENTRIES) at values where the one-dimensional
elastic operator with characteristic boundary penalties has the smallest
spectral radius — no larger than the interior stencil's max |alpha^| — with
positive norm weights, taking the simplest rational among equivalent values:
order 3 A[1][2] = 1/2 (w = 7/12, 3/4, 7/6), order 5 A[2][4] = 1/4,
A[3][4] = 1/2 (w = 323/720, 203/240, 71/48, 451/720, 11/10), order 6
A[4][5] = 101/125, order 7 A[5][6] = 2/3, A[4][6] = A[3][6] = 0,
A[4][5] = 3/5 (radius 1.7495 at N = 120 against the interior 1.7504), order
8 A[6][7] = 5/6, A[5][7] = -1/5, A[5][6] = 3/4 (radius 2.352 at N = 80
against the interior 2.099: the radius depends sharply on these entries and
its minimum over them, about 2.24, lies at irrational values) (a reading; the
paper is silent).  Order 9 leaves seven entries free and is not constructed.
S annihilates polynomials of degree < P, so D+ and D- share the accuracy of
A + B/2.  The SBP identity and the semi-definiteness then hold by
construction and are pinned separately by the tests.
"""
from fractions import Fraction as Fr
from math import comb

import numpy as np

# Table tab:upwind: order -> (r, [alpha_{-r}, ..., alpha_{q}]).
# Order 8: the printed alpha_4 = +1/28 makes sum(alpha) = 1/14 != 0; the
# consistent value is -1/28 (reading).  Order 9: "2.0/21" read as 2/21.
UPWIND_ALPHA = {
    2: (0, [Fr(-3, 2), Fr(2), Fr(-1, 2)]),
    3: (1, [Fr(-1, 3), Fr(-1, 2), Fr(1), Fr(-1, 6)]),
    4: (1, [Fr(-1, 4), Fr(-5, 6), Fr(3, 2), Fr(-1, 2), Fr(1, 12)]),
    5: (2, [Fr(1, 20), Fr(-1, 2), Fr(-1, 3), Fr(1), Fr(-1, 4), Fr(1, 30)]),
    6: (2, [Fr(1, 30), Fr(-2, 5), Fr(-7, 12), Fr(4, 3), Fr(-1, 2), Fr(2, 15),
            Fr(-1, 60)]),
    7: (3, [Fr(-1, 105), Fr(1, 10), Fr(-3, 5), Fr(-1, 4), Fr(1), Fr(-3, 10),
            Fr(1, 15), Fr(-1, 140)]),
    8: (3, [Fr(-1, 168), Fr(1, 14), Fr(-1, 2), Fr(-9, 20), Fr(5, 4), Fr(-1, 2),
            Fr(1, 6), Fr(-1, 28), Fr(1, 280)]),
    9: (4, [Fr(1, 504), Fr(-1, 42), Fr(1, 7), Fr(-2, 3), Fr(-1, 5), Fr(1),
            Fr(-1, 3), Fr(2, 21), Fr(-1, 56), Fr(1, 630)]),
}

# Orders whose boundary closures this oracle constructs.
CLOSED_ORDERS = (2, 3, 4, 5, 6, 7, 8)

# Free closure entries (see module docstring).
ORDER6_FREE_A45 = Fr(101, 125)
FREE_ENTRIES = {
    3: {(1, 2): Fr(1, 2)},
    5: {(2, 4): Fr(1, 4), (3, 4): Fr(1, 2)},
    6: {(4, 5): ORDER6_FREE_A45},
    7: {(5, 6): Fr(2, 3), (4, 6): Fr(0), (3, 6): Fr(0), (4, 5): Fr(3, 5)},
    8: {(6, 7): Fr(5, 6), (5, 7): Fr(-1, 5), (5, 6): Fr(3, 4)},
}


def alpha_dict(order):
    """Interior forward stencil {j: alpha_j} (Table tab:upwind)."""
    r, coeffs = UPWIND_ALPHA[order]
    return {j - r: c for j, c in enumerate(coeffs)}


def beta_dict(order):
    """Interior backward stencil beta_j = -alpha_{-j} (Sec. 6.2)."""
    return {-j: -c for j, c in alpha_dict(order).items()}


def stencil_reach(order):
    """(r, q): the forward stencil reaches r points back and q forward."""
    al = alpha_dict(order)
    return -min(al), max(al)


def _solve_exact(rows, rhs, nunk):
    """Exact Gaussian elimination for a consistent (possibly overdetermined)
    linear system over the rationals.  Raises if inconsistent or if the
    solution is not unique."""
    M = [list(r) + [b] for r, b in zip(rows, rhs)]
    piv_cols = []
    rank = 0
    for col in range(nunk):
        pr = next((i for i in range(rank, len(M)) if M[i][col] != 0), None)
        if pr is None:
            continue
        M[rank], M[pr] = M[pr], M[rank]
        pv = M[rank][col]
        M[rank] = [x / pv for x in M[rank]]
        for i in range(len(M)):
            if i != rank and M[i][col] != 0:
                f = M[i][col]
                M[i] = [a - f * b for a, b in zip(M[i], M[rank])]
        piv_cols.append(col)
        rank += 1
    for i in range(rank, len(M)):
        if M[i][-1] != 0:
            raise ValueError("closure system is inconsistent")
    if rank != nunk:
        raise ValueError("closure system has %d free parameters" % (nunk - rank))
    x = [Fr(0)] * nunk
    for i, col in enumerate(piv_cols):
        x[col] = M[i][-1]
    return x


def closure(order):
    """Solve the boundary-closure conditions for interior order `order`.

    Returns dict with
      m      number of closure rows,
      q      forward reach (= difference order P of the dissipation),
      w      [w_0..w_{m-1}] boundary norm weights (Fractions),
      Ablk   m x m skew block of A (Fractions),
      a, s   antisymmetric / symmetric parts of alpha,
      kappa  dissipation scale.
    """
    if order not in CLOSED_ORDERS:
        raise ValueError("no closure for order %r (available: %s)" % (order, CLOSED_ORDERS))
    al = alpha_dict(order)
    r, q = stencil_reach(order)
    p = order // 2
    m = order
    P = q
    a = {j: (al.get(j, Fr(0)) - al.get(-j, Fr(0))) / 2 for j in range(1, q + 1)}
    s = {j: (al.get(j, Fr(0)) + al.get(-j, Fr(0))) / 2 for j in range(0, q + 1)}
    # interior row of Dp^T Dp is (-1)^j C(2P, P+j); match -kappa * it to 2 s_j
    kappa = -2 * s[0] / comb(2 * P, P)
    for j in range(0, q + 1):
        if -kappa * (-1) ** j * comb(2 * P, P + j) != 2 * s[j]:
            raise AssertionError("symmetric part of alpha is not a multiple of the 2P-th difference")

    # unknowns: w_0..w_{m-1}, then A[i][j] for 0 <= i < j < m
    pairs = [(i, j) for i in range(m) for j in range(i + 1, m)]
    nunk = m + len(pairs)
    uidx = {pr: m + k for k, pr in enumerate(pairs)}

    def A_known(i, j):
        # Toeplitz part outside the free block (rows < m, columns >= m)
        d = j - i
        if d > 0:
            return a.get(d, Fr(0))
        if d < 0:
            return -a.get(-d, Fr(0))
        return Fr(0)

    rows, rhs = [], []
    ncol = m + q  # columns touched by the first m rows
    for k in range(0, p + 1):
        for i in range(m):
            row = [Fr(0)] * nunk
            b = Fr(0)
            for j in range(ncol):
                xk = Fr(j) ** k if (j != 0 or k != 0) else Fr(1)
                if j < m:
                    if i < j:
                        row[uidx[(i, j)]] += xk
                    elif j < i:
                        row[uidx[(j, i)]] -= xk
                else:
                    b -= A_known(i, j) * xk
            if i == 0:  # (B/2)_{00} = -1/2
                b -= Fr(-1, 2) * (Fr(1) if k == 0 else Fr(0))
            # right-hand side k * w_i * x_i^{k-1}
            if k >= 1:
                xkm1 = Fr(i) ** (k - 1) if (i != 0 or k != 1) else Fr(1)
                row[i] -= k * xkm1
            rows.append(row)
            rhs.append(b)
    for pr, val in FREE_ENTRIES.get(order, {}).items():
        row = [Fr(0)] * nunk
        row[uidx[pr]] = Fr(1)
        rows.append(row)
        rhs.append(val)
    x = _solve_exact(rows, rhs, nunk)
    w = x[:m]
    Ablk = [[Fr(0)] * m for _ in range(m)]
    for (i, j), u in uidx.items():
        Ablk[i][j] = x[u]
        Ablk[j][i] = -x[u]
    return dict(order=order, m=m, q=q, r=r, p=p, w=w, Ablk=Ablk, a=a, s=s, kappa=kappa)


def min_points(order):
    """Smallest number of grid points per axis for which the two closures do
    not overlap."""
    return 2 * closure(order)["m"]


def operators_exact(order, npts):
    """Exact (Fraction) matrices for an axis with `npts` points on [0, 1].

    Returns dict with Hdiag (list), Dp, Dm, A, S, B (lists of lists), h.
    """
    c = closure(order)
    m, q, P = c["m"], c["q"], c["q"]
    N = npts
    if N < 2 * m:
        raise ValueError("need at least %d points for order %d" % (2 * m, order))
    h = Fr(1, N - 1)
    A = [[Fr(0)] * N for _ in range(N)]
    for i in range(N):
        for d in range(1, q + 1):
            if i + d < N:
                A[i][i + d] = c["a"][d]
                A[i + d][i] = -c["a"][d]
    for i in range(m):
        for j in range(m):
            A[i][j] = c["Ablk"][i][j]
            A[N - 1 - i][N - 1 - j] = -c["Ablk"][i][j]
    # S = -kappa Dp^T Dp
    drow = [(-1) ** (P - i) * comb(P, i) for i in range(P + 1)]
    S = [[Fr(0)] * N for _ in range(N)]
    for k in range(N - P):
        for i1 in range(P + 1):
            for i2 in range(P + 1):
                S[k + i1][k + i2] += -c["kappa"] * drow[i1] * drow[i2]
    B = [[Fr(0)] * N for _ in range(N)]
    B[0][0] = Fr(-1)
    B[N - 1][N - 1] = Fr(1)
    w = [c["w"][i] if i < m else (c["w"][N - 1 - i] if i >= N - m else Fr(1)) for i in range(N)]
    Hd = [h * wi for wi in w]
    Dp = [[(A[i][j] + B[i][j] / 2 + S[i][j] / 2) / Hd[i] for j in range(N)] for i in range(N)]
    Dm = [[(A[i][j] + B[i][j] / 2 - S[i][j] / 2) / Hd[i] for j in range(N)] for i in range(N)]
    return dict(Hdiag=Hd, Dp=Dp, Dm=Dm, A=A, S=S, B=B, h=h, w=w)


def operators(order, npts):
    """float64 operators for one axis: dict with H (diagonal, 1D array),
    Dp, Dm, D0 = (Dp + Dm)/2 (dense 2D arrays) and h."""
    ex = _operators_cached(order, npts)
    return ex


_cache = {}


def _operators_cached(order, npts):
    key = (order, npts)
    if key not in _cache:
        e = operators_exact(order, npts)
        Dp = np.array([[float(x) for x in row] for row in e["Dp"]])
        Dm = np.array([[float(x) for x in row] for row in e["Dm"]])
        _cache[key] = dict(H=np.array([float(x) for x in e["Hdiag"]]), Dp=Dp, Dm=Dm,
                           D0=0.5 * (Dp + Dm), h=float(e["h"]), w0=float(e["w"][0]))
    return _cache[key]
