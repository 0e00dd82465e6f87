"""Five-stage, fourth-order, 2N-storage Runge-Kutta scheme (oracle side;
test infrastructure only).

The paper integrates in time with the low-storage fourth-order Runge-Kutta
method of Carpenter & Kennedy (1994) (Sec. 1 and Sec. 7) but does not print
its coefficients.  The values below are that method's published rational
coefficients; the tests pin them by the eight classical order-4 conditions of
the equivalent Butcher tableau and by the observed convergence order, not by
re-typing them.

One step from (Q, t) with step dt, for k = 0..4:
    dQ <- A[k] dQ + dt * RHS(Q, t + C[k] dt)
    Q  <- Q + B[k] dQ
(A[0] = 0, so the initial content of dQ is irrelevant.)
"""
from fractions import Fraction as Fr

A = [Fr(0),
     Fr(-567301805773, 1357537059087),
     Fr(-2404267990393, 2016746695238),
     Fr(-3550918686646, 2091501179385),
     Fr(-1275806237668, 842570457699)]
B = [Fr(1432997174477, 9575080441755),
     Fr(5161836677717, 13612068292357),
     Fr(1720146321549, 2090206949498),
     Fr(3134564353537, 4481467310338),
     Fr(2277821191437, 14882151754819)]
C = [Fr(0),
     Fr(1432997174477, 9575080441755),
     Fr(2526269341429, 6820363962896),
     Fr(2006345519317, 3224310063776),
     Fr(2802321613138, 2924317926251)]

A_F = [float(x) for x in A]
B_F = [float(x) for x in B]
C_F = [float(x) for x in C]
NSTAGE = 5


def step(Q, dQ, t, dt, rhs):
    """Advance (Q, dQ) in place by one step of size dt; rhs(Q, t) -> array."""
    for k in range(NSTAGE):
        dQ *= A_F[k]
        dQ += dt * rhs(Q, t + C_F[k] * dt)
        Q += B_F[k] * dQ
    return Q, dQ
