"""Five-stage fourth-order low-storage Runge-Kutta (oracle, FP64).

The paper does not name its time integrator (Sec. II-A ends with the
semi-discrete system (26)-(29); Sec. III gives no scheme).  The reading taken
here is the 2N-storage scheme of Carpenter and Kennedy (1994, "Fourth-order
2N-storage Runge-Kutta schemes", NASA TM-109112, solution 3):

    res <- A_i res + dt * rhs(q, t + c_i dt)
    q   <- q + B_i res,            i = 1..5,  res = 0 at the start of a step.

The published rational constants meet the order conditions to about 1e-25
(far below FP64 rounding), not exactly.

Parity: pinned by tests/test_oracle_lserk.py (rational-arithmetic stability
polynomial 1 + z + z^2/2 + z^3/6 + z^4/24 + z^5/200, stage times equal the
c_i, fourth-order convergence on y' = lambda y + cos t).
"""
from __future__ import annotations

from fractions import Fraction as Fr

A_FR = (Fr(0), Fr(-567301805773, 1357537059087), Fr(-2404267990393, 2016746695238),
        Fr(-3550918686646, 2091501179385), Fr(-1275806237668, 842570457699))
B_FR = (Fr(1432997174477, 9575080441755), Fr(5161836677717, 13612068292357),
        Fr(1720146321549, 2090206949498), Fr(3134564353537, 4481467310338),
        Fr(2277821191437, 14882151754819))
C_FR = (Fr(0), Fr(1432997174477, 9575080441755), Fr(2526269341429, 6820363962896),
        Fr(2006345519317, 3224310063776), Fr(2802321613138, 2924317926251))

A = tuple(float(x) for x in A_FR)
B = tuple(float(x) for x in B_FR)
C = tuple(float(x) for x in C_FR)


def step(rhs, q, t: float, dt: float):
    """One LSERK4 step of q' = rhs(q, t); returns the new q (input not modified)."""
    q = q.copy()
    res = None
    for i in range(5):
        k = rhs(q, t + C[i] * dt)
        res = dt * k if res is None else A[i] * res + dt * k
        q = q + B[i] * res
    return q
