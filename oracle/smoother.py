"""Low-storage additive pseudo-time smoothers (Section 4).

Section 4.1 (preconditioned additive RK) and Section 4.2 (additive W,
low-storage form at the end of the section) share one algorithm:

    u(0) = u
    u(i) = u - alpha_i dt* P^-1 (f^c,(i-1) + f^v,(i-1)),   i = 1..s
    f^c,(i) = f^c(u(i))
    f^v,(0) = f^v(u(0))
    f^v,(i) = beta_{i+1} f^v(u(i)) + (1 - beta_{i+1}) f^v,(i-1)
    new iterate u(s)

(the printed "beta_{j+1}" of the blended line is read as beta_{i+1}).
The additive W method uses P = W ~ I + eta dt* J; the preconditioned ARK
method uses P ~ J.  Coefficients: Table "RK smoothers"; "AW3" is ARK3J's
alpha and beta with the W preconditioner; the five-stage schemes use the
ARK5J beta.  Setting every beta to 1 gives the unsplit (ERK / W) forms.

Reading (local pseudo time step): dt* differs from cell to cell, and W is
row-scaled by it (W ~ I + eta dt* J, eqs. "d-l-u-matrices-W").  The W step
of the locally time-stepped pseudo-time problem u_t* = -dt* F(u) applies
W^-1 to the scaled residual, dt*_c F_c, i.e. it solves
(dt*^-1 + eta J) du = -F.  Multiplying W^-1 F by dt* afterwards, which is
the same thing only for a uniform dt*, is not A-stable even with an exact
W on stretched grids.  The preconditioned ARK methods are explicit in the
preconditioned residual and keep dt* P^-1 F.
"""
from __future__ import annotations

import numpy as np

AW3, PARK3J, AW5J, AW51, AW52, PARK51 = 0, 1, 2, 3, 4, 5

_B3 = (1.0, 0.5, 0.5)
_B5 = (1.0, 0.0, 0.56, 0.0, 0.44)
SCHEMES = {
    # id: (alpha, beta, uses W (True) or P ~ J (False))
    AW3: ((0.1481, 2.0 / 5.0, 1.0), _B3, True),
    PARK3J: ((0.1481, 2.0 / 5.0, 1.0), _B3, False),
    AW5J: ((1.0 / 4.0, 1.0 / 6.0, 3.0 / 8.0, 1.0 / 2.0, 1.0), _B5, True),
    AW51: ((0.0533, 0.1263, 0.2375, 0.4414, 1.0), _B5, True),
    AW52: ((0.0695, 0.1602, 0.2898, 0.5060, 1.0), _B5, True),
    PARK51: ((0.0533, 0.1263, 0.2375, 0.4414, 1.0), _B5, False),
}


def additive_iteration(u0, split, increment, alpha, beta):
    """One smoother iteration.

    split(u)      -> (f^c(u), f^v(u))
    increment(r)  -> the stage increment per unit alpha for the stage
                     residual r: W^-1 (dt* r) for the additive W methods,
                     dt* P^-1 r for the preconditioned ARK methods
    The stage value is u(i) = u(0) - alpha_i * increment(r).
    """
    s = len(alpha)
    fc, fv = split(u0)
    acc = fv
    u = u0
    for i in range(s):
        x = increment(fc + acc)
        u = u0 - alpha[i] * x
        if i < s - 1:
            fc, fv = split(u)
            b = beta[i + 1]
            acc = b * fv + (1.0 - b) * acc
    return u
