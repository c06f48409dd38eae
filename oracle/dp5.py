"""Dormand-Prince 5(4) time stepping with adaptive step size -- oracle side.

Test infrastructure only (see package docstring).

The paper evolves with a high-order Dormand-Prince stepper (section "The
Spectral Einstein Code", citing Numerical Recipes) without giving its
details.  Readings used here:

* the method is the published Dormand & Prince (1980) RK5(4)7M pair: seven
  stages, the fifth-order solution advanced, the embedded fourth-order one
  used only for the error estimate, last stage = first stage of the next step;
* the step control is the one of Numerical Recipes (3rd ed., section 17.2):
  per instance the error is the RMS over all its values of
  e_i / (atol + rtol max(|y_i(t)|, |y_i(t+h)|)); a step is accepted when that
  is <= 1; the next step is h times min(maxscale, max(minscale, safe err^-1/5))
  (maxscale when err = 0), not growing right after a rejection, with
  safe = 0.9, minscale = 0.2, maxscale = 10;
* the angular filter, when enabled, is applied after every accepted step.

The tableau is kept as exact rationals so that its order conditions can be
checked exactly.
"""

from fractions import Fraction as Fr

import numpy as np

C = [Fr(0), Fr(1, 5), Fr(3, 10), Fr(4, 5), Fr(8, 9), Fr(1), Fr(1)]
A = [
    [],
    [Fr(1, 5)],
    [Fr(3, 40), Fr(9, 40)],
    [Fr(44, 45), Fr(-56, 15), Fr(32, 9)],
    [Fr(19372, 6561), Fr(-25360, 2187), Fr(64448, 6561), Fr(-212, 729)],
    [Fr(9017, 3168), Fr(-355, 33), Fr(46732, 5247), Fr(49, 176), Fr(-5103, 18656)],
    [Fr(35, 384), Fr(0), Fr(500, 1113), Fr(125, 192), Fr(-2187, 6784), Fr(11, 84)],
]
B = A[6] + [Fr(0)]                                   # fifth order (advanced)
BHAT = [Fr(5179, 57600), Fr(0), Fr(7571, 16695), Fr(393, 640), Fr(-92097, 339200), Fr(187, 2100),
        Fr(1, 40)]                                   # embedded fourth order
E = [b - bh for b, bh in zip(B, BHAT)]               # error weights

SAFE, MINSCALE, MAXSCALE, EXPONENT = 0.9, 0.2, 10.0, 0.2


def stages(u, h, rhs, k1=None):
    """The seven stage derivatives and the fifth-order solution of one step.

    u: state array; h: step (scalar or array broadcasting against u);
    rhs: u -> du/dt.  Returns (u5, [k1..k7]); k7 = rhs(u5).
    """
    k = [rhs(u) if k1 is None else k1]
    for i in range(1, 7):
        y = u + h * sum(float(a) * kj for a, kj in zip(A[i], k) if a != 0)
        k.append(rhs(y))
    # stage 7 is evaluated at u5 = u + h sum_j B_j k_j, the row A[6]
    u5 = u + h * sum(float(b) * kj for b, kj in zip(B, k) if b != 0)
    return u5, k


def error_vector(k, h):
    """h sum_j (B_j - BHAT_j) k_j, the difference of the 5th and 4th order steps."""
    return h * sum(float(e) * kj for e, kj in zip(E, k) if e != 0)


def error_norm(err, u, u5, atol, rtol):
    """RMS of err / (atol + rtol max(|u|, |u5|)) over all given values."""
    sk = atol + rtol * np.maximum(np.abs(u), np.abs(u5))
    return float(np.sqrt(np.mean((err / sk) ** 2)))


def control(err, prev_rejected):
    """(accept, factor for the next step) from the scaled error norm."""
    if err <= 1.0:
        if err == 0.0:
            scale = MAXSCALE
        else:
            scale = min(MAXSCALE, max(MINSCALE, SAFE * err ** (-EXPONENT)))
        if prev_rejected:
            scale = min(scale, 1.0)
        return True, scale
    return False, max(MINSCALE, SAFE * err ** (-EXPONENT))
