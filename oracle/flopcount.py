"""Floating-point operation counts of the oracle's pointwise GH algebra.

Test infrastructure, like the rest of this package.  A scalar type that
counts every +, -, *, / and square root is pushed through
gh.rhs_pointwise and gh.constraints_pointwise at one point.  The count is
that of the formulas as written (full 4x4 tensors, no use of symmetry), once
with the einsum contractions evaluated in the order they are written and once
in the cheapest pairwise order numpy finds; the second is the figure quoted
for the pointwise kernel's arithmetic (an upper bound on what a symmetric,
register-resident implementation needs).
"""

import functools
import math

import numpy as np

from . import gh


class Counted:
    """A float that counts the arithmetic done on it (shared counter)."""

    n = 0
    __slots__ = ("v",)

    def __init__(self, v):
        self.v = float(v)

    @staticmethod
    def _v(o):
        return o.v if isinstance(o, Counted) else o

    def _op(self, r):
        Counted.n += 1
        return Counted(r)

    def __add__(self, o):
        return self._op(self.v + Counted._v(o))

    def __radd__(self, o):
        return self._op(Counted._v(o) + self.v)

    def __sub__(self, o):
        return self._op(self.v - Counted._v(o))

    def __rsub__(self, o):
        return self._op(Counted._v(o) - self.v)

    def __mul__(self, o):
        return self._op(self.v * Counted._v(o))

    def __rmul__(self, o):
        return self._op(Counted._v(o) * self.v)

    def __truediv__(self, o):
        return self._op(self.v / Counted._v(o))

    def __rtruediv__(self, o):
        return self._op(Counted._v(o) / self.v)

    def __neg__(self):
        return Counted(-self.v)

    def __pos__(self):
        return self

    def sqrt(self):
        return self._op(math.sqrt(self.v))


_wrap = np.vectorize(Counted, otypes=[object])
_unwrap = np.vectorize(lambda x: x.v if isinstance(x, Counted) else float(x), otypes=[float])


def count(fn, *arrays, optimal=False):
    """(flops, float result) of fn(*arrays) evaluated with counting scalars.

    Non-array trailing arguments can be bound with functools.partial.  With
    optimal=True every einsum in the oracle's gh module runs with numpy's
    optimal contraction order for the duration of the call.
    """
    Counted.n = 0
    wrapped = [_wrap(np.asarray(a, dtype=float)) for a in arrays]
    orig = gh.np.einsum
    if optimal:
        gh.np.einsum = functools.partial(orig, optimize="optimal")
    try:
        out = fn(*wrapped)
    finally:
        gh.np.einsum = orig
    return Counted.n, _unwrap(out)


def pointwise_rhs_flops(u, du, H, dH, gammas, optimal=True):
    """Flops of gh.rhs_pointwise at the points given (usually one)."""
    fn = functools.partial(_rhs, gammas=gammas)
    return count(fn, u, du, H, dH, optimal=optimal)


def _rhs(u, du, H, dH, gammas):
    return gh.rhs_pointwise(u, du, H, dH, *gammas)


def constraint_flops(u, du, H, optimal=True):
    """Flops of gh.constraints_pointwise at the points given."""
    return count(gh.constraints_pointwise, u, du, H, optimal=optimal)
