"""Exact closed forms used as pins (test helpers; no oracle code here).

Uniform coupling J = a (11^T - I): when every spin starts at the same
position c and momentum 0, J q = a (N - 1) q for all n, so each spin follows
one scalar recurrence.  When the starting vector is orthogonal to 1 (an
alternating +-c pattern with N even), J q = -a q instead.  Either way the
whole trajectory is a scalar recurrence with k_eff = k - zeta_n * lam, where
lam is the eigenvalue of J on the starting direction, and the walls act
element-wise, so the recurrence with clamps stays exact.  Replaying it in
exact rational arithmetic (fractions.Fraction) pins the vector iteration.

``Dual`` carries a Fraction value and one exact Fraction derivative, which
gives exact schedule derivatives of the same recurrence.
"""
from __future__ import annotations

from fractions import Fraction as Fr


def clamp(x, lo, hi):
    if x < lo:
        return lo
    if x > hi:
        return hi
    return x


def scalar_replay(q0, p0, lam, dt, zeta, k, m, qmax, pmax, order="paper"):
    """Exact trajectory [(q_0, p_0), (q_1, p_1), ...] of the scalar recurrence."""
    q, p = Fr(q0), Fr(p0)
    k, m, lam, qmax, pmax = Fr(k), Fr(m), Fr(lam), Fr(qmax), Fr(pmax)
    out = [(q, p)]
    for d, z in zip(dt, zeta):
        d, z = Fr(d), Fr(z)
        if order == "paper":
            u = q + d / m * p
            v = p + d * (-k * q + z * lam * q)
            q, p = clamp(u, -qmax, qmax), clamp(v, -pmax, pmax)
        else:
            v = p + d * (-k * q + z * lam * q)
            p = clamp(v, -pmax, pmax)
            u = q + d / m * p
            q = clamp(u, -qmax, qmax)
        out.append((q, p))
    return out


class Dual:
    """a + b*eps with eps^2 = 0, over exact Fractions."""

    __slots__ = ("a", "b")

    def __init__(self, a, b=0):
        self.a = Fr(a)
        self.b = Fr(b)

    @staticmethod
    def lift(x):
        return x if isinstance(x, Dual) else Dual(x, 0)

    def __add__(self, o):
        o = Dual.lift(o)
        return Dual(self.a + o.a, self.b + o.b)

    __radd__ = __add__

    def __sub__(self, o):
        o = Dual.lift(o)
        return Dual(self.a - o.a, self.b - o.b)

    def __rsub__(self, o):
        return Dual.lift(o) - self

    def __neg__(self):
        return Dual(-self.a, -self.b)

    def __mul__(self, o):
        o = Dual.lift(o)
        return Dual(self.a * o.a, self.a * o.b + self.b * o.a)

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = Dual.lift(o)
        return Dual(self.a / o.a, (self.b * o.a - self.a * o.b) / (o.a * o.a))


def dual_clamp(x: Dual, lo, hi):
    """Clamp with the derivative 1 on the closed interval, 0 outside."""
    if x.a < lo:
        return Dual(lo, 0)
    if x.a > hi:
        return Dual(hi, 0)
    return x


def scalar_loss_derivative(q0, lam, dt, zeta, k, m, qmax, pmax, n_var, which):
    """Exact d/d(schedule entry n_var) of the relaxed energy of the uniform
    instance, per spin: L_spin = -1/2 lam q_S^2 (each spin has the same q).

    which = "dt" or "zeta".  Returns (value, derivative) as Fractions.
    """
    q, p = Dual(q0), Dual(0)
    k, m, lam = Fr(k), Fr(m), Fr(lam)
    qmax, pmax = Fr(qmax), Fr(pmax)
    for n, (d, z) in enumerate(zip(dt, zeta)):
        d = Dual(d, 1 if (which == "dt" and n == n_var) else 0)
        z = Dual(z, 1 if (which == "zeta" and n == n_var) else 0)
        u = q + d / m * p
        v = p + d * (-k * q + z * lam * q)
        q, p = dual_clamp(u, -qmax, qmax), dual_clamp(v, -pmax, pmax)
    L = Fr(-1, 2) * lam * q * q
    return L.a, L.b
