"""Exact float32 rounding for pin tests (independent of the oracle).

``fma_f32(a, b, c)`` is a*b + c computed exactly with rationals and rounded
once to the nearest float32 (ties to even), which is the IEEE definition of a
fused multiply-add.  numpy's float32 add, subtract and multiply are already
correctly rounded, so only the fused operation needs this.
"""
from fractions import Fraction

import numpy as np

_TWO = Fraction(2)


def f32_round(x: Fraction) -> np.float32:
    if x == 0:
        return np.float32(0.0)
    sign = -1 if x < 0 else 1
    x = abs(x)
    e = x.numerator.bit_length() - x.denominator.bit_length() - 24
    while x / _TWO ** e >= 2 ** 24:
        e += 1
    while x / _TWO ** e < 2 ** 23:
        e -= 1
    e = max(e, -149)
    q = x / _TWO ** e
    k = q.numerator // q.denominator
    r = q - k
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and k % 2 == 1):
        k += 1
    return np.float32(float(sign * k * _TWO ** e))


def fma_f32(a, b, c) -> np.float32:
    return f32_round(Fraction(float(np.float32(a))) * Fraction(float(np.float32(b))) + Fraction(float(np.float32(c))))


def dist2_f32(s, q) -> np.float32:
    """Squared distance with the fixed order dx*dx, fma(dy,dy,.), fma(dz,dz,.)."""
    s = [np.float32(v) for v in s]
    q = [np.float32(v) for v in q]
    dx, dy, dz = (np.float32(s[a] - q[a]) for a in range(3))
    return fma_f32(dz, dz, fma_f32(dy, dy, np.float32(dx * dx)))


def transform_f32(Rt, p):
    """fma(R0, x, fma(R1, y, fma(R2, z, t))) per row, all float32."""
    Rt = np.asarray(Rt, np.float32).reshape(12)
    x, y, z = (np.float32(v) for v in p)
    out = []
    for r in range(3):
        out.append(fma_f32(Rt[3 * r], x, fma_f32(Rt[3 * r + 1], y, fma_f32(Rt[3 * r + 2], z, Rt[9 + r]))))
    return out
