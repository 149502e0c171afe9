"""Exact rational segment/triangle predicate -- TEST INFRASTRUCTURE ONLY.

The same geometric statement as the FP64 oracle predicate, evaluated with
Python Fractions on the exact values of the FP32 inputs, so that every sign
is the sign of the real number.  Used on tiny adversarial inputs to pin the
FP64 predicate: the two must agree whenever no exact quantity lies within a
tiny relative band of zero.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _fr(v):
    return [Fraction(float(np.float32(x))) for x in np.asarray(v, np.float32).reshape(3)]


def _sub(a, b):
    return [a[0] - b[0], a[1] - b[1], a[2] - b[2]]


def _cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _mag_dot(a, b):
    return abs(a[0] * b[0]) + abs(a[1] * b[1]) + abs(a[2] * b[2])


def quantities(O, T, v0, v1, v2):
    """Exact plane sides sO, sT and edge orientations U, V, W, each with a
    magnitude scale (sum of absolute products) for relative-band checks."""
    O, T, v0, v1, v2 = (_fr(x) for x in (O, T, v0, v1, v2))
    m = _cross(_sub(v1, v0), _sub(v2, v0))
    mabs = [abs(x) for x in m]
    dO, dT = _sub(O, v0), _sub(T, v0)
    D = _sub(T, O)
    a, b, c = _sub(v0, O), _sub(v1, O), _sub(v2, O)
    out = {
        "sO": (_dot(dO, m), _mag_dot(dO, mabs)),
        "sT": (_dot(dT, m), _mag_dot(dT, mabs)),
    }
    for name, (p, q) in (("U", (b, c)), ("V", (c, a)), ("W", (a, b))):
        x = _cross(p, q)
        scale = sum(abs(D[i]) * (abs(p[(i + 1) % 3] * q[(i + 2) % 3]) + abs(p[(i + 2) % 3] * q[(i + 1) % 3]))
                    for i in range(3))
        out[name] = (_dot(D, x), scale)
    return out


def hit(O, T, v0, v1, v2) -> int:
    """Open segment O->T against the closed triangle, in exact arithmetic."""
    q = quantities(O, T, v0, v1, v2)
    sO, sT = q["sO"][0], q["sT"][0]
    if not ((sO > 0 and sT < 0) or (sO < 0 and sT > 0)):
        return 0
    U, V, W = q["U"][0], q["V"][0], q["W"][0]
    neg = U < 0 or V < 0 or W < 0
    pos = U > 0 or V > 0 or W > 0
    return int(not (neg and pos))


def near_boundary(O, T, v0, v1, v2, rel: float = 1e-12) -> bool:
    """True when some quantity the decision depends on is within rel of zero
    relative to its magnitude scale (there FP64 rounding may decide)."""
    q = quantities(O, T, v0, v1, v2)
    r = Fraction(rel)
    return any(abs(v) <= r * s for (v, s) in q.values())
