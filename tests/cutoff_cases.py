"""Pair separations whose squared distance lies within a few ulps of rc^2 = 6.25, chosen
so that evaluating r^2 = (dx dx + dy dy) + dz dz with a fused multiply-add in place of a
product and a sum changes the cutoff decision (Algorithm 1 takes a pair when
r^2 <= rc^2).

Each component is an integer multiple of 2^-46, so for positions below 64 in magnitude
both atoms of a pair centred on a multiple of 2^-47 are exact doubles and their
difference is exactly the chosen separation.  The rounded values are computed with exact
rational arithmetic (Fraction -> float rounds to nearest even).
"""
from fractions import Fraction as Fr

import numpy as np

RC2 = Fr(25, 4)
Q = 2.0 ** -46


def _rnd(x: Fr) -> float:
    return float(x)


def r2_unfused(d) -> float:
    """((dx*dx) + (dy*dy)) + (dz*dz), every operation rounded to FP64."""
    dx, dy, dz = (Fr(float(v)) for v in d)
    xx, yy, zz = _rnd(dx * dx), _rnd(dy * dy), _rnd(dz * dz)
    return _rnd(Fr(_rnd(Fr(xx) + Fr(yy))) + Fr(zz))


def r2_fused_variants(d):
    """The values three plausible contractions of the same expression give."""
    dx, dy, dz = (Fr(float(v)) for v in d)
    xx, yy = _rnd(dx * dx), _rnd(dy * dy)
    s = _rnd(Fr(xx) + Fr(yy))
    return (_rnd(dz * dz + Fr(_rnd(dx * dx + Fr(yy)))),
            _rnd(dz * dz + Fr(_rnd(dy * dy + Fr(xx)))),
            _rnd(dz * dz + Fr(s)))


def flip_separations(count=48, seed=2024):
    """`count` separations (n x 3) whose cutoff decision differs between the unfused
    evaluation and at least one fused one; half of them in range unfused."""
    rng = np.random.default_rng(seed)
    inside, outside = [], []
    while len(inside) < count // 2 or len(outside) < count - count // 2:
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        d = np.round(u * 2.5 / Q) * Q
        plain = r2_unfused(d)
        if abs(plain - 6.25) > 4e-15:
            continue
        dp = Fr(plain) <= RC2
        if any((Fr(f) <= RC2) != dp for f in r2_fused_variants(d)):
            (inside if dp else outside).append(d)
    return np.array(inside[: count // 2] + outside[: count - count // 2])


def isolated_pair_system(seps, seed=5):
    """Pairs with the given separations, centred 7.5 apart on a grid in a periodic box
    (no atom has a partner other than its own); every coordinate is an exact double and
    every pair difference equals its separation exactly."""
    rng = np.random.default_rng(seed)
    n = len(seps)
    nx = 4
    ny = int(np.ceil(n / (nx * 4)))
    box = (7.5 * nx, 7.5 * ny if ny >= 3 else 22.5, 30.0)
    pos = []
    for k, d in enumerate(seps):
        i, j, l = k % nx, (k // nx) % max(ny, 3), k // (nx * max(ny, 3))
        c = np.array([3.75 + 7.5 * i, 3.75 + 7.5 * j, 3.75 + 7.5 * l])
        c += np.round(rng.uniform(-1.0, 1.0, 3) * 2.0 ** 20) * 2.0 ** -20
        pos += [c + 0.5 * d, c - 0.5 * d]
    pos = np.array(pos)
    assert (pos > 0).all() and (pos < np.array(box)).all()
    assert (pos[0::2] - pos[1::2] == seps).all()
    return box, pos
