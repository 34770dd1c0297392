"""Pins of the oracle's pair terms (Algorithm 1 neighbour-loop body) against the
Lennard-Jones definition evaluated in exact rational arithmetic.

The test only states the potential, U(r) = 4 (r^-12 - r^-6) shifted to vanish at
rc (Sec. 4: truncated and shifted LJ, sigma = epsilon = 1, rc = 2.5).  The force
is obtained by differentiating that definition (exact rational central difference
with a 1e-40 step), and the virial of a pair is r * |F|.  A dropped factor, a
wrong sign or a wrong power anywhere in the oracle's pair function fails here.
"""
from fractions import Fraction as Fr
import math

import numpy as np
import pytest

from oracle import ref

RC = Fr(5, 2)


def U_def(r: Fr) -> Fr:
    return 4 * (r ** -12 - r ** -6) - 4 * (RC ** -12 - RC ** -6)


def F_def(r: Fr) -> Fr:
    """-dU/dr: positive = repulsive."""
    h = Fr(1, 10 ** 40)
    return -(U_def(r + h) - U_def(r - h)) / (2 * h)


@pytest.fixture(scope="module")
def geom():
    # a large cubic box so that no periodic image interferes
    return ref.geometry([40.0, 40.0, 40.0], 4, 2.5)


RADII = [0.9, 1.0, 2.0 ** (1.0 / 6.0), 1.1, 1.5, 2.0, 2.4, 2.5]


@pytest.mark.parametrize("r", RADII)
def test_pair_matches_lj_definition(geom, r):
    ri = np.array([10.0, 10.0, 10.0])
    rj = np.array([10.0 + r, 10.0, 10.0])
    rr = Fr(rj[0]) - Fr(ri[0])  # exact separation as stored
    inr, f, u, w, s, r2 = ref.pair(geom, ri, rj)
    assert inr
    Fexact = F_def(rr)
    # force on i points away from j when repulsive: f_x = -F(r)
    assert f[0] == pytest.approx(float(-Fexact), rel=1e-13, abs=1e-13)
    assert f[1] == 0.0 and f[2] == 0.0
    assert u == pytest.approx(float(U_def(rr)), rel=1e-13, abs=1e-14)
    assert w == pytest.approx(float(rr * Fexact), rel=1e-13, abs=1e-13)
    # scale = |repulsive term| + |attractive term| of the force magnitude
    assert s >= abs(float(Fexact)) * (1 - 1e-14)


def test_minimum_of_the_potential(geom):
    """At r = 2^(1/6) sigma the LJ force vanishes and the unshifted energy is -epsilon."""
    r = 2.0 ** (1.0 / 6.0)
    _, f, u, w, _, _ = ref.pair(geom, [5.0, 5.0, 5.0], [5.0, 5.0 + r, 5.0])
    assert abs(f[1]) < 1e-14 and abs(w) < 1e-13
    uc = float(4 * (RC ** -12 - RC ** -6))
    assert u == pytest.approx(-1.0 - uc, abs=1e-14)


def test_zero_crossing_at_sigma(geom):
    _, f, u, w, _, _ = ref.pair(geom, [5.0, 5.0, 5.0], [5.0, 5.0, 6.0])
    uc = float(4 * (RC ** -12 - RC ** -6))
    assert u == -uc or u == pytest.approx(-uc, abs=1e-16)
    assert f[2] == -24.0 and w == 24.0  # exact at r = 1


def test_dyadic_separation_is_bit_exact(geom):
    """r = 2: r^-2 = 1/4, r^-6 = 1/64, every intermediate is dyadic."""
    _, f, u, w, _, r2 = ref.pair(geom, [1.0, 7.0, 7.0], [3.0, 7.0, 7.0])
    assert r2 == 4.0
    assert f[0] == 0.181640625      # attraction pulls i (left) towards +x
    assert w == -0.36328125


def test_cutoff_is_inclusive(geom):
    """Algorithm 1 takes a pair when r^2 <= rc^2; r = 2.5 exactly is in range."""
    inr, f, u, w, _, r2 = ref.pair(geom, [1.0, 7.0, 7.0], [3.5, 7.0, 7.0])
    assert r2 == 6.25 and inr
    assert u == 0.0 or abs(u) < 1e-17
    assert f[0] == pytest.approx(float(-F_def(RC)), rel=1e-13)
    assert f[0] == pytest.approx(0.0389994774528, rel=1e-11)
    inr2, f2, _, _, _, _ = ref.pair(geom, [1.0, 7.0, 7.0], [np.nextafter(3.5, 9.0), 7.0, 7.0])
    assert not inr2 and f2[0] == 0.0


def test_newton_pair_antisymmetry(geom):
    rng = np.random.default_rng(1)
    for _ in range(50):
        a = rng.uniform(0, 40, 3)
        b = a + rng.uniform(-1.4, 1.4, 3)
        _, f1, u1, w1, _, _ = ref.pair(geom, a, b)
        _, f2, u2, w2, _, _ = ref.pair(geom, b, a)
        np.testing.assert_array_equal(f1, -f2)
        assert u1 == u2 and w1 == w2


def test_minimum_image_across_the_boundary():
    L = 9.0
    g = ref.geometry([L, L, L], 3, 2.5)
    inr, f, u, w, _, r2 = ref.pair(g, [0.5, 4.0, 4.0], [L - 0.5, 4.0, 4.0])
    assert inr and r2 == 1.0
    assert f[0] == 24.0     # repulsion pushes the atom at 0.5 towards +x
    inr, f, *_ = ref.pair(g, [L - 0.5, 4.0, 4.0], [0.5, 4.0, 4.0])
    assert f[0] == -24.0


def test_energy_shift_value(geom):
    assert geom.uc == pytest.approx(float(4 * (RC ** -12 - RC ** -6)), rel=1e-15)
    assert geom.uc == pytest.approx(-0.016316891136, rel=1e-10)


def test_cutoff_decision_uses_unfused_r2():
    """r^2 is (dx dx + dy dy) + dz dz with every operation rounded (no fused multiply-add):
    on separations whose decision a fused evaluation would flip, the oracle's r^2 is the
    unfused value bit for bit and its decision follows it."""
    from tests.cutoff_cases import flip_separations, r2_unfused
    g = ref.geometry([60.0, 60.0, 60.0], 4, 2.5)
    seps = flip_separations(24)
    n_in = 0
    for d in seps:
        ri = np.array([30.0, 30.0, 30.0])
        rj = ri - d
        assert (ri - rj == d).all()
        inr, _, _, _, _, r2 = ref.pair(g, ri, rj)
        assert r2 == r2_unfused(d)
        assert inr == (r2 <= 6.25)
        n_in += inr
    assert 0 < n_in < len(seps)
