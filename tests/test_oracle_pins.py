"""Pins of the oracle parts that the GPU parity tests at scale lean on:

  * the force-error normaliser S_i = sum over in-range partners of 24 (2 r^-13 + r^-7)
    (the magnitudes of the repulsive and attractive terms of the pair force), pinned
    from both sides: each pair's term equals the exact rational value at eight
    separations, and each atom's sum equals the sum over a pair list enumerated
    independently (all pairs, minimum image, plain numpy) -- so an inflated or
    deflated S_i, which would loosen or tighten every force gate, fails here;
  * the subset force routine (the 1% subsample of the precision study, Sec. 4 LJ
    forces) against the full cell-list routine, row for row and bitwise;
  * the normalised force-error metric on hand-made cases.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import ref
from paper_2507_11289_amd import inputs

RADII = [0.9, 1.0, 2.0 ** (1.0 / 6.0), 1.1, 1.5, 2.0, 2.4, 2.5]


def scale_def(r: Fr) -> Fr:
    """|d/dr of 4 r^-12| + |d/dr of 4 r^-6| = 48 r^-13 + 24 r^-7."""
    return 48 * r ** -13 + 24 * r ** -7


@pytest.mark.parametrize("r", RADII)
def test_pair_scale_equals_the_sum_of_term_magnitudes(r):
    g = ref.geometry([40.0, 40.0, 40.0], 4, 2.5)
    ri = np.array([10.0, 10.0, 10.0])
    rj = np.array([10.0, 10.0 + r, 10.0])
    rr = Fr(rj[1]) - Fr(ri[1])
    inr, _, _, _, s, _ = ref.pair(g, ri, rj)
    assert inr
    assert s == pytest.approx(float(scale_def(rr)), rel=1e-13)


def test_pair_scale_is_zero_out_of_range():
    g = ref.geometry([40.0, 40.0, 40.0], 4, 2.5)
    inr, f, u, w, s, _ = ref.pair(g, [10.0, 10.0, 10.0], [10.0, 10.0, 12.75])
    assert not inr and s == 0.0


def enumerate_pairs(box, pos, rc):
    """Every unordered pair within rc under the minimum-image rule (plain numpy, no cells)."""
    L = np.asarray(box, dtype=np.float64)
    n = len(pos)
    ii, jj = np.triu_indices(n, 1)
    d = pos[ii] - pos[jj]
    d -= L * np.round(d / L)
    r2 = (d * d).sum(axis=1)
    keep = r2 <= rc * rc
    return ii[keep], jj[keep], np.sqrt(r2[keep])


@pytest.mark.parametrize("n,rho,aspect,slices", [(500, 0.8, (1, 1, 1), 3), (700, 0.5, (2, 1, 1), 4),
                                                 (600, 0.3, (1, 1, 1), 3)])
def test_atom_scale_is_the_sum_over_an_independent_pair_list(n, rho, aspect, slices):
    box, pos, _, _ = inputs.homogeneous(n, rho, 1.0, 29, aspect=aspect)
    g = ref.geometry(box, slices, 2.5)
    c = ref.forces_cells(g, pos)
    ii, jj, r = enumerate_pairs(box, pos, 2.5)
    term = 48.0 * r ** -13 + 24.0 * r ** -7
    S = np.zeros(n)
    np.add.at(S, ii, term)
    np.add.at(S, jj, term)
    cnt = np.bincount(ii, minlength=n) + np.bincount(jj, minlength=n)
    np.testing.assert_array_equal(c["inr"], cnt)
    np.testing.assert_allclose(c["scale"], S, rtol=1e-12, atol=0.0)
    # S_i bounds the force: |F_i| <= S_i, and it is not loose by a constant factor
    Fn = np.linalg.norm(c["F"], axis=1)
    assert (Fn <= c["scale"] * (1 + 1e-12)).all()
    assert np.median(Fn / c["scale"]) > 0.01


def test_subset_forces_are_rows_of_the_full_forces_bitwise():
    s = inputs.lj_fluid_2048()
    g = ref.geometry(s.box, s.slices, s.rc)
    full = ref.forces_cells(g, s.pos)
    rng = np.random.default_rng(3)
    n = s.n
    for ids in (np.array([0, n - 1]), np.array([5, 5, 17, 5, n - 1, 0, 0]),
                rng.integers(0, n, 300), np.arange(n)):
        sub = ref.forces_subset(g, s.pos, ids)
        np.testing.assert_array_equal(sub["F"], full["F"][ids])
        np.testing.assert_array_equal(sub["scale"], full["scale"][ids])
        np.testing.assert_array_equal(sub["cand"], full["cand"][ids])
        np.testing.assert_array_equal(sub["inr"], full["inr"][ids])
    # an empty subset and a bad id
    assert len(ref.forces_subset(g, s.pos, np.zeros(0, np.int64))["F"]) == 0
    with pytest.raises(ref.OracleError):
        ref.forces_subset(g, s.pos, np.array([n]))
    with pytest.raises(ref.OracleError):
        ref.forces_subset(g, s.pos, np.array([-1]))


def test_subset_forces_on_a_moved_state_match_full_forces():
    """Positions after some steps (atoms in other cells than at t = 0)."""
    s = inputs.lj_fluid_2048()
    g = ref.geometry(s.box, s.slices, s.rc)
    pos = ref.run(g, s.pos, s.vel, s.dt, 20)["pos"]
    full = ref.forces_cells(g, pos)
    ids = np.arange(0, s.n, 7)
    sub = ref.forces_subset(g, pos, ids)
    np.testing.assert_array_equal(sub["F"], full["F"][ids])
    np.testing.assert_array_equal(sub["scale"], full["scale"][ids])


def test_force_error_hand_made_cases():
    Fref = np.array([[1.0, 2.0, 3.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [-1.0, 0.5, 0.25],
                     [0.0, 0.0, 0.0]])
    Ftest = np.array([[1.0, 2.0, 3.0],      # equal: 0
                      [0.0, 0.0, 0.0],      # no partners, exactly zero: 0
                      [0.0, 1e-300, 0.0],   # no partners, not zero: inf
                      [2.0, 4.5, 0.25],     # difference (3, 4, 0): |d| = 5
                      [3.0, 0.0, 4.0]])     # difference (3, 0, 4), S = 2.5
    S = np.array([7.0, 0.0, 0.0, 10.0, 2.5])
    e = ref.force_error(Ftest, Fref, S)
    assert e[0] == 0.0 and e[1] == 0.0
    assert np.isinf(e[2])
    assert e[3] == 0.5
    assert e[4] == 2.0
    # flat arrays are read as n x 3
    np.testing.assert_array_equal(ref.force_error(Ftest.ravel(), Fref.ravel(), S), e)
    # the error is the Euclidean norm of the difference, symmetric in its arguments
    np.testing.assert_array_equal(ref.force_error(Fref, Ftest, S), e)
