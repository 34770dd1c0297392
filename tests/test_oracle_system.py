"""Pins of the oracle's many-atom parts: cell list vs brute force, Newton's third
law, energy/force and virial consistency (finite differences of the oracle's own
energy), binning on adversarial coordinates, free flight with closed-form
migration steps, NVE conservation, time reversibility and the guards."""
from fractions import Fraction as Fr
import math

import numpy as np
import pytest

from oracle import ref
from paper_2507_11289_amd import inputs


def small_system(n=500, rho=0.8, T=1.0, seed=7, aspect=(1.0, 1.0, 1.0)):
    box, pos, vel, _ = inputs.homogeneous(n, rho, T, seed, aspect=aspect)
    return box, pos, vel


def norm_err(F, Fr_, scale):
    e = ref.force_error(F, Fr_, scale)
    return float(e.max())


@pytest.mark.parametrize("n,rho,aspect,slices", [
    (500, 0.8, (1, 1, 1), 3),
    (700, 0.5, (2, 1, 1), 4),
    (400, 0.3, (1, 1, 1), 3),
    (1200, 0.9, (3, 1, 1), 3),   # w = 2.5*... gives several cell layers per slice
])
def test_cells_equal_brute_force(n, rho, aspect, slices):
    box, pos, _ = small_system(n, rho, aspect=aspect)
    g = ref.geometry(box, slices, 2.5)
    Fb, Ub, Wb, Pb = ref.forces_brute(g, pos)
    c = ref.forces_cells(g, pos)
    assert int(c["inr"].sum()) == 2 * Pb          # identical pair set
    assert norm_err(c["F"], Fb, c["scale"]) <= 1e-13
    assert c["u_half"].sum() == pytest.approx(Ub, rel=1e-12)
    assert c["w_half"].sum() == pytest.approx(Wb, rel=1e-12)


def test_candidate_counts_follow_the_27_cell_stencil():
    box, pos, _ = small_system(900, 0.8, aspect=(2, 1, 1))
    g = ref.geometry(box, 4, 2.5)
    gxyz, _, _ = ref.bin_atoms(g, pos)
    G = np.array(list(g.G))
    occ = np.zeros(G, np.int64)
    np.add.at(occ, (gxyz[:, 0], gxyz[:, 1], gxyz[:, 2]), 1)
    nb = np.zeros_like(occ)
    for ox in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for oz in (-1, 0, 1):
                nb += np.roll(occ, (ox, oy, oz), axis=(0, 1, 2))
    expect = nb[gxyz[:, 0], gxyz[:, 1], gxyz[:, 2]] - 1
    c = ref.forces_cells(g, pos)
    np.testing.assert_array_equal(c["cand"], expect)
    assert (c["inr"] <= c["cand"]).all()


def test_newton_third_law_and_momentum():
    sys_ = inputs.lj_fluid_2048()
    g = ref.geometry(sys_.box, sys_.slices, 2.5)
    c = ref.forces_cells(g, sys_.pos)
    tot = np.abs(c["F"]).sum()
    assert np.linalg.norm(c["F"].sum(axis=0)) <= 1e-12 * tot


def test_energy_force_consistency():
    """F = -dU/dx by central differences of the oracle's total energy."""
    box, pos, vel = small_system(600, 0.7, seed=3)
    g = ref.geometry(box, 3, 2.5)
    F = ref.forces_cells(g, pos)["F"]
    h = 1e-6
    rng = np.random.default_rng(5)
    for i in rng.choice(len(pos), 6, replace=False):
        for d in range(3):
            p1 = pos.copy(); p1[i, d] += h
            p2 = pos.copy(); p2[i, d] -= h
            U1 = ref.energy(g, p1, vel)[0]
            U2 = ref.energy(g, p2, vel)[0]
            fd = -(U1 - U2) / (2 * h)
            assert fd == pytest.approx(F[i, d], rel=2e-5, abs=2e-5)


def test_virial_is_minus_volume_derivative():
    """W = sum r_ij . f_ij = -dU(lambda r)/dlambda at lambda = 1 (box scaled with r)."""
    box, pos, vel = small_system(600, 0.7, seed=4)
    g = ref.geometry(box, 3, 2.5)
    U0, _, W = ref.energy(g, pos, vel)
    h = 1e-7
    vals = []
    for lam in (1 + h, 1 - h):
        b = [x * lam for x in box]
        gl = ref.geometry(b, 3, 2.5)
        vals.append(ref.energy(gl, pos * lam, vel)[0])
    dU = (vals[0] - vals[1]) / (2 * h)
    assert -dU == pytest.approx(W, rel=1e-5)


def exact_floor_cell(x: float, L: float, G: int) -> int:
    """floor(x / (L/G)) in exact arithmetic, clamped."""
    q = Fr(x) * G / Fr(L)
    return min(max(math.floor(q), 0), G - 1)


def test_binning_adversarial_coordinates():
    box = [20.0 * 1.0000001, 9.3, 11.7]
    g = ref.geometry(box, 3, 2.5)
    xs = []
    for d in range(3):
        l = box[d] / g.G[d]
        vals = [0.0, -0.0, box[d], np.nextafter(box[d], 0.0)]
        for k in range(g.G[d] + 1):
            x = k * l
            vals += [x, np.nextafter(x, -1.0), np.nextafter(x, 1e9)]
        xs.append([v for v in vals if 0.0 <= v <= box[d]])
    m = max(len(v) for v in xs)
    pos = np.zeros((m, 3))
    for d in range(3):
        col = np.resize(np.array(xs[d]), m)
        pos[:, d] = col
    gxyz, sl, cell = ref.bin_atoms(g, pos)
    for d in range(3):
        assert gxyz[:, d].min() >= 0 and gxyz[:, d].max() <= g.G[d] - 1
        # monotone in the coordinate
        o = np.argsort(pos[:, d], kind="stable")
        assert (np.diff(gxyz[o, d]) >= 0).all()
        for x, c in zip(pos[:, d], gxyz[:, d]):
            ex = exact_floor_cell(float(x), box[d], g.G[d])
            # a single rounding of x * (1/l) can only move an exact boundary value
            assert abs(int(c) - ex) <= 1
            if x == box[d]:
                assert c == g.G[d] - 1
            lo = Fr(box[d]) / g.G[d] * ex
            if abs(Fr(float(x)) - lo) > Fr(1, 10 ** 9) and abs(Fr(float(x)) - lo - Fr(box[d]) / g.G[d]) > Fr(1, 10 ** 9):
                assert c == ex
    np.testing.assert_array_equal(sl, gxyz[:, 0] // g.ncx)
    # global cell id: slice-major, then x layer within the slice, then y, then z
    local = ((gxyz[:, 0] % g.ncx) * g.G[1] + gxyz[:, 1]) * g.G[2] + gxyz[:, 2]
    np.testing.assert_array_equal(cell, sl.astype(np.int64) * g.cells_per_slice + local)


def test_geometry_rules():
    g = ref.geometry([173.72269, 173.72269, 173.72269], 64, 2.5)
    assert g.ncx == 1 and g.G[0] == 64 and g.G[1] == 69 and g.G[2] == 69
    for d in range(3):
        assert g.l[d] > 2.5
    # an exact multiple of rc loses one cell (cell edge must exceed rc)
    g2 = ref.geometry([30.0, 10.0, 10.0], 3, 2.5)
    assert g2.G[1] == 3 and g2.l[1] > 2.5 and g2.ncx == 3
    with pytest.raises(ref.OracleError):
        ref.geometry([6.0, 10.0, 10.0], 3, 2.5)   # slice narrower than rc
    with pytest.raises(ref.OracleError):
        ref.geometry([30.0, 7.4, 10.0], 3, 2.5)  # fewer than 3 cells in y
    with pytest.raises(ref.OracleError):
        ref.geometry([30.0, 10.0, 10.0], 2, 2.5)


def free_flight_system():
    """Atoms 3 sigma apart (beyond rc) moving together: forces stay exactly zero."""
    box = [12.0, 9.0, 9.0]
    pts = []
    for i in range(4):
        for j in range(3):
            for k in range(3):
                pts.append([0.25 + 3.0 * i, 0.5 + 3.0 * j, 0.75 + 3.0 * k])
    pos = np.array(pts)
    vel = np.tile(np.array([[1.0, -0.5, 0.25]]), (len(pos), 1))
    return box, pos, vel


def test_free_flight_is_exact_and_migrations_follow_closed_form():
    box, pos, vel = free_flight_system()
    g = ref.geometry(box, 3, 2.5)          # slices of width 4 along x
    dt = 2.0 ** -8
    nsteps = 1500
    out = ref.run(g, pos, vel, dt, nsteps, every=0, miglog=True)
    assert np.abs(out["F"]).max() == 0.0
    # exact positions: x0 + n dt v, wrapped
    expect = pos + nsteps * dt * vel
    for d in range(3):
        expect[:, d] = np.mod(expect[:, d], box[d])
    np.testing.assert_array_equal(out["pos"], expect)
    np.testing.assert_array_equal(out["vel"], vel)
    # closed form: an atom leaves slice s to the right at the first step whose
    # new x reaches the next multiple of 4
    mig = np.zeros((nsteps, 3, 2), np.int32)
    for x0 in pos[:, 0]:
        x = Fr(float(x0))
        for n in range(nsteps):
            x1 = x + Fr(1, 256)
            s0 = math.floor(x / 4) % 3
            s1 = math.floor((x1 % 12) / 4) % 3
            if s1 != s0:
                mig[n, s0, 1] += 1
            x = x1 % 12
    np.testing.assert_array_equal(out["miglog"], mig)
    assert mig.sum() > 0


def test_nve_energy_conservation_small_fluid():
    s = inputs.lj_fluid_2048()
    g = ref.geometry(s.box, s.slices, 2.5)
    out = ref.run(g, s.pos, s.vel, 0.005, 100, every=1)
    E = out["elog"][:, 1] + out["elog"][:, 2]
    drift = np.abs(E - E[0]).max() / s.n
    assert drift < 1e-3
    # a kinetic-energy change of order 0.1 per atom takes place meanwhile
    assert np.ptp(out["elog"][:, 2]) / s.n > 1e-3
    # momentum stays zero to rounding
    assert np.abs(out["vel"].sum(axis=0)).max() < 1e-9


def test_time_reversibility():
    s = inputs.lj_fluid_2048()
    g = ref.geometry(s.box, s.slices, 2.5)
    fwd = ref.run(g, s.pos, s.vel, 0.005, 50)
    back = ref.run(g, fwd["pos"], -fwd["vel"], 0.005, 50)
    d = back["pos"] - s.pos
    L = np.array(s.box)
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-9
    np.testing.assert_allclose(-back["vel"], s.vel, atol=1e-9)


def test_slice_jump_is_unstable():
    box, pos, vel = free_flight_system()
    box = [20.0, 9.0, 9.0]
    g = ref.geometry(box, 5, 2.5)          # slices of width 4
    vel = vel.copy()
    vel[0, 0] = 9.0 / 0.01        # moves two slices in one step
    out = ref.run(g, pos, vel, 0.01, 3, check=False)
    assert out["status"] == -6 and out["steps_done"] == 0


def test_non_finite_is_unstable():
    box, pos, vel = free_flight_system()
    g = ref.geometry(box, 3, 2.5)
    vel = vel.copy()
    vel[3, 1] = np.nan
    out = ref.run(g, pos, vel, 0.01, 3, check=False)
    assert out["status"] == -6
