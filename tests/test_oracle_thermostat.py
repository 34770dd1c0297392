"""Pins of the oracle's per-slice velocity-scaling thermostat (Sec. 4: a factor
computed from the new velocities scales them before the positions advance; Sec. 4.2:
canonical-ensemble runs).  The factor of slice s is lambda_s = sqrt(T0 / T_s) with the
kinetic temperature T_s = 2 K_s / (3 n_s).  Pinned by exact free-flight cases (no
forces, powers-of-two arithmetic), the defining invariant T_s(lambda v) = T0, slice
independence, the degenerate slices, and the composition "scale, then one NVE step"."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import ref
from paper_2507_11289_amd import inputs


def free_flight_system():
    """Atoms 3 sigma apart (beyond rc), all with one velocity: forces stay zero."""
    box = [12.0, 9.0, 9.0]
    pts = [[0.25 + 3.0 * i, 0.5 + 3.0 * j, 0.75 + 3.0 * k]
           for i in range(4) for j in range(3) for k in range(3)]
    pos = np.array(pts)
    vel = np.tile(np.array([[1.0, -0.5, 0.25]]), (len(pos), 1))
    return box, pos, vel


def slice_of(pos, box, S):
    return np.floor(pos[:, 0] / (box[0] / S)).astype(int) % S


def slice_temperatures(pos, vel, box, S):
    s = slice_of(pos, box, S)
    T = np.full(S, np.nan)
    for k in range(S):
        v = vel[s == k]
        if len(v):
            T[k] = (2.0 / (3.0 * len(v))) * 0.5 * float((v * v).sum())
    return T


def test_factor_two_is_exact_in_free_flight():
    # |v|^2 = 1.3125, T_s = 0.4375 in every slice; T0 = 1.75 gives lambda = 2 exactly,
    # after which every slice sits at T0 and lambda = 1 exactly
    box, pos, vel = free_flight_system()
    g = ref.geometry(box, 3, 2.5)
    dt = 2.0 ** -8
    nsteps = 700
    out = ref.run(g, pos, vel, dt, nsteps, miglog=True, thermostat=1.75)
    assert np.abs(out["F"]).max() == 0.0
    np.testing.assert_array_equal(out["vel"], 2.0 * vel)
    expect = pos + nsteps * dt * (2.0 * vel)
    for d in range(3):
        expect[:, d] = np.mod(expect[:, d], box[d])
    np.testing.assert_array_equal(out["pos"], expect)
    # migrations: x advances by exactly 1/128 per step
    mig = np.zeros((nsteps, 3, 2), np.int32)
    for x0 in pos[:, 0]:
        x = Fr(float(x0))
        for n in range(nsteps):
            x1 = x + Fr(1, 128)
            s0 = math.floor(x / 4) % 3
            s1 = math.floor((x1 % 12) / 4) % 3
            if s1 != s0:
                mig[n, s0, 1] += 1
            x = x1 % 12
    np.testing.assert_array_equal(out["miglog"], mig)


def test_target_equal_to_current_temperature_is_plain_nve():
    box, pos, vel = free_flight_system()
    g = ref.geometry(box, 3, 2.5)
    a = ref.run(g, pos, vel, 2.0 ** -7, 300, miglog=True, thermostat=0.4375)
    b = ref.run(g, pos, vel, 2.0 ** -7, 300, miglog=True)
    for key in ("pos", "vel", "F", "miglog"):
        np.testing.assert_array_equal(a[key], b[key])


def test_scaled_slices_sit_at_the_target_and_factors_are_per_slice():
    s = inputs.lj_fluid_2048()
    g = ref.geometry(s.box, s.slices, 2.5)
    rng = np.random.default_rng(3)
    vel = s.vel * rng.uniform(0.5, 2.0, size=(s.slices,))[slice_of(s.pos, s.box, s.slices)][:, None]
    T0 = 1.37
    v2, lam = ref.slice_scale(g, s.pos, vel, T0)
    T_before = slice_temperatures(s.pos, vel, s.box, s.slices)
    T_after = slice_temperatures(s.pos, v2, s.box, s.slices)
    np.testing.assert_allclose(T_after, T0, rtol=1e-14)
    np.testing.assert_allclose(lam, np.sqrt(T0 / T_before), rtol=1e-14)
    # each atom is scaled by the factor of its own slice
    sl = slice_of(s.pos, s.box, s.slices)
    np.testing.assert_array_equal(v2, vel * lam[sl][:, None])
    # changing the velocities of one slice changes only that slice's factor
    vel3 = vel.copy()
    vel3[sl == 1] *= 3.0
    _, lam3 = ref.slice_scale(g, s.pos, vel3, T0)
    np.testing.assert_array_equal(np.delete(lam3, 1), np.delete(lam, 1))
    assert lam3[1] == pytest.approx(lam[1] / 3.0, rel=1e-14)


def test_empty_and_motionless_slices_keep_factor_one():
    box, pos, vel = free_flight_system()
    g = ref.geometry(box, 3, 2.5)
    keep = slice_of(pos, box, 3) != 1          # slice 1 empty
    pos2, vel2 = pos[keep], vel[keep].copy()
    vel2[slice_of(pos2, box, 3) == 2] = 0.0    # slice 2 at rest
    v3, lam = ref.slice_scale(g, pos2, vel2, 0.875)
    assert lam[1] == 1.0 and lam[2] == 1.0
    assert lam[0] == math.sqrt(2.0)            # 0.875 / 0.4375 = 2
    np.testing.assert_array_equal(v3[slice_of(pos2, box, 3) == 2], 0.0)


def test_a_step_is_scaling_then_one_nve_step():
    s = inputs.lj_fluid_2048()
    g = ref.geometry(s.box, s.slices, 2.5)
    T0 = 1.5
    out = ref.run(g, s.pos, s.vel, 0.005, 4, every=1, thermostat=T0)
    pos, vel = s.pos.copy(), s.vel.copy()
    for _ in range(4):
        vel, _ = ref.slice_scale(g, pos, vel, T0)
        one = ref.run(g, pos, vel, 0.005, 1)
        pos, vel = one["pos"], one["vel"]
    np.testing.assert_array_equal(out["pos"], pos)
    np.testing.assert_array_equal(out["vel"], vel)
    # energy samples report the unscaled kinetic energy of v(t)
    assert out["elog"][-1, 2] == pytest.approx(0.5 * float((vel * vel).sum()), rel=1e-13)


def test_liquid_relaxes_to_the_target_temperature():
    s = inputs.lj_fluid_2048()
    g = ref.geometry(s.box, s.slices, 2.5)
    out = ref.run(g, s.pos, s.vel, 0.005, 200, every=10, thermostat=1.5)
    n = s.n
    T = 2.0 * out["elog"][:, 2] / (3.0 * n)
    assert abs(T[0] - 1.0) < 0.05            # starts at the generated temperature
    assert np.abs(T[-5:] - 1.5).max() < 0.05  # held near the target
    # the plain run stays well below it
    nve = ref.run(g, s.pos, s.vel, 0.005, 200, every=10)
    assert (2.0 * nve["elog"][-1, 2] / (3.0 * n)) < 1.2


def test_invalid_target_is_rejected():
    box, pos, vel = free_flight_system()
    g = ref.geometry(box, 3, 2.5)
    with pytest.raises(ref.OracleError):
        ref.run(g, pos, vel, 0.01, 2, thermostat=0.0)
    with pytest.raises(ref.OracleError):
        ref.slice_scale(g, pos, vel, -1.0)
