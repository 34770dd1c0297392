"""GPU parity of the per-slice velocity-scaling thermostat (Sec. 4 kernels md_thermo_a,
md_thermo_b, md_v3b; Sec. 4.2 canonical runs) against the oracle, through the C ABI.

Bars: exact free-flight closed forms (bitwise); a target equal to the current
temperature reproduces the NVE run bitwise; FP64 trajectories within the FP64
trajectory bars of the NVE tests (the slice kinetic energies are summed in another
order, so the factors agree to rounding); schedule and launch-split invariance bitwise.
"""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2507_11289_amd import inputs, md

pytestmark = pytest.mark.gpu

PRECS = [md.MD_FP64, md.MD_FP32_FORCE]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def free_flight():
    box = [12.0, 9.0, 9.0]
    pts = [[0.25 + 3.0 * i, 0.5 + 3.0 * j, 0.75 + 3.0 * k] for i in range(4) for j in range(3) for k in range(3)]
    pos = np.array(pts)
    vel = np.tile(np.array([[1.0, -0.5, 0.25]]), (len(pos), 1))
    return box, pos, vel


def test_free_flight_factor_two_is_exact():
    box, pos, vel = free_flight()
    dt = 2.0 ** -8
    g = ref.geometry(box, 3, 2.5)
    o = ref.run(g, pos, vel, dt, 700, miglog=True, thermostat=1.75)
    for prec in PRECS:
        say(f"[gpu-nvt] free flight, factor 2, precision={prec}")
        with md.Sim(box, 3, 2.5, dt, prec) as sim:
            sim.set_thermostat(1.75)
            sim.set_option(md.OPT_MIGRATION_LOG, 1)
            sim.load(pos, vel)
            sim.step(700)
            p, v, F = sim.state()
            np.testing.assert_array_equal(p, o["pos"])
            np.testing.assert_array_equal(v, 2.0 * vel)
            assert np.abs(F).max() == 0.0
            np.testing.assert_array_equal(sim.migration_log(), o["miglog"])


def test_target_at_the_current_temperature_is_the_nve_run():
    box, pos, vel = free_flight()
    dt = 2.0 ** -7
    for prec in PRECS:
        say(f"[gpu-nvt] factor 1 equals NVE, precision={prec}")
        states = []
        for T0 in (0.4375, 0.0):
            with md.Sim(box, 3, 2.5, dt, prec) as sim:
                sim.set_thermostat(T0)
                sim.load(pos, vel)
                sim.step(300)
                states.append(sim.state())
        for a, b in zip(*states):
            np.testing.assert_array_equal(a, b)


@pytest.fixture(scope="module")
def c0():
    return inputs.lj_fluid_2048()


def test_fp64_nvt_trajectory_matches_oracle(c0):
    say("[gpu-nvt] lj_fluid_2048 FP64, T0 = 1.5, 60 steps vs oracle")
    g = ref.geometry(c0.box, c0.slices, c0.rc)
    o = ref.run(g, c0.pos, c0.vel, c0.dt, 60, every=5, miglog=True, thermostat=1.5)
    with md.Sim(c0.box, c0.slices, c0.rc, c0.dt, md.MD_FP64) as sim:
        sim.set_thermostat(1.5)
        sim.set_option(md.OPT_ENERGY_EVERY, 5)
        sim.set_option(md.OPT_MIGRATION_LOG, 1)
        sim.load(c0.pos, c0.vel)
        sim.step(60)
        elog = sim.energy_log()
        U, K, W = sim.energy_virial()
        pos, vel, F = sim.state()
        mig = sim.migration_log()
    oe = o["elog"]
    assert elog.shape == (12, 4)
    np.testing.assert_array_equal(elog[:, 0], oe[:12, 0])
    for col in (1, 2, 3):
        assert np.abs(elog[:, col] - oe[:12, col]).max() <= 1e-10 * np.abs(oe[:, col]).max()
    assert K == pytest.approx(oe[12, 2], rel=1e-10)
    # the thermostat moved the kinetic energy a long way from the NVE run
    assert oe[12, 2] / oe[0, 2] > 1.3
    np.testing.assert_array_equal(mig, o["miglog"])
    d = pos - o["pos"]
    L = np.array(c0.box)
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-9
    np.testing.assert_allclose(vel, o["vel"], atol=1e-8)


def test_fp32_nvt_trajectory_tracks_oracle(c0):
    say("[gpu-nvt] lj_fluid_2048 FP32-force, T0 = 1.5, 60 steps vs oracle")
    g = ref.geometry(c0.box, c0.slices, c0.rc)
    o = ref.run(g, c0.pos, c0.vel, c0.dt, 60, every=10, thermostat=1.5)
    with md.Sim(c0.box, c0.slices, c0.rc, c0.dt, md.MD_FP32_FORCE) as sim:
        sim.set_thermostat(1.5)
        sim.set_option(md.OPT_ENERGY_EVERY, 10)
        sim.load(c0.pos, c0.vel)
        sim.step(60)
        elog = sim.energy_log()
        pos, vel, F = sim.state()
    E = elog[:, 1] + elog[:, 2]
    Eo = o["elog"][:6, 1] + o["elog"][:6, 2]
    assert np.abs(E - Eo).max() / c0.n < 1e-6
    c = ref.forces_cells(g, pos)
    assert ref.force_error(F, c["F"], c["scale"]).max() <= 1e-5


@pytest.fixture(scope="module")
def medium():
    box, pos, vel, _ = inputs.homogeneous(60000, 0.8, 1.0, 21, aspect=(2.0, 1.0, 1.0))
    return inputs.System("medium", box, 12, pos, vel)


def nvt_state(s, prec, nsteps, grid=0, max_launch=0):
    with md.Sim(s.box, s.slices, s.rc, s.dt, prec) as sim:
        sim.set_thermostat(1.2)
        if grid:
            sim.set_option(md.OPT_GRID, grid)
        if max_launch:
            sim.set_option(md.OPT_MAX_STEPS_PER_LAUNCH, max_launch)
        sim.load(s.pos, s.vel)
        if max_launch:
            sim.step(nsteps // 2)
            sim.step(nsteps - nsteps // 2)
        else:
            sim.step(nsteps)
        return sim.state()


@pytest.mark.parametrize("prec", PRECS)
def test_nvt_is_schedule_and_split_invariant(medium, prec):
    say(f"[gpu-nvt] 60k atoms, 12 slices: grid and launch-split invariance, precision={prec}")
    base = nvt_state(medium, prec, 16)
    for grid, ml in [(1, 0), (37, 0), (0, 5)]:
        say(f"    grid={grid} max_steps_per_launch={ml}")
        st = nvt_state(medium, prec, 16, grid, ml)
        for a, b in zip(base, st):
            np.testing.assert_array_equal(a, b)


def test_thermostat_requires_the_dataflow_scheduler():
    box, pos, vel = free_flight()
    with md.Sim(box, 3, 2.5, 0.005) as sim:
        sim.set_thermostat(1.0)
        sim.set_option(md.OPT_CLAIM_ORDER, md.ORDER_SWEEP)
        sim.load(pos, vel)
        with pytest.raises(md.MDError) as e:
            sim.step(1)
        assert e.value.code == md.MD_EINVAL
