"""md_step_noalloc, the stepping entry point for callers that cannot allocate device
memory, against md_step through the C ABI.

Both entry points run the same kernels, so the bar is bitwise equality of everything a
step produces: positions, velocities and forces of the synchronous state, cell ids,
atoms per slice, the energy log and the per-step migration log.  Two calls in a row
share the per-GPU scratch array; the second runs a smaller system, so contents the first
call left in the array (a longer work queue, more energy partials and migration counts)
would show up as a difference if any piece were read before being rewritten.
"""
import sys

import numpy as np
import pytest

from paper_2507_11289_amd import inputs, md

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def fluid_32k():
    box, pos, vel, _ = inputs.homogeneous(32768, 0.8, 1.0, seed=inputs.BASE_SEED + 77)
    return inputs.System("lj_fluid_32k", box, 12, pos, vel)


def run(system, prec, steps, noalloc, every=3, max_launch=None):
    with md.Sim(system.box, system.slices, system.rc, system.dt, prec) as sim:
        sim.load(system.pos, system.vel)
        sim.set_option(md.OPT_ENERGY_EVERY, every)
        sim.set_option(md.OPT_MIGRATION_LOG, 1)
        if max_launch:
            sim.set_option(md.OPT_MAX_STEPS_PER_LAUNCH, max_launch)
        if noalloc:
            sim.step_noalloc(steps)
        else:
            sim.step(steps)
        pos, vel, F = sim.state()
        out = dict(pos=pos, vel=vel, F=F, cells=sim.cells(), counts=sim.slice_counts(),
                   elog=sim.energy_log(), mig=sim.migration_log())
        out["launches"] = sim.stats().last_launches
        out["step"] = sim.stats().step
        return out


def assert_same(a, b):
    for key in ("pos", "vel", "F", "cells", "counts", "elog", "mig"):
        assert a[key].shape == b[key].shape, key
        assert np.array_equal(a[key], b[key]), f"{key} differs"
    assert a["step"] == b["step"]


@pytest.mark.parametrize("prec", [md.MD_FP32_FORCE, md.MD_FP64])
def test_noalloc_equals_md_step_twice_second_smaller(prec):
    big, small = fluid_32k(), inputs.lj_fluid_2048()
    say(f"[gpu] md_step_noalloc vs md_step, precision={prec}: {big.name} 24 steps, then {small.name} 10 steps")
    ref_big = run(big, prec, 24, noalloc=False)
    got_big = run(big, prec, 24, noalloc=True)
    assert_same(got_big, ref_big)
    assert got_big["mig"].sum() > 0 and len(got_big["elog"]) == 8
    ref_small = run(small, prec, 10, noalloc=False, every=2)
    got_small = run(small, prec, 10, noalloc=True, every=2)
    assert_same(got_small, ref_small)
    assert len(got_small["elog"]) == 5


def test_noalloc_splits_launches_like_md_step():
    s = inputs.lj_fluid_2048()
    say("[gpu] md_step_noalloc with at most 7 steps per launch, 20 steps")
    ref = run(s, md.MD_FP32_FORCE, 20, noalloc=False)
    got = run(s, md.MD_FP32_FORCE, 20, noalloc=True, max_launch=7)
    assert got["launches"] == 3
    assert_same(got, ref)


def test_noalloc_rejects_what_needs_allocated_buffers():
    s = inputs.lj_fluid_2048()
    say("[gpu] md_step_noalloc rejects the thermostat and the trace")
    with md.Sim(s.box, s.slices, s.rc, s.dt, md.MD_FP32_FORCE) as sim:
        sim.load(s.pos, s.vel)
        sim.set_thermostat(1.0)
        with pytest.raises(md.MDError) as e:
            sim.step_noalloc(1)
        assert e.value.code == md.MD_EINVAL
        sim.set_thermostat(0.0)
        sim.set_option(md.OPT_TRACE, 1)
        with pytest.raises(md.MDError) as e:
            sim.step_noalloc(1)
        assert e.value.code == md.MD_EINVAL
        sim.set_option(md.OPT_TRACE, 0)
        # nothing ran and the handle is not poisoned
        sim.step_noalloc(2)
        assert sim.stats().step == 2
