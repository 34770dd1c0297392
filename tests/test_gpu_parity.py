"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Bars (the method's contract):
  * binning, slice membership, migration counts, candidate and in-range pair counts:
    bit-exact;
  * forces: max_i |F_i - F_i^ref| / S_i <= 1e-12 (FP64 mode) and <= 1e-5 (FP32-force
    mode), where S_i sums the magnitudes of atom i's pair-force terms;
  * energies of an FP64 trajectory: relative 1e-10 of the oracle's over 100 steps.
"""
import math
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2507_11289_amd import inputs, md

pytestmark = pytest.mark.gpu

TOL = {md.MD_FP64: 1e-12, md.MD_FP32_FORCE: 1e-5}
PRECS = [md.MD_FP64, md.MD_FP32_FORCE]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c0():
    return inputs.lj_fluid_2048()


@pytest.fixture(scope="module")
def c0_oracle(c0):
    g = ref.geometry(c0.box, c0.slices, c0.rc)
    return g, ref.forces_cells(g, c0.pos)


@pytest.mark.parametrize("prec", PRECS)
def test_load_binning_and_forces_at_t0(c0, c0_oracle, prec):
    g, o = c0_oracle
    say(f"[gpu] lj_fluid_2048 load + forces, precision={prec}")
    with md.Sim(c0.box, c0.slices, c0.rc, c0.dt, prec) as sim:
        sim.load(c0.pos, c0.vel)
        _, _, ocell = ref.bin_atoms(g, c0.pos)
        np.testing.assert_array_equal(sim.cells(), ocell)
        pos, vel, F = sim.state()
        np.testing.assert_array_equal(pos, c0.pos)
        np.testing.assert_array_equal(vel, c0.vel)
        e = ref.force_error(F, o["F"], o["scale"])
        say(f"    max e_i = {e.max():.3e}")
        assert e.max() <= TOL[prec]
        U, K, W = sim.energy_virial()
        oU, oK, oW = ref.energy(g, c0.pos, c0.vel)
        rel = 1e-12 if prec == md.MD_FP64 else 1e-6
        assert U == pytest.approx(oU, rel=rel)
        assert W == pytest.approx(oW, rel=rel)
        assert K == pytest.approx(oK, rel=1e-13)
        counts = np.bincount(ref.bin_atoms(g, c0.pos)[1], minlength=c0.slices)
        np.testing.assert_array_equal(sim.slice_counts(), counts)


def test_fp64_trajectory_matches_oracle(c0):
    say("[gpu] lj_fluid_2048 FP64 100 steps vs oracle")
    g = ref.geometry(c0.box, c0.slices, c0.rc)
    o = ref.run(g, c0.pos, c0.vel, c0.dt, 100, every=1, miglog=True)
    with md.Sim(c0.box, c0.slices, c0.rc, c0.dt, md.MD_FP64) as sim:
        sim.set_option(md.OPT_ENERGY_EVERY, 1)
        sim.set_option(md.OPT_MIGRATION_LOG, 1)
        sim.load(c0.pos, c0.vel)
        sim.step(100)
        elog = sim.energy_log()
        mig = sim.migration_log()
        U, K, W = sim.energy_virial()
        pos, vel, F = sim.state()
    assert elog.shape == (100, 4)
    np.testing.assert_array_equal(elog[:, 0], np.arange(100))
    ref_e = o["elog"]
    E = elog[:, 1] + elog[:, 2]
    Eo = ref_e[:100, 1] + ref_e[:100, 2]
    assert np.abs(E - Eo).max() <= 1e-10 * np.abs(Eo).max()
    assert np.abs(elog[:, 3] - ref_e[:100, 3]).max() <= 1e-10 * np.abs(ref_e[:, 3]).max()
    assert U + K == pytest.approx(ref_e[100, 1] + ref_e[100, 2], rel=1e-10)
    np.testing.assert_array_equal(mig, o["miglog"])
    d = pos - o["pos"]
    L = np.array(c0.box)
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-9
    np.testing.assert_allclose(vel, o["vel"], atol=1e-8)
    # the GPU's own binning of its positions follows the binning rule exactly
    c = ref.forces_cells(g, pos)
    assert ref.force_error(F, c["F"], c["scale"]).max() <= 1e-12


def test_fp32_force_trajectory_tracks_fp64(c0):
    say("[gpu] lj_fluid_2048 FP32-force 100 steps vs oracle")
    g = ref.geometry(c0.box, c0.slices, c0.rc)
    o = ref.run(g, c0.pos, c0.vel, c0.dt, 100, every=10, miglog=True)
    with md.Sim(c0.box, c0.slices, c0.rc, c0.dt, md.MD_FP32_FORCE) as sim:
        sim.set_option(md.OPT_ENERGY_EVERY, 10)
        sim.load(c0.pos, c0.vel)
        sim.step(100)
        elog = sim.energy_log()
        U, K, W = sim.energy_virial()
        pos, vel, F = sim.state()
        cells = sim.cells()
        counts = sim.slice_counts()
    E = elog[:, 1] + elog[:, 2]
    Eo = o["elog"][:10, 1] + o["elog"][:10, 2]
    # 1e-5-accurate forces keep the short trajectory within 1e-6 per atom
    assert np.abs(E - Eo).max() / c0.n < 1e-6
    c = ref.forces_cells(g, pos)
    assert ref.force_error(F, c["F"], c["scale"]).max() <= 1e-5
    # the GPU's binning of its own positions after 100 steps follows the binning rule
    _, osl, ocell = ref.bin_atoms(g, pos)
    np.testing.assert_array_equal(cells, ocell)
    np.testing.assert_array_equal(counts, np.bincount(osl, minlength=c0.slices))


def migrations_from_binning(g, p0, p1):
    """Per-slice (left, right) migration counts of one step from the oracle's binning of
    the positions before and after it."""
    s0 = ref.bin_atoms(g, p0)[1].astype(np.int64)
    s1 = ref.bin_atoms(g, p1)[1].astype(np.int64)
    delta = (s1 - s0) % g.S
    assert np.isin(delta, [0, 1, g.S - 1]).all()
    out = np.zeros((g.S, 2), np.int64)
    np.add.at(out[:, 0], s0[delta == g.S - 1], 1)
    np.add.at(out[:, 1], s0[delta == 1], 1)
    return out


@pytest.mark.parametrize("prec", PRECS)
def test_migration_log_step_by_step_against_oracle_binning(c0, prec):
    """Each step's per-slice migration counts equal the oracle's binning of the GPU's own
    positions before and after the step (bit-exact); so do cells and slice counts."""
    say(f"[gpu] lj_fluid_2048 migration log step by step, precision={prec}")
    g = ref.geometry(c0.box, c0.slices, c0.rc)
    # a hotter copy of the fluid so that atoms cross slice boundaries every few steps
    vel = 4.0 * c0.vel
    total = 0
    with md.Sim(c0.box, c0.slices, c0.rc, c0.dt, prec) as sim:
        sim.set_option(md.OPT_MIGRATION_LOG, 1)
        sim.load(c0.pos, vel)
        p0 = c0.pos
        for t in range(25):
            sim.step(1)
            p1, _, _ = sim.state()
            mig = sim.migration_log()
            assert mig.shape == (1, c0.slices, 2)
            np.testing.assert_array_equal(mig[0], migrations_from_binning(g, p0, p1))
            _, osl, ocell = ref.bin_atoms(g, p1)
            np.testing.assert_array_equal(sim.cells(), ocell)
            np.testing.assert_array_equal(sim.slice_counts(), np.bincount(osl, minlength=c0.slices))
            total += int(mig.sum())
            p0 = p1
    assert total > 20


def test_brute_force_tiny_systems():
    for n, rho, aspect, slices in [(500, 0.8, (1, 1, 1), 3), (700, 0.5, (2, 1, 1), 4),
                                   (1200, 0.9, (3, 1, 1), 3)]:
        box, pos, vel, _ = inputs.homogeneous(n, rho, 1.0, 7, aspect=aspect)
        g = ref.geometry(box, slices, 2.5)
        Fb, Ub, Wb, Pb = ref.forces_brute(g, pos)
        c = ref.forces_cells(g, pos)
        for prec in PRECS:
            say(f"[gpu] brute force n={n} slices={slices} precision={prec}")
            with md.Sim(box, slices, 2.5, 0.005, prec) as sim:
                sim.set_option(md.OPT_COUNT_PAIRS, 1)
                sim.load(pos, vel)
                _, _, F = sim.state()
                assert ref.force_error(F, Fb, c["scale"]).max() <= TOL[prec]
                U, K, W = sim.energy_virial()
                assert U == pytest.approx(Ub, rel=1e-12 if prec == 0 else 1e-6)
                sim.step(1)
                st = sim.stats()
                assert st.in_range == 2 * Pb
                assert st.candidates == int(c["cand"].sum())


def test_dense_cells_many_batches_and_mask_groups():
    """Jittered lattices at rho = 3 (about 48 atoms per cell, up to 62; nearest
    neighbours about 0.8 apart): several 16-atom batches per cell, windows of 80 and more
    16-candidate tiles (more than one group of pre-filter mask words in the FP32 pair
    walk), staged blocks cut below 4 cells by the staging capacity, and periodic images
    on every side.  Forces, energy and pair counts against the oracle."""
    for n, aspect, slices in [(1300, (1, 1, 1), 3), (2600, (2, 1, 1), 3)]:
        box, pos, vel, _ = inputs.homogeneous(n, 3.0, 1.0, 17, aspect=aspect)
        g = ref.geometry(box, slices, 2.5)
        cnt = np.bincount(ref.bin_atoms(g, pos)[2])
        assert cnt.max() <= 64 and cnt.mean() > 40  # the case this test is for
        o = ref.forces_cells(g, pos)
        oU, oK, oW = ref.energy(g, pos, vel)
        assert (o["cand"].max() + 15) // 16 > 64  # windows beyond two mask groups
        for prec in PRECS:
            say(f"[gpu] dense cells n={n} aspect={aspect} slices={slices} precision={prec}")
            # a tiny step: the counting step then moves no atom into a full cell
            with md.Sim(box, slices, 2.5, 1e-5, prec) as sim:
                sim.set_option(md.OPT_COUNT_PAIRS, 1)
                sim.load(pos, vel)
                np.testing.assert_array_equal(sim.cells(), ref.bin_atoms(g, pos)[2])
                _, _, F = sim.state()
                e = ref.force_error(F, o["F"], o["scale"])
                say(f"    max e_i = {e.max():.3e}")
                assert e.max() <= TOL[prec]
                U, K, W = sim.energy_virial()
                rel = 1e-12 if prec == md.MD_FP64 else 1e-6
                assert U == pytest.approx(oU, rel=rel)
                assert W == pytest.approx(oW, rel=rel)
                sim.step(1)
                st = sim.stats()
                assert st.candidates == int(o["cand"].sum())
                assert st.in_range == int(o["inr"].sum())


def cutoff_pairs(seed=11):
    """Isolated atom pairs at separations rc (1 + delta), delta from -2^-12 to +2^-12:
    some pairs lie inside the FP32 guard band |r2 - rc^2| <= 2^-16 rc^2 (decided again in
    FP64), some just outside it, some exactly at the FP64 cutoff decision.  Pair centres
    are 7.5 apart, so no atom has a partner other than its own (at most 2.25 from the
    centre)."""
    rc = 2.5
    rng = np.random.default_rng(seed)
    deltas = [-2.0 ** -12, -2.0 ** -17, -2.0 ** -20, -2.0 ** -26, 0.0,
              2.0 ** -26, 2.0 ** -20, 2.0 ** -17, 2.0 ** -12]
    box = (45.0, 30.0, 30.0)
    pos = []
    n = 0
    for i in range(6):
        for j in range(4):
            for k in range(4):
                d = rc * (1.0 + deltas[n % len(deltas)])
                u = rng.normal(size=3)
                u /= np.linalg.norm(u)
                if n % 4 == 0:
                    u = np.array([1.0, 0.0, 0.0])
                c = np.array([3.75 + 7.5 * i, 3.75 + 7.5 * j, 3.75 + 7.5 * k]) + rng.uniform(-1.0, 1.0, 3)
                pos += [c - 0.5 * d * u, c + 0.5 * d * u]
                n += 1
    return box, rc, np.mod(np.array(pos), box)


def test_cutoff_decisions_at_the_guard_band():
    box, rc, pos = cutoff_pairs()
    g = ref.geometry(box, 3, rc)
    Fb, Ub, Wb, Pb = ref.forces_brute(g, pos)
    c = ref.forces_cells(g, pos)
    # the construction reaches both sides of the cutoff and the inside of the FP32 band
    a, b = pos[0::2], pos[1::2]
    dd = a - b
    dd -= np.array(box) * np.round(dd / np.array(box))
    r2 = (dd[:, 0] * dd[:, 0] + dd[:, 1] * dd[:, 1]) + dd[:, 2] * dd[:, 2]
    band = np.abs(r2 - rc * rc) <= 2.0 ** -16 * rc * rc
    assert band.sum() >= 20 and 0 < Pb < len(r2)
    assert ((r2 <= rc * rc) & band).any() and ((r2 > rc * rc) & band).any()
    vel = np.zeros_like(pos)
    for prec in PRECS:
        say(f"[gpu] cutoff pairs: {len(r2)} pairs, {int(band.sum())} in the FP32 band, precision={prec}")
        with md.Sim(box, 3, rc, 0.005, prec) as sim:
            sim.set_option(md.OPT_COUNT_PAIRS, 1)
            sim.load(pos, vel)
            _, _, F = sim.state()
            # an atom whose only partner is out of range feels exactly nothing
            np.testing.assert_array_equal(F[np.all(Fb == 0.0, axis=1)], 0.0)
            assert ref.force_error(F, Fb, c["scale"]).max() <= TOL[prec]
            sim.step(1)
            st = sim.stats()
            assert st.in_range == 2 * Pb
            assert st.candidates == int(c["cand"].sum())


def run_state(s, prec, nsteps, order=None, seed=1, chunk=0):
    with md.Sim(s.box, s.slices, s.rc, s.dt, prec) as sim:
        if order is not None:
            sim.set_option(md.OPT_CLAIM_ORDER, order)
            sim.set_option(md.OPT_ORDER_SEED, seed)
        if chunk:
            sim.set_option(md.OPT_CHUNK_CELLS, chunk)
        sim.load(s.pos, s.vel)
        sim.step(nsteps)
        return sim.state()


@pytest.fixture(scope="module")
def medium():
    box, pos, vel, _ = inputs.homogeneous(60000, 0.8, 1.0, 21, aspect=(2.0, 1.0, 1.0))
    return inputs.System("medium", box, 12, pos, vel)


@pytest.mark.parametrize("prec", PRECS)
def test_schedule_invariance_is_bitwise(medium, prec):
    ref_state = None
    for order, seed, chunk in [(md.ORDER_SWEEP, 1, 0), (md.ORDER_PHASED, 1, 0),
                               (md.ORDER_DESCENDING, 1, 7), (md.ORDER_RANDOM, 5, 0),
                               (md.ORDER_RANDOM, 9, 33)]:
        say(f"[gpu] schedule invariance order={order} seed={seed} chunk={chunk} precision={prec}")
        st = run_state(medium, prec, 20, order, seed, chunk)
        if ref_state is None:
            ref_state = st
        else:
            for a, b in zip(ref_state, st):
                np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("prec", PRECS)
def test_block_integration_equals_per_wave_integration(medium, prec):
    """Plain steps finish each block on one wave (the waves leave their forces in LDS, one
    wave advances the atoms of all the block's cells, in FP32 while the other waves stage
    the next block); steps with an energy sample integrate each cell on its own wave.  All
    give bitwise the same trajectory and binning: 15 plain steps against 15 sampled ones and
    against a sample every third step (both kinds of step in one launch), on the liquid and
    on a dense liquid (about 19 atoms per cell), where many blocks hold more than 64 atoms
    and integrate per wave in every run."""
    box, pos, vel, _ = inputs.homogeneous(20000, 1.2, 1.5, 31)
    dense = inputs.System("dense", box, 4, pos, vel)
    for sysm in (medium, dense):
        say(f"[gpu] block vs per-wave integration, {sysm.name}, precision={prec}")
        outs = []
        for every in (0, 1, 3):
            with md.Sim(sysm.box, sysm.slices, sysm.rc, sysm.dt, prec) as sim:
                if every:
                    sim.set_option(md.OPT_ENERGY_EVERY, every)
                sim.load(sysm.pos, sysm.vel)
                sim.step(15)
                p, v, _ = sim.state()
                outs.append((p, v, sim.cells()))
        for other in outs[1:]:
            for a, b in zip(outs[0], other):
                assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", PRECS)
def test_bitwise_resume(medium, prec):
    say(f"[gpu] resume precision={prec}")
    whole = run_state(medium, prec, 20)
    with md.Sim(medium.box, medium.slices, medium.rc, medium.dt, prec) as a:
        a.load(medium.pos, medium.vel)
        a.step(10)
        p, v, _ = a.state()
    with md.Sim(medium.box, medium.slices, medium.rc, medium.dt, prec) as b:
        b.load(p, v)
        b.step(10)
        split = b.state()
    for x, y in zip(whole, split):
        np.testing.assert_array_equal(x, y)


def test_split_launches_equal_one_launch(medium):
    say("[gpu] launch splitting")
    whole = run_state(medium, md.MD_FP32_FORCE, 12)
    with md.Sim(medium.box, medium.slices, medium.rc, medium.dt, md.MD_FP32_FORCE) as sim:
        sim.set_option(md.OPT_MAX_STEPS_PER_LAUNCH, 5)
        sim.load(medium.pos, medium.vel)
        sim.step(7)
        sim.step(5)
        st = sim.state()
    for x, y in zip(whole, st):
        np.testing.assert_array_equal(x, y)


def test_free_flight_exact_and_migrations():
    say("[gpu] free flight")
    box = [12.0, 9.0, 9.0]
    pts = [[0.25 + 3.0 * i, 0.5 + 3.0 * j, 0.75 + 3.0 * k] for i in range(4) for j in range(3) for k in range(3)]
    pos = np.array(pts)
    vel = np.tile(np.array([[1.0, -0.5, 0.25]]), (len(pos), 1))
    dt = 2.0 ** -8
    g = ref.geometry(box, 3, 2.5)
    o = ref.run(g, pos, vel, dt, 1500, miglog=True)
    for prec in PRECS:
        with md.Sim(box, 3, 2.5, dt, prec) as sim:
            sim.set_option(md.OPT_MIGRATION_LOG, 1)
            sim.load(pos, vel)
            sim.step(1500)
            p, v, F = sim.state()
            np.testing.assert_array_equal(p, o["pos"])
            np.testing.assert_array_equal(v, vel)
            assert np.abs(F).max() == 0.0
            np.testing.assert_array_equal(sim.migration_log(), o["miglog"])
            st = sim.stats()
            assert st.migrations_right == int(o["miglog"][:, :, 1].sum()) and st.migrations_left == 0


def test_empty_system_and_boundary_positions():
    say("[gpu] empty system")
    with md.Sim((12.0, 9.0, 9.0), 3, 2.5, 0.005) as sim:
        sim.load(np.zeros((0, 3)), np.zeros((0, 3)))
        sim.step(3)
        assert sim.energy_virial() == (0.0, 0.0, 0.0)
        assert sim.stats().step == 3
    say("[gpu] positions at 0 and L")
    box = (12.0, 9.0, 9.0)
    # coordinates exactly 0 and exactly L (the last cell), all pairs beyond rc
    pos = np.array([[0.0, 0.0, 0.0], [12.0, 4.5, 9.0], [6.0, 9.0, 4.5]])
    vel = np.array([[0.5, -0.25, 0.125], [-1.0, 0.5, 0.25], [0.0, 1.0, -1.0]])
    g = ref.geometry(box, 3, 2.5)
    o = ref.run(g, pos, vel, 0.005, 2)
    with md.Sim(box, 3, 2.5, 0.005) as sim:
        sim.load(pos, vel)
        np.testing.assert_array_equal(sim.cells(), ref.bin_atoms(g, pos)[2])
        sim.step(2)
        p, v, F = sim.state()
        np.testing.assert_array_equal(p, o["pos"])
        np.testing.assert_array_equal(v, o["vel"])


def test_errors_are_reported_and_poison():
    box = (20.0, 9.0, 9.0)
    say("[gpu] capacity overflow at load")
    pos = np.full((70, 3), 1.0) + np.linspace(0, 0.9, 70)[:, None] * np.array([1, 0, 0])
    with md.Sim(box, 5, 2.5, 0.005) as sim:
        with pytest.raises(md.MDError) as e:
            sim.load(pos, np.zeros_like(pos))
        assert e.value.code == md.MD_ECAPACITY
        with pytest.raises(md.MDError) as e:
            sim.step(1)
        assert e.value.code == md.MD_ESTATE
    say("[gpu] slice jump")
    pos = np.array([[0.5, 1.0, 1.0], [10.5, 5.0, 5.0]])
    vel = np.array([[9.0 / 0.01, 0.0, 0.0], [0.0, 0.0, 0.0]])
    with md.Sim(box, 5, 2.5, 0.01) as sim:
        sim.load(pos, vel)
        assert sim.step_rc(3) == md.MD_EUNSTABLE
        assert sim.stats().poisoned == 1
        assert sim.step_rc(1) == md.MD_ESTATE
    say("[gpu] injected fault")
    s = inputs.lj_fluid_2048()
    with md.Sim(s.box, s.slices, s.rc, s.dt) as sim:
        sim.set_option(md.OPT_FAIL_AT_STEP, 4)
        sim.load(s.pos, s.vel)
        assert sim.step_rc(10) == md.MD_EUNSTABLE
    say("[gpu] invalid input")
    with md.Sim(box, 5, 2.5, 0.005) as sim:
        with pytest.raises(md.MDError) as e:
            sim.load(np.array([[21.0, 1.0, 1.0]]), np.zeros((1, 3)))
        assert e.value.code == md.MD_EINVAL
        with pytest.raises(md.MDError) as e:
            sim.step(1)
        assert e.value.code == md.MD_ESTATE


def test_cutoff_decisions_without_fused_r2():
    """Pairs whose squared distance is within ulps of rc^2 and whose decision a fused
    multiply-add in r^2 would flip: the FP64 decision (every pair in FP64 mode, the
    guard band in FP32-force mode) must be the unfused one of the oracle."""
    from tests.cutoff_cases import flip_separations, isolated_pair_system, r2_unfused
    seps = flip_separations(48)
    box, pos = isolated_pair_system(seps)
    g = ref.geometry(box, 3, 2.5)
    inside = np.array([r2_unfused(d) <= 6.25 for d in seps])
    Fb, Ub, Wb, Pb = ref.forces_brute(g, pos)
    c = ref.forces_cells(g, pos)
    assert Pb == int(inside.sum()) and 0 < Pb < len(seps)
    vel = np.zeros_like(pos)
    for prec in PRECS:
        say(f"[gpu] {len(seps)} pairs at rc^2 within ulps, {Pb} in range, precision={prec}")
        with md.Sim(box, 3, 2.5, 0.005, prec) as sim:
            sim.set_option(md.OPT_COUNT_PAIRS, 1)
            sim.load(pos, vel)
            _, _, F = sim.state()
            out = np.repeat(~inside, 2)
            np.testing.assert_array_equal(F[out], 0.0)
            assert (np.abs(F[~out]).sum(axis=1) > 0).all()
            assert ref.force_error(F, Fb, c["scale"]).max() <= TOL[prec]
            sim.step(1)
            assert sim.stats().in_range == 2 * Pb


@pytest.mark.parametrize("order,thermo", [(None, 0.0), (md.ORDER_RANDOM, 0.0), (None, 1.2)])
def test_trace_has_no_races(medium, order, thermo):
    """Race detection: every work item of two persistent launches ran exactly once and
    became ready only after every item whose results it reads had finished (device clock
    of the per-item trace)."""
    from paper_2507_11289_amd import tracecheck
    say(f"[gpu] trace race check order={order} thermostat={thermo}")
    with md.Sim(medium.box, medium.slices, medium.rc, medium.dt, md.MD_FP32_FORCE) as sim:
        if order is not None:
            sim.set_option(md.OPT_CLAIM_ORDER, order)
            sim.set_option(md.OPT_ORDER_SEED, 3)
        if thermo:
            sim.set_thermostat(thermo)
        sim.set_option(md.OPT_TRACE, 1)
        sim.set_option(md.OPT_MAX_STEPS_PER_LAUNCH, 6)
        sim.load(medium.pos, medium.vel)
        sim.step(12)
        rec, hz = sim.trace()
        st = sim.stats()
    assert st.last_launches == 2 and hz > 0
    rep = tracecheck.check(rec, medium.slices)
    say(f"    {rep['items']} items, {rep['launches']} launches, violations: {rep['violations']}")
    assert rep["violations"] == []
    u = tracecheck.utilisation(rec, st.persistent_grid)
    say(f"    execute {u['execute']:.3f} wait {u['wait']:.3f} levels {u['levels_in_flight']:.2f}")
    assert 0.0 < u["execute"] <= 1.0


def test_cell_capacity_option_forces_the_guard(c0):
    """A lowered cell capacity turns a load or a step that fills a cell beyond it into
    MD_ECAPACITY (the step poisons the handle)."""
    say("[gpu] capacity option")
    counts = np.bincount(ref.bin_atoms(ref.geometry(c0.box, c0.slices, c0.rc), c0.pos)[2])
    with md.Sim(c0.box, c0.slices, c0.rc, c0.dt) as sim:
        sim.set_option(md.OPT_CELL_CAPACITY, int(counts.max()) - 1)
        with pytest.raises(md.MDError) as e:
            sim.load(c0.pos, c0.vel)
        assert e.value.code == md.MD_ECAPACITY
    with md.Sim(c0.box, c0.slices, c0.rc, c0.dt) as sim:
        sim.set_option(md.OPT_CELL_CAPACITY, int(counts.max()))
        sim.load(c0.pos, c0.vel)
        assert sim.stats().cell_capacity == counts.max()
        sim.set_option(md.OPT_CELL_CAPACITY, 2)
        assert sim.step_rc(1) == md.MD_ECAPACITY
        assert sim.stats().poisoned == 1
    with pytest.raises(md.MDError):
        with md.Sim(c0.box, c0.slices, c0.rc, c0.dt) as sim:
            sim.set_option(md.OPT_CELL_CAPACITY, 65)


def test_torch_caching_allocator_gives_the_same_trajectory(c0):
    """md_set_allocator with torch's caching allocator: device memory comes from torch
    (its allocated bytes grow while the simulation lives) and results are bitwise those
    of the library's own hipMalloc."""
    import torch
    say("[gpu] torch caching allocator")
    with md.Sim(c0.box, c0.slices, c0.rc, c0.dt, md.MD_FP32_FORCE) as sim:
        sim.load(c0.pos, c0.vel)
        sim.step(10)
        want = sim.state()
    torch.cuda.init()
    base = torch.cuda.memory_allocated()
    md.use_torch_allocator()
    try:
        with md.Sim(c0.box, c0.slices, c0.rc, c0.dt, md.MD_FP32_FORCE) as sim:
            sim.load(c0.pos, c0.vel)
            sim.step(10)
            got = sim.state()
            held = torch.cuda.memory_allocated() - base
        assert held >= 2 * 4352 * (c0.slices * 25)
        assert torch.cuda.memory_allocated() == base
    finally:
        md.set_allocator(None, None)
    for a, b in zip(want, got):
        np.testing.assert_array_equal(a, b)


def test_longer_launch_after_a_shorter_one_allocates_nothing(c0):
    """When its launch buffers (work queue, round tables, energy partials, migration log)
    grow, md_step sizes them for the longest launch the run may make (its steps-per-launch
    cap): after a 5-step launch, 20-step launches allocate no device memory (counted
    through md_set_allocator), without and with energy samples and the migration log."""
    import torch
    say("[gpu] no allocation when a longer launch follows a shorter one")
    torch.cuda.init()
    sizes = []

    def alloc(n):
        sizes.append(n)
        return torch.cuda.caching_allocator_alloc(n)

    md.set_allocator(alloc, lambda p: torch.cuda.caching_allocator_delete(p))
    try:
        for every, miglog in ((0, 0), (5, 1)):
            with md.Sim(c0.box, c0.slices, c0.rc, c0.dt, md.MD_FP32_FORCE) as sim:
                sim.set_option(md.OPT_MAX_STEPS_PER_LAUNCH, 100)
                if every:
                    sim.set_option(md.OPT_ENERGY_EVERY, every)
                sim.set_option(md.OPT_MIGRATION_LOG, miglog)
                sim.load(c0.pos, c0.vel)
                sim.step(5)
                before = len(sizes)
                sim.step(20)
                sim.step(20)
                assert len(sizes) == before, (every, miglog, sizes[before:])
    finally:
        md.set_allocator(None, None)


@pytest.fixture(scope="module")
def long_fluid():
    # 32 slices: at least 3 slices for each of the GPU's XCD work queues
    box, pos, vel, _ = inputs.homogeneous(32768, 0.8, 1.0, 23, aspect=(4.0, 1.0, 1.0))
    return inputs.System("long", box, 32, pos, vel)


def run_queues(system, prec, xcd_queues):
    """20 plain steps, then 20 with energy samples (both persistent kernel variants)."""
    from paper_2507_11289_amd import tracecheck

    with md.Sim(system.box, system.slices, system.rc, system.dt, prec) as sim:
        sim.set_option(md.OPT_XCD_QUEUES, xcd_queues)
        sim.set_option(md.OPT_MIGRATION_LOG, 1)
        sim.set_option(md.OPT_TRACE, 1)
        sim.load(system.pos, system.vel)
        sim.step(20)
        mig_a = sim.migration_log()
        rec, _ = sim.trace()
        st = sim.stats()
        first = list(st.queue_first)[: st.work_queues + 1]
        sim.set_option(md.OPT_ENERGY_EVERY, 5)
        sim.step(20)
        out = {"state": sim.state(), "cells": sim.cells(), "elog": sim.energy_log(),
               "mig": np.concatenate([mig_a, sim.migration_log()]), "queues": st.work_queues,
               "first": first, "rec": rec}
    assert tracecheck.check(rec, system.slices)["violations"] == []
    return out


@pytest.mark.parametrize("prec", PRECS)
def test_xcd_queues_are_bitwise_the_single_queue(long_fluid, prec):
    """One work queue per XCD (items of slices whose neighbours share the XCD synchronise
    through its L2 only) gives bitwise the results of one device-wide queue; every item
    ran on the XCD of its queue, and each queue owns a contiguous range of slices."""
    say(f"[gpu] XCD work queues vs one queue, precision={prec}")
    one = run_queues(long_fluid, prec, 0)
    xq = run_queues(long_fluid, prec, 1)
    assert one["queues"] == 1
    say(f"    queues {xq['queues']}, ranges {xq['first']}")
    assert xq["queues"] > 1
    first = np.array(xq["first"])
    assert first[0] == 0 and first[-1] == long_fluid.slices and (np.diff(first) >= 3).all()
    rec = xq["rec"]
    owner = np.searchsorted(first, rec["slice"], side="right") - 1
    np.testing.assert_array_equal(rec["queue"], owner)
    np.testing.assert_array_equal(rec["xcd"], rec["queue"])
    for a, b in zip(one["state"], xq["state"]):
        np.testing.assert_array_equal(a, b)
    for key in ("cells", "elog", "mig"):
        np.testing.assert_array_equal(one[key], xq[key])


@pytest.mark.parametrize("prec", PRECS)
def test_wavefront_sweep_is_bitwise_the_dataflow_run(long_fluid, prec):
    """The multi-time-level sweep (W steps dealt as outward wavefronts, each step three
    slices behind the one before) gives bitwise the dataflow run's state, energies and
    migrations, with whole rounds of W steps and a shorter rest launch (7 = 3 + 3 + 1)."""
    from paper_2507_11289_amd import tracecheck

    say(f"[gpu] wavefront sweep, precision={prec}")
    outs = []
    for order, levels in ((md.ORDER_DATAFLOW, 0), (md.ORDER_WAVEFRONT, 3), (md.ORDER_WAVEFRONT, 8)):
        with md.Sim(long_fluid.box, long_fluid.slices, long_fluid.rc, long_fluid.dt, prec) as sim:
            sim.set_option(md.OPT_CLAIM_ORDER, order)
            if levels:
                sim.set_option(md.OPT_WAVEFRONT_LEVELS, levels)
            sim.set_option(md.OPT_MIGRATION_LOG, 1)
            sim.set_option(md.OPT_ENERGY_EVERY, 2)
            sim.set_option(md.OPT_TRACE, 1)
            sim.load(long_fluid.pos, long_fluid.vel)
            sim.step(7)
            rec, _ = sim.trace()
            launches = sim.stats().last_launches
            outs.append((sim.state(), sim.energy_log(), sim.migration_log(), sim.cells()))
        assert tracecheck.check(rec, long_fluid.slices)["violations"] == []
        if levels == 3:
            assert launches == 2      # 6 steps in whole rounds, then the 1-step rest
        if levels:
            # items of several steps ran at once: a later step's first item started before
            # an earlier step's last item finished
            ph0 = rec[(rec["phase"] == 0) & (rec["launch"] == 0)]
            k = ph0["k"]
            assert any(ph0["t_ready"][k == j + 1].min() < ph0["t_done"][k == j].max()
                       for j in range(int(k.max())))
    for other in outs[1:]:
        for a, b in zip(outs[0][0], other[0]):
            np.testing.assert_array_equal(a, b)
        for a, b in zip(outs[0][1:], other[1:]):
            np.testing.assert_array_equal(a, b)
