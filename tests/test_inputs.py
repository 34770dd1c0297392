"""The seeded input generator: published SplitMix64 outputs, determinism and the
statistics the workloads are defined by (density, temperature, momentum, lattice)."""
import math

import numpy as np
import pytest

from paper_2507_11289_amd import inputs


def test_splitmix64_reference_outputs():
    # first outputs of SplitMix64 for seed 0 (Steele, Lea, Flood; Vigna's reference code)
    out = [int(x) for x in inputs.splitmix64(0, 0, 3)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    # counter-based: any window equals the same part of the full sequence
    np.testing.assert_array_equal(inputs.splitmix64(42, 5, 10), inputs.splitmix64(42, 0, 15)[5:])


def test_uniform_and_normal_ranges():
    st = inputs.Stream(3)
    u = st.uniform(100000)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01
    z = inputs.Stream(4).normal(100001)
    assert len(z) == 100001 and abs(z.mean()) < 0.02 and abs(z.std() - 1.0) < 0.02


def test_small_fluid_properties_and_determinism():
    s = inputs.lj_fluid_2048()
    t = inputs.lj_fluid_2048()
    np.testing.assert_array_equal(s.pos, t.pos)
    np.testing.assert_array_equal(s.vel, t.vel)
    L = s.box[0]
    assert s.n / L ** 3 == pytest.approx(0.8, rel=1e-12)
    assert (s.pos >= 0).all() and (s.pos < L).all()
    assert np.abs(s.vel.sum(axis=0)).max() < 1e-10
    assert (s.vel ** 2).sum() / (3 * s.n - 3) == pytest.approx(1.0, rel=1e-12)
    assert s.meta["fcc"] == [8, 8, 8] and s.meta["vacancies"] == 0


def test_lattice_counts_of_the_large_workloads():
    # without generating the atoms: the lattice each workload is cut from
    L4 = (4194304 / 0.8) ** (1 / 3)
    assert inputs.fcc_counts((L4, L4, L4), 4194304, 0.8) == [102, 102, 102]
    u = (33554432 / 0.85 / 4) ** (1 / 3)
    assert inputs.fcc_counts((4 * u, u, u), 33554432, 0.85) == [512, 128, 128]
    vol = 8388608 / (0.73 / 3 + 2 * 0.02 / 3)
    ly = (vol / 16) ** (1 / 3)
    assert inputs.fcc_counts((16 * ly / 3, ly, ly), round(0.73 * vol / 3), 0.73) == [384, 72, 72]


def test_vacancies_keep_order_and_count():
    sites = np.arange(30.0).reshape(10, 3)
    kept = inputs.remove_vacancies(sites, 7, inputs.Stream(1))
    assert len(kept) == 7
    assert (np.diff(kept[:, 0]) > 0).all()


def test_slab_regions():
    box, pos, vel, meta = inputs.slab(20000, 0.73, 0.02, 0.8, 5)
    x = pos[:, 0]
    n_l = meta["n_liquid"]
    liquid = (x >= box[0] / 3) & (x < 2 * box[0] / 3)
    assert liquid[:n_l].mean() > 0.99 and liquid[n_l:].mean() < 0.05
    assert box[0] == pytest.approx(16 * box[1])


def test_served_ensemble_distribution():
    reqs = inputs.served_ensemble(count=2000)
    n = np.array([r.n for r in reqs])
    assert n.min() >= 500 and n.max() <= 200000
    assert abs(np.log(n).mean() - (math.log(500) + math.log(2e5)) / 2) < 0.2
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() - 1 / 50) < 0.002
    assert all(200 <= r.steps <= 2000 for r in reqs)
    assert all(0.3 <= r.rho <= 0.9 and 0.8 <= r.T <= 2.0 for r in reqs)
    s = reqs[3].system()
    assert s.box[0] / s.slices >= 2.5 and s.slices >= 3
