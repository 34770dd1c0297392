"""C-ABI checks that need no GPU: the library loads, exports every function declared in
include/md.h, validates arguments before touching the device, and the serving engine's
admission logic (first come, first served by device footprint) runs against a fake
executor."""
import os
import re
import time

import numpy as np
import pytest

from paper_2507_11289_amd import md, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "md.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(md_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = md.lib()
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(md.EXPORTED)


def test_strerror_covers_all_codes():
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7, -8, -9):
        assert md.md_strerror(code) != "unknown status"


@pytest.mark.parametrize("box,slices,rc,dt,prec", [
    ((20.0, 10.0, 10.0), 2, 2.5, 0.005, 0),     # fewer than 3 slices
    ((6.0, 10.0, 10.0), 3, 2.5, 0.005, 0),      # slice narrower than rc
    ((20.0, 7.0, 10.0), 3, 2.5, 0.005, 0),      # fewer than 3 cells in y
    ((20.0, 10.0, 10.0), 3, -1.0, 0.005, 0),    # rc <= 0
    ((20.0, 10.0, 10.0), 3, 2.5, 0.0, 0),       # dt <= 0
    ((20.0, float("nan"), 10.0), 3, 2.5, 0.005, 0),
    ((20.0, 10.0, 10.0), 3, 2.5, 0.005, 7),     # unknown precision
])
def test_md_init_rejects_invalid_geometry(box, slices, rc, dt, prec):
    with pytest.raises(md.MDError) as e:
        md.Sim(box, slices, rc, dt, prec)
    assert e.value.code == md.MD_EINVAL


def test_footprint_is_positive_and_grows_with_the_box():
    a = md.md_footprint_bytes((20.0, 10.0, 10.0), 3, 2.5, 1000)
    b = md.md_footprint_bytes((40.0, 10.0, 10.0), 6, 2.5, 1000)
    assert 0 < a < b
    assert md.md_footprint_bytes((6.0, 10.0, 10.0), 3, 2.5, 10) == -1


def _fake_runs(k, n=600, steps=300):
    out = []
    for i in range(k):
        box, pos, vel, _ = inputs.homogeneous(n, 0.8, 1.0, 100 + i)
        out.append((box, int(box[0] // 2.5), pos, vel, steps))
    return out


def test_fake_server_admits_fcfs_within_budget():
    runs = _fake_runs(6)
    fp = md.md_footprint_bytes(runs[0][0], runs[0][1], 2.5, len(runs[0][2]))
    budget = 2 * fp + fp // 2     # room for two resident runs
    sv = md.Server(budget, 8, quantum_steps=50, flags=md.SERVER_FAKE_EXECUTOR)
    try:
        tickets = [sv.submit(b, s, p, v, st, tag=i) for i, (b, s, p, v, st) in enumerate(runs)]
        peak = 0
        results = {}
        deadline = time.time() + 60
        while len(results) < len(tickets) and time.time() < deadline:
            st = sv.stats()
            peak = max(peak, st["bytes_in_use"])
            assert st["bytes_in_use"] <= budget
            assert st["running"] <= 2
            for t in tickets:
                if t in results:
                    continue
                rc, r = sv.poll(t)
                if rc != md.MD_PENDING:
                    assert rc == md.MD_OK
                    results[t] = r
            time.sleep(0.002)
        assert len(results) == len(tickets)
        admits = [results[t].t_admit for t in tickets]
        assert admits == sorted(admits)                 # first come, first served
        for i, t in enumerate(tickets):
            assert results[t].tag == i and results[t].steps_done == runs[i][4]
            assert results[t].t_submit <= results[t].t_admit <= results[t].t_done
        assert peak > fp          # two runs were resident together
        with pytest.raises(md.MDError):
            sv.poll(tickets[0])   # released by the first poll that reported it
    finally:
        sv.close()


def test_fake_server_rejects_runs_that_never_fit():
    runs = _fake_runs(1)
    b, s, p, v, st = runs[0]
    fp = md.md_footprint_bytes(b, s, 2.5, len(p))
    sv = md.Server(fp - 1, 4, flags=md.SERVER_FAKE_EXECUTOR)
    try:
        with pytest.raises(md.MDError) as e:
            sv.submit(b, s, p, v, st)
        assert e.value.code == md.MD_ENOMEM
        with pytest.raises(md.MDError) as e:
            sv.submit(b, 2, p, v, st)
        assert e.value.code == md.MD_EINVAL
        bad = p.copy()
        bad[0, 0] = -1.0
        with pytest.raises(md.MDError) as e:
            sv.submit(b, s, bad, v, st)
        assert e.value.code == md.MD_EINVAL
    finally:
        sv.close()


def test_fake_server_slot_cap_and_late_arrivals():
    runs = _fake_runs(5, steps=2000)
    sv = md.Server(1 << 40, 2, quantum_steps=20, flags=md.SERVER_FAKE_EXECUTOR)
    try:
        t0 = [sv.submit(b, s, p, v, st) for (b, s, p, v, st) in runs[:3]]
        time.sleep(0.002)
        t1 = [sv.submit(b, s, p, v, st) for (b, s, p, v, st) in runs[3:]]
        done = {}
        deadline = time.time() + 60
        while len(done) < 5 and time.time() < deadline:
            assert sv.stats()["running"] <= 2
            for t in t0 + t1:
                if t not in done:
                    rc, r = sv.poll(t)
                    if rc != md.MD_PENDING:
                        done[t] = r
            time.sleep(0.002)
        assert len(done) == 5 and all(r.status == 0 for r in done.values())
        # the late arrivals were admitted while earlier runs were still resident
        assert min(done[t].t_admit for t in t1) < max(done[t].t_done for t in t0)
    finally:
        sv.close()


def test_server_queue_limit_returns_busy():
    """At most MD_SERVER_MAX_QUEUED runs wait for admission; the next submission gets
    MD_EBUSY (fake executor: one long resident run, nothing else is admitted)."""
    box, pos, vel, _ = inputs.homogeneous(400, 0.8, 1.0, 3)
    slices = int(box[0] // 2.5)
    sv = md.Server(1 << 40, 1, quantum_steps=50, flags=md.SERVER_FAKE_EXECUTOR)
    try:
        sv.submit(box, slices, pos, vel, 10 ** 9)
        time.sleep(0.05)
        k = 0
        with pytest.raises(md.MDError) as e:
            for k in range(md.SERVER_MAX_QUEUED + 2):
                sv.submit(box, slices, pos, vel, 10)
        assert e.value.code == md.MD_EBUSY
        assert md.SERVER_MAX_QUEUED - 1 <= k <= md.SERVER_MAX_QUEUED
        assert sv.stats()["queued"] >= md.SERVER_MAX_QUEUED - 1
    finally:
        sv.close()


def test_allocator_hook_rules():
    L = md.lib()
    # only one of the two functions: invalid
    a = md.ALLOC_FN(lambda n, c: None)
    assert L.md_set_allocator(a, md.FREE_FN(), None) == md.MD_EINVAL
    # no handle alive: setting and clearing succeed
    md.set_allocator(lambda n: 0, lambda p: None)
    md.set_allocator(None, None)
    # a live server (fake executor) blocks changes
    sv = md.Server(1 << 30, 1, flags=md.SERVER_FAKE_EXECUTOR)
    try:
        with pytest.raises(md.MDError) as e:
            md.set_allocator(lambda n: 0, lambda p: None)
        assert e.value.code == md.MD_ESTATE
    finally:
        sv.close()
    md.set_allocator(None, None)
