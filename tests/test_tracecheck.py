"""The trace checker (race detection over per-item records) on synthetic traces: a valid
schedule passes; an item that starts before one of its inputs finished, a missing item
and an item run twice are each reported."""
import numpy as np

from paper_2507_11289_amd import tracecheck
from paper_2507_11289_amd.md import TRACE_DTYPE


def sweep_trace(S=6, K=3, nch=2, ncha=1, nvt=False, launches=1):
    """Items in a valid order (step by step: updates, then finalises), each running alone
    for 10 ticks."""
    recs = []
    t = 100
    for L in range(launches):
        for k in range(K):
            phases = [(0, nch), (2, nch), (1, ncha)] if nvt else [(0, nch), (1, ncha)]
            for ph, n in phases:
                for s in range(S):
                    for c in range(n):
                        recs.append((k, s, c, ph, 0, L, 0, 0, t, t + 1, t + 10))
                        t += 11
    return np.array(recs, dtype=TRACE_DTYPE)


def test_valid_traces_pass():
    for nvt in (False, True):
        rep = tracecheck.check(sweep_trace(nvt=nvt, launches=2), 6)
        assert rep["violations"] == [] and rep["launches"] == 2


def test_early_start_is_a_race():
    r = sweep_trace()
    # force item of slice 3 at step 2 made ready before slice 4's finalise of step 1 finished
    fin = np.where((r["phase"] == 1) & (r["k"] == 1) & (r["slice"] == 4))[0][0]
    f = np.where((r["phase"] == 0) & (r["k"] == 2) & (r["slice"] == 3))[0][0]
    r["t_claim"][f] = r["t_ready"][f] = r["t_done"][fin] - 1
    rep = tracecheck.check(r, 6)
    assert any("force items started before" in v for v in rep["violations"])
    # a finalise of slice 0 (periodic neighbour 5) before the update of slice 5 finished
    r = sweep_trace()
    up = np.where((r["phase"] == 0) & (r["k"] == 0) & (r["slice"] == 5))[0][-1]
    fin = np.where((r["phase"] == 1) & (r["k"] == 0) & (r["slice"] == 0))[0][0]
    r["t_claim"][fin] = r["t_ready"][fin] = r["t_done"][up] - 5
    rep = tracecheck.check(r, 6)
    assert any("finalise items started before" in v for v in rep["violations"])


def test_thermostat_integrate_before_forces_is_a_race():
    r = sweep_trace(nvt=True)
    f = np.where((r["phase"] == 0) & (r["k"] == 1) & (r["slice"] == 2))[0][-1]
    it = np.where((r["phase"] == 2) & (r["k"] == 1) & (r["slice"] == 2))[0][0]
    r["t_claim"][it] = r["t_ready"][it] = r["t_done"][f] - 3
    rep = tracecheck.check(r, 6)
    assert any("thermostat integrate" in v for v in rep["violations"])


def test_missing_and_duplicate_items_are_reported():
    r = sweep_trace()
    rep = tracecheck.check(np.delete(r, 7), 6)
    assert any("1 items missing" in v for v in rep["violations"])
    r2 = r.copy()
    r2[8] = r2[9]
    rep = tracecheck.check(r2, 6)
    assert any("run twice" in v for v in rep["violations"])


def test_utilisation_of_a_serial_trace():
    r = sweep_trace(S=4, K=2, nch=1, ncha=1)
    u = tracecheck.utilisation(r, workers=1)
    # each item: 1 tick waiting, 9 executing, 1 tick between items
    assert abs(u["execute"] - 9 / 11) < 0.01 and abs(u["wait"] - 1 / 11) < 0.01
    assert u["levels_in_flight"] == 1.0
