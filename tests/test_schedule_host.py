"""Host logic of the cyclic schedule: the per-step claim tables of the persistent
kernel (checked without a GPU) and their relation to the paper's Table 1."""
import os

import numpy as np
import pytest

from paper_2507_11289_amd import md

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_one_worker.txt")


def valid_step_order(table, S):
    """Every entry once; a finalise entry of slice i after the integrate entries of i-1, i, i+1."""
    seen = set()
    done = np.zeros(S, bool)
    for phase, s in table:
        assert (phase, s) not in seen
        seen.add((phase, s))
        if phase == 0:
            done[s] = True
        else:
            assert done[(s - 1) % S] and done[s] and done[(s + 1) % S]
    assert len(seen) == 2 * S


@pytest.mark.parametrize("S", [3, 4, 5, 17, 64, 512])
@pytest.mark.parametrize("order", [md.ORDER_SWEEP, md.ORDER_PHASED, md.ORDER_DESCENDING, md.ORDER_RANDOM])
def test_claim_tables_respect_the_dependencies(S, order):
    for seed in (1, 2, 3):
        valid_step_order(md.md_claim_table(S, order, seed), S)


def test_random_orders_differ_by_seed():
    a = md.md_claim_table(64, md.ORDER_RANDOM, 1)
    b = md.md_claim_table(64, md.ORDER_RANDOM, 2)
    assert not np.array_equal(a, b)
    assert np.array_equal(a, md.md_claim_table(64, md.ORDER_RANDOM, 1))


def parse_table1(N):
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        stage, store, recv, worker, partial, send = [c.strip() for c in line.split("|")]
        ev = lambda x: None if x in ("-", "idle") else eval(x.replace("N", str(N)))
        rows.append((ev(stage), ev(worker), ev(send)))
    return rows


@pytest.mark.parametrize("N", [6, 9, 64])
def test_sweep_order_follows_table_1(N):
    """Table 1: at stage s the worker processes slice s-2 and slice s-3 is complete and
    sent.  In the sweep table (0-based slices), integrating slice k is immediately
    followed by finalising slice k-1, for every stage of the table's interior.  The
    paper's first slice has no left neighbour; here slices are periodic, so slice 0 is
    completed only after the last slice (stage 4 of the table is the exception)."""
    t = [tuple(x) for x in md.md_claim_table(N, md.ORDER_SWEEP)]
    pos = {e: i for i, e in enumerate(t)}
    checked = 0
    for stage, worker, send in parse_table1(N):
        if worker is None or send is None or not (5 <= stage <= N):
            continue
        assert worker == stage - 2 and send == stage - 3
        assert pos[(1, send - 1)] == pos[(0, worker - 1)] + 1
        checked += 1
    assert checked == 2   # the printed interior rows: stage 5 and stage N
    # integration sweeps the slices in ascending order, as the worker does
    integ = [s for ph, s in t if ph == 0]
    assert integ == list(range(N))
    # the periodic exception: slice 0 is finalised last, right after slice N-1
    assert t[-1] == (1, 0) and t[-2] == (1, N - 1)


def valid_wavefront(table, S, W):
    """Every (step, phase, slice) of W steps once; finalise of slice i (for step j+1) after the
    integrates of i-1, i, i+1 at step j; integrate of slice i at step j >= 1 after the
    finalises of i-1, i, i+1 for step j."""
    seen = set()
    integ = np.zeros((W, S), bool)
    fin = np.zeros((W, S), bool)
    for j, phase, s in table:
        assert (j, phase, s) not in seen
        seen.add((j, phase, s))
        nb = [(s - 1) % S, s, (s + 1) % S]
        if phase == 0:
            if j > 0:
                assert all(fin[j - 1, t] for t in nb)
            integ[j, s] = True
        else:
            assert all(integ[j, t] for t in nb)
            fin[j, s] = True
    assert len(seen) == 2 * S * W


@pytest.mark.parametrize("S", [3, 4, 5, 17, 64, 512])
@pytest.mark.parametrize("W", [1, 2, 3, 8, 64])
def test_wavefront_tables_respect_the_dependencies(S, W):
    valid_wavefront(md.md_wavefront_table(S, W), S, W)


def test_wavefront_keeps_levels_in_flight_in_a_window():
    """S = 64, W = 8: the sweep starts every step at slice 0 and moves outward in both
    directions; a later step starts before an earlier one has reached the far side, and
    over the middle of the table the entries of any 64 consecutive table positions touch
    several steps but only a window of slices."""
    S, W = 64, 8
    t = md.md_wavefront_table(S, W)
    first = {j: min(i for i, e in enumerate(t) if e[0] == j) for j in range(W)}
    last = {j: max(i for i, e in enumerate(t) if e[0] == j) for j in range(W)}
    for j in range(1, W):
        assert first[j] < last[j - 1]            # levels overlap
    mid = t[len(t) // 3: 2 * len(t) // 3]
    for k in range(0, len(mid) - 64, 16):
        w = mid[k:k + 64]
        assert len(set(w[:, 0])) >= 2
        d = np.minimum(w[:, 2], S - w[:, 2])     # distance from slice 0
        assert d.max() - d.min() <= 3 * W + 4
    # the first entries: integrate of slice 0, then its neighbours
    assert tuple(t[0]) == (0, 0, 0)


def test_wavefront_table_rejects_bad_arguments():
    with pytest.raises(md.MDError):
        md.md_wavefront_table(2, 4)
    with pytest.raises(md.MDError):
        md.md_wavefront_table(64, 0)
    with pytest.raises(md.MDError):
        md.md_wavefront_table(64, 65)
