"""Race detection and utilisation from the per-item trace of a persistent launch.

`md_step` with MD_OPT_TRACE records one record per work item: which item (step k within
its launch, slice, chunk, phase), when its worker claimed a queue slot, when the item's
inputs were known to be complete (after the acquire), and when it finished (after the
release).  The dependency rule of the cyclic schedule (slice i advances from step t to
t+1 once slices i-1 and i+1 have reached step t; the data flow of Sec. 3.1, Table 1,
generalised to work items) gives, for every item, the items whose results it reads:

  * force/integrate of slice i at step k >= 1 (phase 0) reads the finalised cells of
    slices i-1, i, i+1 for step k, i.e. the finalise items (phase 1) of step k-1 of those
    slices (every chunk);
  * finalise of slice i for step k+1 (phase 1, recorded with k) reads what the update
    items of slices i-1, i, i+1 at step k wrote (phase 0, or phase 2 with the thermostat);
  * thermostat integrate of slice i at step k (phase 2) needs every force item (phase 0)
    of slice i at step k.

`check` verifies that each launch ran every item exactly once and that every item became
ready no earlier than each of its inputs finished; a violation is a race.  The device
clock is one counter for the whole GPU.  This module only reads records; it computes
nothing of the method.
"""
from __future__ import annotations

import numpy as np


def _per_key_max(keys, vals, shape):
    out = np.full(shape, -1, dtype=np.int64)
    np.maximum.at(out, keys, vals.astype(np.int64))
    return out


def _per_key_min(keys, vals, shape):
    out = np.full(shape, np.iinfo(np.int64).max, dtype=np.int64)
    np.minimum.at(out, keys, vals.astype(np.int64))
    return out


def check(rec, slices: int):
    """Returns a dict: items, launches, violations (list of strings, empty when clean)."""
    bad = []
    rec = np.asarray(rec)
    if len(rec) == 0:
        return {"items": 0, "launches": 0, "violations": ["empty trace"]}
    order_ok = (rec["t_claim"] <= rec["t_ready"]) & (rec["t_ready"] <= rec["t_done"])
    if not order_ok.all():
        bad.append(f"{int((~order_ok).sum())} records with claim/ready/done out of order")
    S = int(slices)
    for L in np.unique(rec["launch"]):
        r = rec[rec["launch"] == L]
        K = int(r["k"].max()) + 1
        phases = set(int(p) for p in np.unique(r["phase"]))
        if not phases <= {0, 1, 2}:
            bad.append(f"launch {L}: unknown phase in {sorted(phases)}")
            continue
        nvt = 2 in phases
        done, ready = {}, {}
        for ph in sorted(phases):
            m = r["phase"] == ph
            nch = int(r["chunk"][m].max()) + 1
            key = (r["k"][m].astype(np.int64) * S + r["slice"][m].astype(np.int64)) * nch + r["chunk"][m]
            cnt = np.bincount(key, minlength=K * S * nch)
            if len(cnt) != K * S * nch or (cnt != 1).any():
                missing = int((cnt[: K * S * nch] == 0).sum())
                dup = int((cnt > 1).sum())
                bad.append(f"launch {L} phase {ph}: {missing} items missing, {dup} run twice")
            ks = r["k"][m].astype(np.int64) * S + r["slice"][m].astype(np.int64)
            done[ph] = _per_key_max(ks, r["t_done"][m], K * S).reshape(K, S)
            ready[ph] = _per_key_min(ks, r["t_ready"][m], K * S).reshape(K, S)
        upd = 2 if nvt else 0

        def nb_max(a):  # max over slices i-1, i, i+1 (periodic)
            return np.maximum(np.maximum(np.roll(a, 1, axis=1), a), np.roll(a, -1, axis=1))

        # phase 0 at step k >= 1 after the finalise items of step k-1 of i-1, i, i+1
        if K > 1 and 1 in done:
            need = nb_max(done[1][:-1])
            late = ready[0][1:] < need
            if late.any():
                k, i = np.argwhere(late)[0]
                bad.append(f"launch {L}: {int(late.sum())} force items started before their "
                           f"neighbours were finalised (first: step {k + 1}, slice {i})")
        # phase 1 at step k after the update items of step k of i-1, i, i+1
        if 1 in ready:
            need = nb_max(done[upd])
            late = ready[1] < need
            if late.any():
                k, i = np.argwhere(late)[0]
                bad.append(f"launch {L}: {int(late.sum())} finalise items started before the "
                           f"neighbouring updates finished (first: step {k}, slice {i})")
        if nvt:
            late = ready[2] < done[0]
            if late.any():
                bad.append(f"launch {L}: {int(late.sum())} thermostat integrate items started "
                           "before all force items of their slice finished")
    return {"items": int(len(rec)), "launches": int(len(np.unique(rec["launch"]))), "violations": bad}


def utilisation(rec, workers: int):
    """Fractions of the workers' time (workers x span of each launch, summed) spent
    executing items and waiting for a ready item; time-weighted mean number of distinct
    steps among the force items executing at once."""
    rec = np.asarray(rec)
    span = 0
    execute = wait = 0
    lev_area = lev_time = 0.0
    for L in np.unique(rec["launch"]):
        r = rec[rec["launch"] == L]
        t0, t1 = int(r["t_claim"].min()), int(r["t_done"].max())
        span += workers * (t1 - t0)
        execute += int((r["t_done"].astype(np.int64) - r["t_ready"].astype(np.int64)).sum())
        wait += int((r["t_ready"].astype(np.int64) - r["t_claim"].astype(np.int64)).sum())
        f = r[r["phase"] == 0]
        if len(f):
            ev_t = np.concatenate([f["t_ready"], f["t_done"]]).astype(np.int64)
            ev_k = np.concatenate([f["k"], f["k"]]).astype(np.int64)
            ev_s = np.concatenate([np.ones(len(f), np.int64), -np.ones(len(f), np.int64)])
            o = np.lexsort((-ev_s, ev_t))
            active = {}
            last_t = None
            for t, k, s in zip(ev_t[o], ev_k[o], ev_s[o]):
                if last_t is not None and active and t > last_t:
                    lev_area += (t - last_t) * len(active)
                    lev_time += t - last_t
                active[k] = active.get(k, 0) + s
                if active[k] == 0:
                    del active[k]
                last_t = t
    return {"execute": execute / span if span else 0.0, "wait": wait / span if span else 0.0,
            "levels_in_flight": lev_area / lev_time if lev_time else 0.0}
