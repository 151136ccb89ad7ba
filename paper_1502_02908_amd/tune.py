"""Choice of launch shape and level grouping for one workload, by timing.

Every setting of sim_device_opts gives the same trajectory bit for bit: the
random streams are keyed by node, event and day (include/episim.h), never by
launch shape, grouping or node order. So a setting can be chosen on speed
alone. The tuner runs the workload once with the default settings up to a
day typical of the horizon (half of it by default), keeps that state, and
then, for each candidate, loads the state into a handle built with the
candidate's settings and times the same window of days (once untimed, then
timed). It also checks that every candidate ends the window in the same state.

Candidates vary what the per-day schedule leaves open, and only what changes
the schedule of the workload at hand (candidates_for):
  launch             per-day kernels, or one cooperative kernel for the whole run;
  small_level        up to which size event levels run several per launch in
                     one workgroup (0: default 512);
  few_chains         how many live chains of a wavefront may be walked one after
                     another by the whole wavefront (0: default 4, negative: never);
one lane per node (one trajectory per instance):
  group_herds        how many of the largest herds of a large instance get a
                     whole workgroup for their chains (0: default 4, negative: none);
  group_min_attempts how many attempts a chain must still expect in the day for
                     the workgroup to walk it (0: default 4096);
  tile_nodes         nonzero: tiles of this many nodes instead, each wavefront
                     walking one node's chain with all its lanes;
replicate tiles (several replicates per instance):
  tile_nodes         nodes per tile of 64 replicate lanes (0: default 128), taken
                     one at a time by the tile's four wavefronts;
  heavy_herds        how many of the largest herds get a wavefront per (herd,
                     replicate) chain (0: default 64, negative: none).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from .sim import LAUNCH_KERNELS, LAUNCH_PERSISTENT, Simulator

LANE_CANDIDATES = (
    dict(),
    dict(group_herds=-1),
    dict(group_herds=8),
    dict(group_min_attempts=1024),
    dict(group_min_attempts=16384),
    dict(small_level=128),
    dict(small_level=4096),
    dict(few_chains=1),
    dict(few_chains=8),
    dict(launch=LAUNCH_PERSISTENT),
    dict(tile_nodes=4),
    dict(tile_nodes=16),
)
TILE_CANDIDATES = (
    dict(),
    dict(tile_nodes=64),
    dict(tile_nodes=256),
    dict(heavy_herds=-1),
    dict(heavy_herds=32),
    dict(heavy_herds=128),
    dict(few_chains=1),
    dict(few_chains=-1),
    dict(small_level=4096),
    dict(launch=LAUNCH_PERSISTENT),
)
CANDIDATES = LANE_CANDIDATES


def candidates_for(p):
    """The candidate settings that change the schedule of problem p (or of a
    list of instances packed in one handle)."""
    first = p[0] if isinstance(p, (list, tuple)) else p
    return TILE_CANDIDATES if first.n_rep > 1 else LANE_CANDIDATES


@dataclass
class Tuning:
    best: dict                                  # the fastest candidate's options
    table: list = field(default_factory=list)   # (options, ms per day of the window) per candidate
    start_day: int = 0
    window: int = 0

    def summary(self):
        rows = [dict(opts=o, ms_per_day=round(ms, 4)) for o, ms in self.table]
        return dict(best=self.best, start_day=self.start_day, window=self.window, candidates=rows)


def _sync_time(sim, n_days):
    sim.sync()
    t0 = time.perf_counter()
    sim.run(n_days)
    sim.sync()
    return time.perf_counter() - t0


def autotune(p, *, start_day=None, window=None, candidates=None, margin=0.03, log=None) -> Tuning:
    """Time each candidate's settings over days [start_day, start_day + window)
    of problem p (a farmnet.Problem, or a list of instances packed in one
    handle) from the state the default settings reach at start_day; return the
    fastest (the first candidate, the defaults, unless another beats it by
    more than `margin`). Raises if two candidates end the window in different
    states (they must not). log, if given, is called with a line per
    candidate as it is timed."""
    if candidates is None:
        candidates = candidates_for(p)
    D = (p[0] if isinstance(p, (list, tuple)) else p).n_days
    start = D // 2 if start_day is None else int(start_day)
    if not 0 <= start < D:
        raise ValueError("start_day must lie in [0, n_days)")
    win = min(60, D - start) if window is None else int(window)
    if not 1 <= win <= D - start:
        raise ValueError("window must lie in [1, n_days - start_day]")
    with Simulator(p) as sim:
        if start:
            sim.run(start)
        u0, v0, day = sim.get_state()
    table, ends = [], []
    for cand in candidates:
        cand = dict(cand)
        with Simulator(p, **cand) as sim:
            sim.set_state(u0, v0, day)
            _sync_time(sim, win)           # untimed: code objects, caches
            sim.set_state(u0, v0, day)
            dt = _sync_time(sim, win)
            u, v, d_end = sim.get_state()
        table.append((dict(cand), 1e3 * dt / win))
        ends.append((u, v.view(np.int64), d_end))
        if log is not None:
            log(f"candidate {len(table)}/{len(candidates)} {cand}: {1e3 * dt / win:.4f} ms per day")
    ref = ends[0]
    for (cand, _), (u, v, d_end) in zip(table, ends):
        if d_end != ref[2] or not np.array_equal(u, ref[0]) or not np.array_equal(v, ref[1]):
            raise RuntimeError(f"candidate {cand} ended the window in another state")
    # a candidate replaces the first (the defaults) only if it is faster by
    # more than the margin: closer calls are within the timing noise of a
    # short window and need not carry over to the whole horizon
    fastest = min(table, key=lambda row: row[1])
    best = fastest[0] if fastest[1] < table[0][1] * (1.0 - margin) else table[0][0]
    return Tuning(best=best, table=table, start_day=start, window=win)
