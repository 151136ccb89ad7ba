"""Request loop over slot handles: many simulation requests against a few
resident networks, served from one GPU.

The paper's parameter-fitting workload runs many trajectories with different
rate parameters over one event database (Sec. 4.3). Here those trajectories
arrive as requests over time: each names a network, a horizon, up to 64
replicates with their own parameters, and the replicate ids that key its
random streams. The server keeps every network resident in a slot handle
(include/episim.h) and runs iteration-level batching: one step advances every
running slot of a network by one day (SSA, the day's events, phi update) in
shared launches, a finished slot's records are downloaded while the handle
goes on, and the freed slot takes the next queued request of that network at
the next step. Networks run on their own streams and overlap on the device.

Admission is bounded by an HBM budget: the budget is split between the
networks in proportion to the lane-days their requests are expected to need,
and each network gets as many slots (slot_lanes replicate lanes each, with
their own state, parameters and records) as its share holds. A request of
n replicates takes ceil(n / slot_lanes) slots, each running a contiguous part
of its replicates; narrow slots waste fewer idle lanes on small requests. A
request waits in its network's FIFO queue until enough slots are free.
A step's launches cover only the 64-lane columns that hold a running slot,
so idle slots cost nothing, and a request's parts go to the free slots of the
columns that already run the most slots: fewer columns, fewer idle lanes.

Every result is bit-identical to the same request run alone (sim_create with
the same network, parameters and replicate ids, run for its horizon): a slot
computes its lanes exactly as a plain handle does, whatever else runs.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from .sim import SimError, SlotHandle


@dataclass
class Result:
    rid: int
    net: int
    n_rep: int
    horizon: int
    arrival: float            # seconds since the serve() start
    admitted: float
    done: float               # records on the host
    prevalence: np.ndarray    # [horizon][n_rep] infected-node counts after each day
    transitions: np.ndarray   # [horizon][n_rep] SSA transitions per day
    error: str | None = None  # the request's own device-side error (its records are then void)

    @property
    def latency(self):
        return self.done - self.arrival


@dataclass
class Stats:
    wall_s: float = 0.0
    completed: int = 0
    node_days: float = 0.0     # sum over results of n_nodes * horizon * n_rep
    transitions: int = 0
    steps: list = field(default_factory=list)   # steps issued per network
    slots: list = field(default_factory=list)   # slots per network
    busy_lanes: float = 0.0    # mean fraction of slot lanes that held a live replicate per step
    column_lanes: float = 0.0  # the same over the lanes of the columns a step launched

    def summary(self, results):
        lat = np.array([r.latency for r in results]) if results else np.zeros(1)
        return dict(requests=self.completed, wall_s=round(self.wall_s, 3),
                    requests_per_s=round(self.completed / self.wall_s, 3) if self.wall_s else 0.0,
                    node_days_per_s=self.node_days / self.wall_s if self.wall_s else 0.0,
                    transitions_per_s=self.transitions / self.wall_s if self.wall_s else 0.0,
                    p50_s=round(float(np.percentile(lat, 50)), 3), p99_s=round(float(np.percentile(lat, 99)), 3),
                    mean_s=round(float(lat.mean()), 3), steps=self.steps, slots=self.slots,
                    lane_occupancy=round(self.busy_lanes, 3), column_occupancy=round(self.column_lanes, 3))


def pick_slot(free, running, per_col):
    """The free slot (from the set `free`) in the column of 64 lanes that
    already runs the most slots of `running`, then the lowest column and slot:
    the parts of small requests share columns, so a step launches fewer."""
    busy = {}
    for sl in running:
        busy[sl // per_col] = busy.get(sl // per_col, 0) + 1
    return min(free, key=lambda sl: (-busy.get(sl // per_col, 0), sl))


def plan_slots(networks, hbm_budget, demand, max_slots=None, slot_lanes=64):
    """Slots per network from an HBM byte budget split in proportion to
    `demand` (expected lane-days per network); at least one column of 64
    lanes each, whole columns only."""
    per_col = 64 // slot_lanes
    max_slots = 256 * per_col if max_slots is None else max_slots
    per, base = [], []
    for net in networks:
        one = SlotHandle.workspace_bytes(net, per_col, slot_lanes)
        two = SlotHandle.workspace_bytes(net, 2 * per_col, slot_lanes)
        if one == 0 or two == 0:
            raise ValueError("network rejected by the slot handle")
        per.append((two - one) / per_col)
        base.append(one - (two - one))
    w = np.asarray(demand, float)
    w = w / w.sum()
    out = []
    for j, net in enumerate(networks):
        n = int((hbm_budget * w[j] - base[j]) // per[j])
        # lane indices stay below 2^31: positions (nodes plus padding and the
        # units of the largest herds) times the lanes of all slots
        cap = (2 ** 31 - 1) // (slot_lanes * (net.n_nodes + 512))
        n = int(min(max(n, per_col), max_slots, cap))
        out.append(max(per_col, n // per_col * per_col))
    return out, [int(b + n * p) for b, n, p in zip(base, out, per)]


class Server:
    """Slot handles for the given networks, one stream each."""

    def __init__(self, networks, slots, *, max_ahead=4, device=0, slot_lanes=64):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the server needs a GPU")
        self.torch = torch
        self.networks = networks
        self.max_ahead = max_ahead
        self.W = int(slot_lanes)
        self.streams = [torch.cuda.Stream(device=device) for _ in networks]  # default priority
        self.handles = []
        for net, n, st in zip(networks, slots, self.streams):
            with torch.cuda.stream(st):
                self.handles.append(SlotHandle(net, n, stream=st.cuda_stream, device=device, slot_lanes=self.W))
        # pinned download buffers, one pair per slot (a slot fetches only after
        # its previous fetch was collected)
        self.bufs = [[(torch.empty(net.n_days * self.W, dtype=torch.int32, pin_memory=True),
                       torch.empty(net.n_days * self.W, dtype=torch.int64, pin_memory=True)) for _ in range(n)]
                     for net, n in zip(networks, slots)]

    def close(self):
        for h in self.handles:
            h.close()
        self.handles = []

    def serve(self, requests, *, realtime=True, on_step=None):
        """Serve the requests (dicts from farmnet.synth.serving_requests, sorted
        by arrival). With realtime, a request enters its queue once the wall
        clock passes its arrival time; otherwise all are queued at once.
        Returns (results in completion order, Stats)."""
        J, W = len(self.handles), self.W
        for q in requests:
            if not 1 <= q["n_rep"] <= 64:
                raise ValueError(f"request {q['rid']}: n_rep must be in [1, 64]")
            if not 1 <= q["horizon"] <= self.networks[q["net"]].n_days:
                raise ValueError(f"request {q['rid']}: horizon beyond its network")
            if -(-q["n_rep"] // W) > self.handles[q["net"]].n_slots:
                raise ValueError(f"request {q['rid']}: more replicates than its network's slots hold")
        queues = [deque() for _ in range(J)]
        free = [set(range(h.n_slots)) for h in self.handles]
        per_col = 64 // W
        running = [dict() for _ in range(J)]     # slot -> (request, part, admitted)
        fetching = [dict() for _ in range(J)]    # slot -> (request, part, admitted)
        parts = {}                               # request id -> {part: (prevalence, transitions, error)}
        stats = Stats(steps=[0] * J, slots=[h.n_slots for h in self.handles])
        results = []
        lanes_used = lanes_total = col_lanes = 0

        def take_slot(j):
            best = pick_slot(free[j], running[j], per_col)
            free[j].discard(best)
            return best
        order = deque(sorted(requests, key=lambda q: q["arrival"]))
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        errors = {}

        def landed(j, slot):
            """Whether the download of slot has landed; a request's own error
            is kept with its result."""
            try:
                ok = self.handles[j].query(slot)
            except SimError as e:
                errors[(j, slot)] = str(e)
                return True
            return ok

        def collect(j, slot):
            """A part's records are on the host; the request is done once all
            its parts are."""
            q, part, adm = fetching[j].pop(slot)
            H, R = q["horizon"], q["n_rep"]
            n = min(W, R - part * W)
            pv, tr = self.bufs[j][slot]
            got = parts.setdefault(q["rid"], {})
            got[part] = (pv[:H * n].numpy().reshape(H, n).copy(), tr[:H * n].numpy().reshape(H, n).copy(),
                         errors.pop((j, slot), None))
            if len(got) < -(-R // W):
                return
            del parts[q["rid"]]
            ordered = [got[k] for k in range(len(got))]
            err = next((e for _, _, e in ordered if e), None)
            res = Result(q["rid"], j, R, H, q["arrival"] if realtime else 0.0, adm, now(),
                         np.concatenate([a for a, _, _ in ordered], axis=1),
                         np.concatenate([b for _, b, _ in ordered], axis=1), err)
            results.append(res)
            stats.completed += 1
            stats.node_days += float(self.networks[j].n_nodes) * H * R
            stats.transitions += int(res.transitions.sum())

        while len(results) < len(requests):
            progressed = False
            t = now()
            while order and (not realtime or order[0]["arrival"] <= t):
                q = order.popleft()
                queues[q["net"]].append(q)
            for j, h in enumerate(self.handles):
                # collect landed downloads
                for slot in list(fetching[j]):
                    if landed(j, slot):
                        collect(j, slot)
                        progressed = True
                # admit queued requests (first come first served) while their
                # parts find free slots (a slot still being downloaded is free:
                # the download is ordered before its reuse)
                while queues[j] and len(free[j]) >= -(-queues[j][0]["n_rep"] // W):
                    q = queues[j].popleft()
                    adm = now()
                    for part in range(-(-q["n_rep"] // W)):
                        slot = take_slot(j)
                        sl = slice(part * W, min(q["n_rep"], (part + 1) * W))
                        h.start(slot, q["horizon"], q["coef"][sl], q["alpha"][sl], q["beta"][sl],
                                q["replicate_id"][sl])
                        running[j][slot] = (q, part, adm)
                    progressed = True
                if running[j] and h.in_flight() < self.max_ahead:
                    lanes_used += sum(min(W, q["n_rep"] - part * W) for q, part, _ in running[j].values())
                    lanes_total += W * h.n_slots
                    col_lanes += 64 * len({sl // per_col for sl in running[j]})
                    finished = h.step()
                    stats.steps[j] += 1
                    if on_step is not None:
                        on_step(j, stats.steps[j])
                    for slot in finished:
                        # the slot's buffers still hold an earlier download: collect it first
                        while slot in fetching[j]:
                            if landed(j, slot):
                                collect(j, slot)
                        q, part, adm = running[j].pop(slot)
                        pv, tr = self.bufs[j][slot]
                        h.fetch(slot, pv, tr)
                        fetching[j][slot] = (q, part, adm)
                        free[j].add(slot)
                    progressed = True
            if not progressed:
                if realtime and order and not any(running) and not any(fetching):
                    time.sleep(max(0.0, min(order[0]["arrival"] - now(), 0.01)))
                else:
                    time.sleep(0.0002)
        for st in self.streams:
            st.synchronize()
        stats.wall_s = now()
        stats.busy_lanes = lanes_used / lanes_total if lanes_total else 0.0
        stats.column_lanes = lanes_used / col_lanes if col_lanes else 0.0
        return results, stats
