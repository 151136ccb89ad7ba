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
and each network gets as many slots (64 replicate lanes each, with their own
state, parameters and records) as its share holds. A request waits in its
network's FIFO queue until a slot is free.

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

    def summary(self, results):
        lat = np.array([r.latency for r in results]) if results else np.zeros(1)
        return dict(requests=self.completed, wall_s=round(self.wall_s, 3),
                    requests_per_s=round(self.completed / self.wall_s, 3) if self.wall_s else 0.0,
                    node_days_per_s=self.node_days / self.wall_s if self.wall_s else 0.0,
                    transitions_per_s=self.transitions / self.wall_s if self.wall_s else 0.0,
                    p50_s=round(float(np.percentile(lat, 50)), 3), p99_s=round(float(np.percentile(lat, 99)), 3),
                    mean_s=round(float(lat.mean()), 3), steps=self.steps, slots=self.slots,
                    lane_occupancy=round(self.busy_lanes, 3))


def plan_slots(networks, hbm_budget, demand, max_slots=256):
    """Slots per network from an HBM byte budget split in proportion to
    `demand` (expected lane-days per network); at least one slot each."""
    per, base = [], []
    for net in networks:
        one = SlotHandle.workspace_bytes(net, 1)
        two = SlotHandle.workspace_bytes(net, 2)
        if one == 0 or two == 0:
            raise ValueError("network rejected by the slot handle")
        per.append(two - one)
        base.append(one - (two - one))
    w = np.asarray(demand, float)
    w = w / w.sum()
    out = []
    for j, net in enumerate(networks):
        n = int((hbm_budget * w[j] - base[j]) // per[j])
        # lane indices stay below 2^31: positions (nodes plus padding and the
        # units of the largest herds) times 64 lanes per slot
        cap = (2 ** 31 - 1) // (64 * (net.n_nodes + 512))
        out.append(int(min(max(n, 1), max_slots, cap)))
    return out, [b + n * p for b, n, p in zip(base, out, per)]


class Server:
    """Slot handles for the given networks, one stream each."""

    def __init__(self, networks, slots, *, max_ahead=4, device=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the server needs a GPU")
        self.torch = torch
        self.networks = networks
        self.max_ahead = max_ahead
        self.streams = [torch.cuda.Stream(device=device) for _ in networks]  # default priority
        self.handles = []
        for net, n, st in zip(networks, slots, self.streams):
            with torch.cuda.stream(st):
                self.handles.append(SlotHandle(net, n, stream=st.cuda_stream, device=device))
        # pinned download buffers, one pair per slot (a slot fetches only after
        # its previous fetch was collected)
        self.bufs = [[(torch.empty(net.n_days * 64, dtype=torch.int32, pin_memory=True),
                       torch.empty(net.n_days * 64, dtype=torch.int64, pin_memory=True)) for _ in range(n)]
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
        J = len(self.handles)
        for q in requests:
            if not 1 <= q["n_rep"] <= 64:
                raise ValueError(f"request {q['rid']}: n_rep must be in [1, 64]")
            if not 1 <= q["horizon"] <= self.networks[q["net"]].n_days:
                raise ValueError(f"request {q['rid']}: horizon beyond its network")
        queues = [deque() for _ in range(J)]
        free = [deque(range(h.n_slots)) for h in self.handles]
        running = [dict() for _ in range(J)]     # slot -> (request, admitted)
        fetching = [dict() for _ in range(J)]    # slot -> (request, admitted)
        stats = Stats(steps=[0] * J, slots=[h.n_slots for h in self.handles])
        results = []
        lanes_used = lanes_total = 0
        order = deque(sorted(requests, key=lambda q: q["arrival"]))
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        def landed(j, slot):
            """Whether the download of slot has landed; a request's own error
            is kept with its result."""
            try:
                ok = self.handles[j].query(slot)
            except SimError as e:
                errors[(j, slot)] = str(e)
                return True
            return ok

        errors = {}

        def collect(j, slot):
            q, adm = fetching[j].pop(slot)
            H, R = q["horizon"], q["n_rep"]
            pv, tr = self.bufs[j][slot]
            res = Result(q["rid"], j, R, H, q["arrival"] if realtime else 0.0, adm, now(),
                         pv[:H * R].numpy().reshape(H, R).copy(), tr[:H * R].numpy().reshape(H, R).copy(),
                         errors.pop((j, slot), None))
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
                # admit queued requests into free slots (a slot still being
                # downloaded is free: the download is ordered before its reuse)
                while queues[j] and free[j]:
                    q = queues[j].popleft()
                    slot = free[j].popleft()
                    h.start(slot, q["horizon"], q["coef"], q["alpha"], q["beta"], q["replicate_id"])
                    running[j][slot] = (q, now())
                    progressed = True
                if running[j] and h.in_flight() < self.max_ahead:
                    lanes_used += sum(q["n_rep"] for q, _ in running[j].values())
                    lanes_total += 64 * h.n_slots
                    finished = h.step()
                    stats.steps[j] += 1
                    if on_step is not None:
                        on_step(j, stats.steps[j])
                    for slot in finished:
                        # the slot's buffers still hold an earlier download: collect it first
                        while slot in fetching[j]:
                            if landed(j, slot):
                                collect(j, slot)
                        q, adm = running[j].pop(slot)
                        pv, tr = self.bufs[j][slot]
                        h.fetch(slot, pv, tr)
                        fetching[j][slot] = (q, adm)
                        free[j].append(slot)
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
        return results, stats
