"""Slot handles and the request loop: every request served in a mix of other
requests (different replicate counts, horizons, parameters and start days,
slots reused) gives records and state bit-identical to the same request run
alone on a plain handle, which the parity tests pin to the oracle. Calls go
through the C ABI."""
import numpy as np
import pytest

from farmnet import EXIT, synth
from oracle import oracle as O
import paper_1502_02908_amd as P
from paper_1502_02908_amd.serve import Server

from .gpu_common import say

pytestmark = pytest.mark.gpu


def request(rid, n_rep, horizon, seed):
    coef, alpha, beta = synth.prior_draws(n_rep, seed=seed)
    return dict(rid=rid, n_rep=n_rep, horizon=horizon, coef=coef, alpha=alpha, beta=beta,
                replicate_id=np.uint32(rid) * np.uint32(64) + np.arange(n_rep, dtype=np.uint32))


def alone(net, q):
    """The request on a plain handle: records of its horizon and its final state."""
    p = net.with_replicates(q["n_rep"], coef=q["coef"], alpha=q["alpha"], beta=q["beta"],
                            replicate_id=q["replicate_id"])
    with P.Simulator(p) as s:
        s.run(q["horizon"])
        tr = s.trajectory()
        u, v, day = s.get_state()
    H = q["horizon"]
    assert day == H
    return dict(prevalence=tr["prevalence"][:H], transitions=tr["transitions"][:H], totals=tr["totals"][:H], u=u, v=v)


def test_slots_mixed_requests_equal_alone():
    net = synth.sise3_network(n_nodes=1500, n_days=80, seed=21, age_days=(10, 30))
    say(f"[serve] slots on {net.n_nodes} nodes x {net.n_days} days")
    reqs = {"A": request(1, 1, 80, 11), "B": request(2, 17, 30, 12), "C": request(3, 64, 60, 13),
            "D": request(4, 40, 41, 14)}
    got = {}
    H = P.SlotHandle(net, 3)
    try:
        where = {}

        def start(name, slot):
            q = reqs[name]
            H.start(slot, q["horizon"], q["coef"], q["alpha"], q["beta"], q["replicate_id"])
            where[slot] = name

        def fetch(slot):
            q = reqs[where[slot]]
            pv = np.zeros((q["horizon"], q["n_rep"]), np.int32)
            tr = np.zeros((q["horizon"], q["n_rep"]), np.int64)
            to = np.zeros((q["horizon"], q["n_rep"], net.n_comp), np.int64)
            H.fetch(slot, pv, tr, to)
            while not H.query(slot):
                pass
            got[where[slot]] = dict(prevalence=pv, transitions=tr, totals=to)
            if where[slot] != "B":
                got[where[slot]]["u"], got[where[slot]]["v"] = H.state(slot, q["n_rep"])

        start("A", 0)
        start("B", 2)
        step = 0
        while len(got) < 4:
            if step == 5:
                start("C", 1)
            fin = H.step()
            step += 1
            for slot in fin:
                fetch(slot)
                if where[slot] == "B":
                    start("D", 2)  # reuse the slot at once
        assert step == 81
    finally:
        H.close()
    for name, q in reqs.items():
        ref = alone(net, q)
        for k, v in got[name].items():
            assert np.array_equal(v, ref[k]), (name, k)
        assert ref["transitions"].sum() > 0
    say("[serve] slots == alone for A(R=1) B(R=17) C(R=64) D(R=40, reused slot)")


def test_slot_request_against_oracle():
    net = synth.sise3_network(n_nodes=400, n_days=25, seed=22, age_days=(5, 12))
    q = request(9, 5, 19, 15)
    with P.SlotHandle(net, 2) as H:
        H.start(1, q["horizon"], q["coef"], q["alpha"], q["beta"], q["replicate_id"])
        fin = []
        while not fin:
            fin = H.step()
        pv = np.zeros((19, 5), np.int32)
        tr = np.zeros((19, 5), np.int64)
        H.fetch(1, pv, tr)
        while not H.query(1):
            pass
        u, v = H.state(1, 5)
    p = net.truncated(19).with_replicates(5, coef=q["coef"], alpha=q["alpha"], beta=q["beta"],
                                          replicate_id=q["replicate_id"])
    o = O.run(p, threads=8)
    assert np.array_equal(pv, o["prevalence"]) and np.array_equal(tr, o["transitions"])
    assert np.array_equal(u, o["u"]) and np.allclose(v, o["v"], rtol=1e-12, atol=0)


def test_slot_error_stays_in_its_slot():
    # an exit of 3 infected animals on day 1 is feasible only where no
    # infected animal recovered on day 0: with recovery on, some replicate
    # fails; with all rates 0 every replicate succeeds
    m = synth.sis_model(upsilon=0.5, gamma=0.5)
    n = 40
    u0 = np.tile([[3, 3]], (n, 1))
    net = synth.events_only(u0, [(1, EXIT, np.arange(n), -1, 3, 2, -1)], n_days=3)
    net.E = np.concatenate([m["E"], [[0], [1]]], axis=1).astype(np.int32)
    net.uses_phi[:] = 0
    bad = dict(rid=0, n_rep=8, horizon=3, coef=np.tile([0.5, 0.5], (8, 1)), alpha=np.ones(8),
               beta=np.full((8, 4), 0.1), replicate_id=np.arange(8, dtype=np.uint32))
    good = dict(bad, rid=1, coef=np.zeros((8, 2)), replicate_id=np.arange(64, 72, dtype=np.uint32))
    with P.SlotHandle(net, 2) as H:
        for slot, q in ((0, bad), (1, good)):
            H.start(slot, q["horizon"], q["coef"], q["alpha"], q["beta"], q["replicate_id"])
        fin = []
        while len(fin) < 2:
            fin += H.step()
        pv = {s: np.zeros((3, 8), np.int32) for s in (0, 1)}
        for s in (0, 1):
            H.fetch(s, pv[s])
        with pytest.raises(P.SimError) as e:
            while not H.query(0):
                pass
        assert e.value.code == -4 and "slot 0" in str(e.value)
        while not H.query(1):
            pass
    ref = alone(net, good)
    assert np.array_equal(pv[1], ref["prevalence"])


def test_server_results_equal_alone():
    nets = [synth.sise3_network(n_nodes=600, n_days=60, seed=23, age_days=(10, 30)),
            synth.sise3_network(n_nodes=2500, n_days=90, seed=24, age_days=(10, 30))]
    reqs = synth.serving_requests(n_requests=14, rate=400.0, n_networks=2, horizon=(20, 60), seed=7)
    srv = Server(nets, slots=[3, 2], max_ahead=3)
    try:
        results, stats = srv.serve(reqs)
    finally:
        srv.close()
    say(f"[serve] {stats.summary(results)}")
    assert sorted(r.rid for r in results) == list(range(14))
    by_id = {q["rid"]: q for q in reqs}
    for r in results:
        q = by_id[r.rid]
        ref = alone(nets[q["net"]], q)
        assert np.array_equal(r.prevalence, ref["prevalence"]), r.rid
        assert np.array_equal(r.transitions, ref["transitions"]), r.rid
        assert r.latency >= 0


@pytest.mark.parametrize("W", [8, 16, 32])
def test_narrow_slots_at_different_days_equal_alone(W):
    # slots of W lanes share a wavefront column while each runs its own
    # request from its own day: every lane takes its day from its slot
    net = synth.sise3_network(n_nodes=1500, n_days=70, seed=25, u=3.0, age_days=(10, 30), shifted_moves=0.3)
    n_slots = 128 // W
    reqs = [request(10 + k, 1 + (5 * k) % W, 20 + (9 * k) % 45, 40 + k) for k in range(n_slots + 2)]
    starts = {k: (3 * k if k < n_slots else None) for k in range(len(reqs))}
    got, where, step = {}, {}, 0
    with P.SlotHandle(net, n_slots, slot_lanes=W) as H:
        pending = list(range(len(reqs)))
        while len(got) < len(reqs):
            for k in list(pending):
                free = [sl for sl in range(n_slots) if sl not in where.values()]
                if free and (starts[k] is None or starts[k] <= step):
                    q = reqs[k]
                    H.start(free[0], q["horizon"], q["coef"], q["alpha"], q["beta"], q["replicate_id"])
                    where[k] = free[0]
                    pending.remove(k)
            for sl in H.step():
                k = next(k for k, v in where.items() if v == sl)
                q = reqs[k]
                pv = np.zeros((q["horizon"], q["n_rep"]), np.int32)
                tr = np.zeros((q["horizon"], q["n_rep"]), np.int64)
                to = np.zeros((q["horizon"], q["n_rep"], net.n_comp), np.int64)
                H.fetch(sl, pv, tr, to)
                while not H.query(sl):
                    pass
                u, v = H.state(sl, q["n_rep"])
                got[k] = dict(prevalence=pv, transitions=tr, totals=to, u=u, v=v)
                del where[k]
            step += 1
    for k, q in enumerate(reqs):
        ref = alone(net, q)
        for key, val in got[k].items():
            assert np.array_equal(val, ref[key]), (W, k, key)
    say(f"[serve] {len(reqs)} requests in slots of {W} lanes == alone")


def test_server_with_narrow_slots_equals_alone():
    nets = [synth.sise3_network(n_nodes=700, n_days=60, seed=26, age_days=(10, 30)),
            synth.sise3_network(n_nodes=2000, n_days=80, seed=27, age_days=(10, 30))]
    reqs = synth.serving_requests(n_requests=12, rate=400.0, n_networks=2, horizon=(20, 60), seed=8)
    srv = Server(nets, slots=[8, 4], max_ahead=3, slot_lanes=16)
    try:
        results, stats = srv.serve(reqs)
    finally:
        srv.close()
    say(f"[serve] narrow slots: {stats.summary(results)}")
    assert sorted(r.rid for r in results) == list(range(12))
    by_id = {q["rid"]: q for q in reqs}
    for r in results:
        q = by_id[r.rid]
        ref = alone(nets[q["net"]], q)
        assert r.error is None
        assert np.array_equal(r.prevalence, ref["prevalence"]), r.rid
        assert np.array_equal(r.transitions, ref["transitions"]), r.rid


def test_scattered_slots_with_idle_columns_equal_alone():
    # a step launches only the columns that hold a running slot and the slots
    # that have a day of events: running slots far apart, columns idle in
    # between, starts at different steps and the host many steps ahead of the
    # device (the run lists' pinned ring wraps)
    net = synth.sise3_network(n_nodes=1200, n_days=60, seed=28, age_days=(10, 30), shifted_moves=0.2)
    W, n_slots = 16, 32
    plan = [(1, 0, request(50, 16, 40, 61)), (14, 2, request(51, 5, 55, 62)), (15, 2, request(52, 11, 30, 63)),
            (29, 7, request(53, 16, 50, 64)), (30, 7, request(54, 3, 21, 65))]
    got, step = {}, 0
    with P.SlotHandle(net, n_slots, slot_lanes=W) as H:
        while len(got) < len(plan):
            for slot, t0, q in plan:
                if t0 == step:
                    H.start(slot, q["horizon"], q["coef"], q["alpha"], q["beta"], q["replicate_id"])
            for sl in H.step():
                slot, t0, q = next(x for x in plan if x[0] == sl)
                pv = np.zeros((q["horizon"], q["n_rep"]), np.int32)
                tr = np.zeros((q["horizon"], q["n_rep"]), np.int64)
                to = np.zeros((q["horizon"], q["n_rep"], net.n_comp), np.int64)
                H.fetch(sl, pv, tr, to)
                while not H.query(sl):
                    pass
                u, v = H.state(sl, q["n_rep"])
                got[sl] = dict(prevalence=pv, transitions=tr, totals=to, u=u, v=v)
            step += 1
    for slot, t0, q in plan:
        ref = alone(net, q)
        for key, val in got[slot].items():
            assert np.array_equal(val, ref[key]), (slot, key)
    say(f"[serve] {len(plan)} requests in scattered slots == alone")
