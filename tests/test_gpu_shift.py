"""External transfers whose shift column moves the drawn animals into another
compartment at the destination (Sec. 3.2, eq:event), on the GPU against the
oracle: every event path of the library sees such moves (the day's levels in
LDS, large levels with a launch of their own, runs of small levels in one
workgroup, replicate tiles, the persistent launch, packed instances and slot
handles). Counts and records bit-exact, phi within 1e-12 relative."""
import os

import numpy as np
import pytest

from farmnet import EXTERNAL, synth
from oracle import oracle as O
import paper_1502_02908_amd as P

from .gpu_common import assert_parity, gpu_run, say

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


def shifted_network(n_nodes, n_days, seed, e2=235.0 / 37221.0, u=10.0):
    p = synth.sise3_network(n_nodes=n_nodes, n_days=n_days, seed=seed, u=u, age_days=(10, 30),
                            e2_per_node_day=e2, shifted_moves=0.6)
    moves = p.ev_kind == EXTERNAL
    assert (p.ev_shift[moves] >= 0).sum() > 0.2 * moves.sum()
    return p


@pytest.mark.parametrize("launch", [P.LAUNCH_KERNELS, P.LAUNCH_PERSISTENT])
def test_shifted_moves_lds_days(launch):
    # about 20 moves a day: every day's levels run in LDS (k_event_day)
    p = shifted_network(3000, 120, seed=71)
    p.record_days = np.array([0, 60, 119], np.int32)
    say(f"[shift] LDS days launch={launch}: {p.n_events} events")
    g = gpu_run(p, launch=launch)
    o = O.run(p, threads=THREADS)
    assert_parity(g, o)
    assert o["transitions"].sum() > 10000


@pytest.mark.parametrize("small_level", [0, 1])
def test_shifted_moves_large_levels(small_level):
    # about 1200 moves a day: past the LDS day's capacity, so large levels get
    # a launch of their own; small_level = 1 sends every level to its own
    # launch, the default groups the small ones into one workgroup
    p = shifted_network(4000, 40, seed=72, e2=0.3)
    p.record_days = np.array([39], np.int32)
    say(f"[shift] large levels small_level={small_level}: {p.n_events} events")
    g = gpu_run(p, small_level=small_level)
    o = O.run(p, threads=THREADS)
    assert_parity(g, o)


def test_shifted_moves_replicate_tiles():
    base = shifted_network(900, 60, seed=73, e2=0.05)
    coef, alpha, beta = synth.prior_draws(64, seed=74)
    p = base.with_replicates(64, coef=coef * 3, alpha=alpha, beta=beta,
                             replicate_id=np.arange(500, 564, dtype=np.uint32))
    p.record_days = np.array([30, 59], np.int32)
    say(f"[shift] replicate tiles R=64: {p.n_events} events")
    g = gpu_run(p)
    o = O.run(p, threads=THREADS)
    assert_parity(g, o)


def test_shifted_moves_packed_instances():
    probs = []
    for k, n in enumerate((700, 2100, 300)):
        q = shifted_network(n, 50, seed=80 + k, e2=0.02)
        q.seed = 900 + k
        probs.append(q)
    with P.Simulator(probs) as sim:
        sim.run(0)
        traj = sim.trajectory()
        u, v, _ = sim.get_state()
    off = 0
    for k, q in enumerate(probs):
        o = O.run(q, threads=THREADS)
        sl = slice(off, off + q.n_nodes)
        assert np.array_equal(u[:, sl], o["u"]), k
        assert np.array_equal(v[:, sl].view(np.int64), o["v"].view(np.int64)), k
        assert np.array_equal(traj["prevalence"][:, k:k + 1], o["prevalence"]), k
        assert np.array_equal(traj["totals"][:, k:k + 1], o["totals"]), k
        off += q.n_nodes


def test_shifted_moves_slot_handle():
    net = shifted_network(600, 30, seed=75, e2=0.05)
    coef, alpha, beta = synth.prior_draws(9, seed=76)
    rid = np.arange(64, 73, dtype=np.uint32)
    with P.SlotHandle(net, 2) as H:
        H.start(1, 30, coef, alpha, beta, rid)
        fin = []
        while not fin:
            fin = H.step()
        pv = np.zeros((30, 9), np.int32)
        tr = np.zeros((30, 9), np.int64)
        to = np.zeros((30, 9, 6), np.int64)
        H.fetch(1, pv, tr, to)
        while not H.query(1):
            pass
        u, v = H.state(1, 9)
    p = net.with_replicates(9, coef=coef, alpha=alpha, beta=beta, replicate_id=rid)
    o = O.run(p, threads=THREADS)
    assert np.array_equal(pv, o["prevalence"]) and np.array_equal(tr, o["transitions"])
    assert np.array_equal(to, o["totals"]) and np.array_equal(u, o["u"])
    assert np.array_equal(v.view(np.int64), o["v"].view(np.int64))
