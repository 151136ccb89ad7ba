"""The C-ABI library on the CPU: it loads, exports every symbol the header
declares, rejects invalid problems before touching a device, and its
dependency pass over the events has the properties the event semantics need.
No compute is launched here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1502_02908_amd as P
from paper_1502_02908_amd import sim as S
from farmnet import ENTER, EXIT, EXTERNAL, INTERNAL, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "episim.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = P.lib()
    names = header_functions()
    assert len(names) >= 10, names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(S.SIGNATURES), set(names) ^ set(S.SIGNATURES)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(S, "_lib", None)
    monkeypatch.setattr(S, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        S.lib()


def _create_error(p):
    s, keep = S._marshal(p)
    h = C.c_void_p()
    rc = P.lib().sim_create(C.byref(s), None, C.byref(h))
    return rc, P.lib().sim_last_error(None).decode()


def _base():
    return synth.config1().truncated(20)


BAD = {
    "negative count": lambda p: p.u0.__setitem__((3, 0), -1),
    "unsorted days": lambda p: p.ev_day.__setitem__(slice(0, 2), [5, 1]),
    "node out of range": lambda p: p.ev_node.__setitem__(0, p.n_nodes),
    "dest out of range": lambda p: p.ev_dest.__setitem__(np.flatnonzero(p.ev_kind == EXTERNAL)[0], -1),
    "unknown kind": lambda p: p.ev_kind.__setitem__(0, 7),
    "enter selects two compartments": lambda p: p.ev_select.__setitem__(np.flatnonzero(p.ev_kind == ENTER)[0], 1),
    "reactant not decremented": lambda p: p.S.__setitem__((0, 0), 0),
    "other compartment decremented": lambda p: p.S.__setitem__((1, 0), -1),
    "negative rate": lambda p: p.coef.__setitem__((0, 1), -0.5),
    "beta above one": lambda p: p.beta.__setitem__((0, 2), 1.5),
    "mask beyond compartments": lambda p: setattr(p, "phi_I_mask", 0b100),
    "select out of range": lambda p: p.ev_select.__setitem__(0, 9),
    "shift out of range": lambda p: p.ev_shift.__setitem__(0, 3),
    "day past horizon": lambda p: p.ev_day.__setitem__(-1, p.n_days),
    "negative n": lambda p: p.ev_n.__setitem__(0, -2),
    "record days not ascending": lambda p: setattr(p, "record_days", np.array([5, 5], np.int32)),
    "region out of range": lambda p: (setattr(p, "n_regions", 3),
                                      setattr(p, "region", np.full(p.n_nodes, 3, np.int32))),
    "region below -1": lambda p: (setattr(p, "n_regions", 3),
                                  setattr(p, "region", np.full(p.n_nodes, -2, np.int32))),
    "too many regions": lambda p: (setattr(p, "n_regions", 4097),
                                   setattr(p, "region", np.zeros(p.n_nodes, np.int32))),
}


@pytest.mark.parametrize("name", sorted(BAD))
def test_invalid_problem_rejected_before_device(name):
    p = _base()
    BAD[name](p)
    rc, msg = _create_error(p)
    assert rc == S.SIM_EINVAL, (rc, msg)
    assert msg
    assert S.workspace_bytes(p) == 0


def test_shift_landing_outside_compartments_rejected():
    p = synth.sise3_network(n_nodes=50, n_days=30, seed=3, age_days=(5, 10), e1_per_node_day=0.5)
    i = np.flatnonzero(p.ev_kind == INTERNAL)[0]
    p.ev_select[i] = 3              # adults {S3, I3} ...
    p.ev_shift[i] = 0
    p.N[4, 0] = 2                   # ... with S3 shifted by +2: compartment 6 does not exist
    rc, msg = _create_error(p)
    assert rc == S.SIM_EINVAL and "shift" in msg


def test_long_event_lists_report_their_first_fault():
    # validation runs over ranges of events on host threads when the list is
    # long: the message still names the first faulting event, whichever
    # range holds it, and a list without faults passes
    p = synth.sise3_network(n_nodes=20000, n_days=1000, seed=5, age_days=(20, 60), e1_per_node_day=0.06)
    n = p.n_events
    assert n > 1 << 20
    assert S.workspace_bytes(p) > 0
    late, early = n - 7, n // 3 + 11
    p.ev_node[late] = p.n_nodes        # node out of range
    rc, msg = _create_error(p)
    assert rc == S.SIM_EINVAL and msg == f"event {late}: node out of range", msg
    p.ev_n[early] = -1                 # an earlier fault, in another range
    rc, msg = _create_error(p)
    assert rc == S.SIM_EINVAL and msg.startswith(f"event {early}: n must be in"), msg


def test_valid_problem_passes_validation():
    p = _base()
    assert S.workspace_bytes(p) > 0
    rc, msg = _create_error(p)
    assert rc in (S.SIM_OK, S.SIM_EDEVICE, S.SIM_ENOMEM), (rc, msg)


# --- the dependency pass ------------------------------------------------------

def touches(kind, node, dest):
    """(nodes drawn from, nodes added to) by one event."""
    if kind == ENTER:
        return {node}, set(), {node}
    if kind == EXTERNAL:
        return {node, dest}, {node}, {dest}
    return {node}, {node}, set()


def check_levels(day, kind, node, dest, level, task):
    """Tasks are single external transfers or maximal runs of one node's
    single-node events with no external transfer touching the node in
    between; a task's events share a level; events of different tasks that
    conflict keep list order across levels; and every task's level is as small
    as the rules allow (one more than the largest level it must follow)."""
    n = len(day)
    for d in np.unique(day):
        idx = np.flatnonzero(day == d)
        info = [touches(kind[i], node[i], dest[i] if kind[i] == EXTERNAL else -1) for i in idx]
        # task shape
        for t in np.unique(task[idx]):
            mine = idx[task[idx] == t]
            assert len(set(level[mine])) == 1
            if len(mine) > 1:
                assert (kind[mine] != EXTERNAL).all() and len(set(node[mine])) == 1
        # maximal runs: walk the events touching each node in list order
        last = {}
        for a, i in enumerate(idx):
            nodes, _, _ = info[a]
            for x in nodes:
                prev = last.get(x)
                if prev is not None:
                    both_local = kind[prev] != EXTERNAL and kind[i] != EXTERNAL
                    assert (task[prev] == task[i]) == both_local, (prev, i)
                last[x] = i
        # order and minimality
        need = {}
        for a in range(len(idx)):
            _, draw_a, add_a = info[a]
            for b in range(a):
                if task[idx[b]] == task[idx[a]]:
                    continue
                _, draw_b, add_b = info[b]
                if bool(draw_a & (draw_b | add_b)) or bool(add_a & draw_b):
                    assert level[idx[b]] < level[idx[a]]
                    need[task[idx[a]]] = max(need.get(task[idx[a]], 0), level[idx[b]])
        for a in range(len(idx)):
            assert level[idx[a]] == need.get(task[idx[a]], 0) + 1


def random_events(rng, n_nodes, n_events, n_days):
    day = np.sort(rng.integers(0, n_days, n_events))
    kind = rng.integers(0, 4, n_events)
    node = rng.integers(0, n_nodes, n_events)
    dest = rng.integers(0, n_nodes, n_events)
    dest[kind != EXTERNAL] = -1
    return day, kind, node, dest


@pytest.mark.parametrize("seed", range(6))
def test_levels_random_lists(seed):
    rng = np.random.default_rng(seed)
    n_nodes = [3, 5, 20, 50, 8, 2][seed]
    day, kind, node, dest = random_events(rng, n_nodes, 300, 4)
    level, task = P.plan_levels(day, kind, node, dest, n_nodes, tasks=True)
    check_levels(day, kind, node, dest, level, task)


def test_levels_hub_additions_share_a_level():
    # twenty moves into one hub from distinct sources: one level
    n = 20
    level = P.plan_levels(np.zeros(n), np.full(n, EXTERNAL), np.arange(1, n + 1), np.zeros(n), n + 1)
    assert (level == 1).all()
    # a draw from the hub in between splits them
    kind = np.r_[np.full(10, EXTERNAL), EXIT, np.full(10, EXTERNAL)]
    node = np.r_[np.arange(1, 11), 0, np.arange(11, 21)]
    dest = np.r_[np.zeros(10), -1, np.zeros(10)]
    level = P.plan_levels(np.zeros(21), kind, node, dest, 21)
    assert level.tolist() == [1] * 10 + [2] + [3] * 10


def test_levels_on_generated_network():
    p = synth.sise3_network(n_nodes=2000, n_days=60, seed=9)
    level, task = P.plan_levels(p.ev_day, p.ev_kind, p.ev_node, p.ev_dest, p.n_nodes, tasks=True)
    sub = p.ev_day < 3
    check_levels(p.ev_day[sub], p.ev_kind[sub], p.ev_node[sub], p.ev_dest[sub], level[sub], task[sub])
    assert level.max() < 20
    assert len(np.unique(task)) < len(task)


def test_long_lists_plan_each_day_as_alone():
    # days are independent in the dependency pass: a list long enough to be
    # planned in ranges of days on several host threads gets, day by day, the
    # levels of that day planned alone and its tasks offset by the tasks of
    # the days before; tasks stay numbered in order of their first event
    rng = np.random.default_rng(21)
    n_nodes, n_days = 20000, 37
    per_day = rng.integers(5000, 60000, n_days)
    day = np.repeat(np.arange(n_days), per_day)
    n = len(day)
    assert n > 1 << 20
    kind = rng.integers(0, 4, n)
    node = rng.integers(0, n_nodes, n)
    dest = np.where(kind == EXTERNAL, rng.integers(0, n_nodes, n), -1)
    level, task = P.plan_levels(day, kind, node, dest, n_nodes, tasks=True)
    first = np.unique(task, return_index=True)[1]
    assert np.array_equal(np.unique(task), np.arange(task.max() + 1)) and (np.diff(first) > 0).all()
    off = 0
    for d, (b, e) in enumerate(zip(np.r_[0, np.cumsum(per_day)[:-1]], np.cumsum(per_day))):
        lv, tk = P.plan_levels(day[b:e], kind[b:e], node[b:e], dest[b:e], n_nodes, tasks=True)
        assert np.array_equal(level[b:e], lv), d
        assert np.array_equal(task[b:e], tk + off), d
        off += tk.max() + 1


def test_single_node_runs_form_one_task():
    # node 0: enter, exit, internal, exit -> one task at level 1; a move out of
    # node 0 follows it; the next exit at node 0 starts a new task after the move
    kind = np.array([ENTER, EXIT, INTERNAL, EXIT, EXTERNAL, EXIT, ENTER])
    node = np.array([0, 0, 0, 0, 0, 0, 1])
    dest = np.array([-1, -1, -1, -1, 1, -1, -1])
    level, task = P.plan_levels(np.zeros(7), kind, node, dest, 2, tasks=True)
    assert level.tolist() == [1, 1, 1, 1, 2, 3, 1]
    assert task.tolist() == [0, 0, 0, 0, 1, 2, 3]
    # additions only, then a draw: the task moves past every earlier event at the node
    kind = np.array([EXTERNAL, EXTERNAL, ENTER, EXIT])
    node = np.array([1, 2, 0, 0])
    dest = np.array([0, 0, -1, -1])
    level, task = P.plan_levels(np.zeros(4), kind, node, dest, 3, tasks=True)
    assert level.tolist() == [1, 1, 2, 2] and task[2] == task[3]


def test_plan_levels_rejects_bad_input():
    with pytest.raises(S.SimError):
        P.plan_levels([1, 0], [EXIT, EXIT], [0, 0], [-1, -1], 2)
    with pytest.raises(S.SimError):
        P.plan_levels([0], [EXTERNAL], [0], [5], 2)


def test_workspace_covers_every_events_mode():
    p = synth.sise3_network(n_nodes=300, n_days=40, seed=4, age_days=(5, 15), e1_per_node_day=0.5)
    lv = S.workspace_bytes(p, events_mode=S.EVENTS_LEVELS)
    se = S.workspace_bytes(p, events_mode=S.EVENTS_SERIAL)
    assert 0 < lv < se


def test_batch_rejects_mixed_models():
    a = synth.config1().truncated(10)
    b = synth.sise3_network(n_nodes=50, n_days=10, seed=1)
    structs = [S._marshal(a), S._marshal(b)]
    arr = (C.POINTER(S.sim_problem) * 2)(*[C.pointer(s) for s, _ in structs])
    h = C.c_void_p()
    rc = P.lib().sim_create_batch(arr, 2, None, C.byref(h))
    assert rc == S.SIM_EINVAL
    assert "share" in P.lib().sim_last_error(None).decode()
    c = synth.config1().truncated(10)
    c.n_days = 12
    structs = [S._marshal(a), S._marshal(c)]
    arr = (C.POINTER(S.sim_problem) * 2)(*[C.pointer(s) for s, _ in structs])
    assert P.lib().sim_workspace_bytes_batch(arr, 2, None) == 0


def test_slot_handle_sizing_and_rejects():
    net = synth.sise3_network(n_nodes=300, n_days=40, seed=4, age_days=(5, 15))
    one, four = S.SlotHandle.workspace_bytes(net, 1), S.SlotHandle.workspace_bytes(net, 4)
    assert 0 < one < four
    # per slot: 64 lanes of state over the padded positions, records of every day
    per = (four - one) / 3
    assert per >= 64 * net.n_nodes * (net.n_comp * 4 + 8) + 64 * net.n_days * (4 + 8 + 8 * net.n_comp)
    assert S.SlotHandle.workspace_bytes(net, 0) == 0
    rec = synth.sise3_network(n_nodes=300, n_days=40, seed=4, age_days=(5, 15))
    rec.record_days = np.array([3], np.int32)
    assert S.SlotHandle.workspace_bytes(rec, 2) == 0
    s, keep = S._marshal(rec)
    h = C.c_void_p()
    assert P.lib().sim_slots_create(C.byref(s), 2, None, C.byref(h)) == S.SIM_EINVAL
    assert "snapshots" in P.lib().sim_last_error(None).decode()
    s, keep = S._marshal(net)
    assert P.lib().sim_slots_create(C.byref(s), 0, None, C.byref(h)) == S.SIM_EINVAL
    assert not h.value


def test_device_options_validated_before_device():
    p = _base()
    assert S.workspace_bytes(p) > 0
    assert S.workspace_bytes(p, group_herds=17) == 0
    assert S.workspace_bytes(p, small_level=-1) == 0
    for bad in (2, 12, 48, 1024):
        assert S.workspace_bytes(p, tile_nodes=bad) == 0
    for good in (4, 16, 32, 64, 256, 512):
        assert S.workspace_bytes(p, tile_nodes=good) > 0
    assert S.workspace_bytes(p, heavy_herds=257) == 0 and S.workspace_bytes(p, heavy_herds=256) > 0
    assert S.workspace_bytes(p, few_chains=65) == 0 and S.workspace_bytes(p, few_chains=-1) > 0
    assert S.workspace_bytes(p, group_min_attempts=-1) == 0 and S.workspace_bytes(p, group_min_attempts=100) > 0
    with pytest.raises(TypeError):
        S.workspace_bytes(p, tile_width=64)
    s, keep = S._marshal(p)
    for field, value in (("block", 128), ("group_herds", 17), ("small_level", -5), ("launch", 7)):
        o = S.sim_device_opts()
        setattr(o, field, value)
        h = C.c_void_p()
        assert P.lib().sim_create(C.byref(s), C.byref(o), C.byref(h)) == S.SIM_EINVAL, field
        assert P.lib().sim_last_error(None).decode()


def test_tuner_rejects_bad_windows_before_device():
    from paper_1502_02908_amd.tune import autotune
    p = _base()
    for kw in (dict(start_day=p.n_days), dict(start_day=-1), dict(start_day=5, window=0),
               dict(start_day=5, window=p.n_days)):
        with pytest.raises(ValueError):
            autotune(p, **kw)


def test_request_parts_go_to_the_busiest_column():
    from paper_1502_02908_amd.serve import pick_slot
    # 16-lane slots: four to a column of 64 lanes
    assert pick_slot({0, 1, 2, 3, 4, 5, 6, 7}, [], 4) == 0
    # slot 5 runs: its column (4-7) fills first
    assert pick_slot({0, 1, 2, 3, 4, 6, 7}, [5], 4) == 4
    # two columns busy: the one with more running slots wins, then the lowest
    assert pick_slot({1, 2, 3, 6, 7, 9}, [0, 4, 5, 8], 4) == 6
    assert pick_slot({1, 6, 9}, [0, 4, 8], 4) == 1
    # a request's parts in a row fill one column before opening another
    free, running = set(range(8)), []
    for _ in range(3):
        sl = pick_slot(free, running, 4)
        free.discard(sl)
        running.append(sl)
    assert sorted(running) == [0, 1, 2]
