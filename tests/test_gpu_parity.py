"""GPU path against the oracle, element by element, on seeded inputs: every
compartment count, daily record and snapshot bit-exact, phi within 1e-12
relative (and in practice bit-identical). Calls go through the C ABI."""
import os

import numpy as np
import pytest

from farmnet import ENTER, EXIT, EXTERNAL, INTERNAL, synth
from oracle import oracle as O
import paper_1502_02908_amd as P

from .gpu_common import assert_parity, gpu_run, say

pytestmark = pytest.mark.gpu


def both(p, **kw):
    say(f"[parity] {p.name} Nn={p.n_nodes} R={p.n_rep} D={p.n_days} events={p.n_events} {kw}")
    g = gpu_run(p, **kw)
    o = O.run(p, threads=min(16, os.cpu_count() or 1))
    return g, o


def test_config1_full():
    p = synth.config1()
    p.record_days = np.array([0, 1, 90, 91, 182, 364], np.int32)
    g, o = both(p)
    assert_parity(g, o)
    assert o["transitions"].sum() > 1000


@pytest.mark.parametrize("launch", [P.LAUNCH_KERNELS, P.LAUNCH_PERSISTENT])
def test_sise3_small_network(launch):
    p = synth.sise3_network(n_nodes=3000, n_days=120, seed=5, u=10.0, age_days=(15, 40))
    p.record_days = np.array([7, 60, 119], np.int32)
    g, o = both(p, launch=launch)
    assert_parity(g, o)
    assert o["transitions"].sum() > 10000


def test_serial_events_equal_levels():
    p = synth.sise3_network(n_nodes=500, n_days=60, seed=6, age_days=(10, 30),
                            e1_per_node_day=0.4, e2_per_node_day=0.1)
    a = gpu_run(p, events_mode=P.EVENTS_LEVELS)
    b = gpu_run(p, events_mode=P.EVENTS_SERIAL)
    for k in ("u", "v", "prevalence", "transitions", "totals"):
        assert np.array_equal(a[k], b[k]), k
    assert a["levels"][0] < b["levels"][0]
    assert_parity(a, O.run(p))


def test_replicates_with_own_parameters():
    base = synth.sise3_network(n_nodes=700, n_days=90, seed=8, age_days=(10, 30))
    coef, alpha, beta = synth.prior_draws(5, seed=4)
    p = base.with_replicates(5, coef=coef * 5, alpha=alpha, beta=beta,
                             replicate_id=np.array([3, 1, 4, 1, 5], np.uint32))
    p.record_days = np.array([10, 89], np.int32)
    g, o = both(p)
    assert_parity(g, o)


@pytest.mark.parametrize("launch", [P.LAUNCH_KERNELS, P.LAUNCH_PERSISTENT])
def test_many_replicates_ragged(launch):
    p = synth.config1().truncated(40).with_replicates(67)
    g, o = both(p, launch=launch)
    assert_parity(g, o)


def test_flip_model_heavy_ssa():
    # the paper's synthetic benchmark model: ~2000 transitions per node-day
    p = synth.flip_model(n_nodes=333, n_days=3)
    g, o = both(p)
    assert_parity(g, o)
    assert o["transitions"].sum() > 1_900_000


def test_two_node_replicates():
    from .laws import TWO_NODE_KW
    p = synth.two_node(**TWO_NODE_KW).with_replicates(4099)
    p.record_days = np.array([0, 1, 2], np.int32)
    g, o = both(p)
    assert_parity(g, o)


def test_phi_closed_form_system():
    p = synth.constant_infection(n_days=400, day0=50)
    p.record_days = np.arange(400, dtype=np.int32)
    g, o = both(p)
    assert_parity(g, o)


def test_chunked_runs_and_checkpoint():
    p = synth.config1()
    p.record_days = np.array([3, 100, 250, 364], np.int32)
    full = gpu_run(p)
    chunked = gpu_run(p, chunks=[1, 99, 165, 100])
    for k in ("u", "v", "prevalence", "transitions", "totals", "snap_u", "snap_v"):
        assert np.array_equal(full[k], chunked[k]), k
    # save at day 137, restore into a fresh handle, finish
    with P.Simulator(p) as a:
        a.run(137)
        u, v, day = a.get_state()
    with P.Simulator(p) as b:
        b.set_state(u, v, day)
        b.run(0)
        u2, v2, day2 = b.get_state()
        tb = b.trajectory()
    assert day == 137 and day2 == 365
    assert np.array_equal(u2, full["u"]) and np.array_equal(v2, full["v"])
    assert np.array_equal(tb["prevalence"][137:], full["prevalence"][137:])


def test_empty_and_degenerate_inputs():
    # no events at all, a single node, zero-day run
    p = synth.sis_decay(n_nodes=1, I0=7, gamma=0.9, n_days=5)
    g, o = both(p)
    assert_parity(g, o)
    p0 = synth.config1().truncated(10)
    with P.Simulator(p0) as s:
        s.run(3)
        s.run(0)
        with pytest.raises(P.SimError):
            s.run(1)
        u, v, d = s.get_state()
        assert d == 10


def test_deterministic_events_and_order():
    u0 = [[5, 0], [0, 0], [0, 0]]
    ev = [(0, EXTERNAL, 0, 1, 3, 1, -1), (0, EXTERNAL, 1, 2, 3, 1, -1), (1, ENTER, 2, -1, 4, 0, -1),
          (1, EXIT, 2, -1, 2, 1, -1)]
    p = synth.events_only(u0, ev, n_days=2)
    g = gpu_run(p)
    assert g["u"][0].tolist() == [[2, 0], [0, 0], [5, 0]]


def test_event_levels_in_lds_take_every_selection_and_size():
    # events drawn after an addition at their node sit past level 1, so they
    # run in the day's LDS levels: selections of one, two and all six
    # compartments, moves of up to twelve animals (past the six draws computed
    # ahead), shifts on internal and external transfers, and runs of one
    # node's exit, internal transfer and entry; all against the oracle
    rng = np.random.default_rng(41)
    n_nodes = 64
    u0 = rng.integers(100, 300, size=(n_nodes, 6))
    plan = [  # external (select, shift, n), exit (select, n), internal n, entry n
        ((1, 0, 3), (4, 2), 7, 1),
        ((2, 1, 9), (1, 8), 3, 4),
        ((4, -1, 12), (2, 11), 1, 20),
        ((3, -1, 5), (3, 4), 10, 2),
    ]
    ev = []
    for d in range(3):
        for i in range(0, n_nodes, 2):
            (sel_e, sh_e, n_e), (sel_x, n_x), n_i, n_en = plan[(i // 2) % 4]
            src = (i + 1 + 2 * d) % n_nodes
            ev += [(d, EXTERNAL, src, i, n_e, sel_e, sh_e), (d, EXIT, i, -1, n_x, sel_x, -1),
                   (d, INTERNAL, i, -1, n_i, 1, 0), (d, ENTER, i, -1, n_en, 0, -1)]
    p = synth.events_only(u0, ev, n_days=3, model="sise3")
    E = np.concatenate([p.E, np.ones((6, 1), np.int32)], axis=1)  # select 4: every compartment
    p.E = np.ascontiguousarray(E, np.int32)
    g, o = both(p)
    assert_parity(g, o)
    assert g["levels"] == (6, 2)  # each day: the external transfers, then the runs


def test_infeasible_event_reports_smallest_index():
    u0 = [[5, 0], [0, 0], [0, 0]]
    ev = [(0, EXTERNAL, 1, 2, 3, 1, -1), (0, EXTERNAL, 0, 1, 3, 1, -1), (0, EXIT, 2, -1, 9, 1, -1)]
    p = synth.events_only(u0, ev, n_days=2)
    o = O.run(p, raise_on_error=False)
    assert o["rc"] == -4
    with P.Simulator(p) as s:
        s.run(0)
        with pytest.raises(P.SimError) as e:
            s.sync()
        assert e.value.code == -4
        assert f"infeasible event {o['err_event']} (replicate {o['err_rep']})" in str(e.value)


def test_infeasible_depends_on_replicate():
    m = synth.sis_model(upsilon=0.5, gamma=0.5)
    E = np.concatenate([m["E"], [[0], [1]]], axis=1)
    n = 40
    u0 = np.tile([[3, 3]], (n, 1))
    ev = [(1, EXIT, np.arange(n), -1, 3, 2, -1)]
    p = synth.events_only(u0, ev, n_days=2, n_rep=8)
    p.E = E.astype(np.int32)
    p.coef[:] = [0.5, 0.5]
    p.uses_phi[:] = 0
    o = O.run(p, raise_on_error=False)
    assert o["rc"] == -4
    with P.Simulator(p) as s:
        s.run(0)
        with pytest.raises(P.SimError) as e:
            s.sync()
        assert f"infeasible event {o['err_event']} (replicate {o['err_rep']})" in str(e.value)


@pytest.mark.parametrize("launch", [P.LAUNCH_KERNELS, P.LAUNCH_PERSISTENT])
def test_config2_full_37k_nodes_1461_days(launch):
    p = synth.config2()
    p.record_days = np.array([0, 400, 1000, 1460], np.int32)
    g, o = both(p, launch=launch)
    assert_parity(g, o)
    n_lv, mx = g["levels"]
    say(f"[parity] config2 levels total={n_lv} max/day={mx} transitions={o['transitions'].sum()}")


@pytest.mark.parametrize("heavy_per_wave", [1, 4, 5, 64])
def test_heavy_chains_per_wavefront(heavy_per_wave):
    # flip model (S<->I at rate 1): herds of 2000 run ~2000 transitions a day,
    # herds of 2 almost none; the node order deals the big herds out across
    # wavefronts, so each of the 10 wavefronts gets heavy_per_wave of them
    n = 640
    p = synth.flip_model(n_nodes=n, n_days=2)
    big = np.zeros(n, bool)
    big[np.random.default_rng(1).choice(n, 10 * heavy_per_wave, replace=False)] = True
    p.u0[~big] = [1, 1]
    p.record_days = np.array([0, 1], np.int32)
    g, o = both(p)
    assert_parity(g, o)
    assert o["transitions"].sum() > 10 * heavy_per_wave * 3000


def sir_network(n_days=60, waning=0.05):
    """S -> I (upsilon*phi*S), I -> R (gamma*I), R -> S (waning*R): a model
    outside the paired S<->I form, so the general stoichiometry path runs."""
    base = synth.sis_network(n_nodes=800, n_days=n_days, seed=31, p_exit=0.01, p_enter=0.01, p_ext=0.005)
    S = np.array([[-1, 0, 1], [1, -1, 0], [0, 1, -1]], np.int32)
    u0 = np.zeros((base.n_nodes, 3), np.int32)
    u0[:, :2] = base.u0
    u0[::7, 1] += 5
    E = np.array([[1, 1], [0, 1], [0, 1]], np.int32)
    import dataclasses
    return dataclasses.replace(
        base, n_comp=3, n_trans=3, u0=u0, S=S, reactant=np.array([0, 1, 2], np.int32),
        uses_phi=np.array([1, 0, 0], np.int32), coef=np.array([[0.3, 0.2, waning]]),
        phi_I_mask=0b010, phi_N_mask=0b111, E=E, N=np.zeros((3, 0), np.int32), name="sir")


@pytest.mark.parametrize("launch", [P.LAUNCH_KERNELS, P.LAUNCH_PERSISTENT])
def test_general_stoichiometry_sir(launch):
    p = sir_network()
    p.record_days = np.array([5, 59], np.int32)
    g, o = both(p, launch=launch)
    assert_parity(g, o)
    assert o["transitions"].sum() > 5000


def test_config3_full_1m_nodes_1461_days():
    # the full-size scale-up network: every count and record against the oracle
    p = synth.config3()
    p.record_days = np.array([730, 1460], np.int32)
    g, o = both(p)
    assert_parity(g, o)
    say(f"[parity] config3 transitions={o['transitions'].sum()} levels={g['levels']}")


# --- method variants ----------------------------------------------------------

@pytest.mark.parametrize("launch", [P.LAUNCH_KERNELS, P.LAUNCH_PERSISTENT])
def test_phi_from_pre_event_state(launch):
    # eq:numstep5 as written: phi fed by the state after the SSA, before the events
    import dataclasses
    p = dataclasses.replace(synth.sise3_network(n_nodes=2000, n_days=90, seed=41, u=10.0, age_days=(10, 30)),
                            phi_pre_events=1)
    p.record_days = np.array([5, 89], np.int32)
    g, o = both(p, launch=launch)
    assert_parity(g, o)
    post = O.run(dataclasses.replace(p, phi_pre_events=0), threads=8)
    assert not np.array_equal(post["v"], o["v"])


def test_phi_from_pre_event_state_replicate_tiles():
    import dataclasses
    base = dataclasses.replace(synth.sise3_network(n_nodes=900, n_days=60, seed=42, age_days=(10, 30)),
                               phi_pre_events=1)
    coef, alpha, beta = synth.prior_draws(70, seed=43)
    p = base.with_replicates(70, coef=coef, alpha=alpha, beta=beta)
    g, o = both(p)
    assert_parity(g, o)


@pytest.mark.parametrize("launch", [P.LAUNCH_KERNELS, P.LAUNCH_PERSISTENT])
def test_mass_action_sir(launch):
    # S + I -> 2I at rate c S I (the bimolecular rate of the SIR example), I -> R, R -> S
    import dataclasses
    p = dataclasses.replace(sir_network(n_days=50), uses_phi=np.zeros(3, np.int32),
                            coef=np.array([[0.004, 0.2, 0.05]]), reactant2=np.array([1, -1, -1], np.int32))
    p.record_days = np.array([3, 49], np.int32)
    g, o = both(p, launch=launch)
    assert_parity(g, o)
    assert o["transitions"].sum() > 5000


@pytest.mark.parametrize("density", [1.0, 3.0])
def test_private_tasks_around_lds_capacity(density):
    # the day kernel applies a unit's private tasks in LDS when the unit-day
    # has at most 256 private events and on global memory otherwise; 512 nodes
    # (two units) at about one single-node event per node-day put unit-days on
    # both sides of that bound, three per node-day puts all of them past it
    p = synth.sise3_network(n_nodes=512, n_days=60, seed=31, age_days=(10, 30), e1_per_node_day=density)
    p.record_days = np.array([0, 30, 59], np.int32)
    g, o = both(p)
    assert_parity(g, o)
    assert o["transitions"].sum() > 0


@pytest.mark.parametrize("launch", [P.LAUNCH_KERNELS, P.LAUNCH_PERSISTENT])
def test_group_walk_of_very_long_chains(launch):
    # the paper's synthetic model (Sec. 4.2) on 8200 nodes, four of them with
    # 6k to 40k transitions expected per day: with per-day launches their
    # chains are walked by all four wavefronts of a workgroup (256 attempts per
    # round) while thousands of attempts remain, then by one wavefront
    p = synth.flip_model(n_nodes=8200, S0=5, I0=5, n_days=4)
    for node, half in ((7, 3000), (100, 6000), (5000, 10000), (8199, 20000)):
        p.u0[node] = (half, half)
    p.record_days = np.array([0, 3], np.int32)
    g, o = both(p, launch=launch)
    assert_parity(g, o)
    assert o["transitions"].sum() > 4 * 78000


def test_group_units_on_a_farm_network():
    # from 8192 nodes up, the four largest herds get a workgroup each (the
    # workgroup walk when their chains are long, one wavefront otherwise);
    # regions check the records of those units
    p = synth.sise3_network(n_nodes=9000, n_days=150, seed=32, u=10.0, age_days=(20, 60))
    rng = np.random.default_rng(3)
    p.n_regions = 21
    p.region = rng.integers(-1, 21, p.n_nodes).astype(np.int32)
    p.record_days = np.array([0, 75, 149], np.int32)
    g, o = both(p)
    assert_parity(g, o)
    assert np.array_equal(g["regional"], o["regional"])
    assert o["transitions"].sum() > 100000
