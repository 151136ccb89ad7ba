"""The oracle against laws fixed by the paper and the mathematics (CPU only)."""
import numpy as np
import pytest

from farmnet import ENTER, EXIT, EXTERNAL, synth
from oracle import oracle as O

from . import laws


def test_sis_decay_is_binomial_thinning():
    ok, pv = laws.check_sis_decay()
    assert ok, pv


def test_flip_model_state_law():
    ok, pv = laws.check_flip_state()
    assert ok, pv


def test_flip_model_transitions_are_poisson_2000():
    ok, pv = laws.check_flip_clock()
    assert ok, pv


def test_three_class_flip_transitions_are_poisson():
    # the six-compartment chain the critical-path probe times
    ok, pv = laws.check_flip_classes()
    assert ok, pv


def test_longest_chain_of_a_day():
    ok, pv = laws.check_max_transitions()
    assert ok, pv


def test_two_node_exact_master_equation():
    ok, pv = laws.check_two_node()
    assert ok, pv


def test_two_node_distinguishes_phi_reading():
    """The same samples reject the reading that feeds phi from the pre-event state,
    so the exact test above really pins the order SSA -> events -> phi."""
    p, snap = laws.two_node_samples()
    pv = laws.two_node_pvalues(snap, laws.two_node_exact_pre(p))
    assert min(pv) < 1e-8, pv


def test_two_node_pre_event_variant():
    """The variant that feeds phi from the state before the events (eq:numstep5
    as written) follows its own exact law, and the same samples reject the
    default reading's law."""
    p, snap = laws.two_node_samples(pre=True)
    pv = laws.two_node_pvalues(snap, laws.two_node_exact_pre(p))
    assert min(pv) > laws.P_MIN, pv
    pv = laws.two_node_pvalues(snap, laws.two_node_exact(p))
    assert min(pv) < 1e-8, pv


def test_mass_action_sir_master_equation():
    """Bimolecular S + I -> 2I (rate c S I) with recovery: the (S, I) law after
    one and two days is the exact matrix exponential of the chain's generator;
    the same samples reject a rate that ignores the second reactant."""
    kw = dict(S0=6, I0=2, c_inf=0.3, c_rec=0.5)
    p, snap = laws.sir_samples(**kw)
    pv = laws.sir_pvalues(snap, **kw)
    assert min(pv) > laws.P_MIN, pv
    pv = laws.sir_pvalues(snap, bimolecular=False, **kw)
    assert min(pv) < 1e-8, pv
    # conservation: S + I + R stays 8
    assert (snap.sum(axis=2) == 8).all()


@pytest.mark.parametrize("day0", [0, 50, 300])
def test_phi_closed_form(day0):
    ok, worst = laws.check_phi_closed_form(day0=day0)
    assert ok, worst


def test_two_node_shifted_external_transfers():
    """External transfers whose shift column moves the drawn animals into
    other compartments at the destination (Sec. 3.2): the exact master
    equation of the two-node system, and the same samples reject the law in
    which the shift is ignored."""
    import dataclasses
    ok, pv = laws.check_two_node_shifted()
    assert ok, pv
    p, snap = laws.two_node_shifted_samples()
    unshifted = dataclasses.replace(p, ev_shift=np.full_like(p.ev_shift, -1))
    pv = laws.two_node_pvalues(snap, laws.two_node_exact(unshifted))
    assert min(pv) < 1e-8, pv


def test_prevalence_is_binomial_in_pure_recovery():
    ok, pv = laws.check_prevalence_law()
    assert ok, pv


def test_prevalence_is_taken_after_the_events():
    # rates zero; select column 2 = {I}: node 0 loses its two infected, node 1
    # sends its one infected to node 2 (every draw forced), so after day 0's
    # events only node 2 holds an infected animal
    m = synth.sis_model()
    u0 = [[0, 2], [3, 1], [5, 0]]
    ev = [(0, EXIT, 0, -1, 2, 1, -1), (0, EXTERNAL, 1, 2, 1, 2, -1)]
    p = synth.events_only(u0, ev, n_days=2)
    p.E = np.concatenate([m["E"], [[0], [1]]], axis=1).astype(np.int32)
    r = O.run(p)
    assert r["prevalence"][:, 0].tolist() == [1, 1]
    assert r["u"][0].tolist() == [[0, 0], [3, 0], [5, 1]]


def test_hypergeometric_removal():
    ok, pv = laws.check_hypergeometric()
    assert ok, pv


def test_multivariate_walk():
    ok, pv = laws.check_multivariate_walk()
    assert ok, pv


def test_class_totals_follow_the_events():
    ok, diff = laws.check_conservation()
    assert ok, diff


def test_single_compartment_events_are_deterministic():
    # node 0 holds only susceptibles: every removal is forced (Sec. 3.3)
    u0 = [[5, 0], [0, 0], [0, 0]]
    ev = [(0, EXTERNAL, 0, 1, 3, 1, -1), (0, EXTERNAL, 1, 2, 3, 1, -1), (1, ENTER, 2, -1, 4, 0, -1),
          (1, EXIT, 2, -1, 2, 1, -1)]
    p = synth.events_only(u0, ev, n_days=2)
    for seed in (1, 2, 3):
        p.seed = seed
        r = O.run(p)
        assert r["u"][0].tolist() == [[2, 0], [0, 0], [5, 0]]


def test_events_apply_in_list_order():
    u0 = [[5, 0], [0, 0], [0, 0]]
    ev = [(0, EXTERNAL, 1, 2, 3, 1, -1), (0, EXTERNAL, 0, 1, 3, 1, -1)]
    p = synth.events_only(u0, ev, n_days=1)
    r = O.run(p, raise_on_error=False)
    assert r["rc"] == -4 and r["err_event"] == 0 and r["err_day"] == 0


def test_infeasible_reports_smallest_event_and_replicate():
    # select column 2 = {I}: whether 3 infected can leave depends on the SSA
    m = synth.sis_model(upsilon=0.5, gamma=0.5)
    E = np.concatenate([m["E"], [[0], [1]]], axis=1)
    n = 40
    u0 = np.tile([[3, 3]], (n, 1))
    ev = [(1, EXIT, np.arange(n), -1, 3, 2, -1)]
    p = synth.events_only(u0, ev, n_days=2, n_rep=8)
    p.E = E.astype(np.int32)
    p.coef[:] = [0.5, 0.5]
    p.uses_phi[:] = 0
    r = O.run(p, raise_on_error=False)
    assert r["rc"] == -4
    # recompute per replicate which events were infeasible, from the state before day 1's events
    per_rep = []
    for rep in range(8):
        q = synth.events_only(u0, ev, n_days=2)
        q.E = p.E; q.coef[:] = p.coef[0]; q.uses_phi[:] = 0
        q.replicate_id = np.array([rep], np.uint32)
        s = O.run(q, d_begin=0, d_end=1)
        rr = O.run(q, d_begin=1, d_end=2, u=s["u"], v=s["v"], raise_on_error=False)
        if rr["rc"] == -4:
            per_rep.append((rr["err_event"], rep))
    assert per_rep and (r["err_event"], r["err_rep"]) == min(per_rep)


def test_threads_are_bit_identical():
    p = synth.config1()
    a = O.run(p, threads=1)
    b = O.run(p, threads=4)
    for k in ("u", "v", "prevalence", "transitions", "totals"):
        assert np.array_equal(a[k], b[k]), k


def test_resume_is_bit_identical():
    p = synth.config1()
    p.record_days = np.array([10, 200, 364], np.int32)
    full = O.run(p)
    a = O.run(p, d_begin=0, d_end=137)
    b = O.run(p, d_begin=137, d_end=365, u=a["u"], v=a["v"])
    assert np.array_equal(full["u"], b["u"]) and np.array_equal(full["v"], b["v"])
    assert np.array_equal(full["prevalence"], np.r_[a["prevalence"], b["prevalence"]])
    assert np.array_equal(full["snap_u"], np.r_[a["snap_u"], b["snap_u"]])


def test_replicates_are_independent_streams():
    p = synth.config1().with_replicates(3, replicate_id=np.array([5, 9, 5], np.uint32))
    r = O.run(p)
    assert np.array_equal(r["u"][0], r["u"][2]) and not np.array_equal(r["u"][0], r["u"][1])
    one = O.run(synth.config1().with_replicates(1, replicate_id=np.array([9], np.uint32)))
    assert np.array_equal(one["u"][0], r["u"][1])
