"""Laws that pin the oracle: each check runs the oracle (or a variant build of
it) on a small seeded system whose answer the paper and the mathematics fix,
and returns (passed, statistic). The expected values never come from the
oracle itself: they come from matrix exponentials of the chain's generator,
binomial / hypergeometric / Poisson laws, mpmath closed forms, and integer
bookkeeping of the event list.
"""
from __future__ import annotations

import math
from collections import defaultdict
from fractions import Fraction

import mpmath as mp
import numpy as np
from scipy import linalg, stats

from farmnet import EXIT, ENTER, EXTERNAL, INTERNAL, synth
from oracle import oracle as O

P_MIN = 1e-4   # acceptance level of the goodness-of-fit tests (inputs are seeded)


def gof(observed_counts, probs, min_expected=5.0):
    """Pearson chi-square goodness of fit with sparse bins pooled. Returns p."""
    obs = np.asarray(observed_counts, float)
    p = np.asarray(probs, float)
    n = obs.sum()
    exp = n * p
    big = exp >= min_expected
    o = np.r_[obs[big], obs[~big].sum()]
    e = np.r_[exp[big], exp[~big].sum()]
    if e[-1] < min_expected:            # fold the pooled tail into the largest bin
        j = np.argmax(e[:-1])
        o[j] += o[-1]; e[j] += e[-1]
        o, e = o[:-1], e[:-1]
    stat = ((o - e) ** 2 / e).sum()
    return float(stats.chi2.sf(stat, len(e) - 1))


# ---------------------------------------------------------------------------
# SSA law: pure recovery is a binomial thinning (each infected animal recovers
# independently at rate gamma), so I(t) ~ Bin(I0, exp(-gamma t)).
# ---------------------------------------------------------------------------

def check_sis_decay(lib_path=None):
    p = synth.sis_decay(n_nodes=4000, I0=20, gamma=0.3, n_days=3)
    r = O.run(p, record_days=[0, 1, 2], lib_path=lib_path)
    pv = []
    for d in range(3):
        I = r["snap_u"][d, 0, :, 1]
        q = math.exp(-0.3 * (d + 1))
        pv.append(gof(np.bincount(I, minlength=21), stats.binom.pmf(np.arange(21), 20, q)))
    return min(pv) > P_MIN, min(pv)


# ---------------------------------------------------------------------------
# The paper's synthetic benchmark model (Sec. 4.2): S->I and I->S at rate 1 per
# individual with S = I = 1000. lambda = S + I = 2000 never changes, so the
# transitions of a node-day are Poisson(2000); each individual is a two-state
# chain, so I(t) = Bin(1000, (1+e^-2t)/2) + Bin(1000, (1-e^-2t)/2).
# ---------------------------------------------------------------------------

def _flip_pmf(t, n=1000):
    a = stats.binom.pmf(np.arange(n + 1), n, (1 + math.exp(-2 * t)) / 2)
    b = stats.binom.pmf(np.arange(n + 1), n, (1 - math.exp(-2 * t)) / 2)
    return np.convolve(a, b)


def check_flip_state(lib_path=None):
    p = synth.flip_model(n_nodes=3000, n_days=2)
    r = O.run(p, record_days=[0, 1], lib_path=lib_path)
    pv = []
    for d in range(2):
        I = r["snap_u"][d, 0, :, 1]
        pmf = _flip_pmf(d + 1)
        edges = np.arange(850, 1151, 10)
        cdf = np.cumsum(pmf)
        probs = np.diff(np.r_[0.0, cdf[edges[1:] - 1], 1.0])
        counts = np.histogram(I, bins=np.r_[-1, edges[1:] - 0.5, 3000])[0]
        pv.append(gof(counts, probs))
    return min(pv) > P_MIN, min(pv)


def check_flip_clock(lib_path=None):
    p = synth.flip_model(n_nodes=1, n_days=2).with_replicates(3000)
    r = O.run(p, lib_path=lib_path)
    k = r["transitions"].ravel()
    edges = np.arange(1850, 2151, 10)
    probs = np.diff(np.r_[0.0, stats.poisson.cdf(edges[1:] - 1, 2000), 1.0])
    counts = np.histogram(k, bins=np.r_[-1, edges[1:] - 0.5, 10**9])[0]
    pv = gof(counts, probs)
    return pv > P_MIN, pv


def check_flip_classes(lib_path=None, R=3000, each=333):
    """The same dynamics on the six SISe3 compartments (three classes, S_j <->
    I_j at rate 1 each): every class keeps S_j + I_j, so lambda = 6 * each
    never changes and a node-day fires Poisson(6 each) transitions; the three
    pairs of rates must all enter lambda and each draw must move an animal
    within its own class."""
    p = synth.flip_classes(n_nodes=1, S0=each, I0=each, n_days=2).with_replicates(R)
    r = O.run(p, lib_path=lib_path)
    lam = 6 * each
    k = r["transitions"].ravel()
    edges = np.arange(lam - 150, lam + 151, 10)
    probs = np.diff(np.r_[0.0, stats.poisson.cdf(edges[1:] - 1, lam), 1.0])
    counts = np.histogram(k, bins=np.r_[-1, edges[1:] - 0.5, 10**9])[0]
    pv = gof(counts, probs)
    u = r["u"].reshape(R, 6)
    kept = (u[:, 0::2] + u[:, 1::2] == 2 * each).all()
    return pv > P_MIN and kept, pv


def check_max_transitions(lib_path=None, n_nodes=20, R=2000, half=100):
    """The longest chain of a day (the most transitions of one node): in the
    synthetic model with S = I = half per node, lambda = 2 half never changes,
    so each node's transitions in a day are Poisson(2 half), independent over
    nodes and days, and their maximum over n nodes has cdf F(x)^n."""
    p = synth.flip_model(n_nodes=n_nodes, S0=half, I0=half, n_days=2).with_replicates(R)
    r = O.run(p, lib_path=lib_path)
    m = r["max_transitions"].ravel()
    x = np.arange(0, 6 * half)
    cdf_max = stats.poisson.cdf(x, 2 * half) ** n_nodes
    pmf = np.diff(np.r_[0.0, cdf_max])
    counts = np.bincount(np.minimum(m, len(x) - 1), minlength=len(x))[:len(x)]
    pv = gof(counts, pmf / pmf.sum())
    ok = pv > P_MIN and (r["max_transitions"] <= r["transitions"]).all()
    return ok, pv


# ---------------------------------------------------------------------------
# Exact master equation of a two-node system over whole days: the per-node
# chain over [d, d+1) with phi frozen (eq:numstep3) is exp(Q), the events are
# exact hypergeometric draws in list order (eq:numstep4), and phi follows the
# Euler step (eq:numstep5) from the post-event state (two_node_exact) or, for
# the alternative reading, from the pre-event state (two_node_exact_pre).
# ---------------------------------------------------------------------------

def _sis_day_matrix(n, inf_rate_per_s, gamma):
    Q = np.zeros((n + 1, n + 1))
    for I in range(n + 1):
        S = n - I
        a, b = inf_rate_per_s * S, gamma * I
        if I < n:
            Q[I, I + 1] = a
        if I > 0:
            Q[I, I - 1] = b
        Q[I, I] = -(a + b)
    return linalg.expm(Q)


def _hyper(S, I, n):
    """P(i infected among n drawn without replacement from S susceptible, I infected)."""
    tot = math.comb(S + I, n)
    return {i: math.comb(I, i) * math.comb(S, n - i) / tot
            for i in range(max(0, n - S), min(n, I) + 1)}


def _events_exact(dist, evs, N):
    """Push a distribution over ((S0, I0, S1, I1), phi) through one day's events
    in list order: removals are exact hypergeometric draws from {S, I}, and a
    moved animal of compartment c lands in c + N[c, shift] at the destination
    (or in c without a shift)."""
    for e in evs:
        _, kind, node, dest, n, sel, sh = map(int, e)
        land = [c + (int(N[c, sh]) if sh >= 0 else 0) for c in range(2)]
        new = defaultdict(float)
        for (x, phi), pr in dist.items():
            x = list(x)
            if kind == ENTER:
                x[2 * node] += n
                new[(tuple(x), phi)] += pr
                continue
            S, I = x[2 * node], x[2 * node + 1]
            for i, ph in _hyper(S, I, n).items():
                y = list(x)
                y[2 * node] -= n - i
                y[2 * node + 1] -= i
                if kind == EXTERNAL:
                    y[2 * dest + land[0]] += n - i
                    y[2 * dest + land[1]] += i
                new[(tuple(y), phi)] += pr * ph
        dist = new
    return dist


def _ssa_exact(dist, ups, gam, pre=None):
    """The stochastic step of one day per node (phi frozen): the row of exp(Q)
    of each node's (S, I) chain. With pre = (alpha, beta) the phi update from
    the post-SSA state follows (the pre-event reading)."""
    new = defaultdict(float)
    for (x, phi), pr in dist.items():
        rows = [_sis_day_matrix(x[2 * k] + x[2 * k + 1], ups * phi[k], gam)[x[2 * k + 1]] for k in range(2)]
        for I0n, p0 in enumerate(rows[0]):
            for I1n, p1 in enumerate(rows[1]):
                if p0 * p1 == 0.0:
                    continue
                n0, n1 = x[0] + x[1], x[2] + x[3]
                y = (n0 - I0n, I0n, n1 - I1n, I1n)
                nphi = phi
                if pre is not None:
                    alpha, beta = pre
                    nphi = tuple((1.0 - beta) * phi[k] +
                                 (alpha * y[2 * k + 1] / (y[2 * k] + y[2 * k + 1]) if y[2 * k] + y[2 * k + 1] else 0.0)
                                 for k in range(2))
                new[(y, nphi)] += pr * p0 * p1
    return new


def _marginal(dist):
    m = defaultdict(float)
    for (x, _), pr in dist.items():
        m[x] += pr
    return dict(m)


def two_node_exact(p):
    """Exact law of the two-node system day by day: SSA -> events -> phi update
    from the post-event state (Algorithm 1)."""
    ups, gam = p.coef[0]
    alpha, beta = p.alpha[0], p.beta[0]
    ev = list(zip(p.ev_day, p.ev_kind, p.ev_node, p.ev_dest, p.ev_n, p.ev_select, p.ev_shift))
    dist = {(tuple(map(int, p.u0.ravel())), tuple(map(float, p.v0))): 1.0}
    marg = []
    for d in range(p.n_days):
        dist = _ssa_exact(dist, ups, gam)
        dist = _events_exact(dist, [e for e in ev if e[0] == d], p.N)
        new = defaultdict(float)
        for (x, phi), pr in dist.items():
            nphi = []
            for k in range(2):
                S, I = x[2 * k], x[2 * k + 1]
                nphi.append((1.0 - beta[0]) * phi[k] + (alpha * I / (S + I) if S + I > 0 else 0.0))
            new[(x, tuple(nphi))] += pr
        dist = new
        marg.append(_marginal(dist))
    return marg


def two_node_exact_pre(p):
    """Alternative reading: phi from the pre-event (post-SSA) state."""
    ups, gam = p.coef[0]
    alpha, beta = p.alpha[0], p.beta[0]
    ev = list(zip(p.ev_day, p.ev_kind, p.ev_node, p.ev_dest, p.ev_n, p.ev_select, p.ev_shift))
    dist = {(tuple(map(int, p.u0.ravel())), tuple(map(float, p.v0))): 1.0}
    marg = []
    for d in range(p.n_days):
        dist = _ssa_exact(dist, ups, gam, pre=(alpha, beta[0]))
        dist = _events_exact(dist, [e for e in ev if e[0] == d], p.N)
        marg.append(_marginal(dist))
    return marg


TWO_NODE_KW = dict(n_days=3, upsilon=0.9, gamma=0.4, alpha=1.0, beta=(0.3, 0.3, 0.3, 0.3),
                   u0=((3, 1), (2, 0)), phi0=(1.6, 0.0))


def two_node_samples(R=200000, lib_path=None, pre=False):
    import dataclasses
    p = synth.two_node(**TWO_NODE_KW).with_replicates(R)
    if pre:
        p = dataclasses.replace(p, phi_pre_events=1)
    r = O.run(p, record_days=[0, 1, 2], lib_path=lib_path)
    return p, r["snap_u"]  # [day, R, 2, 2]


def two_node_pvalues(snap, marg):
    pv = []
    for d, m in enumerate(marg):
        keys = sorted(m)
        index = {k: i for i, k in enumerate(keys)}
        x = snap[d].reshape(snap.shape[1], 4)
        counts = np.zeros(len(keys) + 1)
        for row, c in zip(*np.unique(x, axis=0, return_counts=True)):
            counts[index.get(tuple(int(v) for v in row), len(keys))] += c
        probs = np.r_[[m[k] for k in keys], 0.0]
        if counts[-1] > 0:          # a state the exact law gives probability 0
            pv.append(0.0)
            continue
        pv.append(gof(counts[:-1], probs[:-1] / probs[:-1].sum()))
    return pv


# A shift column that exchanges S and I: an external transfer with it lands
# each moved susceptible as infected at the destination and each moved infected
# as susceptible. Physically odd, but it makes the destination's composition
# depend on exactly where each drawn compartment lands.
SWAP_SHIFT = np.array([[1], [-1]], np.int32)
TWO_NODE_SHIFTED_EVENTS = [(0, EXTERNAL, 0, 1, 2, 1, 0), (1, ENTER, 1, -1, 1, 0, -1),
                           (2, EXTERNAL, 1, 0, 1, 1, 0)]


def two_node_shifted_samples(R=200000, lib_path=None):
    import dataclasses
    p = dataclasses.replace(synth.two_node(events=TWO_NODE_SHIFTED_EVENTS, **TWO_NODE_KW), N=SWAP_SHIFT)
    p = p.with_replicates(R)
    r = O.run(p, record_days=[0, 1, 2], lib_path=lib_path)
    return p, r["snap_u"]


def check_two_node_shifted(lib_path=None, R=200000):
    """The two-node master equation with external transfers that carry a shift
    (Sec. 3.2, eq:event: the event's column moves the drawn individuals into
    other compartments at the destination)."""
    p, snap = two_node_shifted_samples(R, lib_path)
    pv = two_node_pvalues(snap, two_node_exact(p))
    return min(pv) > P_MIN, min(pv)


def check_two_node(lib_path=None, R=200000):
    p, snap = two_node_samples(R, lib_path)
    pv = two_node_pvalues(snap, two_node_exact(p))
    return min(pv) > P_MIN, min(pv)


# ---------------------------------------------------------------------------
# Daily prevalence (nodes with an infected individual after the day's events).
# In pure recovery (no infection, no events) each of a node's I0 infected
# animals has recovered by day t with probability 1 - e^{-gamma t}
# independently, so a node is still infected with probability
# 1 - (1 - e^{-gamma t})^I0, and the prevalence over n identical nodes is
# Binomial(n, that probability). The nodes also hold susceptibles, so
# counting the node size in place of the infected is seen.
# ---------------------------------------------------------------------------

def check_prevalence_law(lib_path=None, n_nodes=40, I0=3, S0=2, gamma=0.3, R=3000):
    p = synth.sis_decay(n_nodes=n_nodes, I0=I0, S0=S0, gamma=gamma, n_days=3).with_replicates(R)
    r = O.run(p, lib_path=lib_path)
    pv = []
    for d in range(3):
        q = 1.0 - (1.0 - math.exp(-gamma * (d + 1))) ** I0
        prev = r["prevalence"][d]
        pv.append(gof(np.bincount(prev, minlength=n_nodes + 1)[:n_nodes + 1],
                      stats.binom.pmf(np.arange(n_nodes + 1), n_nodes, q)))
    return min(pv) > P_MIN, min(pv)


# ---------------------------------------------------------------------------
# phi with I/N constant (all rates zero, no events): within a season beta is
# constant and phi_n = (1-beta)^n phi_0 + alpha c (1 - (1-beta)^n) / beta.
# ---------------------------------------------------------------------------

def season_table(path):
    rows = [tuple(map(int, l.split())) for l in open(path) if l.strip() and not l.startswith("#")]
    return dict(rows)


def paper_season(t):
    """Quarter of beta(t) from the inequalities printed in Sec. 4.1."""
    doy = t % 365
    return 0 if doy <= 91 else 1 if doy <= 182 else 2 if doy <= 273 else 3


def phi_closed_form(phi0, c, alpha, betas, day0, n_steps):
    """phi after each of n_steps Euler steps, segment by segment in mpmath."""
    mp.mp.dps = 40
    out = []
    phi = mp.mpf(phi0)
    seg_start_phi, seg_len, seg_q = phi, 0, paper_season(day0)
    for k in range(n_steps):
        q = paper_season(day0 + k)
        if q != seg_q:
            b = mp.mpf(betas[seg_q])
            a = (1 - b) ** seg_len
            seg_start_phi = a * seg_start_phi + mp.mpf(alpha) * c * (1 - a) / b
            seg_len, seg_q = 0, q
        seg_len += 1
        b = mp.mpf(betas[seg_q])
        a = (1 - b) ** seg_len
        out.append(a * seg_start_phi + mp.mpf(alpha) * c * (1 - a) / b)
    return out


def check_phi_closed_form(lib_path=None, day0=0, n_days=400):
    beta = (0.10, 0.12, 0.10, 0.08)
    p = synth.constant_infection(n_days=n_days, day0=day0, beta=beta, alpha=0.7)
    r = O.run(p, record_days=np.arange(n_days), lib_path=lib_path)
    worst = 0.0
    for i in range(p.n_nodes):
        S, I = p.u0[i]
        c = mp.mpf(int(I)) / (int(S) + int(I)) if S + I > 0 else mp.mpf(0)
        exact = phi_closed_form(p.v0[i], c, 0.7, [mp.mpf(b) for b in beta], day0, n_days)
        got = r["snap_v"][:, 0, i]
        for g, e in zip(got, exact):
            if e != 0:
                worst = max(worst, float(abs((mp.mpf(g) - e) / e)))
            elif g != 0:
                worst = max(worst, 1.0)
    return worst <= 1e-12, worst


# ---------------------------------------------------------------------------
# Events
# ---------------------------------------------------------------------------

def check_hypergeometric(lib_path=None, n_nodes=6000):
    """EXIT of 4 animals from (S, I) = (7, 5): the infected count removed is
    Hypergeometric(12, 5, 4)."""
    u0 = np.tile([[7, 5]], (n_nodes, 1))
    ev = [(0, EXIT, np.arange(n_nodes), -1, 4, 1, -1)]
    p = synth.events_only(u0, ev, n_days=1)
    r = O.run(p, lib_path=lib_path)
    removed_I = 5 - r["u"][0, :, 1]
    pmf = stats.hypergeom.pmf(np.arange(5), 12, 5, 4)
    pv = gof(np.bincount(removed_I, minlength=5)[:5], pmf)
    return pv > P_MIN and (r["u"] >= 0).all(), pv


def check_multivariate_walk(lib_path=None, n_nodes=6000):
    """EXIT of 3 from the selection {S1, S2, I2} holding (4, 5, 3), with 6
    animals in the unselected I1 between them: the composition is multivariate
    hypergeometric and I1 is never touched."""
    m = synth.sise3_model(coef=np.zeros(6))
    E = np.zeros((6, 1), np.int32)
    sel = [0, 2, 3]
    E[sel, 0] = 1
    u0 = np.zeros((n_nodes, 6), np.int64)
    u0[:, 0], u0[:, 1], u0[:, 2], u0[:, 3] = 4, 6, 5, 3
    z = np.zeros(n_nodes, np.int32)
    from farmnet import Problem
    m.update(E=E)
    p = Problem(n_nodes=n_nodes, n_rep=1, n_days=1, u0=u0, v0=np.zeros(n_nodes),
                ev_day=z, ev_kind=z + EXIT, ev_node=np.arange(n_nodes), ev_dest=z - 1, ev_n=z + 3,
                ev_select=z, ev_shift=z - 1, **m)
    r = O.run(p, lib_path=lib_path)
    taken = np.array([4, 5, 3]) - r["u"][0][:, sel]
    keys, counts = np.unique(taken, axis=0, return_counts=True)
    probs = [stats.multivariate_hypergeom.pmf(k, [4, 5, 3], 3) for k in keys]
    ok_support = (taken.sum(axis=1) == 3).all() and (taken >= 0).all() and (r["u"][0][:, 1] == 6).all()
    if not ok_support:
        return False, 0.0
    pv = gof(counts, np.array(probs) / np.sum(probs))
    return pv > P_MIN and abs(np.sum(probs) - 1.0) < 1e-9, pv


def class_totals_replay(p):
    """Per node and class, the deterministic animal count after all events:
    SSA transitions never move an animal between classes, so only the events
    change these totals (integer bookkeeping)."""
    if p.n_comp == 2:
        cls_of = np.array([0, 0])
    else:
        cls_of = np.array([0, 0, 1, 1, 2, 2])
    ncls = cls_of.max() + 1
    T = np.zeros((p.n_nodes, ncls), np.int64)
    np.add.at(T, (np.repeat(np.arange(p.n_nodes), p.n_comp), np.tile(cls_of, p.n_nodes)), p.u0.ravel())
    for d, kind, node, dest, n, sel, sh in zip(p.ev_day, p.ev_kind, p.ev_node, p.ev_dest, p.ev_n,
                                              p.ev_select, p.ev_shift):
        comps = np.flatnonzero(p.E[:, sel])
        c = cls_of[comps[0]]
        if kind == ENTER:
            T[node, c] += n
        elif kind == EXIT:
            T[node, c] -= n
        elif kind == INTERNAL:
            T[node, c] -= n
            T[node, cls_of[comps[0] + p.N[comps[0], sh]]] += n
        else:
            # an external transfer with a shift lands each animal of compartment
            # c in c + N[c, shift] at the destination (Sec. 3.2)
            T[node, c] -= n
            T[dest, cls_of[comps[0] + (p.N[comps[0], sh] if sh >= 0 else 0)]] += n
    return T, cls_of


def check_conservation(lib_path=None):
    p = synth.sise3_network(n_nodes=300, n_days=150, seed=21, u=10.0, age_days=(20, 60),
                            e1_per_node_day=0.6, e2_per_node_day=0.2, shifted_moves=0.5)
    assert (p.ev_shift[p.ev_kind == EXTERNAL] >= 0).sum() > 1000   # the law covers shifted moves
    want, cls_of = class_totals_replay(p)
    ok = True
    for seed in (1, 2):
        p.seed = seed
        r = O.run(p, lib_path=lib_path)
        got = np.zeros_like(want)
        for c in range(p.n_comp):
            got[:, cls_of[c]] += r["u"][0, :, c]
        ok = ok and (got == want).all() and (r["u"] >= 0).all() and r["transitions"].sum() > 300
    return ok, int(np.abs(got - want).sum())


# ---------------------------------------------------------------------------
# Mass-action (bimolecular) rates: the SIR example of Sec. 2.1, one node,
# S + I -> 2I at rate c_1 * S * I and I -> R at rate c_2 * I. Its master
# equation on the (S, I) lattice is small enough to solve exactly.
# ---------------------------------------------------------------------------

def sir_mass_action(S0=6, I0=2, c_inf=0.3, c_rec=0.5, n_days=2, R=1, second_reactant=True):
    from farmnet.problem import Problem
    none = np.zeros(0, np.int32)
    return Problem(n_nodes=1, n_comp=3, n_trans=2, n_rep=R, n_days=n_days,
                   u0=np.array([[S0, I0, 0]]), v0=np.zeros(1),
                   S=np.array([[-1, 0], [1, -1], [0, 1]]), reactant=np.array([0, 1]),
                   uses_phi=np.array([0, 0]), coef=np.tile([c_inf, c_rec], (R, 1)), alpha=np.zeros(R),
                   beta=np.zeros((R, 4)), phi_I_mask=0b010, phi_N_mask=0b111,
                   E=np.ones((3, 1), np.int32), N=np.zeros((3, 0), np.int32),
                   ev_day=none, ev_kind=none, ev_node=none, ev_dest=none, ev_n=none, ev_select=none,
                   ev_shift=none, seed=17, reactant2=np.array([1 if second_reactant else -1, -1]),
                   name="sir-mass-action")


def sir_exact(S0, I0, c_inf, c_rec, t, bimolecular=True):
    """P(S, I) at time t from the generator of the chain (exact matrix exponential)."""
    states = [(S, I) for S in range(S0 + 1) for I in range(S0 + I0 + 1 - S)]
    idx = {st: k for k, st in enumerate(states)}
    Q = np.zeros((len(states), len(states)))
    for (S, I), k in idx.items():
        a = c_inf * S * (I if bimolecular else 1)
        b = c_rec * I
        if S > 0 and a > 0:
            Q[k, idx[(S - 1, I + 1)]] += a
        if I > 0:
            Q[k, idx[(S, I - 1)]] += b
        Q[k, k] = -(a + b)
    row = linalg.expm(Q * t)[idx[(S0, I0)]]
    return {st: row[k] for st, k in idx.items()}


def sir_samples(R=200000, lib_path=None, **kw):
    p = sir_mass_action(R=R, **kw)
    r = O.run(p, record_days=list(range(p.n_days)), lib_path=lib_path)
    return p, r["snap_u"][:, :, 0, :]  # [day, R, c]


def sir_pvalues(snap, S0, I0, c_inf, c_rec, bimolecular=True):
    pv = []
    for d in range(snap.shape[0]):
        law = sir_exact(S0, I0, c_inf, c_rec, d + 1.0, bimolecular)
        keys = sorted(law)
        counts = defaultdict(int)
        for S, I, _ in snap[d]:
            counts[(int(S), int(I))] += 1
        obs = np.array([counts[k] for k in keys], float)
        pv.append(gof(obs, [law[k] for k in keys]))
    return pv
