"""Seeded synthetic farm networks standing in for the paper's workloads.

The paper's national-scale runs (Sec. 4.1) use the Swedish cattle register,
which is not available. These generators produce inputs with the paper's
shapes instead: node sizes with a heavy tail, an age-structured SIS model
(eq:vtectrans with the constants of Sec. 4.1), per-window counts of single-node
(E1: enter, exit, aging) and two-node (E2: movement) events close to the
3707 +/- 670 and 235 +/- 104 reported per window at 37221 nodes, and movement
destinations drawn from a power-law in-degree so that a few hubs receive most
moves. Every removal is feasible by construction: the per-class totals of a node
are deterministic (SSA transitions never change S_j + I_j), so the generator
tracks them exactly and drops an event that would ask for more animals than the
class holds.

This module produces inputs only. It contains no step of the simulation method
and is shared, as an input source, by the oracle's tests and the GPU path.
"""
from __future__ import annotations

import math

import numpy as np

from .problem import ENTER, EXIT, EXTERNAL, INTERNAL, Problem

LN2 = math.log(2.0)


# ---------------------------------------------------------------------------
# Model definitions (parameters only)
# ---------------------------------------------------------------------------

def sis_model(upsilon=0.02, gamma=0.1, alpha=1.0, beta=(0.10, 0.12, 0.10, 0.08)):
    """Compartments [S, I]; transitions [S->I at upsilon*phi*S, I->S at gamma*I]."""
    return dict(
        n_comp=2, n_trans=2,
        S=np.array([[-1, 1], [1, -1]], dtype=np.int32),
        reactant=np.array([0, 1], dtype=np.int32),
        uses_phi=np.array([1, 0], dtype=np.int32),
        coef=np.array([[upsilon, gamma]], dtype=np.float64),
        alpha=np.array([alpha], dtype=np.float64),
        beta=np.array([beta], dtype=np.float64),
        phi_I_mask=0b10, phi_N_mask=0b11,
        # select columns: 0 = {S} (births), 1 = {S, I} (any animal)
        E=np.array([[1, 1], [0, 1]], dtype=np.int32),
        N=np.zeros((2, 0), dtype=np.int32),
    )


def sise3_params(u=1.0, upsilon=(8e-3, 7e-3, 1e-3), delta=(28.0, 25.0, 22.0)):
    """Rate constants of eq:rate_s_to_i and eq:recovery_rates, in transition order."""
    coef = []
    for j in range(3):
        coef += [u * upsilon[j], u / delta[j]]
    return np.array(coef, dtype=np.float64)


PAPER_BETA = (LN2 / 14.0, LN2 / 26.0, LN2 / 20.0, LN2 / 12.0)


def sise3_model(u=1.0, alpha=1.0, beta=PAPER_BETA, coef=None):
    """Compartments [S1, I1, S2, I2, S3, I3] (calves, young stock, adults);
    transitions [S1->I1, I1->S1, S2->I2, I2->S2, S3->I3, I3->S3] (eq:vtectrans)."""
    S = np.zeros((6, 6), dtype=np.int32)
    for j in range(3):
        s, i = 2 * j, 2 * j + 1
        S[s, 2 * j], S[i, 2 * j] = -1, 1          # infection S_j -> I_j
        S[i, 2 * j + 1], S[s, 2 * j + 1] = -1, 1  # recovery I_j -> S_j
    E = np.zeros((6, 4), dtype=np.int32)
    E[0, 0] = 1                       # 0: {S1}: births
    for j in range(3):                # 1..3: whole age class j
        E[2 * j, 1 + j] = E[2 * j + 1, 1 + j] = 1
    N = np.zeros((6, 2), dtype=np.int32)
    N[0, 0] = N[1, 0] = 2             # 0: age 1 -> 2
    N[2, 1] = N[3, 1] = 2             # 1: age 2 -> 3
    return dict(
        n_comp=6, n_trans=6, S=S,
        reactant=np.arange(6, dtype=np.int32),
        uses_phi=np.array([1, 0, 1, 0, 1, 0], dtype=np.int32),
        coef=(sise3_params(u) if coef is None else np.asarray(coef, np.float64)).reshape(1, 6),
        alpha=np.array([alpha], dtype=np.float64),
        beta=np.array([beta], dtype=np.float64),
        phi_I_mask=0b101010, phi_N_mask=0b111111,
        E=E, N=N,
    )


def _events_to_arrays(blocks):
    """Concatenate per-day event blocks [(day, kind, node, dest, n, sel, shift), ...]."""
    if not blocks:
        z = np.zeros(0, np.int32)
        return dict(ev_day=z, ev_kind=z, ev_node=z, ev_dest=z, ev_n=z, ev_select=z, ev_shift=z)
    cols = list(zip(*blocks))
    names = ("ev_day", "ev_kind", "ev_node", "ev_dest", "ev_n", "ev_select", "ev_shift")
    return {k: np.concatenate(c).astype(np.int32) for k, c in zip(names, cols)}


def _block(day, kind, node, dest, n, sel, shift):
    m = len(node)
    f = lambda v: np.full(m, v, np.int32) if np.isscalar(v) else np.asarray(v, np.int32)
    return (f(day), f(kind), f(node), f(dest), f(n), f(sel), f(shift))


def _keep_prefix(keys, amounts, available):
    """Keep events (in list order) while the running demand of their key fits.

    keys: int array of group ids; amounts: demand of each event; available:
    callable mapping group ids to what the group holds. Returns a boolean mask.
    The running sum includes dropped events, which only makes the test stricter.
    """
    if len(keys) == 0:
        return np.zeros(0, bool)
    order = np.argsort(keys, kind="stable")
    k = keys[order]
    a = amounts[order].astype(np.int64)
    cs = np.cumsum(a)
    start = np.r_[0, np.flatnonzero(k[1:] != k[:-1]) + 1]
    grp_first = np.repeat(start, np.diff(np.r_[start, len(k)]))
    before = cs - a - np.where(grp_first > 0, cs[grp_first - 1], 0)
    ok_sorted = before + a <= available(k)
    ok = np.empty(len(keys), bool)
    ok[order] = ok_sorted
    return ok


def _lognormal_sizes(rng, n, median, sigma, lo, hi):
    return np.clip(np.rint(rng.lognormal(math.log(median), sigma, n)), lo, hi).astype(np.int64)


# ---------------------------------------------------------------------------
# Plain SIS network (1 age class)
# ---------------------------------------------------------------------------

def sis_network(n_nodes=1000, n_days=365, seed=1, median=50.0, sigma=1.0, max_size=5000,
                seeded_frac=0.01, seeded_I=0.10, p_exit=0.002, p_enter=0.002, p_ext=0.001,
                max_move=5, record_days=None, **model_kw):
    """SIS on a farm network: lognormal herd sizes, 1% of herds seeded with 10%
    infected, per node-day Bernoulli exits, births and movements of 1-5 animals
    to a uniformly drawn other herd."""
    rng = np.random.default_rng(seed)
    size = _lognormal_sizes(rng, n_nodes, median, sigma, 1, max_size)
    I0 = np.zeros(n_nodes, np.int64)
    seeded = rng.choice(n_nodes, max(1, int(round(seeded_frac * n_nodes))), replace=False)
    I0[seeded] = np.maximum(1, np.rint(seeded_I * size[seeded])).astype(np.int64)
    u0 = np.stack([size - I0, I0], axis=1)
    tot = size.copy()
    blocks = []
    for d in range(n_days):
        ent = np.flatnonzero(rng.random(n_nodes) < p_enter)
        tot[ent] += 1
        if len(ent):
            blocks.append(_block(d, ENTER, ent, -1, 1, 0, -1))
        ex = np.flatnonzero(rng.random(n_nodes) < p_exit)
        ex = ex[tot[ex] >= 1]
        tot[ex] -= 1
        if len(ex):
            blocks.append(_block(d, EXIT, ex, -1, 1, 1, -1))
        src = np.flatnonzero(rng.random(n_nodes) < p_ext)
        if len(src):
            src = rng.permutation(src)
            dst = rng.integers(0, n_nodes - 1, len(src))
            dst = dst + (dst >= src)                       # uniform over the other herds
            n = rng.integers(1, max_move + 1, len(src))
            ok = _keep_prefix(src, n, lambda k: tot[k])
            src, dst, n = src[ok], dst[ok], n[ok]
            np.subtract.at(tot, src, n)
            np.add.at(tot, dst, n)
            if len(src):
                blocks.append(_block(d, EXTERNAL, src, dst, n, 1, -1))
    model = sis_model(**model_kw)
    return Problem(n_nodes=n_nodes, n_rep=1, n_days=n_days, u0=u0, v0=np.zeros(n_nodes),
                   seed=seed, record_days=record_days, name=f"sis_{n_nodes}x{n_days}",
                   **model, **_events_to_arrays(blocks))


# ---------------------------------------------------------------------------
# SISe3 farm network (3 age classes, enter/exit/aging/movement events)
# ---------------------------------------------------------------------------

def sise3_network(n_nodes=37000, n_days=1461, seed=2, u=1.0, median=60.0, sigma=1.2,
                  max_size=10000, seeded_frac=0.01, seeded_I=0.10,
                  e1_per_node_day=3707.0 / 37221.0, e2_per_node_day=235.0 / 37221.0,
                  in_degree_exponent=2.1, age_days=(100, 400), record_days=None,
                  model_kw=None, shifted_moves=0.0):
    """Age-structured farm network. Births (ENTER into S1) and exits arrive at a
    per-animal rate chosen so that births, exits and the two aging transfers
    per birth (INTERNAL 1->2 after age_days[0], 2->3 after age_days[1]) add up
    to e1_per_node_day; movements (EXTERNAL, 1-5 animals of one age class) pick
    the source in proportion to herd size and the destination in proportion to
    a Pareto weight whose density falls as w^-in_degree_exponent. Within a
    day, single-node events come first (births, aging, exits, each by node),
    then movements in random order. With shifted_moves > 0, that fraction of
    the movements of calves and young stock carries the aging shift of its
    class, so the animals land one age class up at the destination (an
    external transfer whose column moves individuals between compartments,
    Sec. 3.2); 0 draws no extra numbers, so the default networks do not
    change."""
    rng = np.random.default_rng(seed)
    size = _lognormal_sizes(rng, n_nodes, median, sigma, 1, max_size)
    cls = np.zeros((n_nodes, 3), np.int64)
    cls[:, 0] = np.rint(0.2 * size)
    cls[:, 1] = np.rint(0.2 * size)
    cls[:, 2] = size - cls[:, 0] - cls[:, 1]
    neg = cls[:, 2] < 0
    cls[neg, 1] += cls[neg, 2]
    cls[neg, 2] = 0
    Icls = np.zeros_like(cls)
    seeded = rng.choice(n_nodes, max(1, int(round(seeded_frac * n_nodes))), replace=False)
    Icls[seeded] = np.ceil(seeded_I * cls[seeded]).astype(np.int64)
    u0 = np.zeros((n_nodes, 6), np.int64)
    u0[:, 0::2] = cls - Icls
    u0[:, 1::2] = Icls
    T = cls.copy()                                    # exact per-class totals

    # births, exits and two aging steps per birth share the E1 budget
    total = float(size.sum())
    rate_b = e1_per_node_day * n_nodes / 4.0 / total  # per animal and day
    size_cdf = np.cumsum(size + 1.0)
    size_cdf /= size_cdf[-1]
    w = (1.0 - rng.random(n_nodes)) ** (-1.0 / (in_degree_exponent - 1.0))
    dst_cdf = np.cumsum(w)
    dst_cdf /= dst_cdf[-1]
    def draw(cdf, m):
        # node whose cdf interval holds each uniform; the uniforms are searched
        # in ascending order (far fewer cache misses on a large cdf) and the
        # answers put back in draw order
        x = rng.random(m)
        o = np.argsort(x, kind="stable")
        out = np.empty(m, np.int64)
        out[o] = np.searchsorted(cdf, x[o], side="right")
        return np.minimum(out, n_nodes - 1)
    exit_cls_p = np.array([0.1, 0.2, 0.7])
    move_cls_p = np.array([0.2, 0.3, 0.5])
    pending12 = [[] for _ in range(n_days)]
    pending23 = [[] for _ in range(n_days)]
    blocks = []
    for d in range(n_days):
        # births -> S1
        nb = rng.poisson(rate_b * total)
        b = np.sort(draw(size_cdf, nb))
        if nb:
            np.add.at(T[:, 0], b, 1)
            blocks.append(_block(d, ENTER, b, -1, 1, 0, -1))
            if d + age_days[0] < n_days:
                pending12[d + age_days[0]].append(b)
            if d + age_days[1] < n_days:
                pending23[d + age_days[1]].append(b)
        # aging 1 -> 2, then 2 -> 3
        for j, pend in ((0, pending12), (1, pending23)):
            if pend[d]:
                a = np.sort(np.concatenate(pend[d]))
                ok = _keep_prefix(a, np.ones(len(a), np.int64), lambda k, j=j: T[k, j])
                a = a[ok]
                np.subtract.at(T[:, j], a, 1)
                np.add.at(T[:, j + 1], a, 1)
                if len(a):
                    blocks.append(_block(d, INTERNAL, a, -1, 1, 1 + j, j))
                pend[d] = None
        # exits, one animal of a drawn age class
        ne = rng.poisson(rate_b * total)
        if ne:
            x = draw(size_cdf, ne)
            c = rng.choice(3, ne, p=exit_cls_p)
            o = np.lexsort((c, x))
            x, c = x[o], c[o]
            ok = _keep_prefix(x * 3 + c, np.ones(ne, np.int64), lambda k: T[k // 3, k % 3])
            x, c = x[ok], c[ok]
            np.subtract.at(T, (x, c), 1)
            if len(x):
                blocks.append(_block(d, EXIT, x, -1, 1, 1 + c, -1))
        # movements
        nm = rng.poisson(e2_per_node_day * n_nodes)
        if nm:
            s = draw(size_cdf, nm)
            t = draw(dst_cdf, nm)
            same = t == s
            t[same] = (t[same] + 1 + rng.integers(0, n_nodes - 1, same.sum())) % n_nodes
            c = rng.choice(3, nm, p=move_cls_p)
            n = rng.integers(1, 6, nm)
            if shifted_moves > 0.0:
                sh = np.where((c < 2) & (rng.random(nm) < shifted_moves), c, -1)
            else:
                sh = np.full(nm, -1)
            ok = _keep_prefix(s * 3 + c, n, lambda k: T[k // 3, k % 3])
            s, t, c, n, sh = s[ok], t[ok], c[ok], n[ok], sh[ok]
            np.subtract.at(T, (s, c), n)
            np.add.at(T, (t, c + (sh >= 0)), n)
            if len(s):
                blocks.append(_block(d, EXTERNAL, s, t, n, 1 + c, sh))
    model = sise3_model(u=u, **(model_kw or {}))
    return Problem(n_nodes=n_nodes, n_rep=1, n_days=n_days, u0=u0, v0=np.zeros(n_nodes),
                   seed=seed, record_days=record_days, name=f"sise3_{n_nodes}x{n_days}",
                   **model, **_events_to_arrays(blocks))


# ---------------------------------------------------------------------------
# The workload configurations
# ---------------------------------------------------------------------------

def config1(seed=1, **kw):
    """Plain SIS, 1 age class: 1,000 nodes, 365 days."""
    return sis_network(n_nodes=1000, n_days=365, seed=seed, **kw)


def config2(seed=2, n_nodes=37000, n_days=1461, **kw):
    """SISe3, 37,000 nodes, 1461 days (about 5.3M events). A shorter horizon
    gives the same network and the same events, cut at n_days."""
    return sise3_network(n_nodes=n_nodes, n_days=n_days, seed=seed, **kw)


def config3(seed=3, n_nodes=1_000_000, n_days=1461, **kw):
    """SISe3 scale-up: 1,000,000 nodes, 1461 days (about 150M events)."""
    return sise3_network(n_nodes=n_nodes, n_days=n_days, seed=seed, **kw)


PRIOR_BOX = dict(upsilon=(0.005, 0.05), gamma=(0.05, 0.2), beta=(0.05, 0.15))


def prior_draws(n, seed):
    """Parameter vectors drawn uniformly from the prior box: per row
    (upsilon_1..3, gamma_1..3) as SISe3 rate constants, and beta_1..4."""
    rng = np.random.default_rng(seed)
    ups = rng.uniform(*PRIOR_BOX["upsilon"], (n, 3))
    gam = rng.uniform(*PRIOR_BOX["gamma"], (n, 3))
    coef = np.empty((n, 6))
    coef[:, 0::2] = ups
    coef[:, 1::2] = gam
    beta = rng.uniform(*PRIOR_BOX["beta"], (n, 4))
    return coef, np.ones(n), beta


def batched_replicates(R=256, n_days=730, seed=4):
    """The batched workload of the fitting pattern (Sec. 4.3): R replicates of
    the 37,000-node network over its first n_days days, each with its own
    prior-box parameter vector (seed) and replicate id r."""
    base = config2(n_days=n_days)
    coef, alpha, beta = prior_draws(R, seed=seed)
    return base.with_replicates(R, coef=coef, alpha=alpha, beta=beta, replicate_id=np.arange(R, dtype=np.uint32))


def uneven_sizes(n_inst=64, seed=4, lo=1e3, hi=2e5):
    """Node counts of the uneven instances, log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n_inst)).astype(int)


def uneven_instance(j, n_nodes, n_days=730, seed=4, n_inst=64):
    """Instance j of the uneven-instances workload: config 2's generator at
    n_nodes nodes with seed 4000 + j, one trajectory with row j of the
    prior-box draws."""
    coef, alpha, beta = prior_draws(n_inst, seed=seed)
    return sise3_network(n_nodes=int(n_nodes), n_days=n_days, seed=4000 + j).with_replicates(
        1, coef=coef[j:j + 1], alpha=alpha[j:j + 1], beta=beta[j:j + 1])


def uneven_instances(n_inst=64, n_days=730, seed=4):
    """The 64 uneven instances (1k-200k nodes) of the batched workload."""
    return [uneven_instance(j, n, n_days, seed, n_inst) for j, n in enumerate(uneven_sizes(n_inst, seed))]


SERVING_SIZES = (1000, 37000, 250000)


def serving_networks(n_days=1461, sizes=SERVING_SIZES, seeds=(51, 52, 53), **kw):
    """The pre-generated networks a serving run draws its requests over:
    config 2's generator at each size, one seed each."""
    return [sise3_network(n_nodes=n, n_days=n_days, seed=sd, **kw) for n, sd in zip(sizes, seeds)]


def serving_requests(n_requests=None, rate=20.0, duration=60.0, n_networks=3, horizon=(365, 1461),
                     reps=(1, 64), seed=5):
    """Open-loop request stream: Poisson arrivals at `rate` per second over
    `duration` seconds (or the first n_requests), each naming a network
    uniformly, a horizon uniform on [horizon[0], horizon[1]] days, a replicate
    count uniform on [reps[0], reps[1]], per-replicate parameters from the
    prior box, and replicate ids (request id * 64 + r) that key its random
    streams. Returns a list of dicts sorted by arrival time (seconds)."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if (n_requests is None and t > duration) or (n_requests is not None and len(out) >= n_requests):
            break
        i = len(out)
        n_rep = int(rng.integers(reps[0], reps[1] + 1))
        coef, alpha, beta = prior_draws(n_rep, seed=int(rng.integers(1 << 31)))
        out.append(dict(rid=i, arrival=t, net=int(rng.integers(n_networks)),
                        horizon=int(rng.integers(horizon[0], horizon[1] + 1)), n_rep=n_rep,
                        coef=coef, alpha=alpha, beta=beta,
                        replicate_id=(np.uint32(i) * np.uint32(64) + np.arange(n_rep, dtype=np.uint32))))
    return out


# ---------------------------------------------------------------------------
# Small systems with known laws (test inputs)
# ---------------------------------------------------------------------------

def _no_events():
    return _events_to_arrays([])


def sis_decay(n_nodes=4000, I0=20, S0=0, gamma=0.3, n_days=3, seed=11):
    """SIS with no infection and no events: each infected recovers at rate gamma."""
    m = sis_model(upsilon=0.0, gamma=gamma)
    u0 = np.tile(np.array([[S0, I0]]), (n_nodes, 1))
    return Problem(n_nodes=n_nodes, n_rep=1, n_days=n_days, u0=u0, v0=np.zeros(n_nodes),
                   seed=seed, name="sis_decay", **m, **_no_events())


def flip_model(n_nodes=400, S0=1000, I0=1000, n_days=2, seed=12):
    """The paper's synthetic benchmark model (Sec. 4.2): S->I and I->S at rate 1
    per individual, 1000 of each per node, no coupling."""
    m = sis_model(upsilon=1.0, gamma=1.0)
    m["uses_phi"] = np.array([0, 0], np.int32)
    u0 = np.tile(np.array([[S0, I0]]), (n_nodes, 1))
    return Problem(n_nodes=n_nodes, n_rep=1, n_days=n_days, u0=u0, v0=np.zeros(n_nodes),
                   seed=seed, name="flip", **m, **_no_events())


def flip_classes(n_nodes=400, S0=333, I0=333, n_days=2, seed=12):
    """The synthetic model's dynamics on the SISe3 compartments: in each of the
    three classes S_j -> I_j and I_j -> S_j at rate 1 per individual, S0 and
    I0 of each per node, no coupling and no events (a chain of the
    six-compartment model whose length is known in advance)."""
    m = sise3_model(coef=np.ones(6))
    m["uses_phi"] = np.zeros(6, np.int32)
    u0 = np.tile(np.array([[S0, I0] * 3]), (n_nodes, 1))
    return Problem(n_nodes=n_nodes, n_rep=1, n_days=n_days, u0=u0, v0=np.zeros(n_nodes),
                   seed=seed, name="flip3", **m, **_no_events())


def constant_infection(n_nodes=3, S0=(90, 50, 0), I0=(10, 50, 0), phi0=(0.0, 1.5, 2.0),
                       n_days=400, day0=0, beta=(0.10, 0.12, 0.10, 0.08), alpha=0.7, seed=13):
    """SIS with all rates zero and no events: I/N is constant, so phi follows a
    linear recurrence with a closed form per season."""
    m = sis_model(upsilon=0.0, gamma=0.0, alpha=alpha, beta=beta)
    u0 = np.stack([np.asarray(S0), np.asarray(I0)], axis=1)
    return Problem(n_nodes=n_nodes, n_rep=1, n_days=n_days, u0=u0, v0=np.asarray(phi0, float),
                   seed=seed, day0=day0, name="constant_infection", **m, **_no_events())


def events_only(u0, events, n_days, model="sis", seed=14, n_rep=1):
    """Given state and an explicit event list, with all stochastic rates zero."""
    m = sis_model(upsilon=0.0, gamma=0.0) if model == "sis" else sise3_model(coef=np.zeros(6))
    blocks = [_block(*ev) if np.ndim(ev[2]) else _block(ev[0], ev[1], [ev[2]], ev[3], ev[4], ev[5], ev[6])
              for ev in events]
    u0 = np.asarray(u0)
    p = Problem(n_nodes=u0.shape[0], n_rep=1, n_days=n_days, u0=u0, v0=np.zeros(u0.shape[0]),
                seed=seed, name="events_only", **m, **_events_to_arrays(blocks))
    return p.with_replicates(n_rep) if n_rep > 1 else p


def two_node(n_days=3, seed=15, upsilon=0.4, gamma=0.5, alpha=1.0, beta=(0.3, 0.3, 0.3, 0.3),
             u0=((2, 1), (1, 0)), phi0=(0.2, 0.0), events=None):
    """A two-node SIS system small enough for an exact master-equation solution:
    infection upsilon*phi*S, recovery gamma*I, phi forced by I/N, and a few
    scheduled events (an animal moved from node 0 to node 1 on day 0, a birth
    at node 1 on day 1, a death at node 0 on day 2)."""
    m = sis_model(upsilon=upsilon, gamma=gamma, alpha=alpha, beta=beta)
    if events is None:
        events = [(0, EXTERNAL, 0, 1, 1, 1, -1), (1, ENTER, 1, -1, 1, 0, -1),
                  (2, EXIT, 0, -1, 1, 1, -1)]
    blocks = [_block(ev[0], ev[1], [ev[2]], ev[3], ev[4], ev[5], ev[6]) for ev in events]
    return Problem(n_nodes=2, n_rep=1, n_days=n_days, u0=np.asarray(u0), v0=np.asarray(phi0, float),
                   seed=seed, name="two_node", **m, **_events_to_arrays(blocks))
