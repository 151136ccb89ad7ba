"""sim_goal_noalloc, the goal function for callers that cannot allocate device
memory, against sim_goal on the same handle through the C ABI: two calls in a
row (the second over a smaller input: fewer replicates, regions and days) give
the same G^2 and VG^2 bit for bit, and a range larger than the static array
is rejected before any device work. Runs alone in a fresh process and after
every other test."""
import dataclasses
import os

import numpy as np
import pytest

from farmnet import synth
from oracle import oracle as O
import paper_1502_02908_amd as P

from .gpu_common import say

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


def regioned(p, J, seed):
    rng = np.random.default_rng(seed)
    reg = rng.integers(-1, J, p.n_nodes).astype(np.int32)
    return dataclasses.replace(p, n_regions=J, region=reg)


def reference_of(p, rid):
    """Regional sums of a reference trajectory (another replicate id), from the oracle."""
    q = p.with_replicates(1, coef=p.coef[:1], alpha=p.alpha[:1], beta=p.beta[:1],
                          replicate_id=np.array([rid], np.uint32))
    return O.run(q, threads=THREADS)["regional"][:, 0]


def same_bits(a, b):
    return np.float64(a).view(np.int64) == np.float64(b).view(np.int64)


def test_goal_noalloc_equals_goal_twice():
    cases = [(3000, 80, 21, 64, 91), (700, 40, 5, 3, 92)]  # the second call's input is smaller
    for n_nodes, n_days, J, R, seed in cases:
        base = regioned(synth.sise3_network(n_nodes=n_nodes, n_days=n_days, seed=seed, u=6.0,
                                            age_days=(10, 30)), J, seed)
        coef, alpha, beta = synth.prior_draws(R, seed=seed)
        p = base.with_replicates(R, coef=coef * 3, alpha=alpha, beta=beta,
                                 replicate_id=np.arange(R, dtype=np.uint32) + 7)
        ref = reference_of(p, 4000 + seed)
        say(f"[no-alloc] Nn={n_nodes} D={n_days} J={J} R={R}")
        with P.Simulator(p) as sim:
            sim.run(0)
            sim.sync()
            for d0, d1 in ((0, n_days), (n_days // 3, n_days - 1), (5, 5)):
                want = sim.goal(ref, d_begin=d0, d_end=d1)
                got = sim.goal_noalloc(ref, d_begin=d0, d_end=d1)
                assert same_bits(got[0], want[0]) and same_bits(got[1], want[1]), (d0, d1, got, want)
                if d1 > d0:
                    assert want[0] > 0 and (R == 1 or want[1] > 0)


def test_goal_noalloc_rejects_oversized_range():
    # 4096 regions x 6 compartments x 8 bytes = 192 KiB per day: 60 days pass 8 MiB
    base = synth.sise3_network(n_nodes=300, n_days=60, seed=93, age_days=(10, 30))
    p = regioned(base, 4096, 93)
    ref = np.zeros((p.n_days, 4096, 6), np.int64)
    with P.Simulator(p) as sim:
        sim.run(0)
        want = sim.goal(ref, d_begin=0, d_end=30)
        assert same_bits(sim.goal_noalloc(ref, d_begin=0, d_end=30)[0], want[0])
        with pytest.raises(P.SimError) as e:
            sim.goal_noalloc(ref, d_begin=0, d_end=60)
        assert e.value.code == P.SIM_EINVAL and "scratch" in str(e.value)
        # the handle and the array are still fine after the rejected call
        assert same_bits(sim.goal_noalloc(ref, d_begin=10, d_end=40)[0], sim.goal(ref, d_begin=10, d_end=40)[0])
