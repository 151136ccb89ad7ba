"""Regional records and the goal function of the fitting study (Sec. 4.3) on
the GPU: the daily regional sums bit-exact against the oracle in every layout
(single replicate, replicate tiles with heavy herds, packed instances, both
launch modes), and G^2 / VG^2 from the device reduction within 1e-12 relative
of the oracle's goal on the oracle's own regional sums. Calls go through the
C ABI."""
import dataclasses
import os

import numpy as np
import pytest

from farmnet import synth
from oracle import goal as OG
from oracle import oracle as O
import paper_1502_02908_amd as P

from .gpu_common import first_mismatch, say

pytestmark = pytest.mark.gpu

GOAL_RTOL = 1e-12
THREADS = min(16, os.cpu_count() or 1)


def regioned(p, J, seed, unassigned=0.05):
    """Uneven regions (sizes drawn from a Dirichlet), a few nodes in none."""
    rng = np.random.default_rng(seed)
    w = rng.dirichlet(np.full(J, 0.7))
    reg = rng.choice(J, size=p.n_nodes, p=w).astype(np.int32)
    reg[rng.random(p.n_nodes) < unassigned] = -1
    return dataclasses.replace(p, n_regions=J, region=reg)


def reference_of(p, seed):
    """Regional sums of one reference trajectory (another replicate id), from the oracle."""
    q = p.with_replicates(1, coef=p.coef[:1], alpha=p.alpha[:1], beta=p.beta[:1],
                          replicate_id=np.array([seed], np.uint32))
    return O.run(q, threads=THREADS)["regional"][:, 0]


def close(a, b):
    return abs(a - b) <= GOAL_RTOL * max(abs(b), 1e-300)


def check_regional(got, want, what):
    assert got.shape == want.shape, (what, got.shape, want.shape)
    mm = first_mismatch(got, want)
    assert mm is None, f"{what}: first mismatch at {mm[0]}: gpu {mm[1]} oracle {mm[2]} ({mm[3]} differ)"


@pytest.mark.parametrize("launch", [P.LAUNCH_KERNELS, P.LAUNCH_PERSISTENT])
def test_regional_single_replicate(launch):
    p = regioned(synth.sise3_network(n_nodes=3000, n_days=90, seed=81, u=8.0, age_days=(15, 40)), 21, seed=1)
    say(f"[goal] R=1 Nn={p.n_nodes} J={p.n_regions} launch={launch}")
    with P.Simulator(p, launch=launch) as sim:
        sim.run(0)
        tr = sim.trajectory()
        ref = reference_of(p, 999)
        g2, vg2 = sim.goal(ref)
    o = O.run(p, threads=THREADS)
    check_regional(tr["regional"], o["regional"], "regional")
    assert np.array_equal(tr["totals"], o["totals"])
    G2, VG2 = OG.goal(o["regional"], ref)
    assert close(g2, G2) and vg2 == 0.0 and VG2 == 0.0, (g2, G2)
    assert G2 > 0


@pytest.mark.parametrize("R,launch", [(64, P.LAUNCH_KERNELS), (100, P.LAUNCH_KERNELS), (64, P.LAUNCH_PERSISTENT)])
def test_goal_over_replicate_tiles(R, launch):
    # 4000 nodes: the TILE layout walks its largest herds as heavy units
    base = regioned(synth.sise3_network(n_nodes=4000, n_days=60, seed=82, u=6.0, age_days=(10, 30)), 21, seed=2)
    coef, alpha, beta = synth.prior_draws(1, seed=9)
    p = base.with_replicates(R, coef=np.repeat(coef * 3, R, 0), alpha=np.repeat(alpha, R),
                             beta=np.repeat(beta, R, 0), replicate_id=np.arange(R, dtype=np.uint32) + 11)
    say(f"[goal] tiles R={R} launch={launch}")
    ref = reference_of(p, 5000)
    with P.Simulator(p, launch=launch) as sim:
        sim.run(0)
        tr = sim.trajectory()
        g2, vg2 = sim.goal(ref)
        part = sim.goal(ref, d_begin=10, d_end=35)
    o = O.run(p, threads=THREADS)
    check_regional(tr["regional"], o["regional"], "regional")
    G2, VG2 = OG.goal(o["regional"], ref)
    assert close(g2, G2) and close(vg2, VG2), (g2, G2, vg2, VG2)
    G2p, VG2p = OG.goal(o["regional"][10:35], ref[10:35])
    assert close(part[0], G2p) and close(part[1], VG2p)
    assert VG2 > 0 and G2 > 0


@pytest.mark.parametrize("R", [1, 3, 64])
def test_goal_per_packed_instance(R):
    sizes = [300, 1000, 77, 2500]
    probs = []
    for k, n in enumerate(sizes):
        b = synth.sise3_network(n_nodes=n, n_days=40, seed=90 + k, u=4.0, age_days=(10, 30))
        b.seed = 2000 + k
        coef, alpha, beta = synth.prior_draws(R, seed=95 + k)
        b = b.with_replicates(R, coef=coef * 3, alpha=alpha, beta=beta,
                              replicate_id=np.arange(R, dtype=np.uint32) + 5 * k)
        probs.append(regioned(b, 6, seed=10 + k))
    say(f"[goal] pack of {len(probs)} instances R={R}")
    refs = [reference_of(q, 777 + k) for k, q in enumerate(probs)]
    with P.Simulator(probs) as sim:
        sim.run(0)
        tr = sim.trajectory()
        goals = [sim.goal(refs[k], instance=k) for k in range(len(probs))]
    for k, q in enumerate(probs):
        o = O.run(q, threads=THREADS)
        check_regional(tr["regional"][:, k * R:(k + 1) * R], o["regional"], f"instance {k}")
        G2, VG2 = OG.goal(o["regional"], refs[k])
        assert close(goals[k][0], G2) and close(goals[k][1], VG2), (k, goals[k], G2, VG2)


def test_goal_after_chunked_runs_and_errors():
    p = regioned(synth.sise3_network(n_nodes=800, n_days=50, seed=83, age_days=(10, 30)), 4, seed=3)
    p = p.with_replicates(8, replicate_id=np.arange(8, dtype=np.uint32))
    ref = reference_of(p, 1234)
    with P.Simulator(p) as sim:
        sim.run(20)
        early = sim.goal(ref, d_end=20)
        with pytest.raises(P.SimError) as e:
            sim.goal(ref, d_end=21)
        assert e.value.code == P.SIM_ESTATE
        with pytest.raises(P.SimError):
            sim.goal(ref, instance=1)
        sim.run(0)
        tr = sim.trajectory()
        full = sim.goal(ref)
        assert sim.goal(ref, d_begin=7, d_end=7) == (0.0, 0.0)
    o = O.run(p, threads=THREADS)
    check_regional(tr["regional"], o["regional"], "regional")
    for got, (a, b) in ((early, (0, 20)), (full, (0, 50))):
        G2, VG2 = OG.goal(o["regional"][a:b], ref[a:b])
        assert close(got[0], G2) and close(got[1], VG2)


def test_handle_without_regions_rejects_goal():
    p = synth.sise3_network(n_nodes=200, n_days=5, seed=84, age_days=(5, 10))
    with P.Simulator(p) as sim:
        sim.run(0)
        assert "regional" not in sim.trajectory()
        with pytest.raises(P.SimError) as e:
            sim.goal(np.zeros((5, 0, p.n_comp), np.int64))
        assert e.value.code == P.SIM_ESTATE
