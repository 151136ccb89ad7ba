"""Batched trajectories on the GPU: many replicates with their own parameter
vectors (replicate tiles), and several uneven instances packed into one
handle. Each trajectory must equal the oracle's, and a packed instance must
equal the same instance run alone."""
import numpy as np
import pytest

from farmnet import EXIT, synth
from oracle import oracle as O
import paper_1502_02908_amd as P

from .gpu_common import assert_parity, gpu_run, say

pytestmark = pytest.mark.gpu


def prior_replicates(base, R, seed):
    coef, alpha, beta = synth.prior_draws(R, seed=seed)
    rid = np.arange(100, 100 + R, dtype=np.uint32)
    return base.with_replicates(R, coef=coef * 3, alpha=alpha, beta=beta, replicate_id=rid)


@pytest.mark.parametrize("R,launch", [(64, P.LAUNCH_KERNELS), (128, P.LAUNCH_KERNELS), (256, P.LAUNCH_KERNELS),
                                      (64, P.LAUNCH_PERSISTENT)])
def test_replicate_tiles_match_oracle(R, launch):
    base = synth.sise3_network(n_nodes=700, n_days=60, seed=41, age_days=(10, 30))
    p = prior_replicates(base, R, seed=5)
    p.record_days = np.array([0, 59], np.int32)
    say(f"[batch] tiles R={R} launch={launch}")
    g = gpu_run(p, launch=launch)
    o = O.run(p, threads=8)
    assert_parity(g, o)


def test_replicate_equals_plain_run():
    base = synth.sise3_network(n_nodes=1500, n_days=90, seed=42, u=5.0, age_days=(10, 30))
    p = prior_replicates(base, 64, seed=6)
    g = gpu_run(p)
    for r in (0, 17, 63):
        one = base.with_replicates(1, coef=p.coef[r:r + 1], alpha=p.alpha[r:r + 1], beta=p.beta[r:r + 1],
                                   replicate_id=p.replicate_id[r:r + 1])
        a = gpu_run(one)
        assert np.array_equal(a["u"][0], g["u"][r]) and np.array_equal(a["v"][0], g["v"][r])
        assert np.array_equal(a["prevalence"][:, 0], g["prevalence"][:, r])


def instances(R=1, n_days=50):
    sizes = [300, 1000, 77, 2500]
    out = []
    for k, n in enumerate(sizes):
        base = synth.sise3_network(n_nodes=n, n_days=n_days, seed=60 + k, u=4.0, age_days=(10, 30))
        base.seed = 1000 + k
        coef, alpha, beta = synth.prior_draws(R, seed=70 + k)
        out.append(base.with_replicates(R, coef=coef * 3, alpha=alpha, beta=beta,
                                        replicate_id=np.arange(R, dtype=np.uint32) + 7 * k))
    return out


@pytest.mark.parametrize("R,launch,tile", [(1, P.LAUNCH_KERNELS, 0), (1, P.LAUNCH_PERSISTENT, 0),
                                           (64, P.LAUNCH_KERNELS, 0), (3, P.LAUNCH_KERNELS, 0),
                                           (1, P.LAUNCH_KERNELS, 8)])
def test_packed_instances_match_oracle(R, launch, tile):
    # tile > 0 with R = 1: one-replicate tiles, a wavefront per node
    probs = instances(R)
    say(f"[batch] pack of {len(probs)} instances R={R} launch={launch} tile_nodes={tile}")
    with P.Simulator(probs, launch=launch, tile_nodes=tile) as sim:
        sim.run(0)
        traj = sim.trajectory()
        u, v, day = sim.get_state()
    off = 0
    for k, q in enumerate(probs):
        o = O.run(q, threads=8)
        sl = slice(off, off + q.n_nodes)
        assert np.array_equal(u[:, sl], o["u"]), k
        assert np.array_equal(v[:, sl].view(np.int64), o["v"].view(np.int64)), k
        sets = slice(k * R, (k + 1) * R)
        assert np.array_equal(traj["prevalence"][:, sets], o["prevalence"]), k
        assert np.array_equal(traj["transitions"][:, sets], o["transitions"]), k
        assert np.array_equal(traj["totals"][:, sets], o["totals"]), k
        off += q.n_nodes


def test_packed_instance_equals_alone():
    probs = instances(1, n_days=40)
    with P.Simulator(probs) as sim:
        sim.run(0)
        u, v, _ = sim.get_state()
    off = 0
    for q in probs:
        a = gpu_run(q)
        assert np.array_equal(a["u"], u[:, off:off + q.n_nodes])
        off += q.n_nodes


def test_packed_infeasible_names_instance():
    probs = instances(1, n_days=10)
    bad = probs[2]
    bad.ev_kind = bad.ev_kind.copy()
    i = int(np.flatnonzero(bad.ev_day == 3)[0])
    bad.ev_kind[i] = EXIT
    bad.ev_n = bad.ev_n.copy()
    bad.ev_n[i] = 10**6
    with P.Simulator(probs) as sim:
        sim.run(0)
        with pytest.raises(P.SimError) as e:
            sim.sync()
    assert e.value.code == -4
    assert f"infeasible event {i} (replicate 0) of instance 2 on day 3" in str(e.value)
