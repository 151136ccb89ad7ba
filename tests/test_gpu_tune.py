"""The tuner of launch shape and level grouping on the GPU: every candidate
setting ends the timed window in the same state, bit for bit (the tuner
checks it and raises otherwise), and the fastest candidate is returned. Calls
go through the C ABI."""
import numpy as np
import pytest

from farmnet import synth
import paper_1502_02908_amd as P
from oracle import oracle as O
from paper_1502_02908_amd.tune import LANE_CANDIDATES, TILE_CANDIDATES, autotune

from .gpu_common import assert_parity

from .gpu_common import say

pytestmark = pytest.mark.gpu


def test_candidates_agree_and_fastest_is_chosen():
    # 9000 nodes: the group-herd placement applies, so the candidates differ in
    # node order, launch shape and level grouping
    p = synth.sise3_network(n_nodes=9000, n_days=90, seed=33, u=10.0, age_days=(20, 60))
    t = autotune(p, start_day=45, window=15)
    say(f"[tune] {t.summary()}")
    assert len(t.table) == len(LANE_CANDIDATES)
    assert t.best in [dict(c) for c in LANE_CANDIDATES]
    fastest = min(t.table, key=lambda row: row[1])
    assert t.best == (fastest[0] if fastest[1] < 0.97 * t.table[0][1] else t.table[0][0])
    assert all(ms > 0 for _, ms in t.table)


def test_group_and_grouping_options_match_the_default_run():
    p = synth.sise3_network(n_nodes=9000, n_days=40, seed=34, u=10.0, age_days=(20, 60))
    out = []
    for kw in (dict(), dict(group_herds=-1), dict(group_herds=16, small_level=64)):
        with P.Simulator(p, **kw) as sim:
            sim.run(0)
            tr = sim.trajectory()
            u, v, _ = sim.get_state()
        out.append((tr, u, v))
    for tr, u, v in out[1:]:
        assert np.array_equal(u, out[0][1]) and np.array_equal(v.view(np.int64), out[0][2].view(np.int64))
        for k in ("prevalence", "transitions", "totals"):
            assert np.array_equal(tr[k], out[0][0][k]), k


def test_tile_candidates_agree_and_fastest_is_chosen():
    # replicate tiles: tile width, heavy herds and the few-chain walk vary
    base = synth.sise3_network(n_nodes=3000, n_days=60, seed=35, u=5.0, age_days=(10, 30))
    coef, alpha, beta = synth.prior_draws(64, seed=36)
    p = base.with_replicates(64, coef=coef * 3, alpha=alpha, beta=beta)
    t = autotune(p, start_day=30, window=10)
    say(f"[tune] tiles {t.summary()}")
    assert len(t.table) == len(TILE_CANDIDATES)
    fastest = min(t.table, key=lambda row: row[1])
    assert t.best == (fastest[0] if fastest[1] < 0.97 * t.table[0][1] else t.table[0][0])


@pytest.mark.parametrize("kw", [dict(tile_nodes=32), dict(tile_nodes=512), dict(heavy_herds=-1),
                                dict(heavy_herds=32, few_chains=-1), dict(few_chains=16)])
def test_tile_options_match_the_oracle(kw):
    base = synth.sise3_network(n_nodes=2500, n_days=40, seed=37, u=5.0, age_days=(10, 30))
    coef, alpha, beta = synth.prior_draws(70, seed=38)
    p = base.with_replicates(70, coef=coef * 3, alpha=alpha, beta=beta,
                             replicate_id=np.arange(70, dtype=np.uint32) + 300)
    p.record_days = np.array([39], np.int32)
    with P.Simulator(p, **kw) as sim:
        sim.run(0)
        g = sim.trajectory()
        g["u"], g["v"], _ = sim.get_state()
    assert_parity(g, O.run(p, threads=8))


@pytest.mark.parametrize("kw", [dict(group_min_attempts=256), dict(few_chains=-1), dict(few_chains=64),
                                dict(tile_nodes=4), dict(tile_nodes=16)])
def test_lane_options_match_the_oracle(kw):
    p = synth.sise3_network(n_nodes=9000, n_days=40, seed=39, u=10.0, age_days=(20, 60))
    p.record_days = np.array([39], np.int32)
    with P.Simulator(p, **kw) as sim:
        sim.run(0)
        g = sim.trajectory()
        g["u"], g["v"], _ = sim.get_state()
    assert_parity(g, O.run(p, threads=8))


@pytest.mark.parametrize("tile", [4, 32])
def test_one_replicate_tiles_on_the_synthetic_model(tile):
    # Sec. 4.2's SSA-heavy model (S <-> I at rate 1, no events): with one
    # replicate in tiles every wavefront walks one node's long chain with all
    # its lanes; records and state against the oracle
    p = synth.flip_model(n_nodes=200, n_days=12)
    p.record_days = np.array([5, 11], np.int32)
    with P.Simulator(p, tile_nodes=tile) as sim:
        sim.run(0)
        g = sim.trajectory()
        g["u"], g["v"], _ = sim.get_state()
    o = O.run(p, threads=8)
    assert o["transitions"].sum() > 10 ** 6
    assert_parity(g, o)
