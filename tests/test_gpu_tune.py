"""The tuner of launch shape and level grouping on the GPU: every candidate
setting ends the timed window in the same state, bit for bit (the tuner
checks it and raises otherwise), and the fastest candidate is returned. Calls
go through the C ABI."""
import numpy as np
import pytest

from farmnet import synth
import paper_1502_02908_amd as P
from paper_1502_02908_amd.tune import CANDIDATES, autotune

from .gpu_common import say

pytestmark = pytest.mark.gpu


def test_candidates_agree_and_fastest_is_chosen():
    # 9000 nodes: the group-herd placement applies, so the candidates differ in
    # node order, launch shape and level grouping
    p = synth.sise3_network(n_nodes=9000, n_days=90, seed=33, u=10.0, age_days=(20, 60))
    t = autotune(p, start_day=45, window=15)
    say(f"[tune] {t.summary()}")
    assert len(t.table) == len(CANDIDATES)
    assert t.best in [dict(c) for c in CANDIDATES]
    assert t.best == min(t.table, key=lambda row: row[1])[0]
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
