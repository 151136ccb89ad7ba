"""The goal function of the fitting study (Sec. 4.3) and the regional
aggregates it is computed from, pinned by identities that hold whatever the
numbers: the mean squared distance of the sample trajectories to the
reference splits into G^2 and (N-1)/N VG^2; identical trajectories give 0;
regions partition the totals; and the oracle's regional sums match the
snapshot states summed region by region."""
import numpy as np

from farmnet import synth
from oracle import goal as Gf
from oracle import oracle as O


def regioned(p, J, seed=0):
    import dataclasses
    rng = np.random.default_rng(seed)
    return dataclasses.replace(p, n_regions=J, region=rng.integers(0, J, p.n_nodes).astype(np.int32))


def test_bias_variance_identity():
    rng = np.random.default_rng(3)
    for N in (1, 2, 5, 17):
        x = rng.integers(0, 1000, (7, N, 4, 6))
        ref = rng.integers(0, 1000, (7, 4, 6))
        G2, VG2 = Gf.goal(x, ref)
        msd = ((x - ref[:, None]) ** 2).sum() / N
        assert np.isclose(msd, G2 + (N - 1) / N * VG2, rtol=1e-12, atol=0), (N, msd, G2, VG2)
        assert G2 >= 0 and VG2 >= 0


def test_identical_trajectories_have_zero_goal():
    p = regioned(synth.sise3_network(n_nodes=300, n_days=30, seed=4, age_days=(5, 15)), 5)
    ref = O.run(p)["regional"][:, 0]
    # four trajectories with the reference's replicate id: the same trajectory
    same = O.run(p.with_replicates(4, replicate_id=np.zeros(4, np.uint32)))["regional"]
    assert Gf.goal(same, ref) == (0.0, 0.0)
    other = O.run(p.with_replicates(4, replicate_id=np.arange(1, 5, dtype=np.uint32)))["regional"]
    G2, VG2 = Gf.goal(other, ref)
    assert G2 > 0 and VG2 > 0


def test_regions_partition_the_totals_and_match_snapshots():
    p = regioned(synth.sise3_network(n_nodes=400, n_days=20, seed=5, age_days=(5, 15)), 7, seed=1)
    p.record_days = np.array([0, 9, 19], np.int32)
    o = O.run(p.with_replicates(3))
    assert np.array_equal(o["regional"].sum(axis=2), o["totals"])
    for k, d in enumerate(p.record_days):
        for r in range(3):
            snap = o["snap_u"][k, r]                     # [node][c]
            by_region = np.zeros((7, p.n_comp), np.int64)
            np.add.at(by_region, p.region, snap)
            assert np.array_equal(by_region, o["regional"][d, r])


def test_nodes_without_region_are_left_out():
    import dataclasses
    p = regioned(synth.sise3_network(n_nodes=200, n_days=10, seed=6, age_days=(5, 15)), 3, seed=2)
    reg = p.region.copy()
    reg[::4] = -1
    q = dataclasses.replace(p, region=reg)
    o = O.run(q)
    assert not np.array_equal(o["regional"].sum(axis=2), o["totals"])
    assert np.array_equal(O.run(dataclasses.replace(q, region=np.where(reg < 0, 0, reg)))["regional"][:, :, 1:],
                          o["regional"][:, :, 1:])


def test_goal_is_smallest_at_the_reference_parameters():
    # the fitting setup of Sec. 4.3: a reference trajectory at k*, samples at
    # k* and with the infection rates halved or doubled; the goal prefers k*
    p = regioned(synth.sise3_network(n_nodes=1500, n_days=120, seed=7, u=10.0, age_days=(20, 60)), 21, seed=3)
    ref = O.run(p.with_replicates(1, replicate_id=np.array([999], np.uint32)))["regional"][:, 0]
    ids = np.arange(8, dtype=np.uint32)
    G = {}
    for f in (0.5, 1.0, 2.0):
        c = p.coef[0].copy()
        c[0::2] *= f  # upsilon_1..3
        G[f] = Gf.goal(O.run(p.with_replicates(8, coef=np.tile(c, (8, 1)), replicate_id=ids),
                             threads=8)["regional"], ref)[0]
    assert G[1.0] < G[0.5] and G[1.0] < G[2.0], G
    assert Gf.residual(np.sqrt(G[2.0]), np.sqrt(G[1.0])) > 1.0
