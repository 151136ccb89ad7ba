"""Oracle samples of the batched and serving workloads at their full size,
run on the GPU exactly as the benchmark runs them (Sec. 4.3's fitting pattern:
many trajectories over one event database):

* 256 replicates of the 37,000-node network over 730 days, each with its own
  prior-box parameters, in one handle (replicate tiles): 8 replicate ids
  against the oracle;
* the 64 uneven instances (1k-200k nodes, one trajectory each, 730 days)
  packed into one handle: 8 of them against the oracle, most of at least
  8,192 nodes (their largest herds are walked by whole workgroups);
* 16 requests of the serving stream (Poisson arrivals, networks of 1k, 37k
  and 250k nodes over 1461 days, horizons 365-1461 days, 1-64 replicates)
  through the request server: sampled replicates of every request against
  the oracle.

Every count and record compared element by element, bit-exact; phi bit-exact
(the stated tolerance is 1e-12 relative)."""
import os
import time

import numpy as np
import pytest

from farmnet import synth
from oracle import oracle as O
import paper_1502_02908_amd as P

from .gpu_common import first_mismatch, say

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


def same(a, b, what):
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if a.dtype == np.float64:
        a, b = a.view(np.int64), b.view(np.int64)
    mm = first_mismatch(a, b)
    assert mm is None, f"{what}: first mismatch at {mm[0]}: gpu {mm[1]} oracle {mm[2]} ({mm[3]} differ)"


def subset(p, idx):
    return p.with_replicates(len(idx), coef=p.coef[idx], alpha=p.alpha[idx], beta=p.beta[idx],
                             replicate_id=np.asarray(p.replicate_id)[idx])


@pytest.mark.timeout(900)
def test_batched_256_replicates_sample():
    p = synth.batched_replicates()
    say(f"[configs] batched: {p.n_rep} replicates x {p.n_nodes} nodes x {p.n_days} days, {p.n_events} events")
    with P.Simulator(p) as sim:
        sim.run(0)
        tr = sim.trajectory()
        u, v, day = sim.get_state()
    assert day == p.n_days
    idx = np.array([0, 37, 64, 101, 128, 190, 211, 255])
    t0 = time.perf_counter()
    o = O.run(subset(p, idx), threads=THREADS)
    say(f"[configs] oracle on replicates {idx.tolist()}: {time.perf_counter() - t0:.1f} s")
    for k in ("prevalence", "transitions"):
        same(tr[k][:, idx], o[k], k)
    same(tr["totals"][:, idx], o["totals"], "totals")
    same(u[idx], o["u"], "u")
    same(v[idx], o["v"], "v")
    assert o["transitions"].sum() > 10 ** 6


@pytest.mark.timeout(1200)
def test_uneven_instances_sample():
    sizes = synth.uneven_sizes()
    t0 = time.perf_counter()
    insts = synth.uneven_instances()
    say(f"[configs] {len(insts)} instances, {int(sizes.sum())} nodes, generated in {time.perf_counter() - t0:.0f} s")
    with P.Simulator(insts) as sim:
        sim.run(0)
        tr = sim.trajectory()
        u, v, day = sim.get_state()
    assert day == 730
    order = np.argsort(sizes)
    pick = order[np.linspace(0, len(order) - 1, 8).round().astype(int)]
    assert (sizes[pick] >= 8192).sum() >= 4
    off = np.r_[0, np.cumsum(sizes)]
    for j in pick:
        q = insts[j]
        t0 = time.perf_counter()
        o = O.run(q, threads=THREADS)
        say(f"[configs] instance {j} ({q.n_nodes} nodes): oracle {time.perf_counter() - t0:.1f} s")
        sl = slice(off[j], off[j + 1])
        same(u[:, sl], o["u"], f"u of instance {j}")
        same(v[:, sl], o["v"], f"v of instance {j}")
        for k in ("prevalence", "transitions", "totals"):
            same(tr[k][:, j:j + 1], o[k], f"{k} of instance {j}")


@pytest.mark.timeout(1200)
def test_serving_requests_sample():
    from paper_1502_02908_amd.serve import Server, plan_slots
    t0 = time.perf_counter()
    nets = synth.serving_networks()
    reqs = synth.serving_requests(n_requests=16, rate=20.0, seed=5)
    say(f"[configs] serving networks generated in {time.perf_counter() - t0:.0f} s; requests "
        f"{[(q['net'], q['horizon'], q['n_rep']) for q in reqs]}")
    slots, _ = plan_slots(nets, 96 * 2 ** 30, [net.n_nodes for net in nets])
    srv = Server(nets, slots, max_ahead=4)
    try:
        results, stats = srv.serve(reqs, realtime=False)
    finally:
        srv.close()
    say(f"[configs] served: {stats.summary(results)}")
    assert sorted(r.rid for r in results) == list(range(16)) and not any(r.error for r in results)
    by_id = {q["rid"]: q for q in reqs}
    for r in sorted(results, key=lambda r: r.rid):
        q = by_id[r.rid]
        net = nets[q["net"]]
        # the first and the last replicate of every request (lane 0 and the
        # request's last lane of its slot)
        idx = np.unique([0, q["n_rep"] - 1])
        p = net.truncated(q["horizon"]).with_replicates(
            len(idx), coef=q["coef"][idx], alpha=q["alpha"][idx], beta=q["beta"][idx],
            replicate_id=q["replicate_id"][idx])
        t0 = time.perf_counter()
        o = O.run(p, threads=THREADS)
        say(f"[configs] request {r.rid} ({net.n_nodes} nodes, {q['horizon']} days, replicates {idx.tolist()} "
            f"of {q['n_rep']}): oracle {time.perf_counter() - t0:.1f} s")
        same(r.prevalence[:, idx], o["prevalence"], f"prevalence of request {r.rid}")
        same(r.transitions[:, idx], o["transitions"], f"transitions of request {r.rid}")
