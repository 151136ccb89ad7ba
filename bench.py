#!/usr/bin/env python3
"""Throughput of the per-day hot path on one MI355X.

Workload: the SISe3 farm network of 37,000 nodes over 1461 days (about 5.3M
scheduled events, seed 2), synthetic (see farmnet/synth.py). One step is one
full simulation of the horizon from the initial state: every day runs the SSA
of every node, the day's events in dependency levels, and the phi update.
Inputs are resident in HBM before the timed region; the state is reset between
steps outside it.

Prints one JSON line: node-days/s (value), SSA transitions/s, the dominant
kernel's achieved algorithmic bandwidth against the HBM peak, and the oracle
timed on the host's cores on the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, vendor peak

WORKLOADS = {
    "sise3-37k": dict(desc="SISe3 farm network, 37,000 nodes x 1461 days, seed 2",
                      make=lambda synth: synth.config2()),
    "sis-1k": dict(desc="SIS farm network, 1,000 nodes x 365 days, seed 1",
                   make=lambda synth: synth.config1()),
    "sise3-1m": dict(desc="SISe3 farm network, 1,000,000 nodes x 1461 days, seed 3",
                     make=lambda synth: synth.config3()),
    # the 37k network with the rate constants scaled by u = 10 (Sec. 4.1's load variant)
    "sise3-37k-u10": dict(desc="SISe3 farm network, 37,000 nodes x 1461 days, seed 2, u = 10",
                          make=lambda synth: synth.config2(u=10.0)),
    # the paper's synthetic SSA-heavy model (Sec. 4.2): S <-> I at rate 1, S = I = 1000, no events
    "synthetic-1k": dict(desc="synthetic S<->I model, 1,000 nodes x 1000 days, S = I = 1000, rates 1",
                         make=lambda synth: synth.flip_model(n_nodes=1000, n_days=1000)),
}


def algorithmic_bytes(p, day_launches, ev_counts_by_kind):
    """Bytes the method must move: per node-day the state u (4 B per
    compartment) and phi (8 B), read and written; per event a 20 B record plus
    4 B read and 4 B written per compartment touched."""
    per_node_day = 2 * (4 * p.n_comp + 8)
    node_days = p.n_nodes * p.n_rep * day_launches
    ev_bytes = 0
    for kind, n in ev_counts_by_kind.items():
        width = {0: 2, 1: 1, 2: 4, 3: 4}[kind] if p.n_comp == 6 else {0: 2, 1: 1, 2: 2, 3: 4}[kind]
        ev_bytes += n * p.n_rep * (20 + 8 * width)
    return node_days * per_node_day, ev_bytes, per_node_day


def counter_traffic(kernel, workload):
    """HBM bytes per launch of kernel from the committed rocprofv3 counter
    summary of the workload (FETCH_SIZE and WRITE_SIZE scaled by a copy of
    known size), or None if there is none or the kernel source changed since
    the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_counters_{workload.replace('-', '_')}.txt")
    src = os.path.join(ROOT, "paper_1502_02908_amd", "csrc", "episim_device.hip")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip().split()[0] if v.strip() else ""
    now = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if fields.get("source_sha256") != now:
        return None
    v = fields.get(f"traffic_bytes_per_launch {kernel}")
    return int(v) if v else None


def counter_occupancy(tag):
    """Occupancy and VALU use of a day kernel from the committed rocprofv3 SQ
    counter summary (the run named tag), or None if there is none or the
    kernel source changed since the counters were taken. SQ_WAVE_CYCLES and
    SQ_ACTIVE_INST_VALU count in units of 4 clocks over the device,
    GRBM_GUI_ACTIVE the busy clocks of each of the 8 XCDs."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "sq_counters_day_kernels.txt")
    src = os.path.join(ROOT, "paper_1502_02908_amd", "csrc", "episim_device.hip")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    now = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if f"source_sha256: {now}" not in text:
        return None
    for line in text.splitlines():
        if line.startswith(f"  {tag} ") and ":" in line:
            v = {k: float(x) for k, x in (kv.split("=") for kv in line.split(":", 1)[1].split())}
            waves = 4 * v["SQ_WAVE_CYCLES"] / (v["GRBM_GUI_ACTIVE"] / 8) / 1024
            per_wave = v["SQ_ACTIVE_INST_VALU"] / v["SQ_WAVE_CYCLES"]
            return dict(resident_waves_per_simd=round(waves, 3),
                        valu_issue_share_per_simd=round(waves * per_wave, 3),
                        active_lanes=round(v["SQ_THREAD_CYCLES_VALU"] / (64 * v["SQ_ACTIVE_INST_VALU"]), 3),
                        wait_share=round(v["SQ_WAIT_ANY"] / v["SQ_WAVE_CYCLES"], 3),
                        source="profiles/sq_counters_day_kernels.txt")
    return None


# Clock of the MI355X compute units (2.4 GHz peak engine clock) and its VALU
# width: 256 compute units x 4 SIMDs x 16 lanes issue one lane-operation per
# cycle each (binary64 add/mul and int32 operations alike), 39.3e12 per
# second; the fp64 vector peak of 78.6 TFLOP/s counts a fused multiply-add
# as two.
CLOCK_GHZ = 2.4
VALU_PEAK_OPS = 256 * 4 * 16 * CLOCK_GHZ * 1e9
# Lane-operations one SSA attempt of the SISe3 / S<->I models requires: a
# Philox4x32-10 block (10 rounds of two 32x32->64 products, low and high
# word, and four xors, plus 18 key additions: 98), two 53-bit uniforms (10),
# -log(u) (bit split and fold 7, (m-1)/(m+1) with a division of about 10
# operations, ten Horner steps of a multiply and an add, and the
# reconstruction: 50), the waiting time (a division: 10) and the clock test
# (2), the target (1), the inversion over the running sums (12), the state
# update (2) and the dependent rates with the re-summed lambda (11).
OPS_PER_ATTEMPT = 98 + 10 + 50 + 10 + 2 + 1 + 12 + 2 + 11


def chain_probe(P, synth, torch, half=1000, days=40, n_nodes=1, classes=1):
    """Time per attempt of one long chain (the serial critical path of a
    plain step): the synthetic model of Sec. 4.2 with one node of S = I =
    half (lambda = 2 half per day, no events) among n_nodes - 1 empty ones,
    its day kernel's duration less that of the same network with no
    animals, over the attempts of a day (transitions + 1). classes = 3 runs
    the same dynamics on the SISe3 compartments (S_j = I_j = half / 3 in each
    class), so the chain walks the six-compartment model as the farm
    networks' herds do. With one node the chain is walked by a wavefront;
    from 8192 nodes on, the largest herd has a workgroup as on the farm
    networks (the block walk fed by a second wavefront, and the workgroup walk
    while the chain expects 4096 attempts or more)."""
    import numpy as np

    def day_us(S0):
        if classes == 3:
            p = synth.flip_classes(n_nodes=n_nodes, S0=0, I0=0, n_days=days)
            row = [S0 // 3] * 6
        else:
            p = synth.flip_model(n_nodes=n_nodes, S0=0, I0=0, n_days=days)
            row = [S0, S0]
        p.u0 = np.ascontiguousarray(p.u0)
        p.u0[0] = row
        with P.Simulator(p) as sim:
            sim.run(0)
            sim.sync()
            sim.set_state(p.u0[None], p.v0[None], 0)
            sim.kernel_times(-1)
            sim.kernel_times(1)
            sim.run(0)
            kt = sim.kernel_times(0)
            trans = int(sim.trajectory()["transitions"].sum())
        ms, n = kt["day"]
        return ms * 1e3 / n, trans / days
    t_big, per_day = day_us(half)
    t_empty, _ = day_us(0)
    us = (t_big - t_empty) / (per_day + 1.0)
    where = "one node" if n_nodes == 1 else f"one node of {n_nodes}"
    model = ("the synthetic S<->I model" if classes == 1 else
             "the synthetic S<->I dynamics on the six SISe3 compartments")
    size = f"S = I = {half}" if classes == 1 else f"S_j = I_j = {half // 3}"
    return dict(us_per_attempt=us, cycles_per_attempt=us * 1e3 * CLOCK_GHZ, attempts_per_day=per_day + 1.0,
                day_kernel_us=t_big, empty_day_kernel_us=t_empty,
                probe=f"{where} of {model} with {size}, {days} days")


def tuned(p, start_day, window, enabled):
    """The tuner's choice of device options for p (timed candidates over a
    window of days from a mid-horizon state), or the defaults."""
    if not enabled:
        return {}, None
    from paper_1502_02908_amd.tune import autotune
    t0 = time.perf_counter()
    t = autotune(p, start_day=start_day, window=window,
                 log=lambda line: print(f"[bench] tuner {line}", file=sys.stderr, flush=True))
    summary = t.summary()
    summary["seconds"] = round(time.perf_counter() - t0, 1)
    print(f"[bench] tuner: {t.best} ({summary['seconds']} s)", file=sys.stderr, flush=True)
    return t.best, summary


def batched_leg(P, synth, torch, steps, plain_sample, tune=True):
    """Trajectories per second, batched against the plain per-trajectory loop:
    256 replicates of the 37k-node network over its first 730 days, each with
    its own (upsilon_1..3, gamma_1..3, beta_1..4) drawn from the prior box, in
    one handle (replicate tiles, options chosen by the tuner), against the
    same trajectories run one handle and one launch sequence each (timed on
    plain_sample of them)."""
    import numpy as np
    R = 256
    pb = synth.batched_replicates(R=R, n_days=730, seed=4)
    base = pb.with_replicates(1)
    coef, alpha, beta, rid = pb.coef, pb.alpha, pb.beta, pb.replicate_id
    best, tuning = tuned(pb, 365, 20, tune)
    sim = P.Simulator(pb, **best)
    u0 = np.tile(pb.u0[None], (R, 1, 1))
    v0 = np.tile(pb.v0[None], (R, 1))
    times = []
    for k in range(steps + 1):
        sim.set_state(u0, v0, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(0)
        sim.sync()
        torch.cuda.synchronize()
        if k > 0:
            times.append(time.perf_counter() - t0)
        print(f"[bench] batched {R} replicates: {(time.perf_counter() - t0) * 1e3:.1f} ms", file=sys.stderr, flush=True)
    trans = int(sim.trajectory()["transitions"].sum())
    # the tile kernel's launches, timed with HIP events on the launch stream
    sim.kernel_times(-1)
    sim.kernel_times(1)
    sim.set_state(u0, v0, 0)
    sim.run(0)
    kt = sim.kernel_times(0)
    sim.close()
    t_batch = sum(times) / len(times)
    day_ms, day_n = kt["day"]
    avg_s = day_ms / 1e3 / day_n
    per_launch = R * base.n_nodes * 2 * (4 * base.n_comp + 8)
    attempts = trans + R * base.n_nodes * base.n_days   # at most one rejected attempt per node-day
    ops_per_launch = attempts * OPS_PER_ATTEMPT / day_n
    roofline = dict(bound="hbm", achieved=round(per_launch / avg_s / 1e9, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(per_launch / avg_s / 1e9 / HBM_PEAK_GBS, 5), traffic=None, kernel="day (replicate tiles)",
                    avg_launch_us=round(avg_s * 1e6, 2),
                    per_unit=f"64 B per replicate-node-day x {R * base.n_nodes} per launch",
                    alu=dict(achieved=round(ops_per_launch / avg_s / 1e12, 3), peak=round(VALU_PEAK_OPS / 1e12, 2),
                             unit="T lane-ops/s", frac=round(ops_per_launch / avg_s / VALU_PEAK_OPS, 4),
                             per_unit=f"{OPS_PER_ATTEMPT} lane-ops per SSA attempt, attempts <= transitions + "
                                      f"node-days"))
    if R == 256 and base.n_days == 730 and base.n_nodes == 37000 and not best:
        roofline["traffic"] = counter_traffic("k_day_tile", "batched-256x730")
        roofline["occupancy"] = counter_occupancy("sq_batched")
    roofline["binding"] = ("issue and latency of the chains' dependent binary64 arithmetic at the resident waves "
                           "the kernel's 168 VGPRs allow (3 per SIMD), not HBM")
    plain = []
    pick = np.linspace(0, R - 1, plain_sample).astype(int)
    for r in pick:
        one = base.with_replicates(1, coef=coef[r:r + 1], alpha=alpha[r:r + 1], beta=beta[r:r + 1],
                                   replicate_id=rid[r:r + 1])
        with P.Simulator(one) as s1:
            s1.run(0)           # warm-up of this handle
            s1.sync()
            s1.set_state(one.u0[None], one.v0[None], 0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s1.run(0)
            s1.sync()
            torch.cuda.synchronize()
            plain.append(time.perf_counter() - t0)
    t_plain = sum(plain) / len(plain)
    return dict(
        workload=f"{R} replicates with prior-box parameters of the 37,000-node network, 730 days",
        replicates_per_s=round(R / t_batch, 3),
        ms_per_batch=round(t_batch * 1e3, 2),
        node_days_per_s=round(R * base.n_nodes * base.n_days / t_batch, 1),
        transitions_per_s=round(trans / t_batch, 1),
        plain_replicates_per_s=round(1.0 / t_plain, 3),
        plain_sample=f"{plain_sample} of the {R} trajectories, one handle and one per-day launch sequence each",
        speedup_vs_plain=round(t_plain / t_batch * R, 2), roofline=roofline, options=best, tuning=tuning)


def instances_leg(P, synth, torch, n_inst=64, days=730):
    """Uneven instances: 64 SISe3 networks with node counts log-uniform in
    [1e3, 2e5] (seeds 4000 + j), one trajectory each with its own prior-box
    parameters, over 730 days, packed into one handle against the same
    instances run one handle each."""
    import numpy as np
    sizes = synth.uneven_sizes(n_inst, seed=4)
    t0 = time.perf_counter()
    insts = synth.uneven_instances(n_inst, n_days=days, seed=4)
    print(f"[bench] {n_inst} instances ({int(sizes.sum())} nodes) generated in {time.perf_counter() - t0:.0f} s",
          file=sys.stderr, flush=True)
    sim = P.Simulator(insts)
    u0 = np.concatenate([q.u0 for q in insts])[None]
    v0 = np.concatenate([q.v0 for q in insts])[None]
    times = []
    for k in range(3):
        sim.set_state(u0, v0, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(0)
        sim.sync()
        torch.cuda.synchronize()
        if k > 0:
            times.append(time.perf_counter() - t0)
    sim.close()
    t_pack = min(times)
    t_plain = 0.0
    for q in insts:
        with P.Simulator(q) as s1:
            s1.run(0)
            s1.sync()
            s1.set_state(q.u0[None], q.v0[None], 0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s1.run(0)
            s1.sync()
            torch.cuda.synchronize()
            t_plain += time.perf_counter() - t0
    nd = float(sizes.sum()) * days
    return dict(workload=f"{n_inst} SISe3 instances, {int(sizes.min())}-{int(sizes.max())} nodes "
                         f"({int(sizes.sum())} in all), 1 trajectory each, {days} days",
                instances_per_s=round(n_inst / t_pack, 3), ms_packed=round(t_pack * 1e3, 2),
                node_days_per_s=round(nd / t_pack, 1), plain_ms=round(t_plain * 1e3, 2),
                speedup_vs_plain=round(t_plain / t_pack, 2))


def serving_leg(P, synth, torch, rate, seconds, budget_gb, slot_lanes=16):
    """Requests over the three resident serving networks (1k, 37k and 250k
    nodes, 1461 days): Poisson arrivals at `rate` per second for `seconds`,
    horizons 365-1461 days, 1-64 replicates with prior-box parameters."""
    import numpy as np
    from paper_1502_02908_amd.serve import Server, plan_slots
    t0 = time.perf_counter()
    nets = synth.serving_networks()
    reqs = synth.serving_requests(rate=rate, duration=seconds, seed=5)
    print(f"[bench] serving: networks generated in {time.perf_counter() - t0:.0f} s, {len(reqs)} requests",
          file=sys.stderr, flush=True)
    demand = [net.n_nodes for net in nets]  # requests pick networks uniformly
    slots, nbytes = plan_slots(nets, budget_gb * 2 ** 30, demand, slot_lanes=slot_lanes)
    srv = Server(nets, slots, max_ahead=4, slot_lanes=slot_lanes)
    last = [time.perf_counter()]

    def progress(j, k):
        if time.perf_counter() - last[0] > 10:
            last[0] = time.perf_counter()
            print(f"[bench] serving: network {j} step {k}", file=sys.stderr, flush=True)
    try:
        results, stats = srv.serve(reqs, on_step=progress)
    finally:
        srv.close()
    out = stats.summary(results)
    work = np.mean([nets[q["net"]].n_nodes * q["horizon"] * q["n_rep"] for q in reqs])
    # the offered load in replicate-node-days per second, against which
    # node_days_per_s (what the day kernels got through) is the bound
    out.update(offered_rate=rate, arrival_seconds=seconds, hbm_budget_gb=budget_gb, slot_lanes=slot_lanes,
               slot_bytes_gb=[round(b / 2 ** 30, 2) for b in nbytes],
               mean_request_node_days=float(work), offered_node_days_per_s=float(work) * rate,
               errors=sum(r.error is not None for r in results))
    return out


def slot_capacity(P, synth, torch, slot_lanes=16, warm=200, steps=60, budget_gb=96.0):
    """Throughput of the slot step with every slot of a serving network busy
    and all slots at one day (from day `warm` on), one network at a time:
    the device-side bound of the serving leg, and how much of a step's wall
    time the host leaves the device idle."""
    import numpy as np
    from paper_1502_02908_amd.serve import plan_slots
    nets = synth.serving_networks()
    slots, _ = plan_slots(nets, budget_gb * 2 ** 30, [net.n_nodes for net in nets], slot_lanes=slot_lanes)
    out = []
    for net, n in zip(nets, slots):
        st = torch.cuda.Stream()  # default priority
        h = P.SlotHandle(net, n, stream=st.cuda_stream, slot_lanes=slot_lanes)
        coef, alpha, beta = synth.prior_draws(slot_lanes, seed=9)
        for k in range(h.n_slots):
            h.start(k, net.n_days, coef, alpha, beta, np.arange(slot_lanes, dtype=np.uint32) + np.uint32(k * slot_lanes))

        def run(m):
            for _ in range(m):
                h.step()
                while h.in_flight() > 4:
                    time.sleep(0.0002)
            st.synchronize()
        run(warm)
        h.kernel_times(-1)
        h.kernel_times(1)
        t0 = time.perf_counter()
        run(steps)
        wall = time.perf_counter() - t0
        kt = h.kernel_times(0)
        h.close()
        busy = sum(a for a, b in kt.values() if b) / 1e3
        out.append(dict(nodes=net.n_nodes, slots=n, lanes=n * slot_lanes, ms_per_step=round(wall / steps * 1e3, 3),
                        node_days_per_s=n * slot_lanes * net.n_nodes * steps / wall,
                        device_busy=round(busy / wall, 3)))
        print(f"[bench] slot capacity: {out[-1]}", file=sys.stderr, flush=True)
    return dict(slot_lanes=slot_lanes, from_day=warm, steps=steps, networks=out)


def plan_stats(P, synth, workload):
    """Levels per day of the dependency pass (host side of sim_create) and
    the events of each level, as a histogram over the days."""
    import numpy as np
    from farmnet import EXTERNAL
    p = WORKLOADS[workload]["make"](synth)
    lv, task = P.plan_levels(p.ev_day, p.ev_kind, p.ev_node, p.ev_dest, p.n_nodes, tasks=True)
    D = p.n_days
    per_day = np.zeros(D, np.int64)
    np.maximum.at(per_day, p.ev_day, lv)
    ev_per_day = np.bincount(p.ev_day, minlength=D)
    moves = np.bincount(p.ev_day[p.ev_kind == EXTERNAL], minlength=D)
    print(f"# dependency levels per day, {WORKLOADS[workload]['desc']}: {p.n_events} events, "
          f"{int(task.max()) + 1 if len(task) else 0} tasks")
    print(f"events per day: mean {ev_per_day.mean():.1f}, max {ev_per_day.max()}; "
          f"external transfers per day: mean {moves.mean():.1f}, max {moves.max()}")
    print(f"levels per day: mean {per_day.mean():.2f}, median {np.median(per_day):.0f}, max {per_day.max()}")
    print("levels  days")
    for k, n in enumerate(np.bincount(per_day)):
        if n:
            print(f"{k:6d}  {n}")
    sizes = np.bincount(lv.astype(np.int64) + p.ev_day.astype(np.int64) * (per_day.max() + 1))
    sizes = sizes[sizes > 0]
    print(f"events per (day, level): mean {sizes.mean():.1f}, median {np.median(sizes):.0f}, max {sizes.max()}")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, seconds, runs=5):
    """The oracle on the host over a bounded sample of the workload: a window
    of days from the middle of the horizon (the state at its start computed
    first, untimed, by the oracle itself), timed once on one thread and once
    fork-join over the host's cores (at most 16, the CPU share of one GPU),
    each the median of `runs` runs after a warm-up run. The window is sized
    so that the timed runs take about `seconds` in all."""
    import numpy as np
    from oracle import oracle as O
    cores = max(1, min(os.cpu_count() or 1, 16))
    start = p.n_days // 2
    pre = O.run(p, d_begin=0, d_end=start, threads=cores)
    # size the window from a short probe on one thread
    probe = min(5, p.n_days - start)
    t0 = time.perf_counter()
    O.run(p, d_begin=start, d_end=start + probe, u=pre["u"], v=pre["v"], threads=1)
    per_day_1 = (time.perf_counter() - t0) / probe
    share = seconds / (runs * (1.0 + 1.0 / max(cores / 2.0, 1.0)))
    days = int(max(probe, min(p.n_days - start, share / per_day_1)))

    def leg(threads):
        O.run(p, d_begin=start, d_end=start + days, u=pre["u"], v=pre["v"], threads=threads)  # warm-up
        times, trans = [], 0
        for _ in range(runs):
            t0 = time.perf_counter()
            r = O.run(p, d_begin=start, d_end=start + days, u=pre["u"], v=pre["v"], threads=threads)
            times.append(time.perf_counter() - t0)
            trans = int(r["transitions"].sum())
        med = float(np.median(times))
        nd = p.n_nodes * p.n_rep * days
        return dict(value=nd / med, transitions_per_s=trans / med, median_s=med, runs=runs)

    one = leg(1)
    many = leg(cores)
    return dict(value=many["value"], unit="node-days/s", cores=cores, kind="oracle",
                sample=f"days {start}-{start + days - 1} of {p.n_days} ({p.n_nodes} nodes, state at day {start} "
                       f"from the oracle), median of {runs} runs after a warm-up, fork-join over {cores} threads "
                       f"(SSA and phi node loops; events serial)",
                transitions_per_s=many["transitions_per_s"], cpu_model=cpu_model(), host_threads=os.cpu_count(),
                single_thread=dict(value=one["value"], unit="node-days/s", cores=1,
                                   transitions_per_s=one["transitions_per_s"]))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="sise3-37k", choices=sorted(WORKLOADS))
    ap.add_argument("--launch", default="kernels", choices=["kernels", "persistent"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-replicates leg")
    ap.add_argument("--no-tune", action="store_true", help="default device options instead of the tuner's")
    ap.add_argument("--no-chain-probe", action="store_true",
                    help="leave out the critical-path probe (profiled runs: its launches share the day kernel)")
    ap.add_argument("--options", default="", metavar="JSON",
                    help="device options of the plain leg, e.g. '{\"tile_nodes\": 4}' (no tuner)")
    ap.add_argument("--instances", action="store_true", help="add the 64-uneven-instances leg (slow to generate)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--serving-rate", type=float, default=20.0, help="request arrivals per second")
    ap.add_argument("--serving-seconds", type=float, default=8.0, help="seconds of arrivals")
    ap.add_argument("--serving-budget-gb", type=float, default=96.0, help="HBM budget for the slots")
    ap.add_argument("--serving-slot-lanes", type=int, default=16, choices=[8, 16, 32, 64],
                    help="replicate lanes per slot of the serving handles")
    ap.add_argument("--plain-sample", type=int, default=6)
    ap.add_argument("--slot-capacity", action="store_true",
                    help="only the slot step's throughput with every slot of each serving network busy")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--plan-stats", action="store_true",
                    help="only print the dependency pass's levels per day and events per level (host only)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (profiler calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): the per-node hot path "
              "is measured on a single MI355X. Independent trajectories would shard across GPUs with no "
              "communication; one trajectory would shard by node ranges, exchanging the counts of "
              "cross-range movements once per event level.", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import paper_1502_02908_amd as P
    from farmnet import synth

    if args.plan_stats:
        plan_stats(P, synth, args.workload)
        return
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        # a copy of known size: the hardware counters of the profiled kernels
        # are scaled by what the same counters read for it
        n = args.calibrate_copy // 4
        a = torch.arange(n, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(calibration="copy", bytes_read=n * 4, bytes_written=n * 4, launches=3)))
        return
    if args.slot_capacity:
        print(json.dumps(dict(slot_capacity=slot_capacity(P, synth, torch, args.serving_slot_lanes))))
        return
    wl = WORKLOADS[args.workload]
    p = wl["make"](synth)
    launch = P.LAUNCH_PERSISTENT if args.launch == "persistent" else P.LAUNCH_KERNELS
    print(f"[bench] {wl['desc']}: {p.n_events} events, launch={args.launch}", file=sys.stderr, flush=True)
    if args.options:
        best, tuning = json.loads(args.options), None
    else:
        best, tuning = tuned(p, p.n_days // 2, min(30, p.n_days - p.n_days // 2),
                             not args.no_tune and args.launch == "kernels")
    opts = dict(launch=launch)
    opts.update(best)
    sim = P.Simulator(p, **opts)
    u0 = np.tile(p.u0[None], (p.n_rep, 1, 1))
    v0 = np.tile(p.v0[None], (p.n_rep, 1))

    def one_step():
        sim.run(0)

    for _ in range(args.warmup):
        sim.set_state(u0, v0, 0)
        one_step()
        sim.sync()
    times = []
    for k in range(args.steps):
        sim.set_state(u0, v0, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one_step()
        sim.sync()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        print(f"[bench] step {k}: {times[-1] * 1e3:.2f} ms", file=sys.stderr, flush=True)
    traj = sim.trajectory()
    trans_per_step = int(traj["transitions"].sum())
    most = traj["max_transitions"].max(axis=1).astype(np.int64)   # the day's longest chain
    total = sum(times)
    node_days = p.n_nodes * p.n_days * p.n_rep * args.steps
    value = node_days / total

    # per-kernel durations, HIP events on the launch stream, same configuration
    sim.kernel_times(-1)
    sim.kernel_times(1)
    for _ in range(max(1, min(args.steps, 3))):
        sim.set_state(u0, v0, 0)
        one_step()
    kt = sim.kernel_times(0)
    steps_timed = max(1, min(args.steps, 3))
    dom = max(kt, key=lambda k: kt[k][0])
    dom_ms, dom_n = kt[dom]
    counts = {k: int((p.ev_kind == k).sum()) for k in range(4)}
    nd_bytes, ev_bytes, per_nd = algorithmic_bytes(p, p.n_days, counts)
    if dom == "day":
        bytes_per_launch = p.n_nodes * p.n_rep * per_nd
        unit_desc = f"{per_nd} B per node-day x {p.n_nodes * p.n_rep} node-days per launch"
    elif dom == "persist":
        bytes_per_launch = nd_bytes + ev_bytes
        unit_desc = (f"{per_nd} B per node-day x {p.n_nodes * p.n_days * p.n_rep} node-days + "
                     f"event bytes {ev_bytes} per launch")
    elif dom == "events":
        n_lv = sim.levels()[0]
        bytes_per_launch = ev_bytes / max(n_lv, 1)
        unit_desc = f"event bytes {ev_bytes} over {n_lv} level launches"
    else:
        bytes_per_launch = p.n_nodes * p.n_rep * per_nd / 2
        unit_desc = f"{per_nd // 2} B per node (read) per launch"
    avg_s = dom_ms / 1e3 / dom_n
    achieved = bytes_per_launch / avg_s / 1e9
    # committed counters hold for the default options (or, for occupancy, the
    # options named in the run's tag)
    traffic = counter_traffic("k_day", args.workload) if dom == "day" and not best else None
    roofline = dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 5), traffic=traffic,
                    kernel=dom, avg_launch_us=round(avg_s * 1e6, 3), launches_per_step=dom_n // steps_timed,
                    per_unit=unit_desc)
    kernel_breakdown = {k: dict(ms_per_step=round(v[0] / steps_timed, 4), launches_per_step=v[1] // steps_timed)
                        for k, v in kt.items() if v[1]}
    sim.close()

    # the serial critical path: each day's longest SSA chain at the
    # per-attempt time of a long chain walked as the day kernel walks the
    # largest herd (from 8192 nodes with one lane per node: its own workgroup,
    # the workgroup walk for chains of 4096 expected attempts or more)
    hub_layout = p.n_nodes >= 8192 and p.n_rep == 1 and not best.get("tile_nodes")
    # the probe walks the workload's own rules: three S<->I classes on the
    # six-compartment networks, one on the synthetic model (its launches are
    # those of the step's own day kernel, so profiled runs leave it out)
    classes = 3 if p.n_comp == 6 else 1
    critical = None
    if not args.no_chain_probe:
        if hub_layout:
            short = chain_probe(P, synth, torch, half=1000, n_nodes=8192, classes=classes)
            long_ = chain_probe(P, synth, torch, half=10000, days=20, n_nodes=8192, classes=classes)
            per_day_us = np.where(most + 1 >= 4096, long_["us_per_attempt"], short["us_per_attempt"]) * (most + 1)
            probes = [short, long_]
        else:
            one = chain_probe(P, synth, torch, classes=classes)
            per_day_us = one["us_per_attempt"] * (most + 1)
            probes = [one]
        chain_ms = float(per_day_us.sum()) / 1e3
        step_ms = total / args.steps * 1e3
        critical = dict(longest_chain_attempts_per_step=int((most + 1).sum()),
                        longest_chain_per_day=dict(max=int(most.max()), median=float(np.median(most)),
                                                   p99=float(np.percentile(most, 99))),
                        us_per_attempt=[round(q["us_per_attempt"], 5) for q in probes],
                        cycles_per_attempt=[round(q["cycles_per_attempt"], 1) for q in probes],
                        chain_ms_per_step=round(chain_ms, 3), step_ms=round(step_ms, 3),
                        frac=round(chain_ms / step_ms, 4), probe=[q["probe"] for q in probes],
                        rule="longest chains of 4096 attempts or more at the second probe's rate" if hub_layout else "")
    roofline["binding"] = ("serial SSA chain of the day's largest herd (critical_path.frac of the step), "
                           "not HBM")
    tag = {"sise3-37k": "sq_37k", "sise3-1m": "sq_1m", "sise3-37k-u10": "sq_u10",
           "synthetic-1k": "sq_synthetic"}.get(args.workload, "")
    if tag and best:
        tag += "_" + "_".join(f"{k}{v}" for k, v in sorted(best.items()))
    roofline["occupancy"] = counter_occupancy(tag) if tag else None
    # SSA-heavy workloads: VALU lane-operations of the attempts against the VALU peak
    alu = None
    if args.workload in ("synthetic-1k", "sise3-37k-u10"):
        attempts = trans_per_step + p.n_nodes * p.n_rep * p.n_days   # at most one rejected attempt per node-day
        day_s = kt["day"][0] / 1e3 / steps_timed
        ops = attempts * OPS_PER_ATTEMPT
        alu = dict(bound="alu", achieved=round(ops / day_s / 1e12, 4), peak=round(VALU_PEAK_OPS / 1e12, 2),
                   unit="T lane-ops/s", frac=round(ops / day_s / VALU_PEAK_OPS, 5), traffic=None,
                   kernel="day", per_unit=f"{OPS_PER_ATTEMPT} lane-ops per SSA attempt x {attempts} attempts "
                                          f"(transitions + node-days) per step, over the day kernels' time")

    batched = None
    if not args.no_batched and args.workload == "sise3-37k":
        batched = batched_leg(P, synth, torch, max(1, min(args.steps, 3)), args.plain_sample, not args.no_tune)

    instances = instances_leg(P, synth, torch) if args.instances else None
    serving = (serving_leg(P, synth, torch, args.serving_rate, args.serving_seconds, args.serving_budget_gb,
                           args.serving_slot_lanes)
               if not args.no_serving and args.workload == "sise3-37k" else None)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(p, args.cpu_seconds)
        cpu = {k: (round(v, 1) if isinstance(v, float) else v) for k, v in cpu.items()}

    line = dict(
        metric="SISe3 node-days/s + SSA transitions/s at 37k nodes; batched replicates/s vs plain",
        value=round(value, 1), unit="node-days/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(total / args.steps * 1e3, 3), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload=wl["desc"], nodes=p.n_nodes, days=p.n_days, replicates=p.n_rep,
                    events=p.n_events, launch=args.launch, options=best, step="one full-horizon simulation"),
        transitions_per_s=round(trans_per_step * args.steps / total, 1),
        transitions_per_step=trans_per_step,
        roofline=roofline, critical_path=critical, kernels=kernel_breakdown, tuning=tuning, batched=batched,
        cpu_baseline=cpu)
    if alu:
        line["alu_roofline"] = alu
    if instances:
        line["instances"] = instances
    if serving:
        line["serving"] = serving
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
