"""Helpers for the GPU parity tests: run a problem through the C ABI and
through the oracle on the same seeded input, and compare."""
import sys

import numpy as np

import paper_1502_02908_amd as P
from oracle import oracle as O

# phi tolerance: relative 1e-12 (the aim, and what the tests observe, is
# bit-identity: both sides run the same binary64 operations in the same order)
PHI_RTOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_run(p, chunks=None, **kw):
    """Run p on the GPU (optionally in chunks of days); return state + records."""
    with P.Simulator(p, **kw) as sim:
        if chunks:
            for n in chunks:
                sim.run(n)
        else:
            sim.run(0)
        out = sim.trajectory()
        u, v, day = sim.get_state()
        out.update(u=u, v=v, day=day)
        out["levels"] = sim.levels()
    return out


def first_mismatch(a, b):
    idx = np.argwhere(a != b)
    return None if len(idx) == 0 else (tuple(idx[0]), a[tuple(idx[0])], b[tuple(idx[0])], len(idx))


def assert_parity(g, o, check_phi_bits=True):
    for k in ("u", "prevalence", "transitions", "totals", "snap_u", "max_transitions"):
        a, b = np.asarray(g[k]), np.asarray(o[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        mm = first_mismatch(a, b)
        assert mm is None, f"{k}: first mismatch at {mm[0]}: gpu {mm[1]} oracle {mm[2]} ({mm[3]} differ)"
    for k in ("v", "snap_v"):
        a, b = np.asarray(g[k]), np.asarray(o[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        denom = np.maximum(np.abs(b), 1e-300)
        rel = np.where((a == b), 0.0, np.abs(a - b) / denom)
        assert rel.max(initial=0.0) <= PHI_RTOL, f"{k}: max relative difference {rel.max()}"
        if check_phi_bits:
            mm = first_mismatch(a.view(np.int64), b.view(np.int64))
            assert mm is None, f"{k}: not bit-identical at {mm[0]} ({mm[3]} differ)"
