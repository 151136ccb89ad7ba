"""ctypes binding of the episim C ABI (include/episim.h).

Argument marshalling only: every step of the simulation runs in the gfx950
library. PyTorch, when present, provides the stream (torch's current stream)
and owns the device workspace (a uint8 tensor), so the library's memory shows
up in torch's allocator. There is no CPU fallback: without the built library
every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libepisim.so")

SIM_OK, SIM_EINVAL, SIM_ENOMEM, SIM_EDEVICE, SIM_EINFEASIBLE, SIM_ESTATE, SIM_ELIMIT = 0, -1, -2, -3, -4, -5, -6
EVENTS_LEVELS, EVENTS_SERIAL = 0, 1
LAUNCH_KERNELS, LAUNCH_PERSISTENT = 0, 1

_i32p = C.POINTER(C.c_int32)
_u32p = C.POINTER(C.c_uint32)
_i64p = C.POINTER(C.c_int64)
_f64p = C.POINTER(C.c_double)


class sim_problem(C.Structure):
    _fields_ = [
        ("n_nodes", C.c_int32), ("n_comp", C.c_int32), ("n_trans", C.c_int32), ("n_rep", C.c_int32),
        ("n_days", C.c_int32), ("day0", C.c_int32),
        ("u0", _i32p), ("v0", _f64p),
        ("S", _i32p), ("reactant", _i32p), ("uses_phi", _i32p),
        ("coef", _f64p), ("alpha", _f64p), ("beta", _f64p),
        ("phi_I_mask", C.c_uint32), ("phi_N_mask", C.c_uint32),
        ("n_select", C.c_int32), ("E", _i32p),
        ("n_shift", C.c_int32), ("N", _i32p),
        ("n_events", C.c_int64),
        ("ev_day", _i32p), ("ev_kind", _i32p), ("ev_node", _i32p), ("ev_dest", _i32p),
        ("ev_n", _i32p), ("ev_select", _i32p), ("ev_shift", _i32p),
        ("n_record", C.c_int32), ("record_days", _i32p),
        ("seed", C.c_uint32), ("replicate_id", _u32p),
        ("reactant2", _i32p), ("phi_pre_events", C.c_int32),
        ("n_regions", C.c_int32), ("region", _i32p),
    ]


class sim_device_opts(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("events_mode", C.c_int32), ("block", C.c_int32), ("launch", C.c_int32),
                ("group_herds", C.c_int32), ("small_level", C.c_int32),
                ("tile_nodes", C.c_int32), ("heavy_herds", C.c_int32), ("few_chains", C.c_int32),
                ("group_min_attempts", C.c_int32), ("slot_lanes", C.c_int32)]
# device options a handle takes (every setting gives the same results)
OPTION_NAMES = ("events_mode", "launch", "group_herds", "small_level", "tile_nodes", "heavy_herds",
                "few_chains", "group_min_attempts")


class sim_output(C.Structure):
    _fields_ = [("prevalence", _i32p), ("transitions", _i64p), ("totals", _i64p),
                ("snap_u", _i32p), ("snap_v", _f64p), ("regional", _i64p), ("max_transitions", _i32p)]


# every symbol of include/episim.h with its C signature
SIGNATURES = {
    "sim_workspace_bytes": (C.c_size_t, [C.POINTER(sim_problem), C.POINTER(sim_device_opts)]),
    "sim_create": (C.c_int, [C.POINTER(sim_problem), C.POINTER(sim_device_opts), C.POINTER(C.c_void_p)]),
    "sim_run": (C.c_int, [C.c_void_p, C.c_int32]),
    "sim_sync": (C.c_int, [C.c_void_p]),
    "sim_trajectory": (C.c_int, [C.c_void_p, C.POINTER(sim_output)]),
    "sim_get_state": (C.c_int, [C.c_void_p, _i32p, _f64p, _i32p]),
    "sim_set_state": (C.c_int, [C.c_void_p, _i32p, _f64p, C.c_int32]),
    "sim_levels": (C.c_int64, [C.c_void_p, C.c_int32, _i32p]),
    "sim_destroy": (None, [C.c_void_p]),
    "sim_last_error": (C.c_char_p, [C.c_void_p]),
    "sim_plan_levels": (C.c_int, [C.c_int64, _i32p, _i32p, _i32p, _i32p, C.c_int32, _i32p, _i32p]),
    "sim_kernel_times": (C.c_int, [C.c_void_p, C.c_int32, _f64p, _i64p]),
    "sim_goal": (C.c_int, [C.c_void_p, C.c_int32, _i64p, C.c_int32, C.c_int32, _f64p, _f64p]),
    "sim_goal_noalloc": (C.c_int, [C.c_void_p, C.c_int32, _i64p, C.c_int32, C.c_int32, _f64p, _f64p]),
    "sim_create_batch": (C.c_int, [C.POINTER(C.POINTER(sim_problem)), C.c_int32, C.POINTER(sim_device_opts),
                                   C.POINTER(C.c_void_p)]),
    "sim_workspace_bytes_batch": (C.c_size_t, [C.POINTER(C.POINTER(sim_problem)), C.c_int32,
                                               C.POINTER(sim_device_opts)]),
    "sim_slots_workspace_bytes": (C.c_size_t, [C.POINTER(sim_problem), C.c_int32, C.POINTER(sim_device_opts)]),
    "sim_slots_create": (C.c_int, [C.POINTER(sim_problem), C.c_int32, C.POINTER(sim_device_opts),
                                   C.POINTER(C.c_void_p)]),
    "sim_slot_start": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, _f64p, _f64p, _f64p, _u32p]),
    "sim_slots_step": (C.c_int, [C.c_void_p, _i32p, _i32p]),
    "sim_slots_in_flight": (C.c_int32, [C.c_void_p]),
    "sim_slot_fetch": (C.c_int, [C.c_void_p, C.c_int32, _i32p, _i64p, _i64p]),
    "sim_slot_query": (C.c_int, [C.c_void_p, C.c_int32]),
    "sim_slot_state": (C.c_int, [C.c_void_p, C.c_int32, _i32p, _f64p]),
}
KERNEL_CLASSES = ("day", "events", "close", "persist")

_lib = None


def lib():
    """The built library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1502_02908_amd.build` "
                               "(hipcc, gfx950); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class SimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"episim error {code}: {msg}")
        self.code = code


def _p(a, t):
    return a.ctypes.data_as(t)


def _marshal(p):
    """sim_problem for a farmnet.Problem-like object; returns (struct, keepalive)."""
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    f64 = lambda a: np.ascontiguousarray(a, dtype=np.float64)
    arr = dict(u0=i32(p.u0), v0=f64(p.v0), S=i32(p.S), reactant=i32(p.reactant), uses_phi=i32(p.uses_phi),
               coef=f64(p.coef), alpha=f64(p.alpha), beta=f64(p.beta), E=i32(p.E), N=i32(p.N),
               ev_day=i32(p.ev_day), ev_kind=i32(p.ev_kind), ev_node=i32(p.ev_node), ev_dest=i32(p.ev_dest),
               ev_n=i32(p.ev_n), ev_select=i32(p.ev_select), ev_shift=i32(p.ev_shift),
               record_days=i32(p.record_days if p.record_days is not None else np.zeros(0)),
               replicate_id=np.ascontiguousarray(p.replicate_id, dtype=np.uint32))
    r2 = getattr(p, "reactant2", None)
    arr["reactant2"] = None if r2 is None else i32(r2)
    n_regions = int(getattr(p, "n_regions", 0) or 0)
    arr["region"] = i32(p.region) if n_regions > 0 else None
    s = sim_problem(
        p.n_nodes, p.n_comp, p.n_trans, p.n_rep, p.n_days, getattr(p, "day0", 0),
        _p(arr["u0"], _i32p), _p(arr["v0"], _f64p),
        _p(arr["S"], _i32p), _p(arr["reactant"], _i32p), _p(arr["uses_phi"], _i32p),
        _p(arr["coef"], _f64p), _p(arr["alpha"], _f64p), _p(arr["beta"], _f64p),
        p.phi_I_mask, p.phi_N_mask,
        arr["E"].shape[1] if arr["E"].ndim == 2 else 0, _p(arr["E"], _i32p),
        arr["N"].shape[1] if arr["N"].ndim == 2 else 0, _p(arr["N"], _i32p),
        len(arr["ev_day"]),
        _p(arr["ev_day"], _i32p), _p(arr["ev_kind"], _i32p), _p(arr["ev_node"], _i32p),
        _p(arr["ev_dest"], _i32p), _p(arr["ev_n"], _i32p), _p(arr["ev_select"], _i32p),
        _p(arr["ev_shift"], _i32p),
        len(arr["record_days"]), _p(arr["record_days"], _i32p),
        int(p.seed) & 0xFFFFFFFF, _p(arr["replicate_id"], _u32p),
        None if arr["reactant2"] is None else _p(arr["reactant2"], _i32p), int(getattr(p, "phi_pre_events", 0)),
        n_regions, None if arr["region"] is None else _p(arr["region"], _i32p))
    return s, arr


def workspace_bytes(p, **opts):
    """Device bytes of a handle for p with the given device options (0 if rejected)."""
    s, keep = _marshal(p)
    o = sim_device_opts()
    for k, v in opts.items():
        if k not in OPTION_NAMES:
            raise TypeError(f"unknown device option {k}")
        setattr(o, k, int(v))
    return int(lib().sim_workspace_bytes(C.byref(s), C.byref(o)))


def plan_levels(ev_day, ev_kind, ev_node, ev_dest, n_nodes, tasks=False):
    """Host dependency pass (no GPU needed): the level of each event within its
    day, and with tasks=True also the task of each event."""
    a = [np.ascontiguousarray(x, dtype=np.int32) for x in (ev_day, ev_kind, ev_node, ev_dest)]
    out = np.zeros(len(a[0]), np.int32)
    task = np.zeros(len(a[0]), np.int32)
    rc = lib().sim_plan_levels(len(out), *[_p(x, _i32p) for x in a], int(n_nodes), _p(out, _i32p),
                               _p(task, _i32p))
    if rc != SIM_OK:
        raise SimError(rc, "sim_plan_levels rejected its input")
    return (out, task) if tasks else out


def _torch_cuda():
    try:
        import torch
        return torch if torch.cuda.is_available() else None
    except Exception:
        return None


class Simulator:
    """One handle: one network (or several packed instances of one model),
    R replicates each, state on the device."""

    def __init__(self, p, *, events_mode=EVENTS_LEVELS, launch=LAUNCH_KERNELS, stream=None,
                 torch_workspace=True, device=0, group_herds=0, small_level=0, tile_nodes=0,
                 heavy_herds=0, few_chains=0, group_min_attempts=0):
        probs = list(p) if isinstance(p, (list, tuple)) else [p]
        self.p = probs[0]
        self.n_inst = len(probs)
        self.R, self.Nc, self.D = probs[0].n_rep, probs[0].n_comp, probs[0].n_days
        self.Nn = sum(q.n_nodes for q in probs)
        self.node_counts = [q.n_nodes for q in probs]
        self.n_record = 0 if probs[0].record_days is None else len(probs[0].record_days)
        self.n_regions = int(getattr(probs[0], "n_regions", 0) or 0)
        self._h = C.c_void_p()
        self._ws = None
        torch = _torch_cuda()
        structs, keep = zip(*[_marshal(q) for q in probs])
        arr = (C.POINTER(sim_problem) * len(structs))(*[C.pointer(st) for st in structs])
        self.opts = dict(events_mode=events_mode, launch=launch, group_herds=group_herds, small_level=small_level,
                         tile_nodes=tile_nodes, heavy_herds=heavy_herds,
                         few_chains=few_chains, group_min_attempts=group_min_attempts)
        opts = sim_device_opts()
        for k, v in self.opts.items():
            setattr(opts, k, int(v))
        if torch is not None:
            torch.cuda.set_device(device)
            if stream is None:
                stream = torch.cuda.current_stream().cuda_stream
            if torch_workspace:
                nbytes = int(lib().sim_workspace_bytes_batch(arr, len(structs), C.byref(opts)))
                if nbytes == 0:
                    raise SimError(SIM_EINVAL, "problem rejected (sim_workspace_bytes returned 0)")
                self._ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{device}")
                opts.workspace = self._ws.data_ptr()
                opts.workspace_bytes = nbytes
        opts.stream = stream if stream is not None else None
        rc = lib().sim_create_batch(arr, len(structs), C.byref(opts), C.byref(self._h))
        del keep
        if rc != SIM_OK:
            raise SimError(rc, lib().sim_last_error(None).decode())

    def _check(self, rc):
        if rc != SIM_OK:
            raise SimError(rc, lib().sim_last_error(self._h).decode())

    def run(self, n_days=0):
        self._check(lib().sim_run(self._h, int(n_days)))
        return self

    def sync(self):
        self._check(lib().sim_sync(self._h))

    def trajectory(self):
        """Daily records [D][set] (set = instance * R + replicate), snapshots,
        and with regions the regional sums [D][set][region][compartment]."""
        D, R, Nc, Nn, K = self.D, self.R, self.Nc, self.Nn, self.n_record
        S = self.n_inst * R
        out = dict(prevalence=np.zeros((D, S), np.int32), transitions=np.zeros((D, S), np.int64),
                   totals=np.zeros((D, S, Nc), np.int64), snap_u=np.zeros((K, R, Nn, Nc), np.int32),
                   snap_v=np.zeros((K, R, Nn), np.float64), max_transitions=np.zeros((D, S), np.int32))
        if self.n_regions:
            out["regional"] = np.zeros((D, S, self.n_regions, Nc), np.int64)
        o = sim_output(_p(out["prevalence"], _i32p), _p(out["transitions"], _i64p), _p(out["totals"], _i64p),
                       _p(out["snap_u"], _i32p), _p(out["snap_v"], _f64p),
                       _p(out["regional"], _i64p) if self.n_regions else None, _p(out["max_transitions"], _i32p))
        self._check(lib().sim_trajectory(self._h, C.byref(o)))
        return out

    def goal(self, reference, instance=0, d_begin=0, d_end=None):
        """(G2, VG2) of instance's R replicates against reference[D][region][compartment]
        (the regional sums of the reference trajectory) over days [d_begin, d_end)."""
        ref = np.ascontiguousarray(reference, dtype=np.int64)
        if ref.shape != (self.D, self.n_regions, self.Nc):
            raise ValueError(f"reference must have shape {(self.D, self.n_regions, self.Nc)}")
        g, vg = C.c_double(), C.c_double()
        d_end = self.D if d_end is None else d_end
        self._check(lib().sim_goal(self._h, int(instance), _p(ref, _i64p), int(d_begin), int(d_end),
                                   C.byref(g), C.byref(vg)))
        return g.value, vg.value

    def goal_noalloc(self, reference, instance=0, d_begin=0, d_end=None):
        """goal() through sim_goal_noalloc: the library's static device array
        instead of the handle's workspace (nothing allocated)."""
        ref = np.ascontiguousarray(reference, dtype=np.int64)
        if ref.shape != (self.D, self.n_regions, self.Nc):
            raise ValueError(f"reference must have shape {(self.D, self.n_regions, self.Nc)}")
        g, vg = C.c_double(), C.c_double()
        d_end = self.D if d_end is None else d_end
        self._check(lib().sim_goal_noalloc(self._h, int(instance), _p(ref, _i64p), int(d_begin), int(d_end),
                                           C.byref(g), C.byref(vg)))
        return g.value, vg.value

    def get_state(self):
        u = np.zeros((self.R, self.Nn, self.Nc), np.int32)
        v = np.zeros((self.R, self.Nn), np.float64)
        day = C.c_int32()
        self._check(lib().sim_get_state(self._h, _p(u, _i32p), _p(v, _f64p), C.byref(day)))
        return u, v, day.value

    def set_state(self, u, v, day):
        u = np.ascontiguousarray(u, dtype=np.int32).reshape(self.R, self.Nn, self.Nc)
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(self.R, self.Nn)
        self._check(lib().sim_set_state(self._h, _p(u, _i32p), _p(v, _f64p), int(day)))

    def levels(self, day=-1):
        mx = C.c_int32()
        n = lib().sim_levels(self._h, int(day), C.byref(mx))
        return int(n), mx.value

    def kernel_times(self, enable):
        """enable 1/0/-1: start, stop, clear bracketing of launches; returns
        {class: (total ms, launches)}."""
        ms = np.zeros(4)
        n = np.zeros(4, np.int64)
        self._check(lib().sim_kernel_times(self._h, int(enable), _p(ms, _f64p), _p(n, _i64p)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def close(self):
        if self._h:
            lib().sim_destroy(self._h)
            self._h = C.c_void_p()
        self._ws = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr(x, t):
    """Pointer to a numpy array or a torch CPU tensor (None -> NULL)."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return C.cast(C.c_void_p(x.data_ptr()), t)
    return x.ctypes.data_as(t)


class SlotHandle:
    """One resident network with n_slots slots of slot_lanes (8, 16, 32 or 64)
    replicate lanes; each slot runs its own request from its own day 0 and
    one step() advances every running slot by a day in shared launches
    (include/episim.h, slot handles)."""

    def __init__(self, network, n_slots, *, stream=None, torch_workspace=True, device=0, slot_lanes=64):
        self.p = network
        self.n_slots, self.Nc, self.Nt, self.D = int(n_slots), network.n_comp, network.n_trans, network.n_days
        self.Nn = network.n_nodes
        self.slot_lanes = int(slot_lanes)
        self._h = C.c_void_p()
        self._ws = None
        self._keep = {}
        torch = _torch_cuda()
        st, keep = _marshal(network)
        opts = sim_device_opts()
        opts.slot_lanes = self.slot_lanes
        if torch is not None:
            torch.cuda.set_device(device)
            if stream is None:
                stream = torch.cuda.current_stream().cuda_stream
            if torch_workspace:
                nbytes = int(lib().sim_slots_workspace_bytes(C.byref(st), self.n_slots, C.byref(opts)))
                if nbytes == 0:
                    raise SimError(SIM_EINVAL, "network rejected (sim_slots_workspace_bytes returned 0)")
                self._ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{device}")
                opts.workspace = self._ws.data_ptr()
                opts.workspace_bytes = nbytes
        opts.stream = stream if stream is not None else None
        rc = lib().sim_slots_create(C.byref(st), self.n_slots, C.byref(opts), C.byref(self._h))
        del keep
        if rc != SIM_OK:
            raise SimError(rc, lib().sim_last_error(None).decode())

    @staticmethod
    def workspace_bytes(network, n_slots, slot_lanes=64):
        st, keep = _marshal(network)
        opts = sim_device_opts()
        opts.slot_lanes = int(slot_lanes)
        return int(lib().sim_slots_workspace_bytes(C.byref(st), int(n_slots), C.byref(opts)))

    def _check(self, rc):
        if rc != SIM_OK:
            raise SimError(rc, lib().sim_last_error(self._h).decode())

    def start(self, slot, horizon, coef, alpha, beta, replicate_id=None):
        coef = np.ascontiguousarray(coef, np.float64).reshape(-1, self.Nt)
        n = coef.shape[0]
        alpha = np.ascontiguousarray(alpha, np.float64).reshape(n)
        beta = np.ascontiguousarray(beta, np.float64).reshape(n, 4)
        rid = None if replicate_id is None else np.ascontiguousarray(replicate_id, np.uint32).reshape(n)
        self._check(lib().sim_slot_start(self._h, int(slot), n, int(horizon), _p(coef, _f64p), _p(alpha, _f64p),
                                         _p(beta, _f64p), None if rid is None else _p(rid, _u32p)))

    def step(self):
        """Advance every running slot by one day; returns the slots that finished."""
        fin = np.zeros(self.n_slots, np.int32)
        nf = C.c_int32()
        self._check(lib().sim_slots_step(self._h, _p(fin, _i32p), C.byref(nf)))
        return fin[:nf.value].tolist()

    def in_flight(self):
        return int(lib().sim_slots_in_flight(self._h))

    def fetch(self, slot, prevalence=None, transitions=None, totals=None):
        """Enqueue the download of a finished slot's records into the given
        buffers (numpy arrays or torch CPU tensors; pinned ones keep it
        asynchronous). They are kept alive until query() collects them."""
        self._keep[slot] = (prevalence, transitions, totals)
        self._check(lib().sim_slot_fetch(self._h, int(slot), _ptr(prevalence, _i32p), _ptr(transitions, _i64p),
                                         _ptr(totals, _i64p)))

    def query(self, slot):
        """True once the fetch of slot has landed; raises the slot's own error."""
        rc = lib().sim_slot_query(self._h, int(slot))
        if rc == 1:
            return False
        self._keep.pop(slot, None)
        self._check(rc)
        return True

    def state(self, slot, n_rep):
        u = np.zeros((n_rep, self.Nn, self.Nc), np.int32)
        v = np.zeros((n_rep, self.Nn), np.float64)
        self._check(lib().sim_slot_state(self._h, int(slot), _p(u, _i32p), _p(v, _f64p)))
        return u, v

    def kernel_times(self, enable):
        ms = np.zeros(4)
        n = np.zeros(4, np.int64)
        self._check(lib().sim_kernel_times(self._h, int(enable), _p(ms, _f64p), _p(n, _i64p)))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_CLASSES)}

    def sync(self):
        self._check(lib().sim_sync(self._h))

    def close(self):
        if self._h:
            lib().sim_destroy(self._h)
            self._h = C.c_void_p()
        self._ws = None
        self._keep = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
