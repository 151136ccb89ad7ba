"""ctypes front end of the reference oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg. The GPU library never imports or links it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_i32p = C.POINTER(C.c_int32)
_u32p = C.POINTER(C.c_uint32)
_i64p = C.POINTER(C.c_int64)
_f64p = C.POINTER(C.c_double)


class _Problem(C.Structure):
    _fields_ = [
        ("Nn", C.c_int32), ("Nc", C.c_int32), ("Nt", C.c_int32), ("R", C.c_int32), ("day0", C.c_int32),
        ("S", _i32p), ("reactant", _i32p), ("uses_phi", _i32p),
        ("coef", _f64p), ("alpha", _f64p), ("beta", _f64p),
        ("phi_I_mask", C.c_uint32), ("phi_N_mask", C.c_uint32),
        ("n_select", C.c_int32), ("E", _i32p),
        ("n_shift", C.c_int32), ("Nsh", _i32p),
        ("n_events", C.c_int64),
        ("ev_day", _i32p), ("ev_kind", _i32p), ("ev_node", _i32p), ("ev_dest", _i32p),
        ("ev_n", _i32p), ("ev_select", _i32p), ("ev_shift", _i32p),
        ("seed", C.c_uint32), ("replicate_id", _u32p),
        ("reactant2", _i32p), ("phi_pre_events", C.c_int32),
        ("n_regions", C.c_int32), ("region", _i32p),
    ]


class _Output(C.Structure):
    _fields_ = [
        ("prevalence", _i32p), ("transitions", _i64p), ("totals", _i64p),
        ("n_record", C.c_int32), ("record_days", _i32p),
        ("snap_u", _i32p), ("snap_v", _f64p), ("regional", _i64p), ("max_trans", _i32p),
        ("err_event", C.c_int64), ("err_rep", C.c_int32), ("err_day", C.c_int32),
    ]


_libs = {}


def lib(path=None):
    """The compiled oracle (built on first use); path selects another build."""
    path = LIB_PATH if path is None else path
    if path not in _libs:
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            from . import build as _b  # oracle/build.py
            _b.build()
        L = C.CDLL(path)
        L.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.oracle_u53.argtypes = [C.c_uint32, C.c_uint32]
        L.oracle_u53.restype = C.c_double
        L.oracle_mulhi64.argtypes = [C.c_uint64, C.c_uint64]
        L.oracle_mulhi64.restype = C.c_uint64
        L.oracle_neglog.argtypes = [C.c_double]
        L.oracle_neglog.restype = C.c_double
        L.oracle_quarter.argtypes = [C.c_int64]
        L.oracle_quarter.restype = C.c_int
        L.oracle_run.argtypes = [C.POINTER(_Problem), _i32p, _f64p, C.c_int32, C.c_int32, C.c_int32,
                                 C.POINTER(_Output)]
        L.oracle_run.restype = C.c_int
        _libs[path] = L
    return _libs[path]


def _ptr(a, t):
    return a.ctypes.data_as(t)


# --- primitives -------------------------------------------------------------

def philox(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().oracle_philox4x32_10(_ptr(c, _u32p), _ptr(k, _u32p), _ptr(o, _u32p))
    return o


def u53(lo, hi):
    return lib().oracle_u53(int(lo), int(hi))


def mulhi64(a, b):
    return lib().oracle_mulhi64(int(a), int(b))


def neglog(u):
    return lib().oracle_neglog(float(u))


def quarter(t):
    return lib().oracle_quarter(int(t))


# --- whole runs ---------------------------------------------------------------

class OracleError(RuntimeError):
    def __init__(self, code, event=-1, rep=-1, day=-1):
        super().__init__(f"oracle error {code} (event {event}, replicate {rep}, day {day})")
        self.code, self.event, self.rep, self.day = code, event, rep, day


def run(p, d_begin=0, d_end=None, u=None, v=None, threads=1, record_days=None, raise_on_error=True,
        lib_path=None):
    """Run the oracle on farmnet.Problem p over days [d_begin, d_end).

    u, v: starting state (R*Nn*Nc int32 node-major per replicate, R*Nn float64);
    defaults to the problem's initial state for every replicate. Returns a dict
    with the final state and the per-day records (indices relative to d_begin).
    """
    d_end = p.n_days if d_end is None else d_end
    R, Nn, Nc = p.n_rep, p.n_nodes, p.n_comp
    D = d_end - d_begin
    if u is None:
        u = np.tile(p.u0.reshape(1, Nn, Nc), (R, 1, 1))
    if v is None:
        v = np.tile(p.v0.reshape(1, Nn), (R, 1))
    u = np.ascontiguousarray(np.array(u, dtype=np.int32).reshape(R, Nn, Nc))
    v = np.ascontiguousarray(np.array(v, dtype=np.float64).reshape(R, Nn))
    rec = p.record_days if record_days is None else np.asarray(record_days, np.int32)
    rec = np.ascontiguousarray(rec[(rec >= d_begin) & (rec < d_end)], np.int32)
    r2 = getattr(p, "reactant2", None)
    r2 = None if r2 is None else np.ascontiguousarray(r2, np.int32)
    reg = getattr(p, "region", None)
    J = 0 if reg is None else int(p.n_regions)
    reg = None if reg is None else np.ascontiguousarray(reg, np.int32)
    keep = [p.S, p.reactant, p.uses_phi, p.coef, p.alpha, p.beta, p.E, p.N, p.replicate_id, r2, reg]
    prob = _Problem(
        Nn, Nc, p.n_trans, R, p.day0,
        _ptr(p.S, _i32p), _ptr(p.reactant, _i32p), _ptr(p.uses_phi, _i32p),
        _ptr(p.coef, _f64p), _ptr(p.alpha, _f64p), _ptr(p.beta, _f64p),
        p.phi_I_mask, p.phi_N_mask,
        p.n_select, _ptr(p.E, _i32p), p.n_shift, _ptr(p.N, _i32p),
        p.n_events,
        _ptr(p.ev_day, _i32p), _ptr(p.ev_kind, _i32p), _ptr(p.ev_node, _i32p), _ptr(p.ev_dest, _i32p),
        _ptr(p.ev_n, _i32p), _ptr(p.ev_select, _i32p), _ptr(p.ev_shift, _i32p),
        p.seed & 0xFFFFFFFF, _ptr(p.replicate_id, _u32p),
        None if r2 is None else _ptr(r2, _i32p), int(getattr(p, "phi_pre_events", 0)),
        J, None if reg is None else _ptr(reg, _i32p))
    out = dict(
        prevalence=np.zeros((D, R), np.int32),
        transitions=np.zeros((D, R), np.int64),
        totals=np.zeros((D, R, Nc), np.int64),
        snap_u=np.zeros((len(rec), R, Nn, Nc), np.int32),
        snap_v=np.zeros((len(rec), R, Nn), np.float64),
        regional=np.zeros((D, R, J, Nc), np.int64),
        max_transitions=np.zeros((D, R), np.int32),
    )
    o = _Output(_ptr(out["prevalence"], _i32p), _ptr(out["transitions"], _i64p), _ptr(out["totals"], _i64p),
                len(rec), _ptr(rec, _i32p), _ptr(out["snap_u"], _i32p), _ptr(out["snap_v"], _f64p),
                _ptr(out["regional"], _i64p) if J else None, _ptr(out["max_transitions"], _i32p), -1, -1, -1)
    rc = lib(lib_path).oracle_run(C.byref(prob), _ptr(u, _i32p), _ptr(v, _f64p), d_begin, d_end, threads, C.byref(o))
    del keep
    out.update(u=u, v=v, rc=rc, err_event=o.err_event, err_rep=o.err_rep, err_day=o.err_day,
               record_days=rec)
    if rc != 0 and raise_on_error:
        raise OracleError(rc, o.err_event, o.err_rep, o.err_day)
    return out
